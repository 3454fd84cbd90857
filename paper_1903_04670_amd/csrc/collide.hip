// Launch layer of the collision pipeline and the dgfs_collide entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "collide_kernels.hpp"
#include "vss_kernels.hpp"
#include "pipeline.hpp"
#include "launch.hpp"

namespace dgfs {

template <int N> constexpr int groups_for() { return N >= 64 ? 1 : (64 / N > 0 ? 64 / N : 1); }
// k_shift_x (r, s) loop split per block: $DGFS_SHIFT_SPLIT in {1, 2, 4, 8};
// default 2 in FP64 (HBM-bound, no gain beyond) and 8 in FP32
template <typename T> static int shift_split() {
  static const int v = [] {
    const char *s = std::getenv("DGFS_SHIFT_SPLIT");
    const int x = s ? std::atoi(s) : (sizeof(T) == 8 ? 2 : 8);
    return (x == 1 || x == 2 || x == 4 || x == 8) ? x : 2;
  }();
  return v;
}
// groups of 2N threads per k_gain_yz block: at least 128 threads per block
template <int N> constexpr int gain_groups() { return 128 / (2 * N) > 0 ? 128 / (2 * N) : 1; }

// Launch-schedule choices that do not change results: the x-shift split
// and whether k_gain_x serves a mirrored slot in the same pass.
struct Sched {
  int split;
  bool fuse;
};

template <typename T> static Sched plan_sched(const dgfs_plan_s *pl) {
  Sched s;
  s.split = pl->shift_split > 0 ? pl->shift_split : shift_split<T>();
  s.fuse = pl->gain_x_fuse >= 0 ? pl->gain_x_fuse != 0 : sizeof(T) == 4;
  return s;
}

template <typename T, int N>
static hipError_t launch_pipeline_N(const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa, hipStream_t st,
                                    bool do_fwd, bool vss, Sched sc) {
  constexpr int G = groups_for<N>();
  const int E = a.n_nodes * a.n_pairs, EG = a.n_nodes * a.n_gslots;
  if (do_fwd) {
    const int planes = N * fw.n_nodes * fw.nz;
    DGFS_LAUNCH("k_fwd_yz", (k_fwd_yz<T, N, G>), dim3((planes + G - 1) / G), dim3(G * N), 0, st, fw);
  }
  const int pb2 = (N * N + 31) / 32;  // lane pairs: 32 x-lines per 64-thread block
  if (a.pack && !vss) {
    // real-packed gain: the x-lines with k_z < N/2 only
    const int pbh = (N * (N / 2) + 31) / 32;
    switch (sc.split) {
      case 1: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 1, true>), dim3(pbh, 2, EG), dim3(64), 0, st, a); break;
      case 4: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 4, true>), dim3(pbh, 8, EG), dim3(64), 0, st, a); break;
      case 8: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 8, true>), dim3(pbh, 16, EG), dim3(64), 0, st, a); break;
      default: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 2, true>), dim3(pbh, 4, EG), dim3(64), 0, st, a); break;
    }
  } else {
    switch (sc.split) {
      case 1: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 1>), dim3(pb2, 2, EG), dim3(64), 0, st, a); break;
      case 4: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 4>), dim3(pb2, 8, EG), dim3(64), 0, st, a); break;
      case 8: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 8>), dim3(pb2, 16, EG), dim3(64), 0, st, a); break;
      default: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 2>), dim3(pb2, 4, EG), dim3(64), 0, st, a); break;
    }
  }
  constexpr int GG = literal_gain_groups<T, N>(), GP = packed_gain_groups<N>();
  if (!vss) {
    if constexpr (gain_halves<T, N>()) {
      if (a.pack)
        DGFS_LAUNCH("k_gain_yz", (k_gain_yz_halves_packed<T, N>), dim3(N / 2, a.Nr, EG), dim3(128), 0, st, a);
      else
        DGFS_LAUNCH("k_gain_yz", (k_gain_yz_halves<T, N>), dim3(N / 2, a.Nr, EG), dim3(128), 0, st, a);
    } else {
      if (a.pack)
        DGFS_LAUNCH("k_gain_yz", (k_gain_yz<T, N, GP, 1, true>), dim3(N, a.Nr, EG), dim3(GP * 2 * N), 0, st, a);
      else
        DGFS_LAUNCH("k_gain_yz", (k_gain_yz<T, N, GG>), dim3(N, a.Nr, EG), dim3(GG * 2 * N), 0, st, a);
    }
    if (sc.fuse)
      DGFS_LAUNCH("k_gain_x", (k_gain_x<T, N, true>), dim3(pb2, EG), dim3(64), 0, st, a);
    else
      DGFS_LAUNCH("k_gain_x", (k_gain_x<T, N, false>), dim3(pb2, E), dim3(64), 0, st, a);
  } else {
    constexpr int TE = N >= 48 ? 1 : 2;
    const int egroups = a.n_pairs * ((a.n_nodes + TE - 1) / TE);
    constexpr int GV = gain_groups<N>();
    DGFS_LAUNCH("k_gain_yz_vss", (k_gain_yz_vss<T, N, GV>), dim3(N, a.Nr, EG), dim3(GV * 2 * N), 0, st, a);
    DGFS_LAUNCH("k_gain_x_vss", (k_gain_x_vss<T, N, TE>), dim3(pb2, egroups), dim3(64), 0, st, a);
  }
  const int fplanes = N * a.n_nodes * fa.n_out;
  constexpr int GF = final_groups<N>();
  DGFS_LAUNCH("k_final_yz", (k_final_yz<T, N, GF>), dim3((fplanes + GF - 1) / GF), dim3(GF * 2 * N), 0, st, a, fa);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pipeline_T(int N, const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa,
                                    hipStream_t st, bool do_fwd, bool vss, Sched sc) {
  switch (N) {
    case 4: return launch_pipeline_N<T, 4>(a, fw, fa, st, do_fwd, vss, sc);
    case 6: return launch_pipeline_N<T, 6>(a, fw, fa, st, do_fwd, vss, sc);
    case 8: return launch_pipeline_N<T, 8>(a, fw, fa, st, do_fwd, vss, sc);
    case 12: return launch_pipeline_N<T, 12>(a, fw, fa, st, do_fwd, vss, sc);
    case 16: return launch_pipeline_N<T, 16>(a, fw, fa, st, do_fwd, vss, sc);
    case 18: return launch_pipeline_N<T, 18>(a, fw, fa, st, do_fwd, vss, sc);
    case 24: return launch_pipeline_N<T, 24>(a, fw, fa, st, do_fwd, vss, sc);
    case 32: return launch_pipeline_N<T, 32>(a, fw, fa, st, do_fwd, vss, sc);
    case 36: return launch_pipeline_N<T, 36>(a, fw, fa, st, do_fwd, vss, sc);
    case 10: return launch_pipeline_N<T, 10>(a, fw, fa, st, do_fwd, vss, sc);
    case 14: return launch_pipeline_N<T, 14>(a, fw, fa, st, do_fwd, vss, sc);
    case 40: return launch_pipeline_N<T, 40>(a, fw, fa, st, do_fwd, vss, sc);
    case 56: return launch_pipeline_N<T, 56>(a, fw, fa, st, do_fwd, vss, sc);
    case 48: return launch_pipeline_N<T, 48>(a, fw, fa, st, do_fwd, vss, sc);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pipeline(const dgfs_plan_s *pl, const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa,
                           hipStream_t st, bool do_fwd) {
  if (pl->precision == DGFS_FP64)
    return launch_pipeline_T<double>(pl->N, a, fw, fa, st, do_fwd, !pl->vhs, plan_sched<double>(pl));
  return launch_pipeline_T<float>(pl->N, a, fw, fa, st, do_fwd, !pl->vhs, plan_sched<float>(pl));
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }


// Evaluations per launch when no tuned width is known ($DGFS_CHUNK_EVALS,
// 0 = the default for the plan's precision).
int max_evals_per_chunk() {
  static int v = [] {
    const char *s = std::getenv("DGFS_CHUNK_EVALS");
    const int x = s ? std::atoi(s) : 0;
    return x > 0 ? x : 0;
  }();
  return v;
}

// Nodes per launch.  The width in evaluations comes from the autotuner's
// cache, $DGFS_CHUNK_EVALS, or the default (measured at N = 32: 128 in FP64,
// 256 in FP32; 8-32 leave the GPU underfilled); a chunk's intermediates stay
// within 16 GiB (the VSS path stores every (r, m) term; HBM holds 288 GB);
// and the nodes are split evenly over the launches this needs, so no launch
// is a short tail.
int chunk_nodes(const dgfs_plan_s *pl, int64_t n_nodes, int n_pairs) {
  int evals = pl->chunk_evals > 0 ? pl->chunk_evals : max_evals_per_chunk();
  if (evals <= 0) evals = pl->precision == DGFS_FP64 ? 128 : 256;
  int64_t b = std::max<int64_t>(1, evals / n_pairs);
  const size_t per_node = pipeline_bytes(pl, 1, n_pairs, std::min(pl->ns, 2 * n_pairs));
  const int64_t cap = std::max<int64_t>(1, (int64_t)((size_t)16 << 30) / (int64_t)per_node);
  b = std::max<int64_t>(1, std::min(b, cap));
  if (n_nodes <= b) return (int)std::max<int64_t>(1, n_nodes);
  const int64_t launches = (n_nodes + b - 1) / b;
  return (int)((n_nodes + launches - 1) / launches);
}

size_t pipeline_bytes(const dgfs_plan_s *pl, int B, int n_pairs, int nz) {
  const size_t n3 = (size_t)pl->N * pl->N * pl->N, c = 2 * pl->elt();
  const size_t E = (size_t)B * n_pairs;
  const size_t nc = pl->vhs ? (size_t)pl->Nr : (size_t)pl->Nr * pl->M;  // C arrays per evaluation
  return align256((size_t)B * nz * n3 * c) + align256(E * 2 * pl->Nr * pl->Sx * n3 * c) +
         align256(E * nc * n3 * c) + align256(E * 2 * n3 * c);
}

void pipeline_carve(const dgfs_plan_s *pl, int B, int n_pairs, int nz, void *ws, PipeArgs &a) {
  const size_t n3 = (size_t)pl->N * pl->N * pl->N, c = 2 * pl->elt();
  const size_t E = (size_t)B * n_pairs;
  char *p = static_cast<char *>(ws);
  a.Z = p;
  p += align256((size_t)B * nz * n3 * c);
  a.X = p;
  p += align256(E * 2 * pl->Nr * pl->Sx * n3 * c);
  a.Cb = p;
  p += align256(E * (pl->vhs ? (size_t)pl->Nr : (size_t)pl->Nr * pl->M) * n3 * c);
  a.V = p;
}

bool symmetry_enabled() { return std::getenv("DGFS_NO_SYMMETRY") == nullptr; }

void pipeline_slots(const dgfs_plan_s *pl, PipeArgs &a) {
  const bool share = symmetry_enabled();
  a.Mh = (int)pl->mhalf.size();
  a.mhalf = pl->mhalf_dev;
  a.tinfo_half = pl->tinfo_half_dev;
  a.n_gslots = 0;
  for (int i = 0; i < a.n_pairs; ++i) a.cmirror[i] = -1;
  for (int i = 0; i < a.n_pairs; ++i) {
    const int p = a.pair_id[i] / pl->ns, q = a.pair_id[i] % pl->ns;
    a.csrc[i] = i;
    a.half[i] = (share && p == q && a.xshare[i] && pl->vhs && pl->antipodal) ? 1 : 0;
    int src = -1;
    if (share && p != q && pl->mirror_ok(p, q))
      for (int j = 0; j < i; ++j)
        if (a.csrc[j] == j && a.pair_id[j] == q * pl->ns + p && a.zp[j] == a.zq[i] && a.zq[j] == a.zp[i]) src = j;
    if (src >= 0) {
      a.csrc[i] = src;
      a.cmirror[src] = i;
    } else {
      a.gslot[a.n_gslots++] = i;
    }
  }
}

void pipeline_common(const dgfs_plan_s *pl, PipeArgs &a) {
  a.Nr = pl->Nr;
  a.Sx = pl->Sx;
  a.M = pl->M;
  a.ns = pl->ns;
  a.pairs = pl->pair_dev;
  a.wm = pl->wm_dev;
  a.sidx = pl->sidx_dev;
  a.sx_zero = pl->sxz_dev;
  a.morder = pl->morder_dev;
  a.tinfo_full = pl->tinfo_full_dev;
  a.sneg = pl->sneg_dev;
  a.gs_full = pl->gs_full_dev;
  a.gs_half = pl->gs_half_dev;
  a.gs_T_full = pl->gs_T_full;
  a.gs_T_half = pl->gs_T_half;
  a.pack = pl->nyquist_zero && pl->vhs ? 1 : 0;
}

}  // namespace dgfs

using namespace dgfs;

namespace dgfs {

// Workspace of dgfs_collide for chunks of B nodes: the pipeline's arrays,
// then (for DGFS_PROJECT) the unprojected collision term of the chunk and
// the partial moments.
size_t collide_bytes(const dgfs_plan_s *pl, int B, int nz) {
  const size_t n3 = (size_t)pl->N * pl->N * pl->N;
  return pipeline_bytes(pl, B, 1, nz) + align256((size_t)B * n3 * sizeof(double)) + proj_part_bytes(B);
}

// Largest chunk width (nodes per launch, at most the default one) whose
// workspace fits in `bytes`; 0 if a single node does not fit.
int collide_chunk_fitting(const dgfs_plan_s *pl, int64_t n_nodes, int nz, size_t bytes) {
  int B = chunk_nodes(pl, n_nodes, 1);
  while (B > 0 && collide_bytes(pl, B, nz) > bytes) --B;
  return B;
}

dgfs_status collide_impl(const dgfs_plan_s *pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                         const double *fq, int64_t node_stride, double *Q, int64_t out_stride, uint32_t flags,
                         void *ws, size_t ws_bytes, hipStream_t st, int B, const char *who) {
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  const int nz = (p == q && fp == fq) ? 1 : 2;
  const size_t need = collide_bytes(pl, B, nz);
  if (!ws || ws_bytes < need) { set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need); return DGFS_EWORKSPACE; }
  const bool project = flags & DGFS_PROJECT;
  PipeArgs a{};
  pipeline_common(pl, a);
  pipeline_carve(pl, B, 1, nz, ws, a);
  char *tail = static_cast<char *>(ws) + pipeline_bytes(pl, B, 1, nz);
  double *qc = reinterpret_cast<double *>(tail);
  double *part = reinterpret_cast<double *>(tail + align256((size_t)B * n3 * sizeof(double)));
  a.n_pairs = 1;
  a.nz = nz;
  a.pair_id[0] = p * pl->ns + q;
  a.zp[0] = 0;
  a.zq[0] = nz == 1 ? 0 : 1;
  a.xshare[0] = nz == 1 ? 1 : 0;
  pipeline_slots(pl, a);
  ProjArgs pa{};
  if (project) {
    // Q^{pq} alone conserves the mass of species p; the self-collision term
    // of one distribution (p == q, the same array) also conserves momentum
    // and energy.  Those are the rows projected.
    pa.N = pl->N;
    pa.nsp = 1;
    pa.L = pl->L;
    pa.mass[0] = pl->mass[p];
    pa.nblk = kProjBlocks;
    pa.part = part;
    pa.Q = qc;
    pa.q_stride = n3;
    pa.accumulate = (flags & DGFS_ACCUMULATE) ? 1 : 0;
    if (nz == 1) {
      pa.nrow = 5;
      std::memcpy(pa.ginv, pl->proj_ginv_self[p].data(), 25 * sizeof(double));
    } else {
      const double h = 2.0 * pl->L / pl->N, w = h * h * h;
      pa.nrow = 1;
      pa.ginv[0] = 1.0 / (w * w * (double)n3);
    }
  }
  for (int64_t n0 = 0; n0 < n_nodes; n0 += B) {
    const int nb = (int)std::min<int64_t>(B, n_nodes - n0);
    a.n_nodes = nb;
    FwdArgs fw{};
    fw.src[0] = fp + n0 * node_stride;
    fw.src[1] = fq + n0 * node_stride;
    fw.node_stride = node_stride;
    fw.n_nodes = nb;
    fw.nz = nz;
    fw.Z = a.Z;
    FinalArgs fa{};
    fa.n_out = 1;
    fa.qcount = 1;
    fa.fsrc[0] = fp + n0 * node_stride;
    fa.f_stride = node_stride;
    fa.out[0] = project ? qc : Q + n0 * out_stride;
    fa.out_stride = project ? n3 : out_stride;
    fa.accumulate = (!project && (flags & DGFS_ACCUMULATE)) ? 1 : 0;
    hipError_t e = launch_pipeline(pl, a, fw, fa, st, true);
    if (e == hipSuccess && project) {
      pa.out[0] = Q + n0 * out_stride;
      pa.out_stride = out_stride;
      e = launch_projection(pa, nb, st);
    }
    if (e != hipSuccess) return hip_status(e, "collision launch");
  }
  if (flags & DGFS_CHECK) return check_finite(Q, n_nodes, n3, out_stride, st);
  return DGFS_OK;
}

// Argument checks shared by dgfs_collide and its variants.
dgfs_status collide_validate(const dgfs_plan_s *pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                             const double *fq, int64_t node_stride, const double *Q, int64_t out_stride,
                             uint32_t flags, uint32_t allowed, const char *who) {
  if (!pl) { set_error("%s: NULL plan", who); return DGFS_EINVAL; }
  if (n_nodes < 0) { set_error("%s: n_nodes < 0", who); return DGFS_EINVAL; }
  if (p < 0 || q < 0 || p >= pl->ns || q >= pl->ns) { set_error("%s: species (%d, %d) out of range", who, p, q); return DGFS_EINVAL; }
  if (flags & ~allowed) { set_error("%s: unsupported flags 0x%x", who, flags); return DGFS_EINVAL; }
  if (n_nodes == 0) return DGFS_OK;
  if (!fp || !fq || !Q) { set_error("%s: NULL array", who); return DGFS_EINVAL; }
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  if (n_nodes > 1 && (node_stride < n3 || out_stride < n3)) { set_error("%s: strides must be >= N^3", who); return DGFS_EINVAL; }
  return DGFS_OK;
}

}  // namespace dgfs

extern "C" dgfs_status dgfs_collide(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                    const double *fq, int64_t node_stride, double *Q, int64_t out_stride,
                                    uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = collide_validate(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, flags,
                                   DGFS_ACCUMULATE | DGFS_PROJECT | DGFS_CHECK, "dgfs_collide");
  if (s != DGFS_OK || n_nodes == 0) return s;
  return collide_impl(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, flags, ws, ws_bytes,
                      static_cast<hipStream_t>(stream), chunk_nodes(pl, n_nodes, 1), "dgfs_collide");
}

extern "C" size_t dgfs_workspace_bytes(dgfs_plan pl, int64_t n_nodes, int32_t op) {
  if (!pl || n_nodes <= 0) return 0;
  switch (op) {
    case DGFS_OP_COLLIDE: {
      const int B = chunk_nodes(pl, n_nodes, 1);
      return collide_bytes(pl, B, 2);
    }
    default:
      return extra_workspace_bytes(pl, n_nodes, op);
  }
}
