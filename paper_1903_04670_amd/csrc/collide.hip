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

template <typename T, int N>
static hipError_t launch_pipeline_N(const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa, hipStream_t st,
                                    bool do_fwd, bool vss) {
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
    switch (shift_split<T>()) {
      case 1: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 1, true>), dim3(pbh, 2, EG), dim3(64), 0, st, a); break;
      case 4: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 4, true>), dim3(pbh, 8, EG), dim3(64), 0, st, a); break;
      case 8: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 8, true>), dim3(pbh, 16, EG), dim3(64), 0, st, a); break;
      default: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 2, true>), dim3(pbh, 4, EG), dim3(64), 0, st, a); break;
    }
  } else {
    switch (shift_split<T>()) {
      case 1: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 1>), dim3(pb2, 2, EG), dim3(64), 0, st, a); break;
      case 4: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 4>), dim3(pb2, 8, EG), dim3(64), 0, st, a); break;
      case 8: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 8>), dim3(pb2, 16, EG), dim3(64), 0, st, a); break;
      default: DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N, 2>), dim3(pb2, 4, EG), dim3(64), 0, st, a); break;
    }
  }
  constexpr int GG = literal_gain_groups<T, N>(), GP = packed_gain_groups<N>();
  if (!vss) {
    if (a.pack)
      DGFS_LAUNCH("k_gain_yz", (k_gain_yz<T, N, GP, 1, true>), dim3(N, a.Nr, EG), dim3(GP * 2 * N), 0, st, a);
    else
      DGFS_LAUNCH("k_gain_yz", (k_gain_yz<T, N, GG>), dim3(N, a.Nr, EG), dim3(GG * 2 * N), 0, st, a);
    DGFS_LAUNCH("k_gain_x", (k_gain_x<T, N, sizeof(T) == 4>), dim3(pb2, sizeof(T) == 4 ? EG : E), dim3(64), 0, st, a);
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
                                    hipStream_t st, bool do_fwd, bool vss) {
  switch (N) {
    case 4: return launch_pipeline_N<T, 4>(a, fw, fa, st, do_fwd, vss);
    case 6: return launch_pipeline_N<T, 6>(a, fw, fa, st, do_fwd, vss);
    case 8: return launch_pipeline_N<T, 8>(a, fw, fa, st, do_fwd, vss);
    case 12: return launch_pipeline_N<T, 12>(a, fw, fa, st, do_fwd, vss);
    case 16: return launch_pipeline_N<T, 16>(a, fw, fa, st, do_fwd, vss);
    case 18: return launch_pipeline_N<T, 18>(a, fw, fa, st, do_fwd, vss);
    case 24: return launch_pipeline_N<T, 24>(a, fw, fa, st, do_fwd, vss);
    case 32: return launch_pipeline_N<T, 32>(a, fw, fa, st, do_fwd, vss);
    case 36: return launch_pipeline_N<T, 36>(a, fw, fa, st, do_fwd, vss);
    case 10: return launch_pipeline_N<T, 10>(a, fw, fa, st, do_fwd, vss);
    case 14: return launch_pipeline_N<T, 14>(a, fw, fa, st, do_fwd, vss);
    case 40: return launch_pipeline_N<T, 40>(a, fw, fa, st, do_fwd, vss);
    case 56: return launch_pipeline_N<T, 56>(a, fw, fa, st, do_fwd, vss);
    case 48: return launch_pipeline_N<T, 48>(a, fw, fa, st, do_fwd, vss);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pipeline(const dgfs_plan_s *pl, const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa,
                           hipStream_t st, bool do_fwd) {
  if (pl->precision == DGFS_FP64) return launch_pipeline_T<double>(pl->N, a, fw, fa, st, do_fwd, !pl->vhs);
  return launch_pipeline_T<float>(pl->N, a, fw, fa, st, do_fwd, !pl->vhs);
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
  a.sneg = pl->sneg_dev;
  a.gs_full = pl->gs_full_dev;
  a.gs_half = pl->gs_half_dev;
  a.gs_T_full = pl->gs_T_full;
  a.gs_T_half = pl->gs_T_half;
  a.pack = pl->nyquist_zero && pl->vhs ? 1 : 0;
}

}  // namespace dgfs

using namespace dgfs;

extern "C" dgfs_status dgfs_collide(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                    const double *fq, int64_t node_stride, double *Q, int64_t out_stride,
                                    uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (!pl) { set_error("dgfs_collide: NULL plan"); return DGFS_EINVAL; }
  if (n_nodes < 0) { set_error("dgfs_collide: n_nodes < 0"); return DGFS_EINVAL; }
  if (p < 0 || q < 0 || p >= pl->ns || q >= pl->ns) { set_error("dgfs_collide: species (%d, %d) out of range", p, q); return DGFS_EINVAL; }
  if (flags & ~(DGFS_ACCUMULATE | DGFS_CHECK)) { set_error("dgfs_collide: unsupported flags 0x%x", flags); return DGFS_EINVAL; }
  if (n_nodes == 0) return DGFS_OK;
  if (!fp || !fq || !Q) { set_error("dgfs_collide: NULL array"); return DGFS_EINVAL; }
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  if (n_nodes > 1 && (node_stride < n3 || out_stride < n3)) { set_error("dgfs_collide: strides must be >= N^3"); return DGFS_EINVAL; }
  const int nz = (p == q && fp == fq) ? 1 : 2;
  const int B = chunk_nodes(pl, n_nodes, 1);
  const size_t need = pipeline_bytes(pl, B, 1, nz);
  if (!ws || ws_bytes < need) { set_error("dgfs_collide: workspace %zu bytes, need %zu", ws_bytes, need); return DGFS_EWORKSPACE; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  PipeArgs a{};
  pipeline_common(pl, a);
  pipeline_carve(pl, B, 1, nz, ws, a);
  a.n_pairs = 1;
  a.nz = nz;
  a.pair_id[0] = p * pl->ns + q;
  a.zp[0] = 0;
  a.zq[0] = nz == 1 ? 0 : 1;
  a.xshare[0] = nz == 1 ? 1 : 0;
  pipeline_slots(pl, a);
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
    fa.out[0] = Q + n0 * out_stride;
    fa.out_stride = out_stride;
    fa.accumulate = (flags & DGFS_ACCUMULATE) ? 1 : 0;
    hipError_t e = launch_pipeline(pl, a, fw, fa, st, true);
    if (e != hipSuccess) return hip_status(e, "dgfs_collide launch");
  }
  if (flags & DGFS_CHECK) return check_finite(Q, n_nodes, n3, out_stride, st);
  return DGFS_OK;
}

extern "C" size_t dgfs_workspace_bytes(dgfs_plan pl, int64_t n_nodes, int32_t op) {
  if (!pl || n_nodes <= 0) return 0;
  switch (op) {
    case DGFS_OP_COLLIDE: {
      const int B = chunk_nodes(pl, n_nodes, 1);
      return pipeline_bytes(pl, B, 1, 2);
    }
    default:
      return extra_workspace_bytes(pl, n_nodes, op);
  }
}
