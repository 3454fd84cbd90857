// Launch layer and entry point of the collision operator's vector-Jacobian product.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pipeline.hpp"
#include "launch.hpp"
#include "vjp_kernels.hpp"

namespace dgfs {

static size_t a256(size_t b) { return (b + 255) / 256 * 256; }

struct VjpLayout {
  size_t z, x, zw, vx, y, h;
  size_t total() const { return z + x + zw + vx + y + h; }
};

static VjpLayout vjp_layout(const dgfs_plan_s *pl, int B) {
  const size_t n3 = (size_t)pl->N * pl->N * pl->N, c = 2 * pl->elt();
  VjpLayout l;
  l.z = a256((size_t)B * 2 * n3 * c);
  l.x = a256((size_t)B * 2 * pl->Nr * pl->Sx * n3 * c);
  l.zw = a256((size_t)B * 2 * n3 * c);
  l.vx = a256((size_t)B * pl->Nr * (pl->vhs ? 1 : pl->M) * n3 * c);  // VSS: one array per (r, m)
  l.y = l.x;
  l.h = a256((size_t)B * 3 * n3 * c);
  return l;
}

size_t vjp_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes) {
  return vjp_layout(pl, chunk_nodes(pl, n_nodes, 1)).total();
}

template <int N> constexpr int vgroups() { return 64 / N > 0 ? 64 / N : 1; }

template <typename T, int N>
static hipError_t launch_vjp_N(const VjpArgs &v, const FwdArgs &fw, hipStream_t st) {
  constexpr int G = vgroups<N>();
  const PipeArgs &a = v.a;
  const int E = a.n_nodes * a.n_pairs;
  const int planes_f = N * fw.n_nodes * fw.nz;
  DGFS_LAUNCH("k_fwd_yz", (k_fwd_yz<T, N, G>), dim3((planes_f + G - 1) / G), dim3(G * N), 0, st, fw);
  const int planes_w = N * a.n_nodes * 2;
  DGFS_LAUNCH("k_inv_yz", (k_inv_yz<T, N, G>), dim3((planes_w + G - 1) / G), dim3(G * N), 0, st, v);
  DGFS_LAUNCH("k_shift_x", (k_shift_x<T, N>), dim3((N * N + 31) / 32, 2, E), dim3(64), 0, st, a);
  const int pb2 = (N * N + 31) / 32;  // lane pairs: 32 x-lines per 64-thread block
  constexpr int GV = 128 / (2 * N) > 0 ? 128 / (2 * N) : 1;  // groups per block, as the plan's VJP schedule
  const dim3 gyz(N, a.Nr, E), byz(GV * 2 * N);
  // the scalar-phase path needs unzeroed twiddle rows (no nyquist_zero)
  if (v.vss) {
    DGFS_LAUNCH("k_vjp_v", (k_vjp_v<T, N, true>), dim3(pb2, E), dim3(64), 0, st, v);
    if (v.nyq) DGFS_LAUNCH("k_vjp_yz", (k_vjp_yz<T, N, GV, false, true>), gyz, byz, 0, st, v);
    else DGFS_LAUNCH("k_vjp_yz", (k_vjp_yz<T, N, GV, true, true>), gyz, byz, 0, st, v);
  } else {
    DGFS_LAUNCH("k_vjp_v", (k_vjp_v<T, N>), dim3(pb2, E), dim3(64), 0, st, v);
    if (v.nyq) DGFS_LAUNCH("k_vjp_yz", (k_vjp_yz<T, N, GV, false>), gyz, byz, 0, st, v);
    else DGFS_LAUNCH("k_vjp_yz", (k_vjp_yz<T, N, GV>), gyz, byz, 0, st, v);
  }
  if (v.sym)
    DGFS_LAUNCH("k_vjp_x", (k_vjp_x<T, N, true>), dim3(pb2, E), dim3(64), 0, st, v);
  else
    DGFS_LAUNCH("k_vjp_x", (k_vjp_x<T, N, false>), dim3(pb2, E), dim3(64), 0, st, v);
  const int planes_o = N * a.n_nodes;
  DGFS_LAUNCH("k_vjp_final", (k_vjp_final<T, N, G>), dim3((planes_o + G - 1) / G), dim3(G * N), 0, st, v);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_vjp_T(int N, const VjpArgs &v, const FwdArgs &fw, hipStream_t st) {
  switch (N) {
    case 4: return launch_vjp_N<T, 4>(v, fw, st);
    case 6: return launch_vjp_N<T, 6>(v, fw, st);
    case 8: return launch_vjp_N<T, 8>(v, fw, st);
    case 12: return launch_vjp_N<T, 12>(v, fw, st);
    case 16: return launch_vjp_N<T, 16>(v, fw, st);
    case 18: return launch_vjp_N<T, 18>(v, fw, st);
    case 24: return launch_vjp_N<T, 24>(v, fw, st);
    case 32: return launch_vjp_N<T, 32>(v, fw, st);
    case 36: return launch_vjp_N<T, 36>(v, fw, st);
    case 10: return launch_vjp_N<T, 10>(v, fw, st);
    case 14: return launch_vjp_N<T, 14>(v, fw, st);
    case 40: return launch_vjp_N<T, 40>(v, fw, st);
    case 56: return launch_vjp_N<T, 56>(v, fw, st);
    case 48: return launch_vjp_N<T, 48>(v, fw, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgfs

using namespace dgfs;

extern "C" dgfs_status dgfs_collide_vjp(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                        const double *fq, int64_t node_stride, const double *wbar,
                                        int64_t wbar_stride, double *grad_fp, double *grad_fq, int64_t grad_stride,
                                        uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (!pl) { set_error("dgfs_collide_vjp: NULL plan"); return DGFS_EINVAL; }
  if (n_nodes < 0) { set_error("dgfs_collide_vjp: n_nodes < 0"); return DGFS_EINVAL; }
  if (p < 0 || q < 0 || p >= pl->ns || q >= pl->ns) { set_error("dgfs_collide_vjp: species out of range"); return DGFS_EINVAL; }
  if (flags & ~DGFS_ACCUMULATE) { set_error("dgfs_collide_vjp: unsupported flags 0x%x", flags); return DGFS_EINVAL; }
  if (n_nodes == 0) return DGFS_OK;
  if (!fp || !fq || !wbar || (!grad_fp && !grad_fq)) { set_error("dgfs_collide_vjp: NULL array"); return DGFS_EINVAL; }
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  if (n_nodes > 1 && (node_stride < n3 || wbar_stride < n3 || grad_stride < n3)) {
    set_error("dgfs_collide_vjp: strides must be >= N^3");
    return DGFS_EINVAL;
  }
  const int B = chunk_nodes(pl, n_nodes, 1);
  const VjpLayout l = vjp_layout(pl, B);
  if (!ws || ws_bytes < l.total()) { set_error("dgfs_collide_vjp: workspace %zu bytes, need %zu", ws_bytes, l.total()); return DGFS_EWORKSPACE; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  VjpArgs v{};
  pipeline_common(pl, v.a);
  char *b = static_cast<char *>(ws);
  v.a.Z = b;
  v.a.X = b + l.z;
  v.Zw = b + l.z + l.x;
  v.Vx = b + l.z + l.x + l.zw;
  v.Y = b + l.z + l.x + l.zw + l.vx;
  v.H = b + l.z + l.x + l.zw + l.vx + l.y;
  v.a.n_pairs = 1;
  v.a.nz = 2;
  v.a.pair_id[0] = p * pl->ns + q;
  v.a.zp[0] = 0;
  v.a.zq[0] = 1;
  // p == q on one input: the second side's x-shifted arrays are the first
  // side's of the opposite sigma_x; with an antipodal sphere set the two
  // sides' gain sums coincide as well (the gain part of Q(f, g) is then
  // symmetric in f and g), so only side 0's sums are formed
  const bool same = p == q && fp == fq;
  v.a.xshare[0] = same ? 1 : 0;
  pipeline_slots(pl, v.a);
  // the symmetric shortcut needs a direction-independent table (VHS)
  v.sym = (same && pl->antipodal && pl->vhs) ? 1 : 0;
  v.vss = pl->vhs ? 0 : 1;
  v.nyq = pl->nyquist_zero ? 1 : 0;
  v.f_stride = node_stride;
  v.w_stride = wbar_stride;
  v.g_stride = grad_stride;
  v.accumulate = (flags & DGFS_ACCUMULATE) ? 1 : 0;
  v.sched = v.sym ? pl->vjp_sched_sym_dev : pl->vjp_sched_dev;
  v.sched_T = v.sym ? pl->vjp_T_sym : pl->vjp_T;
  for (int64_t n0 = 0; n0 < n_nodes; n0 += B) {
    const int nb = (int)std::min<int64_t>(B, n_nodes - n0);
    v.a.n_nodes = nb;
    v.f = fp + n0 * node_stride;
    v.w = wbar + n0 * wbar_stride;
    v.gf = grad_fp ? grad_fp + n0 * grad_stride : nullptr;
    v.gg = grad_fq ? grad_fq + n0 * grad_stride : nullptr;
    FwdArgs fw{};
    fw.src[0] = fp + n0 * node_stride;
    fw.src[1] = fq + n0 * node_stride;
    fw.node_stride = node_stride;
    fw.n_nodes = nb;
    fw.nz = 2;
    fw.Z = v.a.Z;
    hipError_t e = pl->precision == DGFS_FP64 ? launch_vjp_T<double>(pl->N, v, fw, st)
                                              : launch_vjp_T<float>(pl->N, v, fw, st);
    if (e != hipSuccess) return hip_status(e, "dgfs_collide_vjp launch");
  }
  return DGFS_OK;
}
