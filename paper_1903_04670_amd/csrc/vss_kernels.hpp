// VSS (alpha != 1) gain path.  The gain table b_rm(k) depends on the
// direction sigma_m (Eq. Fkr_vss), so the sum over m cannot be taken before
// the forward transform: every term's product is transformed and multiplied
// by its own table (Algorithm 2 as written).
//   k_gain_yz_vss : per (eval, r, x-plane) and direction m: u1, u2 (as the VHS
//                   kernel), the product, and its forward yz transform C_rm
//   k_gain_x_vss  : per x-line: QG = sum_{r,m} B_rm(k) FFT_x C_rm with
//                   B_rm = w_r w_m b_rm / N^3 (summed in FP64), then
//                   V1 = iFFT_x QG and V2 = iFFT_x(c FFT_x Z_q).  A thread pair
//                   serves TE nodes of the same ordered pair so each table
//                   x-line is read once per TE evaluations.
#pragma once
#include "collide_kernels.hpp"

namespace dgfs {

template <typename T, int N, int G>
__device__ __forceinline__ void gain_yz_vss_body(const PipeArgs &a, int jx, int r, int e, int tid,
                                                 C<T> (*lds)[N][N + 1], C<T> *phs_all) {
  constexpr int H = N / 2;
  const int g = tid / (2 * N), l = tid % (2 * N);
  const int c = l >> 1, p = l & 1;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  C<T> *Cout = static_cast<C<T> *>(a.Cb) + ((size_t)e * a.Nr + r) * a.M * n3 + (size_t)jx * N * N;
  C<T> u1[H];
  // phase rows of the group's current direction staged in LDS, fetched one
  // direction ahead (as in the VHS gain kernel)
  const bool in_group = g < G;
  C<T> *phs = phs_all + (size_t)(in_group ? g : 0) * 4 * N;
  C<T> pf0{0, 0}, pf1{0, 0};
  auto fetch_ph = [&](int m) {
    pf0 = gload(pyz + ((size_t)r * a.M + m) * 2 * N, l);
    pf1 = gload(pyz + (((size_t)a.Nr + r) * a.M + m) * 2 * N, l);
  };
  // with one group per block the direction index is the same in every lane
  // (lanes outside the group only skip the work), so the plan tables and
  // x_plane are read through the scalar cache
  const int g0 = G == 1 ? 0 : g;
  if (in_group && g0 < a.M) fetch_ph(uload(a.morder, g0));
  const int iters = (a.M + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    const int mi = it * G + g0;
    const bool active = in_group && mi < a.M;
    const int m = mi < a.M ? uload(a.morder, mi) : 0;
    const int s = uload(a.sidx, m);
    if (active) {
      phs[l] = pf0;
      phs[2 * N + l] = pf1;
    }
    group_sync<N>();
    if (active && mi + G < a.M) fetch_ph(uload(a.morder, mi + G));
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      if (active) {
        const C<T> *src = x_plane(a, X, slot, side, r, s, n3) + (size_t)jx * N * N;
        const C<T> *ph = phs + side * 2 * N;
        const C<T> zph = ph[N + c];
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = src[(2 * n + p) * N + c];
        if constexpr (sizeof(T) == 8 && N % 4 == 0 && N >= 8) {
          col_phases_rec<T, N>(h, ph, zph, p);
        } else {
#pragma unroll
          for (int n = 0; n < H; ++n) h[n] = cmul(h[n], cmul(ph[2 * n + p], zph));
        }
        fft_pair<N, +1>(h, p);
#pragma unroll
        for (int k = 0; k < H; ++k) lds[g][p * H + k][c] = h[k];
      }
      group_sync<N>();
      if (active) {
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = lds[g][c][2 * n + p];
        fft_pair<N, +1>(h, p);
        if (side == 0) {
#pragma unroll
          for (int k = 0; k < H; ++k) u1[k] = h[k];
        } else {
          // product (natural z halves), forward z transform by decimation in
          // frequency: lane p ends with kz = 2k + p, exactly the elements of
          // row c it read above, so no other lane's data is overwritten
#pragma unroll
          for (int k = 0; k < H; ++k) h[k] = cmul(u1[k], h[k]);
          fft_pair_dif<N, -1>(h, p);
#pragma unroll
          for (int k = 0; k < H; ++k) lds[g][c][2 * k + p] = h[k];
        }
      }
      group_sync<N>();
    }
    if (active) {
      C<T> h[H];
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = lds[g][2 * n + p][c];
      fft_pair<N, -1>(h, p);
      C<T> *dst = Cout + (size_t)m * n3;
#pragma unroll
      for (int k = 0; k < H; ++k) dst[(p * H + k) * N + c] = h[k];
    }
    group_sync<N>();
  }
}

template <typename T, int N, int G>
__global__ void __launch_bounds__(G * 2 * N) k_gain_yz_vss(PipeArgs a) {
  __shared__ C<T> lds[G][N][N + 1];
  __shared__ C<T> phs[G * 4 * N];
  gain_yz_vss_body<T, N, G>(a, blockIdx.x, blockIdx.y, gain_eval(a, blockIdx.z), threadIdx.x, lds, phs);
}

template <typename T, int N, int TE>
__device__ __forceinline__ void gain_x_vss_body(const PipeArgs &a, int bx, int by, int tid) {
  constexpr int H = N / 2;
  const int pencil = bx * 32 + (tid >> 1), p = tid & 1;
  const int ngroups = (a.n_nodes + TE - 1) / TE;
  const int slot = by / ngroups, node0 = (by % ngroups) * TE;
  const bool valid = pencil < N * N;
  const int pc = valid ? pencil : 0;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int vy = wave_idx(pc / N, N), vz = wave_idx(pc % N, N), kyz = vy * vy + vz * vz;
  const C<T> *B = static_cast<const C<T> *>(pd.btab);
  // QG in FP64 in both precisions: in FP32 each table value and transform
  // are widened and their product fused-multiply-added
  C<double> Q[TE][H];
#pragma unroll
  for (int j = 0; j < TE; ++j)
#pragma unroll
    for (int k = 0; k < H; ++k) Q[j][k] = C<double>{0, 0};
  for (int rm = 0; rm < a.Nr * a.M; ++rm) {
    C<T> b[H];
    const C<T> *bl = B + (size_t)rm * n3;
#pragma unroll
    for (int k = 0; k < H; ++k) b[k] = bl[(size_t)(p * H + k) * N * N + pc];
#pragma unroll
    for (int j = 0; j < TE; ++j) {
      const int node = min(node0 + j, a.n_nodes - 1);
      const int e = node * a.n_pairs + slot;
      const C<T> *src = static_cast<const C<T> *>(a.Cb) + ((size_t)e * a.Nr * a.M + rm) * n3;
      C<T> w[H];
#pragma unroll
      for (int n = 0; n < H; ++n) w[n] = src[(size_t)(2 * n + p) * N * N + pc];
      fft_pair<N, -1>(w, p);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        if constexpr (sizeof(T) == 4) {
          const double bx = b[k].x, by = b[k].y, wx = w[k].x, wy = w[k].y;
          Q[j][k].x = __builtin_fma(bx, wx, __builtin_fma(-by, wy, Q[j][k].x));
          Q[j][k].y = __builtin_fma(bx, wy, __builtin_fma(by, wx, Q[j][k].y));
        } else {
          const C<T> t = cmul(b[k], w[k]);
          Q[j][k].x += t.x;
          Q[j][k].y += t.y;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < TE; ++j) {
    const int node = node0 + j;
    const bool live = valid && node < a.n_nodes;
    const int e = min(node, a.n_nodes - 1) * a.n_pairs + slot;
    C<T> q[H];
#pragma unroll
    for (int k = 0; k < H; ++k) q[k] = C<T>{(T)Q[j][k].x, (T)Q[j][k].y};
    fft_pair_dif<N, +1>(q, p);
    C<T> *V = static_cast<C<T> *>(a.V) + (size_t)e * 2 * n3;
    if (live) {
#pragma unroll
      for (int k = 0; k < H; ++k) V[(size_t)(2 * k + p) * N * N + pc] = q[k];
    }
    // loss: c(|k|) FFT_x Z_q, back along x
    const C<T> *Zq = static_cast<const C<T> *>(a.Z) + ((size_t)min(node, a.n_nodes - 1) * a.nz + a.zq[slot]) * n3;
#pragma unroll
    for (int n = 0; n < H; ++n) q[n] = Zq[(size_t)(2 * n + p) * N * N + pc];
    fft_pair<N, -1>(q, p);
    const T *ct = static_cast<const T *>(pd.ctab) + kyz;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int vx = wave_idx(p * H + k, N);
      q[k] = cscale(q[k], gload(ct, vx * vx));
    }
    fft_pair_dif<N, +1>(q, p);
    if (live) {
#pragma unroll
      for (int k = 0; k < H; ++k) V[n3 + (size_t)(2 * k + p) * N * N + pc] = q[k];
    }
  }
}
template <typename T, int N, int TE>
__global__ void __launch_bounds__(64) k_gain_x_vss(PipeArgs a) {
  gain_x_vss_body<T, N, TE>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}

}  // namespace dgfs
