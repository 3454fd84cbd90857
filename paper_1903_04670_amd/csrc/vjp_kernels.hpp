// Kernels of the vector-Jacobian product of Algorithm 2.
//
// With F = fft3 and iF = ifft3 (both symmetric), u = iF(wbar), W = w_r w_m b_r:
//   grad_f = beta Re F( sum_rm P1_rm * iF(u2_rm * F(W * u)) ) - beta wbar * Re iF(c * F g)
//   grad_g = beta Re F( sum_rm P2_rm * iF(u1_rm * F(W * u)) ) - beta Re F(c * iF(f * wbar))
// P1 = e^{+i th_q sigma.l}, P2 = e^{-i th_p sigma.l}; u1 = iF(P1 F f), u2 = iF(P2 F g)
// are recomputed per (r, m) from the same X arrays as the forward pipeline.
// For VHS, F(W * u) = w_m v_r with v_r = F(w_r b_r * u).
//
// Stages (arrays N^3 complex, [x][y][z]):
//   Zw   = iFFT_yz(wbar), Zfw = iFFT_yz(f * wbar)                         k_inv_yz
//   X1, X2 (as the forward), Vx_r = FFT_x(g_r(|k|) iFFT_x Zw)              k_shift_x, k_vjp_v
//   Y1_rs = sum_{m: s(m)=s} P1yz_rm iFFT_yz(w_m u2_rm v_r)  (plane jx)     k_vjp_yz
//   Y2_rs = sum_{m: s(m)=s} P2yz_rm iFFT_yz(w_m u1_rm v_r)
//   Hf = FFT_x(sum_rs P1x_rs iFFT_x Y1_rs / N^3)                           k_vjp_x
//   Hg = FFT_x(sum_rs P2x_rs iFFT_x Y2_rs / N^3 - c iFFT_x Zfw / N^3)
//   Vf = iFFT_x(c FFT_x Z_g) / N^3
//   grad_f = beta (Re FFT_yz Hf - wbar Re iFFT_yz Vf), grad_g = beta Re FFT_yz Hg   k_vjp_final
#pragma once
#include "collide_kernels.hpp"

namespace dgfs {

struct VjpArgs {
  PipeArgs a;           // n_pairs = 1, nz = 2 (Z slots f, g), Z/X as the forward pipeline
  void *Zw;             // [node][2][N^3] : iFFT_yz(wbar), iFFT_yz(f wbar)
  void *Vx;             // [e][Nr][N^3]
  void *Y;              // [e][2][Nr][Sx][N^3]
  void *H;              // [e][3][N^3] : Hf, Hg, Vf
  const double *f, *w;  // f^p and wbar of node n at + n*f_stride / + n*w_stride
  int64_t f_stride, w_stride;
  double *gf, *gg;      // outputs (may be NULL), node n at + n*g_stride
  int64_t g_stride;
  int accumulate;
};

// iFFT_yz of wbar and of f*wbar on plane jx of each node (rows first through
// LDS, then columns written coalesced).
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_inv_yz(VjpArgs v) {
  __shared__ C<T> lds[G][N][N + 1];
  const int g = threadIdx.x / N, t = threadIdx.x % N;
  const int plane = blockIdx.x * G + g;
  const int jobs = N * v.a.n_nodes * 2;
  const bool active = plane < jobs;
  const int jx = plane % N, job = plane / N, node = job / 2, which = job % 2;
  const size_t n3 = (size_t)N * N * N;
  if (active) {
    const double *w = v.w + (size_t)node * v.w_stride + (size_t)jx * N * N;
    const double *f = v.f + (size_t)node * v.f_stride + (size_t)jx * N * N;
    for (int i = t; i < N * N; i += N) lds[g][i / N][i % N] = C<T>{(T)(which ? f[i] * w[i] : w[i]), (T)0};
  }
  __syncthreads();
  if (active) {
    C<T> row[N];
#pragma unroll
    for (int z = 0; z < N; ++z) row[z] = lds[g][t][z];
    fft<N, +1>(row);
#pragma unroll
    for (int z = 0; z < N; ++z) lds[g][t][z] = row[z];
  }
  __syncthreads();
  if (active) {
    C<T> col[N];
#pragma unroll
    for (int y = 0; y < N; ++y) col[y] = lds[g][y][t];
    fft<N, +1>(col);
    C<T> *Z = static_cast<C<T> *>(v.Zw) + ((size_t)node * 2 + which) * n3 + (size_t)jx * N * N;
#pragma unroll
    for (int y = 0; y < N; ++y) Z[y * N + t] = col[y];
  }
}

// Vx_r = FFT_x(g_r(|k|) iFFT_x Zw) for every r; thread = x-line.
template <typename T, int N>
__global__ void __launch_bounds__(64) k_vjp_v(VjpArgs v) {
  const PipeArgs &a = v.a;
  const int pencil = blockIdx.x * 64 + threadIdx.x;
  const int e = blockIdx.y;
  if (pencil >= N * N) return;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int K2 = 3 * (N / 2) * (N / 2) + 1;
  const int vy = wave_idx(pencil / N, N), vz = wave_idx(pencil % N, N), kyz = vy * vy + vz * vz;
  const C<T> *Zw = static_cast<const C<T> *>(v.Zw) + (size_t)node * 2 * n3;
  C<T> U[N];
#pragma unroll
  for (int x = 0; x < N; ++x) U[x] = Zw[(size_t)x * N * N + pencil];
  fft<N, +1>(U);
  const T *gt = static_cast<const T *>(pd.gtab);
  C<T> *Vx = static_cast<C<T> *>(v.Vx) + (size_t)e * a.Nr * n3;
  for (int r = 0; r < a.Nr; ++r) {
    const T *gr = gt + (size_t)r * K2 + kyz;
    C<T> w[N];
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int vx = wave_idx(x, N);
      w[x] = cscale(U[x], gr[vx * vx]);
    }
    fft<N, -1>(w);
#pragma unroll
    for (int x = 0; x < N; ++x) Vx[(size_t)r * n3 + (size_t)x * N * N + pencil] = w[x];
  }
}

// Plane (e, r, jx): v = FFT_yz(Vx_r) kept in LDS; for each distinct sigma_x
// value s and each side, accumulate Y_side[r][s] over the directions m with
// s(m) = s.  Thread t: column z = t (y passes), row y = t (z passes).
template <typename T, int N>
__global__ void __launch_bounds__(N) k_vjp_yz(VjpArgs v) {
  const PipeArgs &a = v.a;
  __shared__ C<T> vl[N][N + 1];
  __shared__ C<T> lds[N][N + 1];
  const int t = threadIdx.x;
  const int jx = blockIdx.x, r = blockIdx.y, e = blockIdx.z;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  // v_r on this plane: column FFT_y, then row FFT_z, rows stay in vl
  {
    const C<T> *src = static_cast<const C<T> *>(v.Vx) + ((size_t)e * a.Nr + r) * n3 + (size_t)jx * N * N;
    C<T> col[N];
#pragma unroll
    for (int y = 0; y < N; ++y) col[y] = src[y * N + t];
    fft<N, -1>(col);
#pragma unroll
    for (int y = 0; y < N; ++y) vl[y][t] = col[y];
    __syncthreads();
    C<T> row[N];
#pragma unroll
    for (int z = 0; z < N; ++z) row[z] = vl[t][z];
    fft<N, -1>(row);
#pragma unroll
    for (int z = 0; z < N; ++z) vl[t][z] = row[z];
    __syncthreads();
  }
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  C<T> *Y = static_cast<C<T> *>(v.Y) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  for (int s = 0; s < a.Sx; ++s) {
    for (int side = 0; side < 2; ++side) {
      // side 0 accumulates Y1 = sum P1yz iFFT_yz(w u2 v): needs u2 (X side 1)
      // side 1 accumulates Y2 = sum P2yz iFFT_yz(w u1 v): needs u1 (X side 0)
      const int uside = 1 - side;
      C<T> acc[N];
#pragma unroll
      for (int y = 0; y < N; ++y) acc[y] = C<T>{0, 0};
      for (int m = 0; m < a.M; ++m) {
        if (a.sidx[m] != s) continue;
        // u (row y = t) from X_uside with the yz phases of direction m
        {
          const C<T> *src = x_plane(a, X, e % a.n_pairs, uside, r, s, n3) + (size_t)jx * N * N;
          const C<T> *ph = pyz + (((size_t)uside * a.Nr + r) * a.M + m) * 2 * N;
          const C<T> zph = ph[N + t];
          C<T> col[N];
#pragma unroll
          for (int y = 0; y < N; ++y) col[y] = cmul(src[y * N + t], cmul(ph[y], zph));
          fft<N, +1>(col);
#pragma unroll
          for (int y = 0; y < N; ++y) lds[y][t] = col[y];
        }
        __syncthreads();
        {
          C<T> row[N];
          const T w = wm[m];
#pragma unroll
          for (int z = 0; z < N; ++z) row[z] = lds[t][z];
          fft<N, +1>(row);  // u row
#pragma unroll
          for (int z = 0; z < N; ++z) row[z] = cscale(cmul(row[z], vl[t][z]), w);
          fft<N, +1>(row);  // iFFT_z of the product
#pragma unroll
          for (int z = 0; z < N; ++z) lds[t][z] = row[z];
        }
        __syncthreads();
        {
          C<T> col[N];
#pragma unroll
          for (int y = 0; y < N; ++y) col[y] = lds[y][t];
          fft<N, +1>(col);
          const C<T> *ph = pyz + (((size_t)side * a.Nr + r) * a.M + m) * 2 * N;
          const C<T> zph = ph[N + t];
#pragma unroll
          for (int y = 0; y < N; ++y) acc[y] = cadd(acc[y], cmul(col[y], cmul(ph[y], zph)));
        }
        __syncthreads();
      }
      C<T> *dst = Y + (((size_t)side * a.Nr + r) * a.Sx + s) * n3 + (size_t)jx * N * N;
#pragma unroll
      for (int y = 0; y < N; ++y) dst[y * N + t] = acc[y];
    }
  }
}

// Thread = x-line: Hf, Hg (with the g-side loss), Vf.
template <typename T, int N>
__global__ void __launch_bounds__(64) k_vjp_x(VjpArgs v) {
  const PipeArgs &a = v.a;
  const int pencil = blockIdx.x * 64 + threadIdx.x;
  const int e = blockIdx.y;
  if (pencil >= N * N) return;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int vy = wave_idx(pencil / N, N), vz = wave_idx(pencil % N, N), kyz = vy * vy + vz * vz;
  const C<T> *Y = static_cast<const C<T> *>(v.Y) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  C<T> *H = static_cast<C<T> *>(v.H) + (size_t)e * 3 * n3;
  const T *ct = static_cast<const T *>(pd.ctab) + kyz;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const C<T> *px = static_cast<const C<T> *>(pd.px) + (size_t)side * a.Nr * a.Sx * N;
    C<T> G[N];
#pragma unroll
    for (int x = 0; x < N; ++x) G[x] = C<T>{0, 0};
    for (int rs = 0; rs < a.Nr * a.Sx; ++rs) {
      const C<T> *src = Y + ((size_t)side * a.Nr * a.Sx + rs) * n3;
      C<T> w[N];
#pragma unroll
      for (int x = 0; x < N; ++x) w[x] = src[(size_t)x * N * N + pencil];
      fft<N, +1>(w);
      const C<T> *ph = px + (size_t)rs * N;
#pragma unroll
      for (int x = 0; x < N; ++x) G[x] = cadd(G[x], cmul(w[x], ph[x]));
    }
    if (side == 1) {  // minus c(|k|) iFFT_x(Zfw) / N^3
      const C<T> *Zfw = static_cast<const C<T> *>(v.Zw) + ((size_t)node * 2 + 1) * n3;
      C<T> w[N];
#pragma unroll
      for (int x = 0; x < N; ++x) w[x] = Zfw[(size_t)x * N * N + pencil];
      fft<N, +1>(w);
#pragma unroll
      for (int x = 0; x < N; ++x) {
        const int vx = wave_idx(x, N);
        G[x] = csub(G[x], cscale(w[x], ct[vx * vx]));
      }
    }
    fft<N, -1>(G);
#pragma unroll
    for (int x = 0; x < N; ++x) H[(size_t)side * n3 + (size_t)x * N * N + pencil] = G[x];
  }
  // Vf = iFFT_x(c FFT_x Z_g) / N^3
  const C<T> *Zg = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + a.zq[slot]) * n3;
  C<T> w[N];
#pragma unroll
  for (int x = 0; x < N; ++x) w[x] = Zg[(size_t)x * N * N + pencil];
  fft<N, -1>(w);
#pragma unroll
  for (int x = 0; x < N; ++x) {
    const int vx = wave_idx(x, N);
    w[x] = cscale(w[x], ct[vx * vx]);
  }
  fft<N, +1>(w);
#pragma unroll
  for (int x = 0; x < N; ++x) H[2 * n3 + (size_t)x * N * N + pencil] = w[x];
}

// Plane (e, jx): grad_f = beta (Re FFT_yz Hf - wbar Re iFFT_yz Vf),
// grad_g = beta Re FFT_yz Hg.  Rows via LDS, then columns (coalesced output).
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_vjp_final(VjpArgs v) {
  const PipeArgs &a = v.a;
  __shared__ C<T> lds[G][N][N + 1];
  const int g = threadIdx.x / N, t = threadIdx.x % N;
  const int plane = blockIdx.x * G + g;
  const int jobs = N * a.n_nodes;
  const bool active = plane < jobs;
  const int jx = plane % N, node = plane / N;
  const int e = node * a.n_pairs;
  const size_t n3 = (size_t)N * N * N;
  const double beta = a.pairs[a.pair_id[0]].beta;
  double res[N];
#pragma unroll
  for (int which = 0; which < 3; ++which) {
    if (active) {
      const C<T> *src = static_cast<const C<T> *>(v.H) + ((size_t)e * 3 + which) * n3 + (size_t)jx * N * N;
      for (int i = t; i < N * N; i += N) lds[g][i / N][i % N] = src[i];
    }
    __syncthreads();
    if (active) {
      C<T> row[N];
#pragma unroll
      for (int z = 0; z < N; ++z) row[z] = lds[g][t][z];
      if (which == 2) fft<N, +1>(row);
      else fft<N, -1>(row);
#pragma unroll
      for (int z = 0; z < N; ++z) lds[g][t][z] = row[z];
    }
    __syncthreads();
    if (active) {
      C<T> col[N];
#pragma unroll
      for (int y = 0; y < N; ++y) col[y] = lds[g][y][t];
      if (which == 2) fft<N, +1>(col);
      else fft<N, -1>(col);
      if (which == 0) {
#pragma unroll
        for (int y = 0; y < N; ++y) res[y] = beta * (double)col[y].x;
      } else if (which == 1) {
        if (v.gg) {
          double *o = v.gg + (size_t)node * v.g_stride + (size_t)jx * N * N;
#pragma unroll
          for (int y = 0; y < N; ++y) {
            const double val = beta * (double)col[y].x;
            if (v.accumulate) o[y * N + t] += val;
            else o[y * N + t] = val;
          }
        }
      } else if (v.gf) {
        const double *w = v.w + (size_t)node * v.w_stride + (size_t)jx * N * N;
        double *o = v.gf + (size_t)node * v.g_stride + (size_t)jx * N * N;
#pragma unroll
        for (int y = 0; y < N; ++y) {
          const double val = res[y] - beta * w[y * N + t] * (double)col[y].x;
          if (v.accumulate) o[y * N + t] += val;
          else o[y * N + t] = val;
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace dgfs
