// Kernels of the fast spectral collision pipeline (Algorithm 2) for one
// compute type T and one compile-time grid size N.
//
// Data flow per evaluation e = (node, ordered pair p,q), arrays of N^3
// complex values indexed [x][y][z] (z fastest):
//   Z_s   = FFT_yz(f^s)                                         k_fwd_yz
//   X1_rs = iFFT_x(e^{+i th_q s_x v_x} FFT_x Z_p) / N^3           k_shift_x
//   X2_rs = iFFT_x(e^{-i th_p s_x v_x} FFT_x Z_q) / N^3
//           (one per distinct x component s_x of the sphere set)
//   C_r   = FFT_yz( sum_m w_m u1_rm u2_rm ),                      k_gain_yz
//           u1_rm = iFFT_yz(e^{+i th_q (s_y v_y + s_z v_z)} X1_{r s(m)}), u2 likewise
//   V1    = iFFT_x( sum_r g_r(|k|) FFT_x C_r ),   V2 = iFFT_x(c(|k|) FFT_x Z_q)   k_gain_x
//   Q     = beta Re( iFFT_yz V1 - f^p iFFT_yz V2 )                 k_final_yz
// With the 1/N^3 factors folded into the phase and kernel tables, u1 and u2
// are the translated distribution functions of Algorithm 2 (ifft(t1),
// ifft(t2)), sum_r g_r FFT_x C_r is its QG, and V1, V2 are partial inverse
// transforms of QG and c*FTg.  Because the VHS gain table depends on |k| and
// r only, the sum over m is taken before the forward transform (an exact
// reordering of the quadrature sum).
//
// Thread layouts: pencil kernels give one x-line (fixed y, z) to each thread;
// plane kernels give one column (fixed z, varying y) to a thread, read and
// written coalesced, and transpose through LDS for the row (z) transforms.
#pragma once
#include "fft.hpp"
#include "internal.hpp"

namespace dgfs {

template <typename T> using C = cplx<T>;

struct PipeArgs {
  int Nr, Sx, M, ns;
  int n_nodes;   // nodes in this chunk
  int n_pairs;   // pair slots per node
  int nz;        // Z slots per node
  int pair_id[kMaxPairs];
  int zp[kMaxPairs], zq[kMaxPairs];
  const PairDev *pairs;
  const void *wm;
  const int *sidx;
  void *Z, *X, *Cb, *V;
};

struct FwdArgs {
  const double *src[DGFS_MAX_SPECIES];  // per Z slot: block of node n at src + n*node_stride
  int64_t node_stride;
  int n_nodes, nz;
  void *Z;
};

struct FinalArgs {
  int n_out, qcount;             // outputs per node; pair slots summed per output
  const double *fsrc[DGFS_MAX_SPECIES];  // f^p of output o at fsrc[o] + n*f_stride
  int64_t f_stride;
  double *out[DGFS_MAX_SPECIES];  // output o of node n at out[o] + n*out_stride
  int64_t out_stride;
  int accumulate;
};

__device__ __forceinline__ int wave_idx(int j, int N) { return j < N / 2 ? j : j - N; }

// Neumaier-compensated accumulation (used by the FP32 path).
template <typename T> struct Acc {
  T s, c;
};
template <typename T> __device__ __forceinline__ void acc_add(T &s, T &c, T x) {
  T t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// ------------------------------------------------------------------ k_fwd_yz
// One (node, slot, x-plane) per group of N threads; G planes per block.
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_fwd_yz(FwdArgs a) {
  __shared__ C<T> lds[G][N][N + 1];
  const int g = threadIdx.x / N, t = threadIdx.x % N;
  const int plane = blockIdx.x * G + g;   // over N x-planes * n_nodes * nz
  const int jobs = N * a.n_nodes * a.nz;
  const bool active = plane < jobs;
  const int jx = plane % N, job = plane / N;
  const int node = job / a.nz, slot = job % a.nz;
  const size_t n3 = (size_t)N * N * N;
  if (active) {
    const double *f = a.src[slot] + (size_t)node * a.node_stride + (size_t)jx * N * N;
    // stage the real plane: element (y, z) -> lds[y][z]
    for (int i = t; i < N * N; i += N) lds[g][i / N][i % N] = C<T>{(T)f[i], (T)0};
  }
  __syncthreads();
  if (active) {
    C<T> row[N];
#pragma unroll
    for (int z = 0; z < N; ++z) row[z] = lds[g][t][z];
    fft<N, -1>(row);
#pragma unroll
    for (int z = 0; z < N; ++z) lds[g][t][z] = row[z];
  }
  __syncthreads();
  if (active) {
    C<T> col[N];
#pragma unroll
    for (int y = 0; y < N; ++y) col[y] = lds[g][y][t];
    fft<N, -1>(col);
    C<T> *Z = static_cast<C<T> *>(a.Z) + (size_t)job * n3 + (size_t)jx * N * N;
#pragma unroll
    for (int y = 0; y < N; ++y) Z[y * N + t] = col[y];
  }
}

// ------------------------------------------------------------------ k_shift_x
// Thread = x-line (y, z) of one (eval, side); loops over r and the distinct
// sigma_x values.
template <typename T, int N>
__global__ void __launch_bounds__(64) k_shift_x(PipeArgs a) {
  const int pencil = blockIdx.x * 64 + threadIdx.x;
  const int side = blockIdx.y;
  const int e = blockIdx.z;
  if (pencil >= N * N) return;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int zs = side == 0 ? a.zp[slot] : a.zq[slot];
  const C<T> *Z = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + zs) * n3;
  C<T> F[N];
#pragma unroll
  for (int x = 0; x < N; ++x) F[x] = Z[(size_t)x * N * N + pencil];
  fft<N, -1>(F);
  const C<T> *px = static_cast<const C<T> *>(pd.px) + (size_t)side * a.Nr * a.Sx * N;
  C<T> *X = static_cast<C<T> *>(a.X) + ((size_t)e * 2 + side) * a.Nr * a.Sx * n3;
  for (int rs = 0; rs < a.Nr * a.Sx; ++rs) {
    const C<T> *ph = px + (size_t)rs * N;
    C<T> w[N];
#pragma unroll
    for (int x = 0; x < N; ++x) w[x] = cmul(F[x], ph[x]);
    fft<N, +1>(w);
    C<T> *dst = X + (size_t)rs * n3;
#pragma unroll
    for (int x = 0; x < N; ++x) dst[(size_t)x * N * N + pencil] = w[x];
  }
}

// ------------------------------------------------------------------ k_gain_yz
// Block = G groups of N threads on one (eval, r, x-plane); group g takes the
// directions m = g, g+G, ...  Thread t owns column z = t in the y pass and row
// y = t in the z pass, product and accumulation.
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_gain_yz(PipeArgs a) {
  __shared__ C<T> lds[G][N][N + 1];
  const int g = threadIdx.x / N, t = threadIdx.x % N;
  const int jx = blockIdx.x, r = blockIdx.y, e = blockIdx.z;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  C<T> P[N], Pc[N], u1[N];
#pragma unroll
  for (int z = 0; z < N; ++z) P[z] = Pc[z] = C<T>{0, 0};
  const int iters = (a.M + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    const int m = it * G + g;
    const bool active = m < a.M;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (active) {
        const int s = a.sidx[m];
        const C<T> *src = X + (((size_t)side * a.Nr + r) * a.Sx + s) * n3 + (size_t)jx * N * N;
        const C<T> *ph = pyz + (((size_t)side * a.Nr + r) * a.M + m) * 2 * N;
        const C<T> zph = ph[N + t];
        C<T> col[N];
#pragma unroll
        for (int y = 0; y < N; ++y) col[y] = cmul(src[y * N + t], cmul(ph[y], zph));
        fft<N, +1>(col);
#pragma unroll
        for (int y = 0; y < N; ++y) lds[g][y][t] = col[y];
      }
      __syncthreads();
      if (active) {
        C<T> row[N];
#pragma unroll
        for (int z = 0; z < N; ++z) row[z] = lds[g][t][z];
        fft<N, +1>(row);
        if (side == 0) {
#pragma unroll
          for (int z = 0; z < N; ++z) u1[z] = row[z];
        } else {
          const T w = wm[m];
#pragma unroll
          for (int z = 0; z < N; ++z) {
            C<T> pr = cmul(u1[z], row[z]);
            if constexpr (sizeof(T) == 4) {
              acc_add(P[z].x, Pc[z].x, w * pr.x);
              acc_add(P[z].y, Pc[z].y, w * pr.y);
            } else {
              P[z].x += w * pr.x;
              P[z].y += w * pr.y;
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // combine the groups' partial sums in group order, then FFT_yz
  if constexpr (G > 1) {
    if (g > 0) {
#pragma unroll
      for (int z = 0; z < N; ++z) lds[g][t][z] = C<T>{P[z].x + Pc[z].x, P[z].y + Pc[z].y};
    }
    __syncthreads();
    if (g == 0) {
#pragma unroll
      for (int z = 0; z < N; ++z) {
        T sx = P[z].x, cx = Pc[z].x, sy = P[z].y, cy = Pc[z].y;
        for (int h = 1; h < G; ++h) {
          C<T> v = lds[h][t][z];
          if constexpr (sizeof(T) == 4) {
            acc_add(sx, cx, v.x);
            acc_add(sy, cy, v.y);
          } else {
            sx += v.x;
            sy += v.y;
          }
        }
        P[z] = C<T>{sx, sy};
        Pc[z] = C<T>{cx, cy};
      }
    }
    __syncthreads();
  }
  if (g == 0) {
#pragma unroll
    for (int z = 0; z < N; ++z) P[z] = C<T>{P[z].x + Pc[z].x, P[z].y + Pc[z].y};
    fft<N, -1>(P);
#pragma unroll
    for (int z = 0; z < N; ++z) lds[0][t][z] = P[z];
  }
  __syncthreads();
  if (g == 0) {
    C<T> col[N];
#pragma unroll
    for (int y = 0; y < N; ++y) col[y] = lds[0][y][t];
    fft<N, -1>(col);
    C<T> *dst = static_cast<C<T> *>(a.Cb) + ((size_t)e * a.Nr + r) * n3 + (size_t)jx * N * N;
#pragma unroll
    for (int y = 0; y < N; ++y) dst[y * N + t] = col[y];
  }
}

// ------------------------------------------------------------------ k_gain_x
// Thread = x-line (y, z) of one eval: QG = sum_r g_r(|k|) FFT_x C_r, then
// V1 = iFFT_x QG and V2 = iFFT_x(c(|k|) FFT_x Z_q).
template <typename T, int N>
__global__ void __launch_bounds__(64) k_gain_x(PipeArgs a) {
  const int pencil = blockIdx.x * 64 + threadIdx.x;
  const int e = blockIdx.y;
  if (pencil >= N * N) return;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int K2 = 3 * (N / 2) * (N / 2) + 1;
  const int vy = wave_idx(pencil / N, N), vz = wave_idx(pencil % N, N);
  const int kyz = vy * vy + vz * vz;
  const T *gt = static_cast<const T *>(pd.gtab);
  const C<T> *Cb = static_cast<const C<T> *>(a.Cb) + (size_t)e * a.Nr * n3;
  C<T> Q[N], Qc[N];
#pragma unroll
  for (int x = 0; x < N; ++x) Q[x] = Qc[x] = C<T>{0, 0};
  for (int r = 0; r < a.Nr; ++r) {
    C<T> w[N];
    const C<T> *src = Cb + (size_t)r * n3;
#pragma unroll
    for (int x = 0; x < N; ++x) w[x] = src[(size_t)x * N * N + pencil];
    fft<N, -1>(w);
    const T *g = gt + (size_t)r * K2 + kyz;
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int vx = wave_idx(x, N);
      const T gv = g[vx * vx];
      if constexpr (sizeof(T) == 4) {
        acc_add(Q[x].x, Qc[x].x, gv * w[x].x);
        acc_add(Q[x].y, Qc[x].y, gv * w[x].y);
      } else {
        Q[x].x += gv * w[x].x;
        Q[x].y += gv * w[x].y;
      }
    }
  }
#pragma unroll
  for (int x = 0; x < N; ++x) Q[x] = C<T>{Q[x].x + Qc[x].x, Q[x].y + Qc[x].y};
  fft<N, +1>(Q);
  C<T> *V = static_cast<C<T> *>(a.V) + (size_t)e * 2 * n3;
#pragma unroll
  for (int x = 0; x < N; ++x) V[(size_t)x * N * N + pencil] = Q[x];
  // loss: c(|k|) * FFT_x Z_q, back along x
  const C<T> *Zq = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + a.zq[slot]) * n3;
#pragma unroll
  for (int x = 0; x < N; ++x) Q[x] = Zq[(size_t)x * N * N + pencil];
  fft<N, -1>(Q);
  const T *ct = static_cast<const T *>(pd.ctab) + kyz;
#pragma unroll
  for (int x = 0; x < N; ++x) {
    const int vx = wave_idx(x, N);
    Q[x] = cscale(Q[x], ct[vx * vx]);
  }
  fft<N, +1>(Q);
#pragma unroll
  for (int x = 0; x < N; ++x) V[n3 + (size_t)x * N * N + pencil] = Q[x];
}

// ------------------------------------------------------------------ k_final_yz
// One (node, output, x-plane) per group: Q = sum over the output's pair slots
// of beta Re(iFFT_yz V1 - f^p iFFT_yz V2).  Rows first (staged through LDS),
// then columns so the output and f^p are accessed coalesced.
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_final_yz(PipeArgs a, FinalArgs fa) {
  __shared__ C<T> lds[G][N][N + 1];
  const int g = threadIdx.x / N, t = threadIdx.x % N;
  const int plane = blockIdx.x * G + g;
  const int jobs = N * a.n_nodes * fa.n_out;
  const bool active = plane < jobs;
  const int jx = plane % N, job = plane / N;
  const int node = job / fa.n_out, o = job % fa.n_out;
  const size_t n3 = (size_t)N * N * N;
  double acc[N];
#pragma unroll
  for (int y = 0; y < N; ++y) acc[y] = 0.0;
  const double *f = active ? fa.fsrc[o] + (size_t)node * fa.f_stride + (size_t)jx * N * N : nullptr;
  for (int j = 0; j < fa.qcount; ++j) {
    const int slot = o * fa.qcount + j;
    const int e = node * a.n_pairs + slot;
    const double beta = a.pairs[a.pair_id[slot]].beta;
#pragma unroll
    for (int which = 0; which < 2; ++which) {
      if (active) {
        const C<T> *src = static_cast<const C<T> *>(a.V) + ((size_t)e * 2 + which) * n3 + (size_t)jx * N * N;
        for (int i = t; i < N * N; i += N) lds[g][i / N][i % N] = src[i];
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
        // gain part, then the loss part f^p * Re(ifft(c FTg))
        if (which == 0) {
#pragma unroll
          for (int y = 0; y < N; ++y) acc[y] += beta * (double)col[y].x;
        } else {
#pragma unroll
          for (int y = 0; y < N; ++y) acc[y] -= beta * f[y * N + t] * (double)col[y].x;
        }
      }
      __syncthreads();
    }
  }
  if (active) {
    double *out = fa.out[o] + (size_t)node * fa.out_stride + (size_t)jx * N * N;
#pragma unroll
    for (int y = 0; y < N; ++y) {
      if (fa.accumulate) out[y * N + t] += acc[y];
      else out[y * N + t] = acc[y];
    }
  }
}

}  // namespace dgfs
