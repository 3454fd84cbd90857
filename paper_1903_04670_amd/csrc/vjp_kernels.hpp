// Kernels of the vector-Jacobian product of Algorithm 2.
//
// With F = fft3 and iF = ifft3 (both symmetric), u = iF(wbar), W = w_r w_m b_r:
//   grad_f = beta Re F( sum_rm P1_rm * iF(u2_rm * F(W * u)) ) - beta wbar * Re iF(c * F g)
//   grad_g = beta Re F( sum_rm P2_rm * iF(u1_rm * F(W * u)) ) - beta Re F(c * iF(f * wbar))
// P1 = e^{+i th_q sigma.l}, P2 = e^{-i th_p sigma.l}; u1 = iF(P1 F f), u2 = iF(P2 F g)
// are recomputed per (r, m) from the same X arrays as the forward pipeline.
// For VHS, F(W * u) = w_m v_r with v_r = F(w_r b_r * u); for VSS the table
// depends on the direction and v_rm = F(w_r w_m b_rm * u) is formed per term.
//
// Stages (arrays N^3 complex, [x][y][z]):
//   Zw   = iFFT_yz(wbar), Zfw = iFFT_yz(f * wbar)                         k_inv_yz
//   X1, X2 (as the forward), Vx_r = FFT_x(g_r(|k|) iFFT_x Zw)              k_shift_x, k_vjp_v
//     (VSS: Vx_rm = FFT_x(b_rm(k) iFFT_x Zw), b_rm carrying w_r w_m / N^3)
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
  const int *sched;     // [G][sched_T] term schedule of k_vjp_yz (m | side << 16 | last << 17, or -1)
  int sched_T;
  int sym;              // 1: the two sides' gain sums coincide; only side 0's Y is formed
  int vss;              // 1: direction-dependent table, Vx is [e][Nr][M][N^3]
  int nyq;              // 1: the plan's twiddle rows have zeroed Nyquist entries
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

// Vx_r = FFT_x(g_r(|k|) iFFT_x Zw) for every r (VSS: Vx_rm with the complex
// table b_rm(k) for every (r, m)).  Lane pair (pencil, p) = x-line (y, z):
// iFFT_x of the decimated half x = 2n + p gives wave numbers pH + k; after
// the table multiply a decimation-in-frequency FFT_x returns to x = 2k + p.
template <typename T, int N, bool VSS = false>
__global__ void __launch_bounds__(64) k_vjp_v(VjpArgs v) {
  constexpr int H = N / 2;
  const PipeArgs &a = v.a;
  const int pencil = blockIdx.x * 32 + (threadIdx.x >> 1), p = threadIdx.x & 1;
  const bool valid = pencil < N * N;
  const int pc = valid ? pencil : 0;  // idle lanes still take part in the lane swaps
  const int e = blockIdx.y;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int K2 = 3 * (N / 2) * (N / 2) + 1;
  const int vy = wave_idx(pc / N, N), vz = wave_idx(pc % N, N), kyz = vy * vy + vz * vz;
  const C<T> *Zw = static_cast<const C<T> *>(v.Zw) + (size_t)node * 2 * n3;
  C<T> U[H];
#pragma unroll
  for (int n = 0; n < H; ++n) U[n] = Zw[(size_t)(2 * n + p) * N * N + pc];
  fft_pair<N, +1>(U, p);
  if constexpr (VSS) {
    const C<T> *B = static_cast<const C<T> *>(pd.btab);  // [Nr][M][N^3], natural wave order
    C<T> *Vx = static_cast<C<T> *>(v.Vx) + (size_t)e * a.Nr * a.M * n3;
    for (int rm = 0; rm < a.Nr * a.M; ++rm) {
      const C<T> *bl = B + (size_t)rm * n3;
      C<T> w[H];
#pragma unroll
      for (int k = 0; k < H; ++k) w[k] = cmul(U[k], bl[(size_t)(p * H + k) * N * N + pc]);
      fft_pair_dif<N, -1>(w, p);
      if (valid) {
#pragma unroll
        for (int k = 0; k < H; ++k) Vx[(size_t)rm * n3 + (size_t)(2 * k + p) * N * N + pc] = w[k];
      }
    }
    return;
  }
  const T *gt = static_cast<const T *>(pd.gtab);
  C<T> *Vx = static_cast<C<T> *>(v.Vx) + (size_t)e * a.Nr * n3;
  for (int r = 0; r < a.Nr; ++r) {
    const T *gr = gt + (size_t)r * K2 + kyz;
    C<T> w[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int vx = wave_idx(p * H + k, N);
      w[k] = cscale(U[k], gload(gr, vx * vx));
    }
    fft_pair_dif<N, -1>(w, p);
    if (valid) {
#pragma unroll
      for (int k = 0; k < H; ++k) Vx[(size_t)r * n3 + (size_t)(2 * k + p) * N * N + pc] = w[k];
    }
  }
}

// Plane (e, r, jx), G groups of 2N threads; every length-N pencil is split
// over a lane pair (c, p) as in the forward gain kernel.  Each group first
// forms v = FFT_yz(Vx_r) on the plane (row y = c, z = pH + k in registers),
// then works through its list of terms (m, side): u from X of the other
// side (column pass: phases, iFFT_y, to LDS; row pass: iFFT_z), the product
// w_m u v, iFFT_z back into the same LDS slots, iFFT_y of the columns, the
// yz phases of `side`, and accumulation; the last term of a (sigma_x group,
// side) unit writes Y_side[r][s] for the plane.
// SCALAR = false for plans whose twiddle tables have zeroed Nyquist entries
// (the scalar-phase identities of the N = 32 path do not hold for them).
// VSS: each term forms its own v_rm on the plane (two more passes through
// the group's LDS plane), and w_m is already in the table.
template <typename T, int N, int G, bool SCALAR = true, bool VSS = false>
__global__ void __launch_bounds__(G * 2 * N) k_vjp_yz(VjpArgs v) {
  constexpr int H = N / 2;
  const PipeArgs &a = v.a;
  __shared__ C<T> lds[G][N][N + 1];
  const int tid = threadIdx.x, g = tid / (2 * N), l = tid % (2 * N);
  const int c = l >> 1, p = l & 1;
  const int jx = blockIdx.x, r = blockIdx.y, e = blockIdx.z;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  C<T>(*buf)[N + 1] = lds[g < G ? g : 0];
  const bool in_group = g < G;
  C<T> vr[H];
  // v = FFT_yz of the Vx array `arr` on this plane: row y = c, z = pH + k
  auto form_v = [&](bool on, size_t arr) {
    const C<T> *src = static_cast<const C<T> *>(v.Vx) + arr * n3 + (size_t)jx * N * N;
    C<T> h[H];
    if (on) {
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = src[(2 * n + p) * N + c];
      fft_pair<N, -1>(h, p);
#pragma unroll
      for (int k = 0; k < H; ++k) buf[p * H + k][c] = h[k];
    }
    group_sync<N>();
    if (on) {
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = buf[c][2 * n + p];
      fft_pair<N, -1>(h, p);
#pragma unroll
      for (int k = 0; k < H; ++k) vr[k] = h[k];
    }
    group_sync<N>();
  };
  if constexpr (!VSS) form_v(in_group, (size_t)e * a.Nr + r);
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  C<T> *Y = static_cast<C<T> *>(v.Y) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  C<T> acc[H];
#pragma unroll
  for (int k = 0; k < H; ++k) acc[k] = C<T>{0, 0};
  const int *sched = v.sched + (in_group ? g : 0) * v.sched_T;
  for (int t = 0; t < v.sched_T; ++t) {
    const int ent = in_group ? uload(sched, t) : -1;
    const bool active = ent >= 0;
    const int m = active ? (ent & 0xffff) : 0;
    const int side = (ent >> 16) & 1, uside = 1 - side;
    const int s = uload(a.sidx, m);
    if constexpr (VSS) form_v(active, ((size_t)e * a.Nr + r) * a.M + m);
    if (active) {
      const C<T> *src = x_plane(a, X, slot, uside, r, s, n3) + (size_t)jx * N * N;
      C<T> h[H];
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = src[(2 * n + p) * N + c];
      apply_col_phase<T, N, SCALAR>(h, pyz + (((size_t)uside * a.Nr + r) * a.M + m) * 2 * N, c, p);
      fft_pair<N, +1>(h, p);
#pragma unroll
      for (int k = 0; k < H; ++k) buf[p * H + k][c] = h[k];
    }
    group_sync<N>();
    if (active) {
      C<T> h[H];
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = buf[c][2 * n + p];
      fft_pair<N, +1>(h, p);  // u on row y = c, z = pH + k
      const T w = VSS ? (T)1 : uload(wm, m);
#pragma unroll
      for (int k = 0; k < H; ++k) h[k] = cscale(cmul(h[k], vr[k]), w);
      fft_pair_dif<N, +1>(h, p);  // iFFT_z of the product: z = 2k + p
#pragma unroll
      for (int k = 0; k < H; ++k) buf[c][2 * k + p] = h[k];  // the slots this lane read
    }
    group_sync<N>();
    if (active) {
      C<T> h[H];
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = buf[2 * n + p][c];
      fft_pair<N, +1>(h, p);  // column z = c, y = pH + k
      const C<T> *ph = pyz + (((size_t)side * a.Nr + r) * a.M + m) * 2 * N;
      const C<T> zph = gload(ph, N + c);
      if constexpr (2 * N == 64 && SCALAR) {
        // rows y = pH + k: ph_y(pH + k) = ph_y(k) ph_y(H)^p (wave numbers k and k - H)
        const C<T> *phu = wave_uniform(ph);
        const C<T> zH = cmul(zph, uload(phu, H));
        const C<T> L{p ? zH.x : zph.x, p ? zH.y : zph.y};
#pragma unroll
        for (int k = 0; k < H; ++k) acc[k] = cadd(acc[k], cmul(h[k], cmul(uload(phu, k), L)));
      } else {
#pragma unroll
        for (int k = 0; k < H; ++k) acc[k] = cadd(acc[k], cmul(h[k], cmul(gload(ph, p * H + k), zph)));
      }
      if ((ent >> 17) & 1) {
        C<T> *dst = Y + (((size_t)side * a.Nr + r) * a.Sx + s) * n3 + (size_t)jx * N * N;
#pragma unroll
        for (int k = 0; k < H; ++k) {
          dst[(p * H + k) * N + c] = acc[k];
          acc[k] = C<T>{0, 0};
        }
      }
    }
    group_sync<N>();
  }
}

// Lane pair (pencil, p) = x-line: Hf, Hg (with the g-side loss), Vf.  The
// inverse x transforms of the decimated halves give wave numbers pH + k, the
// phases and tables act there, and a decimation-in-frequency transform
// returns to x = 2k + p.
template <typename T, int N, bool SYM>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_vjp_x(VjpArgs v) {
  constexpr int H = N / 2;
  const PipeArgs &a = v.a;
  const int pencil = blockIdx.x * 32 + (threadIdx.x >> 1), p = threadIdx.x & 1;
  const bool valid = pencil < N * N;
  const int pc = valid ? pencil : 0;
  const int e = blockIdx.y;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int vy = wave_idx(pc / N, N), vz = wave_idx(pc % N, N), kyz = vy * vy + vz * vz;
  const C<T> *Y = static_cast<const C<T> *>(v.Y) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  C<T> *Hs = static_cast<C<T> *>(v.H) + (size_t)e * 3 * n3;
  const T *ct = static_cast<const T *>(pd.ctab) + kyz;
  // G = sum_rs P_x,rs iFFT_x Y_side,rs of one side
  auto gain_sum = [&](int side, C<T>(&G)[H]) {
    const C<T> *px = static_cast<const C<T> *>(pd.px) + (size_t)side * a.Nr * a.Sx * N;
#pragma unroll
    for (int k = 0; k < H; ++k) G[k] = C<T>{0, 0};
    for (int rs = 0; rs < a.Nr * a.Sx; ++rs) {
      const C<T> *src = Y + ((size_t)side * a.Nr * a.Sx + rs) * n3;
      C<T> w[H];
#pragma unroll
      for (int n = 0; n < H; ++n) w[n] = src[(size_t)(2 * n + p) * N * N + pc];
      fft_pair<N, +1>(w, p);
      const C<T> *ph = px + (size_t)rs * N + p * H;
#pragma unroll
      for (int k = 0; k < H; ++k) G[k] = cadd(G[k], cmul(w[k], gload(ph, k)));
    }
  };
  // out = G - c(|k|) iFFT_x(Zfw) / N^3 (the g-side loss), in place of w
  auto minus_loss = [&](const C<T>(&G)[H], C<T>(&w)[H]) {
    const C<T> *Zfw = static_cast<const C<T> *>(v.Zw) + ((size_t)node * 2 + 1) * n3;
#pragma unroll
    for (int n = 0; n < H; ++n) w[n] = Zfw[(size_t)(2 * n + p) * N * N + pc];
    fft_pair<N, +1>(w, p);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int vx = wave_idx(p * H + k, N);
      w[k] = csub(G[k], cscale(w[k], gload(ct, vx * vx)));
    }
  };
  auto store_h = [&](int which, C<T>(&G)[H]) {
    fft_pair_dif<N, -1>(G, p);
    if (valid) {
#pragma unroll
      for (int k = 0; k < H; ++k) Hs[(size_t)which * n3 + (size_t)(2 * k + p) * N * N + pc] = G[k];
    }
  };
  C<T> G[H], w[H];
  gain_sum(0, G);
  if constexpr (SYM) {
    // p == q on one input with an antipodal sphere set: side 1's gain sum is
    // side 0's (only side 0's Y was formed)
    minus_loss(G, w);
    store_h(1, w);
    store_h(0, G);
  } else {
    store_h(0, G);
    gain_sum(1, G);
    minus_loss(G, w);
    store_h(1, w);
  }
  // Vf = iFFT_x(c FFT_x Z_g) / N^3
  const C<T> *Zg = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + a.zq[slot]) * n3;
#pragma unroll
  for (int n = 0; n < H; ++n) w[n] = Zg[(size_t)(2 * n + p) * N * N + pc];
  fft_pair<N, -1>(w, p);
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const int vx = wave_idx(p * H + k, N);
    w[k] = cscale(w[k], gload(ct, vx * vx));
  }
  fft_pair_dif<N, +1>(w, p);
  if (valid) {
#pragma unroll
    for (int k = 0; k < H; ++k) Hs[2 * n3 + (size_t)(2 * k + p) * N * N + pc] = w[k];
  }
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
