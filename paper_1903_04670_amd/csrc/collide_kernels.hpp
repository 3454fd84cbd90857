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
  const int *sx_zero;  // [Sx]: 1 if that sigma_x value is zero (X then independent of r)
  const int *morder;   // [M]: directions in sigma_x-group order
  // [M] and [Mh] groups of four ints in morder and mhalf order: m, s =
  // sidx[m], sneg[s], sx_zero[s] | sx_zero[sneg[s]] << 1
  const int *tinfo_full, *tinfo_half;
  const int *sneg;     // [Sx]: index of the opposite sigma_x value, or -1
  int xshare[kMaxPairs];  // 1: the pair has p == q on one input, so X2[s] = X1[sneg[s]]
  // Gain schedule.  The shift and gain kernels run over the n_gslots slots
  // gslot[]; slot i takes its C_r arrays from slot csrc[i].  With a sphere set
  // closed under sigma -> -sigma (equal weights) the m-sum of (q, p) equals
  // that of (p, q), so (q, p) reads (p, q)'s arrays; and for p == q on one
  // input the terms of sigma and -sigma coincide, so half[i] = 1 sums over
  // mhalf (one direction of each antipodal pair) with doubled weights.
  int n_gslots;
  int gslot[kMaxPairs], csrc[kMaxPairs], half[kMaxPairs];
  int cmirror[kMaxPairs];  // the slot that reads this slot's C_r arrays, or -1
  int Mh;
  const int *mhalf;
  // FP32 term schedules of the N = 32 gain kernel with shared column passes
  // (entries m | first << 16), for the full and the half set
  const int *gs_full, *gs_half;
  int gs_T_full, gs_T_half;
  // 1: the plan drops the Nyquist planes from the gain's translates (its
  // twiddle tables are zero there), so k_gain_yz takes the real-packed path
  int pack;
  void *Z, *X, *Cb, *V;
};

// Evaluation index of the eg-th (node, gain slot) of a launch over gain slots.
__device__ __forceinline__ int gain_eval(const PipeArgs &a, int eg) {
  return (eg / a.n_gslots) * a.n_pairs + a.gslot[eg % a.n_gslots];
}

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

// Load from a table that every lane reads at the same address: through the
// constant address space, so the compiler issues scalar (SMEM) loads.
template <typename V>
__device__ __forceinline__ V uload(const V *p, size_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  using CP = const __attribute__((address_space(4))) V *;
  return reinterpret_cast<CP>(reinterpret_cast<uintptr_t>(p))[i];
#else
  return p[i];
#endif
}

// Load from device memory through a pointer the compiler cannot place
// (read from a descriptor): as a global-address-space load, not a flat one.
template <typename V>
__device__ __forceinline__ V gload(const V *p, size_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  using GP = const __attribute__((address_space(1))) V *;
  return reinterpret_cast<GP>(reinterpret_cast<uintptr_t>(p))[i];
#else
  return p[i];
#endif
}

// The same address in every lane of the wavefront, as a scalar value.
template <typename V>
__device__ __forceinline__ const V *wave_uniform(const V *ptr) {
  const uint64_t u = reinterpret_cast<uint64_t>(ptr);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return reinterpret_cast<const V *>(((uint64_t)hi << 32) | lo);
}

// y phases of a column pass, lane pair (c, p) holding rows y = 2n + p (the
// decimated input of fft_pair): h[n] *= ph_y(2n + p) zph.  When a group is
// exactly one wavefront (N = 32) the table row is the same in every lane, so
// the identity ph_y(2n + p) = ph_y(2n) ph_y(1)^p (the wave numbers of rows 2n
// and 2n + 1 differ by one, N/2 being even) turns the 16 per-lane table
// loads into scalar loads of ph_y(2n), and only zph ph_y(1)^p is per lane.
// Per-lane loads that each wait for the previous one are what this avoids.
// A table with its Nyquist entry zeroed breaks the identity: SCALAR = false.
template <typename T, int N, bool SCALAR = true>
__device__ __forceinline__ void apply_col_phase(cplx<T> (&h)[N / 2], const cplx<T> *ph, int c, int p) {
  const cplx<T> zph = gload(ph, N + c);
  if constexpr (2 * N == 64 && SCALAR) {
    const cplx<T> *phu = wave_uniform(ph);
    const cplx<T> z1 = cmul(zph, uload(phu, 1));
    const cplx<T> L{p ? z1.x : zph.x, p ? z1.y : zph.y};
#pragma unroll
    for (int n = 0; n < N / 2; ++n) h[n] = cmul(h[n], cmul(uload(phu, 2 * n), L));
  } else {
#pragma unroll
    for (int n = 0; n < N / 2; ++n) h[n] = cmul(h[n], cmul(gload(ph, 2 * n + p), zph));
  }
}

// Barrier between the phases of one group of 2N threads whose LDS plane no
// other group touches.  When groups tile wavefronts exactly (2N divides 64)
// no hardware barrier is needed: the LDS operations of a wavefront complete
// in issue order, and the wavefront-scope fences keep the compiler from
// moving LDS accesses across this point.  Otherwise a group spans waves and
// the block barrier is used (every thread of the block must reach it).
template <int N> __device__ __forceinline__ void group_sync() {
  if constexpr (64 % (2 * N) == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Column phases of a lane pair (c, p) holding rows y = 2n + p, FP64, by
// recurrence instead of one table read per row: the wave index of row y is
// v = y below N/2 and y - N from N/2 on, so consecutive rows of a lane
// differ by e^{2 i beta} = ph(2) within each half.  Rows 2n + p, n < N/4,
// get zph ph(1)^p ph(2)^n; the upper half restarts from the table at rows
// N/2 + p and N/2 + 2 + p (the first may be a zeroed Nyquist entry, which
// the second skips) and steps by ph(2).  Four staged values per side
// replace 16 per-lane table reads, each an LDS round trip the next
// multiply waits for; the recurrence adds rounding of a few ulp.
// Requires N % 4 == 0 and N >= 8 (ph(2) is not a Nyquist entry).
template <typename T, int N>
__device__ __forceinline__ void col_phases_rec(cplx<T> (&h)[N / 2], const cplx<T> *ph, cplx<T> zph, int p) {
  constexpr int Q = N / 4;
  const cplx<T> rho = ph[2];
  const cplx<T> z1 = cmul(zph, ph[1]);
  cplx<T> phi{p ? z1.x : zph.x, p ? z1.y : zph.y};
#pragma unroll
  for (int n = 0; n < N / 2; ++n) {
    if (n == Q) phi = cmul(zph, ph[N / 2 + p]);
    else if (n == Q + 1) phi = cmul(zph, ph[N / 2 + 2 + p]);
    else if (n > 0) phi = cmul(phi, rho);
    h[n] = cmul(h[n], phi);
  }
}

// Column phases of a whole column held by one lane (rows y < N), FP64, by
// recurrence: consecutive rows differ by rho = ph(1) within each half of the
// wave indices (y below N/2, y - N from N/2 on); the upper half restarts from
// the table values ph(N/2) (possibly a zeroed Nyquist entry) and ph(N/2 + 1).
// Requires N >= 4.
template <typename T, int N>
__device__ __forceinline__ void col_phases_full(cplx<T> (&h)[N], cplx<T> zph, cplx<T> rho, cplx<T> ph_half,
                                                cplx<T> ph_half1) {
  const cplx<T> q0 = cmul(zph, ph_half), q1 = cmul(zph, ph_half1);
  cplx<T> phi = zph;
#pragma unroll
  for (int y = 0; y < N; ++y) {
    if (y == N / 2) phi = q0;
    else if (y == N / 2 + 1) phi = q1;
    else if (y > 0) phi = cmul(phi, rho);
    h[y] = cmul(h[y], phi);
  }
}

// v_permlane32_swap on a 64-bit value in each operand: the upper half-wave
// of a trades places with the lower half-wave of b, so lane l < 32 ends with
// (a_l, a_{l+32}) and lane l + 32 with (b_l, b_{l+32}).  Every lane of the
// wavefront must be active.
__device__ __forceinline__ void half_swap(double &a, double &b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// Streaming store of one complex value: the x-shifted arrays and the C_r
// arrays are written once and read back by the next kernel from HBM (a
// launch writes several GB), so the write need not allocate cache lines.
template <typename T> __device__ __forceinline__ void store_stream(cplx<T> *dst, cplx<T> v) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<V2 *>(dst));
}

// Compensated accumulation (the FP32 paired-lane gain and x kernels): Kahan's summation with
// the correction kept so that s + c is the running sum.  The rounding error
// of each addition, y - (t - s), is recovered exactly and fed into the next
// one; the error of the total is bounded by about 2 eps sum |x_i|,
// independent of the number of terms.
template <typename T> struct Acc {
  T s, c;
};
template <typename T> __device__ __forceinline__ void acc_add(T &s, T &c, T x) {
  const T y = x + c;
  const T t = s + y;
  c = y - (t - s);
  s = t;
}

// Source plane of the x-shifted input of (side, r, s) for evaluation slot
// `slot`.  With p == q on a single input, side 1 uses side 0's array of the
// opposite x component (the phases e^{-i th s v} and e^{+i th (-s) v} agree).
template <typename T>
__device__ __forceinline__ const C<T> *x_plane(const PipeArgs &a, const C<T> *Xe, int slot, int side, int r,
                                               int s, size_t n3) {
  if (side == 1 && a.xshare[slot] && uload(a.sneg, s) >= 0) {
    side = 0;
    s = uload(a.sneg, s);
  }
  const int rx = uload(a.sx_zero, s) ? 0 : r;  // X of a zero x-component does not depend on r
  return Xe + (((size_t)side * a.Nr + rx) * a.Sx + s) * n3;
}

// ------------------------------------------------------------------ k_fwd_yz
// One (node, slot, x-plane) per group of N threads; G planes per block.
template <typename T, int N, int G>
__device__ __forceinline__ void fwd_yz_body(const FwdArgs &a, int bx, int tid, C<T> (*lds)[N][N + 1]) {
  const int g = tid / N, t = tid % N;
  const int plane = bx * G + g;   // over N x-planes * n_nodes * nz
  const int jobs = N * a.n_nodes * a.nz;
  const bool active = g < G && plane < jobs;
  const int jx = plane % N, job = plane / N;
  const int node = job / a.nz, slot = job % a.nz;
  const size_t n3 = (size_t)N * N * N;
  if (active) {
    const double *f = a.src[slot] + (size_t)node * a.node_stride + (size_t)jx * N * N;
    // stage the real plane: element (y, z) -> lds[y][z]; thread t moves
    // column z = t, its N loads issued together (a runtime loop here waited
    // for each load before issuing the next)
    double v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = f[y * N + t];
#pragma unroll
    for (int y = 0; y < N; ++y) lds[g][y][t] = C<T>{(T)v[y], (T)0};
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
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * N) k_fwd_yz(FwdArgs a) {
  __shared__ C<T> lds[G][N][N + 1];
  fwd_yz_body<T, N, G>(a, blockIdx.x, threadIdx.x, lds);
}

// ------------------------------------------------------------------ k_shift_x
// Lane pair (pencil, p) = x-line (y, z) of one (eval, side): forward x
// transform of Z (decimation in time: lane p loads x = 2n + p and ends with
// frequencies p*N/2 + k), then for every r and distinct sigma_x the phase
// and the inverse transform (decimation in frequency back to x = 2n + p).
// HALF (real-packed plans): the x-lines with k_z in [0, N/2) only.  With the
// Nyquist planes dropped, every X plane is the (k_y, k_z) spectrum of a real
// function, so X(k_y, k_z) = conj X(-k_y, -k_z) and the gain kernel rebuilds
// the columns k_z > N/2 from these; the Nyquist column k_z = N/2 has zero
// twiddles and is never needed.
template <typename T, int N, bool HALF = false>
__device__ __forceinline__ void shift_x_body(const PipeArgs &a, int bx, int side, int e, int tid, int part = 0,
                                             int nparts = 1) {
  constexpr int H = N / 2;
  const int pencil = bx * 32 + (tid >> 1), p = tid & 1;
  const bool valid = pencil < (HALF ? N * H : N * N);
  // idle lanes still take part in the lane swaps
  const int pc = !valid ? 0 : HALF ? (pencil / H) * N + pencil % H : pencil;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const int zs = side == 0 ? a.zp[slot] : a.zq[slot];
  const C<T> *Z = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + zs) * n3;
  C<T> F[H];
#pragma unroll
  for (int n = 0; n < H; ++n) F[n] = Z[(size_t)(2 * n + p) * N * N + pc];
  fft_pair<N, -1>(F, p);
  const C<T> *px = static_cast<const C<T> *>(pd.px) + (size_t)side * a.Nr * a.Sx * N;
  C<T> *X = static_cast<C<T> *>(a.X) + ((size_t)e * 2 + side) * a.Nr * a.Sx * n3;
  const bool shared = side == 1 && a.xshare[slot];
  // the (r, s) arrays of this block: part `part` of `nparts` equal ranges
  const int nrs = a.Nr * a.Sx, rs_per = (nrs + nparts - 1) / nparts;
  const int rs_end = min(nrs, (part + 1) * rs_per);
  for (int rs = part * rs_per; rs < rs_end; ++rs) {
    // plan tables through the scalar cache: a vector load here would put a
    // memory round trip before every (r, s) array
    if (rs >= a.Sx && uload(a.sx_zero, rs % a.Sx)) continue;
    if (shared && uload(a.sneg, rs % a.Sx) >= 0) continue;
    const C<T> *ph = px + (size_t)rs * N + p * H;
    C<T> w[H];
#pragma unroll
    for (int k = 0; k < H; ++k) w[k] = cmul(F[k], gload(ph, k));
    fft_pair_dif<N, +1>(w, p);
    C<T> *dst = X + (size_t)rs * n3;
    if (valid) {
#pragma unroll
      for (int k = 0; k < H; ++k) store_stream(&dst[(size_t)(2 * k + p) * N * N + pc], w[k]);
    }
  }
}
// blockIdx.y = side + 2 part: the (r, s) loop is split over NP blocks per
// (x-lines, side, eval), each redoing the cheap forward x transform, so that
// more waves share the latency of the phase loads and stores
template <typename T, int N, int NP = 1, bool HALF = false>
__global__ void __launch_bounds__(64) k_shift_x(PipeArgs a) {
  shift_x_body<T, N, HALF>(a, blockIdx.x, blockIdx.y & 1, gain_eval(a, blockIdx.z), threadIdx.x, blockIdx.y >> 1,
                           NP);
}

// ------------------------------------------------------------------ k_gain_yz
// The paired-lane gain kernel, for N other than 32 (N = 32 runs
// gain_yz_halves_body and gain_yz_halves_packed_body below).
// Block = G groups of 2N threads on one (eval, r, x-plane); group g takes the
// directions m = g, g+G, ...  Every length-N pencil is split over a lane pair
// (fft_pair).  Per direction and side: the column (y) pass reads X coalesced
// (lane pair (c, p) holds rows y = 2n+p of column z = c), transforms, and
// writes the column to the group's LDS buffer; the row (z) pass reads row
// y = c back (z = 2n+p) and transforms it.  u1's row half stays in
// registers while u2 reuses the buffer; the product is accumulated into the
// row-half accumulator P (compensated in FP32).
// LDS planes per group in k_gain_yz: FP32 keeps both sides' columns in
// flight (two buffers); FP64 uses one buffer so that LDS does not limit
// occupancy below what its registers allow.
template <typename T> constexpr int gain_bufs() { return sizeof(T) == 4 ? 2 : 1; }

// Groups per k_gain_yz block: at least 128 threads, except one wave per
// block for the real-packed path at N = 32 (measured faster: the block's
// final transform then idles no second group).  The literal terms at N = 32
// run gain_yz_halves_body instead.  The batched kernel uses the same counts,
// so results match bit for bit.
template <int N> constexpr int default_gain_groups() { return 128 / (2 * N) > 0 ? 128 / (2 * N) : 1; }
template <int N> constexpr int packed_gain_groups() { return N == 32 ? 1 : default_gain_groups<N>(); }
template <typename T, int N> constexpr int literal_gain_groups() { return default_gain_groups<N>(); }

// LDS of k_gain_yz besides its planes: per group the yz phase rows of its
// current direction, [2 sides][2N] (y phases, then z phases).
template <typename T, int N, int G> constexpr size_t gain_phase_elems() { return (size_t)G * 4 * N; }

// The gain kernel's layout at N = 32 (gain_yz_halves_body): one wavefront
// per (evaluation, r, x-plane), the two sides on its half-waves.
template <typename T, int N> constexpr bool gain_halves() { return N == 32; }

__device__ __forceinline__ void half_swap(float &a, float &b) {
  const auto v = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(v[0]);
  b = __uint_as_float(v[1]);
}

// Forward 2-D transform of a wavefront's sum over directions and the store
// of C_r: lane (side, c) holds the sum on row c, z = side N/2 + k, k < N/2;
// it goes through the plane, then lane pairs (cp, pp) take the z pass on row
// cp from the decimated columns 2n + pp and the y pass on column cp.
template <typename T, int N>
__device__ __forceinline__ void halves_forward(const PipeArgs &a, int jx, int r, int e, int l, C<T> (*pw)[N + 1],
                                               const C<T> (&P)[N / 2]) {
  constexpr int H = N / 2;
  const int side = l >> 5, c = l & 31;
  const size_t n3 = (size_t)N * N * N;
#pragma unroll
  for (int k = 0; k < H; ++k) pw[c][side * H + k] = P[k];
  group_sync<N>();
  const int cp = l >> 1, pp = l & 1;
  C<T> f[H];
#pragma unroll
  for (int n = 0; n < H; ++n) f[n] = pw[cp][2 * n + pp];
  fft_pair<N, -1>(f, pp);
  group_sync<N>();
#pragma unroll
  for (int k = 0; k < H; ++k) pw[cp][pp * H + k] = f[k];
  group_sync<N>();
#pragma unroll
  for (int n = 0; n < H; ++n) f[n] = pw[2 * n + pp][cp];
  fft_pair<N, -1>(f, pp);
  C<T> *dst = static_cast<C<T> *>(a.Cb) + ((size_t)e * a.Nr + r) * n3 + (size_t)jx * N * N;
#pragma unroll
  for (int k = 0; k < H; ++k) store_stream(&dst[(pp * H + k) * N + cp], f[k]);
}

// One (evaluation, r, x-plane) per wavefront at N = 32, with the two sides on
// the two half-waves.  Lane (side, c), c < 32, holds a whole pencil: column
// z = c for the y pass, row y = c for the z pass, so each transform runs
// inside one lane, with no lane-pair exchange and no join twiddles that only
// one lane of a pair needs.  After the row pass lane (0, c) holds u1 and lane
// (1, c) holds u2 on row c; one half-wave swap per value leaves lane (h, c)
// with both on z = 16 h + j, j < 16, where the product accumulates.  The
// wavefront then takes the forward transform of its sum over lane pairs and
// writes C_r.  Every direction of the slot is summed in one wavefront, in the
// same order wherever this body runs, so results do not depend on the launch
// (single plan or batch).
//  * FP64: one LDS plane (pl[0]) carries one side's transpose at a time, so
//    the registers of the other side's pencil stay untouched; the column
//    phases come by recurrence from four table values.
//  * FP32-mixed: one plane per side (pl[0], pl[1]), both sides transpose at
//    once, and the column pass of a (sigma_x, sigma_y) class serves every
//    direction of the class (the plan's term schedule); the z phase, constant
//    along a column, is applied in the row pass.  Phase rows are staged in
//    phs ([side][y row, z row]) one direction ahead, and the products, exact
//    in FP64, are summed in FP64.
template <typename T, int N>
__device__ __forceinline__ void gain_yz_halves_body(const PipeArgs &a, int jx, int r, int e, int l,
                                                    C<T> (*pl)[N][N + 1], C<T> *phs) {
  static_assert(gain_halves<T, N>() && 2 * N == 64, "half-wave sides need N = 32");
  constexpr int H = N / 2;
  const int side = l >> 5, c = l & 31;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  // the quadrature weight w_m (doubled on a half set) rides on side 0's z
  // phase, which is constant along each column and enters u1 linearly
  const T wscale = a.half[slot] ? (T)2 : (T)1;
  C<T> P[H];
#pragma unroll
  for (int k = 0; k < H; ++k) P[k] = C<T>{0, 0};
  if constexpr (sizeof(T) == 8) {
    const int Mx = a.half[slot] ? a.Mh : a.M;
    const int4 *tinfo = reinterpret_cast<const int4 *>(a.half[slot] ? a.tinfo_half : a.tinfo_full);
    C<T>(*pw)[N + 1] = pl[0];
    // Direction and x-shifted plane offsets of both sides for term mi (the
    // choice of x_plane made with wave-uniform values), from one scalar load
    // of the plan's term table, taken one term ahead.
    auto term = [&](int mi, int &m, size_t &o0, size_t &o1) {
      const int4 v = uload(tinfo, mi);
      m = v.x;
      const int s = v.y, sn = v.z;
      const int rx = (v.w & 1) ? 0 : r;
      o0 = ((size_t)rx * a.Sx + s) * n3;
      if (a.xshare[slot] && sn >= 0) {
        const int rxn = (v.w & 2) ? 0 : r;
        o1 = ((size_t)rxn * a.Sx + sn) * n3;  // side 0's array of the opposite x component
      } else {
        o1 = (((size_t)a.Nr + rx) * a.Sx + s) * n3;
      }
    };
    int m_n = 0;
    size_t o0_n = 0, o1_n = 0;
    if (Mx > 0) term(0, m_n, o0_n, o1_n);
    for (int mi = 0; mi < Mx; ++mi) {
      const int m = m_n;
      const size_t o = side ? o1_n : o0_n;
      if (mi + 1 < Mx) term(mi + 1, m_n, o0_n, o1_n);
      // phase values first: the recurrence can start as the first rows arrive
      const C<T> *ph = pyz + (((size_t)side * a.Nr + r) * a.M + m) * 2 * N;
      const C<T> zph = gload(ph, N + c), rho = gload(ph, 1), phh = gload(ph, N / 2), phh1 = gload(ph, N / 2 + 1);
      const C<T> *src = X + o + (size_t)jx * N * N + c;
      C<T> h[N];
#pragma unroll
      for (int y = 0; y < N; ++y) h[y] = src[y * N];
      const T ws = side ? (T)1 : uload(wm, m) * wscale;
      col_phases_full<T, N>(h, cscale(zph, ws), rho, phh, phh1);
      fft<N, +1>(h);
      if (side == 0) {
#pragma unroll
        for (int y = 0; y < N; ++y) pw[y][c] = h[y];
      }
      group_sync<N>();
      if (side == 0) {
#pragma unroll
        for (int z = 0; z < N; ++z) h[z] = pw[c][z];
      }
      group_sync<N>();
      if (side == 1) {
#pragma unroll
        for (int y = 0; y < N; ++y) pw[y][c] = h[y];
      }
      group_sync<N>();
      if (side == 1) {
#pragma unroll
        for (int z = 0; z < N; ++z) h[z] = pw[c][z];
      }
      group_sync<N>();
      fft<N, +1>(h);
#pragma unroll
      for (int j = 0; j < H; ++j) {
        half_swap(h[j].x, h[j + H].x);
        half_swap(h[j].y, h[j + H].y);
        // P += u1 u2 as two fused multiply-adds per component
        P[j].x = __builtin_fma(h[j].x, h[j + H].x, __builtin_fma(-h[j].y, h[j + H].y, P[j].x));
        P[j].y = __builtin_fma(h[j].x, h[j + H].y, __builtin_fma(h[j].y, h[j + H].x, P[j].y));
      }
    }
  } else {
    const int nT = a.half[slot] ? a.gs_T_half : a.gs_T_full;
    const int *sch = a.half[slot] ? a.gs_half : a.gs_full;
    // the product of two FP32 values is exact in FP64, and the sum over
    // directions runs in FP64 (as many registers as an FP32 sum with its
    // compensation, and fewer instructions)
    double Px[H], Py[H];
#pragma unroll
    for (int k = 0; k < H; ++k) Px[k] = Py[k] = 0.0;
    C<T> pf0{0, 0}, pf1{0, 0};
    auto fetch_ph = [&](int m) {
      pf0 = gload(pyz + ((size_t)r * a.M + m) * 2 * N, l);
      pf1 = gload(pyz + (((size_t)a.Nr + r) * a.M + m) * 2 * N, l);
    };
    int ent_next = nT > 0 ? uload(sch, 0) : -1;
    if (ent_next >= 0) fetch_ph(ent_next & 0xffff);
    // schedule entries m | first << 16; a one-group schedule pads nothing
    for (int t = 0; t < nT; ++t) {
      const int ent = ent_next;
      if (ent < 0) break;
      ent_next = t + 1 < nT ? uload(sch, t + 1) : -1;
      const int m = ent & 0xffff;
      const T ws = l >= N ? uload(wm, m) * wscale : (T)1;
      phs[l] = C<T>{pf0.x * ws, pf0.y * ws};
      phs[2 * N + l] = pf1;
      group_sync<N>();
      if (ent_next >= 0) fetch_ph(ent_next & 0xffff);
      const C<T> *ph = phs + side * 2 * N;
      if ((ent >> 16) & 1) {
        const C<T> *src = x_plane(a, X, slot, side, r, uload(a.sidx, m), n3) + (size_t)jx * N * N + c;
        C<T> h[N];
#pragma unroll
        for (int y = 0; y < N; ++y) h[y] = cmul(src[y * N], ph[y]);
        fft<N, +1>(h);
#pragma unroll
        for (int y = 0; y < N; ++y) pl[side][y][c] = h[y];
        group_sync<N>();
      }
      C<T> h[N];
#pragma unroll
      for (int z = 0; z < N; ++z) h[z] = cmul(pl[side][c][z], ph[N + z]);
      fft<N, +1>(h);
#pragma unroll
      for (int j = 0; j < H; ++j) {
        half_swap(h[j].x, h[j + H].x);
        half_swap(h[j].y, h[j + H].y);
        const double ax = h[j].x, ay = h[j].y, bx = h[j + H].x, by = h[j + H].y;
        Px[j] = __builtin_fma(ax, bx, __builtin_fma(-ay, by, Px[j]));
        Py[j] = __builtin_fma(ax, by, __builtin_fma(ay, bx, Py[j]));
      }
      group_sync<N>();
    }
#pragma unroll
    for (int k = 0; k < H; ++k) P[k] = C<T>{(T)Px[k], (T)Py[k]};
  }
  halves_forward<T, N>(a, jx, r, e, l, pl[0], P);
}

// Real-packed terms (the Nyquist-zeroed variant) at N = 32, one wavefront per
// (evaluation, r, x-plane): with the Nyquist planes dropped from both
// translates, u1 and u2 are real, so one transform of h = t1 + i t2 gives
// u1 = Re h and u2 = Im h (t1 carrying w_m), and the product is real.  Here
// each half-wave takes its own direction term (directions 2i and 2i + 1 of
// the slot), each lane a whole pencil of h: column z = c, then row y = c.
// The x-shifted arrays hold the columns k_z < N/2 and are Hermitian (their
// x-Nyquist plane is dropped too).  A lane of column c > N/2 reads column
// N - c with rows in natural order, g(k') = X(k', N - c) = conj X(-k', c),
// and transforms psi1 g1 - i psi2 g2 with psi(k') = conj(phi(-k')) (the z
// phase conjugated; the y phase is unchanged away from the zeroed Nyquist
// row): the result is the conjugate of the true column, so the row pass takes
// conj of the entries k_z > N/2.  The lane of the Nyquist column reads column
// 0, which its zero z phase discards.  A half-wave left without a direction
// (odd counts) runs with zero phases.  After each pair of terms one half-wave
// swap per value brings both halves' products of a point to one lane, which
// sums them in the layout of halves_forward.
template <typename T, int N>
__device__ __forceinline__ void gain_yz_halves_packed_body(const PipeArgs &a, int jx, int r, int e, int l,
                                                           C<T> (*pl)[N][N + 1]) {
  static_assert(gain_halves<T, N>() && 2 * N == 64, "half-wave terms need N = 32");
  constexpr int H = N / 2;
  const int half = l >> 5, c = l & 31;
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  const T wscale = a.half[slot] ? (T)2 : (T)1;
  const int Mx = a.half[slot] ? a.Mh : a.M;
  const int4 *tinfo = reinterpret_cast<const int4 *>(a.half[slot] ? a.tinfo_half : a.tinfo_full);
  const bool mr = c > H;
  const int col = c < H ? c : (c == H ? 0 : N - c);
  const T sg = mr ? (T)-1 : (T)1;  // sign of the i t2 term and of the z phase's imaginary part
  C<T>(*pw)[N + 1] = pl[0];
  // sum over the slot's directions on row c, z = half N/2 + j, in FP64 in
  // both precisions (in FP32 as many registers as a compensated sum)
  double P[H];
#pragma unroll
  for (int k = 0; k < H; ++k) P[k] = 0.0;
  for (int mi = 0; mi < Mx; mi += 2) {
    const int my = mi + half;           // this half-wave's direction
    const bool on = my < Mx;
    const int4 v = uload(tinfo, on ? my : mi);
    const int m = v.x, s = v.y, sn = v.z;
    // x-shifted arrays of both sides (side 1 may use side 0's array of -s)
    const int rx = (v.w & 1) ? 0 : r;
    const size_t o0 = ((size_t)rx * a.Sx + s) * n3;
    size_t o1;
    if (a.xshare[slot] && sn >= 0) {
      const int rxn = (v.w & 2) ? 0 : r;
      o1 = ((size_t)rxn * a.Sx + sn) * n3;
    } else {
      o1 = (((size_t)a.Nr + rx) * a.Sx + s) * n3;
    }
    const C<T> *ph0 = pyz + ((size_t)r * a.M + m) * 2 * N;
    const C<T> *ph1 = pyz + (((size_t)a.Nr + r) * a.M + m) * 2 * N;
    const T ws = on ? gload(wm, m) * wscale : (T)0;
    C<T> z0 = cscale(gload(ph0, N + c), ws), z1 = cscale(gload(ph1, N + c), on ? (T)1 : (T)0);
    z0.y *= sg;
    z1.y *= sg;
    const C<T> rho0 = gload(ph0, 1), q00 = gload(ph0, N / 2), q01 = gload(ph0, N / 2 + 1);
    const C<T> rho1 = gload(ph1, 1), q10 = gload(ph1, N / 2), q11 = gload(ph1, N / 2 + 1);
    const C<T> *src0 = X + o0 + (size_t)jx * N * N + col;
    const C<T> *src1 = X + o1 + (size_t)jx * N * N + col;
    C<T> h[N];
#pragma unroll
    for (int y = 0; y < N; ++y) h[y] = src0[y * N];
    col_phases_full<T, N>(h, z0, rho0, q00, q01);
    // h += sg i phi1 X1, phi1 by the same recurrence, one row at a time
    {
      const C<T> a0 = cmul(z1, q10), a1 = cmul(z1, q11);
      C<T> phi = z1;
#pragma unroll
      for (int y = 0; y < N; ++y) {
        if (y == N / 2) phi = a0;
        else if (y == N / 2 + 1) phi = a1;
        else if (y > 0) phi = cmul(phi, rho1);
        const C<T> g = src1[y * N];
        const C<T> t = cmul(g, phi);
        h[y] = C<T>{fmaT(-sg, t.y, h[y].x), fmaT(sg, t.x, h[y].y)};
      }
    }
    fft<N, +1>(h);
    if (half == 0) {
#pragma unroll
      for (int y = 0; y < N; ++y) pw[y][c] = h[y];
    }
    group_sync<N>();
    if (half == 0) {
#pragma unroll
      for (int z = 0; z < N; ++z) h[z] = pw[c][z];
    }
    group_sync<N>();
    if (half == 1) {
#pragma unroll
      for (int y = 0; y < N; ++y) pw[y][c] = h[y];
    }
    group_sync<N>();
    if (half == 1) {
#pragma unroll
      for (int z = 0; z < N; ++z) h[z] = pw[c][z];
    }
    group_sync<N>();
#pragma unroll
    for (int z = H + 1; z < N; ++z) h[z].y = -h[z].y;  // mirrored columns
    fft<N, +1>(h);
    // products of both half-waves' directions on row c: one half-wave swap
    // per value leaves lane (half, c) with both on z = half N/2 + j
#pragma unroll
    for (int j = 0; j < H; ++j) {
      T lo = h[j].x * h[j].y, hi = h[j + H].x * h[j + H].y;
      half_swap(lo, hi);
      if constexpr (sizeof(T) == 4) {
        P[j] += (double)lo;
        P[j] += (double)hi;
      } else {
        P[j] += lo + hi;
      }
    }
  }
  C<T> S[H];
#pragma unroll
  for (int j = 0; j < H; ++j) S[j] = C<T>{(T)P[j], (T)0};
  halves_forward<T, N>(a, jx, r, e, l, pw, S);
}

template <typename T, int N, int G, int NB = gain_bufs<T>(), bool PACK = false>
__device__ __forceinline__ void gain_yz_body(const PipeArgs &a, int jx, int r, int e, int tid, C<T> (*lds)[N][N + 1],
                                             C<T> *phs_all) {
  constexpr int H = N / 2;
  const int g = tid / (2 * N), l = tid % (2 * N);
  const int c = l >> 1, p = l & 1;  // column (then row) index, lane parity
  const bool in_group = g < G;       // threads beyond G groups only join the barriers
  const int slot = e % a.n_pairs;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const size_t n3 = (size_t)N * N * N;
  const C<T> *X = static_cast<const C<T> *>(a.X) + (size_t)e * 2 * a.Nr * a.Sx * n3;
  const T *wm = static_cast<const T *>(a.wm);
  const C<T> *pyz = static_cast<const C<T> *>(pd.pyz);
  C<T> P[H], u1[H];
  T Pcx[sizeof(T) == 4 ? H : 1], Pcy[sizeof(T) == 4 ? H : 1];
#pragma unroll
  for (int k = 0; k < H; ++k) P[k] = C<T>{0, 0};
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < H; ++k) Pcx[k] = Pcy[k] = 0;
  }
  // column pass of one side: rows y = 2n + p of column z = c, phases, iFFT_y,
  // then column c of the buffer
  auto load_col = [&](int side, int s, C<T>(&h)[H]) {
    const C<T> *src = x_plane(a, X, slot, side, r, s, n3) + (size_t)jx * N * N;
#pragma unroll
    for (int n = 0; n < H; ++n) h[n] = src[(2 * n + p) * N + c];
  };
  // The group's phase rows for its current direction are staged in LDS (one
  // entry per lane and side, fetched one direction ahead), so the column
  // passes read them with in-order LDS loads rather than per-lane global
  // loads that each wait for the one before.
  C<T> *phs = phs_all + (size_t)(in_group ? g : 0) * 4 * N;
  C<T> pf0{0, 0}, pf1{0, 0};
  auto fetch_ph = [&](int m) {
    pf0 = gload(pyz + ((size_t)r * a.M + m) * 2 * N, l);
    pf1 = gload(pyz + (((size_t)a.Nr + r) * a.M + m) * 2 * N, l);
  };
  constexpr bool kRec = sizeof(T) == 8 && N % 4 == 0 && N >= 8 && !PACK;
  auto finish_col = [&](int side, int m, C<T>(&h)[H], C<T>(*buf)[N + 1]) {
    const C<T> *ph = phs + side * 2 * N;
    const C<T> zph = ph[N + c];
    if constexpr (kRec) {
      col_phases_rec<T, N>(h, ph, zph, p);
    } else {
#pragma unroll
      for (int n = 0; n < H; ++n) h[n] = cmul(h[n], cmul(ph[2 * n + p], zph));
    }
    fft_pair<N, +1>(h, p);
#pragma unroll
    for (int k = 0; k < H; ++k) buf[p * H + k][c] = h[k];
  };
  auto col_pass = [&](int side, int m, int s, C<T>(*buf)[N + 1]) {
    C<T> h[H];
    load_col(side, s, h);
    finish_col(side, m, h, buf);
  };
  // The quadrature weight w_m (doubled on a half set) rides on side 0's z
  // phase row when it is staged: that row is constant along each column and
  // enters u1 linearly, so the product below needs no separate scaling.
  const T wscale = a.half[slot] ? (T)2 : (T)1;
  auto stage_ph = [&](int m) {
    const T ws = l >= N ? uload(wm, m) * wscale : (T)1;
    phs[l] = C<T>{pf0.x * ws, pf0.y * ws};
    phs[2 * N + l] = pf1;
  };
  auto accumulate = [&](const C<T> (&h)[H]) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const C<T> pr = cmul(u1[k], h[k]);
      if constexpr (sizeof(T) == 4) {
        acc_add(P[k].x, Pcx[k], pr.x);
        acc_add(P[k].y, Pcy[k], pr.y);
      } else {
        // P += u1 h as two fused multiply-adds per component
        P[k].x = __builtin_fma(u1[k].x, h[k].x, __builtin_fma(-u1[k].y, h[k].y, P[k].x));
        P[k].y = __builtin_fma(u1[k].x, h[k].y, __builtin_fma(u1[k].y, h[k].x, P[k].y));
      }
    }
  };
  const int Mx = a.half[slot] ? a.Mh : a.M;
  const int *mo = a.half[slot] ? a.mhalf : a.morder;
  const int iters = (Mx + G - 1) / G;
  if constexpr (PACK) {
    // Real-packed terms.  With the Nyquist planes dropped from both
    // translates, u1 and u2 are real, so one column and one row transform of
    // h = t1 + i t2 give u1 = Re h and u2 = Im h (t1 carrying w_m), and the
    // product accumulates into the real parts of P.  The phase rows of the
    // next direction are staged while the row pass runs, so two group
    // barriers per direction suffice.
    // X holds the columns k_z < N/2 only (shift_x_body<HALF>): a lane of
    // column c > N/2 reads column N - c at the mirrored rows -y mod N and
    // conjugates; the lane of the Nyquist column reads column 0, which its
    // zero twiddle discards.
    const bool mr = c > H;
    const int col = c < H ? c : (c == H ? 0 : N - c);
    const int rbase = (mr ? N - p : p) * N, rstep = mr ? -2 * N : 2 * N;
    const int row0 = mr ? (p ? N - 1 : 0) : p;
    const T csg = mr ? (T)-1 : (T)1;
    auto load_half = [&](int side, int s, C<T>(&h)[H]) {
      const C<T> *src = x_plane(a, X, slot, side, r, s, n3) + (size_t)jx * N * N + col;
#pragma unroll
      for (int n = 0; n < H; ++n) {
        const C<T> v = src[n == 0 ? row0 * N : rbase + n * rstep];
        h[n] = C<T>{v.x, csg * v.y};
      }
    };
    // with one group per block the direction index is the same in every
    // lane, so the plan tables and x_plane are read through the scalar cache
    int mi = G == 1 ? 0 : g;
    bool active = in_group && mi < Mx;
    if (active) {
      fetch_ph(uload(mo, mi));
      stage_ph(uload(mo, mi));
      if (mi + G < Mx) fetch_ph(uload(mo, mi + G));
    }
    group_sync<N>();
    for (int it = 0; it < iters; ++it) {
      if (active) {
        const int s = uload(a.sidx, uload(mo, mi));
        C<T> h[H], h1[H];
        load_half(0, s, h);
        load_half(1, s, h1);
        const C<T> z0 = phs[N + c], z1 = phs[3 * N + c];
#pragma unroll
        for (int n = 0; n < H; ++n) {
          const C<T> t1 = cmul(h[n], cmul(phs[2 * n + p], z0));
          const C<T> t2 = cmul(h1[n], cmul(phs[2 * N + 2 * n + p], z1));
          h[n] = C<T>{t1.x - t2.y, t1.y + t2.x};
        }
        fft_pair<N, +1>(h, p);
#pragma unroll
        for (int k = 0; k < H; ++k) lds[NB * g][p * H + k][c] = h[k];
      }
      group_sync<N>();
      const int mn = mi + G;
      const bool next = in_group && mn < Mx;
      if (next) {
        stage_ph(uload(mo, mn));
        if (mn + G < Mx) fetch_ph(uload(mo, mn + G));
      }
      if (active) {
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = lds[NB * g][c][2 * n + p];
        fft_pair<N, +1>(h, p);
#pragma unroll
        for (int k = 0; k < H; ++k) {
          if constexpr (sizeof(T) == 4) {
            acc_add(P[k].x, Pcx[k], h[k].x * h[k].y);
          } else {
            P[k].x += h[k].x * h[k].y;
          }
        }
      }
      group_sync<N>();
      mi = mn;
      active = next;
    }
  } else {
  // with one group per block the direction index is the same in every lane
  // (lanes outside the group only skip the work), so the plan tables and
  // x_plane are read through the scalar cache
  const int g0 = G == 1 ? 0 : g;
  if (in_group && g0 < Mx) fetch_ph(uload(mo, g0));
  for (int it = 0; it < iters; ++it) {
    const int mi = it * G + g0;
    const bool active = in_group && mi < Mx;
    const int m = mi < Mx ? uload(mo, mi) : 0;
    const int s = uload(a.sidx, m);
    if (active) stage_ph(m);
    group_sync<N>();
    if (active && mi + G < Mx) fetch_ph(uload(mo, mi + G));
    if constexpr (NB == 2) {
      if (active) {
        col_pass(0, m, s, lds[2 * g]);
        col_pass(1, m, s, lds[2 * g + 1]);
      }
      group_sync<N>();
      if (active) {
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = lds[2 * g][c][2 * n + p];
        fft_pair<N, +1>(h, p);
#pragma unroll
        for (int k = 0; k < H; ++k) u1[k] = h[k];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = lds[2 * g + 1][c][2 * n + p];
        fft_pair<N, +1>(h, p);
        accumulate(h);
      }
      group_sync<N>();
    } else {
      // side 0's row pass transforms in u1 itself (no copy); side 1's
      // result goes straight into the product
      if (active) col_pass(0, m, s, lds[g]);
      group_sync<N>();
      if (active) {
#pragma unroll
        for (int n = 0; n < H; ++n) u1[n] = lds[g][c][2 * n + p];
        fft_pair<N, +1>(u1, p);
      }
      group_sync<N>();
      if (active) col_pass(1, m, s, lds[g]);
      group_sync<N>();
      if (active) {
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = lds[g][c][2 * n + p];
        fft_pair<N, +1>(h, p);
        accumulate(h);
      }
      group_sync<N>();
    }
  }
  }
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < H; ++k) P[k] = C<T>{P[k].x + Pcx[k], P[k].y + Pcy[k]};
  }
  // P (row y = c, z = p*H + k) to LDS; groups combined in group order
  if (in_group) {
#pragma unroll
    for (int k = 0; k < H; ++k) lds[NB * g][c][p * H + k] = P[k];
  }
  __syncthreads();
  if (g == 0) {
    // row pass of the forward transform: read z = 2n + p, summing the groups
    C<T> h[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
      T sx = lds[0][c][2 * n + p].x, sy = lds[0][c][2 * n + p].y, cx = 0, cy = 0;
      for (int q = 1; q < G; ++q) {
        const C<T> v = lds[NB * q][c][2 * n + p];
        if constexpr (sizeof(T) == 4) {
          acc_add(sx, cx, v.x);
          acc_add(sy, cy, v.y);
        } else {
          sx += v.x;
          sy += v.y;
        }
      }
      h[n] = C<T>{sx + cx, sy + cy};
    }
    fft_pair<N, -1>(h, p);
#pragma unroll
    for (int k = 0; k < H; ++k) P[k] = h[k];
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < H; ++k) lds[0][c][p * H + k] = P[k];
  }
  __syncthreads();
  if (g == 0) {
    C<T> h[H];
#pragma unroll
    for (int n = 0; n < H; ++n) h[n] = lds[0][2 * n + p][c];
    fft_pair<N, -1>(h, p);
    C<T> *dst = static_cast<C<T> *>(a.Cb) + ((size_t)e * a.Nr + r) * n3 + (size_t)jx * N * N;
#pragma unroll
    for (int k = 0; k < H; ++k) store_stream(&dst[(p * H + k) * N + c], h[k]);
  }
}
template <typename T, int N, int G, int NB = gain_bufs<T>(), bool PACK = false>
__global__ void __launch_bounds__(G * 2 * N) k_gain_yz(PipeArgs a) {
  __shared__ C<T> lds[G * NB][N][N + 1];
  __shared__ C<T> phs[gain_phase_elems<T, N, G>()];
  gain_yz_body<T, N, G, NB, PACK>(a, blockIdx.x, blockIdx.y, gain_eval(a, blockIdx.z), threadIdx.x, lds, phs);
}
// Real-packed terms: two x-planes per block, one per wavefront
// (gain_yz_halves_packed_body, one LDS plane each); grid (N / 2, N_rho,
// gain evaluations).
template <typename T, int N>
__global__ void __launch_bounds__(128) k_gain_yz_halves_packed(PipeArgs a) {
  __shared__ C<T> lds[2][N][N + 1];
  const int w = threadIdx.x >> 6;
  gain_yz_halves_packed_body<T, N>(a, 2 * blockIdx.x + w, blockIdx.y, gain_eval(a, blockIdx.z), threadIdx.x & 63,
                                   lds + w);
}
// Two x-planes per block, one per wavefront (gain_yz_halves_body); grid
// (N / 2, N_rho, gain evaluations).  LDS per wavefront: one plane in FP64,
// two planes and the staged phase rows in FP32 (the same layout as the
// two-group k_gain_yz, which the batched kernel shares).
template <typename T, int N>
__global__ void __launch_bounds__(128) k_gain_yz_halves(PipeArgs a) {
  constexpr int NB = gain_bufs<T>();
  __shared__ C<T> lds[2 * NB][N][N + 1];
  __shared__ C<T> phs[gain_phase_elems<T, N, 2>()];
  const int w = threadIdx.x >> 6;
  gain_yz_halves_body<T, N>(a, 2 * blockIdx.x + w, blockIdx.y, gain_eval(a, blockIdx.z), threadIdx.x & 63,
                            lds + NB * w, phs + w * 4 * N);
}

// ------------------------------------------------------------------ k_gain_x
// Lane pair = x-line (y, z) of one gain slot: QG = sum_r g_r(|k|) FFT_x C_r,
// then V1 = iFFT_x QG and V2 = iFFT_x(c(|k|) FFT_x Z_q).  A slot whose C_r
// are reused by a mirrored slot (q, p) serves it in the same pass when FUSE
// is set: each FFT_x C_r is multiplied by both pairs' gain tables (the FP32
// kernel; in FP64 the second accumulator costs more occupancy than it saves).
template <typename T, int N, bool FUSE = false>
__device__ __forceinline__ void gain_x_body(const PipeArgs &a, int bx, int e, int tid) {
  constexpr int H = N / 2;
  const int pencil = bx * 32 + (tid >> 1), p = tid & 1;
  const bool valid = pencil < N * N;
  const int pc = valid ? pencil : 0;
  const int node = e / a.n_pairs, slot = e % a.n_pairs;
  const int slot2 = FUSE ? a.cmirror[slot] : -1;
  const bool two = slot2 >= 0;
  const PairDev pd = a.pairs[a.pair_id[slot]];
  const PairDev pd2 = a.pairs[a.pair_id[two ? slot2 : slot]];
  const size_t n3 = (size_t)N * N * N;
  const int K2 = 3 * (N / 2) * (N / 2) + 1;
  const int vy = wave_idx(pc / N, N), vz = wave_idx(pc % N, N);
  const int kyz = vy * vy + vz * vz;
  const T *gt = static_cast<const T *>(pd.gtab), *gt2 = static_cast<const T *>(pd2.gtab);
  const C<T> *Cb = static_cast<const C<T> *>(a.Cb) + (size_t)(node * a.n_pairs + a.csrc[slot]) * a.Nr * n3;
  C<T> Q[H], Q2[H];
  T Qcx[sizeof(T) == 4 ? H : 1], Qcy[sizeof(T) == 4 ? H : 1];
  T Qcx2[sizeof(T) == 4 ? H : 1], Qcy2[sizeof(T) == 4 ? H : 1];
#pragma unroll
  for (int k = 0; k < H; ++k) Q[k] = Q2[k] = C<T>{0, 0};
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < H; ++k) Qcx[k] = Qcy[k] = Qcx2[k] = Qcy2[k] = 0;
  }
  auto acc = [&](C<T>(&q)[H], T(&cx)[sizeof(T) == 4 ? H : 1], T(&cy)[sizeof(T) == 4 ? H : 1], const T *g,
                 const C<T>(&w)[H]) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int vx = wave_idx(p * H + k, N);
      const T gv = gload(g, vx * vx);
      if constexpr (sizeof(T) == 4) {
        acc_add(q[k].x, cx[k], gv * w[k].x);
        acc_add(q[k].y, cy[k], gv * w[k].y);
      } else {
        q[k].x += gv * w[k].x;
        q[k].y += gv * w[k].y;
      }
    }
  };
  for (int r = 0; r < a.Nr; ++r) {
    C<T> w[H];
    const C<T> *src = Cb + (size_t)r * n3;
#pragma unroll
    for (int n = 0; n < H; ++n) w[n] = src[(size_t)(2 * n + p) * N * N + pc];
    fft_pair<N, -1>(w, p);
    acc(Q, Qcx, Qcy, gt + (size_t)r * K2 + kyz, w);
    if (two) acc(Q2, Qcx2, Qcy2, gt2 + (size_t)r * K2 + kyz, w);
  }
  // V1 = iFFT_x QG, and the loss part V2 = iFFT_x(c(|k|) FFT_x Z_q), per served slot
  auto finish = [&](C<T>(&q)[H], T(&cx)[sizeof(T) == 4 ? H : 1], T(&cy)[sizeof(T) == 4 ? H : 1], int sl,
                    const PairDev &pdv) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int k = 0; k < H; ++k) q[k] = C<T>{q[k].x + cx[k], q[k].y + cy[k]};
    }
    fft_pair_dif<N, +1>(q, p);
    C<T> *V = static_cast<C<T> *>(a.V) + (size_t)(node * a.n_pairs + sl) * 2 * n3;
    if (valid) {
#pragma unroll
      for (int k = 0; k < H; ++k) V[(size_t)(2 * k + p) * N * N + pc] = q[k];
    }
    const C<T> *Zq = static_cast<const C<T> *>(a.Z) + ((size_t)node * a.nz + a.zq[sl]) * n3;
#pragma unroll
    for (int n = 0; n < H; ++n) q[n] = Zq[(size_t)(2 * n + p) * N * N + pc];
    fft_pair<N, -1>(q, p);
    const T *ct = static_cast<const T *>(pdv.ctab) + kyz;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int vx = wave_idx(p * H + k, N);
      q[k] = cscale(q[k], gload(ct, vx * vx));
    }
    fft_pair_dif<N, +1>(q, p);
    if (valid) {
#pragma unroll
      for (int k = 0; k < H; ++k) V[n3 + (size_t)(2 * k + p) * N * N + pc] = q[k];
    }
  };
  finish(Q, Qcx, Qcy, slot, pd);
  if (two) finish(Q2, Qcx2, Qcy2, slot2, pd2);
}
// FUSE: one block per gain slot (blockIdx.y over gain slots); else one per slot
template <typename T, int N, bool FUSE>
__global__ void __launch_bounds__(64) k_gain_x(PipeArgs a) {
  gain_x_body<T, N, FUSE>(a, blockIdx.x, FUSE ? gain_eval(a, blockIdx.y) : (int)blockIdx.y, threadIdx.x);
}

// ------------------------------------------------------------------ k_final_yz
// One (node, output, x-plane) per group of 2N threads: Q = sum over the
// output's pair slots of beta Re(iFFT_yz V1 - f^p iFFT_yz V2).  Lane pair
// (c, p): the row pass reads row y = c of V (z = 2n + p) and transforms it
// along z; through LDS the column pass transforms column z = c along y and
// ends with rows y = pH + k, so f^p and the output are accessed coalesced.
template <int N> constexpr int final_groups() { return 128 / (2 * N) > 0 ? 128 / (2 * N) : 1; }

template <typename T, int N, int G>
__device__ __forceinline__ void final_yz_body(const PipeArgs &a, const FinalArgs &fa, int bx, int tid,
                                              C<T> (*lds)[N][N + 1]) {
  constexpr int H = N / 2;
  const int g = tid / (2 * N), l = tid % (2 * N);
  const int c = l >> 1, p = l & 1;
  const int plane = bx * G + g;
  const int jobs = N * a.n_nodes * fa.n_out;
  const bool active = g < G && plane < jobs;
  const int jx = plane % N, job = plane / N;
  const int node = job / fa.n_out, o = job % fa.n_out;
  const size_t n3 = (size_t)N * N * N;
  C<T>(*buf)[N + 1] = lds[g < G ? g : 0];
  double acc[H];
#pragma unroll
  for (int k = 0; k < H; ++k) acc[k] = 0.0;
  const double *f = active ? fa.fsrc[o] + (size_t)node * fa.f_stride + (size_t)jx * N * N : nullptr;
  for (int j = 0; j < fa.qcount; ++j) {
    const int slot = o * fa.qcount + j;
    const int e = node * a.n_pairs + slot;
    const double beta = a.pairs[a.pair_id[slot]].beta;
#pragma unroll
    for (int which = 0; which < 2; ++which) {
      if (active) {
        const C<T> *src = static_cast<const C<T> *>(a.V) + ((size_t)e * 2 + which) * n3 + (size_t)jx * N * N;
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = src[c * N + 2 * n + p];
        fft_pair<N, +1>(h, p);
#pragma unroll
        for (int k = 0; k < H; ++k) buf[c][p * H + k] = h[k];
      }
      group_sync<N>();
      if (active) {
        C<T> h[H];
#pragma unroll
        for (int n = 0; n < H; ++n) h[n] = buf[2 * n + p][c];
        fft_pair<N, +1>(h, p);
        // gain part, then the loss part f^p * Re(ifft(c FTg))
        if (which == 0) {
#pragma unroll
          for (int k = 0; k < H; ++k) acc[k] += beta * (double)h[k].x;
        } else {
#pragma unroll
          for (int k = 0; k < H; ++k) acc[k] -= beta * f[(p * H + k) * N + c] * (double)h[k].x;
        }
      }
      group_sync<N>();
    }
  }
  if (active) {
    double *out = fa.out[o] + (size_t)node * fa.out_stride + (size_t)jx * N * N;
    // the branch is uniform; taken outside the loop, the H reads of the
    // accumulated output are issued together instead of one per store
    if (fa.accumulate) {
      double prev[H];
#pragma unroll
      for (int k = 0; k < H; ++k) prev[k] = out[(p * H + k) * N + c];
#pragma unroll
      for (int k = 0; k < H; ++k) out[(p * H + k) * N + c] = prev[k] + acc[k];
    } else {
#pragma unroll
      for (int k = 0; k < H; ++k) out[(p * H + k) * N + c] = acc[k];
    }
  }
}
template <typename T, int N, int G>
__global__ void __launch_bounds__(G * 2 * N) k_final_yz(PipeArgs a, FinalArgs fa) {
  __shared__ C<T> lds[G][N][N + 1];
  final_yz_body<T, N, G>(a, fa, blockIdx.x, threadIdx.x, lds);
}

}  // namespace dgfs
