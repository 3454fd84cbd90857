// Register-resident 1-D complex FFTs of compile-time length for gfx950.
//
// One thread owns one pencil of N complex values and transforms it with a
// fully unrolled mixed-radix decimation-in-time recursion (radix 4, 2, 3, 5
// and 7 codelets).  Twiddle factors are compile-time constants produced by a
// constexpr sine/cosine (octant reduction on the exact rational angle j/n,
// then Taylor series on [0, pi/4]), so no table is read at run time.
//
// Sign convention: DIR = -1 is the forward transform sum_n x_n e^{-2 pi i nk/N},
// DIR = +1 the inverse without the 1/N factor.
#pragma once
#include <hip/hip_runtime.h>

#define DGFS_HD __host__ __device__ __forceinline__

namespace dgfs {

template <typename T> struct alignas(2 * sizeof(T)) cplx { T x, y; };

template <typename T> DGFS_HD cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> DGFS_HD cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> DGFS_HD cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> DGFS_HD cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by DIR * i  (i.e. -i for the forward transform)
template <int DIR, typename T> DGFS_HD cplx<T> mul_dir_i(cplx<T> a) {
  if constexpr (DIR > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// ---------------------------------------------------------------- constexpr sin/cos
namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double taylor_sin(double x) {
  // x - x^3/3! + ... up to x^25/25!, Horner form
  double x2 = x * x, s = 0.0;
  for (int k = 12; k >= 1; --k) s = (1.0 - s * x2 / ((2.0 * k) * (2.0 * k + 1.0)));
  // the loop above builds 1 - x^2/(2*3)(1 - x^2/(4*5)(...)) ; multiply by x
  return x * s;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, s = 0.0;
  for (int k = 12; k >= 1; --k) s = (1.0 - s * x2 / ((2.0 * k - 1.0) * (2.0 * k)));
  return s;
}
struct SC { double s, c; };
// sin and cos of 2 pi num/den for integers 0 <= num < den (any den > 0)
constexpr SC sincos2pi(long long num, long long den) {
  num %= den;
  if (num < 0) num += den;
  // f = num/den in [0,1)
  if (2 * num >= den) {  // f - 1/2
    SC r = sincos2pi(2 * num - den, 2 * den);
    return {-r.s, -r.c};
  }
  if (4 * num >= den) {  // f - 1/4 in [0, 1/4)
    SC r = sincos2pi(4 * num - den, 4 * den);
    return {r.c, -r.s};
  }
  if (8 * num > den) {  // 1/4 - f in [0, 1/8)
    SC r = sincos2pi(den - 4 * num, 4 * den);
    return {r.c, r.s};
  }
  double x = 2.0 * kPi * (double)num / (double)den;
  return {taylor_sin(x), taylor_cos(x)};
}
}  // namespace ct

// W_N^{DIR * e} = exp(DIR * 2 pi i e / N) applied to a
template <int N, int DIR, int E, typename T>
DGFS_HD cplx<T> twiddle(cplx<T> a) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (4 * e == N) {  // exp(DIR i pi/2) = DIR i
    return mul_dir_i<DIR>(a);
  } else if constexpr (2 * e == N) {
    return {-a.x, -a.y};
  } else if constexpr (4 * e == 3 * N) {
    return mul_dir_i<-DIR>(a);
  } else {
    constexpr ct::SC sc = ct::sincos2pi(e, N);
    constexpr T c = (T)sc.c;
    constexpr T s = (T)(DIR * sc.s);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <typename T> DGFS_HD T fmaT(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// (a, b) <- (a + W_N^{DIR E} b, a - W_N^{DIR E} b).  With a general twiddle
// the sum takes two fused multiply-adds per component and the difference
// one more, as 2a - (a + W b): three instructions per component instead of a
// twiddle product, an add and a subtract (four).
template <int N, int DIR, int E, typename T>
DGFS_HD void tw_butterfly(cplx<T> &a, cplx<T> &b) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0 || 4 * e == N || 2 * e == N || 4 * e == 3 * N) {
    const cplx<T> t = twiddle<N, DIR, E>(b);
    b = csub(a, t);
    a = cadd(a, t);
  } else {
    constexpr ct::SC sc = ct::sincos2pi(e, N);
    constexpr T c = (T)sc.c;
    constexpr T s = (T)(DIR * sc.s);
    const cplx<T> sum{fmaT(b.x, c, fmaT(-b.y, s, a.x)), fmaT(b.x, s, fmaT(b.y, c, a.y))};
    b = cplx<T>{fmaT((T)2, a.x, -sum.x), fmaT((T)2, a.y, -sum.y)};
    a = sum;
  }
}

// ---------------------------------------------------------------- codelets
template <int DIR, typename T>
DGFS_HD void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename T>
DGFS_HD void dft3(cplx<T>& a, cplx<T>& b, cplx<T>& c) {
  constexpr T h = (T)0.8660254037844386467637231707529362;  // sqrt(3)/2
  cplx<T> t1 = cadd(b, c);
  cplx<T> t2 = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
  cplx<T> d = csub(b, c);
  cplx<T> t3 = mul_dir_i<DIR>(cplx<T>{h * d.x, h * d.y});
  a = cadd(a, t1);
  b = cadd(t2, t3);
  c = csub(t2, t3);
}

template <int DIR, typename T>
DGFS_HD void dft4(cplx<T>& a, cplx<T>& b, cplx<T>& c, cplx<T>& d) {
  cplx<T> s0 = cadd(a, c), s1 = csub(a, c);
  cplx<T> s2 = cadd(b, d), s3 = mul_dir_i<DIR>(csub(b, d));
  a = cadd(s0, s2);
  c = csub(s0, s2);
  b = cadd(s1, s3);
  d = csub(s1, s3);
}

// Odd-length R-point DFT (R = 5, 7) in place.  Inputs n and R - n are
// paired: with s_n = y_n + y_{R-n} and d_n = y_n - y_{R-n},
//   Y_k     = y_0 + sum_n s_n cos(2 pi nk/R) + DIR i sum_n d_n sin(2 pi nk/R)
//   Y_{R-k} = the same with the sine sum's sign flipped,
// for n, k = 1 .. (R-1)/2; the constants are compile-time.
namespace detail {
template <int R, int K, int NN, typename T>
DGFS_HD void odd_terms(const cplx<T> (&s)[R], const cplx<T> (&d)[R], cplx<T> &a, cplx<T> &b) {
  if constexpr (NN <= (R - 1) / 2) {
    constexpr ct::SC sc = ct::sincos2pi((long long)NN * K, R);
    constexpr T c = (T)sc.c, sn = (T)sc.s;
    a = cplx<T>{a.x + c * s[NN].x, a.y + c * s[NN].y};
    b = cplx<T>{b.x + sn * d[NN].x, b.y + sn * d[NN].y};
    odd_terms<R, K, NN + 1>(s, d, a, b);
  }
}
template <int R, int DIR, int K, typename T>
DGFS_HD void odd_outputs(const cplx<T> &y0, const cplx<T> (&s)[R], const cplx<T> (&d)[R], cplx<T> (&out)[R]) {
  if constexpr (K <= (R - 1) / 2) {
    cplx<T> a = y0, b{(T)0, (T)0};
    odd_terms<R, K, 1>(s, d, a, b);
    const cplx<T> ib = mul_dir_i<DIR>(b);
    out[K] = cadd(a, ib);
    out[R - K] = csub(a, ib);
    odd_outputs<R, DIR, K + 1>(y0, s, d, out);
  }
}
}  // namespace detail

template <int R, int DIR, typename T>
DGFS_HD void dft_odd(cplx<T> (&y)[R]) {
  static_assert(R % 2 == 1 && R >= 5, "odd codelet");
  cplx<T> s[R], d[R], out[R];
  cplx<T> sum = y[0];
#pragma unroll
  for (int n = 1; n <= (R - 1) / 2; ++n) {
    s[n] = cadd(y[n], y[R - n]);
    d[n] = csub(y[n], y[R - n]);
    sum = cadd(sum, s[n]);
  }
  out[0] = sum;
  detail::odd_outputs<R, DIR, 1>(y[0], s, d, out);
#pragma unroll
  for (int k = 0; k < R; ++k) y[k] = out[k];
}

template <int N> constexpr int first_radix() {
  if constexpr (N % 4 == 0) return 4;
  else if constexpr (N % 2 == 0) return 2;
  else if constexpr (N % 3 == 0) return 3;
  else if constexpr (N % 5 == 0) return 5;
  else if constexpr (N % 7 == 0) return 7;
  else return 0;
}

// In-place DFT of a strided register view: elements x[OFF + STRIDE * n], n < N.
template <int N, int DIR, int OFF, int STRIDE, int LEN, typename T>
struct FFTView {
  static DGFS_HD void run(cplx<T> (&x)[LEN]) {
    if constexpr (N == 1) {
    } else if constexpr (N == 2) {
      dft2<DIR>(x[OFF], x[OFF + STRIDE]);
    } else if constexpr (N == 3) {
      dft3<DIR>(x[OFF], x[OFF + STRIDE], x[OFF + 2 * STRIDE]);
    } else if constexpr (N == 4) {
      dft4<DIR>(x[OFF], x[OFF + STRIDE], x[OFF + 2 * STRIDE], x[OFF + 3 * STRIDE]);
    } else if constexpr (N == 5 || N == 7) {
      cplx<T> y[N];
#pragma unroll
      for (int n = 0; n < N; ++n) y[n] = x[OFF + STRIDE * n];
      dft_odd<N, DIR>(y);
#pragma unroll
      for (int n = 0; n < N; ++n) x[OFF + STRIDE * n] = y[n];
    } else {
      constexpr int R = first_radix<N>();
      static_assert(R > 0, "unsupported FFT length");
      constexpr int M = N / R;
      // sub-transforms of the R decimated sequences x[OFF + STRIDE*(R*n1 + n2)]
      run_subs<0, R, M>(x);
      // twiddle and R-point butterflies; results land in digit-reversed slots
      combine<0, R, M>(x);
      // permute from [n2-major] layout to natural order
      permute<R, M>(x);
    }
  }
  template <int n2, int R, int M>
  static DGFS_HD void run_subs(cplx<T> (&x)[LEN]) {
    if constexpr (n2 < R) {
      FFTView<M, DIR, OFF + STRIDE * n2, STRIDE * R, LEN, T>::run(x);
      run_subs<n2 + 1, R, M>(x);
    }
  }
  // after run_subs, sub-transform n2 holds X_{n2}[k1] at x[OFF + STRIDE*(n2 + R*k1)]
  template <int k1, int R, int M>
  static DGFS_HD void combine(cplx<T> (&x)[LEN]) {
    if constexpr (k1 < M) {
      cplx<T> y[R];
      if constexpr (R == 2) {
        // the twiddle product feeds the butterfly (tw_butterfly)
        y[0] = x[OFF + STRIDE * (2 * k1)];
        y[1] = x[OFF + STRIDE * (1 + 2 * k1)];
        tw_butterfly<N, DIR, k1>(y[0], y[1]);
      } else if constexpr (R == 4) {
        // dft4 of (y0, W^k1 y1, W^2k1 y2, W^3k1 y3) with the products of
        // y2 and y3 fused into the butterflies that consume them
        y[0] = x[OFF + STRIDE * (4 * k1)];
        y[1] = twiddle<N, DIR, k1>(x[OFF + STRIDE * (1 + 4 * k1)]);
        y[2] = x[OFF + STRIDE * (2 + 4 * k1)];
        y[3] = x[OFF + STRIDE * (3 + 4 * k1)];
        tw_butterfly<N, DIR, 2 * k1>(y[0], y[2]);  // a + c, a - c
        tw_butterfly<N, DIR, 3 * k1>(y[1], y[3]);  // b + d, b - d
        const cplx<T> s0 = y[0], s1 = y[2], s2 = y[1], s3 = mul_dir_i<DIR>(y[3]);
        y[0] = cadd(s0, s2);
        y[2] = csub(s0, s2);
        y[1] = cadd(s1, s3);
        y[3] = csub(s1, s3);
      } else {
        load_tw<0, k1, R, M>(x, y);
        if constexpr (R == 3) dft3<DIR>(y[0], y[1], y[2]);
        else dft_odd<R, DIR>(y);
      }
      store_back<0, k1, R>(x, y);
      combine<k1 + 1, R, M>(x);
    }
  }
  template <int n2, int k1, int R, int M>
  static DGFS_HD void load_tw(cplx<T> (&x)[LEN], cplx<T> (&y)[R]) {
    if constexpr (n2 < R) {
      y[n2] = twiddle<N, DIR, n2 * k1>(x[OFF + STRIDE * (n2 + R * k1)]);
      load_tw<n2 + 1, k1, R, M>(x, y);
    }
  }
  // output k = k1 + M*k2 is stored (temporarily) in slot n2 := k2 of column k1
  template <int k2, int k1, int R>
  static DGFS_HD void store_back(cplx<T> (&x)[LEN], cplx<T> (&y)[R]) {
    if constexpr (k2 < R) {
      x[OFF + STRIDE * (k2 + R * k1)] = y[k2];
      store_back<k2 + 1, k1, R>(x, y);
    }
  }
  // slot (k2 + R*k1) holds X[k1 + M*k2]; move to natural order
  template <int R, int M>
  static DGFS_HD void permute(cplx<T> (&x)[LEN]) {
    cplx<T> tmp[N];
    copy_out<0, R, M>(x, tmp);
    copy_in<0>(x, tmp);
  }
  template <int j, int R, int M>
  static DGFS_HD void copy_out(cplx<T> (&x)[LEN], cplx<T> (&tmp)[N]) {
    if constexpr (j < N) {
      constexpr int k2 = j % R, k1 = j / R;
      tmp[k1 + M * k2] = x[OFF + STRIDE * j];
      copy_out<j + 1, R, M>(x, tmp);
    }
  }
  template <int j>
  static DGFS_HD void copy_in(cplx<T> (&x)[LEN], cplx<T> (&tmp)[N]) {
    if constexpr (j < N) {
      x[OFF + STRIDE * j] = tmp[j];
      copy_in<j + 1>(x, tmp);
    }
  }
};

template <int N, int DIR, typename T>
DGFS_HD void fft(cplx<T> (&x)[N]) {
  FFTView<N, DIR, 0, 1, N, T>::run(x);
}


// ---------------------------------------------------------------- paired lanes
// A length-N transform split over two adjacent lanes (lane parity p): on
// entry each lane holds its decimated half x[2n + p], n < N/2; on exit lane p
// holds X[p N/2 + k], k < N/2.  The two halves are combined by one radix-2
// stage whose partner values come through a DPP quad permutation [1,0,3,2]
// (lane t <-> lane t^1), so no LDS is used.
namespace detail {
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_pair(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int N, int DIR, int K, int H, typename T>
struct TwHalf {
  static DGFS_HD void run(cplx<T> (&h)[H]) {
    if constexpr (K < H) {
      h[K] = twiddle<N, DIR, K>(h[K]);
      TwHalf<N, DIR, K + 1, H, T>::run(h);
    }
  }
};
}  // namespace detail

template <int N, int DIR, typename T>
__device__ __forceinline__ void fft_pair(cplx<T> (&h)[N / 2], int p) {
  static_assert(N % 2 == 0, "paired transform needs even N");
  fft<N / 2, DIR>(h);
  if (p) detail::TwHalf<N, DIR, 0, N / 2, T>::run(h);
  const T sg = p ? (T)-1 : (T)1;
#pragma unroll
  for (int k = 0; k < N / 2; ++k) {
    const cplx<T> o{detail::swap_pair(h[k].x), detail::swap_pair(h[k].y)};
    h[k] = cplx<T>{sg * h[k].x + o.x, sg * h[k].y + o.y};
  }
}

// Decimation-in-frequency counterpart: on entry lane p holds x[p N/2 + n]
// (natural halves), on exit lane p holds X[2k + p] (decimated).
template <int N, int DIR, typename T>
__device__ __forceinline__ void fft_pair_dif(cplx<T> (&h)[N / 2], int p) {
  static_assert(N % 2 == 0, "paired transform needs even N");
  const T sg = p ? (T)-1 : (T)1;
#pragma unroll
  for (int n = 0; n < N / 2; ++n) {
    const cplx<T> o{detail::swap_pair(h[n].x), detail::swap_pair(h[n].y)};
    // lane 0: x[n] + x[n+N/2]; lane 1: x[n] - x[n+N/2] (then twiddled)
    h[n] = cplx<T>{o.x + sg * h[n].x, o.y + sg * h[n].y};
  }
  if (p) detail::TwHalf<N, DIR, 0, N / 2, T>::run(h);
  fft<N / 2, DIR>(h);
}

}  // namespace dgfs
