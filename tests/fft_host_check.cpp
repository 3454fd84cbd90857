// Host check of the register FFTs (fft.hpp): every length the library
// instantiates, and the radix-5/7 sub-lengths, against a direct DFT in long
// double.  Prints one line per length: N, max error forward, inverse.
#include "../paper_1903_04670_amd/csrc/fft.hpp"

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>

using namespace dgfs;

template <int N, int DIR> double check() {
  cplx<double> x[N];
  std::complex<long double> in[N];
  std::srand(N * 7 + DIR + 3);
  for (int i = 0; i < N; ++i) {
    const double a = std::rand() / (double)RAND_MAX - 0.5, b = std::rand() / (double)RAND_MAX - 0.5;
    in[i] = {a, b};
    x[i] = {a, b};
  }
  fft<N, DIR>(x);
  double err = 0;
  for (int k = 0; k < N; ++k) {
    std::complex<long double> s = 0;
    for (int n = 0; n < N; ++n) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)((n * k) % N) / N;
      s += in[n] * std::complex<long double>(cosl(ang), DIR * sinl(ang));
    }
    err = std::fmax(err, (double)std::abs(std::complex<long double>(x[k].x, x[k].y) - s));
  }
  return err;
}

template <int N> void line() { std::printf("%d %.3e %.3e\n", N, check<N, -1>(), check<N, 1>()); }

int main() {
  line<2>(); line<3>(); line<4>(); line<5>(); line<6>(); line<7>(); line<8>(); line<10>(); line<12>();
  line<14>(); line<16>(); line<18>(); line<20>(); line<24>(); line<28>(); line<32>(); line<36>();
  line<40>(); line<48>(); line<56>();
  return 0;
}
