// VSS gain tables: b_rm(k) = rho_r^{gamma+2} int_{S^2} (1 + sigma_m.u)^eta
// e^{-i x khat.u} du, x = pi/L rho_r m_q/(m_p+m_q) |k| (Eq. Fkr_vss with the
// sphere integral in closed form by the Funk-Hecke theorem):
//   4 pi sum_n a_n (-i)^n j_n(x) P_n(sigma_m . khat),
//   a_n = (2n+1)/2 int_{-1}^{1} (1+t)^eta P_n(t) dt
//       = (2n+1)/2 2^{eta+1} eta(eta-1)..(eta-n+1) / ((eta+1)(eta+2)..(eta+n+1)).
// j_n(x) for every (r, |k|^2) is computed on the host by Miller's downward
// recurrence; the sum over n and the Legendre recurrence run on the GPU in
// FP64.  Stored per pair as w_r w_m b_rm(k) / N^3 in the compute type.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace dgfs {

// j_0..j_nmax at x >= 0: downward recurrence j_{n-1} = (2n+1)/x j_n - j_{n+1}
// from well above max(nmax, x), scaled to whichever of j_0, j_1 is larger.
static void spherical_bessel(int nmax, double x, double *out) {
  for (int n = 0; n <= nmax; ++n) out[n] = 0.0;
  if (x == 0.0) {
    out[0] = 1.0;
    return;
  }
  const int start = nmax + (int)x + 40;
  std::vector<double> v(start + 2, 0.0);
  double jp1 = 0.0, jn = 1e-250;
  v[start] = jn;
  for (int n = start; n >= 1; --n) {
    double jm1 = (2.0 * n + 1.0) / x * jn - jp1;
    jp1 = jn;
    jn = jm1;
    v[n - 1] = jn;
    if (std::fabs(jn) > 1e200) {  // rescale everything computed so far
      for (int k = n - 1; k <= start; ++k) v[k] *= 1e-200;
      jn *= 1e-200;
      jp1 *= 1e-200;
    }
  }
  const double j0 = std::sin(x) / x, j1 = std::sin(x) / (x * x) - std::cos(x) / x;
  const double scale = std::fabs(j0) >= std::fabs(j1) ? j0 / v[0] : j1 / v[1];
  for (int n = 0; n <= nmax; ++n) out[n] = v[n] * scale;
}

static void funk_hecke(double eta, int nmax, std::vector<double> &a) {
  a.assign(nmax + 1, 0.0);
  double ratio = 1.0 / (eta + 1.0);  // eta(eta-1)..(eta-n+1) / ((eta+1)..(eta+n+1)) at n = 0
  for (int n = 0; n <= nmax; ++n) {
    a[n] = 0.5 * (2.0 * n + 1.0) * std::pow(2.0, eta + 1.0) * ratio;
    ratio *= (eta - n) / (eta + n + 2.0);
  }
}

struct VssTabArgs {
  int N, M, K2, nmax;
  const double *J;      // [K2][nmax+1] for one r
  const double *an;     // [nmax+1]
  const double *sigma;  // [M][3]
  const double *wm;     // [M]
  double scale;         // w_r rho_r^{gamma+2} 4 pi / N^3
};

template <typename T>
__global__ void k_vss_table(VssTabArgs a, T *out /* [M][N^3] complex for one r */) {
  const int N = a.N;
  const int n3 = N * N * N;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (idx >= n3) return;
  const int i = idx / (N * N), j = (idx / N) % N, l = idx % N;
  const int vx = i < N / 2 ? i : i - N, vy = j < N / 2 ? j : j - N, vz = l < N / 2 ? l : l - N;
  const int k2 = vx * vx + vy * vy + vz * vz;
  const double kk = sqrt((double)k2);
  const double *s = a.sigma + 3 * m;
  const double t = k2 == 0 ? 1.0 : (s[0] * vx + s[1] * vy + s[2] * vz) / kk;
  const double *J = a.J + (size_t)k2 * (a.nmax + 1);
  double re = 0.0, im = 0.0, pm1 = 0.0, pn = 1.0;
  for (int n = 0; n <= a.nmax; ++n) {
    const double term = a.an[n] * J[n] * pn;
    switch (n & 3) {  // (-i)^n = 1, -i, -1, i
      case 0: re += term; break;
      case 1: im -= term; break;
      case 2: re -= term; break;
      default: im += term; break;
    }
    const double pn1 = ((2.0 * n + 1.0) * t * pn - n * pm1) / (n + 1.0);
    pm1 = pn;
    pn = pn1;
  }
  const double sc = a.scale * a.wm[m];
  out[2 * ((size_t)m * n3 + idx)] = (T)(sc * re);
  out[2 * ((size_t)m * n3 + idx) + 1] = (T)(sc * im);
}

dgfs_status build_vss_tables(dgfs_plan_s *pl) {
  const int N = pl->N, M = pl->M, Nr = pl->Nr, ns = pl->ns, K2 = pl->K2();
  const size_t n3 = (size_t)N * N * N, per_pair = (size_t)Nr * M * n3 * 2 * pl->elt();
  const int npair = ns * ns;
  hipError_t e = hipMalloc(&pl->vss_dev, per_pair * npair);
  if (e != hipSuccess) {
    set_error("VSS tables: hipMalloc(%zu) failed: %s", per_pair * npair, hipGetErrorString(e));
    return DGFS_ENOMEM;
  }
  double *dJ = nullptr, *dA = nullptr, *dS = nullptr, *dW = nullptr;
  auto fail = [&](hipError_t err, const char *what) {
    if (dJ) (void)hipFree(dJ);
    if (dA) (void)hipFree(dA);
    if (dS) (void)hipFree(dS);
    if (dW) (void)hipFree(dW);
    (void)hipFree(pl->vss_dev);
    pl->vss_dev = nullptr;
    return hip_status(err, what);
  };
  if ((e = hipMalloc(&dS, M * 3 * sizeof(double))) != hipSuccess) return fail(e, "VSS tables");
  if ((e = hipMalloc(&dW, M * sizeof(double))) != hipSuccess) return fail(e, "VSS tables");
  if ((e = hipMemcpy(dS, pl->sigma.data(), M * 3 * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "VSS tables");
  if ((e = hipMemcpy(dW, pl->wsig.data(), M * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "VSS tables");
  const double kmax = std::sqrt((double)(K2 - 1));
  for (int pr = 0; pr < npair; ++pr) {
    const PairHost &ph = pl->pairs[pr];
    const double aq = ph.mq / (ph.mp + ph.mq);
    const double xmax = M_PI / pl->L * ph.R * aq * kmax;
    const int nmax = (int)std::ceil(xmax) + (int)(16.0 * std::cbrt(xmax)) + 32;
    std::vector<double> an, J((size_t)K2 * (nmax + 1));
    funk_hecke(ph.eta, nmax, an);
    if ((e = hipMalloc(&dA, an.size() * sizeof(double))) != hipSuccess) return fail(e, "VSS tables");
    if ((e = hipMalloc(&dJ, J.size() * sizeof(double))) != hipSuccess) return fail(e, "VSS tables");
    if ((e = hipMemcpy(dA, an.data(), an.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "VSS tables");
    char *dst = static_cast<char *>(pl->vss_dev) + pr * per_pair;
    for (int r = 0; r < Nr; ++r) {
      for (int k2 = 0; k2 < K2; ++k2)
        spherical_bessel(nmax, M_PI / pl->L * ph.rho[r] * aq * std::sqrt((double)k2), &J[(size_t)k2 * (nmax + 1)]);
      if ((e = hipMemcpy(dJ, J.data(), J.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "VSS tables");
      VssTabArgs ta{N, M, K2, nmax, dJ, dA, dS, dW, ph.wrho[r] * std::pow(ph.rho[r], ph.gamma + 2.0) * 4.0 * M_PI / (double)n3};
      const dim3 grid((unsigned)((n3 + 255) / 256), M);
      char *rdst = dst + (size_t)r * M * n3 * 2 * pl->elt();
      if (pl->precision == DGFS_FP64) hipLaunchKernelGGL(k_vss_table<double>, grid, dim3(256), 0, 0, ta, (double *)rdst);
      else hipLaunchKernelGGL(k_vss_table<float>, grid, dim3(256), 0, 0, ta, (float *)rdst);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e, "VSS table kernel");
      if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "VSS table kernel");
    }
    (void)hipFree(dA);
    (void)hipFree(dJ);
    dA = dJ = nullptr;
    pl->pair_host[pr].btab = dst;
  }
  (void)hipFree(dS);
  (void)hipFree(dW);
  return DGFS_OK;
}

}  // namespace dgfs
