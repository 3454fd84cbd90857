// Host side of libdgfs: parameter validation, the tables of Algorithm 1
// evaluated in closed form, sphere sets, error state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace dgfs {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

dgfs_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return DGFS_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return DGFS_EHIP;
}

// Gauss-Legendre rule on [-1, 1] by Newton's method on P_n, nodes ascending.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

static double sinc(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }

static int wave(int j, int N) { return j < N / 2 ? j : j - N; }

bool dg_setup(int P, std::vector<double> &r, std::vector<double> &Dr, std::vector<double> &Minv);
dgfs_status build_vss_tables(dgfs_plan_s *pl);
void load_tuned(dgfs_plan_s *pl);
bool projection_ginv(const dgfs_plan_s *pl, const std::vector<int> &species, std::vector<double> &G);

}  // namespace dgfs

using namespace dgfs;

extern "C" const char *dgfs_last_error(void) { return g_err; }

extern "C" dgfs_status dgfs_sphere_set(int32_t kind, int32_t M, double *sigma, double *w) {
  if (!sigma || !w) { set_error("dgfs_sphere_set: NULL output"); return DGFS_EINVAL; }
  if (kind == 0) {
    if (M != 6) { set_error("octahedron has M = 6"); return DGFS_EINVAL; }
    const double s[18] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    std::memcpy(sigma, s, sizeof(s));
  } else if (kind == 1) {
    if (M != 12) { set_error("icosahedron has M = 12"); return DGFS_EINVAL; }
    const double phi = 0.5 * (1.0 + std::sqrt(5.0)), nrm = std::sqrt(1.0 + phi * phi);
    int k = 0;
    for (double a : {1.0, -1.0})
      for (double b : {phi, -phi}) {
        const double v[3][3] = {{0, a, b}, {a, b, 0}, {b, 0, a}};
        for (int i = 0; i < 3; ++i) {
          for (int d = 0; d < 3; ++d) sigma[3 * k + d] = v[i][d] / nrm;
          ++k;
        }
      }
  } else if (kind == 2) {
    if (M < 1) { set_error("Fibonacci set needs M >= 1"); return DGFS_EINVAL; }
    for (int i = 0; i < M; ++i) {
      double z = 1.0 - (2.0 * i + 1.0) / M, az = i * M_PI * (3.0 - std::sqrt(5.0));
      double rxy = std::sqrt(std::max(0.0, 1.0 - z * z));
      sigma[3 * i] = rxy * std::cos(az);
      sigma[3 * i + 1] = rxy * std::sin(az);
      sigma[3 * i + 2] = z;
    }
  } else {
    set_error("unknown sphere set kind %d", kind);
    return DGFS_EINVAL;
  }
  for (int i = 0; i < M; ++i) w[i] = 4.0 * M_PI / M;
  return DGFS_OK;
}

// The grid sizes the kernels are instantiated for: the even N = 2^a 3^b up
// to 48, and 10, 14, 40, 56 (radix-5 and radix-7 transforms).
static bool supported_N(int N) {
  for (int n : {4, 6, 8, 10, 12, 14, 16, 18, 24, 32, 36, 40, 48, 56})
    if (N == n) return true;
  return false;
}

extern "C" dgfs_status dgfs_plan_create(const dgfs_params *prm, dgfs_plan *out) {
  if (!prm || !out) { set_error("dgfs_plan_create: NULL argument"); return DGFS_EINVAL; }
  *out = nullptr;
  const int ns = prm->n_species;
  if (ns < 1 || ns > DGFS_MAX_SPECIES) { set_error("n_species = %d outside [1, %d]", ns, DGFS_MAX_SPECIES); return DGFS_EINVAL; }
  if (!prm->mass || !prm->omega || !prm->alpha) { set_error("mass, omega and alpha are required"); return DGFS_EINVAL; }
  if (prm->N < 2 || prm->N % 2) { set_error("N = %d must be even and >= 4", prm->N); return DGFS_EINVAL; }
  if (!supported_N(prm->N)) { set_error("N = %d not supported (4, 6, 8, 10, 12, 14, 16, 18, 24, 32, 36, 40, 48, 56)", prm->N); return DGFS_EUNSUPPORTED; }
  if (!(prm->L > 0.0)) { set_error("L must be > 0"); return DGFS_EINVAL; }
  if (prm->M < 1 || !prm->sigma || !prm->w_sigma) { set_error("M >= 1 with sigma and w_sigma required"); return DGFS_EINVAL; }
  if (prm->N_rho < 1) { set_error("N_rho = %d must be >= 1", prm->N_rho); return DGFS_EINVAL; }
  if (prm->dg_order < 0 || prm->dg_order > 8) { set_error("dg_order = %d outside [0, 8]", prm->dg_order); return DGFS_EINVAL; }
  if (prm->precision != DGFS_FP64 && prm->precision != DGFS_FP32_MIXED) { set_error("unknown precision %d", prm->precision); return DGFS_EINVAL; }
  if (prm->nyquist_zero != 0 && prm->nyquist_zero != 1) { set_error("nyquist_zero = %d must be 0 or 1", prm->nyquist_zero); return DGFS_EINVAL; }
  for (int p = 0; p < ns; ++p)
    if (!(prm->mass[p] > 0.0)) { set_error("mass[%d] must be > 0", p); return DGFS_EINVAL; }
  for (int i = 0; i < ns * ns; ++i) {
    if (!(prm->alpha[i] > 0.0)) { set_error("alpha[%d] must be > 0", i); return DGFS_EINVAL; }
    if (!(prm->omega[i] < 2.5)) { set_error("omega[%d] must be < 2.5", i); return DGFS_EINVAL; }
    if (prm->R && !(prm->R[i] > 0.0)) { set_error("R[%d] must be > 0", i); return DGFS_EINVAL; }
    if (!prm->beta && prm->kn && !(prm->kn[i] > 0.0)) { set_error("kn[%d] must be > 0", i); return DGFS_EINVAL; }
  }
  for (int m = 0; m < prm->M; ++m) {
    const double *s = prm->sigma + 3 * m;
    double n2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    if (std::fabs(n2 - 1.0) > 1e-12) { set_error("sigma[%d] is not a unit vector", m); return DGFS_EINVAL; }
  }

  auto *pl = new dgfs_plan_s();
  pl->ns = ns;
  pl->N = prm->N;
  pl->M = prm->M;
  pl->Nr = prm->N_rho;
  pl->P = prm->dg_order;
  pl->precision = prm->precision;
  pl->nyquist_zero = prm->nyquist_zero != 0;
  pl->L = prm->L;
  pl->S = prm->S;
  pl->mass.assign(prm->mass, prm->mass + ns);
  pl->sigma.assign(prm->sigma, prm->sigma + 3 * prm->M);
  pl->wsig.assign(prm->w_sigma, prm->w_sigma + prm->M);
  const int N = pl->N, M = pl->M, Nr = pl->Nr;

  // group directions by sigma_x (exactly equal values share x transforms)
  for (int m = 0; m < M; ++m) {
    double sx = pl->sigma[3 * m];
    int found = -1;
    for (int s = 0; s < pl->Sx; ++s)
      if (std::fabs(pl->sx_val[s] - sx) <= 1e-15) found = s;
    if (found < 0) {
      pl->sx_val.push_back(sx);
      found = pl->Sx++;
    }
    pl->sx_idx.push_back(found);
  }

  std::vector<double> glx, glw;
  gauss_legendre(Nr, glx, glw);
  pl->pairs.resize(ns * ns);
  for (int p = 0; p < ns; ++p)
    for (int q = 0; q < ns; ++q) {
      PairHost &ph = pl->pairs[p * ns + q];
      ph.mp = pl->mass[p];
      ph.mq = pl->mass[q];
      ph.omega = prm->omega[p * ns + q];
      ph.alpha = prm->alpha[p * ns + q];
      ph.gamma = 2.0 * (1.0 - ph.omega);  // |u|^{2(1-omega)} of Eq. (VSSNonDim)
      ph.eta = ph.alpha - 1.0;
      if (std::fabs(ph.eta) > 0.0) pl->vhs = false;
      double mu = ph.mp * ph.mq / (ph.mp + ph.mq);
      double shape = std::pow(mu, 0.5 - ph.omega) * ph.alpha /
                     (std::pow(2.0, 1.0 + ph.alpha) * std::tgamma(2.5 - ph.omega) * M_PI);
      if (prm->beta) ph.beta = prm->beta[p * ns + q];
      else if (prm->kn) ph.beta = shape / (prm->kn[p * ns + q] * std::sqrt(1.0 + ph.mp / ph.mq));
      else ph.beta = shape;
      ph.R = prm->R ? prm->R[p * ns + q]
                    : 4.0 * pl->L / (1.0 + std::max(4.0 * ph.mq / (ph.mp + ph.mq), 2.0) + std::sqrt(1.0 + ph.mq / ph.mp));
      ph.rho.resize(Nr);
      ph.wrho.resize(Nr);
      for (int r = 0; r < Nr; ++r) {
        ph.rho[r] = 0.5 * ph.R * (glx[r] + 1.0);
        ph.wrho[r] = 0.5 * ph.R * glw[r];
      }
    }

  // ---- tables, built in FP64 on the host
  const int K2 = pl->K2(), Sx = pl->Sx, npair = ns * ns;
  const double n3 = (double)N * N * N;
  const size_t szPX = (size_t)2 * Nr * Sx * N, szPYZ = (size_t)2 * Nr * M * 2 * N;
  const size_t szG = (size_t)Nr * K2, szC = (size_t)K2;
  std::vector<double> hostbuf;  // complex tables as (re, im) pairs, real tables plain
  std::vector<size_t> off_px(npair), off_pyz(npair), off_g(npair), off_c(npair);
  auto push = [&](size_t n) { size_t o = hostbuf.size(); hostbuf.resize(o + n); return o; };
  pl->ctab_host.resize(npair);
  for (int pr = 0; pr < npair; ++pr) {
    const PairHost &ph = pl->pairs[pr];
    const double aq = ph.mq / (ph.mp + ph.mq), ap = ph.mp / (ph.mp + ph.mq);
    off_px[pr] = push(2 * szPX);
    off_pyz[pr] = push(2 * szPYZ);
    off_g[pr] = push(szG);
    off_c[pr] = push(szC);
    for (int side = 0; side < 2; ++side)
      for (int r = 0; r < Nr; ++r) {
        // side 0 (f^p): e^{+i (pi/L) rho m_q/(m_p+m_q) v sigma}; side 1 (f^q): e^{-i (pi/L) rho m_p/(m_p+m_q) v sigma}
        const double th = side == 0 ? M_PI / pl->L * ph.rho[r] * aq : -M_PI / pl->L * ph.rho[r] * ap;
        for (int s = 0; s < Sx; ++s)
          for (int j = 0; j < N; ++j) {
            double a = th * pl->sx_val[s] * wave(j, N);
            size_t o = off_px[pr] + 2 * ((((size_t)side * Nr + r) * Sx + s) * N + j);
            // with nyquist_zero the twiddle is 0 on the Nyquist plane of its
            // axis: the three axes' zeros together mask fft(f) as required
            const double keep = pl->nyquist_zero && j == N / 2 ? 0.0 : 1.0;
            hostbuf[o] = keep * std::cos(a) / n3;
            hostbuf[o + 1] = keep * std::sin(a) / n3;
          }
        for (int m = 0; m < M; ++m)
          for (int ax = 0; ax < 2; ++ax)
            for (int j = 0; j < N; ++j) {
              double a = th * pl->sigma[3 * m + 1 + ax] * wave(j, N);
              size_t o = off_pyz[pr] + 2 * (((((size_t)side * Nr + r) * M + m) * 2 + ax) * N + j);
              const double keep = pl->nyquist_zero && j == N / 2 ? 0.0 : 1.0;
              hostbuf[o] = keep * std::cos(a);
              hostbuf[o + 1] = keep * std::sin(a);
            }
      }
    // VHS gain table: b_r(k) = rho_r^{gamma+2} 4 pi sinc(pi/L rho_r a_q |k|) (Eq. Fkr_vss with alpha = 1)
    // loss table: c(k) = sum_r w_r rho_r^{gamma+2} C_eta 4 pi sinc(pi/L rho_r |k|) (Eq. Gmm_vss)
    const double Ceta = 2.0 * M_PI * std::pow(2.0, ph.eta + 1.0) / (ph.eta + 1.0);
    pl->ctab_host[pr].assign(K2, 0.0);
    for (int k2 = 0; k2 < K2; ++k2) {
      const double kk = std::sqrt((double)k2);
      double c = 0.0;
      for (int r = 0; r < Nr; ++r) {
        const double rg = std::pow(ph.rho[r], ph.gamma + 2.0);
        hostbuf[off_g[pr] + (size_t)r * K2 + k2] = ph.wrho[r] * rg * 4.0 * M_PI * sinc(M_PI / pl->L * ph.rho[r] * aq * kk) / n3;
        c += ph.wrho[r] * rg * Ceta * 4.0 * M_PI * sinc(M_PI / pl->L * ph.rho[r] * kk);
      }
      pl->ctab_host[pr][k2] = c;
      hostbuf[off_c[pr] + k2] = c / n3;
    }
  }
  // sphere weights and x-group index
  const size_t off_wm = push(M);
  for (int m = 0; m < M; ++m) hostbuf[off_wm + m] = pl->wsig[m];

  if (pl->P >= 1 && !dg_setup(pl->P, pl->dg_r, pl->dg_Dr, pl->dg_Minv)) {
    set_error("DG operators for P = %d could not be built", pl->P);
    delete pl;
    return DGFS_EINVAL;
  }
  {
    std::vector<int> all(ns);
    for (int p = 0; p < ns; ++p) all[p] = p;
    if (!projection_ginv(pl, all, pl->proj_ginv)) {
      set_error("conservation constraints are singular");
      delete pl;
      return DGFS_EINVAL;
    }
    // one species on its own (the self-collision term of dgfs_collide)
    pl->proj_ginv_self.resize(ns);
    for (int p = 0; p < ns; ++p)
      if (!projection_ginv(pl, std::vector<int>{p}, pl->proj_ginv_self[p])) {
        set_error("conservation constraints are singular");
        delete pl;
        return DGFS_EINVAL;
      }
  }

  // convert to the compute type and upload in one allocation
  const size_t e = pl->elt();
  const size_t nvals = hostbuf.size();
  const size_t bytes_vals = ((nvals * e + 255) / 256) * 256;
  const size_t bytes_pairs = ((npair * sizeof(PairDev) + 255) / 256) * 256;
  // antipodal pairs of directions with equal weights (see PipeArgs::half)
  {
    std::vector<int> anti(M, -1);
    bool all = M % 2 == 0;
    for (int m = 0; m < M && all; ++m) {
      for (int t = 0; t < M; ++t) {
        const double d = std::fabs(pl->sigma[3 * m] + pl->sigma[3 * t]) + std::fabs(pl->sigma[3 * m + 1] + pl->sigma[3 * t + 1]) +
                         std::fabs(pl->sigma[3 * m + 2] + pl->sigma[3 * t + 2]);
        if (d <= 1e-13 && std::fabs(pl->wsig[m] - pl->wsig[t]) <= 1e-14 * std::fabs(pl->wsig[m])) anti[m] = t;
      }
      if (anti[m] < 0) all = false;
    }
    pl->antipodal = all;
    if (all) {
      // one representative per pair, taken in the half space sigma_x > 0 (then
      // sigma_y > 0, then sigma_z > 0), so that representatives share
      // (sigma_x, sigma_y) values as often as the set allows; ordered by
      // sigma_x group, then sigma_y
      const double tol = 1e-13;
      auto upper = [&](int m) {
        const double *v = &pl->sigma[3 * m];
        if (std::fabs(v[0]) > tol) return v[0] > 0;
        if (std::fabs(v[1]) > tol) return v[1] > 0;
        return v[2] > 0;
      };
      std::vector<char> taken(M, 0);
      for (int m = 0; m < M; ++m)
        if (!taken[m]) {
          taken[m] = taken[anti[m]] = 1;
          pl->mhalf.push_back(upper(m) ? m : anti[m]);
        }
      std::stable_sort(pl->mhalf.begin(), pl->mhalf.end(), [&](int a, int b) {
        if (pl->sx_idx[a] != pl->sx_idx[b]) return pl->sx_idx[a] < pl->sx_idx[b];
        return pl->sigma[3 * a + 1] < pl->sigma[3 * b + 1];
      });
    }
  }
  const int Mh = (int)pl->mhalf.size();
  // FP32 term schedule of the N = 32 gain kernel (gain_yz_halves_body, one
  // wavefront per x-plane): directions sharing (sigma_x, sigma_y) share one
  // column pass, so they run as consecutive terms, largest class first; an
  // entry is m | first << 16 (first: the column pass runs before this term).
  // The table keeps the form of a schedule for G groups (one here), padded
  // with -1 to a common length T.
  auto gain_sched = [&](const std::vector<int> &dirs, std::vector<int> &table) {
    const int G = 1;
    std::vector<std::vector<int>> classes;
    for (int m : dirs) {
      int found = -1;
      for (size_t k = 0; k < classes.size(); ++k) {
        const int m0 = classes[k][0];
        if (pl->sx_idx[m0] == pl->sx_idx[m] && std::fabs(pl->sigma[3 * m0 + 1] - pl->sigma[3 * m + 1]) <= 1e-15)
          found = (int)k;
      }
      if (found < 0) {
        classes.push_back({m});
      } else {
        classes[found].push_back(m);
      }
    }
    std::stable_sort(classes.begin(), classes.end(),
                     [](const std::vector<int> &a, const std::vector<int> &b) { return a.size() > b.size(); });
    std::vector<std::vector<int>> lists(G);
    std::vector<int> load(G, 0);
    for (const auto &cl : classes) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (size_t j = 0; j < cl.size(); ++j) lists[g].push_back(cl[j] | (j == 0 ? 1 << 16 : 0));
      load[g] += 2 + 2 * (int)cl.size();
    }
    int T = 0;
    for (const auto &l : lists) T = std::max<int>(T, (int)l.size());
    table.assign((size_t)G * T, -1);
    for (int g = 0; g < G; ++g)
      for (size_t t = 0; t < lists[g].size(); ++t) table[(size_t)g * T + t] = lists[g][t];
    return T;
  };
  {
    std::vector<int> order(M);
    for (int m = 0; m < M; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pl->sx_idx[a] < pl->sx_idx[b]; });
    pl->gs_T_full = gain_sched(order, pl->gs_full);
    pl->gs_T_half = Mh ? gain_sched(pl->mhalf, pl->gs_half) : 0;
  }
  // VJP term schedules: the (sigma_x group, side) units of the adjoint's yz
  // stage spread over the groups of a block (largest first onto the least
  // loaded group); each group's list holds m | side << 16 | last << 17 per
  // term (last: the unit ends, write its sum), padded with -1 to a common
  // length so every group passes the same barriers.  The second schedule
  // holds the side-0 units only: with p == q on one input and an antipodal
  // sphere set the two sides' gain sums coincide (see dgfs_collide_vjp).
  {
    const int G = std::max(1, 128 / (2 * N));
    std::vector<int> cnt(pl->Sx, 0);
    for (int m = 0; m < M; ++m) ++cnt[pl->sx_idx[m]];
    auto build = [&](int nsides, std::vector<int> &table) {
      std::vector<std::pair<int, int>> units;  // (s, side)
      for (int s = 0; s < pl->Sx; ++s)
        for (int side = 0; side < nsides; ++side) units.push_back({s, side});
      std::stable_sort(units.begin(), units.end(), [&](const std::pair<int, int> &a, const std::pair<int, int> &b) {
        return cnt[a.first] > cnt[b.first];
      });
      std::vector<std::vector<int>> lists(G);
      std::vector<int> load(G, 0);
      for (const auto &u : units) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        int left = cnt[u.first];
        for (int m = 0; m < M; ++m)
          if (pl->sx_idx[m] == u.first) lists[g].push_back(m | (u.second << 16) | ((--left == 0) ? 1 << 17 : 0));
        load[g] += cnt[u.first];
      }
      int T = 0;
      for (const auto &l : lists) T = std::max<int>(T, (int)l.size());
      table.assign((size_t)G * T, -1);
      for (int g = 0; g < G; ++g)
        for (size_t t = 0; t < lists[g].size(); ++t) table[(size_t)g * T + t] = lists[g][t];
      return T;
    };
    pl->vjp_G = G;
    pl->vjp_T = build(2, pl->vjp_sched);
    pl->vjp_T_sym = build(1, pl->vjp_sched_sym);
  }
  const int nsched = (int)pl->vjp_sched.size() + (int)pl->vjp_sched_sym.size();
  const int ngf = (int)pl->gs_full.size(), ngh = (int)pl->gs_half.size();
  // term tables of the N = 32 gain kernel: per direction of the full order
  // (morder) and of the half set (mhalf), four ints: m, s = sidx[m],
  // sneg[s], sx_zero[s] | sx_zero[sneg[s]] << 1
  const int ntinfo = 4 * (M + Mh);
  const size_t bytes_sidx =
      (((2 * M + 2 * pl->Sx + Mh + nsched + ngf + ngh + 4 + ntinfo) * sizeof(int) + 255) / 256) * 256;
  pl->dev_bytes = bytes_vals + bytes_pairs + bytes_sidx;
  hipError_t he = hipMalloc(&pl->dev, pl->dev_bytes);
  if (he != hipSuccess) {
    set_error("plan tables: hipMalloc(%zu) failed: %s", pl->dev_bytes, hipGetErrorString(he));
    delete pl;
    return DGFS_ENOMEM;
  }
  std::vector<unsigned char> img(pl->dev_bytes, 0);
  if (pl->precision == DGFS_FP64) std::memcpy(img.data(), hostbuf.data(), nvals * sizeof(double));
  else {
    float *f = reinterpret_cast<float *>(img.data());
    for (size_t i = 0; i < nvals; ++i) f[i] = (float)hostbuf[i];
  }
  char *base = static_cast<char *>(pl->dev);
  pl->pair_host.resize(npair);
  for (int pr = 0; pr < npair; ++pr) {
    PairDev &d = pl->pair_host[pr];
    d.px = base + off_px[pr] * e;
    d.pyz = base + off_pyz[pr] * e;
    d.gtab = base + off_g[pr] * e;
    d.ctab = base + off_c[pr] * e;
    d.beta = pl->pairs[pr].beta;
  }
  std::memcpy(img.data() + bytes_vals, pl->pair_host.data(), npair * sizeof(PairDev));
  std::memcpy(img.data() + bytes_vals + bytes_pairs, pl->sx_idx.data(), M * sizeof(int));
  {
    std::vector<int> z(pl->Sx);
    for (int s = 0; s < pl->Sx; ++s) z[s] = pl->sx_val[s] == 0.0 ? 1 : 0;
    std::memcpy(img.data() + bytes_vals + bytes_pairs + M * sizeof(int), z.data(), pl->Sx * sizeof(int));
    // directions ordered by their sigma_x group (consecutive terms share X arrays)
    std::vector<int> order(M);
    for (int m = 0; m < M; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pl->sx_idx[a] < pl->sx_idx[b]; });
    std::memcpy(img.data() + bytes_vals + bytes_pairs + (M + pl->Sx) * sizeof(int), order.data(), M * sizeof(int));
    // index of the opposite x component, if present exactly
    std::vector<int> neg(pl->Sx, -1);
    for (int s = 0; s < pl->Sx; ++s)
      for (int t = 0; t < pl->Sx; ++t)
        if (pl->sx_val[t] == -pl->sx_val[s]) neg[s] = t;
    std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + pl->Sx) * sizeof(int), neg.data(), pl->Sx * sizeof(int));
    if (Mh) std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + 2 * pl->Sx) * sizeof(int), pl->mhalf.data(), Mh * sizeof(int));
    std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + 2 * pl->Sx + Mh) * sizeof(int), pl->vjp_sched.data(),
                pl->vjp_sched.size() * sizeof(int));
    std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + 2 * pl->Sx + Mh + pl->vjp_sched.size()) * sizeof(int),
                pl->vjp_sched_sym.data(), pl->vjp_sched_sym.size() * sizeof(int));
    std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + 2 * pl->Sx + Mh + nsched) * sizeof(int),
                pl->gs_full.data(), ngf * sizeof(int));
    if (ngh)
      std::memcpy(img.data() + bytes_vals + bytes_pairs + (2 * M + 2 * pl->Sx + Mh + nsched + ngf) * sizeof(int),
                  pl->gs_half.data(), ngh * sizeof(int));
    // term tables, 16-byte aligned
    const size_t t0 = ((2 * M + 2 * pl->Sx + Mh + nsched + ngf + ngh) + 3) / 4 * 4;
    std::vector<int> tinfo;
    auto add_term = [&](int m) {
      const int sx = pl->sx_idx[m], sn = neg[sx];
      tinfo.insert(tinfo.end(), {m, sx, sn, z[sx] | (sn >= 0 ? z[sn] : 0) << 1});
    };
    for (int m : order) add_term(m);
    for (int m : pl->mhalf) add_term(m);
    std::memcpy(img.data() + bytes_vals + bytes_pairs + t0 * sizeof(int), tinfo.data(), tinfo.size() * sizeof(int));
    pl->tinfo_off = t0;
  }
  pl->pair_dev = reinterpret_cast<PairDev *>(base + bytes_vals);
  pl->wm_dev = base + off_wm * e;
  pl->sidx_dev = reinterpret_cast<const int *>(base + bytes_vals + bytes_pairs);
  pl->sxz_dev = pl->sidx_dev + M;
  pl->morder_dev = pl->sidx_dev + M + pl->Sx;
  pl->sneg_dev = pl->sidx_dev + 2 * M + pl->Sx;
  pl->mhalf_dev = Mh ? pl->sidx_dev + 2 * M + 2 * pl->Sx : nullptr;
  pl->vjp_sched_dev = pl->sidx_dev + 2 * M + 2 * pl->Sx + Mh;
  pl->vjp_sched_sym_dev = pl->vjp_sched_dev + pl->vjp_sched.size();
  pl->gs_full_dev = pl->vjp_sched_dev + nsched;
  pl->gs_half_dev = ngh ? pl->gs_full_dev + ngf : nullptr;
  pl->tinfo_full_dev = pl->sidx_dev + pl->tinfo_off;
  pl->tinfo_half_dev = Mh ? pl->tinfo_full_dev + 4 * M : nullptr;
  if (!pl->vhs) {
    dgfs_status vs = build_vss_tables(pl);
    if (vs != DGFS_OK) {
      (void)hipFree(pl->dev);
      delete pl;
      return vs;
    }
    for (int pr = 0; pr < npair; ++pr)
      std::memcpy(img.data() + bytes_vals + pr * sizeof(PairDev), &pl->pair_host[pr], sizeof(PairDev));
  }
  he = hipMemcpy(pl->dev, img.data(), pl->dev_bytes, hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    set_error("plan tables: upload failed: %s", hipGetErrorString(he));
    hipFree(pl->dev);
    if (pl->vss_dev) hipFree(pl->vss_dev);
    delete pl;
    return DGFS_EHIP;
  }
  if (!std::getenv("DGFS_NO_TUNE_CACHE")) load_tuned(pl);
  *out = pl;
  return DGFS_OK;
}

namespace dgfs { void destroy_graph_cache(dgfs_plan_s *pl); }

extern "C" void dgfs_plan_destroy(dgfs_plan plan) {
  if (!plan) return;
  dgfs::destroy_graph_cache(plan);
  if (plan->dev) (void)hipFree(plan->dev);
  if (plan->vss_dev) (void)hipFree(plan->vss_dev);
  delete plan;
}

extern "C" dgfs_status dgfs_plan_table(dgfs_plan pl, int32_t p, int32_t q, int32_t which, double *out, int64_t n) {
  if (!pl || !out) { set_error("dgfs_plan_table: NULL argument"); return DGFS_EINVAL; }
  if (p < 0 || q < 0 || p >= pl->ns || q >= pl->ns) { set_error("species index out of range"); return DGFS_EINVAL; }
  const PairHost &ph = pl->pairs[p * pl->ns + q];
  const int N = pl->N, Nr = pl->Nr, M = pl->M;
  const int64_t n3 = (int64_t)N * N * N;
  auto need = [&](int64_t k) {
    if (n < k) { set_error("dgfs_plan_table: output holds %lld, need %lld", (long long)n, (long long)k); return false; }
    return true;
  };
  const double aq = ph.mq / (ph.mp + ph.mq);
  switch (which) {
    case 0: if (!need(Nr)) return DGFS_EINVAL; std::copy(ph.rho.begin(), ph.rho.end(), out); return DGFS_OK;
    case 1: if (!need(Nr)) return DGFS_EINVAL; std::copy(ph.wrho.begin(), ph.wrho.end(), out); return DGFS_OK;
    case 2:
      if (!need(n3)) return DGFS_EINVAL;
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
          for (int k = 0; k < N; ++k) {
            int k2 = wave(i, N) * wave(i, N) + wave(j, N) * wave(j, N) + wave(k, N) * wave(k, N);
            out[((int64_t)i * N + j) * N + k] = pl->ctab_host[p * pl->ns + q][k2];
          }
      return DGFS_OK;
    case 3:
    case 4: {
      if (!need((int64_t)Nr * M * n3)) return DGFS_EINVAL;
      if (!pl->vhs) {  // copy the device table back, undoing w_r w_m / N^3
        const size_t cnt = (size_t)Nr * M * n3 * 2;
        std::vector<unsigned char> buf(cnt * pl->elt());
        hipError_t he = hipMemcpy(buf.data(), pl->pair_host[p * pl->ns + q].btab, buf.size(), hipMemcpyDeviceToHost);
        if (he != hipSuccess) return hip_status(he, "dgfs_plan_table");
        for (int r = 0; r < Nr; ++r)
          for (int m = 0; m < M; ++m) {
            const double sc = (double)n3 / (ph.wrho[r] * pl->wsig[m]);
            for (int64_t k = 0; k < n3; ++k) {
              const size_t i = 2 * (((size_t)r * M + m) * n3 + k) + (which == 4 ? 1 : 0);
              const double v = pl->precision == DGFS_FP64 ? reinterpret_cast<double *>(buf.data())[i]
                                                          : (double)reinterpret_cast<float *>(buf.data())[i];
              out[((int64_t)r * M + m) * n3 + k] = v * sc;
            }
          }
        return DGFS_OK;
      }
      for (int r = 0; r < Nr; ++r)
        for (int m = 0; m < M; ++m)
          for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
              for (int k = 0; k < N; ++k) {
                double kk = std::sqrt((double)(wave(i, N) * wave(i, N) + wave(j, N) * wave(j, N) + wave(k, N) * wave(k, N)));
                double b = std::pow(ph.rho[r], ph.gamma + 2.0) * 4.0 * M_PI * sinc(M_PI / pl->L * ph.rho[r] * aq * kk);
                out[(((int64_t)r * M + m) * N + i) * N * N + (int64_t)j * N + k] = which == 3 ? b : 0.0;
              }
      return DGFS_OK;
    }
    case 5: if (!need(1)) return DGFS_EINVAL; out[0] = ph.beta; return DGFS_OK;
    default: set_error("dgfs_plan_table: unknown table %d", which); return DGFS_EINVAL;
  }
}
