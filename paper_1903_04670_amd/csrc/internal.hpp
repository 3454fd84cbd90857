// Internal types of libdgfs shared by the host plan builder and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgfs.h"

namespace dgfs {

constexpr int kMaxPairs = DGFS_MAX_SPECIES * DGFS_MAX_SPECIES;

// Per ordered pair (p, q): device tables, in the plan's compute type T
// (double for DGFS_FP64, float for DGFS_FP32_MIXED).  Complex = (re, im).
struct PairDev {
  const void *px;    // [2][Nr][S][N] cplx: side 0 e^{+i th_q s v}/N^3, side 1 e^{-i th_p s v}/N^3
  const void *pyz;   // [2][Nr][M][2][N] cplx: side 0 e^{+i th_q sigma_a v}, side 1 e^{-i th_p sigma_a v}; a = y, z
  const void *gtab;  // VHS: [Nr][K2] real  w_r b_r(|k|)/N^3, indexed by |k|^2
  const void *ctab;  // [K2] real  c(|k|)/N^3
  const void *btab;  // VSS: [Nr][M][N^3] cplx  w_r w_m b_rm(k)/N^3 (natural wave order); else NULL
  double beta;
};

// Host-side parameters of one ordered pair.
struct PairHost {
  double mp, mq, omega, alpha, gamma, eta, beta, R;
  std::vector<double> rho, wrho;
};

}  // namespace dgfs

struct dgfs_plan_s {
  int ns = 0, N = 0, M = 0, Nr = 0, P = 0, precision = 0;
  double L = 0, S = 0;
  std::vector<double> mass, sigma, wsig;
  // grouping of the sphere directions by their x component
  int Sx = 0;
  std::vector<double> sx_val;  // [Sx]
  std::vector<int> sx_idx;     // [M]
  std::vector<dgfs::PairHost> pairs;  // [ns*ns], p-major
  bool nyquist_zero = false;  // gain translates drop the Nyquist planes (real-packed VHS gain)
  bool vhs = true;      // every pair has alpha == 1 (sigma-independent gain table)
  int chunk_evals = 0;  // evaluations per launch chosen by dgfs_autotune or its cache (0 = default)
  // launch schedule knobs that dgfs_autotune also picks (0 / -1 = default);
  // neither changes a result bit
  int shift_split = 0;   // k_shift_x blocks per x-line set: 1, 2, 4 or 8
  int gain_x_fuse = -1;  // k_gain_x serves a mirrored slot in the same pass: 0 or 1
  void *vss_dev = nullptr;  // VSS gain tables of all pairs (separate allocation)
  // device memory owned by the plan
  void *dev = nullptr;
  size_t dev_bytes = 0;
  dgfs::PairDev *pair_dev = nullptr;   // device array [ns*ns]
  std::vector<dgfs::PairDev> pair_host;  // same pointers, host copy
  const void *wm_dev = nullptr;        // [M] T sphere weights
  const int *sidx_dev = nullptr;       // [M]
  const int *sxz_dev = nullptr;        // [Sx] zero-x-component flags
  const int *morder_dev = nullptr;     // [M] directions ordered by sigma_x group
  const int *sneg_dev = nullptr;       // [Sx] index of -sigma_x (or -1)
  // antipodal symmetry of the sphere set: every sigma_m has -sigma_m in the
  // set with the same weight; mhalf holds one direction of each such pair
  bool antipodal = false;
  std::vector<int> mhalf;
  const int *mhalf_dev = nullptr;      // [M/2] device copy of mhalf
  // per-term index tables of the N = 32 gain kernel ([M] and [M/2] groups of
  // four ints, in morder and mhalf order; see plan.cpp)
  size_t tinfo_off = 0;
  const int *tinfo_full_dev = nullptr, *tinfo_half_dev = nullptr;
  // FP32 N = 32 gain-kernel term schedules with shared column passes, full
  // and half sets
  int gs_T_full = 0, gs_T_half = 0;
  std::vector<int> gs_full, gs_half;
  const int *gs_full_dev = nullptr, *gs_half_dev = nullptr;
  // term schedule of the adjoint's yz stage: [vjp_G][vjp_T] entries
  int vjp_G = 1, vjp_T = 0, vjp_T_sym = 0;
  std::vector<int> vjp_sched, vjp_sched_sym;  // all units; side-0 units only
  const int *vjp_sched_dev = nullptr, *vjp_sched_sym_dev = nullptr;
  // the m-sum of the gain product of (q, p) equals that of (p, q)
  bool mirror_ok(int p, int q) const {
    return vhs && antipodal && pairs[p * ns + q].R == pairs[q * ns + p].R;
  }
  // nodal DG operators on P+1 Gauss-Lobatto points (row-major (P+1)^2)
  std::vector<double> dg_r, dg_Dr, dg_Minv;
  // (C C^T)^{-1} of the conservation constraints of all species (ns+4)^2
  std::vector<double> proj_ginv;
  // the same for each species alone, (1+4)^2 per species
  std::vector<std::vector<double>> proj_ginv_self;
  // graph cache of dgfs_step (guarded by graph_mu)
  void *graph_cache = nullptr;
  // host copies for dgfs_plan_table
  std::vector<std::vector<double>> ctab_host;  // [pair][K2] (c, unscaled)
  int K2() const { return 3 * (N / 2) * (N / 2) + 1; }
  size_t elt() const { return precision == DGFS_FP64 ? sizeof(double) : sizeof(float); }
};

namespace dgfs {
void set_error(const char *fmt, ...);
dgfs_status hip_status(hipError_t e, const char *what);
}  // namespace dgfs
