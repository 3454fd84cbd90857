// Right-hand side of the non-dimensional Boltzmann equation (Eq. bzeNonDim)
// in one space dimension: nodal DG transport with diffuse walls plus the
// mixture collision term, the FP64 conservation projection, and SSP-RK3 /
// Euler time steps captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "pipeline.hpp"
#include "launch.hpp"

namespace dgfs {

bool projection_ginv(const dgfs_plan_s *pl, const std::vector<int> &species, std::vector<double> &G);

constexpr int kMaxDG = 9;  // P <= 8

struct DGArgs {
  int N, ns, K, P;
  double L, h;            // velocity half-width, element width
  double mass[DGFS_MAX_SPECIES];
  double uw[2][3], Tw[2];  // wall 0 = left (x_left), 1 = right
  double Dr[kMaxDG * kMaxDG], Minv[kMaxDG * kMaxDG];
  const double *F;
  double *dF;
  const double *nw;  // [2][ns][kWallSplit][2] partial wall fluxes (k_wall_density)
};

__device__ __forceinline__ double grid_c(int j, int N, double L) { return -L + (j + 0.5) * (2.0 * L / N); }

__device__ __forceinline__ double wall_maxwellian(double m, const double *u, double T, double cx, double cy, double cz) {
  const double dx = cx - u[0], dy = cy - u[1], dz = cz - u[2];
  const double a = m / (M_PI * T);
  return a * sqrt(a) * exp(-m * (dx * dx + dy * dy + dz * dz) / T);
}

// Wall densities n_w from zero discrete net mass flux: n_w is the outgoing
// flux of f over the incoming flux of the unit-density wall Maxwellian.  Each
// (wall, species) is split over kWallSplit blocks, each writing its partial
// sums (outgoing, unit) in fixed order; the transport kernel adds the partials
// in block order where it needs n_w, so the result does not depend on timing.
constexpr int kWallThreads = 1024;  // the 2-D kernel's block
constexpr int kWall1Threads = 256, kWallSplit = 32;

__global__ void __launch_bounds__(kWall1Threads) k_wall_density(DGArgs a, double *nw) {
  const int part = blockIdx.x % kWallSplit, wp = blockIdx.x / kWallSplit;
  const int wall = wp / a.ns, p = wp % a.ns;
  const int N = a.N, n3 = N * N * N;
  const int node = wall == 0 ? 0 : a.K * (a.P + 1) - 1;
  const double *f = a.F + ((size_t)node * a.ns + p) * n3;
  double out = 0.0, unit = 0.0;
  for (int v = part * kWall1Threads + threadIdx.x; v < n3; v += kWall1Threads * kWallSplit) {
    const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
    if (wall == 0) {  // emits c_x > 0, absorbs c_x < 0
      if (cx < 0) out -= cx * f[v];
      else unit += cx * wall_maxwellian(a.mass[p], a.uw[wall], a.Tw[wall], cx, cy, cz);
    } else {
      if (cx > 0) out += cx * f[v];
      else unit -= cx * wall_maxwellian(a.mass[p], a.uw[wall], a.Tw[wall], cx, cy, cz);
    }
  }
  __shared__ double so[kWall1Threads], su[kWall1Threads];
  so[threadIdx.x] = out;
  su[threadIdx.x] = unit;
  __syncthreads();
  for (int s = kWall1Threads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      su[threadIdx.x] += su[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nw[2 * (wp * kWallSplit + part)] = so[0];
    nw[2 * (wp * kWallSplit + part) + 1] = su[0];
  }
}

__device__ __forceinline__ double wall_density(const DGArgs &a, int wall, int p) {
  const double *q = a.nw + 2 * (size_t)((wall * a.ns + p) * kWallSplit);
  double so = 0.0, su = 0.0;
  for (int i = 0; i < kWallSplit; ++i) {
    so += q[2 * i];
    su += q[2 * i + 1];
  }
  return so / su;
}

// dF/dt = -c_x dF/dx by nodal DG (strong form, upwind flux).  One thread per
// (species, velocity point, element); blockIdx.y strides over the elements.
// The degree is a template argument so that the element's P + 1 loads, its
// two neighbour loads and its stores are issued together (with a run-time
// degree each load was waited for before the next).
template <int P>
__global__ void __launch_bounds__(256) k_dg_transport(DGArgs a) {
  constexpr int np1 = P + 1;
  const int N = a.N, n3 = N * N * N;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.z;
  if (v >= n3) return;
  const double cx = grid_c(v / (N * N), N, a.L);
  const size_t ns_stride = (size_t)a.ns * n3;
  const double *f = a.F + (size_t)p * n3 + v;
  double *df = a.dF + (size_t)p * n3 + v;
  const double s = 2.0 / a.h;
  for (int e = blockIdx.y; e < a.K; e += gridDim.y) {
    // neighbour nodes across the two faces; at a wall the index is any valid
    // one and its value is replaced by the wall's inflow below
    const int iL = e > 0 ? e * np1 - 1 : 0, iR = e < a.K - 1 ? (e + 1) * np1 : 0;
    double u[np1];
#pragma unroll
    for (int i = 0; i < np1; ++i) u[i] = f[(size_t)(e * np1 + i) * ns_stride];
    double uL = f[(size_t)iL * ns_stride], uR = f[(size_t)iR * ns_stride];
    if (e == 0) {
      const double cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
      uL = cx > 0 ? wall_density(a, 0, p) * wall_maxwellian(a.mass[p], a.uw[0], a.Tw[0], cx, cy, cz) : 0.0;
    }
    if (e == a.K - 1) {
      const double cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
      uR = cx < 0 ? wall_density(a, 1, p) * wall_maxwellian(a.mass[p], a.uw[1], a.Tw[1], cx, cy, cz) : 0.0;
    }
    // boundary terms n (c u - F*) with the upwind flux F*
    const double termR = cx > 0 ? 0.0 : cx * (u[P] - uR);
    const double termL = cx > 0 ? -cx * (u[0] - uL) : 0.0;
#pragma unroll
    for (int i = 0; i < np1; ++i) {
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < np1; ++j) d += a.Dr[i * np1 + j] * u[j];
      df[(size_t)(e * np1 + i) * ns_stride] = s * (-cx * d + a.Minv[i * np1 + P] * termR + a.Minv[i * np1] * termL);
    }
  }
}

template <int P>
static void launch_dg_transport(dim3 grid, hipStream_t st, const DGArgs &d) {
  DGFS_LAUNCH("k_dg_transport", k_dg_transport<P>, grid, dim3(256), 0, st, d);
}

// ------------------------------------------------------------ 2-D transport
// Tensor-product nodal DG on Kx x Ky rectangles.  With the exact mass
// matrices of the tensor basis the strong form separates into the 1-D
// operator along every x-line of nodes (velocity c_x) plus the 1-D operator
// along every y-line (c_y); both use the same GLL Dr and Minv as the 1-D
// scheme.  Sides: 0 = left (x_left), 1 = right, 2 = bottom (y_bottom),
// 3 = top; each is periodic or a diffuse wall.
constexpr int kMax2D = 5;  // P <= 4
constexpr size_t kWallCap = 8192;  // boundary densities (nodes x species) the workspace holds
static_assert(2 * DGFS_MAX_SPECIES * kWallSplit * 2 <= kWallCap, "1-D partial wall fluxes exceed the buffer");

struct DG2Args {
  int N, ns, Kx, Ky, P;
  int periodic[2];
  double L, hx, hy;
  double mass[DGFS_MAX_SPECIES];
  double uw[4][3], Tw[4];
  double Dr[kMaxDG * kMaxDG], Minv[kMaxDG * kMaxDG];
  const double *F;
  double *dF;
  const double *nw;  // wall densities, see wall_slot()
};

// Index of the wall density of boundary node b (along the side) of side s,
// species p: sides 0, 1 hold Ky (P+1) nodes each, sides 2, 3 Kx (P+1).
__device__ __forceinline__ int wall_slot(const DG2Args &a, int side, int b, int p) {
  const int ny = a.Ky * (a.P + 1), nx = a.Kx * (a.P + 1);
  const int off = side == 0 ? 0 : side == 1 ? ny : side == 2 ? 2 * ny : 2 * ny + nx;
  return (off + b) * a.ns + p;
}

__device__ __forceinline__ int node2(const DG2Args &a, int ex, int ey, int i, int j) {
  return ((ey * a.Kx + ex) * (a.P + 1) + j) * (a.P + 1) + i;
}

// One block per (side, boundary node, species) of the wall sides; fixed-order
// reduction of the outgoing flux and the unit-density incoming flux.
__global__ void __launch_bounds__(kWallThreads) k_wall_density_2d(DG2Args a, double *nw) {
  const int ny = a.Ky * (a.P + 1), nx = a.Kx * (a.P + 1), ns = a.ns;
  int blk = blockIdx.x;
  // walk the sides in order, skipping periodic directions
  int side = -1, b = 0;
  for (int s = 0; s < 4; ++s) {
    if (a.periodic[s / 2]) continue;
    const int cnt = (s < 2 ? ny : nx) * ns;
    if (blk < cnt) {
      side = s;
      b = blk;
      break;
    }
    blk -= cnt;
  }
  if (side < 0) return;
  const int p = b % ns;
  b /= ns;
  const int P = a.P, e = b / (P + 1), l = b % (P + 1);
  const int node = side == 0 ? node2(a, 0, e, 0, l)
                 : side == 1 ? node2(a, a.Kx - 1, e, P, l)
                 : side == 2 ? node2(a, e, 0, l, 0)
                             : node2(a, e, a.Ky - 1, l, P);
  const int N = a.N, n3 = N * N * N;
  const double *f = a.F + ((size_t)node * ns + p) * n3;
  const int axis = side / 2;       // 0: the wall's normal is x, 1: y
  const bool lo = side % 2 == 0;   // lo walls emit c_n > 0 into the domain
  double out = 0.0, unit = 0.0;
  for (int v = threadIdx.x; v < n3; v += kWallThreads) {
    const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
    const double cn = axis == 0 ? cx : cy;
    if (lo) {
      if (cn < 0) out -= cn * f[v];
      else unit += cn * wall_maxwellian(a.mass[p], a.uw[side], a.Tw[side], cx, cy, cz);
    } else {
      if (cn > 0) out += cn * f[v];
      else unit -= cn * wall_maxwellian(a.mass[p], a.uw[side], a.Tw[side], cx, cy, cz);
    }
  }
  __shared__ double so[kWallThreads], su[kWallThreads];
  so[threadIdx.x] = out;
  su[threadIdx.x] = unit;
  __syncthreads();
  for (int s = kWallThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      su[threadIdx.x] += su[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) nw[wall_slot(a, side, b, p)] = so[0] / su[0];
}

// One thread per (species, velocity point, element); blockIdx.y strides over
// the elements.
__global__ void __launch_bounds__(256) k_dg_transport_2d(DG2Args a) {
  const int N = a.N, n3 = N * N * N, P = a.P, np1 = a.P + 1;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.z;
  if (v >= n3) return;
  const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
  const size_t st = (size_t)a.ns * n3;
  const double *f = a.F + (size_t)p * n3 + v;
  double *df = a.dF + (size_t)p * n3 + v;
  const double sx = 2.0 / a.hx, sy = 2.0 / a.hy;
  const int K = a.Kx * a.Ky;
  for (int e = blockIdx.y; e < K; e += gridDim.y) {
    const int ex = e % a.Kx, ey = e / a.Kx;
    double u[kMax2D][kMax2D], du[kMax2D][kMax2D];
    for (int j = 0; j <= P; ++j)
      for (int i = 0; i <= P; ++i) u[j][i] = f[(size_t)node2(a, ex, ey, i, j) * st];
    for (int j = 0; j <= P; ++j)
      for (int i = 0; i <= P; ++i) {
        double dx = 0.0, dy = 0.0;
        for (int k = 0; k <= P; ++k) {
          dx += a.Dr[i * np1 + k] * u[j][k];
          dy += a.Dr[j * np1 + k] * u[k][i];
        }
        du[j][i] = -sx * cx * dx - sy * cy * dy;
      }
    // x faces of every node row j: upwind flux, neighbour, periodic image or wall
    for (int j = 0; j <= P; ++j) {
      double uL = 0.0, uR = 0.0;
      if (cx > 0) {
        if (ex > 0) uL = f[(size_t)node2(a, ex - 1, ey, P, j) * st];
        else if (a.periodic[0]) uL = f[(size_t)node2(a, a.Kx - 1, ey, P, j) * st];
        else uL = a.nw[wall_slot(a, 0, ey * np1 + j, p)] * wall_maxwellian(a.mass[p], a.uw[0], a.Tw[0], cx, cy, cz);
      } else {
        if (ex < a.Kx - 1) uR = f[(size_t)node2(a, ex + 1, ey, 0, j) * st];
        else if (a.periodic[0]) uR = f[(size_t)node2(a, 0, ey, 0, j) * st];
        else uR = a.nw[wall_slot(a, 1, ey * np1 + j, p)] * wall_maxwellian(a.mass[p], a.uw[1], a.Tw[1], cx, cy, cz);
      }
      const double termR = cx > 0 ? 0.0 : cx * (u[j][P] - uR);
      const double termL = cx > 0 ? -cx * (u[j][0] - uL) : 0.0;
      for (int i = 0; i <= P; ++i) du[j][i] += sx * (a.Minv[i * np1 + P] * termR + a.Minv[i * np1] * termL);
    }
    // y faces of every node column i
    for (int i = 0; i <= P; ++i) {
      double uB = 0.0, uT = 0.0;
      if (cy > 0) {
        if (ey > 0) uB = f[(size_t)node2(a, ex, ey - 1, i, P) * st];
        else if (a.periodic[1]) uB = f[(size_t)node2(a, ex, a.Ky - 1, i, P) * st];
        else uB = a.nw[wall_slot(a, 2, ex * np1 + i, p)] * wall_maxwellian(a.mass[p], a.uw[2], a.Tw[2], cx, cy, cz);
      } else {
        if (ey < a.Ky - 1) uT = f[(size_t)node2(a, ex, ey + 1, i, 0) * st];
        else if (a.periodic[1]) uT = f[(size_t)node2(a, ex, 0, i, 0) * st];
        else uT = a.nw[wall_slot(a, 3, ex * np1 + i, p)] * wall_maxwellian(a.mass[p], a.uw[3], a.Tw[3], cx, cy, cz);
      }
      const double termT = cy > 0 ? 0.0 : cy * (u[P][i] - uT);
      const double termB = cy > 0 ? -cy * (u[0][i] - uB) : 0.0;
      for (int j = 0; j <= P; ++j) du[j][i] += sy * (a.Minv[j * np1 + P] * termT + a.Minv[j * np1] * termB);
    }
    for (int j = 0; j <= P; ++j)
      for (int i = 0; i <= P; ++i) df[(size_t)node2(a, ex, ey, i, j) * st] = du[j][i];
  }
}

constexpr int kProjThreads = 256;

// Partial moments C Q over a slice of one node's ns*N^3 values (fixed-order
// tree reduction, so the result is deterministic).  Rows of C: mass of each
// species, then (nrow = nsp + 4) total momentum (x, y, z) and total energy,
// weight h^3.
__global__ void __launch_bounds__(kProjThreads) k_proj_moments(ProjArgs a) {
  const int node = blockIdx.y, blk = blockIdx.x;
  const int N = a.N, n3 = N * N * N, k = a.nrow, total = a.nsp * n3;
  const double h = 2.0 * a.L / N, w = h * h * h;
  const double *Q = a.Q + (size_t)node * a.q_stride;
  double mom[DGFS_MAX_SPECIES + 4];
  for (int i = 0; i < k; ++i) mom[i] = 0.0;
  const int per = (total + a.nblk - 1) / a.nblk;
  const int lo = blk * per, hi = min(total, lo + per);
  // species of the block's range in turn (a uniform loop, so the mass is a
  // scalar read), points unrolled so that several loads are in flight
  double px = 0.0, py = 0.0, pz = 0.0, en = 0.0;
  for (int sp = lo / n3; sp < a.nsp && sp * n3 < hi; ++sp) {
    const int s0 = max(lo, sp * n3), s1 = min(hi, (sp + 1) * n3);
    const double m = a.mass[sp];
    const double *Qs = Q + (size_t)sp * n3;
    double ms = 0.0;
#pragma unroll 4
    for (int i = s0 + threadIdx.x; i < s1; i += kProjThreads) {
      const int v = i - sp * n3;
      const double q = Qs[v];
      const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
      ms += w * q;
      if (k > a.nsp) {
        px += w * m * cx * q;
        py += w * m * cy * q;
        pz += w * m * cz * q;
        en += w * 0.5 * m * (cx * cx + cy * cy + cz * cz) * q;
      }
    }
#pragma unroll
    for (int s = 0; s < DGFS_MAX_SPECIES; ++s)
      if (s == sp) mom[s] += ms;
  }
  if (k > a.nsp) {
    // static indices keep mom in registers; nsp may equal the maximum
#pragma unroll
    for (int s = 0; s <= DGFS_MAX_SPECIES; ++s)
      if (s == a.nsp) {
        mom[s] += px;
        mom[s + 1] += py;
        mom[s + 2] += pz;
        mom[s + 3] += en;
      }
  }
  __shared__ double red[DGFS_MAX_SPECIES + 4][kProjThreads];
  for (int i = 0; i < k; ++i) red[i][threadIdx.x] = mom[i];
  __syncthreads();
  for (int s = kProjThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int i = 0; i < k; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < k) a.part[((size_t)node * a.nblk + blk) * k + threadIdx.x] = red[threadIdx.x][0];
}

// Q~ = Q - C^T (C C^T)^{-1} C Q: every block sums its node's partial moments
// in block order, forms the multipliers and corrects a slice of the node.
__global__ void __launch_bounds__(kProjThreads) k_proj_apply(ProjArgs a) {
  const int node = blockIdx.y, blk = blockIdx.x;
  const int N = a.N, n3 = N * N * N, k = a.nrow, total = a.nsp * n3;
  const double h = 2.0 * a.L / N, w = h * h * h;
  __shared__ double lam[DGFS_MAX_SPECIES + 4];
  if (threadIdx.x < k) {
    double mom[DGFS_MAX_SPECIES + 4];
    for (int j = 0; j < k; ++j) {
      double sum = 0.0;
      for (int b = 0; b < a.nblk; ++b) sum += a.part[((size_t)node * a.nblk + b) * k + j];
      mom[j] = sum;
    }
    double l = 0.0;
    for (int j = 0; j < k; ++j) l += a.ginv[threadIdx.x * k + j] * mom[j];
    lam[threadIdx.x] = l;
  }
  __syncthreads();
  const double *Q = a.Q + (size_t)node * a.q_stride;
  const int per = (total + a.nblk - 1) / a.nblk;
  const int lo = blk * per, hi = min(total, lo + per);
  // species of the block's range in turn (uniform: mass, output pointer and
  // multipliers are scalar reads), points unrolled
  for (int sp = lo / n3; sp < a.nsp && sp * n3 < hi; ++sp) {
    const int s0 = max(lo, sp * n3), s1 = min(hi, (sp + 1) * n3);
    const double m = a.mass[sp], l0 = lam[sp];
    const double lx = k > a.nsp ? lam[a.nsp] : 0.0, ly = k > a.nsp ? lam[a.nsp + 1] : 0.0;
    const double lz = k > a.nsp ? lam[a.nsp + 2] : 0.0, le = k > a.nsp ? lam[a.nsp + 3] : 0.0;
    const double *Qs = Q + (size_t)sp * n3;
    double *o = a.out[sp] + (size_t)node * a.out_stride;
    // chunks of kU points per thread: all loads of a chunk are issued
    // before its first store (a store may alias the next load otherwise)
    constexpr int kU = 4;
    for (int i0 = s0 - sp * n3 + threadIdx.x; i0 < s1 - sp * n3; i0 += kU * kProjThreads) {
      double q[kU], prev[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int v = i0 + u * kProjThreads;
        const bool in = v < s1 - sp * n3;
        q[u] = in ? Qs[v] : 0.0;
        prev[u] = in && a.accumulate ? o[v] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int v = i0 + u * kProjThreads;
        if (v >= s1 - sp * n3) break;
        const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
        const double corr =
            k > a.nsp ? w * (l0 + m * (lx * cx + ly * cy + lz * cz) + 0.5 * m * (cx * cx + cy * cy + cz * cz) * le)
                      : w * l0;
        o[v] = prev[u] + (q[u] - corr);
      }
    }
  }
}

hipError_t launch_projection(const ProjArgs &pa, int n_nodes, hipStream_t st) {
  DGFS_LAUNCH("k_proj_moments", k_proj_moments, dim3(pa.nblk, n_nodes), dim3(kProjThreads), 0, st, pa);
  DGFS_LAUNCH("k_proj_apply", k_proj_apply, dim3(pa.nblk, n_nodes), dim3(kProjThreads), 0, st, pa);
  return hipGetLastError();
}

// out = a*X + b*(Y + dt*R), elementwise
__global__ void k_combine(double *out, const double *X, const double *Y, const double *R, double a, double b,
                          double dt, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * X[i] + b * (Y[i] + dt * R[i]);
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }


struct RhsLayout {
  int B;                      // nodes per collision chunk
  size_t pipe, qc, nw, part;  // byte sizes
  size_t total() const { return pipe + qc + nw + part; }
};

static RhsLayout rhs_layout(const dgfs_plan_s *pl, int64_t n_nodes) {
  RhsLayout l;
  const int npairs = pl->ns * pl->ns;
  l.B = chunk_nodes(pl, n_nodes, npairs);
  l.pipe = pipeline_bytes(pl, l.B, npairs, pl->ns);
  l.qc = align256((size_t)l.B * pl->ns * pl->N * pl->N * pl->N * sizeof(double));
  l.nw = align256(kWallCap * sizeof(double));
  l.part = align256((size_t)l.B * kProjBlocks * (DGFS_MAX_SPECIES + 4) * sizeof(double));
  return l;
}

size_t extra_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes, int32_t op) {
  const size_t state = align256((size_t)n_nodes * pl->ns * pl->N * pl->N * pl->N * sizeof(double));
  switch (op) {
    case DGFS_OP_RHS: return rhs_layout(pl, n_nodes).total();
    case DGFS_OP_STEP: return rhs_layout(pl, n_nodes).total() + 3 * state;
    case DGFS_OP_VJP: return vjp_workspace_bytes(pl, n_nodes);
    default: return 0;
  }
}

static dgfs_status validate_rhs(const dgfs_plan_s *pl, const dgfs_mesh *mesh, int64_t n_nodes, const char *who) {
  if (!pl) { set_error("%s: NULL plan", who); return DGFS_EINVAL; }
  if (n_nodes < 1) { set_error("%s: n_nodes must be >= 1", who); return DGFS_EINVAL; }
  if (mesh) {
    if (pl->P < 1) { set_error("%s: the plan has dg_order %d; a mesh needs dg_order >= 1", who, pl->P); return DGFS_EINVAL; }
    if (mesh->K < 1) { set_error("%s: mesh K must be >= 1", who); return DGFS_EINVAL; }
    if ((int64_t)mesh->K * (pl->P + 1) != n_nodes) {
      set_error("%s: n_nodes %lld != K*(P+1) = %d", who, (long long)n_nodes, mesh->K * (pl->P + 1));
      return DGFS_EINVAL;
    }
    if (!(mesh->x_right > mesh->x_left) || !(mesh->T_left > 0) || !(mesh->T_right > 0)) {
      set_error("%s: invalid mesh extent or wall temperature", who);
      return DGFS_EINVAL;
    }
  }
  return DGFS_OK;
}

// Enqueues one right-hand side evaluation; no validation, no sync.
// The transport term of a right-hand side: none, a 1-D mesh or a 2-D mesh.
struct Transport {
  const dgfs_mesh *m1 = nullptr;
  const dgfs_mesh2d *m2 = nullptr;
  bool any() const { return m1 || m2; }
};

static hipError_t enqueue_rhs(const dgfs_plan_s *pl, const Transport &tr, int64_t n_nodes, const double *F,
                              double *dF, uint32_t flags, void *ws, hipStream_t st) {
  const dgfs_mesh *mesh = tr.m1;
  const int ns = pl->ns, N = pl->N;
  const int64_t n3 = (int64_t)N * N * N;
  const RhsLayout l = rhs_layout(pl, n_nodes);
  char *base = static_cast<char *>(ws);
  double *qc = reinterpret_cast<double *>(base + l.pipe);
  double *nw = reinterpret_cast<double *>(base + l.pipe + l.qc);
  double *part = reinterpret_cast<double *>(base + l.pipe + l.qc + l.nw);
  const bool project = flags & DGFS_PROJECT;
  if (mesh) {
    DGArgs d{};
    d.N = N;
    d.ns = ns;
    d.K = mesh->K;
    d.P = pl->P;
    d.L = pl->L;
    d.h = (mesh->x_right - mesh->x_left) / mesh->K;
    for (int p = 0; p < ns; ++p) d.mass[p] = pl->mass[p];
    for (int c = 0; c < 3; ++c) {
      d.uw[0][c] = mesh->u_left[c];
      d.uw[1][c] = mesh->u_right[c];
    }
    d.Tw[0] = mesh->T_left;
    d.Tw[1] = mesh->T_right;
    const int np1 = pl->P + 1;
    for (int i = 0; i < np1 * np1; ++i) {
      d.Dr[i] = pl->dg_Dr[i];
      d.Minv[i] = pl->dg_Minv[i];
    }
    d.F = F;
    d.dF = dF;
    d.nw = nw;
    DGFS_LAUNCH("k_wall_density", k_wall_density, dim3(2 * ns * kWallSplit), dim3(kWall1Threads), 0, st, d, nw);
    // element slices in y (each thread strides over the rest); species in z
    const unsigned ey = (unsigned)std::min(mesh->K, 64);
    const dim3 grid((unsigned)((n3 + 255) / 256), ey, ns);
    switch (pl->P) {  // a mesh needs 1 <= P; the plan admits P <= 8
      case 1: launch_dg_transport<1>(grid, st, d); break;
      case 2: launch_dg_transport<2>(grid, st, d); break;
      case 3: launch_dg_transport<3>(grid, st, d); break;
      case 4: launch_dg_transport<4>(grid, st, d); break;
      case 5: launch_dg_transport<5>(grid, st, d); break;
      case 6: launch_dg_transport<6>(grid, st, d); break;
      case 7: launch_dg_transport<7>(grid, st, d); break;
      default: launch_dg_transport<8>(grid, st, d); break;
    }
  }
  if (tr.m2) {
    const dgfs_mesh2d *m = tr.m2;
    DG2Args d{};
    d.N = N;
    d.ns = ns;
    d.Kx = m->Kx;
    d.Ky = m->Ky;
    d.P = pl->P;
    d.periodic[0] = m->periodic_x ? 1 : 0;
    d.periodic[1] = m->periodic_y ? 1 : 0;
    d.L = pl->L;
    d.hx = (m->x_right - m->x_left) / m->Kx;
    d.hy = (m->y_top - m->y_bottom) / m->Ky;
    for (int p = 0; p < ns; ++p) d.mass[p] = pl->mass[p];
    const double *uws[4] = {m->u_left, m->u_right, m->u_bottom, m->u_top};
    const double Tws[4] = {m->T_left, m->T_right, m->T_bottom, m->T_top};
    for (int sd = 0; sd < 4; ++sd) {
      for (int c = 0; c < 3; ++c) d.uw[sd][c] = uws[sd][c];
      d.Tw[sd] = Tws[sd];
    }
    const int np1 = pl->P + 1;
    for (int i = 0; i < np1 * np1; ++i) {
      d.Dr[i] = pl->dg_Dr[i];
      d.Minv[i] = pl->dg_Minv[i];
    }
    d.F = F;
    d.dF = dF;
    d.nw = nw;
    const int walls = ((m->periodic_x ? 0 : 2 * m->Ky) + (m->periodic_y ? 0 : 2 * m->Kx)) * np1 * ns;
    if (walls > 0)
      DGFS_LAUNCH("k_wall_density_2d", k_wall_density_2d, dim3(walls), dim3(kWallThreads), 0, st, d, nw);
    const unsigned ey = (unsigned)std::min(m->Kx * m->Ky, 64);
    DGFS_LAUNCH("k_dg_transport_2d", k_dg_transport_2d, dim3((unsigned)((n3 + 255) / 256), ey, ns), dim3(256), 0,
                st, d);
  }
  const int npairs = ns * ns;
  PipeArgs a{};
  pipeline_common(pl, a);
  pipeline_carve(pl, l.B, npairs, ns, ws, a);
  a.n_pairs = npairs;
  a.nz = ns;
  for (int p = 0; p < ns; ++p)
    for (int q = 0; q < ns; ++q) {
      a.pair_id[p * ns + q] = p * ns + q;
      a.zp[p * ns + q] = p;
      a.zq[p * ns + q] = q;
      a.xshare[p * ns + q] = p == q ? 1 : 0;
    }
  pipeline_slots(pl, a);
  const int64_t node_stride = ns * n3;
  for (int64_t n0 = 0; n0 < n_nodes; n0 += l.B) {
    const int nb = (int)std::min<int64_t>(l.B, n_nodes - n0);
    a.n_nodes = nb;
    FwdArgs fw{};
    for (int p = 0; p < ns; ++p) fw.src[p] = F + n0 * node_stride + p * n3;
    fw.node_stride = node_stride;
    fw.n_nodes = nb;
    fw.nz = ns;
    fw.Z = a.Z;
    FinalArgs fa{};
    fa.n_out = ns;
    fa.qcount = ns;
    for (int p = 0; p < ns; ++p) {
      fa.fsrc[p] = F + n0 * node_stride + p * n3;
      fa.out[p] = project ? qc + p * n3 : dF + n0 * node_stride + p * n3;
    }
    fa.f_stride = node_stride;
    fa.out_stride = project ? node_stride : node_stride;
    fa.accumulate = (!project && tr.any()) ? 1 : 0;
    hipError_t e = launch_pipeline(pl, a, fw, fa, st, true);
    if (e != hipSuccess) return e;
    if (project) {
      ProjArgs pa{};
      pa.N = N;
      pa.nsp = ns;
      pa.nrow = ns + 4;
      pa.accumulate = tr.any() ? 1 : 0;
      pa.L = pl->L;
      for (int p = 0; p < ns; ++p) pa.mass[p] = pl->mass[p];
      std::memcpy(pa.ginv, pl->proj_ginv.data(), pl->proj_ginv.size() * sizeof(double));
      pa.Q = qc;
      pa.q_stride = node_stride;
      for (int p = 0; p < ns; ++p) pa.out[p] = dF + n0 * node_stride + p * n3;
      pa.out_stride = node_stride;
      pa.nblk = kProjBlocks;
      pa.part = part;
      if ((e = launch_projection(pa, nb, st)) != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

static hipError_t enqueue_step(const dgfs_plan_s *pl, const Transport &tr, int64_t n_nodes, double *F, double dt,
                               uint32_t flags, void *ws, hipStream_t st) {
  const RhsLayout l = rhs_layout(pl, n_nodes);
  const int64_t n = n_nodes * pl->ns * (int64_t)pl->N * pl->N * pl->N;
  const size_t state = align256((size_t)n * sizeof(double));
  char *base = static_cast<char *>(ws) + l.total();
  double *R = reinterpret_cast<double *>(base);
  double *F1 = reinterpret_cast<double *>(base + state);
  double *F2 = reinterpret_cast<double *>(base + 2 * state);
  const dim3 g((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), b(256);
  hipError_t e;
  if (flags & DGFS_EULER) {
    if ((e = enqueue_rhs(pl, tr, n_nodes, F, R, flags, ws, st)) != hipSuccess) return e;
    DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F, F, F, R, 0.0, 1.0, dt, n);
    return hipGetLastError();
  }
  // Shu-Osher SSP-RK3
  if ((e = enqueue_rhs(pl, tr, n_nodes, F, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F1, F, F, R, 0.0, 1.0, dt, n);
  if ((e = enqueue_rhs(pl, tr, n_nodes, F1, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F2, F, F1, R, 0.75, 0.25, dt, n);
  if ((e = enqueue_rhs(pl, tr, n_nodes, F2, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F, F, F2, R, 1.0 / 3.0, 2.0 / 3.0, dt, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- graph cache
// Everything a captured step depends on: the arguments, and the workspace
// layout (the chunk width, which dgfs_autotune may change, and the bytes the
// layout spans).
struct GraphKey {
  bool has_mesh;
  dgfs_mesh mesh;
  bool has_mesh2;
  dgfs_mesh2d mesh2;
  int64_t n_nodes;
  double *F;
  double dt;
  uint32_t flags;
  void *ws;
  int chunk_nodes;
  size_t ws_span;
  bool operator==(const GraphKey &o) const {
    return has_mesh == o.has_mesh && (!has_mesh || std::memcmp(&mesh, &o.mesh, sizeof(mesh)) == 0) &&
           has_mesh2 == o.has_mesh2 && (!has_mesh2 || std::memcmp(&mesh2, &o.mesh2, sizeof(mesh2)) == 0) &&
           n_nodes == o.n_nodes && F == o.F && dt == o.dt && flags == o.flags && ws == o.ws &&
           chunk_nodes == o.chunk_nodes && ws_span == o.ws_span;
  }
};
// One captured step per plan.  `done` is recorded on the caller's stream
// after the last replay, so that a recapture waits for every queued replay
// of the old executable graph before destroying it.
struct GraphCache {
  std::mutex mu;
  bool valid = false;
  GraphKey key{};
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

static std::mutex g_cache_create_mu;

static GraphCache *cache_of(dgfs_plan_s *pl) {
  std::lock_guard<std::mutex> lk(g_cache_create_mu);
  if (!pl->graph_cache) pl->graph_cache = new GraphCache();
  return static_cast<GraphCache *>(pl->graph_cache);
}

void destroy_graph_cache(dgfs_plan_s *pl) {
  if (!pl->graph_cache) return;
  auto *c = static_cast<GraphCache *>(pl->graph_cache);
  if (c->done && c->launched) (void)hipEventSynchronize(c->done);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->done) (void)hipEventDestroy(c->done);
  delete c;
  pl->graph_cache = nullptr;
}

static bool use_graphs() {
  static int v = [] {
    const char *s = std::getenv("DGFS_NO_GRAPH");
    return (s && s[0] == '1') ? 0 : 1;
  }();
  // kernel timing brackets every launch with events, which a graph would not replay
  return v != 0 && !prof::enabled();
}

}  // namespace dgfs

using namespace dgfs;

static dgfs_status validate_mesh2d(const dgfs_plan_s *pl, const dgfs_mesh2d *m, int64_t n_nodes, const char *who) {
  if (!pl) { set_error("%s: NULL plan", who); return DGFS_EINVAL; }
  if (!m) { set_error("%s: NULL mesh", who); return DGFS_EINVAL; }
  if (pl->P < 1 || pl->P + 1 > kMax2D) {
    set_error("%s: a 2-D mesh needs the plan's dg_order in 1 .. %d (it is %d)", who, kMax2D - 1, pl->P);
    return pl->P < 1 ? DGFS_EINVAL : DGFS_EUNSUPPORTED;
  }
  if (m->Kx < 1 || m->Ky < 1) { set_error("%s: mesh Kx and Ky must be >= 1", who); return DGFS_EINVAL; }
  const int64_t np1 = pl->P + 1;
  if ((int64_t)m->Kx * m->Ky * np1 * np1 != n_nodes) {
    set_error("%s: n_nodes %lld != Kx*Ky*(P+1)^2 = %lld", who, (long long)n_nodes,
              (long long)((int64_t)m->Kx * m->Ky * np1 * np1));
    return DGFS_EINVAL;
  }
  if (!(m->x_right > m->x_left) || !(m->y_top > m->y_bottom)) { set_error("%s: invalid mesh extent", who); return DGFS_EINVAL; }
  if ((!m->periodic_x && !(m->T_left > 0 && m->T_right > 0)) || (!m->periodic_y && !(m->T_bottom > 0 && m->T_top > 0))) {
    set_error("%s: wall temperatures must be > 0", who);
    return DGFS_EINVAL;
  }
  if ((size_t)(2 * ((int64_t)m->Kx + m->Ky) * np1 * pl->ns) > kWallCap) {
    set_error("%s: %lld boundary node densities exceed the %zu the workspace holds", who,
              (long long)(2 * ((int64_t)m->Kx + m->Ky) * np1 * pl->ns), kWallCap);
    return DGFS_EUNSUPPORTED;
  }
  return DGFS_OK;
}

static dgfs_status rhs_common(const dgfs_plan_s *pl, const Transport &tr, int64_t n_nodes, const double *F,
                              double *dFdt, uint32_t flags, void *ws, size_t ws_bytes, void *stream, const char *who) {
  if (flags & ~(DGFS_PROJECT | DGFS_CHECK)) { set_error("%s: unsupported flags 0x%x", who, flags); return DGFS_EINVAL; }
  if (!F || !dFdt) { set_error("%s: NULL array", who); return DGFS_EINVAL; }
  const size_t need = rhs_layout(pl, n_nodes).total();
  if (!ws || ws_bytes < need) { set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need); return DGFS_EWORKSPACE; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_rhs(pl, tr, n_nodes, F, dFdt, flags, ws, st);
  if (e != hipSuccess) return hip_status(e, "right-hand side launch");
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  if (flags & DGFS_CHECK) return check_finite(dFdt, n_nodes * pl->ns, n3, n3, st);
  return DGFS_OK;
}

static dgfs_status step_common(dgfs_plan_s *pl, const Transport &tr, int64_t n_nodes, double *F, double dt,
                               int32_t n_steps, uint32_t flags, void *ws, size_t ws_bytes, void *stream,
                               const char *who) {
  if (flags & ~(DGFS_PROJECT | DGFS_CHECK | DGFS_EULER)) { set_error("%s: unsupported flags 0x%x", who, flags); return DGFS_EINVAL; }
  if (!F) { set_error("%s: NULL state", who); return DGFS_EINVAL; }
  if (n_steps < 0 || !std::isfinite(dt)) { set_error("%s: n_steps >= 0 and finite dt required", who); return DGFS_EINVAL; }
  const size_t need = extra_workspace_bytes(pl, n_nodes, DGFS_OP_STEP);
  if (!ws || ws_bytes < need) { set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need); return DGFS_EWORKSPACE; }
  if (n_steps == 0) return DGFS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t sflags = flags & ~DGFS_CHECK;
  hipError_t e = hipSuccess;
  if (!use_graphs()) {
    for (int i = 0; i < n_steps && e == hipSuccess; ++i) e = enqueue_step(pl, tr, n_nodes, F, dt, sflags, ws, st);
    if (e != hipSuccess) return hip_status(e, "step launch");
  } else {
    GraphCache *c = cache_of(pl);
    std::lock_guard<std::mutex> lk(c->mu);
    GraphKey key{};
    key.has_mesh = tr.m1 != nullptr;
    if (tr.m1) key.mesh = *tr.m1;
    key.has_mesh2 = tr.m2 != nullptr;
    if (tr.m2) key.mesh2 = *tr.m2;
    key.n_nodes = n_nodes;
    key.F = F;
    key.dt = dt;
    key.flags = sflags;
    key.ws = ws;
    key.chunk_nodes = rhs_layout(pl, n_nodes).B;
    key.ws_span = need;
    if (!c->valid || !(c->key == key)) {
      if (c->exec) {
        // earlier replays may still be queued on some stream: wait for them
        if (c->launched && (e = hipEventSynchronize(c->done)) != hipSuccess)
          return hip_status(e, "step: wait for earlier replays");
        (void)hipGraphExecDestroy(c->exec);
        c->exec = nullptr;
        c->launched = false;
      }
      c->valid = false;
      if (!c->done && (e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming)) != hipSuccess)
        return hip_status(e, "step event");
      if (!c->cap && (e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_status(e, "step capture stream");
      hipGraph_t graph = nullptr;
      if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_status(e, "step begin capture");
      hipError_t le = enqueue_step(pl, tr, n_nodes, F, dt, sflags, ws, c->cap);
      e = hipStreamEndCapture(c->cap, &graph);
      if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_status(le, "step capture"); }
      if (e != hipSuccess) return hip_status(e, "step end capture");
      e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_status(e, "step instantiate");
      c->key = key;
      c->valid = true;
    }
    for (int i = 0; i < n_steps && e == hipSuccess; ++i) e = hipGraphLaunch(c->exec, st);
    if (e == hipSuccess) {
      e = hipEventRecord(c->done, st);
      c->launched = true;
    }
    if (e != hipSuccess) return hip_status(e, "step graph launch");
  }
  if (flags & DGFS_CHECK) {
    const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
    return check_finite(F, n_nodes * pl->ns, n3, n3, st);
  }
  return DGFS_OK;
}

extern "C" dgfs_status dgfs_rhs(dgfs_plan pl, const dgfs_mesh *mesh, int64_t n_nodes, const double *F, double *dFdt,
                                uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_rhs(pl, mesh, n_nodes, "dgfs_rhs");
  if (s != DGFS_OK) return s;
  Transport tr;
  tr.m1 = mesh;
  return rhs_common(pl, tr, n_nodes, F, dFdt, flags, ws, ws_bytes, stream, "dgfs_rhs");
}

extern "C" dgfs_status dgfs_step(dgfs_plan pl, const dgfs_mesh *mesh, int64_t n_nodes, double *F, double dt,
                                 int32_t n_steps, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_rhs(pl, mesh, n_nodes, "dgfs_step");
  if (s != DGFS_OK) return s;
  Transport tr;
  tr.m1 = mesh;
  return step_common(pl, tr, n_nodes, F, dt, n_steps, flags, ws, ws_bytes, stream, "dgfs_step");
}

extern "C" dgfs_status dgfs_rhs_2d(dgfs_plan pl, const dgfs_mesh2d *mesh, int64_t n_nodes, const double *F,
                                   double *dFdt, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_mesh2d(pl, mesh, n_nodes, "dgfs_rhs_2d");
  if (s != DGFS_OK) return s;
  Transport tr;
  tr.m2 = mesh;
  return rhs_common(pl, tr, n_nodes, F, dFdt, flags, ws, ws_bytes, stream, "dgfs_rhs_2d");
}

extern "C" dgfs_status dgfs_step_2d(dgfs_plan pl, const dgfs_mesh2d *mesh, int64_t n_nodes, double *F, double dt,
                                    int32_t n_steps, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_mesh2d(pl, mesh, n_nodes, "dgfs_step_2d");
  if (s != DGFS_OK) return s;
  Transport tr;
  tr.m2 = mesh;
  return step_common(pl, tr, n_nodes, F, dt, n_steps, flags, ws, ws_bytes, stream, "dgfs_step_2d");
}
