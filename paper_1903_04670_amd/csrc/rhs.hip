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
  const double *nw;  // [2][ns] wall densities
};

__device__ __forceinline__ double grid_c(int j, int N, double L) { return -L + (j + 0.5) * (2.0 * L / N); }

__device__ __forceinline__ double wall_maxwellian(double m, const double *u, double T, double cx, double cy, double cz) {
  const double dx = cx - u[0], dy = cy - u[1], dz = cz - u[2];
  const double a = m / (M_PI * T);
  return a * sqrt(a) * exp(-m * (dx * dx + dy * dy + dz * dz) / T);
}

// Wall densities n_w from zero discrete net mass flux (one block per wall and
// species; fixed-order reduction).
constexpr int kWallThreads = 1024;

__global__ void __launch_bounds__(kWallThreads) k_wall_density(DGArgs a, double *nw) {
  const int wall = blockIdx.x / a.ns, p = blockIdx.x % a.ns;
  const int N = a.N, n3 = N * N * N;
  const int node = wall == 0 ? 0 : a.K * (a.P + 1) - 1;
  const double *f = a.F + ((size_t)node * a.ns + p) * n3;
  double out = 0.0, unit = 0.0;
  for (int v = threadIdx.x; v < n3; v += kWallThreads) {
    const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
    if (wall == 0) {  // emits c_x > 0, absorbs c_x < 0
      if (cx < 0) out -= cx * f[v];
      else unit += cx * wall_maxwellian(a.mass[p], a.uw[wall], a.Tw[wall], cx, cy, cz);
    } else {
      if (cx > 0) out += cx * f[v];
      else unit -= cx * wall_maxwellian(a.mass[p], a.uw[wall], a.Tw[wall], cx, cy, cz);
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
  if (threadIdx.x == 0) nw[wall * a.ns + p] = so[0] / su[0];
}

// dF/dt = -c_x dF/dx by nodal DG (strong form, upwind flux).  One thread per
// (species, velocity point, element); blockIdx.y strides over the elements.
__global__ void __launch_bounds__(256) k_dg_transport(DGArgs a) {
  const int N = a.N, n3 = N * N * N, P = a.P, np1 = a.P + 1;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.z;
  if (v >= n3) return;
  const double cx = grid_c(v / (N * N), N, a.L);
  const size_t ns_stride = (size_t)a.ns * n3;
  const double *f = a.F + (size_t)p * n3 + v;
  double *df = a.dF + (size_t)p * n3 + v;
  const double s = 2.0 / a.h;
  for (int e = blockIdx.y; e < a.K; e += gridDim.y) {
    double u[kMaxDG];
    for (int i = 0; i <= P; ++i) u[i] = f[(size_t)(e * np1 + i) * ns_stride];
    double uL, uR;
    if (e == 0) {
      const double cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
      uL = cx > 0 ? a.nw[p] * wall_maxwellian(a.mass[p], a.uw[0], a.Tw[0], cx, cy, cz) : 0.0;
    } else {
      uL = f[(size_t)(e * np1 - 1) * ns_stride];
    }
    if (e == a.K - 1) {
      const double cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
      uR = cx < 0 ? a.nw[a.ns + p] * wall_maxwellian(a.mass[p], a.uw[1], a.Tw[1], cx, cy, cz) : 0.0;
    } else {
      uR = f[(size_t)((e + 1) * np1) * ns_stride];
    }
    // boundary terms n (c u - F*) with the upwind flux F*
    const double termR = cx > 0 ? 0.0 : cx * (u[P] - uR);
    const double termL = cx > 0 ? -cx * (u[0] - uL) : 0.0;
    for (int i = 0; i <= P; ++i) {
      double d = 0.0;
      for (int j = 0; j <= P; ++j) d += a.Dr[i * np1 + j] * u[j];
      df[(size_t)(e * np1 + i) * ns_stride] = s * (-cx * d + a.Minv[i * np1 + P] * termR + a.Minv[i * np1] * termL);
    }
  }
}

struct ProjArgs {
  int N, nsp, accumulate, nblk;  // nblk: partial-moment blocks per node
  double L;
  double mass[DGFS_MAX_SPECIES];
  double ginv[(DGFS_MAX_SPECIES + 4) * (DGFS_MAX_SPECIES + 4)];
  const double *Q;   // node n, species a block at Q + n*q_stride + a*n3
  int64_t q_stride;
  double *out[DGFS_MAX_SPECIES];  // species a of node n at out[a] + n*out_stride
  int64_t out_stride;
  double *part;      // [node][nblk][nsp+4] partial moments
};

constexpr int kProjThreads = 256;

// Partial moments C Q over a slice of one node's ns*N^3 values (fixed-order
// tree reduction, so the result is deterministic).  Rows of C: mass of each
// species, total momentum (x, y, z) and total energy, weight h^3.
__global__ void __launch_bounds__(kProjThreads) k_proj_moments(ProjArgs a) {
  const int node = blockIdx.y, blk = blockIdx.x;
  const int N = a.N, n3 = N * N * N, k = a.nsp + 4, total = a.nsp * n3;
  const double h = 2.0 * a.L / N, w = h * h * h;
  const double *Q = a.Q + (size_t)node * a.q_stride;
  double mom[DGFS_MAX_SPECIES + 4];
  for (int i = 0; i < k; ++i) mom[i] = 0.0;
  const int per = (total + a.nblk - 1) / a.nblk;
  const int lo = blk * per, hi = min(total, lo + per);
  for (int i = lo + threadIdx.x; i < hi; i += kProjThreads) {
    const int sp = i / n3, v = i % n3;
    const double q = Q[(size_t)sp * n3 + v], m = a.mass[sp];
    const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
    mom[sp] += w * q;
    mom[a.nsp + 0] += w * m * cx * q;
    mom[a.nsp + 1] += w * m * cy * q;
    mom[a.nsp + 2] += w * m * cz * q;
    mom[a.nsp + 3] += w * 0.5 * m * (cx * cx + cy * cy + cz * cz) * q;
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
  const int N = a.N, n3 = N * N * N, k = a.nsp + 4, total = a.nsp * n3;
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
  for (int i = lo + threadIdx.x; i < hi; i += kProjThreads) {
    const int sp = i / n3, v = i % n3;
    const double m = a.mass[sp];
    const double cx = grid_c(v / (N * N), N, a.L), cy = grid_c((v / N) % N, N, a.L), cz = grid_c(v % N, N, a.L);
    const double corr = w * (lam[sp] + m * (lam[a.nsp] * cx + lam[a.nsp + 1] * cy + lam[a.nsp + 2] * cz) +
                             0.5 * m * (cx * cx + cy * cy + cz * cz) * lam[a.nsp + 3]);
    const double val = Q[(size_t)sp * n3 + v] - corr;
    double *o = a.out[sp] + (size_t)node * a.out_stride;
    if (a.accumulate) o[v] += val;
    else o[v] = val;
  }
}

// out = a*X + b*(Y + dt*R), elementwise
__global__ void k_combine(double *out, const double *X, const double *Y, const double *R, double a, double b,
                          double dt, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * X[i] + b * (Y[i] + dt * R[i]);
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

constexpr int kProjBlocks = 32;  // partial-moment blocks per node

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
  l.nw = 256;
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
static hipError_t enqueue_rhs(const dgfs_plan_s *pl, const dgfs_mesh *mesh, int64_t n_nodes, const double *F,
                              double *dF, uint32_t flags, void *ws, hipStream_t st) {
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
    DGFS_LAUNCH("k_wall_density", k_wall_density, dim3(2 * ns), dim3(kWallThreads), 0, st, d, nw);
    // element slices in y (each thread strides over the rest); species in z
    const unsigned ey = (unsigned)std::min(mesh->K, 64);
    DGFS_LAUNCH("k_dg_transport", k_dg_transport, dim3((unsigned)((n3 + 255) / 256), ey, ns), dim3(256), 0, st, d);
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
    fa.accumulate = (!project && mesh) ? 1 : 0;
    hipError_t e = launch_pipeline(pl, a, fw, fa, st, true);
    if (e != hipSuccess) return e;
    if (project) {
      ProjArgs pa{};
      pa.N = N;
      pa.nsp = ns;
      pa.accumulate = mesh ? 1 : 0;
      pa.L = pl->L;
      for (int p = 0; p < ns; ++p) pa.mass[p] = pl->mass[p];
      std::memcpy(pa.ginv, pl->proj_ginv.data(), pl->proj_ginv.size() * sizeof(double));
      pa.Q = qc;
      pa.q_stride = node_stride;
      for (int p = 0; p < ns; ++p) pa.out[p] = dF + n0 * node_stride + p * n3;
      pa.out_stride = node_stride;
      pa.nblk = kProjBlocks;
      pa.part = part;
      DGFS_LAUNCH("k_proj_moments", k_proj_moments, dim3(kProjBlocks, nb), dim3(kProjThreads), 0, st, pa);
      DGFS_LAUNCH("k_proj_apply", k_proj_apply, dim3(kProjBlocks, nb), dim3(kProjThreads), 0, st, pa);
    }
  }
  return hipGetLastError();
}

static hipError_t enqueue_step(const dgfs_plan_s *pl, const dgfs_mesh *mesh, int64_t n_nodes, double *F, double dt,
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
    if ((e = enqueue_rhs(pl, mesh, n_nodes, F, R, flags, ws, st)) != hipSuccess) return e;
    DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F, F, F, R, 0.0, 1.0, dt, n);
    return hipGetLastError();
  }
  // Shu-Osher SSP-RK3
  if ((e = enqueue_rhs(pl, mesh, n_nodes, F, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F1, F, F, R, 0.0, 1.0, dt, n);
  if ((e = enqueue_rhs(pl, mesh, n_nodes, F1, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F2, F, F1, R, 0.75, 0.25, dt, n);
  if ((e = enqueue_rhs(pl, mesh, n_nodes, F2, R, flags, ws, st)) != hipSuccess) return e;
  DGFS_LAUNCH("k_combine", k_combine, g, b, 0, st, F, F, F2, R, 1.0 / 3.0, 2.0 / 3.0, dt, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- graph cache
struct GraphKey {
  bool has_mesh;
  dgfs_mesh mesh;
  int64_t n_nodes;
  double *F;
  double dt;
  uint32_t flags;
  void *ws;
  bool operator==(const GraphKey &o) const {
    return has_mesh == o.has_mesh && (!has_mesh || std::memcmp(&mesh, &o.mesh, sizeof(mesh)) == 0) &&
           n_nodes == o.n_nodes && F == o.F && dt == o.dt && flags == o.flags && ws == o.ws;
  }
};
struct GraphCache {
  std::mutex mu;
  bool valid = false;
  GraphKey key{};
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
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
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->cap) (void)hipStreamDestroy(c->cap);
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

extern "C" dgfs_status dgfs_rhs(dgfs_plan pl, const dgfs_mesh *mesh, int64_t n_nodes, const double *F, double *dFdt,
                                uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_rhs(pl, mesh, n_nodes, "dgfs_rhs");
  if (s != DGFS_OK) return s;
  if (flags & ~(DGFS_PROJECT | DGFS_CHECK)) { set_error("dgfs_rhs: unsupported flags 0x%x", flags); return DGFS_EINVAL; }
  if (!F || !dFdt) { set_error("dgfs_rhs: NULL array"); return DGFS_EINVAL; }
  const size_t need = rhs_layout(pl, n_nodes).total();
  if (!ws || ws_bytes < need) { set_error("dgfs_rhs: workspace %zu bytes, need %zu", ws_bytes, need); return DGFS_EWORKSPACE; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_rhs(pl, mesh, n_nodes, F, dFdt, flags, ws, st);
  if (e != hipSuccess) return hip_status(e, "dgfs_rhs launch");
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  if (flags & DGFS_CHECK) return check_finite(dFdt, n_nodes * pl->ns, n3, n3, st);
  return DGFS_OK;
}

extern "C" dgfs_status dgfs_step(dgfs_plan pl, const dgfs_mesh *mesh, int64_t n_nodes, double *F, double dt,
                                 int32_t n_steps, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  dgfs_status s = validate_rhs(pl, mesh, n_nodes, "dgfs_step");
  if (s != DGFS_OK) return s;
  if (flags & ~(DGFS_PROJECT | DGFS_CHECK | DGFS_EULER)) { set_error("dgfs_step: unsupported flags 0x%x", flags); return DGFS_EINVAL; }
  if (!F) { set_error("dgfs_step: NULL state"); return DGFS_EINVAL; }
  if (n_steps < 0 || !std::isfinite(dt)) { set_error("dgfs_step: n_steps >= 0 and finite dt required"); return DGFS_EINVAL; }
  const size_t need = extra_workspace_bytes(pl, n_nodes, DGFS_OP_STEP);
  if (!ws || ws_bytes < need) { set_error("dgfs_step: workspace %zu bytes, need %zu", ws_bytes, need); return DGFS_EWORKSPACE; }
  if (n_steps == 0) return DGFS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t sflags = flags & ~DGFS_CHECK;
  hipError_t e = hipSuccess;
  if (!use_graphs()) {
    for (int i = 0; i < n_steps && e == hipSuccess; ++i) e = enqueue_step(pl, mesh, n_nodes, F, dt, sflags, ws, st);
    if (e != hipSuccess) return hip_status(e, "dgfs_step launch");
  } else {
    GraphCache *c = cache_of(pl);
    std::lock_guard<std::mutex> lk(c->mu);
    GraphKey key{};
    key.has_mesh = mesh != nullptr;
    if (mesh) key.mesh = *mesh;
    key.n_nodes = n_nodes;
    key.F = F;
    key.dt = dt;
    key.flags = sflags;
    key.ws = ws;
    if (!c->valid || !(c->key == key)) {
      if (c->exec) { (void)hipGraphExecDestroy(c->exec); c->exec = nullptr; }
      c->valid = false;
      if (!c->cap && (e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_status(e, "dgfs_step capture stream");
      hipGraph_t graph = nullptr;
      if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_status(e, "dgfs_step begin capture");
      hipError_t le = enqueue_step(pl, mesh, n_nodes, F, dt, sflags, ws, c->cap);
      e = hipStreamEndCapture(c->cap, &graph);
      if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_status(le, "dgfs_step capture"); }
      if (e != hipSuccess) return hip_status(e, "dgfs_step end capture");
      e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_status(e, "dgfs_step instantiate");
      c->key = key;
      c->valid = true;
    }
    for (int i = 0; i < n_steps && e == hipSuccess; ++i) e = hipGraphLaunch(c->exec, st);
    if (e != hipSuccess) return hip_status(e, "dgfs_step graph launch");
  }
  if (flags & DGFS_CHECK) {
    const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
    return check_finite(F, n_nodes * pl->ns, n3, n3, st);
  }
  return DGFS_OK;
}
