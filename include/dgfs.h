/*
 * dgfs.h -- C ABI of the MI355X fast spectral collision library.
 *
 * The library evaluates the multi-species fast Fourier-spectral Boltzmann
 * collision operator Q^{pq}(f^p, f^q) of Jaiswal, Hu, Brillon and Alexeenko,
 * "A discontinuous Galerkin fast spectral method for multi-species full
 * Boltzmann on streaming multi-processors" (PASC'19, arXiv:1903.04670):
 *   - the operator itself: Algorithm 2 (collision algorithm), with the tables
 *     of Algorithm 1 (pre-computation) evaluated in closed form,
 *   - its adjoint (vector-Jacobian product),
 *   - the right-hand side of the non-dimensional Boltzmann equation
 *     (Eq. bzeNonDim) with a nodal discontinuous Galerkin transport term in
 *     one space dimension (Sec. 3.3) or on a 2-D box of tensor-product
 *     elements, and SSP-RK3 / Euler time steps.
 *
 * Conventions (every entry point):
 *   - Array arguments are DEVICE pointers owned by the caller unless marked
 *     "host".  Nothing is retained after a call returns.
 *   - A distribution array F holds n_nodes x n_species blocks of N^3 doubles,
 *     block (node, p) at F + node*node_stride + p*N^3, each block indexed
 *     [x][y][z] with z fastest, velocity c_j = -L + (j + 1/2) h, h = 2L/N.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are stream
 *     ordered and asynchronous: they neither allocate device memory nor
 *     synchronise the host, with these exceptions:
 *       * dgfs_plan_create / dgfs_plan_destroy allocate and free the plan's
 *         tables and synchronise (destroy first waits for queued replays of
 *         the plan's captured step);
 *       * DGFS_CHECK allocates a 4-byte counter (stream-ordered
 *         hipMallocAsync) and synchronises the stream to read it;
 *       * dgfs_step, when its key (mesh, n_nodes, F, dt, flags, workspace,
 *         chunk width) differs from the captured one (always on the first
 *         call for a plan), creates a private capture stream and an event,
 *         captures and instantiates a HIP graph, and first waits on the host
 *         for the earlier graph's queued replays;
 *       * dgfs_collide_batched stages its item descriptors in a pinned host
 *         buffer (hipHostMalloc when a larger one is needed), waits on the
 *         host for the previous call's copy from that buffer, and serialises
 *         concurrent callers on a process-wide lock;
 *       * dgfs_autotune and dgfs_autotune_rhs synchronise the stream and
 *         create timing events;
 *       * while dgfs_profile_enable is on, every launch creates two events.
 *   - `ws` / `ws_bytes`: caller-owned device workspace of at least
 *     dgfs_workspace_bytes(plan, n_nodes, op) bytes, 256-byte aligned.
 *   - Validation errors are returned before anything is launched.  A HIP
 *     launch error is returned as DGFS_EHIP.  Nothing throws across the ABI;
 *     dgfs_last_error() gives a thread-local message for the last non-OK
 *     status.
 *   - A plan is immutable after creation, except that dgfs_autotune and
 *     dgfs_autotune_rhs store the schedule they pick in it, and may be used
 *     concurrently on different streams with distinct workspaces (the two
 *     autotuners excepted).
 */
#ifndef DGFS_H
#define DGFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgfs_plan_s *dgfs_plan;

typedef enum {
  DGFS_OK = 0,
  DGFS_EINVAL = -1,       /* invalid argument */
  DGFS_EUNSUPPORTED = -2, /* valid but not supported (e.g. an N the kernels are not built for) */
  DGFS_ENOMEM = -3,       /* plan tables could not be allocated */
  DGFS_EHIP = -4,         /* a HIP runtime call or launch failed */
  DGFS_EWORKSPACE = -5,   /* ws NULL or ws_bytes too small */
  DGFS_ENONFINITE = -6    /* DGFS_CHECK found a NaN/Inf in the result */
} dgfs_status;

typedef enum { DGFS_FP64 = 0, DGFS_FP32_MIXED = 1 } dgfs_precision;

/* Workspace queries */
typedef enum { DGFS_OP_COLLIDE = 0, DGFS_OP_VJP = 1, DGFS_OP_RHS = 2, DGFS_OP_STEP = 3 } dgfs_op;

/* flags */
#define DGFS_ACCUMULATE 0x1u /* add into the output instead of overwriting it        */
#define DGFS_PROJECT    0x2u /* conservation projection of the collision term (FP64)  */
#define DGFS_CHECK      0x4u /* host-synchronous NaN/Inf check of the output          */
#define DGFS_EULER      0x8u /* dgfs_step: forward Euler instead of SSP-RK3           */

/*
 * Problem statement (Sec. 2 and the inputs of Algorithms 1 and 2).  All
 * pointers are HOST pointers, read during dgfs_plan_create only.
 *   n_species      ns >= 1 (at most DGFS_MAX_SPECIES)
 *   mass[ns]       non-dimensional particle masses m_p > 0
 *   omega[ns*ns]   VSS viscosity index omega_pq (row p, column q), < 2.5
 *   alpha[ns*ns]   VSS scattering parameter alpha_pq > 0 (1 = VHS)
 *   beta[ns*ns]    kernel prefactor beta^{pq} (Sec. 2, the equation defining
 *                  beta); NULL => computed from kn
 *   kn[ns*ns]      Knudsen numbers Kn_pq (Eq. Kn); used when beta == NULL;
 *                  NULL together with beta == NULL => unit reduced Knudsen
 *                  number, beta = mu^{1/2-omega} alpha/(2^{1+alpha}
 *                  Gamma(5/2-omega) pi), mu = m_p m_q/(m_p+m_q)
 *   N              velocity points per axis: 4, 6, 8, 10, 12, 14, 16, 18, 24,
 *                  32, 36, 40, 48 or 56
 *   L              velocity box half-width: D_L = [-L, L]^3
 *   S              support radius of f (informational; R defaults from L)
 *   R[ns*ns]       truncation radius of the relative-velocity ball; NULL =>
 *                  R = 4L/(1 + max(4 m_q/(m_p+m_q), 2) + sqrt(1 + m_q/m_p))
 *                  (Sec. 2.1)
 *   M, sigma[M*3], w_sigma[M]
 *                  sphere quadrature: unit vectors and weights (sum 4 pi)
 *   N_rho          Gauss-Legendre points on [0, R] (the radial rule)
 *   dg_order       DG polynomial degree P (P+1 Gauss-Lobatto nodes per
 *                  element); only used by dgfs_rhs/dgfs_step, 0 otherwise
 *   precision      DGFS_FP64, or DGFS_FP32_MIXED (FP32 transforms; the
 *                  sums over directions and radii compensated in FP32 or
 *                  carried in FP64; inputs/outputs stay FP64)
 *   nyquist_zero   0: Algorithm 2 as it stands.  1: the gain's translates
 *                  t1, t2 are formed from fft(f^p), fft(f^q) with their
 *                  Nyquist planes (wave index -N/2 on any axis) set to zero;
 *                  the loss term is unchanged.  Not in the paper: it changes
 *                  Q by the Nyquist content of the inputs, which is at
 *                  roundoff level for distributions supported well inside
 *                  D_L.  t1 and t2 are then Hermitian, so u1 and u2 are real
 *                  and the VHS gain evaluates both with one complex
 *                  transform of t1 + i t2.  Applies to every entry point
 *                  (dgfs_collide_vjp differentiates this operator).
 */
#define DGFS_MAX_SPECIES 4
typedef struct {
  int32_t n_species;
  const double *mass;
  const double *omega;
  const double *alpha;
  const double *beta;
  const double *kn;
  int32_t N;
  double L;
  double S;
  const double *R;
  int32_t M;
  const double *sigma;
  const double *w_sigma;
  int32_t N_rho;
  int32_t dg_order;
  int32_t precision;
  int32_t nyquist_zero;
} dgfs_params;

/* Builds the tables of Algorithm 1 for every ordered pair (host FP64, then
 * uploaded).  Synchronous; allocates device memory owned by the plan. */
dgfs_status dgfs_plan_create(const dgfs_params *params, dgfs_plan *out);
void dgfs_plan_destroy(dgfs_plan plan);

/* Device workspace needed by `op` for n_nodes spatial nodes. */
size_t dgfs_workspace_bytes(dgfs_plan plan, int64_t n_nodes, int32_t op);

/*
 * Q^{pq}(f^p, f^q) at n_nodes nodes (Algorithm 2, including the prefactor
 * beta^{pq}):
 *   Q = beta Re( ifft(QG) - f^p * ifft(c * fft(f^q)) ),
 *   QG = sum_{r,m} w_r w_m b_rm * fft( ifft(e^{i m_q/(m_p+m_q) a} fft f^p)
 *                                     * ifft(e^{-i m_p/(m_p+m_q) a} fft f^q) ).
 *   fp, fq     device, node n block at fp + n*node_stride (N^3 doubles each)
 *   Q          device, node n block at Q + n*out_stride
 *   flags      DGFS_ACCUMULATE, DGFS_PROJECT, DGFS_CHECK
 * DGFS_PROJECT replaces each node's Q by its FP64 least-squares projection
 * Q - C^T (C C^T)^{-1} C Q onto the invariants this single term conserves
 * (Sec. 2: collisions conserve the mass of each species and the total
 * momentum and energy).  Q^{pq} alone conserves the mass of species p, the
 * one row of C (weight h^3).  The self-collision term of one distribution
 * (p == q and fp == fq, the same pointer) also conserves momentum and
 * energy: rows m_p c_d h^3 (d = x, y, z) and m_p |c|^2/2 h^3.  With
 * DGFS_ACCUMULATE the projected term is added into Q.
 */
dgfs_status dgfs_collide(dgfs_plan plan, int64_t n_nodes, int32_t p, int32_t q,
                         const double *fp, const double *fq, int64_t node_stride,
                         double *Q, int64_t out_stride, uint32_t flags,
                         void *ws, size_t ws_bytes, void *stream);

/*
 * dgfs_collide for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument; the pipeline's arrays live in a 256 MiB device array
 * of the library, one per GPU, held from the first call on that GPU until
 * the process ends.  Same operator, arguments and results as dgfs_collide
 * (bit for bit); nodes run in chunks that fit the array (N = 32, M = 12,
 * N_rho = 16: 2 nodes per launch in FP64, 5 in FP32-mixed).  Calls no
 * hipMalloc, hipFree or other allocating routine.
 *   flags    DGFS_ACCUMULATE, DGFS_PROJECT (DGFS_CHECK, which allocates and
 *            synchronises, is refused with DGFS_EINVAL)
 * Returns DGFS_EUNSUPPORTED when one node needs more than 256 MiB (e.g.
 * N = 48 with N_rho = 24 in FP64).  Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one
 * GPU (different streams or threads) race, so serialise them.
 */
dgfs_status dgfs_collide_noalloc(dgfs_plan plan, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                 const double *fq, int64_t node_stride, double *Q, int64_t out_stride,
                                 uint32_t flags, void *stream);

/*
 * Vector-Jacobian product of dgfs_collide: for a cotangent wbar (same layout
 * as Q) returns grad_fp = (dQ/df^p)^T wbar and grad_fq = (dQ/df^q)^T wbar.
 * Intermediates of the (r, m) loop are recomputed, not stored (VSS plans
 * keep one transformed cotangent per (r, m) in the workspace, VHS plans one
 * per r).  When fp and
 * fq are the same array (p == q) the gradient with respect to it is the sum
 * of the two outputs.  flags: DGFS_ACCUMULATE (add into grad_*).
 * grad_fp or grad_fq may be NULL to skip that side.
 */
dgfs_status dgfs_collide_vjp(dgfs_plan plan, int64_t n_nodes, int32_t p, int32_t q,
                             const double *fp, const double *fq, int64_t node_stride,
                             const double *wbar, int64_t wbar_stride,
                             double *grad_fp, double *grad_fq, int64_t grad_stride,
                             uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * One-dimensional (x) physical mesh for the DG transport term.  Host struct.
 *   K            number of elements on [x_left, x_right], uniform
 *   x_left/right domain ends (the paper's Couette case uses [0, 1])
 *   u_left[3], T_left, u_right[3], T_right
 *                purely diffuse (Maxwell) walls at the two ends; the wall
 *                density is fixed each stage by zero net mass flux
 * Nodes are element-major: node = e*(P+1) + i, i over the P+1 Gauss-Lobatto
 * points of element e.
 */
typedef struct {
  int32_t K;
  double x_left, x_right;
  double u_left[3], T_left;
  double u_right[3], T_right;
} dgfs_mesh;

/*
 * Right-hand side of Eq. (bzeNonDim):
 *   dF^p/dt = -c_x dF^p/dx (nodal DG, upwind flux, diffuse walls)
 *             + sum_q Q^{pq}(F^p, F^q).
 * mesh == NULL: space-homogeneous problem, n_nodes independent points and
 * no transport term.  Otherwise n_nodes must equal mesh->K*(dg_order+1).
 * F, dFdt: [node][species][N^3], contiguous (node stride ns*N^3).
 * flags: DGFS_PROJECT projects the collision term of each node onto zero
 * mass (per species), momentum and energy change (FP64, Lagrange multipliers).
 */
dgfs_status dgfs_rhs(dgfs_plan plan, const dgfs_mesh *mesh, int64_t n_nodes,
                     const double *F, double *dFdt, uint32_t flags,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * n_steps time steps of size dt on F in place: SSP-RK3 (Shu-Osher), or
 * forward Euler with DGFS_EULER.  Same mesh/flags meaning as dgfs_rhs.  The
 * stage sequence is captured once into a HIP graph per (plan, stream shape)
 * and replayed.
 */
dgfs_status dgfs_step(dgfs_plan plan, const dgfs_mesh *mesh, int64_t n_nodes,
                      double *F, double dt, int32_t n_steps, uint32_t flags,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Two-dimensional (x, y) physical mesh for the DG transport term: the
 * extension to higher spatial dimensions that Sec. 3.3 leaves to future
 * work (its footnote).  Host struct.
 *   Kx, Ky       elements in x and y: uniform rectangles on
 *                [x_left, x_right] x [y_bottom, y_top]
 *   periodic_x   1: periodic in x (the left/right wall fields are unused);
 *                0: purely diffuse (Maxwell) walls at x_left and x_right
 *   periodic_y   the same for y and the bottom/top walls
 *   u_*[3], T_*  wall velocity and temperature of each side; the wall
 *                density of every boundary node is fixed each stage by zero
 *                net mass flux through that node
 * Tensor-product Gauss-Lobatto nodes, (P+1)^2 per element (P = the plan's
 * dg_order, 1 <= P <= 4), upwind flux on every face.  Node order:
 *   node = ((ey*Kx + ex)*(P+1) + j)*(P+1) + i,  i along x, j along y.
 * The boundary nodes of all walls and species must number at most 8192
 * (2 (Kx + Ky) (P+1) ns <= 8192).
 */
typedef struct {
  int32_t Kx, Ky;
  double x_left, x_right, y_bottom, y_top;
  int32_t periodic_x, periodic_y;
  double u_left[3], T_left;
  double u_right[3], T_right;
  double u_bottom[3], T_bottom;
  double u_top[3], T_top;
} dgfs_mesh2d;

/*
 * dgfs_rhs and dgfs_step on a 2-D mesh: dF^p/dt = -(c_x dF^p/dx + c_y
 * dF^p/dy) + sum_q Q^{pq}(F^p, F^q), the collision term as in dgfs_rhs
 * (flags DGFS_PROJECT and DGFS_CHECK; DGFS_EULER for the step).  n_nodes
 * must equal Kx*Ky*(P+1)^2; F and dFdt are [node][species][N^3]; the
 * workspace is that of DGFS_OP_RHS / DGFS_OP_STEP for n_nodes.
 */
dgfs_status dgfs_rhs_2d(dgfs_plan plan, const dgfs_mesh2d *mesh, int64_t n_nodes, const double *F,
                        double *dFdt, uint32_t flags, void *ws, size_t ws_bytes, void *stream);
dgfs_status dgfs_step_2d(dgfs_plan plan, const dgfs_mesh2d *mesh, int64_t n_nodes, double *F, double dt,
                         int32_t n_steps, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * Heterogeneous batch: items of different plans (different N, species,
 * quadratures) evaluated by one launch per pipeline stage.
 *   plans[n_plans]  host array of plans
 *   items[n_items]  host array; item i evaluates Q^{pq} of plans[plan] on
 *                   n_nodes nodes, like dgfs_collide
 * The results equal those of one dgfs_collide call per item bit for bit.
 * Items run concurrently: the output ranges of different items must not
 * share an element (with or without DGFS_ACCUMULATE); interleaved strided
 * outputs that touch distinct elements are fine.  Items with n_nodes == 0
 * are skipped.  flags: DGFS_ACCUMULATE only.
 */
typedef struct {
  int32_t plan;
  int32_t p, q;
  int64_t n_nodes;
  const double *fp, *fq;
  int64_t node_stride;
  double *Q;
  int64_t out_stride;
} dgfs_item;
size_t dgfs_batched_workspace_bytes(const dgfs_plan *plans, int32_t n_plans,
                                    const dgfs_item *items, int64_t n_items);
dgfs_status dgfs_collide_batched(const dgfs_plan *plans, int32_t n_plans,
                                 const dgfs_item *items, int64_t n_items, uint32_t flags,
                                 void *ws, size_t ws_bytes, void *stream);

/*
 * Per-kernel timing for measurement tools.  While enabled (process-wide),
 * every kernel this library launches is bracketed by two HIP events recorded
 * on the stream it is launched on, and dgfs_step enqueues its stages directly
 * instead of replaying a captured graph.  dgfs_profile_enable(on) discards
 * earlier records.  dgfs_profile_read waits for the recorded events and
 * fills, for up to `cap` kernel families, names[i*64 .. i*64+63] (host,
 * NUL-terminated), counts[i] (launches) and total_ms[i] (summed durations);
 * it returns the number of families recorded (may exceed cap).
 */
dgfs_status dgfs_profile_enable(int32_t on);
int32_t dgfs_profile_read(int32_t cap, char *names, int64_t *counts, double *total_ms);

/*
 * Launch-schedule autotuning.  Times dgfs_collide on the given inputs over
 * three schedule dimensions, none of which changes a result bit: the chunk
 * width (evaluations per launch: 8 .. 256, those whose workspace fits in
 * ws_bytes), then at the best width the number of blocks splitting each
 * x-line set's (r, sigma_x) loop in the x-shift stage (1, 2, 4, 8), then
 * whether the x stage of the gain serves a mirrored pair slot in the same
 * pass.  After a warm-up the default schedule is timed first and kept in
 * each dimension unless a candidate is more than 3% faster; a pick other
 * than the default is then timed against the default alternately, three
 * times each, and kept only if its median still wins by that margin (so
 * that timing noise does not move the schedule).  The pick is kept in the
 * plan; `chosen` (host int32[3], may be
 * NULL) receives (width, split, fusion), width 0, split 0 and fusion -1
 * meaning the default was kept.  Give it at least as many evaluations as a
 * launch of the widest candidate holds (256 in FP64), or the wide widths
 * time the same work.  The choice is appended to a text cache
 * (path $DGFS_TUNE_CACHE, default ~/.cache/dgfs_tune.txt) keyed by GPU
 * architecture and plan shape, and dgfs_plan_create reads it unless
 * DGFS_NO_TUNE_CACHE is set.  Synchronises the stream; overwrites Q; must
 * not run concurrently with other calls on the same plan.  Query the
 * workspace again afterwards: it depends on the chunk width.
 */
dgfs_status dgfs_autotune(dgfs_plan plan, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                          const double *fq, int64_t node_stride, double *Q, int64_t out_stride,
                          void *ws, size_t ws_bytes, void *stream, int32_t *chosen);

/*
 * The same search as dgfs_autotune, timing dgfs_rhs (mesh, n_nodes, F, dFdt
 * and flags as there) instead of one ordered pair: the schedule a
 * right-hand side or a time step of this shape should run (all its pairs,
 * the reuse of gain sums, the transport).  ws must hold the right-hand side
 * of the default schedule; wider candidates that do not fit are skipped.
 * Overwrites dFdt; otherwise as dgfs_autotune.
 */
dgfs_status dgfs_autotune_rhs(dgfs_plan plan, const dgfs_mesh *mesh, int64_t n_nodes, const double *F,
                              double *dFdt, uint32_t flags, void *ws, size_t ws_bytes, void *stream,
                              int32_t *chosen);

/* Thread-local message describing the last non-OK status of this thread. */
const char *dgfs_last_error(void);

/* ------------------------------------------------------------ host helpers */
/* Sphere quadrature sets on the full sphere, equal weights 4 pi/M:
 * kind 0 = octahedron (M = 6), 1 = icosahedron (M = 12), 2 = Fibonacci
 * lattice (any M >= 1).  sigma[M*3], w[M]: host outputs. */
dgfs_status dgfs_sphere_set(int32_t kind, int32_t M, double *sigma, double *w);

/* Copies a plan table to host memory (for tests): which = 0: radial
 * Gauss-Legendre nodes rho[N_rho]; 1: weights w_rho[N_rho]; 2: loss table
 * c(k) on the N^3 wave grid; 3: gain table b_{r m}(k) [N_rho][M][N^3]
 * (real part); 4: its imaginary part; 5: beta (1 value).  `n` is the
 * capacity of `out` in doubles. */
dgfs_status dgfs_plan_table(dgfs_plan plan, int32_t p, int32_t q, int32_t which,
                            double *out, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* DGFS_H */
