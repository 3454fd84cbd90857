// Shared host-side helpers of the collision pipeline (used by every entry point).
#pragma once
#include "collide_kernels.hpp"

namespace dgfs {
hipError_t launch_pipeline(const dgfs_plan_s *pl, const PipeArgs &a, const FwdArgs &fw, const FinalArgs &fa,
                           hipStream_t st, bool do_fwd);
int max_evals_per_chunk();
int chunk_nodes(const dgfs_plan_s *pl, int64_t n_nodes, int n_pairs);
size_t pipeline_bytes(const dgfs_plan_s *pl, int B, int n_pairs, int nz);
void pipeline_carve(const dgfs_plan_s *pl, int B, int n_pairs, int nz, void *ws, PipeArgs &a);
void pipeline_common(const dgfs_plan_s *pl, PipeArgs &a);
// Gain schedule of a PipeArgs whose n_pairs, pair_id, zp, zq and xshare are
// set: which slots compute their gain sums, which reuse another slot's, and
// which sum over half of an antipodal sphere set.  DGFS_NO_SYMMETRY turns the
// reuse off (every slot computes its full sum).
void pipeline_slots(const dgfs_plan_s *pl, PipeArgs &a);
bool symmetry_enabled();
// dgfs_collide's workspace for chunks of B nodes (pipeline arrays, then the
// unprojected term and partial moments of DGFS_PROJECT).
size_t collide_bytes(const dgfs_plan_s *pl, int B, int nz);
// Largest chunk width (at most the default) whose workspace fits `bytes`; 0 if none.
int collide_chunk_fitting(const dgfs_plan_s *pl, int64_t n_nodes, int nz, size_t bytes);
dgfs_status collide_validate(const dgfs_plan_s *pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                             const double *fq, int64_t node_stride, const double *Q, int64_t out_stride,
                             uint32_t flags, uint32_t allowed, const char *who);
// The collision of dgfs_collide in chunks of B nodes on a workspace of
// ws_bytes >= collide_bytes(pl, B, nz) (arguments already validated).
dgfs_status collide_impl(const dgfs_plan_s *pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                         const double *fq, int64_t node_stride, double *Q, int64_t out_stride, uint32_t flags,
                         void *ws, size_t ws_bytes, hipStream_t st, int B, const char *who);
// NaN/Inf scan of n_nodes blocks of n3 doubles at stride; synchronises the stream.
dgfs_status check_finite(const double *x, int64_t n_nodes, int64_t n3, int64_t stride, hipStream_t st);
// Conservation projection Q~ = Q - C^T (C C^T)^{-1} C Q of each node's
// collision term (FP64).  Rows of C: the mass of each of the nsp species,
// then, when nrow = nsp + 4, total momentum (x, y, z) and total energy.
constexpr int kProjBlocks = 32;  // partial-moment blocks per node
struct ProjArgs {
  int N, nsp, nrow, accumulate, nblk;  // nblk: partial-moment blocks per node
  double L;
  double mass[DGFS_MAX_SPECIES];
  double ginv[(DGFS_MAX_SPECIES + 4) * (DGFS_MAX_SPECIES + 4)];  // (C C^T)^{-1}, nrow x nrow
  const double *Q;   // node n, species a block at Q + n*q_stride + a*n3
  int64_t q_stride;
  double *out[DGFS_MAX_SPECIES];  // species a of node n at out[a] + n*out_stride
  int64_t out_stride;
  double *part;      // [node][nblk][nrow] partial moments
};
// Bytes of the partial-moment buffer for B nodes.
inline size_t proj_part_bytes(int B) {
  return ((size_t)B * kProjBlocks * (DGFS_MAX_SPECIES + 4) * sizeof(double) + 255) / 256 * 256;
}
hipError_t launch_projection(const ProjArgs &pa, int n_nodes, hipStream_t st);
size_t extra_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes, int32_t op);
size_t vjp_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes);
void destroy_graph_cache(dgfs_plan_s *pl);
}  // namespace dgfs
