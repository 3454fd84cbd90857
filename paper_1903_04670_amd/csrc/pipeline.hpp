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
// NaN/Inf scan of n_nodes blocks of n3 doubles at stride; synchronises the stream.
dgfs_status check_finite(const double *x, int64_t n_nodes, int64_t n3, int64_t stride, hipStream_t st);
size_t extra_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes, int32_t op);
size_t vjp_workspace_bytes(const dgfs_plan_s *pl, int64_t n_nodes);
void destroy_graph_cache(dgfs_plan_s *pl);
}  // namespace dgfs
