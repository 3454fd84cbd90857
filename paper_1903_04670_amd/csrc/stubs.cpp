// Entry points not yet implemented in this build.
#include "internal.hpp"
#include <hip/hip_runtime.h>

namespace dgfs {
}
using namespace dgfs;
extern "C" size_t dgfs_batched_workspace_bytes(const dgfs_plan *, int32_t, const dgfs_item *, int64_t) { return 0; }
extern "C" dgfs_status dgfs_collide_batched(const dgfs_plan *, int32_t, const dgfs_item *, int64_t, uint32_t, void *,
                                            size_t, void *) {
  set_error("dgfs_collide_batched: not implemented");
  return DGFS_EUNSUPPORTED;
}
