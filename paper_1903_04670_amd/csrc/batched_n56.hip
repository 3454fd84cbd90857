// The N <= 56 class of the batched launch (radix-5/7 grids N = 40, 56 and
// everything below), in a translation unit of its own so that it compiles
// in parallel with the smaller classes.
#include "batched_kernels.hpp"

namespace dgfs {
template hipError_t launch_batch<double, 56>(const SubItem *, const int *, const int *, int, size_t, hipStream_t);
template hipError_t launch_batch<float, 56>(const SubItem *, const int *, const int *, int, size_t, hipStream_t);
}  // namespace dgfs
