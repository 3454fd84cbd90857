// Kernel launch wrapper with optional per-kernel HIP-event timing.
#pragma once
#include <hip/hip_runtime.h>

namespace dgfs {
namespace prof {
bool enabled();
void *begin(const char *name, hipStream_t st);
void end(void *token, hipStream_t st);
}  // namespace prof
}  // namespace dgfs

#define DGFS_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHM, ST, ...)                              \
  do {                                                                                    \
    void *dgfs_tok_ = ::dgfs::prof::enabled() ? ::dgfs::prof::begin(NAME, ST) : nullptr; \
    hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, ST, __VA_ARGS__);                        \
    if (dgfs_tok_) ::dgfs::prof::end(dgfs_tok_, ST);                                      \
  } while (0)
