// dgfs_collide_noalloc: the collision of dgfs_collide for callers that cannot
// allocate device memory.  The chunk arrays of the pipeline live in a
// file-scope device array instead of a caller workspace; everything else
// (kernels, chunk loop, projection) is dgfs_collide's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pipeline.hpp"

namespace dgfs {

// 256 MiB per device, held from the first call on that device until the
// process ends.  At N = 32 (icosahedron, N_rho = 16, FP64) one node needs
// about 90 MiB, so chunks of 2 nodes run; N = 40 with N_rho = 20 fits one
// node; larger plans are refused.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct ScratchSlot {
  std::once_flag once;
  void *ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];
}  // namespace

// Device address of `scratch` on the current device.  Host code must not use
// the array's name as an address (it is a host-side stand-in); the runtime
// resolves the symbol once per device, with that device current, and the
// address is kept.
static dgfs_status scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "dgfs_collide_noalloc: current device");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("dgfs_collide_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    return DGFS_EUNSUPPORTED;
  }
  ScratchSlot &s = g_scratch[dev];
  std::call_once(s.once, [&s] { s.err = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch)); });
  if (s.err != hipSuccess) return hip_status(s.err, "dgfs_collide_noalloc: scratch address");
  if (!s.ptr) {
    set_error("dgfs_collide_noalloc: scratch address is NULL");
    return DGFS_EHIP;
  }
  *out = s.ptr;
  return DGFS_OK;
}

}  // namespace dgfs

using namespace dgfs;

extern "C" dgfs_status dgfs_collide_noalloc(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                            const double *fq, int64_t node_stride, double *Q, int64_t out_stride,
                                            uint32_t flags, void *stream) {
  // DGFS_CHECK allocates a counter and synchronises, so it is not accepted here
  dgfs_status s = collide_validate(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, flags,
                                   DGFS_ACCUMULATE | DGFS_PROJECT, "dgfs_collide_noalloc");
  if (s != DGFS_OK || n_nodes == 0) return s;
  const int nz = (p == q && fp == fq) ? 1 : 2;
  const int B = collide_chunk_fitting(pl, n_nodes, nz, kScratchBytes);
  if (B < 1) {
    set_error("dgfs_collide_noalloc: one node needs %zu bytes of scratch; the limit is %zu",
              collide_bytes(pl, 1, nz), kScratchBytes);
    return DGFS_EUNSUPPORTED;
  }
  void *ws = nullptr;
  if ((s = scratch_address(&ws)) != DGFS_OK) return s;
  return collide_impl(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, flags, ws, kScratchBytes,
                      static_cast<hipStream_t>(stream), B, "dgfs_collide_noalloc");
}
