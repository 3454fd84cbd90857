// Device side of the heterogeneous batched launch: item descriptors, the
// per-stage kernels (a block finds its item by binary search and runs the
// N-specialised body of the single-plan kernels) and the launch of one N
// class.  The classes are instantiated in separate translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "launch.hpp"
#include "pipeline.hpp"
#include "vss_kernels.hpp"

namespace dgfs {

struct SubItem {
  PipeArgs a;
  FwdArgs fw;
  FinalArgs fa;
  int N, vss;
};

enum { kFwd = 0, kShift, kGainYZ, kGainX, kFinal, kStages };

template <int N> constexpr int g_small() { return 64 / N > 0 ? 64 / N : 1; }    // fwd / final groups
template <int N> constexpr int g_gain() { return 128 / (2 * N) > 0 ? 128 / (2 * N) : 1; }
template <int N> constexpr int te_vss() { return N >= 48 ? 1 : 2; }

// N classes: every supported N up to NC
template <int NC, typename F>
__device__ __forceinline__ void dispatch_N(int N, F &&f) {
  switch (N) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 14: f(std::integral_constant<int, 14>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 18: if constexpr (NC >= 32) f(std::integral_constant<int, 18>{}); break;
    case 24: if constexpr (NC >= 32) f(std::integral_constant<int, 24>{}); break;
    case 32: if constexpr (NC >= 32) f(std::integral_constant<int, 32>{}); break;
    case 36: if constexpr (NC >= 48) f(std::integral_constant<int, 36>{}); break;
    case 40: if constexpr (NC >= 48) f(std::integral_constant<int, 40>{}); break;
    case 48: if constexpr (NC >= 48) f(std::integral_constant<int, 48>{}); break;
    case 56: if constexpr (NC >= 56) f(std::integral_constant<int, 56>{}); break;
    default: break;
  }
}

__device__ __forceinline__ int find_item(const int *start, int n, int b) {
  int lo = 0, hi = n - 1;  // largest i with start[i] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int NC>
__global__ void __launch_bounds__(64) kb_fwd(const SubItem *items, const int *start, int n) {
  extern __shared__ __align__(16) char smem[];
  const int it = find_item(start, n, blockIdx.x), local = blockIdx.x - start[it];
  const SubItem &si = items[it];
  dispatch_N<NC>(si.N, [&](auto nn) {
    constexpr int NN = decltype(nn)::value;
    fwd_yz_body<T, NN, g_small<NN>()>(si.fw, local, threadIdx.x, reinterpret_cast<C<T>(*)[NN][NN + 1]>(smem));
  });
}

template <typename T, int NC>
__global__ void __launch_bounds__(64) kb_shift(const SubItem *items, const int *start, int n) {
  const int it = find_item(start, n, blockIdx.x), local = blockIdx.x - start[it];
  const SubItem &si = items[it];
  dispatch_N<NC>(si.N, [&](auto nn) {
    constexpr int NN = decltype(nn)::value;
    if (si.a.pack && !si.vss) {
      const int pb = (NN * (NN / 2) + 31) / 32;  // x-lines with k_z < N/2 (real-packed gain)
      shift_x_body<T, NN, true>(si.a, local % pb, (local / pb) % 2, local / (2 * pb), threadIdx.x);
    } else {
      const int pb = (NN * NN + 31) / 32;
      shift_x_body<T, NN>(si.a, local % pb, (local / pb) % 2, local / (2 * pb), threadIdx.x);
    }
  });
}

template <typename T, int NC>
__global__ void __launch_bounds__(128) kb_gain_yz(const SubItem *items, const int *start, int n) {
  extern __shared__ __align__(16) char smem[];
  const int it = find_item(start, n, blockIdx.x), local = blockIdx.x - start[it];
  const SubItem &si = items[it];
  dispatch_N<NC>(si.N, [&](auto nn) {
    constexpr int NN = decltype(nn)::value;
    auto *lds = reinterpret_cast<C<T>(*)[NN][NN + 1]>(smem);
    // the phase rows follow the planes of the non-VSS body
    auto *phs = reinterpret_cast<C<T> *>(smem + (size_t)g_gain<NN>() * gain_bufs<T>() * NN * (NN + 1) * sizeof(C<T>));
    const int jx = local % NN, r = (local / NN) % si.a.Nr, e = local / (NN * si.a.Nr);
    if (si.vss) {
      gain_yz_vss_body<T, NN, g_gain<NN>()>(si.a, jx, r, e, threadIdx.x, lds, phs);
    } else if constexpr (gain_halves<T, NN>()) {
      // two x-planes per block, one per wavefront (blocks_of counts N / 2)
      const int w = threadIdx.x >> 6, jx2 = 2 * (local % (NN / 2)) + w;
      const int r2 = (local / (NN / 2)) % si.a.Nr, e2 = local / ((NN / 2) * si.a.Nr);
      if (si.a.pack)
        gain_yz_halves_packed_body<T, NN>(si.a, jx2, r2, e2, threadIdx.x & 63, lds + gain_bufs<T>() * w);
      else
        gain_yz_halves_body<T, NN>(si.a, jx2, r2, e2, threadIdx.x & 63, lds + gain_bufs<T>() * w, phs + w * 4 * NN);
    } else if (si.a.pack) {
      gain_yz_body<T, NN, packed_gain_groups<NN>(), 1, true>(si.a, jx, r, e, threadIdx.x, lds, phs);
    } else {
      gain_yz_body<T, NN, literal_gain_groups<T, NN>()>(si.a, jx, r, e, threadIdx.x, lds, phs);
    }
  });
}

template <typename T, int NC>
__global__ void __launch_bounds__(64) kb_gain_x(const SubItem *items, const int *start, int n) {
  const int it = find_item(start, n, blockIdx.x), local = blockIdx.x - start[it];
  const SubItem &si = items[it];
  dispatch_N<NC>(si.N, [&](auto nn) {
    constexpr int NN = decltype(nn)::value;
    const int pb = (NN * NN + 31) / 32;
    if (si.vss) gain_x_vss_body<T, NN, te_vss<NN>()>(si.a, local % pb, local / pb, threadIdx.x);
    // the single-plan FP32 kernel's body (its mirrored-slot pass is idle for
    // a one-pair item), so that both compile to the same arithmetic
    else gain_x_body<T, NN, sizeof(T) == 4>(si.a, local % pb, local / pb, threadIdx.x);
  });
}

template <typename T, int NC>
__global__ void __launch_bounds__(128) kb_final(const SubItem *items, const int *start, int n) {
  extern __shared__ __align__(16) char smem[];
  const int it = find_item(start, n, blockIdx.x), local = blockIdx.x - start[it];
  const SubItem &si = items[it];
  dispatch_N<NC>(si.N, [&](auto nn) {
    constexpr int NN = decltype(nn)::value;
    final_yz_body<T, NN, final_groups<NN>()>(si.a, si.fa, local, threadIdx.x,
                                              reinterpret_cast<C<T>(*)[NN][NN + 1]>(smem));
  });
}

// ---------------------------------------------------------------- host side
static int blocks_of(int stage, const SubItem &s) {
  const int N = s.N, pb = (N * N + 31) / 32, E = s.a.n_nodes;
  const int gs = 64 / N > 0 ? 64 / N : 1, te = N >= 48 ? 1 : 2;
  switch (stage) {
    case kFwd: return (N * s.fw.n_nodes * s.fw.nz + gs - 1) / gs;
    case kShift: return (s.a.pack && !s.vss ? (N * (N / 2) + 31) / 32 : pb) * 2 * E;
    case kGainYZ: {
      // the N = 32 bodies (literal and real-packed) take two x-planes per block
      const bool halves = N == 32 && !s.vss;
      return (halves ? N / 2 : N) * s.a.Nr * E;
    }
    case kGainX: return s.vss ? pb * ((E + te - 1) / te) : pb * E;
    default: {
      const int gf = 128 / (2 * N) > 0 ? 128 / (2 * N) : 1;  // final_groups<N>()
      return (N * E + gf - 1) / gf;
    }
  }
}

static size_t lds_bytes(int stage, int nmax, size_t elt) {
  size_t best = 0;
  for (int N : {4, 6, 8, 10, 12, 14, 16, 18, 24, 32, 36, 40, 48, 56}) {
    if (N > nmax) continue;
    const int gs = 64 / N > 0 ? 64 / N : 1, gg = 128 / (2 * N) > 0 ? 128 / (2 * N) : 1;
    const size_t plane = (size_t)N * (N + 1) * 2 * elt;
    if (stage == kGainYZ) best = std::max(best, gg * plane * (elt == 4 ? 2 : 1) + (size_t)gg * 4 * N * 2 * elt);
    else if (stage == kFwd) best = std::max(best, gs * plane);
    else if (stage == kFinal) best = std::max(best, (size_t)(128 / (2 * N) > 0 ? 128 / (2 * N) : 1) * plane);
  }
  return best;
}

template <typename T, int NC>
hipError_t launch_batch(const SubItem *d_items, const int *d_start, const int *h_total, int n, size_t elt,
                               hipStream_t st) {
  if (h_total[kFwd]) DGFS_LAUNCH("kb_fwd", (kb_fwd<T, NC>), dim3(h_total[kFwd]), dim3(64), lds_bytes(kFwd, NC, elt), st, d_items, d_start + 0 * (n + 1), n);
  if (h_total[kShift]) DGFS_LAUNCH("kb_shift", (kb_shift<T, NC>), dim3(h_total[kShift]), dim3(64), 0, st, d_items, d_start + 1 * (n + 1), n);
  if (h_total[kGainYZ]) DGFS_LAUNCH("kb_gain_yz", (kb_gain_yz<T, NC>), dim3(h_total[kGainYZ]), dim3(128), lds_bytes(kGainYZ, NC, elt), st, d_items, d_start + 2 * (n + 1), n);
  if (h_total[kGainX]) DGFS_LAUNCH("kb_gain_x", (kb_gain_x<T, NC>), dim3(h_total[kGainX]), dim3(64), 0, st, d_items, d_start + 3 * (n + 1), n);
  if (h_total[kFinal]) DGFS_LAUNCH("kb_final", (kb_final<T, NC>), dim3(h_total[kFinal]), dim3(128), lds_bytes(kFinal, NC, elt), st, d_items, d_start + 4 * (n + 1), n);
  return hipGetLastError();
}

}  // namespace dgfs
