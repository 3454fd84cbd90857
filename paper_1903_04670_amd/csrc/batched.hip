// Heterogeneous batch: items of different plans (N, species, quadratures)
// run through the five pipeline stages with ONE launch per stage per
// workspace chunk.  Every block finds its item by binary search over the
// stage's block offsets and runs the item's N-specialised stage body, the
// same device code the single-plan kernels use, so results are identical
// bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "batched_kernels.hpp"

namespace dgfs {

// the N <= 56 class is instantiated in batched_n56.hip
extern template hipError_t launch_batch<double, 56>(const SubItem *, const int *, const int *, int, size_t, hipStream_t);
extern template hipError_t launch_batch<float, 56>(const SubItem *, const int *, const int *, int, size_t, hipStream_t);

struct SubRef {
  int item;
  int64_t n0;
  int nb;
  size_t bytes;
};

static size_t a256(size_t b) { return (b + 255) / 256 * 256; }

static dgfs_status plan_batch(const dgfs_plan *plans, int32_t n_plans, const dgfs_item *items, int64_t n_items,
                              std::vector<SubRef> &subs, std::vector<size_t> &chunk_end, size_t &ws_need) {
  subs.clear();
  chunk_end.clear();
  ws_need = 0;
  if (!plans || n_plans < 1 || (n_items > 0 && !items)) { set_error("dgfs_collide_batched: NULL plans or items"); return DGFS_EINVAL; }
  for (int i = 0; i < n_plans; ++i)
    if (!plans[i]) { set_error("dgfs_collide_batched: plan %d is NULL", i); return DGFS_EINVAL; }
  for (int i = 1; i < n_plans; ++i)
    if (plans[i]->precision != plans[0]->precision) { set_error("dgfs_collide_batched: plans differ in precision"); return DGFS_EINVAL; }
  for (int64_t i = 0; i < n_items; ++i) {
    const dgfs_item &it = items[i];
    if (it.plan < 0 || it.plan >= n_plans) { set_error("item %lld: plan index out of range", (long long)i); return DGFS_EINVAL; }
    const dgfs_plan_s *pl = plans[it.plan];
    if (it.p < 0 || it.q < 0 || it.p >= pl->ns || it.q >= pl->ns) { set_error("item %lld: species out of range", (long long)i); return DGFS_EINVAL; }
    if (it.n_nodes < 0) { set_error("item %lld: n_nodes < 0", (long long)i); return DGFS_EINVAL; }
    if (it.n_nodes == 0) continue;
    if (!it.fp || !it.fq || !it.Q) { set_error("item %lld: NULL array", (long long)i); return DGFS_EINVAL; }
    const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
    if (it.n_nodes > 1 && (it.node_stride < n3 || it.out_stride < n3)) { set_error("item %lld: strides must be >= N^3", (long long)i); return DGFS_EINVAL; }
    const int B = chunk_nodes(pl, it.n_nodes, 1);
    const int nz = (it.p == it.q && it.fp == it.fq) ? 1 : 2;
    for (int64_t n0 = 0; n0 < it.n_nodes; n0 += B) {
      const int nb = (int)std::min<int64_t>(B, it.n_nodes - n0);
      subs.push_back(SubRef{(int)i, n0, nb, pipeline_bytes(pl, nb, 1, nz)});
    }
  }
  // pack sub-items into chunks of at most 8 GiB of intermediates (or one sub-item)
  const size_t budget = (size_t)8 << 30;
  size_t cur = 0, worst = 0, max_count = 0, count = 0;
  for (size_t k = 0; k < subs.size(); ++k) {
    if (count > 0 && cur + subs[k].bytes > budget) {
      chunk_end.push_back(k);
      worst = std::max(worst, cur);
      max_count = std::max(max_count, count);
      cur = 0;
      count = 0;
    }
    cur += subs[k].bytes;
    ++count;
  }
  if (count > 0) {
    chunk_end.push_back(subs.size());
    worst = std::max(worst, cur);
    max_count = std::max(max_count, count);
  }
  ws_need = a256(max_count * sizeof(SubItem)) + a256(kStages * (max_count + 1) * sizeof(int)) + worst;
  if (ws_need == 0) ws_need = 256;
  return DGFS_OK;
}

// pinned staging for the descriptor tables (process-wide, reused after the
// previous call's copies have completed)
static std::mutex g_stage_mu;
static void *g_stage = nullptr;
static size_t g_stage_bytes = 0;
static hipEvent_t g_stage_done = nullptr;


}  // namespace dgfs

using namespace dgfs;

extern "C" size_t dgfs_batched_workspace_bytes(const dgfs_plan *plans, int32_t n_plans, const dgfs_item *items,
                                               int64_t n_items) {
  std::vector<SubRef> subs;
  std::vector<size_t> ends;
  size_t need = 0;
  if (plan_batch(plans, n_plans, items, n_items, subs, ends, need) != DGFS_OK) return 0;
  return need;
}

extern "C" dgfs_status dgfs_collide_batched(const dgfs_plan *plans, int32_t n_plans, const dgfs_item *items,
                                            int64_t n_items, uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (flags & ~DGFS_ACCUMULATE) { set_error("dgfs_collide_batched: unsupported flags 0x%x", flags); return DGFS_EINVAL; }
  std::vector<SubRef> subs;
  std::vector<size_t> ends;
  size_t need = 0;
  dgfs_status s = plan_batch(plans, n_plans, items, n_items, subs, ends, need);
  if (s != DGFS_OK) return s;
  if (subs.empty()) return DGFS_OK;
  if (!ws || ws_bytes < need) { set_error("dgfs_collide_batched: workspace %zu bytes, need %zu", ws_bytes, need); return DGFS_EWORKSPACE; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t elt = plans[0]->elt();
  int nmax = 0;
  for (const SubRef &r : subs) nmax = std::max(nmax, plans[items[r.item].plan]->N);
  // host descriptor tables of every chunk, staged in one pinned buffer
  size_t max_count = 0;
  {
    size_t b = 0;
    for (size_t e : ends) { max_count = std::max(max_count, e - b); b = e; }
  }
  const size_t desc_bytes = a256(max_count * sizeof(SubItem)) + a256(kStages * (max_count + 1) * sizeof(int));
  const size_t stage_need = desc_bytes * ends.size();
  std::lock_guard<std::mutex> lk(g_stage_mu);
  hipError_t e = hipSuccess;
  if (g_stage_done && (e = hipEventSynchronize(g_stage_done)) != hipSuccess) return hip_status(e, "batched staging");
  if (g_stage_bytes < stage_need) {
    if (g_stage) (void)hipHostFree(g_stage);
    g_stage = nullptr;
    g_stage_bytes = 0;
    if ((e = hipHostMalloc(&g_stage, stage_need, hipHostMallocDefault)) != hipSuccess) return hip_status(e, "batched staging");
    g_stage_bytes = stage_need;
  }
  if (!g_stage_done && (e = hipEventCreateWithFlags(&g_stage_done, hipEventDisableTiming)) != hipSuccess)
    return hip_status(e, "batched staging");
  char *wsb = static_cast<char *>(ws);
  // enqueue every chunk; the staging event is recorded whatever the outcome,
  // so the next call never rewrites descriptors a pending copy still reads
  auto enqueue = [&]() -> dgfs_status {
    hipError_t e = hipSuccess;
    size_t begin = 0;
    for (size_t c = 0; c < ends.size(); ++c) {
      const size_t end = ends[c], n = end - begin;
      char *host = static_cast<char *>(g_stage) + c * desc_bytes;
      SubItem *hi = reinterpret_cast<SubItem *>(host);
      int *hs = reinterpret_cast<int *>(host + a256(max_count * sizeof(SubItem)));
      char *region = wsb + desc_bytes;
      int total[kStages] = {0, 0, 0, 0, 0};
      for (size_t k = 0; k < n; ++k) {
        const SubRef &r = subs[begin + k];
        const dgfs_item &it = items[r.item];
        const dgfs_plan_s *pl = plans[it.plan];
        const int nz = (it.p == it.q && it.fp == it.fq) ? 1 : 2;
        SubItem si{};
        pipeline_common(pl, si.a);
        pipeline_carve(pl, r.nb, 1, nz, region, si.a);
        region += r.bytes;
        si.a.n_nodes = r.nb;
        si.a.n_pairs = 1;
        si.a.nz = nz;
        si.a.pair_id[0] = it.p * pl->ns + it.q;
        si.a.zp[0] = 0;
        si.a.zq[0] = nz == 1 ? 0 : 1;
        si.a.xshare[0] = nz == 1 ? 1 : 0;
        pipeline_slots(pl, si.a);
        si.fw.src[0] = it.fp + r.n0 * it.node_stride;
        si.fw.src[1] = it.fq + r.n0 * it.node_stride;
        si.fw.node_stride = it.node_stride;
        si.fw.n_nodes = r.nb;
        si.fw.nz = nz;
        si.fw.Z = si.a.Z;
        si.fa.n_out = 1;
        si.fa.qcount = 1;
        si.fa.fsrc[0] = it.fp + r.n0 * it.node_stride;
        si.fa.f_stride = it.node_stride;
        si.fa.out[0] = it.Q + r.n0 * it.out_stride;
        si.fa.out_stride = it.out_stride;
        si.fa.accumulate = (flags & DGFS_ACCUMULATE) ? 1 : 0;
        si.N = pl->N;
        si.vss = pl->vhs ? 0 : 1;
        hi[k] = si;
        for (int sg = 0; sg < kStages; ++sg) {
          hs[sg * (n + 1) + k] = total[sg];
          total[sg] += blocks_of(sg, si);
        }
      }
      for (int sg = 0; sg < kStages; ++sg) hs[sg * (n + 1) + n] = total[sg];
      // descriptors to the head of the workspace, then the five stage launches
      SubItem *d_items = reinterpret_cast<SubItem *>(wsb);
      int *d_start = reinterpret_cast<int *>(wsb + a256(max_count * sizeof(SubItem)));
      if ((e = hipMemcpyAsync(d_items, hi, n * sizeof(SubItem), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_status(e, "batched descriptors");
      if ((e = hipMemcpyAsync(d_start, hs, kStages * (n + 1) * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_status(e, "batched descriptors");
      // the start arrays were laid out with stride (n + 1) per stage
      const bool f64 = plans[0]->precision == DGFS_FP64;
      if (nmax <= 16) e = f64 ? launch_batch<double, 16>(d_items, d_start, total, (int)n, elt, st)
                              : launch_batch<float, 16>(d_items, d_start, total, (int)n, elt, st);
      else if (nmax <= 32) e = f64 ? launch_batch<double, 32>(d_items, d_start, total, (int)n, elt, st)
                                   : launch_batch<float, 32>(d_items, d_start, total, (int)n, elt, st);
      else if (nmax <= 48) e = f64 ? launch_batch<double, 48>(d_items, d_start, total, (int)n, elt, st)
                                   : launch_batch<float, 48>(d_items, d_start, total, (int)n, elt, st);
      else e = f64 ? launch_batch<double, 56>(d_items, d_start, total, (int)n, elt, st)
                   : launch_batch<float, 56>(d_items, d_start, total, (int)n, elt, st);
      if (e != hipSuccess) return hip_status(e, "dgfs_collide_batched launch");
      begin = end;
    }
    return DGFS_OK;
  };
  const dgfs_status st_enq = enqueue();
  if ((e = hipEventRecord(g_stage_done, st)) != hipSuccess && st_enq == DGFS_OK) return hip_status(e, "batched staging");
  return st_enq;
}
