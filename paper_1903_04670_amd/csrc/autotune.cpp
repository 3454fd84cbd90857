// Launch-schedule autotuner.  Three schedule dimensions, none of which
// changes a result bit: evaluations per launch (the chunk width that sets the
// grid of every pipeline stage and the workspace footprint), the number of
// blocks that split the (r, sigma_x) loop of one x-line set in k_shift_x, and
// whether k_gain_x serves a mirrored pair slot in the same pass.  They are
// searched one after the other (chunk width with the defaults, then the
// split at the best width, then the fusion), each candidate timed with HIP
// events on the caller's inputs; the fastest schedule is stored in the plan
// and appended to an on-disk cache keyed by device and plan shape, which
// later plan creations read.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

namespace dgfs {

size_t collide_bytes(const dgfs_plan_s *pl, int B, int nz);

static std::mutex g_tune_mu;

// evaluations per launch the tuner tries (powers of two in this range)
constexpr int kTuneMin = 8, kTuneMax = 256;

static std::string cache_path() {
  if (const char *p = std::getenv("DGFS_TUNE_CACHE")) return p;
  const char *home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/dgfs_tune.txt";
}

static std::string tune_key(const dgfs_plan_s *pl) {
  hipDeviceProp_t prop{};
  int dev = 0;
  std::string name = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) name = prop.gcnArchName;
  for (char &c : name)
    if (c == ' ' || c == ':') c = '_';
  std::ostringstream k;
  k << name << " N" << pl->N << " M" << pl->M << " R" << pl->Nr << " S" << pl->Sx << " P" << pl->precision << " V"
    << (pl->vhs ? 0 : 1) << " ns" << pl->ns;
  return k.str();
}

void load_tuned(dgfs_plan_s *pl) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::ifstream in(cache_path());
  if (!in) return;
  const std::string key = tune_key(pl);
  std::string line;
  while (std::getline(in, line)) {
    const size_t bar = line.rfind('|');
    if (bar == std::string::npos) continue;
    if (line.substr(0, bar) != key) continue;
    // last entry wins; "width" or "width,split,fuse"; values outside the
    // tuner's candidate ranges are ignored (the schedule then keeps its
    // default in that dimension)
    int v = 0, split = 0, fuse = -1;
    const int got = std::sscanf(line.c_str() + bar + 1, "%d,%d,%d", &v, &split, &fuse);
    if (got < 1) continue;
    pl->chunk_evals = (v >= kTuneMin && v <= kTuneMax) ? v : 0;
    pl->shift_split = (got >= 2 && (split == 1 || split == 2 || split == 4 || split == 8)) ? split : 0;
    pl->gain_x_fuse = (got >= 3 && (fuse == 0 || fuse == 1)) ? fuse : -1;
  }
}

static void store_tuned(const dgfs_plan_s *pl) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string path = cache_path();
  // create the parent directories (ignore failures: the open below reports nothing either)
  for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
    (void)::mkdir(path.substr(0, pos).c_str(), 0755);
  std::ofstream out(path, std::ios::app);
  if (out) out << tune_key(pl) << "|" << pl->chunk_evals << "," << pl->shift_split << "," << pl->gain_x_fuse << "\n";
}

}  // namespace dgfs

using namespace dgfs;

namespace dgfs {
namespace {
struct Timer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};
}  // namespace
}  // namespace dgfs

extern "C" dgfs_status dgfs_autotune(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                     const double *fq, int64_t node_stride, double *Q, int64_t out_stride, void *ws,
                                     size_t ws_bytes, void *stream, int32_t *chosen) {
  if (!pl || n_nodes < 1 || !fp || !fq || !Q || !ws) { set_error("dgfs_autotune: invalid argument"); return DGFS_EINVAL; }
  if (p < 0 || q < 0 || p >= pl->ns || q >= pl->ns) { set_error("dgfs_autotune: species out of range"); return DGFS_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nz = (p == q && fp == fq) ? 1 : 2;
  const int saved[3] = {pl->chunk_evals, pl->shift_split, pl->gain_x_fuse};
  auto restore = [&] {
    pl->chunk_evals = saved[0];
    pl->shift_split = saved[1];
    pl->gain_x_fuse = saved[2];
  };
  Timer tm;
  hipError_t he;
  if ((he = hipEventCreate(&tm.e0)) != hipSuccess || (he = hipEventCreate(&tm.e1)) != hipSuccess)
    return hip_status(he, "dgfs_autotune events");
  // time of the current schedule: one untimed call, then three timed ones
  auto time_it = [&](float &ms) -> dgfs_status {
    dgfs_status s = dgfs_collide(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, 0, ws, ws_bytes, stream);
    if (s != DGFS_OK) return s;
    (void)hipEventRecord(tm.e0, st);
    for (int rep = 0; rep < 3; ++rep)
      (void)dgfs_collide(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, 0, ws, ws_bytes, stream);
    (void)hipEventRecord(tm.e1, st);
    if ((he = hipEventSynchronize(tm.e1)) != hipSuccess) return hip_status(he, "dgfs_autotune");
    ms = 0.0f;
    (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
    return DGFS_OK;
  };
  // 1. chunk width with the default split and fusion
  pl->shift_split = 0;
  pl->gain_x_fuse = -1;
  float best = 0.0f;
  int best_e = 0;
  for (int E = kTuneMin; E <= kTuneMax; E *= 2) {
    if (E > 2 * n_nodes && E > 8) break;
    if (collide_bytes(pl, (int)std::min<int64_t>(E, n_nodes), nz) > ws_bytes) continue;
    pl->chunk_evals = E;
    float ms;
    dgfs_status s = time_it(ms);
    if (s != DGFS_OK) { restore(); return s; }
    if (best_e == 0 || ms < best) {
      best = ms;
      best_e = E;
    }
  }
  if (best_e == 0) {
    restore();
    set_error("dgfs_autotune: the workspace fits no candidate schedule");
    return DGFS_EWORKSPACE;
  }
  pl->chunk_evals = best_e;
  // 2. x-shift split at that width
  int best_split = 0;
  for (int split : {1, 2, 4, 8}) {
    pl->shift_split = split;
    float ms;
    dgfs_status s = time_it(ms);
    if (s != DGFS_OK) { restore(); return s; }
    if (ms < best) {
      best = ms;
      best_split = split;
    }
  }
  pl->shift_split = best_split;
  // 3. fused k_gain_x pass for mirrored slots
  int best_fuse = -1;
  for (int fuse : {0, 1}) {
    pl->gain_x_fuse = fuse;
    float ms;
    dgfs_status s = time_it(ms);
    if (s != DGFS_OK) { restore(); return s; }
    if (ms < best) {
      best = ms;
      best_fuse = fuse;
    }
  }
  pl->gain_x_fuse = best_fuse;
  store_tuned(pl);
  if (chosen) {
    chosen[0] = pl->chunk_evals;
    chosen[1] = pl->shift_split;
    chosen[2] = pl->gain_x_fuse;
  }
  return DGFS_OK;
}
