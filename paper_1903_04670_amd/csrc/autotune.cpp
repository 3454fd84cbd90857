// Launch-schedule autotuner: evaluations per launch (the chunk width that sets
// the grid of every pipeline stage and the workspace footprint).  Candidates
// are timed with HIP events on the caller's inputs; the fastest is stored in
// the plan and appended to an on-disk cache keyed by device and plan shape,
// which later plan creations read.
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

size_t pipeline_bytes(const dgfs_plan_s *pl, int B, int n_pairs, int nz);

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
    // last entry wins; a value outside the tuner's candidate range is ignored
    const int v = std::atoi(line.c_str() + bar + 1);
    if (v >= kTuneMin && v <= kTuneMax) pl->chunk_evals = v;
  }
}

static void store_tuned(const dgfs_plan_s *pl) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string path = cache_path();
  // create the parent directories (ignore failures: the open below reports nothing either)
  for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
    (void)::mkdir(path.substr(0, pos).c_str(), 0755);
  std::ofstream out(path, std::ios::app);
  if (out) out << tune_key(pl) << "|" << pl->chunk_evals << "\n";
}

}  // namespace dgfs

using namespace dgfs;

extern "C" dgfs_status dgfs_autotune(dgfs_plan pl, int64_t n_nodes, int32_t p, int32_t q, const double *fp,
                                     const double *fq, int64_t node_stride, double *Q, int64_t out_stride, void *ws,
                                     size_t ws_bytes, void *stream, int32_t *chosen) {
  if (!pl || n_nodes < 1 || !fp || !fq || !Q || !ws) { set_error("dgfs_autotune: invalid argument"); return DGFS_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nz = (p == q && fp == fq) ? 1 : 2;
  const int saved = pl->chunk_evals;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he;
  if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_status(he, "dgfs_autotune events");
  }
  float best = 0.0f;
  int best_e = 0;
  for (int E = kTuneMin; E <= kTuneMax; E *= 2) {
    if (E > 2 * n_nodes && E > 8) break;
    if (pipeline_bytes(pl, (int)std::min<int64_t>(E, n_nodes), 1, nz) > ws_bytes) continue;
    pl->chunk_evals = E;
    dgfs_status s = dgfs_collide(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, 0, ws, ws_bytes, stream);
    if (s != DGFS_OK) {
      pl->chunk_evals = saved;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return s;
    }
    (void)hipEventRecord(e0, st);
    for (int rep = 0; rep < 3; ++rep)
      (void)dgfs_collide(pl, n_nodes, p, q, fp, fq, node_stride, Q, out_stride, 0, ws, ws_bytes, stream);
    (void)hipEventRecord(e1, st);
    if ((he = hipEventSynchronize(e1)) != hipSuccess) {
      pl->chunk_evals = saved;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return hip_status(he, "dgfs_autotune");
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best_e == 0 || ms < best) {
      best = ms;
      best_e = E;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_e == 0) {
    pl->chunk_evals = saved;
    set_error("dgfs_autotune: the workspace fits no candidate schedule");
    return DGFS_EWORKSPACE;
  }
  pl->chunk_evals = best_e;
  store_tuned(pl);
  if (chosen) *chosen = best_e;
  return DGFS_OK;
}
