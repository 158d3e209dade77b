// Autotuner of the work tables (option autotune = 1).
//
// Three choices shape an LP's passes without touching the method: the row
// weight of the chunk cost model (how many short rows share a multi-row
// chunk, hence the lanes per row and the chunks per pass), the chunks per
// workgroup of the three-launch passes, and whether the LP may run in the
// persistent loop kernel (unless the options asked for three launches).  The
// tuner times each candidate on the device (the
// loop passes of the LP from its start point, after a short warm-up, with
// tolerance 0 so that no pass is skipped) and keeps the fastest.  Results go
// to a cache file, keyed by the device and the LP's shape class (precision,
// method, memory, the loop kernel asked for, gram_mode, the binary logarithms of m, n,
// the entry count and the longest row and column), so LPs of the same class
// take the cached choice
// without timing.  The choice is part of the LP, so its reduction order, and
// therefore its iterates, are the same alone and in any batch that runs the
// same loop kernel (a member tuned to three launches takes its batch there).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <filesystem>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "runtime.h"

namespace aapdhg {

namespace {

std::mutex g_tune_mu;
constexpr int TUNE_PASSES = 32;
constexpr int TUNE_WARMUP = 4;

std::string cache_path() {
  if (const char* p = std::getenv("AAPDHG_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : ".") + "/.cache/aapdhg/tune.txt";
}

int lg(double v) { return v <= 1.0 ? 0 : (int)std::lround(std::log2(v)); }

struct Choice {
  int w = 4, cpb = 0, lk = 0;
  double ms = 0.0;
};

// The last line of the cache with this key wins.
bool lookup(const std::string& key, Choice* c) {
  std::ifstream f(cache_path());
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    Choice ch;
    if (is >> k >> ch.w >> ch.cpb >> ch.lk >> ch.ms && k == key) {
      *c = ch;
      found = true;
    }
  }
  return found && c->w >= 1 && c->w <= 64 && c->cpb >= 0 && c->cpb <= 4096 && (c->lk == 0 || c->lk == 1);
}

void store(const std::string& key, const Choice& c) {
  const std::string path = cache_path();
  std::error_code ec;
  const auto dir = std::filesystem::path(path).parent_path();
  if (!dir.empty()) std::filesystem::create_directories(dir, ec);
  std::ofstream f(path, std::ios::app);
  if (f) f << key << ' ' << c.w << ' ' << c.cpb << ' ' << c.lk << ' ' << c.ms << '\n';
  // a cache that cannot be written costs a new tuning next time, nothing else
}

}  // namespace

std::string Problem::tune_key() const {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "device");
  hipDeviceProp_t prop{};
  hip_check(hipGetDeviceProperties(&prop, dev), "device properties");
  int maxr = 0, maxc = 0;
  for (size_t i = 0; i + 1 < dev_ptrB.size(); ++i) maxr = std::max(maxr, dev_ptrB[i + 1] - dev_ptrB[i]);
  for (size_t j = 0; j + 1 < dev_ptrA.size(); ++j) maxc = std::max(maxc, dev_ptrA[j + 1] - dev_ptrA[j]);
  const bool ext = opt.pw_period > 0 || opt.variant == AAPDHG_VARIANT_RPDHG;
  // the processor name without its feature suffixes (gfx950:sramecc+:xnack- -> gfx950)
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s:%d:%s:v%d:M%d:e%d:k%d:g%d:m%d:n%d:z%d:r%d:c%d", arch.c_str(),
                prop.multiProcessorCount, fp64 ? "f64" : "f32", opt.variant, opt.memory, ext ? 1 : 0,
                opt.loop_kernel, opt.gram_mode, lg(m), lg(n), lg(nnz), lg(maxr), lg(maxc));
  for (char* p = buf; *p; ++p)
    if (*p == ' ') *p = '_';
  return buf;
}

// Milliseconds per loop pass of the current tables, from the start point.
double Problem::time_candidate() {
  enqueue_reset(nullptr);
  enqueue_init(nullptr);
  solo->enqueue_passes(nullptr, TUNE_WARMUP);
  hip_check(hipDeviceSynchronize(), "tuning warm-up");
  double ms4[4] = {0.0, 0.0, 0.0, 0.0};
  solo->timed_passes(nullptr, TUNE_PASSES, ms4);
  return ms4[0] == 1.0 ? ms4[1] / TUNE_PASSES : ms4[1] + ms4[2] + ms4[3];
}

void Problem::autotune() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string key = tune_key();
  Choice best;
  if (!lookup(key, &best)) {
    // no pass may stop early while candidates are timed
    const double tol = desc.tol;
    const long long max_iter = desc.max_iter;
    desc.tol = 0.0;
    desc.max_iter = (long long)1 << 60;
    bool have = false;
    // loop_kernel = 1 asked for three launches: only the tables are tuned
    const int lk0 = opt.loop_kernel;
    for (int lkc = lk0; lkc <= 1; ++lkc) {
      for (int w : {2, 4, 8}) {
        for (int cpb : {0, 2}) {
          row_weight = w;
          opt.loop_kernel = lkc;
          opt.chunks_per_block = cpb;
          rebuild_tables();
          // the persistent kernel takes one chunk per workgroup, and a set that
          // does not fit it runs the three launches of loop_kernel = 1
          if (solo->t.persistent ? cpb != 0 : lkc == 0) continue;
          const double ms = time_candidate();
          if (!have || ms < best.ms) {
            best = Choice{w, cpb, lkc, ms};
            have = true;
          }
        }
      }
    }
    desc.tol = tol;
    desc.max_iter = max_iter;
    store(key, best);
  }
  row_weight = best.w;
  opt.chunks_per_block = best.cpb;
  opt.loop_kernel = best.lk;
  rebuild_tables();
  // the next solve or iterate starts from u^0
  started = false;
  pending_init = false;
}

}  // namespace aapdhg
