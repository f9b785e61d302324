// hp_common.hip -- status strings, last-error slot, device facts, strategy
// and tuning state of libhullprep.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <dlfcn.h>

#include "hp_host.h"

namespace hp {

static thread_local char g_last_error[512] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

static std::mutex g_mu;
static DeviceInfo g_dev[64];
static bool g_dev_ok[64];

const DeviceInfo &device_info() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) d = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_dev_ok[d]) {
    DeviceInfo D;
    D.device = d;
    int v = 0;
    D.cus = (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) == hipSuccess && v > 0) ? v : 256;
    D.lds_bytes = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d) == hipSuccess && v > 0) ? v : 65536;
    D.max_threads_cu = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxThreadsPerMultiProcessor, d) == hipSuccess && v > 0) ? v : 2048;
    D.lds_max_p = D.lds_bytes / 8 - 2;  // p pairs plus the reduce's flag and grab words
    g_dev[d] = D;
    g_dev_ok[d] = true;
  }
  return g_dev[d];
}

static int g_forced = -1;  // -1: not read yet

int forced_strategy() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_forced < 0) {
    g_forced = HP_STRATEGY_AUTO;
    const char *e = getenv("HP_FORCE_STRATEGY");
    if (e) {
      if (!strcmp(e, "lds")) g_forced = HP_STRATEGY_LDS;
      else if (!strcmp(e, "global")) g_forced = HP_STRATEGY_GLOBAL;
      else if (!strcmp(e, "lds_partial")) g_forced = HP_STRATEGY_LDS_PARTIAL;
      else if (!strcmp(e, "window")) g_forced = HP_STRATEGY_WINDOW;
      else if (!strcmp(e, "sampled")) g_forced = HP_STRATEGY_SAMPLED;
      else if (!strcmp(e, "binned")) g_forced = HP_STRATEGY_BINNED;
      else if (!strcmp(e, "sparse")) g_forced = HP_STRATEGY_SPARSE;
    }
  }
  return g_forced;
}

// ---------------------------------------------------------------------------
// Tuning table.  Keyed by the regime bucket (floor(log2 n), floor(log2 p));
// each entry fixes strategy, block size, vectors per lane and grid size.  It
// is filled by the tuner (paper_1505_00914_amd/tune.py) through
// hp_tune_load, and an explicit hp_tune_set override wins over it.
// ---------------------------------------------------------------------------
struct TuneEntry {
  int ln, lp, strategy, block, vpt, G;
};
static std::vector<TuneEntry> g_table;
static int g_set_strategy = 0, g_set_block = 0, g_set_vpt = 0, g_set_G = 0;

static int ilog2(int64_t v) {
  int l = 0;
  while (v > 1) { v >>= 1; ++l; }
  return l;
}

int tune_load(const char *path);

// The table shipped beside the library (tuning_gfx950.txt in the directory
// of libhullprep.so) is loaded on first use; HP_TUNING_FILE names another
// file, or disables it when empty.  A missing file leaves the defaults.
static void load_default_table() {
  static std::once_flag once;
  std::call_once(once, [] {
    std::string path;
    if (const char *env = getenv("HP_TUNING_FILE")) {
      path = env;
    } else {
      Dl_info di;
      if (dladdr(reinterpret_cast<void *>(&load_default_table), &di) && di.dli_fname) {
        path = di.dli_fname;
        const size_t slash = path.rfind('/');
        path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tuning_gfx950.txt";
      }
    }
    if (path.empty()) return;
    if (FILE *f = fopen(path.c_str(), "r")) {
      fclose(f);
      (void)tune_load(path.c_str());
    }
  });
}

static const TuneEntry *lookup(int64_t n, int32_t p) {
  const int ln = ilog2(n < 1 ? 1 : n), lp = ilog2(p);
  for (const TuneEntry &t : g_table)
    if (t.ln == ln && t.lp == lp) return &t;
  return nullptr;
}

int tuned_strategy(int64_t n, int32_t p) {
  load_default_table();
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_set_strategy) return g_set_strategy;
  if (const TuneEntry *t = lookup(n, p)) return t->strategy;
  // untuned default: a private L per workgroup pays off once every
  // workgroup sees several points per column
  const DeviceInfo *D = nullptr;
  (void)D;
  return ((int64_t)n >= 4 * (int64_t)p) ? HP_STRATEGY_LDS_PARTIAL : HP_STRATEGY_GLOBAL;
}

void tune_override(int64_t n, int32_t p, int *block, int *vpt, int *G) {
  load_default_table();
  std::lock_guard<std::mutex> lk(g_mu);
  if (const TuneEntry *t = lookup(n, p)) {
    if (t->block) *block = t->block;
    if (t->vpt) *vpt = t->vpt;
    if (t->G) *G = t->G;
  }
  if (g_set_block) *block = g_set_block;
  if (g_set_vpt) *vpt = g_set_vpt;
  if (g_set_G) *G = g_set_G;
}

int tune_set(int strategy, int block, int vpt, int G) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_set_strategy = strategy;
  g_set_block = block;
  g_set_vpt = vpt;
  g_set_G = G;
  return HP_OK;
}

int tune_load(const char *path) {
  FILE *f = fopen(path, "r");
  if (!f) return set_error(HP_EINVAL, "cannot open tuning table %s", path);
  std::vector<TuneEntry> tab;
  char line[256];
  int lineno = 0;
  while (fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneEntry t;
    if (sscanf(line, "%d %d %d %d %d %d", &t.ln, &t.lp, &t.strategy, &t.block, &t.vpt, &t.G) != 6) continue;
    // a line the launch code cannot honour fails the whole load, and the
    // table in use stays as it was
    const bool ok = t.ln >= 0 && t.ln < 64 && t.lp >= 0 && t.lp < 32 && t.strategy >= HP_STRATEGY_LDS &&
                    t.strategy <= HP_STRATEGY_BINNED && (t.block == 256 || t.block == 512 || t.block == 1024) &&
                    (t.vpt == 2 || t.vpt == 4 || t.vpt == 8) && t.G >= 0 && t.G <= (1 << 20);
    if (!ok) {
      fclose(f);
      return set_error(HP_EINVAL, "tuning table %s line %d: unsupported entry", path, lineno);
    }
    tab.push_back(t);
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_mu);
  g_table = tab;
  return HP_OK;
}

// ---------------------------------------------------------------------------
// Reduce-kernel timing (events on the launch stream)
// ---------------------------------------------------------------------------
constexpr int kTimingSlots = 4096;
static bool g_timing_on = false;
static bool g_timing_pool = false;
static hipEvent_t g_ev0[kTimingSlots], g_ev1[kTimingSlots];
static int g_timing_used = 0;

bool timing_slot(hipEvent_t *e0, hipEvent_t *e1) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_timing_on || g_timing_used >= kTimingSlots) return false;
  const int slot = g_timing_used++;
  *e0 = g_ev0[slot];
  *e1 = g_ev1[slot];
  return true;
}

int timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (on && !g_timing_pool) {
    // default events: their durations track the kernel-trace durations of
    // the profiler; fence-free events read noisier on this path
    for (int i = 0; i < kTimingSlots; ++i) {
      if (hipEventCreate(&g_ev0[i]) != hipSuccess || hipEventCreate(&g_ev1[i]) != hipSuccess)
        return set_error(HP_EDEVICE, "hipEventCreate failed");
    }
    g_timing_pool = true;
  }
  g_timing_on = on != 0;
  g_timing_used = 0;
  return HP_OK;
}

int timing_read(int32_t *count, double *total, double *mn, double *mx) {
  std::lock_guard<std::mutex> lk(g_mu);
  double t = 0, lo = 0, hi = 0;
  for (int i = 0; i < g_timing_used; ++i) {
    if (hipEventSynchronize(g_ev1[i]) != hipSuccess) return set_error(HP_EDEVICE, "hipEventSynchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_ev0[i], g_ev1[i]) != hipSuccess)
      return set_error(HP_EDEVICE, "hipEventElapsedTime failed");
    t += ms;
    lo = i == 0 ? ms : std::min(lo, (double)ms);
    hi = i == 0 ? ms : std::max(hi, (double)ms);
  }
  if (count) *count = g_timing_used;
  if (total) *total = t;
  if (mn) *mn = lo;
  if (mx) *mx = hi;
  g_timing_used = 0;
  return HP_OK;
}

}  // namespace hp

using namespace hp;

extern "C" int hp_timing_enable(int on) { return timing_enable(on); }

extern "C" int hp_timing_read(int32_t *count, double *total_ms, double *min_ms, double *max_ms) {
  return timing_read(count, total_ms, min_ms, max_ms);
}

extern "C" const char *hp_status_string(int code) {
  switch (code) {
    case HP_OK: return "HP_OK";
    case HP_EINVAL: return "HP_EINVAL: invalid argument";
    case HP_ERANGE: return "HP_ERANGE: a coordinate lies outside [1, p]";
    case HP_ECAPACITY: return "HP_ECAPACITY: output or workspace too small";
    case HP_EDEVICE: return "HP_EDEVICE: HIP call failed";
    case HP_ENOMEM: return "HP_ENOMEM: allocation failed";
    case HP_ETIMEOUT: return "HP_ETIMEOUT: not completed yet";
    default: return "unknown status";
  }
}

extern "C" const char *hp_last_error(void) { return g_last_error; }

extern "C" int hp_abi_version(void) { return HP_ABI_VERSION; }

extern "C" int32_t hp_lds_max_p(void) { return (int32_t)device_info().lds_max_p; }

extern "C" int hp_set_strategy(int strategy) {
  if (strategy < HP_STRATEGY_AUTO || strategy > HP_STRATEGY_SPARSE)
    return set_error(HP_EINVAL, "unknown strategy %d", strategy);
  forced_strategy();
  std::lock_guard<std::mutex> lk(g_mu);
  g_forced = strategy;
  return HP_OK;
}

extern "C" int hp_tune_set(int32_t strategy, int32_t block, int32_t vpt, int32_t grid) {
  if (strategy < 0 || strategy > HP_STRATEGY_BINNED)   // the sparse path has fixed launch shapes
    return set_error(HP_EINVAL, "unknown strategy %d", strategy);
  const bool ok_shape = (block == 0 && vpt == 0) ||
                        ((block == 256 || block == 512 || block == 1024) && (vpt == 2 || vpt == 4 || vpt == 8));
  if (!ok_shape) return set_error(HP_EINVAL, "unsupported block %d / vpt %d", block, vpt);
  if (grid < 0 || grid > 1 << 20) return set_error(HP_EINVAL, "grid %d out of range", grid);
  return tune_set(strategy, block, vpt, grid);
}

extern "C" int hp_tune_load(const char *path) {
  if (!path) return set_error(HP_EINVAL, "path is NULL");
  return tune_load(path);
}
