// hp_host.h -- host-side helpers shared by the entry points of libhullprep:
// error reporting, device facts, strategy and tuning choices.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "hullprep.h"

namespace hp {

// Record a synchronous error for hp_last_error() and return `code`.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

struct DeviceInfo {
  int device;
  int cus;              // compute units
  int lds_bytes;        // LDS per workgroup
  int64_t lds_max_p;    // largest p whose (lo, hi) pairs fit in LDS
  int max_threads_cu;   // resident threads per CU
  int lds_groups_per_cu(int32_t p) const {
    const int64_t by_lds = (int64_t)lds_bytes / std::max<int64_t>(1, 8 * (int64_t)p);
    const int64_t by_threads = max_threads_cu / 1024;
    return (int)std::max<int64_t>(1, std::min(by_lds, by_threads));
  }
};

// Facts of the current device (queried once per device).
const DeviceInfo &device_info();

// HP_STRATEGY_* forced by hp_set_strategy / HP_FORCE_STRATEGY, else AUTO.
int forced_strategy();

// The strategy the tuning table picks for (n, p).
int tuned_strategy(int64_t n, int32_t p);

// Launch-shape overrides from the tuning table or hp_tune_set (leaves the
// arguments unchanged when nothing applies).
void tune_override(int64_t n, int32_t p, int *block, int *vpt, int *G);

// Reduce-kernel timing hook: when enabled (and not full) hands out the next
// pair of events, which the launch passes to hipExtLaunchKernelGGL so that
// they carry the dispatch's own start and end timestamps.
bool timing_slot(hipEvent_t *e0, hipEvent_t *e1);

// Single-cloud sequence (defined in hp_single.hip).
int run_single(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi, uint64_t *mask,
               int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx, int32_t *hy,
               int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes, hipStream_t s,
               bool do_hull, int32_t ox = 0, int32_t oy = 0, int32_t q = 0);
size_t single_ws_bytes(int64_t n, int32_t p);

// Hull-tree shape over `positions` slots (slabs of 64, fan-in 64).
struct TreeShape;
void tree_shape(int64_t positions, TreeShape *out);

// Batched launch steps (defined in hp_single.hip).
struct BatchItem;
struct BCloud;
hipError_t launch_b_fill(int B, const BCloud *cl, const uint8_t *needs_fill, int32_t *counter,
                         hipStream_t s);
hipError_t prepare_b_reduce();
hipError_t launch_b_reduce(int grid, size_t lds_bytes, const BatchItem *items, int32_t nitems,
                           int32_t *counter, const BCloud *cl, hipStream_t s);
hipError_t launch_b_tiles(int ntiles, const int2 *tiles, const BCloud *cl, hipStream_t s);
hipError_t launch_b_nodes(bool small, int lev, int nwork, const int4 *work, const BCloud *cl,
                          hipStream_t s);
hipError_t launch_b_root(int B, const BCloud *cl, hipStream_t s);
hipError_t launch_b_chain(int nwork, const int2 *work, const BCloud *cl, hipStream_t s);
}  // namespace hp
