// hp_batch.h -- work tables of one batch of clouds, shared by the recorded
// batched plan and the server: per-cloud workspace slots, the work items of
// the persistent reduce, the finish work lists, and their packing into one
// device image that a fixed launch sequence consumes.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "hp_host.h"
#include "hp_args.h"

namespace hp {

constexpr int32_t kBatchPMax = 65536;    // largest p of a batched cloud

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace slots of one cloud as byte offsets from the cloud's own base;
// `total` is the span of all of them (a multiple of 256).
struct CloudSlots {
  size_t slab_k, slab_s, slab_off, Lm, cand, ccount, total;
};
CloudSlots cloud_slots(int32_t p, const TreeShape &T);

// Output capacities of one cloud: min(n, p) chain columns, twice that many
// hull vertices.
inline int64_t chain_cap_for(int64_t n, int32_t p) { return std::min<int64_t>(n, p); }

// Caller buffers of one cloud.
struct CloudOut {
  int32_t *cx, *clo, *chi;
  int32_t chain_cap;
  int32_t *hx, *hy;
  int32_t hull_cap;
  int32_t *info;
  uint64_t *mask;   // may be null
};

BCloud make_bcloud(int32_t p, const TreeShape &T, char *slots_base, const CloudSlots &S, const CloudOut &o);

// One reduce work item before its points are bound: `offset` counts points
// from the start of the cloud.
struct HostItem {
  int32_t cloud, mode;
  int64_t offset, count;
};

// Host tables of one batch.  Clouds are added in cloud-index order.
struct BatchTables {
  int32_t B = 0;
  int maxlev = 1;
  int32_t pmax_lds = 1;                 // largest p of a cloud reduced in LDS
  std::vector<HostItem> items;
  std::vector<uint8_t> needs_fill;      // per cloud: L starts at the sentinel in device memory
  std::vector<int2> tiles;              // (cloud, tile of 64 slabs)
  std::vector<int2> chain;              // (cloud, slab)
  std::vector<int4> nodes[2][kMaxLevels + 1];  // [p < 2^15][level >= 3] (cloud, node, side, 0)

  void clear();
  void add_cloud(int64_t n, int32_t p, const TreeShape &T, int64_t lds_p_max);
  // Upper bound of the image bytes one cloud adds to a batch.
  static size_t cloud_image_bound(int64_t n, int32_t p, const TreeShape &T);
  static constexpr size_t kImageSlack = 256 * (8 + 2 * (kMaxLevels + 1));  // alignment of every list
  // Longest items first, so the persistent reduce ends evenly.
  void sort_items();
};

// The device image: cloud array, work lists and the reduce counter packed
// into one buffer, plus the launch shapes.
struct DeviceBatch {
  int32_t B = 0;
  BCloud *clouds = nullptr;
  uint8_t *needs_fill = nullptr;
  int32_t *counter = nullptr;
  BatchItem *items = nullptr;
  int32_t nitems = 0;
  int2 *tiles = nullptr;
  int32_t ntiles = 0;
  int2 *chain = nullptr;
  int32_t nchain = 0;
  int4 *nodes[2][kMaxLevels + 1] = {};
  int32_t nnodes[2][kMaxLevels + 1] = {};
  int maxlev = 1;
  size_t lds_bytes = 0;
  int reduce_grid = 1;
};

size_t batch_image_bytes(const BatchTables &t);

// Write the image of `t` for device address `dev` into `host` (both
// batch_image_bytes(t) long).  cloud_pts[b] is cloud b's first point.
void batch_image(const BatchTables &t, const std::vector<BCloud> &clouds,
                 const std::vector<const int32_t *> &cloud_pts, char *host, char *dev, DeviceBatch &D);

// The fixed launch sequence over an image already in device memory: fill,
// persistent reduce, tiles, upper node levels, roots, chain.
hipError_t enqueue_batch(const DeviceBatch &D, hipStream_t s);

}  // namespace hp
