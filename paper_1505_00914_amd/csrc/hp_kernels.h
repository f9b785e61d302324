// hp_kernels.h -- kernels of the single-cloud path of libhullprep, also used
// cloud-by-cloud by the batched baseline.  See hullprep.h for the contract.
//
// Launch sequence of one cloud (all on the caller's stream):
//   k_init      control words, tree counters, info; the global L when the
//               global strategy is used                     (L initialisation)
//   k_reduce_*  Algorithm 1 over the points                 (Algorithm 1)
//   k_finish    per slab of 64 columns: merge of the partial L arrays, the M
//               word, slab counts, hull levels 0-1; the last slab to finish
//               scans the slab counts; the last child of every hull-tree
//               node merges its children, the root writes the hull
//   k_chain     per slab: the compacted chain at the scanned offsets (Lemma 1)
#pragma once

#include "hp_device.h"

namespace hp {

// Result of Algorithm 1 for one point, into an (lo, hi) pair array that may
// live in LDS or in device memory.  The pair is read first and the atomics
// are issued only when the point improves it: lo only ever falls and hi only
// ever rises, so a stale read can only cause an unnecessary atomic, never a
// missed one.
// With a column window (wc > 0) L holds columns c0 .. c0 + wc - 1 only and
// points of other columns are skipped (after their range check).
__device__ __forceinline__ void fold_point_lds(int2 *L, int p, int x, int y, bool &bad, unsigned c0 = 0,
                                               unsigned wc = 0) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  bool ok = (xi < (unsigned)p) & (yi < (unsigned)p);
  bad |= !ok;
  const unsigned xr = xi - c0;
  if (wc) ok = ok & (xr < wc);
  const unsigned c = ok ? xr : 0u;
  const int2 cur = L[c];
  if (ok && y < cur.x) atomicMin(&L[c].x, y);
  if (ok && y > cur.y) atomicMax(&L[c].y, y);
}

// A partial L entry in 32 bits: lo - 1 in the low half, hi + 1 in the high
// half (the sentinel (p+1, -1) becomes (p, 0)); valid for p < 65535.
__host__ __device__ __forceinline__ bool partial_packs(int64_t p) { return p < 65535; }
__device__ __forceinline__ uint32_t pack_partial(int2 L) {
  return (uint32_t)(L.x - 1) | ((uint32_t)(L.y + 1) << 16);
}
__device__ __forceinline__ int2 unpack_partial(uint32_t w) {
  return make_int2((int)(w & 0xFFFFu) + 1, (int)(w >> 16) - 1);
}

// A coherent 8-byte read of an (lo, hi) pair that other workgroups update
// with device-scope atomics (a plain load could keep hitting a stale cache
// line, which would defeat the filter without breaking correctness).
__device__ __forceinline__ int2 load_coherent(const int2 *a) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(a),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(unsigned)(v & 0xffffffffull), (int)(unsigned)(v >> 32));
}

__device__ __forceinline__ void fold_point_global(int2 *L, int p, int x, int y, bool &bad) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  const bool ok = (xi < (unsigned)p) & (yi < (unsigned)p);
  bad |= !ok;
  if (ok) {
    const int2 cur = load_coherent(&L[xi]);
    if (y < cur.x) __hip_atomic_fetch_min(&L[xi].x, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (y > cur.y) __hip_atomic_fetch_max(&L[xi].y, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Folding 2*VPT points held as VPT int4 vectors is split in two phases so
// that the stream loop can put its next loads between them: gather reads the
// current (lo, hi) pair of every point's column, all issued before any is
// used; apply compares and issues the atomics.  A point that shares a column
// with an earlier point of the batch may see a value that the earlier point
// is about to improve, which only costs an extra atomic.
template <int VPT>
struct Batch {
  int y[2 * VPT];
  unsigned c[2 * VPT];
  bool ok[2 * VPT];
  int2 cur[2 * VPT];
};

template <int VPT, bool LDS, bool WIN = false>
__device__ __forceinline__ void gather(const int2 *L, int p, const int4 (&q)[VPT], Batch<VPT> &b,
                                       bool &bad, unsigned c0 = 0, unsigned wc = 0) {
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int xs[2] = {q[u].x, q[u].z};
    const int ys[2] = {q[u].y, q[u].w};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * u + h;
      const unsigned xi = (unsigned)(xs[h] - 1), yi = (unsigned)(ys[h] - 1);
      b.ok[j] = (xi < (unsigned)p) & (yi < (unsigned)p);
      bad |= !b.ok[j];
      if (WIN) {
        const unsigned xr = xi - c0;
        b.ok[j] = b.ok[j] & (xr < wc);
        b.c[j] = b.ok[j] ? xr : 0u;
      } else {
        b.c[j] = b.ok[j] ? xi : 0u;
      }
      b.y[j] = ys[h];
    }
  }
#pragma unroll
  for (int j = 0; j < 2 * VPT; ++j) b.cur[j] = LDS ? L[b.c[j]] : load_coherent(&L[b.c[j]]);
}

template <int VPT, bool LDS>
__device__ __forceinline__ void apply(int2 *L, const Batch<VPT> &b) {
#pragma unroll
  for (int j = 0; j < 2 * VPT; ++j) {
    const unsigned c = b.c[j];
    const int y = b.y[j];
    if (LDS) {
      if (b.ok[j] && y < b.cur[j].x) atomicMin(&L[c].x, y);
      if (b.ok[j] && y > b.cur[j].y) atomicMax(&L[c].y, y);
    } else {
      if (b.ok[j] && y < b.cur[j].x)
        __hip_atomic_fetch_min(&L[c].x, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b.ok[j] && y > b.cur[j].y)
        __hip_atomic_fetch_max(&L[c].y, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

struct FinishArgs {
  // source: merged partial L (from_chain == 0) or a chain (from_chain == 1)
  const int2 *part;       // G partial L arrays of p packed words each (or the global L)
  int32_t G;
  int32_t packed;         // part holds packed partial words (pack_partial)
  const int32_t *cx, *clo, *chi;  // chain source
  int32_t positions;      // p, or chain capacity
  int32_t p;
  // outputs of the preconditioner (from_chain == 0)
  int2 *Lm;               // merged L, p pairs
  int32_t *lo, *hi;       // optional L export
  uint64_t *mask;         // optional M export
  int32_t *slab_k, *slab_s, *slab_off;
  // hull
  int32_t do_hull;
  int2 *cand;             // [2 buffers][2 sides][positions]
  int32_t *ccount;        // [2 sides][nodes]
  int32_t *tree_ctr;      // [nodes]
  TreeShape tree;
  int32_t *hx, *hy;
  int32_t hull_cap;
  // control
  int32_t *ctl;
  int32_t *info;
  const int32_t *wg_err;  // per-workgroup range-error words of the reduce
  int32_t n_wg_err;
  unsigned long long *dyn_ctr;  // the reduce's grab counter (cleared here), or null
  const int32_t *wg_cnt;        // per-workgroup chunks folded by the reduce
  int64_t dyn_expect;           // chunks of the run
  // chain: scanned by the last slab (scan_root), then written by it
  // (chain_inline) or by k_chain; otherwise written by the first hull level
  int32_t scan_root;
  int32_t chain_inline;
  int32_t *cx_out, *clo_out, *chi_out;
  int32_t chain_cap;
};

// Arguments of the hull levels above the slabs for one cloud.
struct HullArgs {
  int2 *buf[2];             // [2 sides][positions] each
  uint8_t *keep;            // [2][keep_side] survival flags of the current level
  int64_t keep_side;        // bytes per side of keep (positions rounded up to 4096)
  int32_t *l2cnt;           // [level-2 nodes][test shares][2] survivor counts
  int32_t *ccount;          // [2][nodes] hull sizes of nodes
  TreeShape tree;
  int32_t positions;
  int32_t split;            // test workgroups per child node
  int32_t *hx, *hy;
  int32_t hull_cap;
  int32_t *info;
  int32_t *ctl;             // control words (single level-2 node: test arrivals)
  // chain written by the root compaction (two-level tree, small p)
  int32_t chain_fused;
  const int2 *Lm;
  int32_t p;
  const int32_t *slab_k, *slab_s;
  const int32_t *slab_off;  // scanned slab offsets (k, s and status already written), or null
  const int32_t *wg_err;
  int32_t n_wg_err;
  int32_t *cx, *clo, *chi;
  int32_t chain_cap;
};

// Batched form: one work item of the persistent reduce.
struct BatchItem {
  const int32_t *pts;  // first point of the item (device)
  int64_t count;       // points in the item
  int32_t cloud;       // index into the cloud table
  int32_t mode;        // 0: whole cloud in LDS, 1: LDS + atomic merge, 2: global atomics
};

// Batched form: everything the kernels need about one cloud.  All pointers
// are device memory; cand holds [2 levels][2 sides][p] candidate points.
struct BCloud {
  int32_t p;
  TreeShape tree;
  int2 *Lm;                       // p pairs
  uint64_t *mask;                 // optional M export
  int32_t *slab_k, *slab_s, *slab_off;
  int2 *cand;
  int32_t *ccount;                // [2 sides][tree nodes]
  int32_t *cx, *clo, *chi;        // chain
  int32_t chain_cap;
  int32_t *hx, *hy;               // hull
  int32_t hull_cap;
  int32_t *info;                  // HP_INFO_WORDS words
};

}  // namespace hp
