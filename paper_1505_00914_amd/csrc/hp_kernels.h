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
__device__ __forceinline__ void fold_point_lds(int2 *L, int p, int x, int y, bool &bad) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  if (xi < (unsigned)p && yi < (unsigned)p) {
    const int2 cur = L[xi];
    if (y < cur.x) atomicMin(&L[xi].x, y);
    if (y > cur.y) atomicMax(&L[xi].y, y);
  } else {
    bad = true;
  }
}

__device__ __forceinline__ void fold_point_global(int2 *L, int p, int x, int y, bool &bad) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  if (xi < (unsigned)p && yi < (unsigned)p) {
    const int2 cur = L[xi];
    if (y < cur.x) __hip_atomic_fetch_min(&L[xi].x, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (y > cur.y) __hip_atomic_fetch_max(&L[xi].y, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    bad = true;
  }
}

struct FinishArgs {
  // source: merged partial L (from_chain == 0) or a chain (from_chain == 1)
  const int2 *part;       // G partial L arrays of p pairs each (or the global L)
  int32_t G;
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
};

}  // namespace hp
