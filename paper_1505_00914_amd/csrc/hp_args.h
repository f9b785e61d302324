// hp_args.h -- argument blocks of the finish and hull steps of one cloud and
// of the batched form.  See hullprep.h for the contract.
//
// Launch sequence of one cloud (all on the caller's stream):
//   k_init      control words, tree counters, info; the global L when an
//               atomic strategy is used                    (L initialisation)
//   k_reduce_*  Algorithm 1 over the points                 (Algorithm 1)
//   k_finish    per slab of 64 columns: merge of the partial L arrays, the M
//               word, slab counts, the slab hulls
//   k_l2_*      the hull of the slab hulls (all-vertex test) and the chain
//               (Lemma 1); above 4096 columns, tangent levels k_hull_*
#pragma once

#include "hp_kernels.h"

namespace hp {

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
  int32_t n_wg_cnt;             // workgroups of the pass that shared chunks
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
  // chain written by the level-2 test (and the totals, unless slab_off is set)
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
