// hp_device.h -- device-side building blocks shared by the single-cloud and
// batched kernels of libhullprep (gfx950, wave64).
//
// Geometry is exact: coordinates are int32 in [1, 2^31-2] (or their
// negation for the upper side), so every coordinate difference fits in int32
// and every product of two differences in int64 (|.| < 2^62); a cross product
// is the difference of two such products (|.| < 2^63).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hullprep.h"

namespace hp {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSlab = 64;        // columns per slab = one M word = one wave
constexpr int kTile = 16;        // level-0 hull tile (singleton candidates)
constexpr int kFanIn = 64;       // children per hull-tree node above a slab
constexpr int kMaxLevels = 12;   // hull-tree levels (slab level is 1)
constexpr int kSplit = 4;        // hull-test workgroups per child node above the slabs
constexpr int kSplitSlab = 4;    // hull-test workgroups per slab

// The box Algorithm 1 runs on: p columns (x in 1..p) and q rows (y in
// 1..q), an empty column holding (q + 1, -1) (Implementation of the proposed
// heuristic, Step 1 defines p and q).  It converts from a single side (the
// square, q = p) and to its column count, which is what sizes L.
struct Extent {
  int32_t p, q;
  Extent() = default;
  __host__ __device__ constexpr Extent(int32_t s) : p(s), q(s) {}
  __host__ __device__ constexpr Extent(int32_t a, int32_t b) : p(a), q(b) {}
  __host__ __device__ constexpr operator int32_t() const { return p; }
};

// Control words at the head of every workspace.
constexpr int kCtlErr = 0;       // bitmask of data errors seen by kernels
constexpr int kCtlSlabsDone = 1; // slabs finished (last-arriver scan)
constexpr int kCtlTestDone = 2;  // level-2 test workgroups done (single level-2 node)
constexpr int kCtlWords = 64;

constexpr int kErrRange = 1;     // a point outside [1, p]
constexpr int kErrCapacity = 2;  // an output capacity was exceeded
constexpr int kErrBinOverflow = 4;  // the binned reduce ran out of pages (a sizing bug, never expected)

// Status of the per-workgroup error bits of a reduce: a range error is a data
// error; a binning overflow means the L is incomplete (reported as a device
// error rather than as a silently wrong result).
__device__ __forceinline__ void report_reduce_errors(int err, int32_t *info) {
  if (err & kErrRange) atomicMin(&info[HP_INFO_STATUS], HP_ERANGE);
  if (err & kErrBinOverflow) atomicMin(&info[HP_INFO_STATUS], HP_EDEVICE);
}

// Shape of the last-arriver hull tree over `positions` slots: level 1 has one
// node per slab of kSlab positions, level l+1 one node per kFanIn nodes of
// level l, up to a single root.  Node ids are level-major: base[l] + j.
struct TreeShape {
  int32_t nlev;                   // number of levels (>= 1)
  int32_t size[kMaxLevels + 1];   // nodes per level, size[1] = slabs
  int32_t base[kMaxLevels + 1];   // first node id of each level
  int32_t span[kMaxLevels + 1];   // positions covered by one node
  int32_t nodes;                  // total nodes
};

// Exact geometry.  SMALL: every coordinate magnitude is below 2^15, so each
// difference fits in 16 bits, each product of two differences in 30 bits
// (full-rate 24-bit multiplies) and a cross product in int32.  Otherwise the
// products are formed in int64.
template <bool SMALL>
__device__ __forceinline__ long long mulc(int a, int b) {
  if (SMALL) return (long long)__mul24(a, b);
  return (long long)a * (long long)b;
}

template <bool SMALL>
__device__ __forceinline__ bool cross_pos(int2 o, int2 a, int2 b) {  // cross(o, a, b) > 0
  if (SMALL) return __mul24(a.x - o.x, b.y - o.y) > __mul24(a.y - o.y, b.x - o.x);
  return mulc<false>(a.x - o.x, b.y - o.y) > mulc<false>(a.y - o.y, b.x - o.x);
}

template <bool SMALL>
__device__ __forceinline__ bool cross_neg(int2 o, int2 a, int2 b) {  // cross(o, a, b) < 0
  if (SMALL) return __mul24(a.x - o.x, b.y - o.y) < __mul24(a.y - o.y, b.x - o.x);
  return mulc<false>(a.x - o.x, b.y - o.y) < mulc<false>(a.y - o.y, b.x - o.x);
}

// The int64 forms take differences in 64 bits: with coordinates up to
// 2^31 - 2 (or their negation) a difference needs 32 bits plus sign.
template <>
__device__ __forceinline__ bool cross_pos<false>(int2 o, int2 a, int2 b) {
  return ((long long)a.x - o.x) * ((long long)b.y - o.y) > ((long long)a.y - o.y) * ((long long)b.x - o.x);
}

template <>
__device__ __forceinline__ bool cross_neg<false>(int2 o, int2 a, int2 b) {
  return ((long long)a.x - o.x) * ((long long)b.y - o.y) < ((long long)a.y - o.y) * ((long long)b.x - o.x);
}

// slope(u1, v) > slope(u2, v) for u1, u2 strictly left of v.
template <bool SMALL>
__device__ __forceinline__ bool steeper_left(int2 u1, int2 u2, int2 v) {
  if (SMALL) return __mul24(v.y - u1.y, v.x - u2.x) > __mul24(v.y - u2.y, v.x - u1.x);
  return ((long long)v.y - u1.y) * ((long long)v.x - u2.x) > ((long long)v.y - u2.y) * ((long long)v.x - u1.x);
}

// slope(v, w1) < slope(v, w2) for w1, w2 strictly right of v.
template <bool SMALL>
__device__ __forceinline__ bool flatter_right(int2 w1, int2 w2, int2 v) {
  if (SMALL) return __mul24(w1.y - v.y, w2.x - v.x) < __mul24(w2.y - v.y, w1.x - v.x);
  return ((long long)w1.y - v.y) * ((long long)w2.x - v.x) < ((long long)w2.y - v.y) * ((long long)w1.x - v.x);
}

// Lower convex chain a[0..m) entirely left of v: index of the vertex that
// maximises slope(a[t], v) (the lower tangent from v).  Along the chain that
// slope rises while v lies strictly left of the directed edge a[t]->a[t+1]
// and falls afterwards, so a binary search on that predicate finds it.
template <bool SMALL>
__device__ __forceinline__ int tangent_left(const int2 *a, int m, int2 v) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cross_pos<SMALL>(a[mid], a[mid + 1], v)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Lower convex chain b[0..m) entirely right of v: index minimising
// slope(v, b[t]) (mirror image of tangent_left).
template <bool SMALL>
__device__ __forceinline__ int tangent_right(const int2 *b, int m, int2 v) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cross_neg<SMALL>(v, b[mid], b[mid + 1])) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Wave-wide exclusive prefix count of `flag` and the wave total.
__device__ __forceinline__ int wave_rank(bool flag, int *total) {
  const unsigned long long m = __ballot(flag);
  *total = __popcll(m);
  const unsigned lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  return __popcll(m & below);
}

}  // namespace hp
