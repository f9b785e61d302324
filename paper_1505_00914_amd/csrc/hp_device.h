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

namespace hp {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSlab = 64;        // columns per slab = one M word = one wave
constexpr int kTile = 16;        // level-0 hull tile (singleton candidates)
constexpr int kFanIn = 16;       // children per hull-tree node above a slab
constexpr int kMaxLevels = 12;   // hull-tree levels (slab level is 1)

// Control words at the head of every workspace.
constexpr int kCtlErr = 0;       // bitmask of data errors seen by kernels
constexpr int kCtlSlabsDone = 1; // slabs finished (last-arriver scan)
constexpr int kCtlWords = 64;

constexpr int kErrRange = 1;     // a point outside [1, p]
constexpr int kErrCapacity = 2;  // an output capacity was exceeded

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

__device__ __forceinline__ long long cross3(int2 o, int2 a, int2 b) {
  return ((long long)a.x - o.x) * ((long long)b.y - o.y) -
         ((long long)a.y - o.y) * ((long long)b.x - o.x);
}

// slope(u1, v) > slope(u2, v) for u1, u2 strictly left of v.
__device__ __forceinline__ bool steeper_left(int2 u1, int2 u2, int2 v) {
  long long l = ((long long)v.y - u1.y) * ((long long)v.x - u2.x);
  long long r = ((long long)v.y - u2.y) * ((long long)v.x - u1.x);
  return l > r;
}

// slope(v, w1) < slope(v, w2) for w1, w2 strictly right of v.
__device__ __forceinline__ bool flatter_right(int2 w1, int2 w2, int2 v) {
  long long l = ((long long)w1.y - v.y) * ((long long)w2.x - v.x);
  long long r = ((long long)w2.y - v.y) * ((long long)w1.x - v.x);
  return l < r;
}

// Lower convex chain a[0..m) entirely left of v: index of the vertex that
// maximises slope(a[t], v) (the lower tangent from v).  Along the chain that
// slope rises while v lies strictly left of the directed edge a[t]->a[t+1]
// and falls afterwards, so a binary search on that predicate finds it.
__device__ __forceinline__ int tangent_left(const int2 *a, int m, int2 v) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cross3(a[mid], a[mid + 1], v) > 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Lower convex chain b[0..m) entirely right of v: index minimising
// slope(v, b[t]) (mirror image of tangent_left).
__device__ __forceinline__ int tangent_right(const int2 *b, int m, int2 v) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cross3(v, b[mid], b[mid + 1]) < 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Lower-hull membership of candidate r of child j, given that every child is
// the lower hull of an x-separated group of points listed left to right.  v
// is a strict vertex of the lower hull of the union iff the steepest slope
// into v from any point on its left is smaller than the flattest slope out of
// v to any point on its right; both extremes are attained on the children's
// hulls (own neighbours, tangents to the other children).
__device__ inline bool lower_survives(const int2 *data, const int *cs, const int *cc,
                                      int nchild, int j, int r) {
  const int2 v = data[cs[j] + r];
  bool hasL = false, hasR = false;
  int2 uL = v, wR = v;
  if (r > 0) { uL = data[cs[j] + r - 1]; hasL = true; }
  for (int t = 0; t < j; ++t) {
    const int m = cc[t];
    if (m == 0) continue;
    const int2 *a = data + cs[t];
    const int2 u = a[tangent_left(a, m, v)];
    if (!hasL || steeper_left(u, uL, v)) { uL = u; hasL = true; }
  }
  if (r + 1 < cc[j]) { wR = data[cs[j] + r + 1]; hasR = true; }
  for (int t = j + 1; t < nchild; ++t) {
    const int m = cc[t];
    if (m == 0) continue;
    const int2 *b = data + cs[t];
    const int2 w = b[tangent_right(b, m, v)];
    if (!hasR || flatter_right(w, wR, v)) { wR = w; hasR = true; }
  }
  if (!hasL || !hasR) return true;
  return cross3(uL, v, wR) > 0;
}

// Wave-wide exclusive prefix count of `flag` and the wave total.
__device__ __forceinline__ int wave_rank(bool flag, int *total) {
  const unsigned long long m = __ballot(flag);
  *total = __popcll(m);
  const unsigned lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  return __popcll(m & below);
}

// Merge `nchild` x-ordered lower hulls into the lower hull of their union,
// by the whole workgroup.  data/cs/cc describe the children (cs, cc in LDS);
// survivors are written in order to out[0..), and the count is returned to
// every thread.  s_tmp: LDS scratch of BLOCK/kWave + 1 ints.
template <int BLOCK>
__device__ int merge_lower(const int2 *data, const int *cs, const int *cc, int nchild,
                           int2 *out, int *s_tmp) {
  __shared__ int s_pref[kFanIn + 1];
  const int tid = threadIdx.x;
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < nchild; ++t) { s_pref[t] = acc; acc += cc[t]; }
    s_pref[nchild] = acc;
  }
  __syncthreads();
  const int total = s_pref[nchild];
  int written = 0;
  for (int base = 0; base < total; base += BLOCK) {
    const int q = base + tid;
    bool keep = false;
    int2 v = make_int2(0, 0);
    if (q < total) {
      int j = 0;
      while (j + 1 < nchild && s_pref[j + 1] <= q) ++j;
      const int r = q - s_pref[j];
      v = data[cs[j] + r];
      keep = lower_survives(data, cs, cc, nchild, j, r);
    }
    int wt;
    const int wr = wave_rank(keep, &wt);
    const int w = tid / kWave;
    if ((tid & (kWave - 1)) == 0) s_tmp[w] = wt;
    __syncthreads();
    int off = 0, all = 0;
    for (int i = 0; i < BLOCK / kWave; ++i) {
      if (i < w) off += s_tmp[i];
      all += s_tmp[i];
    }
    if (keep) out[written + off + wr] = v;
    written += all;
    __syncthreads();
  }
  return written;
}

}  // namespace hp
