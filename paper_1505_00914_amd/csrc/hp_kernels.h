// hp_kernels.h -- the per-point step of Algorithm 1 on the device: folding
// points into an (lo, hi) pair array in LDS or device memory, and the packed
// partial-L words.  Used by the single-cloud and batched reduce kernels.
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
__device__ __forceinline__ void fold_point_lds(int2 *L, Extent p, int x, int y, bool &bad, unsigned c0 = 0,
                                               unsigned wc = 0) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  bool ok = (xi < (unsigned)p.p) & (yi < (unsigned)p.q);
  bad |= !ok;
  const unsigned xr = xi - c0;
  if (wc) ok = ok & (xr < wc);
  const unsigned c = ok ? xr : 0u;
  const int2 cur = L[c];
  if (ok && y < cur.x) atomicMin(&L[c].x, y);
  if (ok && y > cur.y) atomicMax(&L[c].y, y);
}

// A partial L entry in 32 bits: lo - 1 in the low half, hi + 1 in the high
// half (the sentinel (q+1, -1) becomes (q, 0)); valid for q < 65535 rows.
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

__device__ __forceinline__ void fold_point_global(int2 *L, Extent p, int x, int y, bool &bad) {
  const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
  const bool ok = (xi < (unsigned)p.p) & (yi < (unsigned)p.q);
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

// Filtered device-L folding.  A point goes on to its column of L only when
// its y lies outside the range filt[column >> fshift] (inside it, y can
// improve neither extreme; see k_reduce_filtered).  Passing points are
// queued per wave in LDS as (column, y) and folded kFiltFlush or more at a
// time, up to four coherent reads in flight per lane, so that the reads of
// L cost one round trip per few hundred passing points instead of one per
// batch of the stream.  A wave's LDS program order makes its queue writes
// visible to its own later reads.
constexpr int kFiltFlush = 128;
__host__ __device__ constexpr int filt_queue_cap(int vpt) { return kFiltFlush + 2 * vpt * kWave; }

__device__ __forceinline__ void filt_flush(int2 *L, const int2 *wq, int qn) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int k = 0; k < qn; k += 4 * kWave) {
    int2 e[4], cur[4];
    bool ok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = k + r * kWave + lane;
      ok[r] = i < qn;
      e[r] = ok[r] ? wq[i] : make_int2(0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) cur[r] = ok[r] ? load_coherent(&L[e[r].x]) : make_int2(0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (ok[r] && e[r].y < cur[r].x)
        __hip_atomic_fetch_min(&L[e[r].x].x, e[r].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ok[r] && e[r].y > cur[r].y)
        __hip_atomic_fetch_max(&L[e[r].x].y, e[r].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int VPT, bool LDS, bool WIN = false, bool FILT = false>
__device__ __forceinline__ void gather(const int2 *L, Extent p, const int4 (&q)[VPT], Batch<VPT> &b,
                                       bool &bad, unsigned c0 = 0, unsigned wc = 0,
                                       const int2 *filt = nullptr, int fshift = 0, int2 *wq = nullptr,
                                       int *qn = nullptr) {
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int xs[2] = {q[u].x, q[u].z};
    const int ys[2] = {q[u].y, q[u].w};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * u + h;
      const unsigned xi = (unsigned)(xs[h] - 1), yi = (unsigned)(ys[h] - 1);
      b.ok[j] = (xi < (unsigned)p.p) & (yi < (unsigned)p.q);
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
  if (FILT) {
    const unsigned lane = threadIdx.x & (kWave - 1);
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int n = *qn;
#pragma unroll
    for (int j = 0; j < 2 * VPT; ++j) {
      const int2 f = filt[b.c[j] >> fshift];
      const bool need = b.ok[j] & ((b.y[j] < f.x) | (b.y[j] > f.y));
      const unsigned long long m = __ballot(need);
      if (need) wq[n + __popcll(m & below)] = make_int2((int)b.c[j], b.y[j]);
      n += __popcll(m);
      b.ok[j] = false;   // folded from the queue instead
    }
    *qn = n;
    return;
  }
#pragma unroll
  for (int j = 0; j < 2 * VPT; ++j) b.cur[j] = LDS ? L[b.c[j]] : load_coherent(&L[b.c[j]]);
}

template <int VPT, bool LDS, bool FILT = false>
__device__ __forceinline__ void apply(int2 *L, const Batch<VPT> &b, const int2 *wq = nullptr, int *qn = nullptr) {
  if (FILT) {
    if (*qn >= kFiltFlush) {
      filt_flush(L, wq, *qn);
      *qn = 0;
    }
    return;
  }
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

}  // namespace hp
