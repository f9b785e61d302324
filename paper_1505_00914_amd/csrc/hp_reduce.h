// hp_reduce.h -- Algorithm 1 on the device: the point stream and the
// single-cloud reduce kernels (workgroup-private L in LDS, written out as a
// partial or merged by atomics; or one L in device memory).  The batched
// reduce streams its work items with the same stream_points.
#pragma once

#include <climits>

#include "hp_kernels.h"

namespace hp {

// ---------------------------------------------------------------------------
// Algorithm 1.  Points are read once, 16 bytes (two points) per lane per
// load, VPT loads in flight per lane; consecutive lanes read consecutive
// vectors and consecutive workgroups consecutive chunks.
// ---------------------------------------------------------------------------

// A 16-byte load of the point stream, marked non-temporal: every point is
// read exactly once, so the caches are better left to L and the partials
// (measured: 4 % faster on 80 MB, 8 % on 2 GiB).  The column-window reduce
// keeps plain loads: its W reads of one chunk group are meant to hit L2.
// Translation by an origin (the heuristic's Step 2): a point is read as
// (x - ox, y - oy), computed modulo 2^32 so that any int32 origin works; the
// range check on the result then applies as usual.
__device__ __forceinline__ int shift_by(int v, int o) { return (int)((unsigned)v - (unsigned)o); }
__device__ __forceinline__ int4 shift_by(int4 q, int ox, int oy) {
  return make_int4(shift_by(q.x, ox), shift_by(q.y, oy), shift_by(q.z, ox), shift_by(q.w, oy));
}

typedef int hp_v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 load_stream(const int4 *a) {
  const hp_v4i t = __builtin_nontemporal_load(reinterpret_cast<const hp_v4i *>(a));
  return make_int4(t.x, t.y, t.z, t.w);
}
template <int BLOCK, int VPT, bool LDS, bool WIN = false, bool FILT = false>
__device__ __forceinline__ void stream_points(const int32_t *__restrict__ pts, int64_t n, Extent p,
                                              int2 *L, int64_t wg, int64_t nwg, bool &bad,
                                              unsigned c0 = 0, unsigned wc = 0,
                                              const int2 *filt = nullptr, int fshift = 0,
                                              int2 *wq = nullptr, int ox = 0, int oy = 0) {
  int qn = 0;   // FILT: entries in this wave's queue
  // pts is 8-byte aligned (checked on the host); peel one point if the
  // vector body would otherwise start on an 8-byte boundary.
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int64_t tail = head + 2 * nv;  // index of the odd last point, if any
  if (wg == 0 && threadIdx.x == 0) {
    if (head) {
      const int x = shift_by(pts[0], ox), y = shift_by(pts[1], oy);
      if (LDS) fold_point_lds(L, p, x, y, bad, c0, wc);
      else fold_point_global(L, p, x, y, bad);
    }
    if (tail < n) {
      const int x = shift_by(pts[2 * tail], ox), y = shift_by(pts[2 * tail + 1], oy);
      if (LDS) fold_point_lds(L, p, x, y, bad, c0, wc);
      else fold_point_global(L, p, x, y, bad);
    }
  }
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  constexpr int64_t chunk = (int64_t)BLOCK * VPT;
  const int64_t step = nwg * chunk;
  int64_t t0 = wg * chunk;
  // Full chunks, software-pipelined: the next chunk's loads are issued
  // before the current chunk is folded into L, so VPT 16-byte loads per
  // lane stay in flight.
  int4 q[VPT];
  bool have = t0 + chunk <= nv;
  if (have) {
#pragma unroll
    for (int u = 0; u < VPT; ++u)
      q[u] = shift_by(WIN ? v[t0 + u * BLOCK + threadIdx.x] : load_stream(&v[t0 + u * BLOCK + threadIdx.x]), ox, oy);
  }
  // The loop runs while a next full chunk exists; the workgroup's last full
  // chunk is folded after it with no loads issued, so no vector is read
  // twice (a select of the load address would keep the loop branch-free but
  // re-read the last chunk).
  while (have && t0 + step + chunk <= nv) {
    const int64_t t1 = t0 + step;
    Batch<VPT> b;
    gather<VPT, LDS, WIN, FILT>(L, p, q, b, bad, c0, wc, filt, fshift, wq, &qn);
    int4 qv[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u)
      qv[u] = shift_by(WIN ? v[t1 + u * BLOCK + threadIdx.x] : load_stream(&v[t1 + u * BLOCK + threadIdx.x]), ox, oy);
    apply<VPT, LDS, FILT>(L, b, wq, &qn);
#pragma unroll
    for (int u = 0; u < VPT; ++u) q[u] = qv[u];
    t0 = t1;
  }
  if (have) {
    Batch<VPT> b;
    gather<VPT, LDS, WIN, FILT>(L, p, q, b, bad, c0, wc, filt, fshift, wq, &qn);
    apply<VPT, LDS, FILT>(L, b, wq, &qn);
    t0 += step;
  }
  // at most one partial chunk remains for this workgroup
  if (t0 < nv) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int64_t idx = t0 + u * BLOCK + threadIdx.x;
      if (idx < nv) {
        const int4 r = shift_by(v[idx], ox, oy);
        if (LDS) {
          fold_point_lds(L, p, r.x, r.y, bad, c0, wc);
          fold_point_lds(L, p, r.z, r.w, bad, c0, wc);
        } else {
          fold_point_global(L, p, r.x, r.y, bad);
          fold_point_global(L, p, r.z, r.w, bad);
        }
      }
    }
  }
  if (FILT) filt_flush(L, wq, qn);
}

// Work sharing of the single-cloud reduce.  The vector body is cut into
// chunks of BLOCK * VPT vectors (the last one possibly partial).  Workgroup
// wg first takes chunks wg, wg + nwg, ... below `nstat` (a fixed fraction of
// its equal share); the chunks from nstat on are handed out in pairs by a
// device-wide counter, so that workgroups that started late (whole XCDs are
// dispatched microseconds apart) or stream slowly take fewer of them.
// Thread 0 issues the grab of the next pair when it hands out the current
// one, so the atomic's latency hides behind two chunks of streaming, and
// passes the pair to the workgroup through LDS (the barrier waits on LDS
// only, not on the loads in flight).  The counter is zero at the start of a
// run and is cleared by the finish step; each workgroup records how many
// chunks it folded so that the finish step can check that every chunk was
// folded exactly once.
struct DynArgs {
  unsigned long long *ctr;  // grab counter, zero at the start of the run (null: static only)
  int32_t *wg_cnt;          // per workgroup: chunks folded
  int32_t static_frac8;     // static share, in eighths of the equal share
};

__host__ __device__ __forceinline__ int64_t dyn_chunks(int64_t n, uintptr_t pts, int64_t chunk) {
  const int64_t head = (n > 0 && (pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  return (nv + chunk - 1) / chunk;
}

template <int BLOCK, int VPT, bool LDS, bool FILT = false>
__device__ __forceinline__ void stream_points_dyn(const int32_t *__restrict__ pts, int64_t n, Extent p, int2 *L,
                                                  int64_t wg, int64_t nwg, bool &bad, const DynArgs &D,
                                                  int *s_slot, const int2 *filt = nullptr, int fshift = 0,
                                                  int2 *wq = nullptr, int ox = 0, int oy = 0) {
  int qn = 0;   // FILT: entries in this wave's queue
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int64_t tail = head + 2 * nv;
  if (wg == 0 && threadIdx.x == 0) {
    if (head) {
      const int x = shift_by(pts[0], ox), y = shift_by(pts[1], oy);
      if (LDS) fold_point_lds(L, p, x, y, bad);
      else fold_point_global(L, p, x, y, bad);
    }
    if (tail < n) {
      const int x = shift_by(pts[2 * tail], ox), y = shift_by(pts[2 * tail + 1], oy);
      if (LDS) fold_point_lds(L, p, x, y, bad);
      else fold_point_global(L, p, x, y, bad);
    }
  }
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  constexpr int64_t chunk = (int64_t)BLOCK * VPT;
  const int64_t nfull = nv / chunk;
  const int64_t ntot = (nv + chunk - 1) / chunk;   // nfull, plus a partial chunk
  // static chunks per workgroup: none, or at least two (the first grab goes
  // out two chunks before the static ones run out)
  int64_t mine = (ntot / nwg) * D.static_frac8 / 8;
  if (mine < 2) mine = 0;
  const int64_t nstat = mine * nwg;
  const bool dyn = ntot > nstat;
  int64_t k = 0;                  // static chunks handed out
  int pos = 0;                    // chunks of the current pair handed out (0: need a grab)
  int64_t pair = 0;               // first chunk of the current pair
  int slot = 0;                   // LDS slot of the next refill (two, used in turn)
  unsigned long long g = 0;       // thread 0: the grab in flight
  bool issued = false;            // thread 0: whether g is in flight
  // the next chunk index of this workgroup, or -1; uniform over the workgroup
  auto next = [&]() -> int64_t {
    if (k < mine) {
      const int64_t c = wg + k * nwg;
      ++k;
      if (dyn && threadIdx.x == 0 && k == mine - 2) {
        g = __hip_atomic_fetch_add(D.ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        issued = true;
      }
      return c;
    }
    if (!dyn) return -1;
    if (pos == 1) {
      pos = 0;
      return pair + 1 < ntot ? pair + 1 : -1;
    }
    if (threadIdx.x == 0) {
      if (!issued) g = __hip_atomic_fetch_add(D.ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_slot[slot] = (int)(g < 0x7fffffffull ? g : 0x7fffffffull);   // pairs: far below 2^31
      g = __hip_atomic_fetch_add(D.ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      issued = true;
    }
    // one barrier per refill: a slot is written again only two refills
    // later, after every wave has passed the barrier in between
    __syncthreads();
    pair = nstat + 2 * (int64_t)s_slot[slot];
    slot ^= 1;
    pos = 1;
    return pair < ntot ? pair : -1;
  };
  // chunk indices run one ahead of the loads: the barrier of a refill is
  // taken while the next chunk's loads are in flight
  int folded = 0;
  int64_t part = -1;              // the partial chunk, if this workgroup gets it
  const bool has_part = ntot > nfull;
  auto take = [&](int64_t c) -> int64_t {
    if (has_part && c == nfull) {
      part = c;
      return -1;
    }
    return c;
  };
  int64_t cur = take(next());
  int64_t nx = cur >= 0 ? take(next()) : -1;
  int4 q[VPT];
  if (cur >= 0) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) q[u] = shift_by(load_stream(&v[cur * chunk + u * BLOCK + threadIdx.x]), ox, oy);
  }
  // as in stream_points, the last chunk is folded after the loop with no
  // loads issued
  while (cur >= 0 && nx >= 0) {
    Batch<VPT> b;
    gather<VPT, LDS, false, FILT>(L, p, q, b, bad, 0, 0, filt, fshift, wq, &qn);
    int4 qv[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) qv[u] = shift_by(load_stream(&v[nx * chunk + u * BLOCK + threadIdx.x]), ox, oy);
    apply<VPT, LDS, FILT>(L, b, wq, &qn);
    ++folded;
    const int64_t nn = take(next());
#pragma unroll
    for (int u = 0; u < VPT; ++u) q[u] = qv[u];
    cur = nx;
    nx = nn;
  }
  if (cur >= 0) {
    Batch<VPT> b;
    gather<VPT, LDS, false, FILT>(L, p, q, b, bad, 0, 0, filt, fshift, wq, &qn);
    apply<VPT, LDS, FILT>(L, b, wq, &qn);
    ++folded;
  }
  if (part >= 0) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int64_t idx = part * chunk + u * BLOCK + threadIdx.x;
      if (idx < nv) {
        const int4 r = shift_by(v[idx], ox, oy);
        if (LDS) {
          fold_point_lds(L, p, r.x, r.y, bad);
          fold_point_lds(L, p, r.z, r.w, bad);
        } else {
          fold_point_global(L, p, r.x, r.y, bad);
          fold_point_global(L, p, r.z, r.w, bad);
        }
      }
    }
    ++folded;
  }
  if (FILT) filt_flush(L, wq, qn);
  if (threadIdx.x == 0) D.wg_cnt[wg] = folded;
}

// Control words the finish step relies on.  When no init kernel runs (the
// partial-L strategy), workgroup 0 of the reduce kernel clears them: the
// finish kernel only starts after the reduce kernel has completed.
struct ResetArgs {
  int32_t *ctl;
  int32_t *tree_ctr;
  int32_t nodes;
  int32_t *info;
};

__device__ __forceinline__ void reset_controls(const ResetArgs &R) {
  if (blockIdx.x != 0 || R.ctl == nullptr) return;
  for (int j = threadIdx.x; j < kCtlWords; j += blockDim.x) R.ctl[j] = 0;
  for (int j = threadIdx.x; j < R.nodes; j += blockDim.x) R.tree_ctr[j] = 0;
  if (threadIdx.x < HP_INFO_WORDS) R.info[threadIdx.x] = 0;
}

// Workgroup-private L in LDS.  MERGE_ATOMIC: folded into the device L with
// filtered device-scope atomics (only touched columns that improve on the
// value read first); otherwise written out as one partial L per workgroup
// and merged by k_finish.  Every workgroup writes its own range-error word.
template <int BLOCK, int VPT, bool MERGE_ATOMIC>
__global__ __launch_bounds__(BLOCK) void k_reduce_lds(const int32_t *__restrict__ pts, int64_t n,
                                                      Extent p, int2 *__restrict__ out_L,
                                                      int32_t *__restrict__ wg_err, ResetArgs R, DynArgs D,
                                                      int2 org) {
  extern __shared__ int2 sL[];           // p pairs, then the flag word and the two grab slots
  int &s_bad = sL[p].x;
  int *s_slot = &sL[p].y;                // sL[p].y and sL[p + 1].x
  reset_controls(R);
  if (threadIdx.x == 0) s_bad = 0;
  for (int c = threadIdx.x; c < p; c += BLOCK) sL[c] = make_int2(p.q + 1, -1);
  __syncthreads();
  bool bad = false;
  if (D.ctr)
    stream_points_dyn<BLOCK, VPT, true>(pts, n, p, sL, blockIdx.x, gridDim.x, bad, D, s_slot, nullptr, 0, nullptr,
                                        org.x, org.y);
  else
    stream_points<BLOCK, VPT, true>(pts, n, p, sL, blockIdx.x, gridDim.x, bad, 0, 0, nullptr, 0, nullptr, org.x, org.y);
  if (bad) s_bad = 1;
  __syncthreads();
  if (MERGE_ATOMIC) {
    for (int c = threadIdx.x; c < p; c += BLOCK) {
      const int2 mine = sL[c];
      if (mine.x > mine.y) continue;  // column untouched by this workgroup
      const int2 cur = load_coherent(&out_L[c]);
      if (mine.x < cur.x)
        __hip_atomic_fetch_min(&out_L[c].x, mine.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (mine.y > cur.y)
        __hip_atomic_fetch_max(&out_L[c].y, mine.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else {
    // the partial L packs (lo - 1, hi + 1) into 16 bits each (the strategy
    // is taken only for fewer than 2^16 - 1 rows): half the bytes of the pairs
    uint32_t *out = reinterpret_cast<uint32_t *>(out_L) + (size_t)blockIdx.x * (size_t)p;
    for (int c = threadIdx.x; c < p; c += BLOCK) out[c] = pack_partial(sL[c]);
  }
  if (threadIdx.x == 0) wg_err[blockIdx.x] = s_bad ? kErrRange : 0;
}

// Column windows of L in LDS (p above the LDS limit).  The grid is Gc
// chunk groups times W windows, Gc a multiple of 8; workgroup b runs window
// (b / 8) % W of chunk group (b / 8 / W) * 8 + b % 8, so the W workgroups
// that read one chunk group have consecutive dispatch slots on the same XCD
// (workgroups are dealt to the 8 XCDs in turn) and the repeated reads of its
// points hit that XCD's L2.  Each writes its window of the chunk group's
// partial array (packed words when p allows, else pairs); the finish step
// folds the Gc partials.
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_reduce_window(const int32_t *__restrict__ pts, int64_t n,
                                                         Extent p, int32_t W, int32_t wc,
                                                         uint32_t *__restrict__ out_part,
                                                         int32_t *__restrict__ wg_err, ResetArgs R, int2 org) {
  extern __shared__ int2 sL[];           // wc pairs, then one flag word
  int &s_bad = reinterpret_cast<int &>(sL[wc]);
  const int b = blockIdx.x, k = b >> 3;
  const int w = k % W, cg = (k / W) * 8 + (b & 7);
  const int Gc = (int)(gridDim.x / W);
  const unsigned c0 = (unsigned)w * (unsigned)wc;
  reset_controls(R);
  if (threadIdx.x == 0) s_bad = 0;
  for (int c = threadIdx.x; c < wc; c += BLOCK) sL[c] = make_int2(p.q + 1, -1);
  __syncthreads();
  bool bad = false;
  stream_points<BLOCK, VPT, true, true>(pts, n, p, sL, cg, Gc, bad, c0, (unsigned)wc, nullptr, 0, nullptr, org.x,
                                        org.y);
  if (bad) s_bad = 1;
  __syncthreads();
  const int ncol = min(wc, p - (int)c0);
  if (partial_packs(p.q)) {
    uint32_t *out = out_part + (size_t)cg * (size_t)p + c0;
    for (int c = threadIdx.x; c < ncol; c += BLOCK) out[c] = pack_partial(sL[c]);
  } else {
    int2 *out = reinterpret_cast<int2 *>(out_part) + (size_t)cg * (size_t)p + c0;
    for (int c = threadIdx.x; c < ncol; c += BLOCK) out[c] = sL[c];
  }
  if (threadIdx.x == 0) wg_err[b] = s_bad ? kErrRange : 0;
}

// One L in device memory, updated with filtered device-scope atomics.
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_reduce_global(const int32_t *__restrict__ pts, int64_t n,
                                                         Extent p, int2 *L,
                                                         int32_t *__restrict__ wg_err, ResetArgs R, DynArgs D,
                                                         int2 org) {
  __shared__ int s_bad;
  __shared__ int s_slot[2];
  reset_controls(R);
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  if (D.ctr)
    stream_points_dyn<BLOCK, VPT, false>(pts, n, p, L, blockIdx.x, gridDim.x, bad, D, s_slot, nullptr, 0, nullptr,
                                         org.x, org.y);
  else
    stream_points<BLOCK, VPT, false>(pts, n, p, L, blockIdx.x, gridDim.x, bad, 0, 0, nullptr, 0, nullptr, org.x, org.y);
  if (bad) s_bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) wg_err[blockIdx.x] = s_bad ? kErrRange : 0;
}

// ---------------------------------------------------------------------------
// Sampled filter for a device L (p above what LDS windows cover).  A first
// pass folds a sample of the points into L exactly (k_reduce_global over a
// prefix of the points).  k_filter_build then bounds, per group of 2^fshift
// columns, the largest sampled lo and the smallest sampled hi: F[g] =
// (max lo, min hi), or (q + 1, -1) -- filter nothing -- when a column of the
// group has no sampled point.  The main pass (k_reduce_filtered) keeps F in
// LDS and sends a point on to the read of its column in L only when y < F.x
// or y > F.y.  A point it skips has lo_final <= lo_sample <= F.x <= y and,
// likewise, y <= hi_final, so it cannot change L.  With k sampled points
// per column about 1 / (k + 1) of the remaining points still read L.
// (k_filter_build is in hp_single.hip.)
// ---------------------------------------------------------------------------
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_reduce_filtered(const int32_t *__restrict__ pts, int64_t n,
                                                           Extent p, int2 *L, const int2 *__restrict__ F,
                                                           int32_t fshift, int32_t ngroups,
                                                           int32_t *__restrict__ wg_err, DynArgs D, int2 org) {
  // LDS: ngroups filter pairs, the flag word and two grab slots (2 pairs),
  // then one queue of filt_queue_cap(VPT) entries per wave
  extern __shared__ int2 sF[];
  int &s_bad = sF[ngroups].x;
  int *s_slot = &sF[ngroups].y;          // sF[ngroups].y and sF[ngroups + 1].x
  int2 *wq = sF + ngroups + 2 + (threadIdx.x / kWave) * filt_queue_cap(VPT);
  for (int g = threadIdx.x; g < ngroups; g += BLOCK) sF[g] = F[g];
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  if (D.ctr)
    stream_points_dyn<BLOCK, VPT, false, true>(pts, n, p, L, blockIdx.x, gridDim.x, bad, D, s_slot, sF, fshift, wq,
                                               org.x, org.y);
  else
    stream_points<BLOCK, VPT, false, false, true>(pts, n, p, L, blockIdx.x, gridDim.x, bad, 0, 0, sF, fshift, wq,
                                                  org.x, org.y);
  if (bad) s_bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) wg_err[blockIdx.x] = s_bad ? kErrRange : 0;
}

}  // namespace hp
