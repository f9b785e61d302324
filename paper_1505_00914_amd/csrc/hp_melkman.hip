// hp_melkman.hip -- Melkman's hull of the Lemma 1 polyline on the device.
//
// The reduced sequence, walked column by column as (x, lo) then (x, hi), is a
// simple polyline (Lemma 1), so Melkman's deque algorithm finds its hull in
// one pass over it.  The algorithm is sequential: one wave runs it in step,
// with the deque in LDS when the chain capacity lets it fit (chains of up to
// 5119 columns) and in the caller's workspace otherwise.  It is a second, exact
// hull of the same chain, in the canonical form of hp_hull (straight angles
// removed, counter-clockwise from the lexicographic minimum), not a fast
// path: the parallel hull of hp_hull and hp_run is the one to use for speed.
#include "hp_host.h"
#include "hp_device.h"

namespace hp {

// Twice the signed area of (a, b, c).  Coordinates are int32, so every
// difference fits in 33 bits and each product in 64; when every coordinate
// lies in [0, 2^15) (SMALL) the differences fit in 16 bits and the whole
// expression in 32.
template <bool SMALL>
__device__ __forceinline__ long long melk_orient(int2 a, int2 b, int2 c) {
  if (SMALL) return (long long)((b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x));
  return ((long long)b.x - a.x) * ((long long)c.y - a.y) - ((long long)b.y - a.y) * ((long long)c.x - a.x);
}

// Walks the reduced sequence of a chain: (x, lo), then (x, hi) when hi > lo.
// The whole wave runs the walk in step (every lane computes the same
// values); the chain is loaded 64 columns at a time with one coalesced load
// per array, lane i holding column base + i, and each column is taken from
// its lane by readlane.
struct ChainWalk {
  const int32_t *cx, *clo, *chi;
  int32_t k, t, base, prevx;
  int32_t vx, vlo, vhi;  // this lane's column of the loaded chunk
  bool upper, bad;
  __device__ void load(int32_t b) {
    base = b;
    const int32_t i = b + (int32_t)(threadIdx.x & 63);
    vx = i < k ? cx[i] : 0;
    vlo = i < k ? clo[i] : 0;
    vhi = i < k ? chi[i] : 0;
  }
  __device__ bool next(int2 &v) {
    if (t >= k) return false;
    if (t >= base + 64) load(t & ~63);
    const int lane = t - base;
    const int32_t x = __builtin_amdgcn_readlane(vx, lane);
    if (!upper) {
      const int32_t lo = __builtin_amdgcn_readlane(vlo, lane), hi = __builtin_amdgcn_readlane(vhi, lane);
      if (hi < lo || (t > 0 && prevx >= x)) {
        bad = true;
        return false;
      }
      prevx = x;
      v = make_int2(x, lo);
      if (hi > lo)
        upper = true;
      else
        ++t;
    } else {
      v = make_int2(x, __builtin_amdgcn_readlane(vhi, lane));
      upper = false;
      ++t;
    }
    return true;
  }
};

template <bool SMALL>
__device__ void melkman_walk(const int32_t *__restrict__ cx, const int32_t *__restrict__ clo,
                             const int32_t *__restrict__ chi, int32_t chain_cap, int32_t k,
                             int32_t *__restrict__ hx, int32_t *__restrict__ hy, int32_t *__restrict__ info,
                             int2 *D) {
  const bool lead = threadIdx.x == 0;  // every lane computes; lane 0 stores
  ChainWalk W{cx, clo, chi, k, 0, -64, 0, 0, 0, 0, false, false};
  int2 a, b, c;
  int32_t h = 0;
  if (!W.next(a)) {
    h = 0;
  } else if (!W.next(b)) {
    if (lead) {
      hx[0] = a.x;
      hy[0] = a.y;
    }
    h = 1;
  } else {
    // points collinear with a and b move b along the line (the walk is
    // x-monotone, so the newest point is the far end)
    bool more;
    while ((more = W.next(c)) && melk_orient<SMALL>(a, b, c) == 0) b = c;
    if (!more) {
      if (lead) {
        hx[0] = a.x;
        hy[0] = a.y;
        hx[1] = b.x;
        hy[1] = b.y;
      }
      h = 2;
    } else {
      // the deque D[bot..top], counter-clockwise from bottom to top, with
      // the newest hull point at both ends; the sequence has at most
      // 2 chain_cap points, so bot starts there and never goes below 0.
      // T0 = D[top], T1 = D[top-1], B0 = D[bot], B1 = D[bot+1] are kept in
      // registers; memory is read only when a pop exposes an older entry.
      int64_t bot = 2 * (int64_t)chain_cap, top = bot + 3;
      const bool ccw = melk_orient<SMALL>(a, b, c) > 0;
      int2 B0 = c, B1 = ccw ? a : b, T1 = ccw ? b : a, T0 = c;
      if (lead) {
        D[bot] = B0;
        D[bot + 1] = B1;
        D[bot + 2] = T1;
        D[top] = T0;
      }
      __syncthreads();
      // The rest of the walk.  The chain comes in increasing x, so nearly
      // every point lies outside the hull so far and takes the deque update;
      // the skip test rarely fires.
      int2 v;
      while (W.next(v)) {
        if (melk_orient<SMALL>(T1, T0, v) > 0 && melk_orient<SMALL>(B0, B1, v) > 0) continue;
        while (top - bot >= 2 && melk_orient<SMALL>(T1, T0, v) <= 0) {
          --top;
          T0 = T1;
          T1 = D[top - 1];
        }
        T1 = T0;
        T0 = v;
        ++top;
        if (lead) D[top] = v;
        __syncthreads();
        // the bottom's cached pair may have been the entries just popped
        // from the top when the deque was short: reload it from memory
        if (top - bot <= 4) {
          B0 = D[bot];
          B1 = D[bot + 1];
        }
        while (top - bot >= 2 && melk_orient<SMALL>(B0, B1, v) <= 0) {
          ++bot;
          B0 = B1;
          B1 = D[bot + 1];
        }
        B1 = B0;
        B0 = v;
        --bot;
        if (lead) D[bot] = v;
        __syncthreads();
        if (top - bot <= 4) {
          T0 = D[top];
          T1 = D[top - 1];
        }
      }
      if (!W.bad) {
        // the hull is D[bot..top-1], convex; a vertex with a straight angle
        // has both neighbours on its line, so one pass against the original
        // neighbours removes exactly those.  Then start at the lexicographic
        // minimum of what is kept.
        const int64_t m = top - bot;
        const int2 *H = D + bot;
        int64_t first = -1;
        for (int64_t i = 0; i < m; ++i) {
          const int2 cur = H[i];
          if (melk_orient<SMALL>(H[(i + m - 1) % m], cur, H[(i + 1) % m]) == 0) continue;
          if (first < 0 || cur.x < H[first].x || (cur.x == H[first].x && cur.y < H[first].y)) first = i;
        }
        if (first < 0) first = 0;  // unreachable: a non-degenerate hull has corners
        for (int64_t j = 0; j < m; ++j) {
          const int64_t i = (first + j) % m;
          const int2 cur = H[i];
          if (melk_orient<SMALL>(H[(i + m - 1) % m], cur, H[(i + 1) % m]) == 0) continue;
          if (lead) {
            hx[h] = cur.x;
            hy[h] = cur.y;
          }
          ++h;
        }
      }
    }
  }
  if (lead) {
    if (W.bad) info[HP_INFO_STATUS] = HP_EINVAL;
    info[HP_INFO_H] = W.bad ? 0 : h;
  }
}

__global__ __launch_bounds__(64) void k_melkman(const int32_t *__restrict__ cx, const int32_t *__restrict__ clo,
                                                const int32_t *__restrict__ chi, int32_t chain_cap,
                                                int32_t *__restrict__ hx, int32_t *__restrict__ hy,
                                                int32_t *__restrict__ info, int2 *__restrict__ gdeque,
                                                int32_t use_lds) {
  extern __shared__ int2 s_deque[];
  int2 *D = use_lds ? s_deque : gdeque;
  const int32_t k = info[HP_INFO_K];
  __syncthreads();
  if (k < 0 || k > chain_cap) {
    if (threadIdx.x == 0) {
      info[HP_INFO_STATUS] = HP_ECAPACITY;
      info[HP_INFO_H] = 0;
    }
    return;
  }
  // one pass of the wave over the chain: is it well formed (x strictly
  // increasing, lo <= hi), and does every coordinate lie in [0, 2^15), where
  // the 32-bit orientation applies
  bool small = true, bad = false;
  for (int32_t t = threadIdx.x; t < k; t += 64) {
    const int32_t x = cx[t], lo = clo[t], hi = chi[t];
    small = small && (unsigned)x < 32768u && (unsigned)lo < 32768u && (unsigned)hi < 32768u;
    bad = bad || hi < lo || (t > 0 && cx[t - 1] >= x);
  }
  small = __ballot(!small) == 0;
  if (__ballot(bad) != 0) {
    if (threadIdx.x == 0) {
      info[HP_INFO_STATUS] = HP_EINVAL;
      info[HP_INFO_H] = 0;
    }
    return;
  }
  if (small)
    melkman_walk<true>(cx, clo, chi, chain_cap, k, hx, hy, info, D);
  else
    melkman_walk<false>(cx, clo, chi, chain_cap, k, hx, hy, info, D);
}

static int64_t melkman_deque_entries(int32_t chain_cap) { return 4 * (int64_t)chain_cap + 4; }

static bool melkman_in_lds(int32_t chain_cap) {
  return melkman_deque_entries(chain_cap) * (int64_t)sizeof(int2) <= device_info().lds_bytes;
}

}  // namespace hp

using namespace hp;

extern "C" int hp_hull_melkman_workspace_bytes(int32_t chain_cap, size_t *bytes) {
  if (chain_cap < 0) return set_error(HP_EINVAL, "chain_cap < 0");
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  *bytes = (size_t)melkman_deque_entries(chain_cap) * sizeof(int2);
  return HP_OK;
}

extern "C" int hp_hull_melkman(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t chain_cap,
                               int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                               size_t ws_bytes, void *stream) {
  if (chain_cap < 0) return set_error(HP_EINVAL, "chain_cap < 0");
  if (chain_cap > 0 && (!cx || !clo || !chi)) return set_error(HP_EINVAL, "chain arrays must not be NULL");
  if (!hx || !hy || !info) return set_error(HP_EINVAL, "NULL output or info");
  if ((int64_t)hull_cap < 2 * (int64_t)chain_cap || hull_cap < 2)
    return set_error(HP_ECAPACITY, "hull_cap %d < max(2, 2 chain_cap)", hull_cap);
  const bool lds = melkman_in_lds(chain_cap);
  if (!lds && (!ws || ws_bytes < (size_t)melkman_deque_entries(chain_cap) * sizeof(int2)))
    return set_error(HP_ECAPACITY, "workspace too small for the deque");
  const size_t shmem = lds ? (size_t)melkman_deque_entries(chain_cap) * sizeof(int2) : 0;
  hipLaunchKernelGGL(k_melkman, dim3(1), dim3(64), shmem, (hipStream_t)stream, cx, clo, chi, chain_cap, hx, hy,
                     info, static_cast<int2 *>(ws), (int32_t)lds);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_melkman launch: %s", hipGetErrorString(e));
  return HP_OK;
}
