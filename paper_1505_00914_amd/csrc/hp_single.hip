// hp_single.hip -- single-cloud kernels and entry points of libhullprep.
#include <climits>
#include <cstring>

#include "hp_host.h"
#include "hp_kernels.h"

namespace hp {

// ---------------------------------------------------------------------------
// L initialisation and control words
// ---------------------------------------------------------------------------
__global__ void k_init(int32_t *ctl, int32_t *tree_ctr, int32_t nodes, int32_t *info,
                       int32_t info_mode, int2 *L, int32_t p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < kCtlWords; j += stride) ctl[j] = 0;
  for (int64_t j = i; j < nodes; j += stride) tree_ctr[j] = 0;
  if (i == 0 && info) {
    if (info_mode == 0) {  // full run: every field
      info[HP_INFO_STATUS] = HP_OK;
      info[HP_INFO_K] = 0;
      info[HP_INFO_S] = 0;
      info[HP_INFO_H] = 0;
    } else {               // hull only: k is an input, status is kept
      info[HP_INFO_H] = 0;
    }
  }
  if (L)
    for (int64_t c = i; c < p; c += stride) L[c] = make_int2(p + 1, -1);
}

// ---------------------------------------------------------------------------
// Algorithm 1.  Points are read once, 16 bytes (two points) per lane per
// load, VPT loads in flight per lane; consecutive lanes read consecutive
// vectors and consecutive workgroups consecutive chunks.
// ---------------------------------------------------------------------------
template <int BLOCK, int VPT, bool LDS>
__device__ __forceinline__ void stream_points(const int32_t *__restrict__ pts, int64_t n, int p,
                                              int2 *L, int64_t wg, int64_t nwg, bool &bad) {
  // pts is 8-byte aligned (checked on the host); peel one point if the
  // vector body would otherwise start on an 8-byte boundary.
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int64_t tail = head + 2 * nv;  // index of the odd last point, if any
  if (wg == 0 && threadIdx.x == 0) {
    if (head) {
      if (LDS) fold_point_lds(L, p, pts[0], pts[1], bad);
      else fold_point_global(L, p, pts[0], pts[1], bad);
    }
    if (tail < n) {
      if (LDS) fold_point_lds(L, p, pts[2 * tail], pts[2 * tail + 1], bad);
      else fold_point_global(L, p, pts[2 * tail], pts[2 * tail + 1], bad);
    }
  }
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  constexpr int64_t chunk = (int64_t)BLOCK * VPT;
  for (int64_t t0 = wg * chunk; t0 < nv; t0 += nwg * chunk) {
    if (t0 + chunk <= nv) {
      int4 q[VPT];
#pragma unroll
      for (int u = 0; u < VPT; ++u) q[u] = v[t0 + u * BLOCK + threadIdx.x];
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        if (LDS) {
          fold_point_lds(L, p, q[u].x, q[u].y, bad);
          fold_point_lds(L, p, q[u].z, q[u].w, bad);
        } else {
          fold_point_global(L, p, q[u].x, q[u].y, bad);
          fold_point_global(L, p, q[u].z, q[u].w, bad);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int64_t idx = t0 + u * BLOCK + threadIdx.x;
        if (idx < nv) {
          const int4 q = v[idx];
          if (LDS) {
            fold_point_lds(L, p, q.x, q.y, bad);
            fold_point_lds(L, p, q.z, q.w, bad);
          } else {
            fold_point_global(L, p, q.x, q.y, bad);
            fold_point_global(L, p, q.z, q.w, bad);
          }
        }
      }
    }
  }
}

// Workgroup-private L in LDS; written out as one partial L per workgroup.
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_reduce_lds(const int32_t *__restrict__ pts, int64_t n,
                                                      int32_t p, int2 *__restrict__ part,
                                                      int32_t *__restrict__ ctl) {
  extern __shared__ int2 sL[];
  for (int c = threadIdx.x; c < p; c += BLOCK) sL[c] = make_int2(p + 1, -1);
  __syncthreads();
  bool bad = false;
  stream_points<BLOCK, VPT, true>(pts, n, p, sL, blockIdx.x, gridDim.x, bad);
  __syncthreads();
  int2 *out = part + (size_t)blockIdx.x * (size_t)p;
  for (int c = threadIdx.x; c < p; c += BLOCK) out[c] = sL[c];
  if (bad) atomicOr(&ctl[kCtlErr], kErrRange);
}

// One L in device memory, updated with filtered device-scope atomics.
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_reduce_global(const int32_t *__restrict__ pts, int64_t n,
                                                         int32_t p, int2 *L,
                                                         int32_t *__restrict__ ctl) {
  bool bad = false;
  stream_points<BLOCK, VPT, false>(pts, n, p, L, blockIdx.x, gridDim.x, bad);
  if (bad) atomicOr(&ctl[kCtlErr], kErrRange);
}

// ---------------------------------------------------------------------------
// Finish: one workgroup of 256 threads per slab of 64 positions.
// ---------------------------------------------------------------------------
constexpr int kFinBlock = 256;
constexpr int kStage = 4096;  // candidates per side staged in LDS for a merge

struct FinishShared {
  int2 red[4][kSlab];          // partial-merge scratch
  int2 pt[2][kSlab];           // slab points: side 0 (x, lo), side 1 (x, -hi)
  int2 lvl0[2][kSlab];         // tile hulls
  int2 stage[kStage];          // children of a tree node
  int cs[kFanIn], cc[kFanIn];
  int l1cs[2][4], l1cc[2][4];
  int tmp[kFinBlock / kWave + 1];
  int slab_cnt[2];
  int flag;
  int scan_carry;
};

// Exclusive scan of n ints in place (by one workgroup); returns the total.
__device__ int block_exclusive_scan(int32_t *a, int32_t n, int *s_tmp, int *s_carry) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += kFinBlock) {
    const int i = base + tid;
    const int v = i < n ? a[i] : 0;
    // inclusive scan inside the wave
    int incl = v;
    const int lane = tid & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    const int w = tid / kWave;
    if (lane == kWave - 1) s_tmp[w] = incl;
    __syncthreads();
    int off = *s_carry, all = 0;
    for (int j = 0; j < kFinBlock / kWave; ++j) {
      if (j < w) off += s_tmp[j];
      all += s_tmp[j];
    }
    if (i < n) a[i] = off + incl - v;
    __syncthreads();
    if (tid == 0) *s_carry += all;
    __syncthreads();
  }
  return *s_carry;
}

// The final hull from the lower hull of (x, lo) and the lower hull of
// (x, -hi) (both left to right): lower chain, then the upper chain walked
// back, without the shared end points.  Returns h.
__device__ int assemble_hull(const int2 *low, int nl, const int2 *upn, int nu, int32_t *hx,
                             int32_t *hy, int32_t cap, bool &overflow) {
  if (nl == 0 || nu == 0) return 0;
  const int2 l0 = low[0], la = low[nl - 1];
  const int2 u0 = make_int2(upn[0].x, -upn[0].y), ub = make_int2(upn[nu - 1].x, -upn[nu - 1].y);
  const bool dropL = (la.x == ub.x && la.y == ub.y);
  const bool dropU = (u0.x == l0.x && u0.y == l0.y);
  const bool single = (nl == 1 && nu == 1 && dropL);
  const int cntL = nl - (dropL ? 1 : 0);
  const int cntU = nu - (dropU ? 1 : 0);
  const int h = single ? 1 : cntL + cntU;
  if (h > cap) {
    overflow = true;
    return h;
  }
  if (single) {
    if (threadIdx.x == 0) { hx[0] = l0.x; hy[0] = l0.y; }
    return 1;
  }
  for (int i = threadIdx.x; i < cntL; i += blockDim.x) { hx[i] = low[i].x; hy[i] = low[i].y; }
  for (int j = threadIdx.x; j < cntU; j += blockDim.x) {
    const int2 u = upn[nu - 1 - j];
    hx[cntL + j] = u.x;
    hy[cntL + j] = -u.y;
  }
  return h;
}

// Merge the children of tree node (lev, j) for both sides; writes the node's
// hulls into cand buffer lev&1 (or, for the root, assembles the hull).
__device__ void tree_merge_node(const FinishArgs &A, FinishShared &S, int lev, int j) {
  const TreeShape &T = A.tree;
  const int c0 = j * kFanIn;
  const int nch = min(kFanIn, T.size[lev - 1] - c0);
  const int64_t P = A.positions;
  const bool root = (lev == T.nlev);
  int nkeep[2];
  for (int side = 0; side < 2; ++side) {
    const int2 *src = A.cand + ((size_t)((lev - 1) & 1) * 2 + side) * (size_t)P;
    int2 *dst = A.cand + ((size_t)(lev & 1) * 2 + side) * (size_t)P;
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int t = 0; t < nch; ++t) {
        const int child = c0 + t;
        S.cc[t] = A.ccount[side * T.nodes + T.base[lev - 1] + child];
        S.cs[t] = acc;
        acc += S.cc[t];
      }
      S.flag = acc;
    }
    __syncthreads();
    const int total = S.flag;
    const int2 *data;
    if (total <= kStage) {
      // stage the children contiguously in LDS
      for (int t = 0; t < nch; ++t) {
        const int2 *cp = src + (size_t)(c0 + t) * (size_t)T.span[lev - 1];
        for (int r = threadIdx.x; r < S.cc[t]; r += kFinBlock) S.stage[S.cs[t] + r] = cp[r];
      }
      data = S.stage;
    } else {
      // too many to stage: point the children at device memory
      __syncthreads();
      if (threadIdx.x == 0)
        for (int t = 0; t < nch; ++t) S.cs[t] = (int)((size_t)(c0 + t) * (size_t)T.span[lev - 1]);
      data = src;
    }
    __syncthreads();
    int2 *out = dst + (size_t)j * (size_t)T.span[lev];
    nkeep[side] = merge_lower<kFinBlock>(data, S.cs, S.cc, nch, out, S.tmp);
    if (threadIdx.x == 0) A.ccount[side * T.nodes + T.base[lev] + j] = nkeep[side];
    __syncthreads();
  }
  if (root) {
    __threadfence_block();
    __syncthreads();
    const int2 *low = A.cand + ((size_t)(lev & 1) * 2 + 0) * (size_t)P;
    const int2 *upn = A.cand + ((size_t)(lev & 1) * 2 + 1) * (size_t)P;
    bool overflow = false;
    const int h = assemble_hull(low, nkeep[0], upn, nkeep[1], A.hx, A.hy, A.hull_cap, overflow);
    if (threadIdx.x == 0) {
      A.info[HP_INFO_H] = overflow ? 0 : h;
      if (overflow) atomicMin(&A.info[HP_INFO_STATUS], HP_ECAPACITY);
    }
  }
}

__device__ bool last_arrival(int32_t *ctr, int expected, FinishShared &S) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int old = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    S.flag = (old == expected - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = S.flag != 0;
  if (last) __threadfence();
  return last;
}

template <int FROM_CHAIN>
__global__ __launch_bounds__(kFinBlock) void k_finish(FinishArgs A) {
  __shared__ FinishShared S;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int grp = tid / kWave;
  const int slab = blockIdx.x;
  const int64_t pos = (int64_t)slab * kSlab + lane;
  const bool inside = pos < A.positions;

  // ---- the slab's points --------------------------------------------------
  int x = 0, lo = 0, hi = -1;
  bool valid = false;
  if (!FROM_CHAIN) {
    int mlo = INT_MAX, mhi = INT_MIN;
    if (inside) {
      const int2 *src = A.part + pos;
      const int G = A.G;
      int g = grp;
      for (; g + 12 < G; g += 16) {
        const int2 a = src[(size_t)g * A.p], b = src[(size_t)(g + 4) * A.p];
        const int2 c = src[(size_t)(g + 8) * A.p], d = src[(size_t)(g + 12) * A.p];
        mlo = min(mlo, min(min(a.x, b.x), min(c.x, d.x)));
        mhi = max(mhi, max(max(a.y, b.y), max(c.y, d.y)));
      }
      for (; g < G; g += 4) {
        const int2 a = src[(size_t)g * A.p];
        mlo = min(mlo, a.x);
        mhi = max(mhi, a.y);
      }
    }
    S.red[grp][lane] = make_int2(mlo, mhi);
    __syncthreads();
    if (grp == 0) {
      for (int k = 1; k < 4; ++k) {
        mlo = min(mlo, S.red[k][lane].x);
        mhi = max(mhi, S.red[k][lane].y);
      }
      lo = mlo;
      hi = mhi;
      x = (int)pos + 1;
      valid = inside && lo <= hi;
      if (inside) {
        A.Lm[pos] = make_int2(lo, hi);
        if (A.lo) { A.lo[pos] = lo; A.hi[pos] = hi; }
      }
    }
  } else {
    if (grp == 0) {
      const int k = A.info[HP_INFO_K];
      valid = inside && pos < k;
      if (valid) {
        x = A.cx[pos];
        lo = A.clo[pos];
        hi = A.chi[pos];
      }
    }
  }

  // ---- M word and counts (wave 0) ------------------------------------------
  if (grp == 0) {
    const unsigned long long vm = __ballot(valid);
    const unsigned long long sm = __ballot(valid && lo < hi);
    if (!FROM_CHAIN && lane == 0) {
      if (A.mask) A.mask[slab] = vm;
      A.slab_k[slab] = __popcll(vm);
      A.slab_s[slab] = __popcll(vm) + __popcll(sm);
    }
    if (A.do_hull) {
      S.pt[0][lane] = make_int2(x, lo);
      S.pt[1][lane] = make_int2(x, -hi);
    }
  }
  __syncthreads();

  // ---- hull level 0 (tiles of 16) and level 1 (the slab), wave 0 -----------
  if (A.do_hull) {
    if (grp == 0) {
      const unsigned long long vm = __ballot(valid);
      const int t0 = lane & ~(kTile - 1);
      for (int side = 0; side < 2; ++side) {
        const int2 v = S.pt[side][lane];
        bool keep = false;
        if (valid) {
          bool hasL = false, hasR = false;
          int2 uL = v, wR = v;
          for (int jj = t0; jj < lane; ++jj) {
            if (!((vm >> jj) & 1ull)) continue;
            const int2 u = S.pt[side][jj];
            if (!hasL || steeper_left(u, uL, v)) { uL = u; hasL = true; }
          }
          for (int jj = lane + 1; jj < t0 + kTile; ++jj) {
            if (!((vm >> jj) & 1ull)) continue;
            const int2 w = S.pt[side][jj];
            if (!hasR || flatter_right(w, wR, v)) { wR = w; hasR = true; }
          }
          keep = !hasL || !hasR || cross3(uL, v, wR) > 0;
        }
        const unsigned long long km = __ballot(keep);
        const unsigned tb = (unsigned)((km >> t0) & 0xFFFFull);
        const int r = __popc(tb & ((1u << (lane - t0)) - 1u));
        if (keep) S.lvl0[side][t0 + r] = v;
        if (lane == t0) {
          S.l1cs[side][lane / kTile] = t0;
          S.l1cc[side][lane / kTile] = __popc(tb);
        }
      }
    }
    __syncthreads();
    if (grp == 0) {
      for (int side = 0; side < 2; ++side) {
        const int T = lane / kTile, r = lane % kTile;
        bool keep = false;
        int2 v = make_int2(0, 0);
        if (r < S.l1cc[side][T]) {
          v = S.lvl0[side][lane];
          keep = lower_survives(S.lvl0[side], S.l1cs[side], S.l1cc[side], 4, T, r);
        }
        int tot;
        const int rk = wave_rank(keep, &tot);
        if (A.tree.nlev == 1) {
          if (keep) S.stage[side * kSlab + rk] = v;   // single slab: keep in LDS
        } else {
          int2 *dst = A.cand + ((size_t)1 * 2 + side) * (size_t)A.positions + (size_t)slab * kSlab;
          if (keep) dst[rk] = v;
        }
        if (lane == 0) {
          A.ccount[side * A.tree.nodes + slab] = tot;
          S.slab_cnt[side] = tot;
        }
      }
    }
    __syncthreads();
    if (A.tree.nlev == 1) {
      bool overflow = false;
      const int h = assemble_hull(S.stage, S.slab_cnt[0], S.stage + kSlab, S.slab_cnt[1], A.hx,
                                  A.hy, A.hull_cap, overflow);
      if (tid == 0) {
        A.info[HP_INFO_H] = overflow ? 0 : h;
        if (overflow) atomicMin(&A.info[HP_INFO_STATUS], HP_ECAPACITY);
      }
    }
  }

  // ---- last slab: scan the slab counts (preconditioner only) ---------------
  if (!FROM_CHAIN) {
    if (last_arrival(&A.ctl[kCtlSlabsDone], gridDim.x, S)) {
      const int nslab = gridDim.x;
      // slab_off = exclusive scan of slab_k; k and s totals
      for (int i = tid; i < nslab; i += kFinBlock) A.slab_off[i] = A.slab_k[i];
      __syncthreads();
      const int k = block_exclusive_scan(A.slab_off, nslab, S.tmp, &S.scan_carry);
      int s_part = 0;
      for (int i = tid; i < nslab; i += kFinBlock) s_part += A.slab_s[i];
      // block sum of s
      for (int d = kWave / 2; d > 0; d >>= 1) s_part += __shfl_down(s_part, d, kWave);
      __syncthreads();
      if (lane == 0) S.tmp[grp] = s_part;
      __syncthreads();
      if (tid == 0) {
        int s = 0;
        for (int w = 0; w < kFinBlock / kWave; ++w) s += S.tmp[w];
        A.info[HP_INFO_K] = k;
        A.info[HP_INFO_S] = s;
        const int err = __hip_atomic_load(&A.ctl[kCtlErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (err & kErrRange) atomicMin(&A.info[HP_INFO_STATUS], HP_ERANGE);
      }
    }
  }

  // ---- hull tree above the slabs: the last child merges its parent ---------
  if (A.do_hull && A.tree.nlev > 1) {
    int lev = 1, j = slab;
    while (lev < A.tree.nlev) {
      const int parent = j / kFanIn;
      const int nch = min(kFanIn, A.tree.size[lev] - parent * kFanIn);
      if (!last_arrival(&A.tree_ctr[A.tree.base[lev + 1] + parent], nch, S)) break;
      ++lev;
      j = parent;
      tree_merge_node(A, S, lev, j);
    }
  }
}

// Chain write: one wave per slab, at the scanned offset (Lemma 1 order).
__global__ __launch_bounds__(256) void k_chain(const int2 *__restrict__ Lm, int32_t p,
                                               const int32_t *__restrict__ slab_off, int32_t nslab,
                                               int32_t *cx, int32_t *clo, int32_t *chi,
                                               int32_t cap, int32_t *info) {
  const int lane = threadIdx.x & (kWave - 1);
  const int slab = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (slab >= nslab) return;
  const int64_t pos = (int64_t)slab * kSlab + lane;
  int2 L = make_int2(1, 0);
  const bool inside = pos < p;
  if (inside) L = Lm[pos];
  const bool valid = inside && L.x <= L.y;
  int tot;
  const int r = wave_rank(valid, &tot);
  const int off = slab_off[slab] + r;
  if (valid) {
    if (off < cap) {
      cx[off] = (int)pos + 1;
      clo[off] = L.x;
      chi[off] = L.y;
    } else {
      atomicMin(&info[HP_INFO_STATUS], HP_ECAPACITY);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static TreeShape make_tree(int64_t positions) {
  TreeShape T;
  memset(&T, 0, sizeof(T));
  const int64_t P = positions < 1 ? 1 : positions;
  T.size[1] = (int32_t)((P + kSlab - 1) / kSlab);
  T.span[1] = kSlab;
  T.base[1] = 0;
  int l = 1;
  while (T.size[l] > 1 && l < kMaxLevels) {
    T.size[l + 1] = (T.size[l] + kFanIn - 1) / kFanIn;
    T.base[l + 1] = T.base[l] + T.size[l];
    const int64_t sp = (int64_t)T.span[l] * kFanIn;
    T.span[l + 1] = (int32_t)(sp > INT32_MAX ? INT32_MAX : sp);
    ++l;
  }
  T.nlev = l;
  T.nodes = T.base[l] + T.size[l];
  return T;
}

struct Layout {
  size_t ctl, tree, slab_k, slab_s, slab_off, Lm, part, cand, ccount, total;
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

static Layout make_layout(int64_t positions, int32_t p, int64_t part_pairs, const TreeShape &T) {
  Layout Y;
  size_t o = 0;
  Y.ctl = o;      o = align_up(o + sizeof(int32_t) * kCtlWords);
  Y.tree = o;     o = align_up(o + sizeof(int32_t) * (size_t)T.nodes);
  Y.slab_k = o;   o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.slab_s = o;   o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.slab_off = o; o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.Lm = o;       o = align_up(o + sizeof(int2) * (size_t)(p > 0 ? p : 0));
  Y.part = o;     o = align_up(o + sizeof(int2) * (size_t)part_pairs);
  Y.cand = o;     o = align_up(o + sizeof(int2) * 4 * (size_t)positions);
  Y.ccount = o;   o = align_up(o + sizeof(int32_t) * 2 * (size_t)T.nodes);
  Y.total = o;
  return Y;
}

static int64_t lds_grid_max();

struct Plan1 {
  int strategy;
  int block, vpt, G;
};

static Plan1 choose(int64_t n, int32_t p) {
  const DeviceInfo &D = device_info();
  Plan1 P;
  int s = forced_strategy();
  if (s == HP_STRATEGY_AUTO) s = tuned_strategy(n, p);
  if (s == HP_STRATEGY_LDS && (int64_t)p > D.lds_max_p) s = HP_STRATEGY_GLOBAL;
  P.strategy = s;
  P.block = 1024;
  P.vpt = 4;
  if (s == HP_STRATEGY_LDS) {
    // enough points per workgroup that the partial L (8p bytes) stays small
    // next to the points it summarises, but never fewer groups than needed
    // to keep every CU streaming when n is large
    const int64_t per_wg_min = 8 * (int64_t)p;
    int64_t G = per_wg_min > 0 ? n / per_wg_min : 1;
    const int64_t gmax = (int64_t)D.cus * D.lds_groups_per_cu(p);
    if (G > gmax) G = gmax;
    if (G < 1) G = 1;
    P.G = (int)G;
  } else {
    const int64_t vecs = (n + 1) / 2;
    int64_t G = (vecs + (int64_t)P.block * P.vpt - 1) / ((int64_t)P.block * P.vpt);
    const int64_t gmax = (int64_t)D.cus * 2;
    if (G > gmax) G = gmax;
    if (G < 1) G = 1;
    P.G = (int)G;
  }
  tune_override(n, p, &P.block, &P.vpt, &P.G);
  if (P.strategy == HP_STRATEGY_LDS && P.G > lds_grid_max()) P.G = (int)lds_grid_max();
  if (P.G < 1) P.G = 1;
  return P;
}

static int64_t part_pairs_for(const Plan1 &P, int32_t p) {
  return P.strategy == HP_STRATEGY_LDS ? (int64_t)P.G * p : (int64_t)p;
}

// Largest grid the LDS strategy may use (also bounds tuned overrides).
static int64_t lds_grid_max() { return (int64_t)device_info().cus * 4; }

static size_t ws_bytes_for(int64_t n, int32_t p) {
  // sized for the largest partial-L array any strategy or override may use,
  // so that a later strategy change still fits the same workspace
  (void)n;
  const TreeShape T = make_tree(p);
  const int64_t part = (int64_t)p <= device_info().lds_max_p ? lds_grid_max() * p : (int64_t)p;
  return make_layout(p, p, part, T).total;
}

template <int BLOCK, int VPT>
static hipError_t launch_reduce(const Plan1 &P, const int32_t *pts, int64_t n, int32_t p, int2 *part,
                                int32_t *ctl, hipStream_t s) {
  if (P.strategy == HP_STRATEGY_LDS) {
    const size_t lds = sizeof(int2) * (size_t)p;
    static bool attr_set = false;
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute((const void *)k_reduce_lds<BLOCK, VPT>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               device_info().lds_bytes);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL((k_reduce_lds<BLOCK, VPT>), dim3(P.G), dim3(BLOCK), lds, s, pts, n, p, part, ctl);
  } else {
    hipLaunchKernelGGL((k_reduce_global<BLOCK, VPT>), dim3(P.G), dim3(BLOCK), 0, s, pts, n, p, part,
                       ctl);
  }
  return hipGetLastError();
}

static hipError_t dispatch_reduce(const Plan1 &P, const int32_t *pts, int64_t n, int32_t p, int2 *part,
                                  int32_t *ctl, hipStream_t s) {
#define HP_CASE(B, V) \
  if (P.block == B && P.vpt == V) return launch_reduce<B, V>(P, pts, n, p, part, ctl, s);
  HP_CASE(1024, 4)
  HP_CASE(1024, 2)
  HP_CASE(1024, 8)
  HP_CASE(512, 2)
  HP_CASE(512, 4)
  HP_CASE(512, 8)
  HP_CASE(256, 2)
  HP_CASE(256, 4)
  HP_CASE(256, 8)
#undef HP_CASE
  return hipErrorInvalidValue;
}

// Enqueue the whole single-cloud sequence.  Shared by hp_precondition,
// hp_run and the per-cloud baseline of the batched form.
int run_single(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi, uint64_t *mask,
               int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx, int32_t *hy,
               int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes, hipStream_t s,
               bool do_hull) {
  const Plan1 P = choose(n, p);
  const TreeShape T = make_tree(p);
  const Layout Y = make_layout(p, p, part_pairs_for(P, p), T);
  if (ws_bytes < Y.total) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, Y.total);
  char *w = static_cast<char *>(ws);
  int32_t *ctl = reinterpret_cast<int32_t *>(w + Y.ctl);
  int32_t *tree = reinterpret_cast<int32_t *>(w + Y.tree);
  int2 *part = reinterpret_cast<int2 *>(w + Y.part);

  const int ninit = (int)std::min<int64_t>(1024, std::max<int64_t>(1, ((int64_t)std::max<int64_t>(p, T.nodes) + 255) / 256));
  hipLaunchKernelGGL(k_init, dim3(ninit), dim3(256), 0, s, ctl, tree, T.nodes, info, 0,
                     P.strategy == HP_STRATEGY_GLOBAL ? part : nullptr, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_init launch: %s", hipGetErrorString(e));
  e = dispatch_reduce(P, pts, n, p, part, ctl, s);
  if (e != hipSuccess) return set_error(HP_EDEVICE, "reduce launch: %s", hipGetErrorString(e));

  FinishArgs A;
  memset(&A, 0, sizeof(A));
  A.part = part;
  A.G = P.strategy == HP_STRATEGY_LDS ? P.G : 1;
  A.positions = p;
  A.p = p;
  A.Lm = reinterpret_cast<int2 *>(w + Y.Lm);
  A.lo = lo;
  A.hi = hi;
  A.mask = mask;
  A.slab_k = reinterpret_cast<int32_t *>(w + Y.slab_k);
  A.slab_s = reinterpret_cast<int32_t *>(w + Y.slab_s);
  A.slab_off = reinterpret_cast<int32_t *>(w + Y.slab_off);
  A.do_hull = do_hull ? 1 : 0;
  A.cand = reinterpret_cast<int2 *>(w + Y.cand);
  A.ccount = reinterpret_cast<int32_t *>(w + Y.ccount);
  A.tree_ctr = tree;
  A.tree = T;
  A.hx = hx;
  A.hy = hy;
  A.hull_cap = hull_cap;
  A.ctl = ctl;
  A.info = info;
  hipLaunchKernelGGL(k_finish<0>, dim3(T.size[1]), dim3(kFinBlock), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_finish launch: %s", hipGetErrorString(e));
  const int nslab = T.size[1];
  hipLaunchKernelGGL(k_chain, dim3((nslab + 3) / 4), dim3(256), 0, s, A.Lm, p, A.slab_off, nslab, cx,
                     clo, chi, chain_cap, info);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_chain launch: %s", hipGetErrorString(e));
  return HP_OK;
}

size_t single_ws_bytes(int64_t n, int32_t p) { return ws_bytes_for(n, p); }

static int check_common(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi,
                        int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *info,
                        void *ws) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (n > 0 && !pts) return set_error(HP_EINVAL, "pts is NULL");
  if (pts && ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is not 8-byte aligned");
  if ((lo == nullptr) != (hi == nullptr)) return set_error(HP_EINVAL, "lo and hi must both be set or both NULL");
  if (!cx || !clo || !chi) return set_error(HP_EINVAL, "chain arrays must not be NULL");
  if (!info) return set_error(HP_EINVAL, "info is NULL");
  if (!ws) return set_error(HP_EINVAL, "workspace is NULL");
  const int64_t need = std::min<int64_t>(n, p);
  if ((int64_t)chain_cap < need)
    return set_error(HP_ECAPACITY, "chain_cap %d < min(n, p) = %lld", chain_cap, (long long)need);
  return HP_OK;
}

}  // namespace hp

using namespace hp;

extern "C" int hp_workspace_bytes(int64_t n, int32_t p, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (p < 1 || p > HP_P_MAX || n < 0) return set_error(HP_EINVAL, "bad n or p");
  *bytes = ws_bytes_for(n, p);
  return HP_OK;
}

extern "C" int hp_precondition(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi,
                               uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                               int32_t chain_cap, int32_t *info, void *ws, size_t ws_bytes,
                               void *stream) {
  const int rc = check_common(pts, n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc != HP_OK) return rc;
  return run_single(pts, n, p, lo, hi, mask, cx, clo, chi, chain_cap, nullptr, nullptr, 0, info, ws,
                    ws_bytes, (hipStream_t)stream, false);
}

extern "C" int hp_run(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi,
                      uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                      int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                      size_t ws_bytes, void *stream) {
  const int rc = check_common(pts, n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc != HP_OK) return rc;
  if (!hx || !hy) return set_error(HP_EINVAL, "hull arrays must not be NULL");
  const int64_t need = 2 * std::min<int64_t>(n, p);
  if ((int64_t)hull_cap < need)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 min(n, p) = %lld", hull_cap, (long long)need);
  return run_single(pts, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, ws,
                    ws_bytes, (hipStream_t)stream, true);
}

extern "C" int hp_hull_workspace_bytes(int32_t chain_cap, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (chain_cap < 0) return set_error(HP_EINVAL, "chain_cap < 0");
  const TreeShape T = make_tree(chain_cap);
  *bytes = make_layout(chain_cap, 0, 0, T).total;
  return HP_OK;
}

extern "C" int hp_hull(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t chain_cap,
                       int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                       size_t ws_bytes, void *stream) {
  if (chain_cap < 0) return set_error(HP_EINVAL, "chain_cap < 0");
  if (chain_cap > 0 && (!cx || !clo || !chi)) return set_error(HP_EINVAL, "chain arrays must not be NULL");
  if (!hx || !hy || !info || !ws) return set_error(HP_EINVAL, "NULL output, info or workspace");
  if ((int64_t)hull_cap < 2 * (int64_t)chain_cap)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 chain_cap", hull_cap);
  const TreeShape T = make_tree(chain_cap);
  const Layout Y = make_layout(chain_cap, 0, 0, T);
  if (ws_bytes < Y.total) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, Y.total);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  int32_t *ctl = reinterpret_cast<int32_t *>(w + Y.ctl);
  int32_t *tree = reinterpret_cast<int32_t *>(w + Y.tree);
  hipLaunchKernelGGL(k_init, dim3(std::max(1, std::min(1024, (T.nodes + 255) / 256))), dim3(256), 0, s,
                     ctl, tree, T.nodes, info, 1, (int2 *)nullptr, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_init launch: %s", hipGetErrorString(e));
  FinishArgs A;
  memset(&A, 0, sizeof(A));
  A.cx = cx;
  A.clo = clo;
  A.chi = chi;
  A.positions = chain_cap;
  A.do_hull = 1;
  A.cand = reinterpret_cast<int2 *>(w + Y.cand);
  A.ccount = reinterpret_cast<int32_t *>(w + Y.ccount);
  A.tree_ctr = tree;
  A.tree = T;
  A.hx = hx;
  A.hy = hy;
  A.hull_cap = hull_cap;
  A.ctl = ctl;
  A.info = info;
  hipLaunchKernelGGL(k_finish<1>, dim3(T.size[1]), dim3(kFinBlock), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_finish launch: %s", hipGetErrorString(e));
  return HP_OK;
}
