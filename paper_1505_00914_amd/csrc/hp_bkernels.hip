// hp_bkernels.hip -- kernels of the batched form and their launchers.
//
// Every cloud of a batch is described by one BCloud in device memory; work
// lists map each workgroup (or lane) to a (cloud, local index) pair, so one
// launch per step covers all clouds of the batch.
#include "hp_args.h"
#include "hp_host.h"
#include "hp_output.h"
#include "hp_reduce.h"

namespace hp {

// Zero each cloud's info words; set the L of clouds that are reduced with
// atomics to the sentinel; reset the reduce work counter.
__global__ __launch_bounds__(256) void k_b_fill(const BCloud *cl, const uint8_t *needs_fill,
                                                int32_t *counter) {
  const int b = blockIdx.x;
  const BCloud &A = cl[b];
  if (b == 0 && threadIdx.x == 0) *counter = 0;
  if (threadIdx.x < HP_INFO_WORDS) A.info[threadIdx.x] = 0;
  if (needs_fill[b])
    for (int c = threadIdx.x; c < A.p; c += 256) A.Lm[c] = make_int2(A.p + 1, -1);
}

// Persistent reduce: workgroups take chunks from a shared counter until the
// list is exhausted (every wave leaves the loop once the counter passes the
// end).  Modes: 0 = the chunk is the whole cloud, LDS L stored as is;
// 1 = LDS L merged into the cloud's L by filtered atomics; 2 = filtered
// atomics straight into the cloud's L (sparse clouds).
template <int BLOCK, int VPT>
__global__ __launch_bounds__(BLOCK) void k_b_reduce(const BatchItem *__restrict__ items,
                                                    int32_t nitems, int32_t *counter,
                                                    const BCloud *cl) {
  extern __shared__ int2 sL[];
  __shared__ int s_item, s_bad;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      s_item = atomicAdd(counter, 1);
      s_bad = 0;
    }
    __syncthreads();
    const int it = s_item;
    if (it >= nitems) break;
    const BatchItem I = items[it];
    const BCloud &A = cl[I.cloud];
    const int p = A.p;
    int2 *L = A.Lm;
    const int32_t *src = I.pts;
    bool bad = false;
    if (I.mode == 2) {
      stream_points<BLOCK, VPT, false>(src, I.count, p, L, 0, 1, bad);
    } else {
      for (int c = threadIdx.x; c < p; c += BLOCK) sL[c] = make_int2(p + 1, -1);
      __syncthreads();
      stream_points<BLOCK, VPT, true>(src, I.count, p, sL, 0, 1, bad);
      __syncthreads();
      if (I.mode == 0) {
        for (int c = threadIdx.x; c < p; c += BLOCK) L[c] = sL[c];
      } else {
        for (int c = threadIdx.x; c < p; c += BLOCK) {
          const int2 mine = sL[c];
          if (mine.x > mine.y) continue;
          const int2 cur = load_coherent(&L[c]);
          if (mine.x < cur.x)
            __hip_atomic_fetch_min(&L[c].x, mine.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (mine.y > cur.y)
            __hip_atomic_fetch_max(&L[c].y, mine.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_bad) atomicMin(&A.info[HP_INFO_STATUS], HP_ERANGE);
  }
}

// ---------------------------------------------------------------------------
// Batched finish, shaped for throughput across many clouds: each lower hull
// is built by Andrew's monotone chain run by one lane over x-sorted input
// held in LDS, so a step costs one LDS read and there is no cross-lane
// traffic.
//   k_b_tiles   per tile of 64 slabs (= one level-2 node): each slab's M
//               word and counts, each slab's two hulls (a lane per slab and
//               side), then the node's two hulls from the slab hulls (a lane
//               per side)
//   k_b_nodes   per node above level 2 and side: the chain over its
//               children's hulls staged in LDS
//   k_b_root    per cloud: slab offsets (scan), k, s, the final vertex list
//   k_b_chain   per slab: the chain at the scanned offset (Lemma 1 order)
// ---------------------------------------------------------------------------
constexpr int kTileSlabs = kFanIn;               // slabs per tile
constexpr int kTileCols = kTileSlabs * kSlab;    // 4096 columns
constexpr int kRow = kSlab + 2;                  // LDS row stride (entries)
constexpr int kSideWords = kTileSlabs * kRow + 1;
constexpr int kNodeCap = 4096;                   // points a k_b_nodes wave stages

// A tile entry packs one point in tile-local coordinates: column in the
// tile (12 bits) above a 16-bit height, lo - 1 for the lower side and p - hi
// for the upper side.  Both are translations of (x, lo) and (x, -hi), so the
// turn tests are unchanged; every difference fits in 17 signed bits and the
// 24-bit products are exact.
struct TilePt {
  __device__ __forceinline__ int2 operator()(uint32_t e) const {
    return make_int2((int)(e >> 16), (int)(e & 0xFFFFu));
  }
};
struct PlainPt {
  __device__ __forceinline__ int2 operator()(int2 e) const { return e; }
};

// Lower chain of the points of E[0..nL) followed by those of R[0..nR), both
// already lower chains (strict left turns) and R entirely right of E; the
// result is left in E[0..), count returned.  The left chain stays the
// bottom of Andrew's stack, so only the right chain is scanned, and once an
// entry R[j] (j >= 1) is pushed without a pop the stack ends in R[j-1],
// R[j], and the rest of R extends it with left turns: it is copied without
// tests.  R may lie in the same array at or after E + nL: every write goes
// at or before the entry just read.
template <bool SMALL, typename T, typename Pt>
__device__ __forceinline__ int merge_right(T *E, int nL, const T *R, int nR, Pt pt) {
  int top = nL;
  int2 a = make_int2(0, 0), b = make_int2(0, 0);
  if (top >= 2) a = pt(E[top - 2]);
  if (top >= 1) b = pt(E[top - 1]);
  int j = 0;
  while (j < nR) {
    const T e = R[j];
    const int2 v = pt(e);
    bool popped = false;
    while (top >= 2 && !cross_pos<SMALL>(a, b, v)) {
      --top;
      b = a;
      if (top >= 2) a = pt(E[top - 2]);
      popped = true;
    }
    E[top++] = e;
    a = b;
    b = v;
    ++j;
    if (j >= 2 && !popped) break;
  }
  for (; j + 4 <= nR; j += 4) {
    const T e0 = R[j], e1 = R[j + 1], e2 = R[j + 2], e3 = R[j + 3];
    E[top] = e0;
    E[top + 1] = e1;
    E[top + 2] = e2;
    E[top + 3] = e3;
    top += 4;
  }
  for (; j < nR; ++j) E[top++] = R[j];
  return top;
}

__global__ __launch_bounds__(2 * kTileSlabs) void k_b_tiles(const int2 *__restrict__ work,
                                                             const BCloud *cl) {
  __shared__ uint32_t sE[2 * kSideWords];       // per side, per slab: a row of entries
  __shared__ unsigned long long sVm[kTileSlabs], sSm[kTileSlabs];
  __shared__ int sTop[2][kTileSlabs];
  const int2 w = work[blockIdx.x];
  const BCloud &A = cl[w.x];
  const int p = A.p;
  const int2 *const Lm = A.Lm;
  uint64_t *const mask = A.mask;
  int32_t *const slab_k = A.slab_k;
  int32_t *const slab_s = A.slab_s;
  const int64_t c0 = (int64_t)w.y * kTileCols;
  const int ncol = (int)min<int64_t>(kTileCols, p - c0);
  const int nslab = (ncol + kSlab - 1) / kSlab;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  constexpr int kIter = kTileSlabs / 2;
  // columns -> entries and ballots (wave w takes slabs w, w + 2, ...)
  int2 Lr[kIter];
#pragma unroll
  for (int k = 0; k < kIter; ++k) {
    const int col = (2 * k + wave) * kSlab + lane;
    Lr[k] = col < ncol ? Lm[c0 + col] : make_int2(1, 0);
  }
#pragma unroll
  for (int k = 0; k < kIter; ++k) {
    const int sl = 2 * k + wave;
    const int col = sl * kSlab + lane;
    const int2 L = Lr[k];
    const bool valid = L.x <= L.y;
    const unsigned long long vm = __ballot(valid);
    const unsigned long long sm = __ballot(valid && L.x < L.y);
    sE[sl * kRow + lane] = ((uint32_t)col << 16) | (uint32_t)(L.x - 1);
    sE[kSideWords + sl * kRow + lane] = ((uint32_t)col << 16) | (uint32_t)(p - L.y);
    if (lane == 0) {
      sVm[sl] = vm;
      sSm[sl] = sm;
    }
  }
  __syncthreads();
  if (tid < nslab) {
    const int gs = w.y * kTileSlabs + tid;
    const unsigned long long vm = sVm[tid];
    if (mask) mask[gs] = vm;
    slab_k[gs] = __popcll(vm);
    slab_s[gs] = __popcll(vm) + __popcll(sSm[tid]);
  }
  // a lane per (slab, side): the slab's hull, in place over its row
  {
    const int sl = tid >> 1, side = tid & 1;
    uint32_t *row = sE + side * kSideWords + sl * kRow;
    unsigned long long vm = sVm[sl];
    int top = 0;
    int2 a = make_int2(0, 0), b = make_int2(0, 0);
    while (vm) {
      const int i = __ffsll((long long)vm) - 1;
      vm &= vm - 1;
      const uint32_t e = row[i];
      const int2 v = TilePt()(e);
      while (top >= 2 && !cross_pos<true>(a, b, v)) {
        --top;
        b = a;
        if (top >= 2) a = TilePt()(row[top - 2]);
      }
      row[top++] = e;
      a = b;
      b = v;
    }
    sTop[side][sl] = top;
  }
  // binary merge tree over the slab hulls: at step h, the lane of (group g,
  // side) joins the hulls of slabs g*2h and g*2h + h, leaving the result at
  // the first one's row
  for (int h = 1; h < kTileSlabs; h <<= 1) {
    __syncthreads();
    const int g = tid >> 1, side = tid & 1;
    const int s0 = g * 2 * h, s1 = s0 + h;
    if (s1 < nslab) {
      uint32_t *E = sE + side * kSideWords + s0 * kRow;
      sTop[side][s0] = merge_right<true>(E, sTop[side][s0], E + h * kRow, sTop[side][s1], TilePt());
    }
  }
  __syncthreads();
  // write the node's hulls (level 2, or level 1 when the cloud is one slab)
  const TreeShape &T = A.tree;
  const int lev = T.nlev >= 2 ? 2 : 1;
  const int64_t x0 = c0 + 1;
  int2 *const cand = A.cand;
  const int span = T.span[lev];
  for (int side = 0; side < 2; ++side) {
    const int cnt = sTop[side][0];
    const uint32_t *E = sE + side * kSideWords;
    int2 *out = cand + (size_t)((lev - 1) & 1) * 2 * (size_t)p + (size_t)side * p + (size_t)w.y * span;
    for (int j = tid; j < cnt; j += 2 * kTileSlabs) {
      const uint32_t e = E[j];
      const int y = (int)(e & 0xFFFFu);
      out[j] = make_int2((int)(x0 + (e >> 16)), side ? y - p : y + 1);
    }
    if (tid == 0) A.ccount[side * T.nodes + T.base[lev] + w.y] = cnt;
  }
}

// A wave per (node at level lev >= 3, side): the children's hulls (level
// lev-1, buffer (lev-2)&1) staged in LDS in order and joined child by child
// by lane 0, the result copied to the node's slot of buffer (lev-1)&1.  A
// node whose children hold more than kNodeCap points is joined the same way
// in global memory.
template <bool SMALL>
__global__ __launch_bounds__(kWave) void k_b_nodes(const int4 *__restrict__ work, const BCloud *cl,
                                                   int lev) {
  __shared__ int2 sP[kNodeCap];
  __shared__ int sOff[kFanIn + 1];
  __shared__ int sTop;
  const int4 w = work[blockIdx.x];        // (cloud, node, side, -)
  const BCloud &H = cl[w.x];
  const TreeShape &T = H.tree;
  const int node = w.y, side = w.z;
  const int lane = threadIdx.x;
  const int64_t P = H.p;
  const int2 *in = H.cand + (size_t)((lev - 2) & 1) * 2 * P + (size_t)side * P;
  int2 *out = H.cand + (size_t)((lev - 1) & 1) * 2 * P + (size_t)side * P + (size_t)node * T.span[lev];
  const int c0 = node * kFanIn, nc = min(kFanIn, T.size[lev - 1] - c0);
  const int32_t *cnt = H.ccount + side * T.nodes + T.base[lev - 1];
  int32_t *const ccount_out = H.ccount + side * T.nodes + T.base[lev] + node;
  const size_t span = (size_t)T.span[lev - 1];
  // child offsets (wave scan)
  const int mine = lane < nc ? cnt[c0 + lane] : 0;
  int incl = mine;
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  const int m = __shfl(incl, kWave - 1, kWave);
  sOff[lane] = incl - mine;
  if (lane == 0) sOff[kFanIn] = m;
  __syncthreads();
  if (m <= kNodeCap) {
    for (int j = lane; j < m; j += kWave) {
      int lo = 0, hi = nc - 1;            // last child with sOff[c] <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sOff[mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      sP[j] = in[(size_t)(c0 + lo) * span + (j - sOff[lo])];
    }
    __syncthreads();
    if (lane == 0) {
      int top = sOff[1] - sOff[0];
      for (int c = 1; c < nc; ++c)
        top = merge_right<SMALL>(sP, top, sP + sOff[c], sOff[c + 1] - sOff[c], PlainPt());
      sTop = top;
    }
    __syncthreads();
    const int top = sTop;
    for (int j = lane; j < top; j += kWave) out[j] = sP[j];
    if (lane == 0) *ccount_out = top;
    return;
  }
  if (lane != 0) return;
  int top = 0;
  for (int c = 0; c < nc; ++c)
    top = merge_right<SMALL>(out, top, in + (size_t)(c0 + c) * span, cnt[c0 + c], PlainPt());
  *ccount_out = top;
}

// Per cloud (one wave): slab offsets and totals, then the final hull from
// the root's two sides (lower left to right, then upper back).
__global__ __launch_bounds__(64) void k_b_root(const BCloud *cl) {
  const BCloud &A = cl[blockIdx.x];
  const TreeShape &T = A.tree;
  const int lane = threadIdx.x;
  const int nslab = T.size[1];
  int carry = 0, stot = 0;
  for (int base = 0; base < nslab; base += kWave) {
    const int i = base + lane;
    const int kk = i < nslab ? A.slab_k[i] : 0;
    stot += i < nslab ? A.slab_s[i] : 0;
    int incl = kk;
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    if (i < nslab) A.slab_off[i] = carry + incl - kk;
    carry += __shfl(incl, kWave - 1, kWave);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) stot += __shfl_xor(stot, d, kWave);
  const int64_t P = A.p;
  const int2 *root = A.cand + (size_t)((T.nlev - 1) & 1) * 2 * P;
  const int nl = A.ccount[0 * T.nodes + T.base[T.nlev]];
  const int nu = A.ccount[1 * T.nodes + T.base[T.nlev]];
  bool overflow = false;
  const int h = assemble_hull(root, nl, root + P, nu, A.hx, A.hy, A.hull_cap, overflow);
  if (lane == 0) {
    A.info[HP_INFO_K] = carry;
    A.info[HP_INFO_S] = stot;
    A.info[HP_INFO_H] = overflow ? 0 : h;
    if (overflow) atomicMin(&A.info[HP_INFO_STATUS], HP_ECAPACITY);
  }
}

// Per slab (one wave): its valid columns at the scanned offset.
__global__ __launch_bounds__(256) void k_b_chain(const int2 *__restrict__ work, int nwork,
                                                 const BCloud *cl) {
  const int t = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (t >= nwork) return;
  const int2 w = work[t];
  const BCloud &A = cl[w.x];
  write_chain_slab(A.Lm, A.p, A.slab_off, w.y, A.cx, A.clo, A.chi, A.chain_cap, A.info);
}

hipError_t launch_b_fill(int B, const BCloud *cl, const uint8_t *needs_fill, int32_t *counter,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_b_fill, dim3(B), dim3(256), 0, s, cl, needs_fill, counter);
  return hipGetLastError();
}

hipError_t prepare_b_reduce() {
  return hipFuncSetAttribute((const void *)k_b_reduce<1024, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             device_info().lds_bytes - 64);
}

hipError_t launch_b_reduce(int grid, size_t lds_bytes, const BatchItem *items, int32_t nitems,
                           int32_t *counter, const BCloud *cl, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_b_reduce<1024, 4>), dim3(grid), dim3(1024), lds_bytes, s, items, nitems, counter, cl);
  return hipGetLastError();
}

hipError_t launch_b_tiles(int ntiles, const int2 *tiles, const BCloud *cl, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_tiles, dim3(ntiles), dim3(2 * kTileSlabs), 0, s, tiles, cl);
  return hipGetLastError();
}

hipError_t launch_b_nodes(bool small, int lev, int nwork, const int4 *work, const BCloud *cl,
                          hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (small) hipLaunchKernelGGL((k_b_nodes<true>), dim3(nwork), dim3(kWave), 0, s, work, cl, lev);
  else hipLaunchKernelGGL((k_b_nodes<false>), dim3(nwork), dim3(kWave), 0, s, work, cl, lev);
  return hipGetLastError();
}

hipError_t launch_b_root(int B, const BCloud *cl, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_root, dim3(B), dim3(64), 0, s, cl);
  return hipGetLastError();
}

hipError_t launch_b_chain(int nwork, const int2 *work, const BCloud *cl, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_chain, dim3((nwork + 3) / 4), dim3(256), 0, s, work, nwork, cl);
  return hipGetLastError();
}

}  // namespace hp
