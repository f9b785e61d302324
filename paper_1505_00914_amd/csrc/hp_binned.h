// hp_binned.h -- Algorithm 1 for large p (L beyond what LDS windows cover):
// the points are first binned by column window, then every window is folded
// in LDS.  Included by hp_single.hip.
//
// A device L of 2^20 columns is 8 MiB: folding points into it one at a time
// costs a random read (and sometimes an atomic) per point, which the memory
// system serves far below the streaming rate.  Here the fold of Algorithm 1
// is split in two passes that each touch memory in long runs:
//
//   k_bin       streams the points once.  Each point that may change L
//               becomes a 32-bit entry (column within its window of 4096
//               columns, y - 1), sorted in LDS by window per tile of 8192
//               points and written out in 128-byte blocks to the pages of
//               its workgroup's stream for that window.
//   k_bin_fold  one workgroup per (window, slice of the binning workgroups):
//               folds the entries of those streams into the window's L in
//               LDS and writes the window of a partial L.
//
// Min and max commute, so the order in which entries are folded does not
// matter.  Between rounds (consecutive ranges of the points) k_bin_merge
// folds the partial arrays into the running L and rebuilds the filter: per
// group of 64 columns the largest lo and the smallest hi, quantised inwards
// to 8 bits each.  A later round drops a point whose y lies inside its
// group's range: its column already holds points at or below and at or
// above it, so it cannot change L.  The later round first streams its
// points through k_bin_compact, which keeps only those the filter cannot
// drop, back to back in one segment per binning workgroup; k_bin then bins
// those short lists, unfiltered.  When a segment overflows, k_bin bins the
// whole range with the filter.
#pragma once

#include <climits>

#include "hp_reduce.h"

namespace hp {

constexpr int kBinXBits = 12;                       // column within a window
constexpr int kBinWc = 1 << kBinXBits;              // columns per window
constexpr int kBinYBits = 20;                       // y - 1
constexpr int64_t kBinPMax = (int64_t)1 << kBinYBits;
constexpr int kBinNwMax = (int)(kBinPMax / kBinWc); // 256 windows at most
constexpr int kBinBlk = 32;                         // entries per written block (128 bytes)
constexpr int kBinPage = 1024;                      // entries per page (4 KiB)
constexpr int kBinThreads = 1024;                   // k_bin workgroup: one bookkeeping wave, 15 point waves
constexpr int kBinWorkers = kBinThreads - 64;       // lanes that hold points
constexpr int kBinVpt = 4;                          // 16-byte vectors per point lane per tile
constexpr int kBinTileV = kBinWorkers * kBinVpt;    // vectors per tile (7680 points)
constexpr int kBinFilterShift = 6;                  // 64 columns per filter group
constexpr int kCpFilterShift = 5;                   // 32 columns per group of the compaction's filter
constexpr int kBinFoldThreads = 512;
// blocks one tile can complete: its 8192 points (2 more in the tile of the
// odd points) plus every window's carry of fewer than kBinBlk entries
constexpr int kBinMaxBlocks = ((2 * kBinTileV + 2) + kBinNwMax * (kBinBlk - 1)) / kBinBlk + 2;
constexpr int kBinBlkWinInts = ((kBinMaxBlocks + 1) / 2 + 1) & ~1;   // ints holding the block map (even)

struct BinArgs {
  uint32_t *pool;     // [G][pages][kBinPage] entries
  int32_t *E;         // [G][nw] entries per stream
  int32_t *pg_off;    // [G][nw + 1] first page of each window's stream in pg_list
  int32_t *pg_list;   // [G][pages] page ids of every stream, window by window
  int32_t *pwin;      // [G][pages] (window << 16 | page index in its stream) of each page
  int32_t pages;      // pages per workgroup
  int32_t nw;         // windows
  int32_t G;          // binning workgroups
};

// Exclusive scan over the WAVES waves of the workgroup, every thread of
// which calls it; tmp holds one partial sum per wave.
template <int WAVES>
__device__ __forceinline__ unsigned long long bin_scan3(unsigned long long v, unsigned long long *tmp,
                                                        unsigned long long *total) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  unsigned long long incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const unsigned long long o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  if (lane == kWave - 1) tmp[wv] = incl;
  __syncthreads();
  unsigned long long off = 0, all = 0;
#pragma unroll
  for (int j = 0; j < WAVES; ++j) {
    if (j < wv) off += tmp[j];
    all += tmp[j];
  }
  *total = all;
  return off + incl - v;
}

// Inclusive prefix sum over the 64 lanes of a wave (row shifts, then the
// row broadcasts of lanes 15 and 31).
__device__ __forceinline__ int wave_incl_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr 1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr 2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr 4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr 8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast 15 into rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast 31 into rows 2 and 3
  return v;
}

// LDS of k_bin, carved from the dynamic allocation.  Per window the state
// that wave 0 keeps from tile to tile (four windows per lane, read and
// written 16 bytes at a time): the previous tile's blocks, new pages, their
// page offset and which carry buffer holds the carry (packed in pk), its
// entries (tot), the stream's entries written so far (Es) and its open page
// (cur).  The other waves read two packed records per window: winA = (entry
// offset in sbuf, carry count, entries in full blocks, carry buffer) and
// winB = (first block, stream position, open page, first new page).
struct BinLds {
  uint32_t *sbuf;     // this tile's entries that complete blocks, by window
  uint32_t *carry;    // [2][kBinNwMax][kBinBlk]: entries not yet written (< kBinBlk per window)
  uint16_t *filt;     // filter words (nf of them), or unused
  int *cnt, *pk, *tot, *Es, *cur;   // cnt: [2][kBinNwMax]
  int4 *winA, *winB;
  uint16_t *blkwin;   // window of every block written this tile
  int *scalars;       // [0] pages used before this tile's, [1] blocks and [2] new pages of this tile,
                      // [3] error bits, [4] pages in all
};

constexpr int kBinWinArrays = 6;   // cnt takes two
__host__ __device__ constexpr size_t bin_lds_bytes(int nf) {
  return sizeof(uint32_t) * (size_t)(2 * kBinTileV + 8) + sizeof(uint32_t) * (size_t)(2 * kBinNwMax * kBinBlk) +
         sizeof(uint16_t) * (size_t)((nf + 7) & ~7) + sizeof(int) * kBinWinArrays * (size_t)kBinNwMax +
         sizeof(int4) * 2 * (size_t)kBinNwMax + sizeof(int) * (size_t)kBinBlkWinInts + sizeof(int) * 8;
}

__device__ __forceinline__ BinLds bin_carve(uint32_t *smem, int nf) {
  BinLds S;
  uint32_t *q = smem;
  S.sbuf = q;     q += 2 * kBinTileV + 8;
  S.carry = q;    q += 2 * kBinNwMax * kBinBlk;
  S.filt = reinterpret_cast<uint16_t *>(q);
  q += ((nf + 7) & ~7) / 2;
  int *ip = reinterpret_cast<int *>(q);
  S.cnt = ip;   // two count buffers, used by tiles in turn
  ip += 2 * kBinNwMax;
  int **arr[kBinWinArrays - 2] = {&S.pk, &S.tot, &S.Es, &S.cur};
  for (int a = 0; a < kBinWinArrays - 2; ++a) {
    *arr[a] = ip;
    ip += kBinNwMax;
  }
  S.winA = reinterpret_cast<int4 *>(ip);
  S.winB = S.winA + kBinNwMax;
  ip = reinterpret_cast<int *>(S.winB + kBinNwMax);
  S.blkwin = reinterpret_cast<uint16_t *>(ip);
  ip += kBinBlkWinInts;
  S.scalars = ip;
  return S;
}

__device__ __forceinline__ int4 lds4(const int *a, int i) { return *reinterpret_cast<const int4 *>(a + i); }
__device__ __forceinline__ void sto4(int *a, int i, int4 v) { *reinterpret_cast<int4 *>(a + i) = v; }
__device__ __forceinline__ int at(const int4 &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; }
__device__ __forceinline__ int4 mk4(const int (&a)[4]) { return make_int4(a[0], a[1], a[2], a[3]); }

// Per-window bookkeeping, by wave 0 alone (windows lane, lane + 64, lane +
// 128, lane + 192; windows past nw hold zeros and stay so): first the
// previous tile's blocks and pages are applied (carry count, stream
// position, open page, carry buffer), then, with `count`, this tile's counts
// (cnt, which it clears for the tile after next) become the offsets of its
// entries, blocks and new pages (a wave scan per
// group of 64 windows), and the pages the tile opens are recorded for the
// fold.  Every state word is loaded before any is stored.  Returns the pages
// used before this tile's (in every lane: the scalar words are written by
// lane 0 and only read by other lanes after a barrier).
__device__ __forceinline__ int bin_windows(const BinLds &S, const BinArgs &B, int g, int *cnt) {
  const bool count = cnt != nullptr;
  const int lane = threadIdx.x;
  const int U = S.scalars[0], NPG = S.scalars[2];
  const int ucur = U + NPG;
  // pk: blocks (9 bits), new pages (4), their first page offset (9), carry buffer (1)
  int vpk[4], vtot[4], ves[4], vcur[4], vcnt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int w = lane + kWave * k;
    vpk[k] = S.pk[w];
    vtot[k] = S.tot[w];
    ves[k] = S.Es[w];
    vcur[k] = S.cur[w];
    vcnt[k] = count ? cnt[w] : 0;
  }
  int nbw[4], np[4], cc[4], e[4], cur[4], sel[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int pk = vpk[k];
    const int pnb = pk & 0x1FF, pnp = (pk >> 9) & 0xF, ppo = (pk >> 13) & 0x1FF;
    cc[k] = vtot[k] - kBinBlk * pnb;
    e[k] = ves[k] + kBinBlk * pnb;
    cur[k] = pnp > 0 ? U + ppo + pnp - 1 : vcur[k];
    sel[k] = ((pk >> 22) & 1) ^ (pnb > 0 ? 1 : 0);
    const int t = cc[k] + vcnt[k];
    nbw[k] = t / kBinBlk;
    np[k] = (e[k] + kBinBlk * nbw[k] + kBinPage - 1) / kBinPage - (e[k] + kBinPage - 1) / kBinPage;
    const int w = lane + kWave * k;
    S.tot[w] = t;
    S.Es[w] = e[k];
    S.cur[w] = cur[k];
    if (count) cnt[w] = 0;
  }
  // counts 14 bits, blocks 9, pages 9: one 32-bit scan per group of 64
  // windows, groups in window order
  int base = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int w = lane + kWave * k;
    const int packed = vcnt[k] | (nbw[k] << 14) | (np[k] << 23);
    const int incl = wave_incl_sum(packed);
    const unsigned ex = (unsigned)(base + incl - packed);
    const int oc = (int)(ex & 0x3FFFu), ob = (int)((ex >> 14) & 0x1FFu), op = (int)(ex >> 23);
    base += __builtin_amdgcn_readlane(incl, kWave - 1);
    S.pk[w] = nbw[k] | (np[k] << 9) | (op << 13) | (sel[k] << 22);
    S.winA[w] = make_int4(oc, cc[k], kBinBlk * nbw[k], sel[k]);
    S.winB[w] = make_int4(ob, e[k], cur[k], ucur + op);
    for (int i = 0; i < nbw[k]; ++i) S.blkwin[ob + i] = (uint16_t)w;
    const int first = ucur + op, opened = (e[k] + kBinPage - 1) / kBinPage;
    for (int i = 0; i < np[k]; ++i)
      if (first + i < B.pages) B.pwin[(size_t)g * B.pages + first + i] = (w << 16) | (opened + i);
  }
  if (lane == 0) {
    S.scalars[0] = ucur;
    S.scalars[1] = (int)(((unsigned)base >> 14) & 0x1FFu);
    S.scalars[2] = (int)((unsigned)base >> 23);
  }
  return ucur;
}

// The three steps of a tile for the point lanes.  bin_rank: up to
// 2 * kBinVpt points per lane (x, y already moved by the origin), `in` per
// point; the entries that pass the filter are ranked by window.  bin_scatter
// (after the bookkeeping wave has turned the counts into offsets): entries
// that complete a block go to sbuf, the others extend their window's carry
// (in the other buffer when the window writes blocks this tile, whose old
// carry bin_flush still reads).  bin_flush, by every lane: each completed
// block (old carry first, then sbuf) is written to its window's stream.
__device__ __forceinline__ void bin_rank(const BinLds &S, int *cnt, Extent p, bool filtered, int qs,
                                         const int (&xs)[2 * kBinVpt], const int (&ys)[2 * kBinVpt],
                                         const bool (&in)[2 * kBinVpt], bool &bad, int (&wr)[2 * kBinVpt],
                                         uint32_t (&val)[2 * kBinVpt]) {
  constexpr int PP = 2 * kBinVpt;
  // every filter word is read before any rank is taken, so the reads share
  // one wait and the atomics another
  bool pass[PP];
  unsigned f[PP];
#pragma unroll
  for (int j = 0; j < PP; ++j) {
    const unsigned xi = (unsigned)(xs[j] - 1), yi = (unsigned)(ys[j] - 1);
    const bool ok = in[j] & (xi < (unsigned)p.p) & (yi < (unsigned)p.q);
    bad |= in[j] & !ok;
    pass[j] = ok;
    val[j] = ((xi & (unsigned)(kBinWc - 1)) << kBinYBits) | yi;
    wr[j] = (int)(xi >> kBinXBits);
    if (filtered) f[j] = S.filt[ok ? (xi >> kBinFilterShift) : 0u];
  }
  if (filtered) {
#pragma unroll
    for (int j = 0; j < PP; ++j) {
      const unsigned yi = val[j] & ((1u << kBinYBits) - 1);
      const unsigned lo_b = (f[j] & 0xFFu) << qs, hi_b = (f[j] >> 8) << qs;
      pass[j] = pass[j] & ((yi < lo_b) | (yi > hi_b));
    }
  }
  // (window << 16) | rank in the window, or -1 when dropped
#pragma unroll
  for (int j = 0; j < PP; ++j) wr[j] = pass[j] ? (wr[j] << 16) | atomicAdd(&cnt[wr[j]], 1) : -1;
}

__device__ __forceinline__ void bin_scatter(const BinLds &S, const int (&wr)[2 * kBinVpt],
                                            const uint32_t (&val)[2 * kBinVpt]) {
  constexpr int PP = 2 * kBinVpt;
  int4 wa[PP];
#pragma unroll
  for (int j = 0; j < PP; ++j)
      wa[j] = S.winA[wr[j] < 0 ? 0 : wr[j] >> 16];
#pragma unroll
  for (int j = 0; j < PP; ++j) {
    if (wr[j] < 0) continue;
    const int w = wr[j] >> 16, rk = wr[j] & 0xFFFF;
    const int idx = wa[j].y + rk, full = wa[j].z;
    if (idx < full) S.sbuf[wa[j].x + rk] = val[j];
    else S.carry[((wa[j].w ^ (full > 0 ? 1 : 0)) * kBinNwMax + w) * kBinBlk + idx - full] = val[j];
  }
}

__device__ __forceinline__ void bin_flush(const BinLds &S, const BinArgs &B, int g, bool &over) {
  const int tid = threadIdx.x;
  const int used = S.scalars[0], nblk = S.scalars[1], nnew = S.scalars[2];
  over |= used + nnew > B.pages;
  // half a wave per block of 32 entries (128 bytes), four blocks per step
  // with every LDS read of the step issued before the stores
  constexpr int kHalves = kBinThreads / kBinBlk;
  constexpr int kStep = 4;
  const int l = tid & (kBinBlk - 1);
  for (int b0 = tid / kBinBlk; b0 < nblk; b0 += kStep * kHalves) {
    int w[kStep];
#pragma unroll
    for (int r = 0; r < kStep; ++r) w[r] = b0 + r * kHalves < nblk ? S.blkwin[b0 + r * kHalves] : 0;
    int4 A[kStep], Bv[kStep];
#pragma unroll
    for (int r = 0; r < kStep; ++r) {
      A[r] = S.winA[w[r]];
      Bv[r] = S.winB[w[r]];
    }
    uint32_t v[kStep];
    int idx[kStep];
#pragma unroll
    for (int r = 0; r < kStep; ++r) {
      idx[r] = b0 + r * kHalves < nblk ? (b0 + r * kHalves - Bv[r].x) * kBinBlk + l : 0;
      v[r] = idx[r] < A[r].y ? S.carry[(A[r].w * kBinNwMax + w[r]) * kBinBlk + idx[r]]
                             : S.sbuf[A[r].x + idx[r] - A[r].y];
    }
#pragma unroll
    for (int r = 0; r < kStep; ++r) {
      if (b0 + r * kHalves >= nblk) continue;
      const int es = Bv[r].y, e = es + idx[r];
      const int ip = e / kBinPage, opened = (es + kBinPage - 1) / kBinPage;
      const int pid = ip < opened ? Bv[r].z : Bv[r].w + (ip - opened);
      if (pid >= 0 && pid < B.pages) B.pool[((size_t)g * B.pages + pid) * kBinPage + (e & (kBinPage - 1))] = v[r];
      else over = true;
    }
  }
}

// Binning pass over n points (pts 8-byte aligned).  Workgroup g takes the
// tiles [g * tpw, (g + 1) * tpw); workgroup 0 also takes the one point that
// precedes the 16-byte-aligned body and the odd last point.  F (nf 16-bit
// words, bounds in steps of 2^qs) is the filter of the previous rounds, or
// null in the first round.  Workgroup 0 of the first round also clears the
// finish step's control words (R).
// With `cpts`, workgroup g bins segment g of the points k_bin_compact kept
// (ccount[g] of them, moved by the origin) in place of its share of pts,
// unfiltered and with no origin, unless a segment overflowed (*cover).
__global__ __launch_bounds__(kBinThreads) void k_bin(const int32_t *__restrict__ pts, int64_t n, Extent p,
                                                     const uint16_t *__restrict__ F, int32_t nf, int32_t qs,
                                                     BinArgs B, int32_t *__restrict__ wg_err, int2 org,
                                                     ResetArgs R, const int2 *__restrict__ cpts,
                                                     const int64_t *__restrict__ ccount, int64_t segcap,
                                                     const int32_t *__restrict__ cover) {
  extern __shared__ uint32_t bin_smem[];
  reset_controls(R);
  const bool segment = cpts != nullptr && *cover == 0;
  if (segment) {
    pts = reinterpret_cast<const int32_t *>(cpts + (size_t)blockIdx.x * (size_t)segcap);
    n = ccount[blockIdx.x];
    F = nullptr;
    org = make_int2(0, 0);
  }
  const BinLds S = bin_carve(bin_smem, F ? nf : 0);
  const int tid = threadIdx.x, g = blockIdx.x;
  const bool filtered = F != nullptr;
  for (int w = tid; w < kBinNwMax; w += kBinThreads) {
    S.cnt[w] = 0;
    S.cnt[kBinNwMax + w] = 0;
    S.pk[w] = 0;
    S.tot[w] = 0;
    S.Es[w] = 0;
    S.cur[w] = -1;
  }
  if (filtered)
    for (int i = tid; i < nf; i += kBinThreads) S.filt[i] = F[i];
  if (tid < 8) S.scalars[tid] = 0;
  __syncthreads();
  bool bad = false, over = false;
  constexpr int PP = 2 * kBinVpt;
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int64_t tail = head + 2 * nv;
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  // a workgroup's share: its segment, or its tiles of the whole range
  const int64_t ntiles = (nv + kBinTileV - 1) / kBinTileV;
  const int64_t tpw = segment ? ntiles : (ntiles + B.G - 1) / B.G;
  const int64_t vbeg = segment ? 0 : (int64_t)g * tpw * kBinTileV;
  const int64_t vend = min(nv, vbeg + tpw * kBinTileV);
  const int nvt = vbeg < vend ? (int)((vend - vbeg + kBinTileV - 1) / kBinTileV) : 0;
  const bool ht = (segment || g == 0) && (head || tail < n);   // a first tile of the odd points
  // Wave 0 keeps the per-window books; the other waves hold the points.
  // Tiles run as a two-stage pipeline: while wave 0 turns tile t's counts
  // into offsets, the point waves rank tile t + 1 (into the other count
  // buffer); then tile t's entries are placed and its blocks written.  Both
  // sides take the same barriers (one before the first tile, three per
  // tile), so the bookkeeping wave holds no point registers and the point
  // waves none of the books.
  const int T = nvt + (ht ? 1 : 0);
  if (tid < kWave) {
    if (T > 0) __syncthreads();   // tile 0 ranked
    for (int t = 0; t < T; ++t) {
      bin_windows(S, B, g, S.cnt + (t & 1) * kBinNwMax);
      __syncthreads();   // offsets of tile t ready, tile t + 1 ranked
      __syncthreads();   // entries of tile t in place
      bin_flush(S, B, g, over);
      __syncthreads();   // tile t written: its records may change
    }
  } else {
    const int wt = tid - kWave;
    // the points of tile i (the tile of odd points first, then the vector
    // tiles) into xs, ys, in; vector tiles come from q
    auto unpack = [&](const int4 (&q)[kBinVpt], int64_t base, int (&xs)[PP], int (&ys)[PP], bool (&in)[PP]) {
#pragma unroll
      for (int u = 0; u < kBinVpt; ++u) {
        const bool ok = base + u * kBinWorkers + wt < vend;
        const int4 r = shift_by(q[u], org.x, org.y);
        xs[2 * u] = r.x;
        ys[2 * u] = r.y;
        xs[2 * u + 1] = r.z;
        ys[2 * u + 1] = r.w;
        in[2 * u] = ok;
        in[2 * u + 1] = ok;
      }
    };
    auto odd_points = [&](int (&xs)[PP], int (&ys)[PP], bool (&in)[PP]) {
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        xs[j] = 0;
        ys[j] = 0;
        in[j] = false;
      }
      if (wt == 0) {
        if (head) {
          xs[0] = shift_by(pts[0], org.x);
          ys[0] = shift_by(pts[1], org.y);
          in[0] = true;
        }
        if (tail < n) {
          xs[1] = shift_by(pts[2 * tail], org.x);
          ys[1] = shift_by(pts[2 * tail + 1], org.y);
          in[1] = true;
        }
      }
    };
    // a lane past the end loads the last vector of the range (always a
    // valid address) and its points are not used
    auto load = [&](int4 (&q)[kBinVpt], int64_t base) {
#pragma unroll
      for (int u = 0; u < kBinVpt; ++u) q[u] = load_stream(&v[min(base + u * kBinWorkers + wt, vend - 1)]);
    };
    int wr[PP], wr1[PP];
    uint32_t val[PP], val1[PP];
    int4 q[kBinVpt];          // the next vector tile to rank
    int64_t qbase = vbeg;     // its first vector
    if (nvt > 0) load(q, qbase);
    if (T > 0) {
      int xs[PP], ys[PP];
      bool in[PP];
      if (ht) {
        odd_points(xs, ys, in);
      } else {
        unpack(q, qbase, xs, ys, in);
        qbase += kBinTileV;
        load(q, qbase);
      }
      bin_rank(S, S.cnt, p, filtered, qs, xs, ys, in, bad, wr, val);
      __syncthreads();
    }
    for (int t = 0; t < T; ++t) {
      const bool more = t + 1 < T;
      int4 qn[kBinVpt];
      if (more) {
        // rank tile t + 1 (a vector tile) while wave 0 books tile t; the
        // loads of the tile after it are issued first and only waited for
        // at the end of this step
        int xs[PP], ys[PP];
        bool in[PP];
        load(qn, qbase + kBinTileV);
        unpack(q, qbase, xs, ys, in);
        bin_rank(S, S.cnt + ((t + 1) & 1) * kBinNwMax, p, filtered, qs, xs, ys, in, bad, wr1, val1);
      }
      __syncthreads();
      bin_scatter(S, wr, val);
      __syncthreads();
      bin_flush(S, B, g, over);
      __syncthreads();
      if (more) {
#pragma unroll
        for (int j = 0; j < PP; ++j) {
          wr[j] = wr1[j];
          val[j] = val1[j];
        }
#pragma unroll
        for (int u = 0; u < kBinVpt; ++u) q[u] = qn[u];
        qbase += kBinTileV;
      }
    }
  }
  // the last tile's bookkeeping, then each window's carry as a last, partial
  // block, and the streams' entry and page counts; winB then holds, per
  // window, (first page in the page list, page of the last block, carry
  // count, stream position)
  __syncthreads();
  const int nw = B.nw;
  if (tid < kWave) {
    const int ucur = bin_windows(S, B, g, nullptr);
    const int lane = tid;
    // the windows of this lane are the ones bin_windows gave it (lane +
    // 64 k), so every record read here was written by this lane; one scan
    // per group of 64 windows, groups in window order
    int base_n = 0, base_p = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int w = lane + kWave * k;
      const int4 a = S.winA[w], b = S.winB[w];
      const int cc = a.y, es = b.y, cur = b.z;
      const int npf = (cc > 0 && (es & (kBinPage - 1)) == 0) ? 1 : 0;
      const int ef = es + cc;
      const int pw = (ef + kBinPage - 1) / kBinPage;
      const int in_n = wave_incl_sum(npf), in_p = wave_incl_sum(pw);
      const int on = base_n + in_n - npf, opw = base_p + in_p - pw;
      base_n += __builtin_amdgcn_readlane(in_n, kWave - 1);
      base_p += __builtin_amdgcn_readlane(in_p, kWave - 1);
      const int pid = npf ? ucur + on : cur;
      S.winB[w] = make_int4(opw, pid, cc, es);
      if (w < nw) {
        B.E[(size_t)g * nw + w] = ef;
        B.pg_off[(size_t)g * (nw + 1) + w] = opw;
        if (npf && pid < B.pages) B.pwin[(size_t)g * B.pages + pid] = (w << 16) | (es / kBinPage);
      }
    }
    if (lane == 0) {
      B.pg_off[(size_t)g * (nw + 1) + nw] = base_p;
      S.scalars[4] = base_p;
    }
  }
  __syncthreads();
  // a wave per window writes its carry
  for (int w = tid / kWave; w < nw; w += kBinThreads / kWave) {
    const int lane = tid & (kWave - 1);
    const int4 f = S.winB[w];
    const int cc = f.z;
    if (lane < cc) {
      const int e = f.w + lane, pid = f.y;
      if (pid >= 0 && pid < B.pages)
        B.pool[((size_t)g * B.pages + pid) * kBinPage + (e & (kBinPage - 1))] =
            S.carry[(S.winA[w].w * kBinNwMax + w) * kBinBlk + lane];
      else
        over = true;
    }
  }
  __syncthreads();
  // the page list ordered by window, each window's pages in stream order
  const int npages = min(S.scalars[4], B.pages);
  for (int pid = tid; pid < npages; pid += kBinThreads) {
    const int word = B.pwin[(size_t)g * B.pages + pid];
    const int w = word >> 16, ip = word & 0xFFFF;
    if (w < nw) {
      const int li = S.winB[w].x + ip;
      if (li < B.pages) B.pg_list[(size_t)g * B.pages + li] = pid;
    }
  }
  if (bad) atomicOr(&S.scalars[3], kErrRange);
  if (over) atomicOr(&S.scalars[3], kErrBinOverflow);
  __syncthreads();
  if (tid == 0) wg_err[g] = S.scalars[3];
}

// First pass of a filtered round, one workgroup per binning workgroup g:
// the points of its share of [pts, pts + 2n) (a contiguous range of 16-byte
// vectors; workgroup 0 also takes the point before the aligned body and the
// odd last point), moved by the origin, each tested against the filter F
// (nf words, one per 32 columns: a finer filter than bin_rank's, which the
// LDS of this kernel has room for; bounds in steps of 2^qs).  Every point that
// passes, or lies outside the box (which the binning pass then reports), is
// written to segment g of out (segcap points), back to back in an arbitrary
// order; count[g] receives the number kept.  A workgroup that keeps more than
// segcap writes no further and sets *over, and k_bin then bins the whole
// range instead.  Each wave takes its room in the segment with an LDS
// atomic, so the waves never wait for one another, and gathers its kept
// points in LDS first, so that they leave in whole 512-byte stores.
constexpr int kCpThreads = 1024;
constexpr int kCpVpt = 4;                          // 16-byte vectors per lane and step
constexpr int kCpStepV = kCpThreads * kCpVpt;      // 8192 points per step
constexpr int kCpFilterMax = (int)(kBinPMax >> kCpFilterShift);

__global__ __launch_bounds__(kCpThreads) void k_bin_compact(const int32_t *__restrict__ pts, int64_t n, Extent p,
                                                            const uint16_t *__restrict__ F, int32_t nf, int32_t qs,
                                                            int2 org, int2 *__restrict__ out, int64_t segcap,
                                                            int64_t *__restrict__ count, int32_t *__restrict__ over) {
  constexpr int PP = 2 * kCpVpt;   // points per lane and step
  __shared__ uint16_t sF[kCpFilterMax];
  __shared__ int2 stg[kCpThreads / kWave][kWave * PP];   // a wave's kept points, in order
  __shared__ unsigned long long skept;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave, g = blockIdx.x;
  for (int i = tid; i < nf; i += kCpThreads) sF[i] = F[i];
  auto keep = [&](int x, int y) -> bool {
    const unsigned xi = (unsigned)(x - 1), yi = (unsigned)(y - 1);
    if (!((xi < (unsigned)p.p) & (yi < (unsigned)p.q))) return true;
    const unsigned f = sF[xi >> kCpFilterShift];
    return (yi < ((f & 0xFFu) << qs)) | (yi > ((f >> 8) << qs));
  };
  int2 *const seg = out + (size_t)g * (size_t)segcap;
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int64_t tail = head + 2 * nv;
  const int64_t vpw = (nv + gridDim.x - 1) / gridDim.x;
  const int64_t vb = (int64_t)g * vpw, ve = min(nv, vb + vpw);
  if (tid == 0) skept = 0;
  __syncthreads();
  if (g == 0 && tid == 0) {
    unsigned long long c = 0;
    for (int k = 0; k < 2; ++k) {
      const int64_t i = k == 0 ? 0 : tail;
      if ((k == 0 && !head) || (k == 1 && tail >= n)) continue;
      const int x = shift_by(pts[2 * i], org.x), y = shift_by(pts[2 * i + 1], org.y);
      if (!keep(x, y)) continue;
      if (c < (unsigned long long)segcap) seg[c] = make_int2(x, y);
      ++c;
    }
    skept = c;
  }
  __syncthreads();
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  int4 q[kCpVpt], qn[kCpVpt];
  // a lane past the end loads the last vector of the range (a valid
  // address, since the loop runs only when the range is not empty) and its
  // points are not used; no branch, so the loads of a step stay in flight
  // together and only the previous step's are waited for
  auto load = [&](int4 (&r)[kCpVpt], int64_t b0) {
#pragma unroll
    for (int u = 0; u < kCpVpt; ++u) r[u] = load_stream(&v[min(b0 + (int64_t)u * kCpThreads + tid, ve - 1)]);
  };
  if (vb < ve) load(q, vb);
  for (int64_t b0 = vb; b0 < ve; b0 += kCpStepV) {
    // the next step's vectors are in flight meanwhile; issued on every step
    // (past the end they repeat the last vector), so that the wait for this
    // step's vectors counts the same loads on every path
    load(qn, b0 + kCpStepV);
    __builtin_amdgcn_sched_barrier(0);   // keep those loads ahead of this step's work
    // every filter word is read before any test, so the LDS reads share one wait
    int xs[PP], ys[PP];
    bool ok[PP], in[PP];
    unsigned f[PP];
#pragma unroll
    for (int u = 0; u < kCpVpt; ++u) {
      const int4 r = shift_by(q[u], org.x, org.y);
      xs[2 * u] = r.x;
      ys[2 * u] = r.y;
      xs[2 * u + 1] = r.z;
      ys[2 * u + 1] = r.w;
      in[2 * u] = in[2 * u + 1] = b0 + (int64_t)u * kCpThreads + tid < ve;
    }
#pragma unroll
    for (int j = 0; j < PP; ++j) {
      const unsigned xi = (unsigned)(xs[j] - 1), yi = (unsigned)(ys[j] - 1);
      ok[j] = (xi < (unsigned)p.p) & (yi < (unsigned)p.q);
      f[j] = sF[ok[j] ? (xi >> kCpFilterShift) : 0u];
    }
    unsigned km = 0;   // bit j: point j of the lane is kept
#pragma unroll
    for (int j = 0; j < PP; ++j) {
      const unsigned yi = (unsigned)(ys[j] - 1);
      const bool kept = !ok[j] | (yi < ((f[j] & 0xFFu) << qs)) | (yi > ((f[j] >> 8) << qs));
      km |= (in[j] & kept ? 1u : 0u) << j;
    }
    const int c = __popc(km);
    const int incl = wave_incl_sum(c);
    const int wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
    if (wtot > 0) {   // the same in every lane
      unsigned long long wb = 0;
      if (lane == 0) wb = atomicAdd(&skept, (unsigned long long)wtot);
      wb = __shfl(wb, 0, kWave);
      int k = incl - c;
#pragma unroll
      for (int j = 0; j < PP; ++j)
        if ((km >> j) & 1u) stg[wv][k++] = make_int2(xs[j], ys[j]);
      // LDS accesses of one wave complete in order: the gathered points are
      // read back in place, a run of 64 consecutive points per store
      for (int i = lane; i < wtot; i += kWave) {
        const unsigned long long o = wb + (unsigned long long)i;
        if (o < (unsigned long long)segcap) seg[o] = stg[wv][i];
      }
    }
#pragma unroll
    for (int u = 0; u < kCpVpt; ++u) q[u] = qn[u];
  }
  __syncthreads();
  if (tid == 0) {
    count[g] = (int64_t)skept;
    if (skept > (unsigned long long)segcap) atomicOr(over, 1);
  }
}

// Fold of the binned entries: workgroup (w, s) folds the streams for window
// w of binning workgroups [s G / S, (s + 1) G / S) into the window's L in
// LDS, then writes that window of partial array s (pairs).  Every workgroup
// writes its window, so the S partial arrays cover every column.  The pages
// to fold are listed in LDS first (kBinFoldList at a time: page id and
// entry count), then read sixteen pages per step: each half of the
// workgroup takes every other page, each lane one 16-byte vector (four
// entries) of its half's pages.
constexpr int kBinFoldList = 1024;
constexpr int kBinFoldStep = 16;

__global__ __launch_bounds__(kBinFoldThreads) void k_bin_fold(BinArgs B, Extent p, int32_t S_,
                                                              int2 *__restrict__ part) {
  __shared__ int2 sL[kBinWc];
  __shared__ int lpid[kBinFoldList];
  __shared__ int lcnt[kBinFoldList];
  __shared__ unsigned long long tmp[16];
  const int tid = threadIdx.x;
  const int w = blockIdx.x / S_, s = blockIdx.x % S_;
  const int nw = B.nw;
  // a page is 256 vectors of 16 bytes: the workgroup's halves take
  // alternate pages of a step, kFoldPer pages per lane
  constexpr int kFoldLanes = kBinPage / 4;
  constexpr int kFoldHalves = kBinFoldThreads / kFoldLanes;
  constexpr int kFoldPer = kBinFoldStep / kFoldHalves;
  static_assert(kFoldPer * kFoldHalves == kBinFoldStep, "whole pages per lane and step");
  const int half = tid / kFoldLanes, lt = tid % kFoldLanes;
  const int64_t c0 = (int64_t)w * kBinWc;
  const int ncol = (int)min<int64_t>(kBinWc, (int64_t)p - c0);
  for (int c = tid; c < kBinWc; c += kBinFoldThreads) sL[c] = make_int2(p.q + 1, -1);
  const int g0 = (int)((int64_t)s * B.G / S_), g1 = (int)((int64_t)(s + 1) * B.G / S_);
  for (int gc = g0; gc < g1; gc += kBinFoldThreads) {
    // slot tid: binning workgroup gc + tid, its stream for window w
    const int g = gc + tid;
    int np = 0, base = 0, ent = 0;
    if (g < g1) {
      base = B.pg_off[(size_t)g * (nw + 1) + w];
      np = B.pg_off[(size_t)g * (nw + 1) + w + 1] - base;
      ent = B.E[(size_t)g * nw + w];
    }
    unsigned long long total;
    const int ex = (int)bin_scan3<kBinFoldThreads / kWave>((unsigned long long)np, tmp, &total);
    const int npages = (int)total;
    for (int qb = 0; qb < npages; qb += kBinFoldList) {
      __syncthreads();   // the previous list is no longer read
      for (int i = max(0, qb - ex); i < np && ex + i < qb + kBinFoldList; ++i) {
        const int li = base + i;
        const int pid = li < B.pages ? B.pg_list[(size_t)g * B.pages + li] : -1;
        // (a page id outside the pool can only follow a binning overflow,
        // which the binning pass has already reported)
        const bool okp = pid >= 0 && pid < B.pages;
        lpid[ex + i - qb] = okp ? g * B.pages + pid : 0;
        lcnt[ex + i - qb] = okp ? min(kBinPage, ent - i * kBinPage) : 0;
      }
      __syncthreads();
      const int nq = min(kBinFoldList, npages - qb);
      for (int q0 = 0; q0 < nq; q0 += kBinFoldStep) {
        uint4 e[kFoldPer];
        int cnt[kFoldPer];
#pragma unroll
        for (int r = 0; r < kFoldPer; ++r) {
          const int qq = q0 + r * kFoldHalves + half;
          cnt[r] = qq < nq ? lcnt[qq] : 0;
          e[r] = make_uint4(0, 0, 0, 0);
          if (4 * lt < cnt[r])
            e[r] = *reinterpret_cast<const uint4 *>(B.pool + (size_t)lpid[qq] * kBinPage + 4 * lt);
        }
#pragma unroll
        for (int r = 0; r < kFoldPer; ++r) {
          const uint32_t ev[4] = {e[r].x, e[r].y, e[r].z, e[r].w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (4 * lt + k < cnt[r]) {
              // atomics whose results are not used (no return, no wait):
              // testing the column first made every entry wait for an LDS
              // round trip, since an atomic on one entry may change the
              // column the next one reads
              const int c = (int)(ev[k] >> kBinYBits);
              const int y = (int)(ev[k] & ((1u << kBinYBits) - 1)) + 1;
              atomicMin(&sL[c].x, y);
              atomicMax(&sL[c].y, y);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  int2 *out = part + (size_t)s * (size_t)p + c0;
  for (int c = tid; c < ncol; c += kBinFoldThreads) out[c] = sL[c];
}

// Between rounds: the S_ partial arrays of the round just folded and the
// running L (array `at` of part; absent after the first round) folded into
// array `at`; the overflow flag of the next round's k_bin_compact cleared;
// and the filters of the next round: per group of 64 columns (one wave; F,
// for k_bin) and of 32 columns (F32, for k_bin_compact), the largest lo
// rounded up and the smallest hi rounded down to multiples of 2^qs in y - 1
// (8 bits each), or a range that holds nothing when a column of the group is
// empty or the lo bound does not fit 8 bits.
__global__ __launch_bounds__(256) void k_bin_merge(int2 *__restrict__ part, int32_t S_, int32_t has_prev, int32_t at,
                                                   Extent p, int32_t qs, uint16_t *__restrict__ F,
                                                   uint16_t *__restrict__ F32, int32_t *__restrict__ cover) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c == 0 && cover) *cover = 0;   // the next round's k_bin_compact starts with no overflow
  const int lane = threadIdx.x & (kWave - 1);
  int2 L = make_int2(p.q + 1, -1);
  if (c < p) {
    int2 a[8];
    int s = 0;
    for (; s + 8 <= S_; s += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = part[(size_t)(s + u) * p + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        L.x = min(L.x, a[u].x);
        L.y = max(L.y, a[u].y);
      }
    }
    for (; s < S_; ++s) {
      const int2 b = part[(size_t)s * p + c];
      L.x = min(L.x, b.x);
      L.y = max(L.y, b.y);
    }
    if (has_prev) {
      const int2 b = part[(size_t)at * p + c];
      L.x = min(L.x, b.x);
      L.y = max(L.y, b.y);
    }
    part[(size_t)at * p + c] = L;   // every array of this column was read above
  }
  const bool inside = c < p;
  const unsigned long long em = __ballot(inside && L.x > L.y);   // empty columns of the wave
  // lo bound rounded up and hi bound rounded down, never outwards; a group
  // with an empty column, or whose lo bound does not fit 8 bits, drops
  // nothing (lo bound 255 << qs, hi bound 0)
  auto word = [&](int mlo, int mhi, bool empty) -> uint16_t {
    if (empty) return 0xFFu;
    const unsigned qlo = ((unsigned)(mlo - 1) + (1u << qs) - 1) >> qs;
    const unsigned qhi = (unsigned)(mhi - 1) >> qs;
    return qlo <= 0xFFu ? (uint16_t)(qlo | (min(qhi, 0xFFu) << 8)) : (uint16_t)0xFFu;
  };
  int mlo = inside ? L.x : INT_MIN, mhi = inside ? L.y : INT_MAX;
#pragma unroll
  for (int d = kWave / 4; d > 0; d >>= 1) {   // each half wave: 32 columns
    mlo = max(mlo, __shfl_xor(mlo, d, kWave));
    mhi = min(mhi, __shfl_xor(mhi, d, kWave));
  }
  const int64_t g32 = c >> kCpFilterShift;
  if (F32 && (lane & 31) == 0 && (g32 << kCpFilterShift) < p)
    F32[g32] = word(mlo, mhi, ((em >> (lane & 32)) & 0xFFFFFFFFull) != 0);
  mlo = max(mlo, __shfl_xor(mlo, kWave / 2, kWave));
  mhi = min(mhi, __shfl_xor(mhi, kWave / 2, kWave));
  const int64_t grp = c >> kBinFilterShift;
  if (lane == 0 && (grp << kBinFilterShift) < p) F[grp] = word(mlo, mhi, em != 0);
}

}  // namespace hp
