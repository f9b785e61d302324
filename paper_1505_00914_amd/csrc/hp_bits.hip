// hp_bits.hip -- the bit array M and its w-ary tree on the device (w = 64):
// inserts of columns, and extraction of the set columns in ascending order.
//
// Layout (Discussion, extraction by an array of bits and by a tree
// structure): level 0 is the array itself, column i at bit (i-1) & 63 of
// word (i-1) >> 6.  A word of level k+1 holds one bit per word of level k,
// set when that word is non-zero; levels are added until one has a single
// word, and they are stored one after another, level 0 first.
//
// Insert: one device-scope OR per column into its level-0 word.  In the
// tree, the thread whose OR found the word empty (exactly one per word) goes
// on to the level above, so the upper levels see one OR per non-empty word,
// not one per column.  The bulk build (further down) gives the same words
// without device-scope atomics on level 0, by partitioning the columns by
// window and assembling each window in LDS.
//
// Extraction: three launches.  k_bits_count gives each workgroup of 128
// level-0 words its number of set bits, k_bits_scan turns those counts into
// output offsets, and k_bits_write expands the set bits of each word with
// the count-trailing-zeros loop of Table I into LDS and then copies the
// workgroup's columns out with coalesced stores.  With the tree, each wave
// reads the level-1 word over its 64 level-0 words first and reads only the
// non-empty ones; a wave whose level-1 word is zero reads nothing.
#include <climits>

#include "hp_host.h"
#include "hp_device.h"

namespace hp {

constexpr int kBitsBlock = 128;         // level-0 words per workgroup (two waves)
constexpr int kBitsScanBlock = 1024;
constexpr int kBitsMaxLevels = 8;

struct BitLevels {
  int64_t off[kBitsMaxLevels + 1];      // word offset of each level, total at [levels]
  int32_t levels;
};

static BitLevels bit_levels(int32_t p, int32_t tree) {
  BitLevels L{};
  int64_t words = ((int64_t)p + 63) / 64, at = 0;
  L.levels = 0;
  for (;;) {
    L.off[L.levels++] = at;
    at += words;
    if (!tree || words == 1) break;
    words = (words + 63) / 64;
  }
  L.off[L.levels] = at;
  return L;
}

__global__ void k_bits_fill(uint64_t *__restrict__ w, int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) w[i] = 0;
}

__global__ void k_bits_info(int32_t *info) {
  info[HP_INFO_STATUS] = HP_OK;
  info[HP_INFO_K] = 0;
}

template <bool TREE>
__global__ __launch_bounds__(256) void k_bits_insert(const int32_t *__restrict__ cols, int64_t s, int32_t p,
                                                     uint64_t *__restrict__ words, BitLevels L,
                                                     int32_t *__restrict__ info) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < s; j += stride) {
    const int32_t c = cols[j];
    if ((unsigned)(c - 1) >= (unsigned)p) {
      bad = true;
      continue;
    }
    uint64_t bit = (uint64_t)(c - 1);
    unsigned long long old = atomicOr((unsigned long long *)&words[bit >> 6], 1ull << (bit & 63));
    if (TREE) {
      for (int k = 1; k < L.levels && old == 0; ++k) {
        bit >>= 6;
        old = atomicOr((unsigned long long *)&words[L.off[k] + (bit >> 6)], 1ull << (bit & 63));
      }
    }
  }
  if (bad) info[HP_INFO_STATUS] = HP_ERANGE;
}

// The level-0 word w as extraction sees it: bits beyond p cleared, and with
// the tree, zero unless its bit in the level-1 word l1 is set.
template <bool TREE>
__device__ __forceinline__ uint64_t bits_leaf(const uint64_t *__restrict__ words, int64_t w, int64_t W0,
                                              uint64_t lastmask, uint64_t l1) {
  if (w >= W0) return 0;
  if (TREE && !((l1 >> (w & 63)) & 1)) return 0;
  const uint64_t v = __builtin_nontemporal_load(&words[w]);
  return w == W0 - 1 ? (v & lastmask) : v;
}

template <bool TREE>
__device__ __forceinline__ uint64_t bits_level1(const uint64_t *__restrict__ words, int64_t w, int64_t W0,
                                                int64_t off1) {
  // the level-1 word over the wave's 64 level-0 words (w is this lane's word)
  if (!TREE || W0 <= 1) return ~0ull;
  return words[off1 + (w >> 6)];
}

template <bool TREE>
__global__ __launch_bounds__(kBitsBlock) void k_bits_count(const uint64_t *__restrict__ words, int64_t W0,
                                                           uint64_t lastmask, int64_t off1,
                                                           int32_t *__restrict__ blockcnt) {
  __shared__ int s_part[kBitsBlock / kWave];
  const int64_t w = (int64_t)blockIdx.x * kBitsBlock + threadIdx.x;
  const int64_t wave0 = w & ~(int64_t)63;
  const uint64_t l1 = wave0 < W0 ? bits_level1<TREE>(words, w, W0, off1) : 0;
  int c = 0;
  if (l1) c = __popcll(bits_leaf<TREE>(words, w, W0, lastmask, l1));
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < kBitsBlock / kWave; ++i) t += s_part[i];
    blockcnt[blockIdx.x] = t;
  }
}

// One workgroup: exclusive offsets of the nb block counts, total at [nb].
__global__ __launch_bounds__(kBitsScanBlock) void k_bits_scan(const int32_t *__restrict__ blockcnt, int64_t nb,
                                                              int64_t *__restrict__ blockoff) {
  __shared__ int64_t s_sum[kBitsScanBlock];
  const int64_t per = (nb + kBitsScanBlock - 1) / kBitsScanBlock;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
  int64_t mine = 0;
  for (int64_t b = b0; b < b1; ++b) mine += blockcnt[b];
  s_sum[threadIdx.x] = mine;
  __syncthreads();
  for (int d = 1; d < kBitsScanBlock; d <<= 1) {  // Hillis-Steele over the thread sums
    const int64_t add = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0;
    __syncthreads();
    s_sum[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = s_sum[threadIdx.x] - mine;
  for (int64_t b = b0; b < b1; ++b) {
    blockoff[b] = run;
    run += blockcnt[b];
  }
  if (threadIdx.x == kBitsScanBlock - 1) blockoff[nb] = s_sum[threadIdx.x];
}

template <bool TREE>
__global__ __launch_bounds__(kBitsBlock) void k_bits_write(const uint64_t *__restrict__ words, int64_t W0,
                                                           uint64_t lastmask, int64_t off1,
                                                           const int64_t *__restrict__ blockoff, int64_t nb,
                                                           int32_t *__restrict__ cols, int32_t cap,
                                                           int32_t *__restrict__ info) {
  __shared__ int32_t s_out[kBitsBlock * 64];
  __shared__ int s_wave[kBitsBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t w = (int64_t)blockIdx.x * kBitsBlock + threadIdx.x;
  const int64_t wave0 = w & ~(int64_t)63;
  const uint64_t l1 = wave0 < W0 ? bits_level1<TREE>(words, w, W0, off1) : 0;
  uint64_t v = l1 ? bits_leaf<TREE>(words, w, W0, lastmask, l1) : 0;
  const int c = __popcll(v);
  int x = c;  // inclusive scan over the wave
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_wave[wave] = x;
  __syncthreads();
  int local = x - c, total = 0;
  for (int i = 0; i < kBitsBlock / kWave; ++i) {
    if (i < wave) local += s_wave[i];
    total += s_wave[i];
  }
  const int32_t base = (int32_t)(w * 64 + 1);
  // the set bits in ascending order (Table I's order): the position of the
  // lowest one, then that bit cleared (v & (v - 1))
  for (; v != 0; v &= v - 1) s_out[local++] = base + __builtin_ctzll(v);
  __syncthreads();
  const int64_t off = blockoff[blockIdx.x];
  // the run cols[off .. off + n), n = total clipped to cap: 4-byte stores
  // up to a 16-byte boundary of cols, 16-byte stores, 4-byte stores after
  const int n = (int)(off + total <= cap ? total : (cap > off ? cap - off : 0));
  const int head = (int)min<int64_t>(n, (4 - ((((uintptr_t)(cols + off)) >> 2) & 3)) & 3);
  const int nq = (n - head) >> 2;
  if (threadIdx.x < head) cols[off + threadIdx.x] = s_out[threadIdx.x];
  int4 *c4 = reinterpret_cast<int4 *>(cols + off + head);
  for (int q = threadIdx.x; q < nq; q += kBitsBlock) {
    const int i = head + 4 * q;
    c4[q] = make_int4(s_out[i], s_out[i + 1], s_out[i + 2], s_out[i + 3]);
  }
  for (int i = head + 4 * nq + threadIdx.x; i < n; i += kBitsBlock) cols[off + i] = s_out[i];
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) {
    const int64_t all = blockoff[nb];
    info[HP_INFO_K] = (int32_t)(all < INT_MAX ? all : INT_MAX);
    info[HP_INFO_STATUS] = all > cap ? HP_ECAPACITY : HP_OK;
  }
}

// ---------------------------------------------------------------------------
// Bulk build: the same result as the inserts, without device-scope atomics
// on level 0.  The columns are partitioned by window (a run of 64-word-aligned
// level-0 words) with a counting pass, a scan and a scatter; then one
// workgroup per window ORs its columns into an LDS bitmap and writes its
// words (old | new) with plain stores, and with a tree sets the level-1 words
// over them by ballot (a window owns whole level-1 words) and carries the
// non-zero level-1 words up with a few atomics.
// ---------------------------------------------------------------------------
constexpr int kPartBlock = 256;
constexpr int kPartMaxWinWords = 2048;   // level-0 words per window (16 KB of LDS)
constexpr int64_t kPartMaxHist = 262144;  // windows x chunks

struct PartShape {
  int32_t wshift;   // log2 of the columns per window
  int32_t nwin, nchunk;
  int64_t per;      // columns per chunk
  bool bulk;        // false: use the atomic inserts
};

static PartShape part_shape(int64_t s, int32_t p) {
  PartShape P{};
  const int64_t W0 = ((int64_t)p + 63) / 64;
  int64_t ww = 64;
  while (ww < kPartMaxWinWords && ww * 256 < W0) ww <<= 1;
  int sh = 0;
  while ((64ll << sh) < ww * 64) ++sh;
  P.wshift = 6 + sh;  // ww * 64 columns = 2^(6 + sh)
  P.nwin = (int32_t)((W0 + ww - 1) / ww);
  const int64_t want = (s + 4095) / 4096;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(1024, kPartMaxHist / P.nwin));
  P.nchunk = (int32_t)std::max<int64_t>(1, std::min(want, cap));
  P.per = (s + P.nchunk - 1) / P.nchunk;
  P.bulk = P.nwin >= 64 && s < (int64_t)INT_MAX && (int64_t)P.nwin <= 16384;
  return P;
}

__global__ __launch_bounds__(kPartBlock) void k_part_count(const int32_t *__restrict__ cols, int64_t s, int32_t p,
                                                           PartShape P, int32_t *__restrict__ hist,
                                                           int32_t *__restrict__ info) {
  extern __shared__ int32_t s_cnt[];
  for (int w = threadIdx.x; w < P.nwin; w += kPartBlock) s_cnt[w] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * P.per, j1 = j0 + P.per < s ? j0 + P.per : s;
  bool bad = false;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kPartBlock) {
    const int32_t c = cols[j];
    if ((unsigned)(c - 1) >= (unsigned)p) {
      bad = true;
      continue;
    }
    atomicAdd(&s_cnt[(unsigned)(c - 1) >> P.wshift], 1);
  }
  __syncthreads();
  for (int w = threadIdx.x; w < P.nwin; w += kPartBlock) hist[(int64_t)w * P.nchunk + blockIdx.x] = s_cnt[w];
  if (bad) info[HP_INFO_STATUS] = HP_ERANGE;
}

// One workgroup per window: exclusive offsets of the window's chunk counts
// within the window (loc), and the window's total (wtot).  The totals are
// then scanned by k_bits_scan into the windows' bases.
__global__ __launch_bounds__(kPartBlock) void k_part_scan_win(const int32_t *__restrict__ hist, int32_t nchunk,
                                                              int32_t *__restrict__ loc,
                                                              int32_t *__restrict__ wtot) {
  __shared__ int32_t s_sum[kPartBlock];
  const int64_t row = (int64_t)blockIdx.x * nchunk;
  const int per = (nchunk + kPartBlock - 1) / kPartBlock;  // at most 4
  const int j0 = threadIdx.x * per;
  int v[4] = {0, 0, 0, 0};
  int mine = 0;
  for (int u = 0; u < per; ++u)
    if (j0 + u < nchunk) {
      v[u] = hist[row + j0 + u];
      mine += v[u];
    }
  s_sum[threadIdx.x] = mine;
  __syncthreads();
  for (int d = 1; d < kPartBlock; d <<= 1) {
    const int add = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0;
    __syncthreads();
    s_sum[threadIdx.x] += add;
    __syncthreads();
  }
  int run = s_sum[threadIdx.x] - mine;
  for (int u = 0; u < per; ++u)
    if (j0 + u < nchunk) {
      loc[row + j0 + u] = run;
      run += v[u];
    }
  if (threadIdx.x == kPartBlock - 1) wtot[blockIdx.x] = s_sum[threadIdx.x];
}

__global__ __launch_bounds__(kPartBlock) void k_part_scatter(const int32_t *__restrict__ cols, int64_t s, int32_t p,
                                                             PartShape P, const int64_t *__restrict__ base,
                                                             const int32_t *__restrict__ loc,
                                                             int32_t *__restrict__ part) {
  extern __shared__ int32_t s_cur[];
  for (int w = threadIdx.x; w < P.nwin; w += kPartBlock) s_cur[w] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * P.per, j1 = j0 + P.per < s ? j0 + P.per : s;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kPartBlock) {
    const int32_t c = cols[j];
    if ((unsigned)(c - 1) >= (unsigned)p) continue;
    const int w = (int)((unsigned)(c - 1) >> P.wshift);
    const int k = atomicAdd(&s_cur[w], 1);
    part[base[w] + loc[(int64_t)w * P.nchunk + blockIdx.x] + k] = c;
  }
}

// The scatter with a local sort: each tile of kPartTile columns of the chunk
// is ordered by window in LDS (ranks from an LDS histogram, offsets from its
// scan), and then written out in that order, so that consecutive lanes
// store consecutive addresses of one window's run instead of 4 bytes each
// into many windows.  For at most kPartSortMaxWin windows.
constexpr int kPartTile = 2048;
constexpr int kPartSortMaxWin = 2048;
constexpr int kPartPerThread = kPartTile / kPartBlock;   // 8

__global__ __launch_bounds__(kPartBlock) void k_part_scatter_sorted(const int32_t *__restrict__ cols, int64_t s,
                                                                    int32_t p, PartShape P,
                                                                    const int64_t *__restrict__ base,
                                                                    const int32_t *__restrict__ loc,
                                                                    int32_t *__restrict__ part) {
  __shared__ int32_t s_cur[kPartSortMaxWin];    // columns of the chunk already written, per window
  __shared__ int32_t s_hist[kPartSortMaxWin];   // this tile's count, per window
  __shared__ int32_t s_toff[kPartSortMaxWin];   // this tile's first slot, per window
  __shared__ int32_t s_tile[kPartTile];
  __shared__ int32_t s_sum[kPartBlock];
  const int nw = P.nwin;
  for (int w = threadIdx.x; w < nw; w += kPartBlock) s_cur[w] = 0;
  const int64_t j0 = (int64_t)blockIdx.x * P.per, j1 = j0 + P.per < s ? j0 + P.per : s;
  for (int64_t t0 = j0; t0 < j1; t0 += kPartTile) {
    for (int w = threadIdx.x; w < nw; w += kPartBlock) s_hist[w] = 0;
    __syncthreads();
    int32_t c[kPartPerThread];
    int wv[kPartPerThread], rk[kPartPerThread];
#pragma unroll
    for (int u = 0; u < kPartPerThread; ++u) {
      const int64_t j = t0 + u * kPartBlock + threadIdx.x;
      c[u] = j < j1 ? cols[j] : 0;
      const bool ok = j < j1 && (unsigned)(c[u] - 1) < (unsigned)p;
      wv[u] = ok ? (int)((unsigned)(c[u] - 1) >> P.wshift) : -1;
      rk[u] = ok ? atomicAdd(&s_hist[wv[u]], 1) : 0;
    }
    __syncthreads();
    // exclusive scan of the tile's window counts: a run of windows per thread
    const int per = (nw + kPartBlock - 1) / kPartBlock;
    const int w0 = threadIdx.x * per;
    int mine = 0;
    for (int w = w0; w < w0 + per && w < nw; ++w) mine += s_hist[w];
    s_sum[threadIdx.x] = mine;
    __syncthreads();
    for (int d = 1; d < kPartBlock; d <<= 1) {
      const int add = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0;
      __syncthreads();
      s_sum[threadIdx.x] += add;
      __syncthreads();
    }
    int run = s_sum[threadIdx.x] - mine;
    for (int w = w0; w < w0 + per && w < nw; ++w) {
      s_toff[w] = run;
      run += s_hist[w];
    }
    const int valid = s_sum[kPartBlock - 1];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPartPerThread; ++u)
      if (wv[u] >= 0) s_tile[s_toff[wv[u]] + rk[u]] = c[u];
    __syncthreads();
    for (int i = threadIdx.x; i < valid; i += kPartBlock) {
      const int32_t cc = s_tile[i];
      const int w = (int)((unsigned)(cc - 1) >> P.wshift);
      part[base[w] + loc[(int64_t)w * P.nchunk + blockIdx.x] + s_cur[w] + (i - s_toff[w])] = cc;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nw; w += kPartBlock) s_cur[w] += s_hist[w];
  }
}

constexpr int kWinBlock = 1024;   // threads per window workgroup

template <bool TREE>
__global__ __launch_bounds__(kWinBlock) void k_part_window(const int32_t *__restrict__ part,
                                                            const int64_t *__restrict__ base, PartShape P,
                                                            int64_t W0, uint64_t *__restrict__ words,
                                                            BitLevels L) {
  __shared__ unsigned long long s_bm[kPartMaxWinWords];
  const int64_t ww = 1ll << (P.wshift - 6);
  const int64_t g0 = (int64_t)blockIdx.x * ww;
  for (int t = threadIdx.x; t < ww; t += kWinBlock) s_bm[t] = 0;
  __syncthreads();
  const int64_t i0 = base[blockIdx.x], i1 = base[blockIdx.x + 1];
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kWinBlock) {
    const uint32_t b = (uint32_t)(part[i] - 1);
    atomicOr(&s_bm[(int64_t)(b >> 6) - g0], 1ull << (b & 63));
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t t0 = 0; t0 < ww; t0 += kWinBlock) {
    const int64_t t = t0 + threadIdx.x, g = g0 + t;
    uint64_t v = 0;
    if (t < ww && g < W0) {
      v = words[g] | s_bm[t];
      words[g] = v;
    }
    if (TREE && L.levels > 1) {
      // a wave covers 64 consecutive level-0 words: one level-1 word
      const unsigned long long nz = __ballot(v != 0);
      const int64_t g1 = g >> 6;
      if (lane == 0 && t < ww && g < W0 && nz) {
        const uint64_t old = words[L.off[1] + g1];
        words[L.off[1] + g1] = old | nz;
        if (old == 0) {  // the level-1 word became non-zero: carry it up
          uint64_t bit = (uint64_t)g1;
          unsigned long long o = 0;
          for (int k = 2; k < L.levels && o == 0; ++k) {
            o = atomicOr((unsigned long long *)&words[L.off[k] + (bit >> 6)], 1ull << (bit & 63));
            bit >>= 6;
          }
        }
      }
    }
  }
}

static int64_t bits_blocks(int32_t p) {
  const int64_t W0 = ((int64_t)p + 63) / 64;
  return (W0 + kBitsBlock - 1) / kBitsBlock;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace hp

using namespace hp;

extern "C" int hp_bitset_words(int32_t p, int32_t tree, int64_t *words) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (!words) return set_error(HP_EINVAL, "words is NULL");
  *words = bit_levels(p, tree).off[bit_levels(p, tree).levels];
  return HP_OK;
}

extern "C" int hp_bitset_clear(uint64_t *words, int64_t nwords, void *stream) {
  if (nwords < 0) return set_error(HP_EINVAL, "nwords < 0");
  if (nwords == 0) return HP_OK;
  if (!words) return set_error(HP_EINVAL, "words is NULL");
  const int grid = (int)std::min<int64_t>(4 * device_info().cus, (nwords + 255) / 256);
  hipLaunchKernelGGL(k_bits_fill, dim3(grid), dim3(256), 0, (hipStream_t)stream, words, nwords);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bits_fill launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_bitset_insert(const int32_t *cols, int64_t s, int32_t p, int32_t tree, uint64_t *words,
                                int32_t *info, void *stream) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (s < 0) return set_error(HP_EINVAL, "s < 0");
  if ((s > 0 && !cols) || !words || !info) return set_error(HP_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_bits_info, dim3(1), dim3(1), 0, st, info);
  if (s > 0) {
    const BitLevels L = bit_levels(p, tree);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8 * device_info().cus, (s + 255) / 256));
    if (tree)
      hipLaunchKernelGGL(k_bits_insert<true>, dim3(grid), dim3(256), 0, st, cols, s, p, words, L, info);
    else
      hipLaunchKernelGGL(k_bits_insert<false>, dim3(grid), dim3(256), 0, st, cols, s, p, words, L, info);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bits_insert launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_bitset_extract_workspace_bytes(int32_t p, size_t *bytes) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  const int64_t nb = bits_blocks(p);
  *bytes = align256(sizeof(int32_t) * nb) + align256(sizeof(int64_t) * (nb + 1));
  return HP_OK;
}

extern "C" int hp_bitset_extract(const uint64_t *words, int32_t p, int32_t tree, int32_t *cols, int32_t cap,
                                 int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (!words || !info || !ws) return set_error(HP_EINVAL, "NULL argument");
  if (cap < 0 || (cap > 0 && !cols)) return set_error(HP_EINVAL, "bad output capacity");
  if ((uintptr_t)words & 7) return set_error(HP_EINVAL, "words is not 8-byte aligned");
  size_t need = 0;
  hp_bitset_extract_workspace_bytes(p, &need);
  if (ws_bytes < need) return set_error(HP_ECAPACITY, "workspace %zu < %zu bytes", ws_bytes, need);
  const int64_t W0 = ((int64_t)p + 63) / 64, nb = bits_blocks(p);
  const uint64_t lastmask = (p & 63) ? (1ull << (p & 63)) - 1 : ~0ull;
  const int64_t off1 = W0;  // level 1 follows level 0 in a tree
  int32_t *blockcnt = static_cast<int32_t *>(ws);
  int64_t *blockoff = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + align256(sizeof(int32_t) * nb));
  hipStream_t st = (hipStream_t)stream;
  if (tree) {
    hipLaunchKernelGGL(k_bits_count<true>, dim3(nb), dim3(kBitsBlock), 0, st, words, W0, lastmask, off1, blockcnt);
    hipLaunchKernelGGL(k_bits_scan, dim3(1), dim3(kBitsScanBlock), 0, st, (const int32_t *)blockcnt, nb, blockoff);
    hipLaunchKernelGGL(k_bits_write<true>, dim3(nb), dim3(kBitsBlock), 0, st, words, W0, lastmask, off1,
                       (const int64_t *)blockoff, nb, cols, cap, info);
  } else {
    hipLaunchKernelGGL(k_bits_count<false>, dim3(nb), dim3(kBitsBlock), 0, st, words, W0, lastmask, off1, blockcnt);
    hipLaunchKernelGGL(k_bits_scan, dim3(1), dim3(kBitsScanBlock), 0, st, (const int32_t *)blockcnt, nb, blockoff);
    hipLaunchKernelGGL(k_bits_write<false>, dim3(nb), dim3(kBitsBlock), 0, st, words, W0, lastmask, off1,
                       (const int64_t *)blockoff, nb, cols, cap, info);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "bit extraction launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_bitset_build_workspace_bytes(int64_t s, int32_t p, size_t *bytes) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (s < 0 || !bytes) return set_error(HP_EINVAL, "bad argument");
  const PartShape P = part_shape(s, p);
  const int64_t h = (int64_t)P.nwin * P.nchunk;
  *bytes = P.bulk ? align256(sizeof(int32_t) * (size_t)s) + 2 * align256(sizeof(int32_t) * (size_t)h) +
                        align256(sizeof(int32_t) * (size_t)P.nwin) + align256(sizeof(int64_t) * (size_t)(P.nwin + 1))
                  : 0;
  return HP_OK;
}

extern "C" int hp_bitset_build(const int32_t *cols, int64_t s, int32_t p, int32_t tree, uint64_t *words,
                               int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (s < 0) return set_error(HP_EINVAL, "s < 0");
  if ((s > 0 && !cols) || !words || !info) return set_error(HP_EINVAL, "NULL argument");
  const PartShape P = part_shape(s, p);
  if (!P.bulk || s == 0) return hp_bitset_insert(cols, s, p, tree, words, info, stream);
  size_t need = 0;
  hp_bitset_build_workspace_bytes(s, p, &need);
  if (!ws || ws_bytes < need) return set_error(HP_ECAPACITY, "workspace %zu < %zu bytes", ws_bytes, need);
  const int64_t h = (int64_t)P.nwin * P.nchunk;
  char *w = static_cast<char *>(ws);
  size_t at = 0;
  auto take = [&](size_t bytes) { char *q = w + at; at += align256(bytes); return q; };
  int32_t *part = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)s));
  int32_t *hist = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)h));
  int32_t *loc = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)h));
  int32_t *wtot = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)P.nwin));
  int64_t *base = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * (size_t)(P.nwin + 1)));
  const BitLevels L = bit_levels(p, tree);
  const int64_t W0 = ((int64_t)p + 63) / 64;
  const size_t lds = sizeof(int32_t) * (size_t)P.nwin;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_bits_info, dim3(1), dim3(1), 0, st, info);
  hipLaunchKernelGGL(k_part_count, dim3(P.nchunk), dim3(kPartBlock), lds, st, cols, s, p, P, hist, info);
  hipLaunchKernelGGL(k_part_scan_win, dim3(P.nwin), dim3(kPartBlock), 0, st, (const int32_t *)hist, P.nchunk, loc,
                     wtot);
  hipLaunchKernelGGL(k_bits_scan, dim3(1), dim3(kBitsScanBlock), 0, st, (const int32_t *)wtot, (int64_t)P.nwin,
                     base);
  if (P.nwin <= kPartSortMaxWin)
    hipLaunchKernelGGL(k_part_scatter_sorted, dim3(P.nchunk), dim3(kPartBlock), 0, st, cols, s, p, P,
                       (const int64_t *)base, (const int32_t *)loc, part);
  else
    hipLaunchKernelGGL(k_part_scatter, dim3(P.nchunk), dim3(kPartBlock), lds, st, cols, s, p, P,
                       (const int64_t *)base, (const int32_t *)loc, part);
  if (tree)
    hipLaunchKernelGGL(k_part_window<true>, dim3(P.nwin), dim3(kWinBlock), 0, st, (const int32_t *)part,
                       (const int64_t *)base, P, W0, words, L);
  else
    hipLaunchKernelGGL(k_part_window<false>, dim3(P.nwin), dim3(kWinBlock), 0, st, (const int32_t *)part,
                       (const int64_t *)base, P, W0, words, L);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "bulk build launch: %s", hipGetErrorString(e));
  return HP_OK;
}
