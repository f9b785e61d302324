// hp_single.hip -- single-cloud kernels and entry points of libhullprep.
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <cstring>

#include <hip/hip_ext.h>

#include "hp_host.h"
#include "hp_args.h"
#include "hp_output.h"
#include "hp_reduce.h"
#include "hp_binned.h"

namespace hp {

// ---------------------------------------------------------------------------
// L initialisation and control words
// ---------------------------------------------------------------------------
__global__ void k_init(int32_t *ctl, int32_t *tree_ctr, int32_t nodes, int32_t *info,
                       int32_t info_mode, int2 *L, Extent p) {
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
    for (int64_t c = i; c < p; c += stride) L[c] = make_int2(p.q + 1, -1);
}

// The sampled filter of the device-L reduce: per group of 2^fshift columns,
// (largest sampled lo, smallest sampled hi), or (q + 1, -1) when a column of
// the group has no sampled point (see k_reduce_filtered).
__global__ __launch_bounds__(256) void k_filter_build(const int2 *__restrict__ L, Extent p, int32_t fshift,
                                                      int32_t ngroups, int2 *__restrict__ F) {
  // a wave per group (up to 64 columns a pass)
  const int lane = threadIdx.x & (kWave - 1);
  const int g = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (g >= ngroups) return;
  const int64_t first = (int64_t)g << fshift;
  const int64_t last = min<int64_t>((int64_t)p, first + ((int64_t)1 << fshift));
  int mlo = INT_MIN, mhi = INT_MAX;
  bool empty = false;
  for (int64_t c = first + lane; c < last; c += kWave) {
    const int2 e = L[c];
    empty |= e.x > e.y;
    mlo = max(mlo, e.x);
    mhi = min(mhi, e.y);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mlo = max(mlo, __shfl_xor(mlo, d, kWave));
    mhi = min(mhi, __shfl_xor(mhi, d, kWave));
  }
  empty = __any(empty);
  if (lane == 0) F[g] = empty ? make_int2(p.q + 1, -1) : make_int2(mlo, mhi);
}

// ---------------------------------------------------------------------------
// Step 1 of the heuristic: the bounding box of the points.  One grid-stride
// pass, four 16-byte loads in flight per lane; every workgroup writes its
// (xmin, xmax, ymin, ymax) to part[workgroup] and k_bbox_fold folds them.
// ---------------------------------------------------------------------------
constexpr int kBoxBlock = 256;
constexpr int kBoxMaxGrid = 2048;

__device__ __forceinline__ void box_add(int4 &b, int x, int y) {
  b.x = min(b.x, x);
  b.y = max(b.y, x);
  b.z = min(b.z, y);
  b.w = max(b.w, y);
}

__device__ __forceinline__ int4 box_block(int4 b, int4 *s_part) {
  // (xmin, xmax, ymin, ymax) over the workgroup, valid in thread 0
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    b.x = min(b.x, __shfl_xor(b.x, d, kWave));
    b.y = max(b.y, __shfl_xor(b.y, d, kWave));
    b.z = min(b.z, __shfl_xor(b.z, d, kWave));
    b.w = max(b.w, __shfl_xor(b.w, d, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) s_part[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kBoxBlock / kWave; ++w) {
      const int4 o = s_part[w];
      b.x = min(b.x, o.x);
      b.y = max(b.y, o.y);
      b.z = min(b.z, o.z);
      b.w = max(b.w, o.w);
    }
  return b;
}

__global__ __launch_bounds__(kBoxBlock) void k_bbox(const int32_t *__restrict__ pts, int64_t n,
                                                    int4 *__restrict__ part) {
  __shared__ int4 s_part[kBoxBlock / kWave];
  int4 b = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (head) box_add(b, pts[0], pts[1]);
    if (head + 2 * nv < n) box_add(b, pts[2 * (head + 2 * nv)], pts[2 * (head + 2 * nv) + 1]);
  }
  const int64_t stride = (int64_t)gridDim.x * kBoxBlock;
  int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    int4 q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = load_stream(&v[i + u * stride]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      box_add(b, q[u].x, q[u].y);
      box_add(b, q[u].z, q[u].w);
    }
  }
  for (; i < nv; i += stride) {
    const int4 q = load_stream(&v[i]);
    box_add(b, q.x, q.y);
    box_add(b, q.z, q.w);
  }
  b = box_block(b, s_part);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(kBoxBlock) void k_bbox_fold(const int4 *__restrict__ part, int32_t nparts,
                                                         int32_t *__restrict__ box) {
  __shared__ int4 s_part[kBoxBlock / kWave];
  int4 b = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
  for (int i = threadIdx.x; i < nparts; i += kBoxBlock) {
    const int4 o = part[i];
    b.x = min(b.x, o.x);
    b.y = max(b.y, o.y);
    b.z = min(b.z, o.z);
    b.w = max(b.w, o.w);
  }
  b = box_block(b, s_part);
  if (threadIdx.x == 0) {
    box[0] = b.x;
    box[1] = b.y;
    box[2] = b.z;
    box[3] = b.w;
  }
}

// ---------------------------------------------------------------------------
// Float input (the scaling of floating-point data to integers): the box of
// float points, skipping points with a NaN coordinate, and the scaling
// X = floor((x - ox) * s) + 1 in double precision, one rounding per
// operation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void boxf_add(float4 &b, float x, float y) {
  if (x != x || y != y) return;
  b.x = fminf(b.x, x);
  b.y = fmaxf(b.y, x);
  b.z = fminf(b.z, y);
  b.w = fmaxf(b.w, y);
}

__device__ __forceinline__ float4 boxf_block(float4 b, float4 *s_part) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    b.x = fminf(b.x, __shfl_xor(b.x, d, kWave));
    b.y = fmaxf(b.y, __shfl_xor(b.y, d, kWave));
    b.z = fminf(b.z, __shfl_xor(b.z, d, kWave));
    b.w = fmaxf(b.w, __shfl_xor(b.w, d, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) s_part[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kBoxBlock / kWave; ++w) {
      const float4 o = s_part[w];
      b.x = fminf(b.x, o.x);
      b.y = fmaxf(b.y, o.y);
      b.z = fminf(b.z, o.z);
      b.w = fmaxf(b.w, o.w);
    }
  return b;
}

__global__ __launch_bounds__(kBoxBlock) void k_bbox_f32(const float2 *__restrict__ pts, int64_t n,
                                                        float4 *__restrict__ part) {
  __shared__ float4 s_part[kBoxBlock / kWave];
  float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  // two points per 16-byte load, four loads in flight per lane; an odd
  // leading point (8-byte aligned start) and an odd last point on their own
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const float4 *v = reinterpret_cast<const float4 *>(pts + head);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (head) boxf_add(b, pts[0].x, pts[0].y);
    if (head + 2 * nv < n) boxf_add(b, pts[head + 2 * nv].x, pts[head + 2 * nv].y);
  }
  const int64_t stride = (int64_t)gridDim.x * kBoxBlock;
  int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    float4 q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = v[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      boxf_add(b, q[u].x, q[u].y);
      boxf_add(b, q[u].z, q[u].w);
    }
  }
  for (; i < nv; i += stride) {
    const float4 q = v[i];
    boxf_add(b, q.x, q.y);
    boxf_add(b, q.z, q.w);
  }
  b = boxf_block(b, s_part);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(kBoxBlock) void k_bbox_fold_f32(const float4 *__restrict__ part, int32_t nparts,
                                                             float *__restrict__ box) {
  __shared__ float4 s_part[kBoxBlock / kWave];
  float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  for (int i = threadIdx.x; i < nparts; i += kBoxBlock) {
    const float4 o = part[i];
    b.x = fminf(b.x, o.x);
    b.y = fmaxf(b.y, o.y);
    b.z = fminf(b.z, o.z);
    b.w = fmaxf(b.w, o.w);
  }
  b = boxf_block(b, s_part);
  if (threadIdx.x == 0) {
    box[0] = b.x;
    box[1] = b.y;
    box[2] = b.z;
    box[3] = b.w;
  }
}

// Scaled coordinates must lie in [1, 2^31 - 2], the integer range of a point.
constexpr double kScaledMax = 2147483646.0;
__device__ __forceinline__ int32_t scale_one(float v, double o, double s, bool &bad) {
  const double t = floor(__dmul_rn(__dsub_rn((double)v, o), s));
  if (!(t >= 0.0 && t <= kScaledMax - 1.0)) {  // also catches NaN
    bad = true;
    return 0;
  }
  return (int32_t)t + 1;
}

__global__ void k_quantize_init(int32_t *info) { info[HP_INFO_STATUS] = HP_OK; }

__global__ __launch_bounds__(256) void k_quantize_f32(const float2 *__restrict__ pts, int64_t n, double ox, double oy,
                                                      double s, int2 *__restrict__ out, int32_t *__restrict__ info) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float2 q = pts[i];
    const int32_t x = scale_one(q.x, ox, s, bad);
    const int32_t y = scale_one(q.y, oy, s, bad);
    out[i] = make_int2(x, y);
  }
  if (bad) info[HP_INFO_STATUS] = HP_ERANGE;
}

// The second sweep: the reduced set of a chain turned into row points
// (y, x), two per column -- (lo, x) and (hi, x) -- so that Algorithm 1 run
// on them with rows for columns keeps, per row, the smallest and largest x.
// A column with lo == hi gives the same point twice, which changes no
// per-row extreme.
__global__ __launch_bounds__(256) void k_chain_transpose(const int32_t *__restrict__ cx,
                                                         const int32_t *__restrict__ clo,
                                                         const int32_t *__restrict__ chi, int32_t k,
                                                         int2 *__restrict__ out) {
  const int stride = gridDim.x * blockDim.x;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += stride) {
    const int32_t x = cx[t];
    out[2 * t] = make_int2(clo[t], x);
    out[2 * t + 1] = make_int2(chi[t], x);
  }
}

// Sweep axis (Results: sweeping along the shorter side keeps fewer points):
// the points with x and y exchanged, two points per 16-byte load and store;
// an odd leading point (8-byte aligned start) and an odd last point on their
// own.  pts and out must not overlap.
__global__ __launch_bounds__(256) void k_points_transpose(const int32_t *__restrict__ pts, int64_t n,
                                                          int32_t *__restrict__ out) {
  const int64_t head = (n > 0 && ((uintptr_t)pts & 15) != 0) ? 1 : 0;
  const int64_t nv = (n - head) >> 1;
  const int4 *v = reinterpret_cast<const int4 *>(pts + 2 * head);
  const bool out_aligned = (((uintptr_t)(out + 2 * head)) & 15) == 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    if (head) {
      out[0] = pts[1];
      out[1] = pts[0];
    }
    const int64_t t = head + 2 * nv;
    if (t < n) {
      out[2 * t] = pts[2 * t + 1];
      out[2 * t + 1] = pts[2 * t];
    }
  }
  for (int64_t i = i0; i < nv; i += stride) {
    const int4 q = load_stream(&v[i]);
    const int64_t o = 2 * head + 4 * i;
    if (out_aligned) {
      *reinterpret_cast<int4 *>(out + o) = make_int4(q.y, q.x, q.w, q.z);
    } else {
      out[o] = q.y;
      out[o + 1] = q.x;
      out[o + 2] = q.w;
      out[o + 3] = q.z;
    }
  }
}

// ---------------------------------------------------------------------------
// Finish: one workgroup per slab of 64 positions, of FB threads: 1024, or
// 256 when there are many slabs (the launch is then bound by how fast the
// dispatcher starts waves, not by the work of a slab).
// ---------------------------------------------------------------------------
constexpr int kFinBlock = 1024;
constexpr int kFinBlockMany = 256;

template <int FB>
struct FinishSharedT {
  int2 red[FB / kSlab][kSlab]; // partial-merge scratch
  int2 pt[2][kSlab];           // slab points: side 0 (x, lo), side 1 (x, -hi)
  int2 stage[2 * kSlab];       // slab hulls per side
  uint32_t keepw[FB / kWave];  // slab-hull keep bits, one per candidate of the wave
  unsigned long long valid;    // valid positions of the slab
  int tmp[FB / kWave + 1];
  int slab_cnt[2];
  int flag;
  int scan_carry;
  int folded;                  // chunks the reduce workgroups report (slab 0)
};
using FinishShared = FinishSharedT<kFinBlock>;

// Exclusive scan of n ints in place (by one workgroup of FB threads);
// returns the total.
template <int FB = kFinBlock>
__device__ int block_exclusive_scan(int32_t *a, int32_t n, int *s_tmp, int *s_carry) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += FB) {
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
    for (int j = 0; j < FB / kWave; ++j) {
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

// Merge the children of tree node (lev, j) for both sides; writes the node's
// hulls into cand buffer lev&1 (or, for the root, assembles the hull).
// Last-arriver test: the barrier completes every thread's stores, then one
// acquire-release increment publishes them (and, for the last arriver,
// makes every earlier arriver's stores visible to the whole workgroup).
// s_flag is an LDS word.
__device__ bool last_arrival_flag(int32_t *ctr, int expected, int *s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    // release only: an acquire costs every arriver an invalidation of its
    // XCD's L2, and only the last arriver reads what the others wrote
    const int old = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int last = (old == expected - 1) ? 1 : 0;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_flag = last;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <int FB>
__device__ bool last_arrival(int32_t *ctr, int expected, FinishSharedT<FB> &S) {
  return last_arrival_flag(ctr, expected, &S.flag);
}

// Exclusive scan of the slab counts into slab_off, the k and s totals and
// the range status, and (chain_inline) the chain itself: by one workgroup,
// the last slab to finish or the scan launch that follows the slab step.
template <int FB>
__device__ void scan_slabs(const FinishArgs &A, FinishSharedT<FB> &S) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int grp = tid / kWave;
  const int nslab = A.tree.size[1];
  if (tid == 0) S.flag = 0;
  // slab_off = exclusive scan of slab_k; k and s totals.  The counts,
  // the s parts and the error words are all loaded before any is used.
  int s_part = 0, err = 0;
  for (int i = tid; i < nslab || i < A.n_wg_err; i += FB) {
    const int kk = i < nslab ? A.slab_k[i] : 0;
    const int ss = i < nslab ? A.slab_s[i] : 0;
    const int ee = i < A.n_wg_err ? A.wg_err[i] : 0;
    if (i < nslab) A.slab_off[i] = kk;
    s_part += ss;
    err |= ee;
  }
  __syncthreads();
  const int k = block_exclusive_scan<FB>(A.slab_off, nslab, S.tmp, &S.scan_carry);
  // block sum of s
  for (int d = kWave / 2; d > 0; d >>= 1) s_part += __shfl_down(s_part, d, kWave);
  __syncthreads();
  if (lane == 0) S.tmp[grp] = s_part;
  __syncthreads();
  if (err) atomicOr(&S.flag, err);
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int w = 0; w < FB / kWave; ++w) s += S.tmp[w];
    A.info[HP_INFO_K] = k;
    A.info[HP_INFO_S] = s;
    report_reduce_errors(S.flag, A.info);
  }
  if (A.chain_inline) {
    // every wave writes the chain of up to 4 slabs per round, all loads first
    constexpr int kW = FB / kWave;
    for (int sl0 = grp; sl0 < nslab; sl0 += 4 * kW) {
      int2 Lv[4];
      int offv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sl = sl0 + u * kW;
        const int64_t pos = (int64_t)sl * kSlab + lane;
        Lv[u] = (sl < nslab && pos < A.p) ? A.Lm[pos] : make_int2(1, 0);
        offv[u] = sl < nslab ? A.slab_off[sl] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sl = sl0 + u * kW;
        const bool valid = sl < nslab && Lv[u].x <= Lv[u].y;
        int tot;
        const int r = wave_rank(valid, &tot);
        const int off = offv[u] + r;
        if (valid) {
          if (off < A.chain_cap) {
            A.cx_out[off] = sl * kSlab + lane + 1;
            A.clo_out[off] = Lv[u].x;
            A.chi_out[off] = Lv[u].y;
          } else {
            atomicMin(&A.info[HP_INFO_STATUS], HP_ECAPACITY);
          }
        }
      }
    }
  }
}

// Per-slab work of the finish step, for slab `slab` of the cloud described
// by A (the single-cloud kernel passes its block index, the batched kernel
// the slab of its work item).
template <int FROM_CHAIN, bool SMALL, int FB>
__device__ __forceinline__ void finish_body(const FinishArgs &A, FinishSharedT<FB> &S, const int slab) {
  constexpr int kFinGroups = FB / kSlab;   // partial-merge thread groups
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int grp = tid / kWave;
  const int64_t pos = (int64_t)slab * kSlab + lane;
  const bool inside = pos < A.positions;

  // ---- slab 0: the reduce's chunk accounting (loads issued with the fold's)
  const bool check = !FROM_CHAIN && slab == 0 && A.dyn_ctr != nullptr;
  int folded = 0;
  if (check) {
    if (tid == 0) S.folded = 0;
    for (int j = tid; j < A.n_wg_cnt; j += FB) folded += A.wg_cnt[j];
  }

  // ---- the slab's points --------------------------------------------------
  int x = 0, lo = 0, hi = -1;
  bool valid = false;
  if (!FROM_CHAIN) {
    int mlo = INT_MAX, mhi = INT_MIN;
    if (inside && A.packed) {
      const uint32_t *src = reinterpret_cast<const uint32_t *>(A.part) + pos;
      const int G = A.G;
      int g = grp;
      // kFinGroups threads per column, 16 independent loads in flight each
      for (; g + 15 * kFinGroups < G; g += 16 * kFinGroups) {
        uint32_t a[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = src[(size_t)(g + kFinGroups * u) * A.p];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int2 e = unpack_partial(a[u]);
          mlo = min(mlo, e.x);
          mhi = max(mhi, e.y);
        }
      }
      for (; g < G; g += kFinGroups) {
        const int2 e = unpack_partial(src[(size_t)g * A.p]);
        mlo = min(mlo, e.x);
        mhi = max(mhi, e.y);
      }
    } else if (inside) {
      const int2 *src = A.part + pos;
      for (int g = grp; g < A.G; g += kFinGroups) {
        const int2 a = src[(size_t)g * A.p];
        mlo = min(mlo, a.x);
        mhi = max(mhi, a.y);
      }
    }
    S.red[grp][lane] = make_int2(mlo, mhi);
    __syncthreads();
    if (check) {
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) folded += __shfl_xor(folded, d, kWave);
      if (lane == 0 && folded) atomicAdd(&S.folded, folded);
    }
    if (grp == 0) {
      for (int k = 1; k < kFinGroups; ++k) {
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
      if (lane == 0) S.valid = vm;
    }
  }
  __syncthreads();
  if (check && tid == 0) {
    // every chunk folded exactly once; the counter is zero again for the
    // next run that uses its slot
    if ((int64_t)S.folded != A.dyn_expect) atomicMin(&A.info[HP_INFO_STATUS], HP_EDEVICE);
    __hip_atomic_store(A.dyn_ctr, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // ---- slab hull: every valid point against the 63 others of its slab.
  // 128 candidates (64 positions x 2 sides), 8 lanes each; lane g of a
  // candidate's group checks positions g, g+8, ..., g+56, keeping the
  // steepest slope into v from the left and the flattest slope out of v to
  // the right; the group combines them and v is kept iff they make a strict
  // left turn (collinear points dropped, Appendix).  Branch-free selects.
  if (A.do_hull) {
    {
      constexpr int kG = FB / (2 * kSlab);   // lanes per candidate
      const unsigned long long vm = S.valid;
      const int cand = tid / kG, g = tid % kG;
      const int side = cand / kSlab, i = cand % kSlab;
      const int2 v = S.pt[side][i];
      int2 uL = v, wR = v;
      bool hasL = false, hasR = false;
      int2 pk[kSlab / kG];
#pragma unroll
      for (int k = 0; k < kSlab / kG; ++k) pk[k] = S.pt[side][g + k * kG];
#pragma unroll
      for (int k = 0; k < kSlab / kG; ++k) {
        const int jj = g + k * kG;
        const int2 u = pk[k];
        const bool ok = ((vm >> jj) & 1ull) != 0;
        const bool isL = ok & (jj < i), isR = ok & (jj > i);
        const bool tL = isL & (!hasL | steeper_left<SMALL>(u, uL, v));
        const bool tR = isR & (!hasR | flatter_right<SMALL>(u, wR, v));
        uL = tL ? u : uL;
        hasL |= tL;
        wR = tR ? u : wR;
        hasR |= tR;
      }
#pragma unroll
      for (int d = kG / 2; d > 0; d >>= 1) {
        const int2 ou = make_int2(__shfl_xor(uL.x, d, kWave), __shfl_xor(uL.y, d, kWave));
        const int2 ow = make_int2(__shfl_xor(wR.x, d, kWave), __shfl_xor(wR.y, d, kWave));
        const bool ohL = __shfl_xor((int)hasL, d, kWave) != 0;
        const bool ohR = __shfl_xor((int)hasR, d, kWave) != 0;
        const bool tL = ohL & (!hasL | steeper_left<SMALL>(ou, uL, v));
        const bool tR = ohR & (!hasR | flatter_right<SMALL>(ow, wR, v));
        uL = tL ? ou : uL;
        hasL |= tL;
        wR = tR ? ow : wR;
        hasR |= tR;
      }
      const bool keep = (((vm >> i) & 1ull) != 0) & (!hasL | !hasR | cross_pos<SMALL>(uL, v, wR));
      // ballot over the wave: its 8 candidates' keep bits at lanes 0, 8, ...
      const unsigned long long kb = __ballot(keep && g == 0);
      if (lane == 0) {
        unsigned bits = 0;
#pragma unroll
        for (int q = 0; q < kWave / kG; ++q) bits |= (unsigned)((kb >> (q * kG)) & 1ull) << q;
        S.keepw[grp] = bits;
      }
    }
    __syncthreads();
    if (grp < 2) {
      // wave `side` compacts its side: position lane kept iff bit set
      const int side = grp;
      const int bitpos = side * kSlab + lane;   // candidate index
      constexpr int kG = FB / (2 * kSlab);
      constexpr int kPerWave = kWave / kG;      // candidates per wave
      const bool keep = (S.keepw[bitpos / kPerWave] >> (bitpos % kPerWave)) & 1u;
      int tot;
      const int rk = wave_rank(keep, &tot);
      if (keep) S.stage[side * kSlab + rk] = S.pt[side][lane];
      if (lane == 0) S.slab_cnt[side] = tot;
    }
    __syncthreads();
    if (grp < 2) {
      const int side = grp;
      const int tot = S.slab_cnt[side];
      if (A.tree.nlev > 1) {
        int2 *dst = A.cand + (size_t)side * (size_t)A.positions + (size_t)slab * kSlab;
        if (lane < tot) dst[lane] = S.stage[side * kSlab + lane];
        if (lane == 0) A.ccount[side * A.tree.nodes + slab] = tot;
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

  // ---- last slab: scan the slab counts (when the chain is not written by
  // the first hull level and no scan launch follows) ---------------------------
  if (!FROM_CHAIN && A.scan_root) {
    if (last_arrival(&A.ctl[kCtlSlabsDone], A.tree.size[1], S)) {
      __syncthreads();
      scan_slabs(A, S);
    }
  }
}

template <int FROM_CHAIN, bool SMALL, int FB = kFinBlock>
__global__ __launch_bounds__(FB) void k_finish(FinishArgs A) {
  __shared__ FinishSharedT<FB> S;
  finish_body<FROM_CHAIN, SMALL, FB>(A, S, blockIdx.x);
}

// The slab scan as a launch of its own (many slabs: one last-arriver count
// per slab would serialise thousands of device-scope atomics on one word).
__global__ __launch_bounds__(kFinBlock) void k_slab_scan(FinishArgs A) {
  __shared__ FinishShared S;
  scan_slabs(A, S);
}

// ---------------------------------------------------------------------------
// Hull levels above the slabs.  Level l has one node per kFanIn nodes of
// level l-1; a node's hull is the lower hull (per side) of its children's
// hulls.  kSplit workgroups per child test the child's vertices, one
// wavefront per vertex: lane t finds the tangent point on sibling t (binary
// search), lane j (the vertex's own child) contributes its neighbours, and a
// shuffle reduction yields the steepest slope in and the flattest slope out;
// the vertex survives iff they make a strict left turn.  The survivors of all
// siblings, in order, are exactly the parent's hull; the last workgroup of
// the parent to finish writes it (or, at the root, the final vertex list).
// Hulls of level-l nodes live in buffer (l-1)&1, compacted at the node's
// first position, lower side then upper side (y negated).
// ---------------------------------------------------------------------------
constexpr int kHullBlock = 1024;
constexpr int kWaves = kHullBlock / kWave;      // candidates per round
constexpr int kStage = 4096;                    // sibling vertices per side in LDS
constexpr int kTestLanes = 16;                  // lanes per tested vertex, at most

// Copy `total` pairs laid out as nseg segments (segment t: cnt[t] pairs at
// src + seg_pos(t)) into dst[0..total), where cs[t] is the prefix of cnt.
// Each thread resolves all of its (at most kBatch) elements and issues every
// load before storing: one memory latency instead of one per element.
template <int BLOCK, int kBatch, typename SegPos>
__device__ __forceinline__ void gather_segments(int2 *dst, const int2 *src, const int *cs, int nseg,
                                                int total, SegPos seg_pos) {
  for (int base = 0; base < total; base += BLOCK * kBatch) {
    int2 v[kBatch];
    int q[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      q[u] = base + u * BLOCK + (int)threadIdx.x;
      if (q[u] < total) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (cs[mid] <= q[u]) lo = mid;
          else hi = mid - 1;
        }
        v[u] = src[seg_pos(lo) + (size_t)(q[u] - cs[lo])];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (q[u] < total) dst[q[u]] = v[u];
  }
}

struct HullShared {
  int2 stage[2][kStage];
  uint32_t keepw[kStage / 2];      // keep bytes of 64 slots of 64 positions
  int cs[2][kFanIn], cc[2][kFanIn];
  int total[2];
  int wsum[kWaves];
  int sum[3];
  int carry;
};

// Wave-wide combine of each lane's steepest-left / flattest-right extreme
// for the wave's candidate v; true iff v is a strict lower-hull vertex.
template <bool SMALL>
__device__ __forceinline__ bool wave_extremes_keep(int2 v, int2 uL, bool hasL, int2 wR, bool hasR,
                                                   int width = kWave) {
#pragma unroll 1
  for (int d = width / 2; d > 0; d >>= 1) {
    const int2 ou = make_int2(__shfl_xor(uL.x, d, kWave), __shfl_xor(uL.y, d, kWave));
    const int2 ow = make_int2(__shfl_xor(wR.x, d, kWave), __shfl_xor(wR.y, d, kWave));
    const bool ohL = __shfl_xor((int)hasL, d, kWave) != 0;
    const bool ohR = __shfl_xor((int)hasR, d, kWave) != 0;
    // branch-free: both tests are plain integer arithmetic
    const bool tL = ohL & (!hasL | steeper_left<SMALL>(ou, uL, v));
    const bool tR = ohR & (!hasR | flatter_right<SMALL>(ow, wR, v));
    uL = make_int2(tL ? ou.x : uL.x, tL ? ou.y : uL.y);
    wR = make_int2(tR ? ow.x : wR.x, tR ? ow.y : wR.y);
    hasL |= tL;
    hasR |= tR;
  }
  return !hasL | !hasR | cross_pos<SMALL>(uL, v, wR);
}

// Sizes and prefixes of the children of `parent` at level lev-1, both sides
// (waves 0 and 1).
__device__ __forceinline__ void load_children(const HullArgs &H, HullShared &S, int lev, int sib0,
                                              int nsib) {
  const TreeShape &T = H.tree;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  if (wave < 2) {
    const int side = wave;
    const int m = lane < nsib ? H.ccount[side * T.nodes + T.base[lev - 1] + sib0 + lane] : 0;
    int incl = m;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    if (lane < nsib) { S.cc[side][lane] = m; S.cs[side][lane] = incl - m; }
    if (lane == kWave - 1) S.total[side] = incl;
  }
}

// Copy the nsib child slots (span positions each, both sides) into LDS as
// they lie in device memory: all loads first, then the stores.
__device__ __forceinline__ void stage_whole(HullShared &S, const int2 *in, int64_t P, int sib0,
                                            int nsib, int span) {
  constexpr int kPer = 2 * kStage / kHullBlock;
  int2 v[kPer];
  const int n = nsib * span;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = (int)threadIdx.x + u * kHullBlock;
    const int side = idx / kStage, rem = idx % kStage;
    if (rem < n && (int64_t)sib0 * span + rem < P) v[u] = in[(size_t)side * P + (size_t)sib0 * span + rem];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = (int)threadIdx.x + u * kHullBlock;
    const int side = idx / kStage, rem = idx % kStage;
    if (rem < n && (int64_t)sib0 * span + rem < P) S.stage[side][rem] = v[u];
  }
}

// Level test: kSplit workgroups per child node of level lev-1 decide, for
// each of the child's hull vertices, whether it survives among its siblings.
template <bool SMALL>
__device__ __forceinline__ void hull_test_body(const HullArgs &H, HullShared &S, const int lev,
                                               const int item) {
  const TreeShape &T = H.tree;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int c = item / H.split;             // child node at level lev-1
  const int part = item % H.split;
  const int parent = c / kFanIn;
  const int sib0 = parent * kFanIn;
  const int nsib = min(kFanIn, T.size[lev - 1] - sib0);
  const int j = c - sib0;
  const int64_t P = H.positions;
  const size_t span_c = (size_t)T.span[lev - 1];
  const int2 *in = H.buf[(lev - 2) & 1];

  // Siblings' vertices in LDS.  When all of their slots fit (first level:
  // 64-position children), the slots are copied whole, position-indexed, in
  // the same round of loads as the counts; otherwise the counts come first
  // and the vertices are packed, or read in place when even that overflows.
  const bool whole = (size_t)nsib * span_c <= (size_t)kStage;
  if (whole) stage_whole(S, in, P, sib0, nsib, (int)span_c);
  load_children(H, S, lev, sib0, nsib);
  __syncthreads();
  bool staged = whole;
  if (!whole) {
    staged = S.total[0] <= kStage && S.total[1] <= kStage;
    if (staged)
      for (int side = 0; side < 2; ++side)
        gather_segments<kHullBlock, kStage / kHullBlock>(
            S.stage[side], in + (size_t)side * P, S.cs[side], nsib, S.total[side],
            [&](int t) { return (size_t)(sib0 + t) * span_c; });
    __syncthreads();
  }
  auto child_ptr = [&](int side, int t) -> const int2 * {
    if (whole) return S.stage[side] + (size_t)t * span_c;
    return staged ? S.stage[side] + S.cs[side][t] : in + (size_t)side * P + (size_t)(sib0 + t) * span_c;
  };

  // this workgroup's share of the child's vertices: index q runs over the
  // lower side then the upper side; `width` lanes per vertex (the sibling
  // count rounded up to a power of two, at most kTestLanes), lane t of a
  // vertex's group taking siblings t, t + width, ...
  const int n0 = S.cc[0][j], n1 = S.cc[1][j];
  const int nq = n0 + n1;
  uint8_t *keep = H.keep + (size_t)c * span_c * 2;
  int width = 1;
  while (width < nsib && width < kTestLanes) width <<= 1;
  const int per_wave = kWave / width;
  const int t0 = lane & (width - 1);
  for (int q0 = (part * kWaves + wave) * per_wave; q0 < nq; q0 += H.split * kWaves * per_wave) {
    const int q = q0 + lane / width;
    const bool on = q < nq;
    const int side = q < n0 ? 0 : 1;
    const int r = side ? q - n0 : q;
    const int *cc = S.cc[side];
    const int2 *own = child_ptr(side, j);
    const int2 v = on ? own[r] : make_int2(0, 0);
    int2 uL = v, wR = v;
    bool hasL = false, hasR = false;
    for (int t = t0; on && t < nsib; t += width) {
      int2 u = v, w = v;
      bool hu = false, hw = false;
      if (t == j) {
        if (r > 0) { u = own[r - 1]; hu = true; }
        if (r + 1 < cc[j]) { w = own[r + 1]; hw = true; }
      } else if (cc[t] > 0) {
        const int2 *a = child_ptr(side, t);
        if (t < j) { u = a[tangent_left<SMALL>(a, cc[t], v)]; hu = true; }
        else { w = a[tangent_right<SMALL>(a, cc[t], v)]; hw = true; }
      }
      const bool tL = hu & (!hasL | steeper_left<SMALL>(u, uL, v));
      const bool tR = hw & (!hasR | flatter_right<SMALL>(w, wR, v));
      uL = tL ? u : uL;
      hasL |= tL;
      wR = tR ? w : wR;
      hasR |= tR;
    }
    const bool k = wave_extremes_keep<SMALL>(v, uL, hasL, wR, hasR, width);
    if (on && t0 == 0) keep[q] = k ? 1 : 0;
  }
}

// Level compaction: one workgroup per parent concatenates its children's
// surviving vertices in order (the parent's hull); the root assembles the
// final vertex list.  Survivors never move to a higher index, so the root
// compacts in place in LDS.
template <bool SMALL>
__global__ __launch_bounds__(kHullBlock) void k_hull_test(HullArgs H, int lev) {
  __shared__ HullShared S;
  hull_test_body<SMALL>(H, S, lev, blockIdx.x);
}

template <bool SMALL>
__device__ __forceinline__ void hull_compact_body(const HullArgs &H, HullShared &S, const int lev,
                                                  const int parent) {
  const TreeShape &T = H.tree;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int sib0 = parent * kFanIn;
  const int nsib = min(kFanIn, T.size[lev - 1] - sib0);
  const int64_t P = H.positions;
  const size_t span_c = (size_t)T.span[lev - 1];
  const size_t span_p = (size_t)T.span[lev];
  const int2 *in = H.buf[(lev - 2) & 1];
  int2 *out = H.buf[(lev - 1) & 1];
  const bool root = lev == T.nlev;

  const bool whole = (size_t)nsib * span_c <= (size_t)kStage && span_c <= 64;
  if (whole) {
    // child slots and their keep bytes, one round of loads
    stage_whole(S, in, P, sib0, nsib, (int)span_c);
    const uint32_t *kw = reinterpret_cast<const uint32_t *>(H.keep + (size_t)sib0 * span_c * 2);
    const int64_t first = (int64_t)sib0 * (int64_t)span_c * 2;
    const int nw = (int)((std::min<int64_t>(first + (int64_t)nsib * span_c * 2, 2 * P) - first + 3) / 4);
    for (int i = tid; i < nw; i += kHullBlock) S.keepw[i] = kw[i];
  }
  load_children(H, S, lev, sib0, nsib);
  __syncthreads();
  const bool in_lds = root && (whole || (S.total[0] <= kStage && S.total[1] <= kStage));
  int nkeep[2];
  if (whole) {
    // in-LDS ordered compaction: thread i owns child i/16's positions
    // 4*(i%16) .. +3 (64-position slots), per side
    const unsigned char *kb = reinterpret_cast<const unsigned char *>(S.keepw);
    for (int side = 0; side < 2; ++side) {
      const int t = tid / 16, r0 = (tid % 16) * 4;
      int2 vv[4];
      bool kf[4];
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + u;
        kf[u] = false;
        if (t < nsib && r < S.cc[side][t]) {
          kf[u] = kb[t * span_c * 2 + (side ? S.cc[0][t] : 0) + r] != 0;
          vv[u] = S.stage[side][t * span_c + r];
        }
        cnt += kf[u] ? 1 : 0;
      }
      // block exclusive scan of cnt (thread order = (child, position) order)
      int incl = cnt;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
      }
      if (lane == kWave - 1) S.wsum[wave] = incl;
      __syncthreads();
      int off = 0, all = 0;
      for (int w = 0; w < kWaves; ++w) {
        if (w < wave) off += S.wsum[w];
        all += S.wsum[w];
      }
      off += incl - cnt;
      __syncthreads();  // every survivor read before any is written back
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!kf[u]) continue;
        if (in_lds) S.stage[side][off] = vv[u];
        else out[(size_t)side * P + (size_t)parent * span_p + off] = vv[u];
        ++off;
      }
      nkeep[side] = all;
      if (tid == 0) H.ccount[side * T.nodes + T.base[lev] + parent] = all;
      __syncthreads();
    }
  } else {
  for (int side = 0; side < 2; ++side) {
    const int total = S.total[side];
    if (tid == 0) S.carry = 0;
    __syncthreads();
    for (int base = 0; base < total; base += kHullBlock) {
      const int q = base + tid;
      bool kf = false;
      int2 v = make_int2(0, 0);
      if (q < total) {
        int lo = 0, hi = nsib - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (S.cs[side][mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        const int r = q - S.cs[side][lo];
        const size_t cpos = (size_t)(sib0 + lo) * span_c;
        kf = H.keep[cpos * 2 + (side ? S.cc[0][lo] : 0) + r] != 0;
        v = in[(size_t)side * P + cpos + r];
      }
      int wt;
      const int wr = wave_rank(kf, &wt);
      if (lane == 0) S.wsum[wave] = wt;
      __syncthreads();
      int off = S.carry, all = 0;
      for (int w = 0; w < kWaves; ++w) {
        if (w < wave) off += S.wsum[w];
        all += S.wsum[w];
      }
      if (kf) {
        if (in_lds) S.stage[side][off + wr] = v;
        else out[(size_t)side * P + (size_t)parent * span_p + off + wr] = v;
      }
      __syncthreads();
      if (tid == 0) S.carry += all;
      __syncthreads();
    }
    nkeep[side] = S.carry;
    if (tid == 0) H.ccount[side * T.nodes + T.base[lev] + parent] = S.carry;
    __syncthreads();
  }
  }
  if (root) {
    bool overflow = false;
    const int2 *low = in_lds ? S.stage[0] : out;
    const int2 *upn = in_lds ? S.stage[1] : out + P;
    const int h = assemble_hull(low, nkeep[0], upn, nkeep[1], H.hx, H.hy, H.hull_cap, overflow);
    if (tid == 0) {
      H.info[HP_INFO_H] = overflow ? 0 : h;
      if (overflow) atomicMin(&H.info[HP_INFO_STATUS], HP_ECAPACITY);
    }
  }
}

template <bool SMALL>
__global__ __launch_bounds__(kHullBlock) void k_hull_compact(HullArgs H, int lev) {
  __shared__ HullShared S;
  hull_compact_body<SMALL>(H, S, lev, blockIdx.x);
}

// Chain write for large p: one wave per slab, at the scanned offset.
__global__ __launch_bounds__(256) void k_chain(const int2 *__restrict__ Lm, int32_t p,
                                               const int32_t *__restrict__ slab_off, int32_t nslab,
                                               int32_t *cx, int32_t *clo, int32_t *chi,
                                               int32_t cap, int32_t *info) {
  const int slab = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (slab >= nslab) return;
  write_chain_slab(Lm, p, slab_off, slab, cx, clo, chi, cap, info);
}

// ---------------------------------------------------------------------------
// Level 2 of every cloud with more than one slab.  A level-2 node's
// slab-hull vertices (at most 64 x 64 per side) are staged compacted, in x
// order, in LDS.  Every vertex v is then tested against all the node's other
// vertices of its side at once: with uL the one left of v that maximises
// slope(uL, v) and wR the one right of v that minimises slope(v, wR), v is a
// strict lower-hull vertex iff (uL, v, wR) turns strictly left (or one of
// them does not exist).  Exact integer comparisons throughout.  The test
// launch also writes the chain; the compaction launch keeps the survivors
// in order (the node's hulls), assembles the final hull at the root and
// writes k, s and the range status.
// ---------------------------------------------------------------------------
constexpr int kL2MaxSlabs = 1024;            // chain offsets summed in-kernel up to here
constexpr int kNodeVerts = kFanIn * kSlab;   // 4096 positions per level-2 node
constexpr int kL2Waves = kHullBlock / kWave; // one tested vertex per wave

constexpr int kL2MaxParts = 128;             // test workgroups per node, at most
constexpr int kL2TargetWgs = 512;            // test workgroups per launch, about

struct L2Shared {
  int2 P[2][kNodeVerts];     // the node's vertices per side, compacted in x order
  int cnt[2][kFanIn];        // per slab: hull size
  int off[2][kFanIn + 1];    // per slab: first compacted index (off[.][64] = count)
  int soff[2][kL2MaxParts + 1];  // per test share: first survivor index
  uint32_t keepw[2][kNodeVerts / 4];
  int tmp[kL2Waves];
  int sum[3];
};

// The node's slots (every position of its slabs, both sides) and the slab
// hull sizes in one round of loads (and, with KEEP, the survival bytes of
// the compacted vertices), then the vertices compacted in place in x order.
template <bool KEEP>
__device__ __forceinline__ void l2_stage(const HullArgs &H, L2Shared &S, int node) {
  constexpr int kPer = 2 * kNodeVerts / kHullBlock;   // 8 slots per thread
  const TreeShape &T = H.tree;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int sib0 = node * kFanIn, nsib = min(kFanIn, T.size[1] - sib0);
  const int64_t P = H.positions;
  const int64_t first = (int64_t)sib0 * kSlab;
  const int2 *in = H.buf[0];
  int2 v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = tid + u * kHullBlock;
    const int side = idx / kNodeVerts, pos = idx % kNodeVerts;
    if (first + pos < P) v[u] = in[(size_t)side * P + first + pos];
  }
  int m = 0;
  if (wave < 2 && lane < nsib) m = H.ccount[wave * T.nodes + T.base[1] + sib0 + lane];
  // survival bytes: kNodeVerts per side, as words, two per thread
  uint32_t kw[2] = {0, 0};
  if (KEEP) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = tid + u * kHullBlock;
      const int side = idx / (kNodeVerts / 4), w = idx % (kNodeVerts / 4);
      kw[u] = reinterpret_cast<const uint32_t *>(H.keep + (size_t)side * H.keep_side + (size_t)node * kNodeVerts)[w];
    }
  }
  if (wave < 2) {
    int incl = m;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    S.cnt[wave][lane] = m;
    S.off[wave][lane] = incl - m;
    if (lane == kWave - 1) S.off[wave][kFanIn] = incl;
  }
  if (KEEP) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = tid + u * kHullBlock;
      S.keepw[idx / (kNodeVerts / 4)][idx % (kNodeVerts / 4)] = kw[u];
    }
  }
  __syncthreads();
  // every slot's destination first, then the stores.  Slot u of this thread
  // is position lane of slab wave + 16 (u % 4) on side u / 4: the slab is
  // uniform over the wave, so each lane reads slab `lane`'s count and offset
  // once and the wave picks its four with readlane
  static_assert(kHullBlock == 16 * kWave && kPer == 8, "stage layout");
  const int cl[2] = {S.cnt[0][lane], S.cnt[1][lane]};   // written for all 64 slabs
  const int ol[2] = {S.off[0][lane], S.off[1][lane]};
  int dst[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int side = u / 4, t = wave + 16 * (u % 4);
    const int c = __builtin_amdgcn_readlane(cl[side], t), o = __builtin_amdgcn_readlane(ol[side], t);
    dst[u] = (t < nsib && lane < c) ? o + lane : -1;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int side = (tid + u * kHullBlock) / kNodeVerts;
    if (dst[u] >= 0) S.P[side][dst[u]] = v[u];
  }
  __syncthreads();
}

// Chain of slab `sl` by one wave, without barriers: its offset is the
// scanned one when the slab-finish step scanned (many slabs), else the sum
// of the counts of every earlier slab (at most kL2MaxSlabs).
__device__ __forceinline__ void l2_chain_slab(const HullArgs &H, int sl) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t pos = (int64_t)sl * kSlab + lane;
  const int2 L = pos < H.p ? H.Lm[pos] : make_int2(1, 0);
  int base = 0;
  if (H.slab_off) {
    base = H.slab_off[sl];
  } else {
    for (int j = lane; j < sl; j += kWave) base += H.slab_k[j];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) base += __shfl_xor(base, d, kWave);
  }
  const bool valid = L.x <= L.y;
  int tot;
  const int r = wave_rank(valid, &tot);
  if (valid) {
    const int o = base + r;
    if (o < H.chain_cap) {
      H.cx[o] = (int)pos + 1;
      H.clo[o] = L.x;
      H.chi[o] = L.y;
    } else {
      atomicMin(&H.info[HP_INFO_STATUS], HP_ECAPACITY);
    }
  }
}

// k, s and the range status of the whole cloud (one workgroup).
__device__ __forceinline__ void l2_totals(const HullArgs &H, L2Shared &S) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  if (tid < 3) S.sum[tid] = 0;
  __syncthreads();
  int kk = 0, ss = 0, err = 0;
  for (int j = tid; j < H.tree.size[1]; j += kHullBlock) {
    kk += H.slab_k[j];
    ss += H.slab_s[j];
  }
  for (int j = tid; j < H.n_wg_err; j += kHullBlock) err |= H.wg_err[j];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    kk += __shfl_xor(kk, d, kWave);
    ss += __shfl_xor(ss, d, kWave);
    err |= __shfl_xor(err, d, kWave);
  }
  if (lane == 0) {
    atomicAdd(&S.sum[0], kk);
    atomicAdd(&S.sum[1], ss);
    if (err) atomicOr(&S.sum[2], err);
  }
  __syncthreads();
  if (tid == 0) {
    H.info[HP_INFO_K] = S.sum[0];
    H.info[HP_INFO_S] = S.sum[1];
    report_reduce_errors(S.sum[2], H.info);
  }
}

// One step of a wave reduction: every lane receives the value of the lane
// selected by the DPP control CTRL (rows outside ROWS keep their own).
template <int CTRL, int ROWS>
__device__ __forceinline__ int2 dpp_pair(int2 a) {
  return make_int2(__builtin_amdgcn_update_dpp(a.x, a.x, CTRL, ROWS, 0xf, false),
                   __builtin_amdgcn_update_dpp(a.y, a.y, CTRL, ROWS, 0xf, false));
}

// Wave-wide reduction of a point by an idempotent choice `pick` (quad
// swaps, rotations by 4 and 8 within each row of 16, then the last lane of
// each row carried to the next rows); the result, read from lane 63, is
// uniform.
template <typename Pick>
__device__ __forceinline__ int2 wave_pick(int2 a, Pick pick) {
  a = pick(a, dpp_pair<0xb1, 0xf>(a));    // quad_perm 1,0,3,2
  a = pick(a, dpp_pair<0x4e, 0xf>(a));    // quad_perm 2,3,0,1
  a = pick(a, dpp_pair<0x124, 0xf>(a));   // row_ror 4
  a = pick(a, dpp_pair<0x128, 0xf>(a));   // row_ror 8
  a = pick(a, dpp_pair<0x142, 0xa>(a));   // row_bcast 15 into rows 1 and 3
  a = pick(a, dpp_pair<0x143, 0xc>(a));   // row_bcast 31 into rows 2 and 3
  return make_int2(__builtin_amdgcn_readlane(a.x, 63), __builtin_amdgcn_readlane(a.y, 63));
}

// Verdicts of the node's vertices q0 .. q1-1 (index q runs over the lower
// side, then the upper side), one wave per vertex: lanes scan the vertices
// left of v and right of v; an empty extreme stays at v itself (same x),
// which the wave reduction never prefers.  flag[q - q0] = 1 iff v survives.
template <bool SMALL>
__device__ __forceinline__ void l2_test_share(const L2Shared &S, int q0, int q1, int C0, int C1,
                                              uint8_t *flag) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int q = q0 + wave; q < q1; q += kL2Waves) {
    const int side = q < C0 ? 0 : 1;
    const int i = side ? q - C0 : q;
    const int cs = side ? C1 : C0;
    const int2 *Pp = S.P[side];
    const int2 v = Pp[i];
    int2 uL = v, wR = v;
    // branch-free updates: both tests are plain integer arithmetic, so
    // they are evaluated and combined without short-circuit branches
    auto left = [&](int2 u) {
      const bool t = (uL.x == v.x) | steeper_left<SMALL>(u, uL, v);
      uL.x = t ? u.x : uL.x;
      uL.y = t ? u.y : uL.y;
    };
    auto right = [&](int2 w) {
      const bool t = (wR.x == v.x) | flatter_right<SMALL>(w, wR, v);
      wR.x = t ? w.x : wR.x;
      wR.y = t ? w.y : wR.y;
    };
    // four reads in flight per lane before their comparisons
    int k = lane;
    for (; k + 3 * kWave < i; k += 4 * kWave) {
      const int2 u0 = Pp[k], u1 = Pp[k + kWave], u2 = Pp[k + 2 * kWave], u3 = Pp[k + 3 * kWave];
      left(u0);
      left(u1);
      left(u2);
      left(u3);
    }
    for (; k < i; k += kWave) left(Pp[k]);
    k = i + 1 + lane;
    for (; k + 3 * kWave < cs; k += 4 * kWave) {
      const int2 w0 = Pp[k], w1 = Pp[k + kWave], w2 = Pp[k + 2 * kWave], w3 = Pp[k + 3 * kWave];
      right(w0);
      right(w1);
      right(w2);
      right(w3);
    }
    for (; k < cs; k += kWave) right(Pp[k]);
    uL = wave_pick(uL, [&](int2 a, int2 b) {
      const bool t = (b.x != v.x) & ((a.x == v.x) | steeper_left<SMALL>(b, a, v));
      return make_int2(t ? b.x : a.x, t ? b.y : a.y);
    });
    wR = wave_pick(wR, [&](int2 a, int2 b) {
      const bool t = (b.x != v.x) & ((a.x == v.x) | flatter_right<SMALL>(b, a, v));
      return make_int2(t ? b.x : a.x, t ? b.y : a.y);
    });
    const bool keep = (uL.x == v.x) | (wR.x == v.x) | cross_pos<SMALL>(uL, v, wR);
    if (lane == 0) flag[q - q0] = keep ? 1 : 0;
  }
}

// H.split workgroups per level-2 node.  Each tests its share of the node's
// vertices (one wave per vertex), writes its survivors in order to the
// node's slot of buffer 1 at its share's first index, with their count per
// side in l2cnt, and writes the chain of its share of the node's slabs.
template <bool SMALL>
__device__ __forceinline__ void l2_test_body(const HullArgs &H, L2Shared &S, const int node, const int part) {
  const int parts = H.split;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const TreeShape &T = H.tree;
  if (node == 0 && part == 0 && !H.slab_off) l2_totals(H, S);
  l2_stage<false>(H, S, node);
  const int C0 = S.off[0][kFanIn], C1 = S.off[1][kFanIn], total = C0 + C1;
  const int per = (total + parts - 1) / parts;
  const int q0 = min(total, part * per), q1 = min(total, q0 + per);
  uint8_t *flag = reinterpret_cast<uint8_t *>(S.keepw);   // this share's verdicts
  l2_test_share<SMALL>(S, q0, q1, C0, C1, flag);
  __syncthreads();  // survivors of each side of the share, in order (waves 0 and 1; a share
  // is at most a few hundred vertices)
  if (wave < 2) {
    const int side = wave;
    const int a = side ? max(q0, C0) : q0, b = side ? q1 : min(q1, C0);   // share in q space
    const int first = side ? a - C0 : a;                                    // in side index space
    int2 *out = H.buf[1] + (size_t)side * H.positions + (size_t)node * T.span[2] + first;
    int n = 0;
    for (int q = a; q < b; q += kWave) {
      const bool keep = q + lane < b && flag[q + lane - q0] != 0;
      int tot;
      const int r = wave_rank(keep, &tot);
      if (keep) out[n + r] = S.P[side][(side ? q - C0 : q) + lane];
      n += tot;
    }
    if (lane == 0) H.l2cnt[((size_t)node * parts + part) * 2 + side] = n;
  }
  // chain of this workgroup's slabs, one wave each
  const int per_slabs = (kFanIn + parts - 1) / parts;
  const int sl = node * kFanIn + part * per_slabs + wave;
  if (wave < per_slabs && part * per_slabs + wave < kFanIn && sl < T.size[1]) l2_chain_slab(H, sl);
}

template <bool SMALL>
__global__ __launch_bounds__(kHullBlock) void k_l2_test(HullArgs H) {
  __shared__ L2Shared S;
  l2_test_body<SMALL>(H, S, blockIdx.x / H.split, blockIdx.x % H.split);
}

// One workgroup per level-2 node: the shares' survivors joined in order
// (the node's hulls in buffer 1), or, at the root, the final vertex list.
template <bool SMALL>
__device__ __forceinline__ void l2_compact_body(const HullArgs &H, L2Shared &S, const int node) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const TreeShape &T = H.tree;
  const int parts = H.split;
  const int64_t P = H.positions;
  // per side: the shares' counts and their prefix; the shares' first
  // indices follow from the staged counts of the test (per = ceil(C/parts))
  if (wave < 2) {
    const int side = wave;
    int carry = 0;
    for (int h = 0; h < kL2MaxParts; h += kWave) {
      const int sh = h + lane;
      const int m = sh < parts ? H.l2cnt[((size_t)node * parts + sh) * 2 + side] : 0;
      int incl = m;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
      }
      S.soff[side][sh] = carry + incl - m;
      carry += __shfl(incl, kWave - 1, kWave);
    }
    if (lane == 0) S.soff[side][kL2MaxParts] = carry;
  }
  // the test's share boundaries need C0 and C1: the node's slab-hull sizes
  if (wave == 2 || wave == 3) {
    const int side = wave - 2;
    const int sib0 = node * kFanIn, nsib = min(kFanIn, T.size[1] - sib0);
    int m = lane < nsib ? H.ccount[side * T.nodes + T.base[1] + sib0 + lane] : 0;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) m += __shfl_xor(m, d, kWave);
    if (lane == 0) S.sum[side] = m;
  }
  __syncthreads();
  const int C0 = S.sum[0], C1 = S.sum[1], total = C0 + C1;
  const int per = (total + parts - 1) / parts;
  // gather every survivor: thread t takes survivors t, t + 1024, ...
  int nk[2];
  int2 *node_out = H.buf[1] + (size_t)node * T.span[2];
  for (int side = 0; side < 2; ++side) {
    const int all = S.soff[side][kL2MaxParts];
    nk[side] = all;
    for (int j = tid; j < all; j += kHullBlock) {
      int lo = 0, hi = parts - 1;          // last share with soff <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.soff[side][mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      const int q0 = min(total, lo * per);
      const int first = side ? max(q0, C0) - C0 : q0;
      S.P[side][j] = node_out[(size_t)side * P + first + (j - S.soff[side][lo])];
    }
  }
  __syncthreads();
  const bool root = T.nlev == 2;
  if (!root) {
    for (int side = 0; side < 2; ++side)
      for (int j = tid; j < nk[side]; j += kHullBlock) node_out[(size_t)side * P + j] = S.P[side][j];
    if (tid < 2) H.ccount[tid * T.nodes + T.base[2] + node] = nk[tid];
    return;
  }
  bool overflow = false;
  const int h = assemble_hull(S.P[0], nk[0], S.P[1], nk[1], H.hx, H.hy, H.hull_cap, overflow);
  if (tid == 0) {
    H.info[HP_INFO_H] = overflow ? 0 : h;
    if (overflow) atomicMin(&H.info[HP_INFO_STATUS], HP_ECAPACITY);
  }
}

template <bool SMALL>
__global__ __launch_bounds__(kHullBlock) void k_l2_compact(HullArgs H) {
  __shared__ L2Shared S;
  l2_compact_body<SMALL>(H, S, blockIdx.x);
}

// ---------------------------------------------------------------------------
// A cloud whose slabs form a single level-2 node (2 to 64 slabs): the test
// workgroups also finish the cloud, with no compaction launch.  Each issues
// every load it needs in one round (the node's slots and slab-hull sizes;
// the L columns and earlier slab counts of its chain slab; for workgroup 0
// the counts and error words of the totals), tests its share of the
// vertices, and stores its verdict bytes, its chain slab and the totals.
// The last workgroup to finish (acquire-release count) still holds every
// vertex of the node in LDS: it loads all verdicts, compacts the survivors
// of each side in x order and writes the hull.  Needs H.split >= slabs.
// ---------------------------------------------------------------------------
template <bool SMALL>
__global__ __launch_bounds__(kHullBlock) void k_l2_root(HullArgs H) {
  __shared__ L2Shared S;
  __shared__ int s_flag;
  const int parts = H.split, part = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int nslab = H.tree.size[1];
  // chain slab `part` (last wave) and the totals (workgroup 0, wave before
  // it): loads first, used after the test
  const bool chain_w = wave == kL2Waves - 1 && part < nslab;
  const bool tot_w = wave == kL2Waves - 2 && part == 0;
  int2 cL = make_int2(1, 0);
  int cbase = 0, tk = 0, ts = 0, te = 0;
  if (chain_w) {
    const int64_t pos = (int64_t)part * kSlab + lane;
    if (pos < H.p) cL = H.Lm[pos];
    if (lane < part) cbase = H.slab_k[lane];
  }
  if (tot_w) {
    if (lane < nslab) {
      tk = H.slab_k[lane];
      ts = H.slab_s[lane];
    }
    for (int j = lane; j < H.n_wg_err; j += kWave) te |= H.wg_err[j];
  }
  l2_stage<false>(H, S, 0);
  const int C0 = S.off[0][kFanIn], C1 = S.off[1][kFanIn], total = C0 + C1;
  const int per = (total + parts - 1) / parts;
  const int q0 = min(total, part * per), q1 = min(total, q0 + per);
  uint8_t *flag = reinterpret_cast<uint8_t *>(S.keepw);
  l2_test_share<SMALL>(S, q0, q1, C0, C1, flag);
  __syncthreads();
  for (int j = tid; j < q1 - q0; j += kHullBlock) H.keep[q0 + j] = flag[j];
  if (chain_w) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) cbase += __shfl_xor(cbase, d, kWave);
    const bool valid = cL.x <= cL.y;
    int tot;
    const int r = wave_rank(valid, &tot);
    if (valid) {
      const int o = cbase + r;
      if (o < H.chain_cap) {
        H.cx[o] = part * kSlab + lane + 1;
        H.clo[o] = cL.x;
        H.chi[o] = cL.y;
      } else {
        atomicMin(&H.info[HP_INFO_STATUS], HP_ECAPACITY);
      }
    }
  }
  if (tot_w) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      tk += __shfl_xor(tk, d, kWave);
      ts += __shfl_xor(ts, d, kWave);
      te |= __shfl_xor(te, d, kWave);
    }
    if (lane == 0) {
      H.info[HP_INFO_K] = tk;
      H.info[HP_INFO_S] = ts;
      report_reduce_errors(te, H.info);
    }
  }
  if (!last_arrival_flag(&H.ctl[kCtlTestDone], parts, &s_flag)) return;

  // the root: every verdict (at most 2 x 4096 bytes, two words per thread)
  const uint32_t *kw = reinterpret_cast<const uint32_t *>(H.keep);
  const int nw = (total + 3) / 4;
  uint32_t w2[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) w2[u] = tid + u * kHullBlock < nw ? kw[tid + u * kHullBlock] : 0u;
  uint32_t *kl = &S.keepw[0][0];   // both rows, 2 x 1024 words
#pragma unroll
  for (int u = 0; u < 2; ++u) kl[tid + u * kHullBlock] = w2[u];
  __syncthreads();
  // survivors of each side in x order: slot idx = side * 4096 + i, eight
  // per thread; a wave's 64 lanes cover one run of 64 slots (chunk)
  // (slot u of this thread is vertex i = tid + 1024 (u % 4) of side u / 4,
  // in chunk wave + 16 (u % 4); every read below is unconditional and in
  // range: i < 4096 and C0 + i < 8192)
  constexpr int kPer = 2 * kNodeVerts / kHullBlock;
  int2 v[kPer];
  uint8_t fb[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int side = u / 4, i = tid + kHullBlock * (u % 4);
    fb[u] = flag[side ? C0 + i : i];
    v[u] = S.P[side][i];
  }
  bool keep[kPer];
  int rank[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int side = u / 4, i = tid + kHullBlock * (u % 4);
    keep[u] = i < (side ? C1 : C0) && fb[u] != 0;
    int tot;
    rank[u] = wave_rank(keep[u], &tot);
    if (lane == 0) S.soff[side][wave + 16 * (u % 4)] = tot;
  }
  __syncthreads();
  if (wave < 2) {
    // exclusive scan of the 64 chunk counts of side `wave`
    const int m = S.soff[wave][lane];
    int incl = m;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    S.soff[wave][lane] = incl - m;
    if (lane == kWave - 1) S.sum[wave] = incl;
  }
  __syncthreads();
  const int sl[2] = {S.soff[0][lane], S.soff[1][lane]};
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int side = u / 4;
    const int base = __builtin_amdgcn_readlane(sl[side], wave + 16 * (u % 4));
    if (keep[u]) S.P[side][base + rank[u]] = v[u];
  }
  __syncthreads();
  bool overflow = false;
  const int h = assemble_hull(S.P[0], S.sum[0], S.P[1], S.sum[1], H.hx, H.hy, H.hull_cap, overflow);
  if (tid == 0) {
    H.info[HP_INFO_H] = overflow ? 0 : h;
    if (overflow) atomicMin(&H.info[HP_INFO_STATUS], HP_ECAPACITY);
  }
}
// ---------------------------------------------------------------------------
// Clouds of more than one level-2 node: one workgroup per node of 64 slabs
// (4096 columns) finishes its columns and builds the node's hulls.
//  1. the partial L arrays folded per column: the L export, M, the slab
//     counts and, per slab and side, the lowest point and the first and
//     last columns; the node's columns stay in LDS
//  2. the lower hull of the 64 lowest points (each against its neighbours
//     up to 8 slabs away, in single precision: it only picks reference
//     points for the filter); one wave finds the node's
//     first chain index from the nodes before it (a look-back over nodes
//     numbered in the order their workgroups start, so a node only waits
//     for nodes that are already running)
//  3. the filter drops every point on or above the segment between two
//     points of the node around it (the nearest lowest points on that hull,
//     or its slab's end column; the test is exact): such a point is no
//     vertex of the node's hull.  The survivors of each slab are listed
//  4. the slab hulls: each survivor against the others of its slab; the
//     node's part of the chain (Lemma 1)
//  5. the node merge: a slab-hull vertex v is kept when the steepest slope
//     into v from the points left of it is below the flattest slope out of
//     v to the points right of it, both found per slab hull by binary search
//     for the tangent from v (16 lanes per vertex, 4 slabs each)
//  6. the node's hulls to the level-2 slot of the hull tree; the node
//     numbered last writes k, s and the reduce's range status
// Vertices are kept only at a strict left turn, so collinear points are
// dropped (Appendix).  Each side is the lower hull of (x, lo) or of (x, -hi).
// ---------------------------------------------------------------------------
constexpr int kNodeBlock = 1024;
constexpr int kNodeWaves = kNodeBlock / kWave;
constexpr int kNodeCols = kFanIn * kSlab;
constexpr int kNodeGroup = 16;                  // lanes per vertex in the merge
constexpr int kCtlNodeTicket = 3;               // node numbers, in workgroup start order
// look-back words: status in bits 62-63 (1: the node's own counts, 2: the
// counts of every node up to it), counts below
constexpr uint64_t kLbAgg = 1ull << 62, kLbIncl = 2ull << 62, kLbMask = (1ull << 62) - 1;
constexpr int kLbSpinMax = 1 << 20;
constexpr int kMinWin = 8;                      // slabs each way in the hull of the lowest points

struct NodeShared {
  int2 col[kNodeCols];            // (lo, hi) per position, slab-swizzled
  int32_t xs[kNodeCols];          // x per position, slab-swizzled
  int2 hp[2][kNodeCols];          // per slab row of 64: survivors, then the slab hull
  uint16_t vidx[2][kNodeCols];    // slab-hull vertices in x order: their places in hp
  uint8_t keep[2][kNodeCols];     // merge verdicts
  int32_t slab_k[kFanIn], slab_s[kFanIn], slab_off[kFanIn];
  int32_t mn[2][kFanIn];          // column in its slab of the lowest point, -1 when empty
  int32_t first[kFanIn], last[kFanIn];
  // per slab and side, the filter's reference points: the nearest lowest
  // points left and right on the hull of the lowest points (or the slab's
  // first and last columns), the slab's own lowest point, and whether that
  // one is on the hull
  int2 refL[2][kFanIn], refM[2][kFanIn], refR[2][kFanIn];
  uint8_t ish[2][kFanIn];
  int32_t scnt[2][kFanIn];        // survivors per slab
  int32_t cnt[2][kFanIn];         // slab-hull sizes
  int32_t tot[2];
  int32_t ticket, base;
};

// Position t of a slab-major array of 64-entry rows, rotated by the row
// index so that the lanes of a wave, one row each, fall in different banks.
__device__ __forceinline__ int node_sw(int t) { return (t & ~(kSlab - 1)) | ((t + (t >> 6)) & (kSlab - 1)); }

__device__ __forceinline__ int2 node_point(const NodeShared &S, int side, int c) {
  const int2 L = S.col[node_sw(c)];
  return make_int2(S.xs[node_sw(c)], side ? -L.y : L.x);
}

// Exact predicates for the points of one node, in one of three forms:
// kPrecSmall, coordinates below 2^15 (24-bit products); kPrecNode, columns
// of one node (x differences below 2^12, y differences below 2^31, so every
// product is below 2^43 and exact in double precision); kPrecWide, any int32
// coordinates (products in 64-bit integers).
//   ncross_pos / ncross_neg: cross(o, a, b) > 0 / < 0
//   nsteeper_left: slope(u1, v) > slope(u2, v), u1 and u2 left of v
//   nflatter_right: slope(v, w1) < slope(v, w2), w1 and w2 right of v
constexpr int kPrecSmall = 0, kPrecNode = 1, kPrecWide = 2;
template <int PREC>
__device__ __forceinline__ bool ncross_pos(int2 o, int2 a, int2 b) {
  if (PREC == kPrecSmall) return cross_pos<true>(o, a, b);
  if (PREC == kPrecWide) return cross_pos<false>(o, a, b);
  return (double)(a.x - o.x) * (double)(b.y - o.y) > (double)(a.y - o.y) * (double)(b.x - o.x);
}
template <int PREC>
__device__ __forceinline__ bool ncross_neg(int2 o, int2 a, int2 b) {
  if (PREC == kPrecSmall) return cross_neg<true>(o, a, b);
  if (PREC == kPrecWide) return cross_neg<false>(o, a, b);
  return (double)(a.x - o.x) * (double)(b.y - o.y) < (double)(a.y - o.y) * (double)(b.x - o.x);
}
template <int PREC>
__device__ __forceinline__ bool nsteeper_left(int2 u1, int2 u2, int2 v) {
  if (PREC == kPrecSmall) return steeper_left<true>(u1, u2, v);
  if (PREC == kPrecWide) return steeper_left<false>(u1, u2, v);
  return (double)(v.y - u1.y) * (double)(v.x - u2.x) > (double)(v.y - u2.y) * (double)(v.x - u1.x);
}
template <int PREC>
__device__ __forceinline__ bool nflatter_right(int2 w1, int2 w2, int2 v) {
  if (PREC == kPrecSmall) return flatter_right<true>(w1, w2, v);
  if (PREC == kPrecWide) return flatter_right<false>(w1, w2, v);
  return (double)(w1.y - v.y) * (double)(w2.x - v.x) < (double)(w2.y - v.y) * (double)(w1.x - v.x);
}

// CHAIN: the node's positions are chain entries (x, lo, hi) (A.cx, A.clo,
// A.chi, the first info[K] of A.positions valid) rather than columns; the
// chain and the totals are then inputs, and only the hulls are written.
template <int PREC, bool CHAIN>
__global__ __launch_bounds__(kNodeBlock) void k_node_finish(FinishArgs A, int2 *__restrict__ l2_out,
                                                            int32_t *__restrict__ ccount) {
  extern __shared__ __align__(16) unsigned char node_smem[];
  NodeShared &S = *reinterpret_cast<NodeShared *>(node_smem);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const TreeShape &T = A.tree;
  const int nnodes = T.size[2], nslab = T.size[1];
  if (tid == 0) S.ticket = __hip_atomic_fetch_add(&A.ctl[kCtlNodeTicket], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int g = S.ticket;
  if (g >= nnodes) {   // the control words were not cleared: no node to take
    if (tid == 0) atomicMin(&A.info[HP_INFO_STATUS], HP_EDEVICE);
    return;
  }
  const int64_t g0 = (int64_t)g * kNodeCols;
  const int32_t x0 = (int32_t)g0 + 1;   // x of the node's column 0
  const int64_t p = A.p;

  // ---- 1. fold the partial arrays, four columns per thread (column
  // tid + 1024 j is column `lane` of the node's slab wave + 16 j) ----------
  int mlo[4], mhi[4], xv[4];
  bool valid[4];
  if (CHAIN) {
    const int64_t kk = min<int64_t>(A.info[HP_INFO_K], A.positions);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t pos = g0 + tid + j * kNodeBlock;
      valid[j] = pos < kk;
      xv[j] = valid[j] ? A.cx[pos] : 0;
      mlo[j] = valid[j] ? A.clo[pos] : 1;
      mhi[j] = valid[j] ? A.chi[pos] : 0;
    }
  } else {
    int64_t pos[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mlo[j] = INT_MAX;
      mhi[j] = INT_MIN;
      pos[j] = g0 + tid + j * kNodeBlock;
    }
    const int G = A.G;
    const bool full = g0 + kNodeCols <= p;
    if (A.packed) {
      const uint32_t *src = reinterpret_cast<const uint32_t *>(A.part);
      for (int q = 0; q < G; ++q) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = (full || pos[j] < p) ? src[(size_t)q * p + pos[j]] : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int2 e = unpack_partial(w[j]);
          mlo[j] = min(mlo[j], e.x);
          mhi[j] = max(mhi[j], e.y);
        }
      }
    } else {
      // up to 8 partial arrays x 4 columns of loads in flight per thread
      for (int q0 = 0; q0 < G; q0 += 8) {
        int2 w[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            w[u][j] = (q0 + u < G && (full || pos[j] < p)) ? A.part[(size_t)(q0 + u) * p + pos[j]]
                                                          : make_int2(INT_MAX, INT_MIN);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            mlo[j] = min(mlo[j], w[u][j].x);
            mhi[j] = max(mhi[j], w[u][j].y);
          }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool inside = pos[j] < p;
      valid[j] = inside && mlo[j] <= mhi[j];
      xv[j] = x0 + tid + j * kNodeBlock;
      if (inside && A.lo) {
        A.lo[pos[j]] = mlo[j];
        A.hi[pos[j]] = mhi[j];
      }
    }
  }
  {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tid + j * kNodeBlock;
      S.col[node_sw(c)] = valid[j] ? make_int2(mlo[j], mhi[j]) : make_int2(1, 0);
      S.xs[node_sw(c)] = xv[j];
      const unsigned long long vm = __ballot(valid[j]);
      const unsigned long long sm = __ballot(valid[j] && mlo[j] < mhi[j]);
      const int sl = wave + j * kNodeWaves;
      // lowest point of the slab on each side: smallest lo, largest hi (the
      // leftmost of equal ones); the keys order int32 values as unsigned
      uint64_t k0 = valid[j] ? ((uint64_t)((uint32_t)mlo[j] ^ 0x80000000u) << 6) | (uint64_t)lane : ~0ull;
      uint64_t k1 = valid[j] ? ((uint64_t)(~((uint32_t)mhi[j] ^ 0x80000000u)) << 6) | (uint64_t)lane : ~0ull;
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) {
        const uint64_t o0 = __shfl_xor(k0, d, kWave), o1 = __shfl_xor(k1, d, kWave);
        k0 = o0 < k0 ? o0 : k0;
        k1 = o1 < k1 ? o1 : k1;
      }
      if (lane == 0) {
        if (!CHAIN && A.mask && (int64_t)g * kFanIn + sl < nslab) A.mask[(int64_t)g * kFanIn + sl] = vm;
        S.slab_k[sl] = __popcll(vm);
        S.slab_s[sl] = __popcll(vm) + __popcll(sm);
        S.mn[0][sl] = vm ? (int)(k0 & 63) : -1;
        S.mn[1][sl] = vm ? (int)(k1 & 63) : -1;
        S.first[sl] = vm ? __builtin_ctzll(vm) : -1;
        S.last[sl] = vm ? 63 - __builtin_clzll(vm) : -1;
      }
    }
  }
  __syncthreads();

  // ---- 2. the hull of the slabs' lowest points (waves 0 and 1: side, lane
  // = slab); the look-back (last wave); the reduce's chunk check (node 0,
  // the wave before) ---------------------------------------------------------
  if (wave < 2) {
    const int side = wave, sl = lane;
    const int ml = S.mn[side][sl];
    const int2 M = ml >= 0 ? node_point(S, side, sl * kSlab + ml) : make_int2(0, 0);
    // against the lowest points of the slabs up to kMinWin away only: the
    // result is a superset of the hull's vertices, which still gives valid
    // reference points
    float lx = 0.f, ly = 0.f, rx = 0.f, ry = 0.f;   // steepest in, flattest out (as vectors)
    bool hasL = false, hasR = false;
#pragma unroll
    for (int d = -kMinWin; d <= kMinWin; ++d) {
      if (d == 0) continue;
      const int j = sl + d;
      const int src = j < 0 ? 0 : (j > kWave - 1 ? kWave - 1 : j);
      const int mj = __shfl(ml, src, kWave);
      const float dx = (float)(__shfl(M.x, src, kWave) - M.x);
      const float dy = (float)(__shfl(M.y, src, kWave) - M.y);
      const bool there = j >= 0 && j < kWave && mj >= 0;
      // from the left: slope dy/dx (dx < 0) steeper than the best so far
      const bool tL = there & (d < 0) & (!hasL | (dy * lx > ly * dx));
      const bool tR = there & (d > 0) & (!hasR | (dy * rx < ry * dx));
      lx = tL ? dx : lx;
      ly = tL ? dy : ly;
      hasL |= tL;
      rx = tR ? dx : rx;
      ry = tR ? dy : ry;
      hasR |= tR;
    }
    // a strict left turn: slope in below slope out (lx < 0 < rx)
    const bool on = ml >= 0 && (!hasL || !hasR || ly * rx > ry * lx);
    const unsigned long long hm = __ballot(on);
    const unsigned long long lm = hm & ((1ull << sl) - 1ull);
    const unsigned long long rm = sl == kWave - 1 ? 0ull : hm & ~((2ull << sl) - 1ull);
    const int hl = lm ? 63 - __builtin_clzll(lm) : 0, hr = rm ? __builtin_ctzll(rm) : 0;
    const int2 PL = make_int2(__shfl(M.x, hl, kWave), __shfl(M.y, hl, kWave));
    const int2 PR = make_int2(__shfl(M.x, hr, kWave), __shfl(M.y, hr, kWave));
    if (ml >= 0) {
      S.refL[side][sl] = lm ? PL : node_point(S, side, sl * kSlab + S.first[sl]);
      S.refR[side][sl] = rm ? PR : node_point(S, side, sl * kSlab + S.last[sl]);
      S.refM[side][sl] = M;
      S.ish[side][sl] = on ? 1 : 0;
    }
  } else if (!CHAIN && wave == kNodeWaves - 1) {
    const int kk = S.slab_k[lane], ss = S.slab_s[lane];
    int incl = kk, stot = ss;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) stot += __shfl_xor(stot, d, kWave);
    S.slab_off[lane] = incl - kk;
    // the node's (k, s) as one word: k in bits 0-30, s in bits 31-61 (sums
    // of either stay below 2^31, so packed words add field by field)
    const uint64_t mine = (uint64_t)(uint32_t)__shfl(incl, kWave - 1, kWave) | ((uint64_t)(uint32_t)stot << 31);
    uint64_t *flags = reinterpret_cast<uint64_t *>(A.tree_ctr);
    uint64_t prefix = 0;
    if (g > 0) {
      if (lane == 0) __hip_atomic_store(&flags[g], kLbAgg | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int j = g - 1;; j -= kWave) {
        const int idx = j - lane;
        uint64_t v = idx >= 0 ? __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kLbIncl;
        // every node numbered before this one is running and publishes its
        // counts right after its fold; the bound only turns a broken
        // invariant into an error instead of a wait without end
        for (int spin = 0; __ballot((v >> 62) == 0) != 0ull; ++spin) {
          if (spin == kLbSpinMax) {
            if (lane == 0) atomicMin(&A.info[HP_INFO_STATUS], HP_EDEVICE);
            v = (v >> 62) == 0 ? kLbIncl : v;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          if ((v >> 62) == 0) v = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned long long incm = __ballot((v >> 62) == 2);
        const int first = incm ? __builtin_ctzll(incm) : kWave;
        uint64_t add = lane <= first ? (v & kLbMask) : 0ull;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) add += __shfl_xor(add, d, kWave);
        prefix += add;
        if (incm) break;
      }
    }
    if (lane == 0) {
      __hip_atomic_store(&flags[g], kLbIncl | (prefix + mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      S.base = (int)(prefix & 0x7FFFFFFFull);
    }
    if (g == nnodes - 1) {
      // the last node holds the totals; it also reads the reduce's error words
      int err = 0;
      for (int j = lane; j < A.n_wg_err; j += kWave) err |= A.wg_err[j];
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) err |= __shfl_xor(err, d, kWave);
      if (lane == 0) {
        const uint64_t tot = prefix + mine;
        A.info[HP_INFO_K] = (int32_t)(tot & 0x7FFFFFFFull);
        A.info[HP_INFO_S] = (int32_t)((tot >> 31) & 0x7FFFFFFFull);
        report_reduce_errors(err, A.info);
      }
    }
  } else if (!CHAIN && wave == kNodeWaves - 2 && g == 0 && A.dyn_ctr != nullptr) {
    // every chunk of the reduce folded exactly once; the counter is zero
    // again for the next run that uses its slot
    int folded = 0;
    for (int j = lane; j < A.n_wg_cnt; j += kWave) folded += A.wg_cnt[j];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) folded += __shfl_xor(folded, d, kWave);
    if (lane == 0) {
      if ((int64_t)folded != A.dyn_expect) atomicMin(&A.info[HP_INFO_STATUS], HP_EDEVICE);
      __hip_atomic_store(A.dyn_ctr, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();

  // ---- 3. the filter (every wave, its 4 slabs): survivors to their row ---
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sl = wave + j * kNodeWaves;
    const int c = sl * kSlab + lane;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      bool keep = false;
      const int2 v = make_int2(xv[j], side ? -mhi[j] : mlo[j]);
      if (valid[j]) {
        const int2 PM = S.refM[side][sl];
        int2 u = S.refL[side][sl], w = S.refR[side][sl];
        if (S.ish[side][sl]) {
          if (v.x < PM.x) w = PM;
          else u = PM;
        }
        keep = v.x == u.x || v.x == w.x || ncross_neg<PREC>(u, w, v);
      }
      int tot;
      const int r = wave_rank(keep, &tot);
      if (keep) S.hp[side][sl * kSlab + r] = v;
      if (lane == 0) S.scnt[side][sl] = tot;
    }
  }
  __syncthreads();

  // ---- 4. slab hulls (every wave, its 4 slabs: lane k tests survivor k
  // against the others of its slab, then the row is compacted in place);
  // the node's part of the chain -------------------------------------------
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sl = wave + j * kNodeWaves;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int m = S.scnt[side][sl];
      int2 *row = S.hp[side] + sl * kSlab;
      const int2 v = lane < m ? row[lane] : make_int2(0, 0);
      int2 uL = v, wR = v;
      bool hasL = false, hasR = false;
      for (int i = 0; i < m; ++i) {
        const int2 u = row[i];
        const bool tL = (i < lane) & (!hasL | nsteeper_left<PREC>(u, uL, v));
        const bool tR = (i > lane) & (!hasR | nflatter_right<PREC>(u, wR, v));
        uL = tL ? u : uL;
        hasL |= tL;
        wR = tR ? u : wR;
        hasR |= tR;
      }
      const bool keep = lane < m && (!hasL || !hasR || ncross_pos<PREC>(uL, v, wR));
      int tot;
      const int r = wave_rank(keep, &tot);
      if (keep) row[r] = v;
      if (lane == 0) S.cnt[side][sl] = tot;
    }
    if (CHAIN) continue;
    const int c = sl * kSlab + lane;
    int tot;
    const int r = wave_rank(valid[j], &tot);
    if (valid[j]) {
      const int off = S.base + S.slab_off[sl] + r;
      if (off < A.chain_cap) {
        A.cx_out[off] = x0 + c;
        A.clo_out[off] = mlo[j];
        A.chi_out[off] = mhi[j];
      } else {
        atomicMin(&A.info[HP_INFO_STATUS], HP_ECAPACITY);
      }
    }
  }
  __syncthreads();
  // the slab-hull vertices in x order per side (every wave scans the counts)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int cn = S.cnt[side][lane];
    int incl = cn;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    const int excl = incl - cn;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int sl = wave + j * kNodeWaves;
      const int o = __builtin_amdgcn_readlane(excl, sl), m = __builtin_amdgcn_readlane(cn, sl);
      if (lane < m) S.vidx[side][o + lane] = (uint16_t)(sl * kSlab + lane);
    }
    if (wave == 0 && lane == kWave - 1) S.tot[side] = incl;
  }
  __syncthreads();

  // ---- 5. node merge: 16 lanes per vertex, slabs gl, gl + 16, ... each ----
  {
    const int gl = tid & (kNodeGroup - 1), grp = tid / kNodeGroup;
    const int t0 = S.tot[0], all = t0 + S.tot[1];
    for (int q = grp; q < all; q += kNodeBlock / kNodeGroup) {
      const int side = q < t0 ? 0 : 1, idx = side ? q - t0 : q;
      const int2 *Hs = S.hp[side];
      const int at = S.vidx[side][idx];
      const int2 v = Hs[at];
      const int i = at >> 6, k = at & (kSlab - 1);
      int2 uL = v, wR = v;
      bool hasL = false, hasR = false;
#pragma unroll
      for (int r = 0; r < kFanIn / kNodeGroup; ++r) {
        const int jsl = gl + r * kNodeGroup;
        const int m = S.cnt[side][jsl];
        if (m == 0) continue;
        const int2 *H = Hs + jsl * kSlab;
        if (jsl == i) {
          // the vertex's own slab hull: its neighbours there
          if (k > 0) {
            const int2 u = H[k - 1];
            if (!hasL || nsteeper_left<PREC>(u, uL, v)) { uL = u; hasL = true; }
          }
          if (k + 1 < m) {
            const int2 w = H[k + 1];
            if (!hasR || nflatter_right<PREC>(w, wR, v)) { wR = w; hasR = true; }
          }
        } else {
          // tangent from v: on a hull to its left the first vertex whose next
          // edge does not turn left towards v, on a hull to its right the
          // first whose next edge does not turn right
          const bool left = jsl < i;
          int lo = 0, hi = m - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const bool go = left ? ncross_pos<PREC>(H[mid], H[mid + 1], v) : ncross_neg<PREC>(H[mid], H[mid + 1], v);
            if (go) lo = mid + 1;
            else hi = mid;
          }
          const int2 t = H[lo];
          if (left) {
            if (!hasL || nsteeper_left<PREC>(t, uL, v)) { uL = t; hasL = true; }
          } else {
            if (!hasR || nflatter_right<PREC>(t, wR, v)) { wR = t; hasR = true; }
          }
        }
      }
#pragma unroll
      for (int d = kNodeGroup / 2; d > 0; d >>= 1) {
        const int2 ou = make_int2(__shfl_xor(uL.x, d, kNodeGroup), __shfl_xor(uL.y, d, kNodeGroup));
        const int2 ow = make_int2(__shfl_xor(wR.x, d, kNodeGroup), __shfl_xor(wR.y, d, kNodeGroup));
        const bool ohL = __shfl_xor((int)hasL, d, kNodeGroup) != 0;
        const bool ohR = __shfl_xor((int)hasR, d, kNodeGroup) != 0;
        if (ohL && (!hasL || nsteeper_left<PREC>(ou, uL, v))) { uL = ou; hasL = true; }
        if (ohR && (!hasR || nflatter_right<PREC>(ow, wR, v))) { wR = ow; hasR = true; }
      }
      if (gl == 0) S.keep[side][idx] = (!hasL || !hasR || ncross_pos<PREC>(uL, v, wR)) ? 1 : 0;
    }
  }
  __syncthreads();

  // ---- 6. the node's hull per side (waves 0 and 1) ------------------------
  if (wave < 2) {
    const int side = wave, m = S.tot[side];
    int2 *dst = l2_out + (size_t)side * A.positions + (size_t)g * kNodeCols;
    int n = 0;
    for (int j0 = 0; j0 < m; j0 += kWave) {
      const int j = j0 + lane;
      const bool kp = j < m && S.keep[side][j] != 0;
      int tot;
      const int r = wave_rank(kp, &tot);
      if (kp) dst[n + r] = S.hp[side][S.vidx[side][j]];
      n += tot;
    }
    if (lane == 0) ccount[side * T.nodes + T.base[2] + g] = n;
  }
}

// ---------------------------------------------------------------------------
// Sparse clouds (n well below p): the path visits only the occupied columns
// (Proposed heuristic, quick analysis: unused entries are skipped when
// p > n; Discussion, extraction with a w-ary tree of bits, w = 64).
//  1. M (one bit per column) and its summary level (one bit per M word)
//     cleared: ceil(p/64) + ceil(p/4096) words
//  2. every point sets its column's bit; the point whose OR found its M
//     word empty sets the word's summary bit
//  3. per summary word, the occupied columns under it (one wave per summary
//     word, reading only the M words its bits name); their scan
//  4. the chain positions: every occupied column in x order, with (lo, hi)
//     at the sentinel, and per occupied M word the chain index of its first
//     column
//  5. every point folds its y into its column's chain entry (device atomics;
//     the index is the word's first index plus the bits below it)
//  6. s, and the L export when asked for
// ---------------------------------------------------------------------------
constexpr int kSparseRatio = 8;     // n * kSparseRatio < p: the automatic choice takes the sparse path
constexpr int kSparseBlock = 256;
constexpr int kSparseScan = 1024;

__global__ void k_sp_clear(uint64_t *__restrict__ L0, int64_t W0, uint64_t *__restrict__ L1, int64_t W1,
                           int32_t *__restrict__ info) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < W0; i += stride) L0[i] = 0;
  for (int64_t i = i0; i < W1; i += stride) L1[i] = 0;
  if (i0 == 0) {
    info[HP_INFO_STATUS] = HP_OK;
    info[HP_INFO_K] = 0;
    info[HP_INFO_S] = 0;
    info[HP_INFO_H] = 0;
  }
}

__global__ __launch_bounds__(kSparseBlock) void k_sp_mark(const int2 *__restrict__ pts, int64_t n, Extent p,
                                                          int2 org, uint64_t *__restrict__ L0,
                                                          uint64_t *__restrict__ L1, int32_t *__restrict__ info) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int2 q = pts[i];
    const unsigned xi = (unsigned)(shift_by(q.x, org.x) - 1), yi = (unsigned)(shift_by(q.y, org.y) - 1);
    if (xi >= (unsigned)p.p || yi >= (unsigned)p.q) {
      bad = true;
      continue;
    }
    const unsigned long long old = atomicOr((unsigned long long *)&L0[xi >> 6], 1ull << (xi & 63));
    if (old == 0) atomicOr((unsigned long long *)&L1[xi >> 12], 1ull << ((xi >> 6) & 63));
  }
  if (bad) atomicMin(&info[HP_INFO_STATUS], HP_ERANGE);
}

// One wave per summary word: the occupied columns of its M words.
__global__ __launch_bounds__(kSparseBlock) void k_sp_count(const uint64_t *__restrict__ L0,
                                                           const uint64_t *__restrict__ L1, int64_t W1,
                                                           int32_t *__restrict__ cnt1) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (int64_t)blockIdx.x * (kSparseBlock / kWave) + threadIdx.x / kWave;
  if (i >= W1) return;
  const uint64_t s1 = L1[i];
  int c = ((s1 >> lane) & 1ull) ? __popcll(L0[i * kWave + lane]) : 0;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
  if (lane == 0) cnt1[i] = c;
}

// One workgroup: exclusive offsets of the summary words' counts; k.
__global__ __launch_bounds__(kSparseScan) void k_sp_scan(const int32_t *__restrict__ cnt1, int64_t W1,
                                                         int32_t *__restrict__ off1, int32_t chain_cap,
                                                         int32_t *__restrict__ info) {
  __shared__ int32_t s_sum[kSparseScan];
  const int64_t per = (W1 + kSparseScan - 1) / kSparseScan;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < W1 ? b0 + per : W1;
  int32_t mine = 0;
  for (int64_t b = b0; b < b1; ++b) mine += cnt1[b];
  s_sum[threadIdx.x] = mine;
  __syncthreads();
  for (int d = 1; d < kSparseScan; d <<= 1) {
    const int32_t add = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0;
    __syncthreads();
    s_sum[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = s_sum[threadIdx.x] - mine;
  for (int64_t b = b0; b < b1; ++b) {
    off1[b] = run;
    run += cnt1[b];
  }
  if (threadIdx.x == kSparseScan - 1) {
    const int32_t k = s_sum[threadIdx.x];
    info[HP_INFO_K] = k;
    if (k > chain_cap) atomicMin(&info[HP_INFO_STATUS], HP_ECAPACITY);
  }
}

// One wave per summary word: its occupied columns in x order into the chain,
// (lo, hi) at the sentinel, and each occupied M word's first chain index.
__global__ __launch_bounds__(kSparseBlock) void k_sp_write(const uint64_t *__restrict__ L0,
                                                           const uint64_t *__restrict__ L1, int64_t W1,
                                                           const int32_t *__restrict__ off1,
                                                           int32_t *__restrict__ wordbase, int32_t *__restrict__ cx,
                                                           int32_t *__restrict__ clo, int32_t *__restrict__ chi,
                                                           int32_t chain_cap, int32_t q) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (int64_t)blockIdx.x * (kSparseBlock / kWave) + threadIdx.x / kWave;
  if (i >= W1) return;
  const uint64_t s1 = L1[i];
  const int64_t w = i * kWave + lane;
  uint64_t v = ((s1 >> lane) & 1ull) ? L0[w] : 0ull;
  const int c = __popcll(v);
  int incl = c;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  int j = off1[i] + incl - c;
  if (v) wordbase[w] = j;
  for (; v; v &= v - 1, ++j) {
    if (j >= chain_cap) continue;
    cx[j] = (int32_t)(w * kWave + __builtin_ctzll(v) + 1);
    clo[j] = q + 1;
    chi[j] = -1;
  }
}

__global__ __launch_bounds__(kSparseBlock) void k_sp_fold(const int2 *__restrict__ pts, int64_t n, Extent p,
                                                          int2 org, const uint64_t *__restrict__ L0,
                                                          const int32_t *__restrict__ wordbase,
                                                          int32_t *__restrict__ clo, int32_t *__restrict__ chi,
                                                          int32_t chain_cap) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int2 q = pts[i];
    const int y = shift_by(q.y, org.y);
    const unsigned xi = (unsigned)(shift_by(q.x, org.x) - 1), yi = (unsigned)(y - 1);
    if (xi >= (unsigned)p.p || yi >= (unsigned)p.q) continue;
    const int idx = wordbase[xi >> 6] + __popcll(L0[xi >> 6] & ((1ull << (xi & 63)) - 1ull));
    if (idx >= chain_cap) continue;
    atomicMin(&clo[idx], y);
    atomicMax(&chi[idx], y);
  }
}

__global__ void k_sp_fill(int32_t *__restrict__ lo, int32_t *__restrict__ hi, Extent p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += stride) {
    lo[i] = p.q + 1;
    hi[i] = -1;
  }
}

// s (a column with lo < hi gives two chain points) and the L export.
__global__ __launch_bounds__(kSparseBlock) void k_sp_tail(const int32_t *__restrict__ cx,
                                                          const int32_t *__restrict__ clo,
                                                          const int32_t *__restrict__ chi, int32_t chain_cap,
                                                          int32_t *__restrict__ lo, int32_t *__restrict__ hi,
                                                          int32_t *__restrict__ info) {
  const int k = min(info[HP_INFO_K], chain_cap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int s = 0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k; j += stride) {
    const int a = clo[j], b = chi[j];
    s += 1 + (a < b ? 1 : 0);
    if (lo) {
      lo[cx[j] - 1] = a;
      hi[cx[j] - 1] = b;
    }
  }
  // one device atomic per workgroup
  __shared__ int s_part[kSparseBlock / kWave];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < kSparseBlock / kWave; ++i) t += s_part[i];
    if (t) atomicAdd(&info[HP_INFO_S], t);
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

// Grab counters of the reduce's shared chunks: one slot per run, taken in
// turn, zero-initialised with the module and cleared by the finish step of
// the run that used it.  Runs in flight at the same time on one device take
// different slots unless more than kGrabSlots of them overlap.
constexpr int kGrabSlots = 4096;
__device__ unsigned long long g_grab[kGrabSlots];

static unsigned long long *grab_counter() {
  static std::mutex mu;
  static unsigned long long *base[64] = {};
  static std::atomic<uint32_t> seq{0};
  const int d = device_info().device;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!base[d]) {
      void *ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_grab)) != hipSuccess || !ptr) return nullptr;
      base[d] = static_cast<unsigned long long *>(ptr);
    }
  }
  return base[d] + (seq.fetch_add(1, std::memory_order_relaxed) % kGrabSlots);
}

// Chunks per reduce workgroup from which the chunks are shared.
constexpr int64_t kDynMinChunks = 32;

// Static share of the shared-chunk reduce in eighths (HP_DYN_STATIC8, 0..8;
// HP_DYN_OFF=1 turns chunk sharing off).
// HP_NODE_FINISH_OFF=1: the slab-per-workgroup finish and the all-vertex
// level-2 test also for clouds of more than one level-2 node.
static bool node_finish_off() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("HP_NODE_FINISH_OFF");
    v = (e && atoi(e) == 1) ? 1 : 0;
  }
  return v == 1;
}

static int dyn_static8() {
  static int v = -2;
  if (v == -2) {
    const char *off = getenv("HP_DYN_OFF");
    const char *e = getenv("HP_DYN_STATIC8");
    v = (off && atoi(off) == 1) ? -1 : (e ? std::max(0, std::min(8, atoi(e))) : 6);
  }
  return v;
}

struct Layout {
  size_t ctl, tree, wg_err, wg_cnt, filt, slab_k, slab_s, slab_off, Lm, part, cand, keep, l2cnt, ccount, bins,
      total;
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Largest reduce grid any strategy or tuned override may use.
constexpr int kMaxGrid = 4096;
// Largest p whose chain the scan root writes itself (no k_chain launch).
constexpr int32_t kChainInline = 32768;
// Most slabs whose scan the last slab to finish does (above: a scan launch).
constexpr int32_t kScanRootMaxSlabs = 256;

// Survival bytes per side: positions rounded up to whole level-2 nodes, so
// the level-2 test's flags (node * 4096 + vertex) stay in range and aligned.
static size_t keep_side_bytes(int64_t positions) {
  const int64_t P = positions < 1 ? 1 : positions;
  return (size_t)((P + kNodeVerts - 1) / kNodeVerts) * kNodeVerts;
}

static Layout make_layout(int64_t positions, int32_t p, int64_t part_pairs, const TreeShape &T,
                          size_t bins_bytes = 0) {
  Layout Y;
  size_t o = 0;
  Y.ctl = o;      o = align_up(o + sizeof(int32_t) * kCtlWords);
  Y.tree = o;     o = align_up(o + sizeof(int32_t) * (size_t)T.nodes);
  Y.wg_err = o;   o = align_up(o + sizeof(int32_t) * (size_t)kMaxGrid);
  Y.wg_cnt = o;   o = align_up(o + sizeof(int32_t) * (size_t)kMaxGrid);
  // the sampled filter's pairs, or the binned reduce's 16-bit words per 64
  // columns (rounded up to 8 words) followed by its words per 32 columns
  Y.filt = o;     o = align_up(o + sizeof(int2) * (size_t)((p > 0 ? (int64_t)p + 63 : 0) / 64) + 16);
  Y.slab_k = o;   o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.slab_s = o;   o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.slab_off = o; o = align_up(o + sizeof(int32_t) * (size_t)T.size[1]);
  Y.Lm = o;       o = align_up(o + sizeof(int2) * (size_t)(p > 0 ? p : 0));
  Y.part = o;     o = align_up(o + sizeof(int2) * (size_t)part_pairs);
  Y.cand = o;     o = align_up(o + sizeof(int2) * 4 * (size_t)positions);
  Y.keep = o;     o = align_up(o + 2 * keep_side_bytes(positions));
  Y.l2cnt = o;    o = align_up(o + sizeof(int32_t) * 2 * kL2MaxParts * (size_t)(T.nlev >= 2 ? T.size[2] : 1));
  Y.ccount = o;   o = align_up(o + sizeof(int32_t) * 2 * (size_t)T.nodes);
  Y.bins = o;     o = align_up(o + bins_bytes);
  Y.total = o;
  return Y;
}

static int64_t lds_grid_max();

struct Plan1 {
  int strategy;
  int block, vpt, G;   // G: workgroups of the reduce
  int W, wc;           // column windows (HP_STRATEGY_WINDOW): count and columns each
};

// Shape of the binned reduce for (n, p), p <= kBinPMax: G binning workgroups
// (one per CU), S fold slices per window, one round, or two from n >= 32 p
// (the first over the first quarter of the points, an even count so that
// the second round's points keep the alignment of pts), and the pages each
// binning workgroup may need: its points of the larger round over the page
// size, plus one partly filled page per window.
struct BinPlan {
  int G, S, S2, nw, pages, rounds;   // S (S2): partial arrays of the first (second) round
  int64_t split;   // points of the first round
  int64_t segcap;  // points a workgroup's compaction segment holds (0: no compaction)
};

// The second round's compaction keeps at most this fraction of a
// workgroup's points (1 / kBinCompactDiv); when more pass the filter in some
// workgroup, the round bins all of its points with the filter instead.
// HP_BIN_COMPACT_OFF=1 turns it off.
constexpr int64_t kBinCompactDiv = 4;
static bool bin_compact_off() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("HP_BIN_COMPACT_OFF");
    v = (e && atoi(e) == 1) ? 1 : 0;
  }
  return v == 1;
}

constexpr int64_t kBinRoundsMinPerCol = 32;

// Partial arrays of the second round at most: it folds far fewer entries
// than the first, and every array costs the finish a read of 8p bytes.
constexpr int kBinS2 = 3;
// Fold workgroups per CU and round (nw windows x S slices): each holds a
// window's L and its page lists in 40 KB of LDS.  More slices fold fewer
// entries each but write more partial arrays for the merge to read back.
constexpr int kBinFoldPerCu = 3;

// Points per binning workgroup and round at most, so that a stream's page
// index fits the 16 bits the page records give it.
constexpr int64_t kBinMaxPerWg = (int64_t)1 << 25;

static BinPlan bin_plan(int64_t n, int32_t p) {
  BinPlan B;
  B.nw = (int)(((int64_t)p + kBinWc - 1) / kBinWc);
  B.rounds = n >= kBinRoundsMinPerCol * (int64_t)p ? 2 : 1;
  B.split = B.rounds == 2 ? (n / 4) & ~(int64_t)1 : n;
  const int64_t m = std::max<int64_t>(B.split, n - B.split);
  const int64_t nv = m / 2 + 1;
  const int64_t ntiles = (nv + kBinTileV - 1) / kBinTileV;
  B.G = (int)std::max<int64_t>(device_info().cus, (m + kBinMaxPerWg - 1) / kBinMaxPerWg);
  B.S = (int)std::max<int64_t>(1, std::min<int64_t>(B.G, (int64_t)kBinFoldPerCu * device_info().cus / B.nw));
  B.S2 = std::min(B.S, kBinS2);
  const int64_t tpw = (ntiles + B.G - 1) / B.G;
  const int64_t per_wg = tpw * 2 * (int64_t)kBinTileV + 2;
  B.pages = (int)((per_wg + kBinPage - 1) / kBinPage + B.nw + 1);
  B.segcap = 0;
  if (B.rounds == 2 && !bin_compact_off()) {
    const int64_t vpw = ((n - B.split + 1) / 2 + B.G - 1) / B.G;   // vectors per workgroup, at most
    B.segcap = ((2 * vpw + kBinCompactDiv - 1) / kBinCompactDiv + 2 + 1) & ~(int64_t)1;
  }
  return B;
}

// Partial arrays the finish folds: the last round's, plus the running L
// (array S2) when there are two rounds.
static int bin_partials(const BinPlan &B) { return B.rounds > 1 ? B.S2 + 1 : B.S; }
// Partial arrays held: the first round writes S of them, and the running L
// sits at index S2.
static int bin_part_storage(const BinPlan &B) { return B.rounds > 1 ? std::max(B.S, B.S2 + 1) : B.S; }

// Device bytes of the binned reduce's pages and tables.
struct BinLayout {
  size_t pool, E, pg_off, pg_list, pwin, cpts, ccount, cover, total;
};
static BinLayout bin_layout(const BinPlan &B) {
  BinLayout Z;
  size_t o = 0;
  Z.pool = o;    o = align_up(o + sizeof(uint32_t) * (size_t)B.G * (size_t)B.pages * kBinPage);
  Z.E = o;       o = align_up(o + sizeof(int32_t) * (size_t)B.G * (size_t)B.nw);
  Z.pg_off = o;  o = align_up(o + sizeof(int32_t) * (size_t)B.G * (size_t)(B.nw + 1));
  Z.pg_list = o; o = align_up(o + sizeof(int32_t) * (size_t)B.G * (size_t)B.pages);
  Z.pwin = o;    o = align_up(o + sizeof(int32_t) * (size_t)B.G * (size_t)B.pages);
  Z.cpts = o;    o = align_up(o + sizeof(int2) * (size_t)B.G * (size_t)B.segcap);
  Z.ccount = o;  o = align_up(o + sizeof(int64_t) * (size_t)B.G);
  Z.cover = o;   o = align_up(o + sizeof(int32_t));
  Z.total = o;
  return Z;
}

// Sampled filter: used by default from this many points per column; the
// sample is the first 1/sample_div() of the points (HP_SAMPLE_DIV, 2..64).
constexpr int64_t kSampledMinPerCol = 16;
static int64_t sample_div() {
  static int64_t v = 0;
  if (v == 0) {
    const char *e = getenv("HP_SAMPLE_DIV");
    v = e ? std::max<int64_t>(2, std::min<int64_t>(64, atoll(e))) : 8;
  }
  return v;
}

// End of the filtered pass that starts after `lo` points: four times lo, or
// n (a pass that starts at 0, after an empty sample, takes every point).
static int64_t sampled_stage_end(int64_t lo, int64_t n) { return lo <= 0 ? n : std::min<int64_t>(n, 4 * lo); }

// Filtered passes after a sample of ns points, and where the last one starts.
static int sampled_stages(int64_t ns, int64_t n, int64_t *last_start = nullptr) {
  int k = 0;
  int64_t at = ns;
  for (int64_t lo = ns; lo < n; lo = sampled_stage_end(lo, n)) {
    ++k;
    at = lo;
  }
  if (last_start) *last_start = at;
  return k;
}

// Column windows: at most kWinMax windows, at most kWinMaxGroups chunk
// groups (a multiple of 8: one per XCD slot).
constexpr int kWinMax = 8;
constexpr int kWinMaxGroups = 64;

// Partial arrays the reduce writes (each p packed words), or 0.
static int partial_count(const Plan1 &P, int64_t n, int32_t p) {
  if (P.strategy == HP_STRATEGY_LDS_PARTIAL) return P.G;
  if (P.strategy == HP_STRATEGY_WINDOW) return P.G / P.W;
  if (P.strategy == HP_STRATEGY_BINNED) return bin_partials(bin_plan(n, p));
  return 0;
}

static bool is_lds(int s) { return s == HP_STRATEGY_LDS || s == HP_STRATEGY_LDS_PARTIAL; }

// allow_binned: the workspace holds the binned reduce's pages (else a plan
// that would bin uses the sampled filter or the device L instead).
// q: the rows of the box (0: the square, q = p).  Packed partial words need
// fewer than 2^16 - 1 rows and the binned entries at most kBinPMax.
static Plan1 choose(int64_t n, int32_t p, bool allow_binned = true, int32_t q = 0) {
  const DeviceInfo &D = device_info();
  if (q <= 0) q = p;
  Plan1 P;
  int s = forced_strategy();
  if (s == HP_STRATEGY_AUTO) s = n * kSparseRatio < (int64_t)p ? HP_STRATEGY_SPARSE : tuned_strategy(n, p);
  if (s == HP_STRATEGY_SPARSE) {
    P.strategy = s;
    P.block = kSparseBlock;
    P.vpt = 1;
    P.G = 1;
    P.W = 1;
    P.wc = p;
    return P;
  }
  if (s == HP_STRATEGY_BINNED && ((int64_t)p > kBinPMax || (int64_t)q > kBinPMax || !allow_binned))
    s = HP_STRATEGY_SAMPLED;
  if (s == HP_STRATEGY_LDS_PARTIAL && !partial_packs(q)) s = HP_STRATEGY_LDS;
  if (s == HP_STRATEGY_SAMPLED && n < kSampledMinPerCol * (int64_t)p) s = HP_STRATEGY_GLOBAL;
  P.W = 1;
  P.wc = p;
  if ((is_lds(s) && (int64_t)p > D.lds_max_p) || s == HP_STRATEGY_WINDOW) {
    // column windows when the L does not fit LDS (or when asked for)
    const int64_t W = ((int64_t)p + D.lds_max_p - 1) / D.lds_max_p;
    if (W <= kWinMax && (s == HP_STRATEGY_WINDOW || n >= 4 * (int64_t)p)) {
      s = HP_STRATEGY_WINDOW;
      P.W = (int)W;
      P.wc = (int)(((int64_t)p + W - 1) / W);
    } else {
      // beyond the windows: a device L, with the sampled filter when every
      // column gets enough points for the sample to bound it
      s = n >= kSampledMinPerCol * (int64_t)p ? HP_STRATEGY_SAMPLED : HP_STRATEGY_GLOBAL;
    }
  }
  P.strategy = s;
  P.block = 1024;
  P.vpt = 4;
  if (is_lds(s)) {
    // one workgroup per CU (or fewer when the cloud is small: every
    // workgroup should see several points per column, since its private L
    // costs 8p bytes of LDS initialisation and of merge traffic)
    const int64_t per_wg_min = 4 * (int64_t)p;
    int64_t G = per_wg_min > 0 ? n / per_wg_min : 1;
    if (G > D.cus) G = D.cus;
    if (G < 1) G = 1;
    P.G = (int)G;
  } else if (s == HP_STRATEGY_WINDOW) {
    P.G = D.cus;   // chunk groups x windows, fixed below
  } else if (s == HP_STRATEGY_BINNED) {
    P.G = bin_plan(n, p).G;
  } else {
    const int64_t vecs = (n + 1) / 2;
    int64_t G = (vecs + (int64_t)P.block * P.vpt - 1) / ((int64_t)P.block * P.vpt);
    const int64_t gmax = (int64_t)D.cus * 2;
    if (G > gmax) G = gmax;
    if (G < 1) G = 1;
    P.G = (int)G;
  }
  if (s == HP_STRATEGY_BINNED) return P;   // fixed launch shapes
  tune_override(n, p, &P.block, &P.vpt, &P.G);
  if (s == HP_STRATEGY_WINDOW) {
    int groups = (P.G / P.W) / 8 * 8;
    groups = std::max(8, std::min(kWinMaxGroups, groups));
    P.G = groups * P.W;
  }
  if (is_lds(P.strategy) && P.G > lds_grid_max()) P.G = (int)lds_grid_max();
  if (P.G > kMaxGrid) P.G = kMaxGrid;
  if (P.G < 1) P.G = 1;
  return P;
}

// Pairs of the reduce output region: G partial L arrays for the partial
// variant, otherwise nothing (the device L is the merged-L region).
static int64_t part_pairs_for(const Plan1 &P, int64_t n, int32_t p, int32_t q = 0) {
  // the binned reduce writes pairs; the other partials pack into half a pair
  // when the rows allow
  if (P.strategy == HP_STRATEGY_BINNED) return (int64_t)bin_part_storage(bin_plan(n, p)) * p;
  const int64_t entries = (int64_t)partial_count(P, n, p) * p;
  return partial_packs(q > 0 ? q : p) ? (entries + 1) / 2 : entries;
}

static size_t bins_bytes_for(const Plan1 &P, int64_t n, int32_t p) {
  return P.strategy == HP_STRATEGY_BINNED ? bin_layout(bin_plan(n, p)).total : 0;
}

// Largest grid the LDS strategies may use (also bounds tuned overrides).
static int64_t lds_grid_max() { return (int64_t)device_info().cus * 4; }

// Workspace for (n, p): sized for the largest partial-L array any strategy or
// override may use, so that a later strategy change still fits the same
// workspace; with_bins adds the binned reduce's pages (for p <= kBinPMax),
// without them a plan that would bin falls back (see choose).
// The sparse path's workspace: the hull of a chain of min(n, p) positions,
// then M (used when the caller gives no M export), its summary level, the
// summary counts and offsets, and a first chain index per M word.
struct SparseLayout {
  int32_t hpos;
  TreeShape T;
  Layout Yh;
  size_t L0, L1, cnt1, off1, wordbase, total;
};
static SparseLayout sparse_layout(int64_t n, int32_t p) {
  SparseLayout Z;
  Z.hpos = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n, p));
  Z.T = make_tree(Z.hpos);
  Z.Yh = make_layout(Z.hpos, 0, 0, Z.T);
  const int64_t W0 = ((int64_t)p + 63) / 64, W1 = (W0 + 63) / 64;
  size_t o = Z.Yh.total;
  Z.L0 = o;       o = align_up(o + sizeof(uint64_t) * (size_t)W0);
  Z.L1 = o;       o = align_up(o + sizeof(uint64_t) * (size_t)W1);
  Z.cnt1 = o;     o = align_up(o + sizeof(int32_t) * (size_t)W1);
  Z.off1 = o;     o = align_up(o + sizeof(int32_t) * (size_t)W1);
  Z.wordbase = o; o = align_up(o + sizeof(int32_t) * (size_t)W0);
  Z.total = o;
  return Z;
}

static size_t ws_bytes_for(int64_t n, int32_t p, bool with_bins = true, int32_t q = 0) {
  if (q <= 0) q = p;
  const size_t sparse = sparse_layout(n, p).total;
  const TreeShape T = make_tree(p);
  const int64_t lds_max = device_info().lds_max_p;
  int64_t part = 0;
  if ((int64_t)p <= lds_max && partial_packs(q)) part = (lds_grid_max() * p + 1) / 2;
  if ((int64_t)p <= kWinMax * lds_max) {
    const int64_t entries = (int64_t)kWinMaxGroups * p;
    part = std::max<int64_t>(part, partial_packs(q) ? (entries + 1) / 2 : entries);
  }
  size_t bins = 0;
  if (with_bins && (int64_t)p <= kBinPMax && (int64_t)q <= kBinPMax) {
    const BinPlan B = bin_plan(n, p);
    part = std::max<int64_t>(part, (int64_t)bin_part_storage(B) * p);
    bins = bin_layout(B).total;
  }
  return std::max(sparse, make_layout(p, p, part, T, bins).total);
}

template <typename K, typename... Args>
static hipError_t launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, Args... args) {
  if (e0)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  return hipGetLastError();
}

template <int BLOCK, int VPT, bool ATOMIC>
static hipError_t launch_lds(const Plan1 &P, const int32_t *pts, int64_t n, Extent p, int2 *out,
                             int32_t *wg_err, ResetArgs R, DynArgs D, int2 org, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_reduce_lds<BLOCK, VPT, ATOMIC>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             device_info().lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  return launch(k_reduce_lds<BLOCK, VPT, ATOMIC>, dim3(P.G), dim3(BLOCK), sizeof(int2) * ((size_t)p + 2), s,
                e0, e1, pts, n, p, out, wg_err, R, D, org);
}

template <int BLOCK, int VPT>
static hipError_t launch_reduce(const Plan1 &P, const int32_t *pts, int64_t n, Extent p, int2 *Lm,
                                int2 *part, int32_t *wg_err, ResetArgs R, DynArgs D, int2 org, hipStream_t s,
                                hipEvent_t e0, hipEvent_t e1) {
  if (P.strategy == HP_STRATEGY_LDS)
    return launch_lds<BLOCK, VPT, true>(P, pts, n, p, Lm, wg_err, R, D, org, s, e0, e1);
  if (P.strategy == HP_STRATEGY_LDS_PARTIAL)
    return launch_lds<BLOCK, VPT, false>(P, pts, n, p, part, wg_err, R, D, org, s, e0, e1);
  if (P.strategy == HP_STRATEGY_WINDOW) {
    static bool attr_set = false;
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute((const void *)k_reduce_window<BLOCK, VPT>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               device_info().lds_bytes);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    return launch(k_reduce_window<BLOCK, VPT>, dim3(P.G), dim3(BLOCK), sizeof(int2) * ((size_t)P.wc + 1), s,
                  e0, e1, pts, n, p, P.W, P.wc, reinterpret_cast<uint32_t *>(part), wg_err, R, org);
  }
  return launch(k_reduce_global<BLOCK, VPT>, dim3(P.G), dim3(BLOCK), 0, s, e0, e1, pts, n, p, Lm,
                wg_err, R, D, org);
}

static hipError_t dispatch_reduce(const Plan1 &P, const int32_t *pts, int64_t n, Extent p, int2 *Lm,
                                  int2 *part, int32_t *wg_err, ResetArgs R, DynArgs D, int2 org, hipStream_t s,
                                  hipEvent_t e0, hipEvent_t e1) {
#define HP_CASE(B, V) \
  if (P.block == B && P.vpt == V)   \
    return launch_reduce<B, V>(P, pts, n, p, Lm, part, wg_err, R, D, org, s, e0, e1);
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

// The sampled-filter reduce: the sample pass (k_reduce_global over the
// first ns points, G1 workgroups), then filtered passes, each over up to
// three times the points folded before it and each after a filter rebuilt
// from the fuller L (so tighter); with the default sample of n/8 these are
// [n/8, n/2) and [n/2, n).  The filtered passes use P.G workgroups each and
// only the last one shares chunks.  e0 is recorded at the start of the
// sample pass and e1 at the end of the last pass.
template <int BLOCK, int VPT>
static hipError_t launch_sampled(const Plan1 &P, const int32_t *pts, int64_t n, Extent p, int2 *Lm,
                                 int2 *F, int fshift, int ngroups, int64_t ns, int G1,
                                 int32_t *wg_err, DynArgs D, int2 org, hipStream_t s, hipEvent_t e0,
                                 hipEvent_t e1) {
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_reduce_filtered<BLOCK, VPT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             device_info().lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  ResetArgs R;
  memset(&R, 0, sizeof(R));
  DynArgs D0 = D;
  D0.ctr = nullptr;
  if (e0) hipExtLaunchKernelGGL((k_reduce_global<BLOCK, VPT>), dim3(G1), dim3(BLOCK), 0, s, e0, nullptr, 0, pts, ns, p,
                                Lm, wg_err, R, D0, org);
  else hipLaunchKernelGGL((k_reduce_global<BLOCK, VPT>), dim3(G1), dim3(BLOCK), 0, s, pts, ns, p, Lm, wg_err, R, D0,
                          org);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(int2) * ((size_t)ngroups + 2 + (size_t)(BLOCK / kWave) * filt_queue_cap(VPT));
  // the filtered passes: each folds up to three times the points folded
  // before it, with the filter rebuilt from the fuller L in between
  int stage = 0;
  for (int64_t lo = ns; lo < n; ++stage) {
    const int64_t hi = sampled_stage_end(lo, n);
    const bool last = hi == n;
    hipLaunchKernelGGL(k_filter_build, dim3((ngroups + 3) / 4), dim3(256), 0, s, (const int2 *)Lm, p, fshift,
                       ngroups, F);
    int32_t *err = wg_err + G1 + (size_t)stage * P.G;
    if (last && e1)
      hipExtLaunchKernelGGL((k_reduce_filtered<BLOCK, VPT>), dim3(P.G), dim3(BLOCK), (uint32_t)lds, s, nullptr, e1, 0,
                            pts + 2 * lo, hi - lo, p, Lm, (const int2 *)F, fshift, ngroups, err, D, org);
    else
      hipLaunchKernelGGL((k_reduce_filtered<BLOCK, VPT>), dim3(P.G), dim3(BLOCK), lds, s, pts + 2 * lo, hi - lo, p,
                         Lm, (const int2 *)F, fshift, ngroups, err, last ? D : D0, org);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    lo = hi;
  }
  return hipSuccess;
}

static hipError_t dispatch_sampled(const Plan1 &P, const int32_t *pts, int64_t n, Extent p, int2 *Lm, int2 *F,
                                   int fshift, int ngroups, int64_t ns, int G1, int32_t *wg_err,
                                   DynArgs D, int2 org, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
#define HP_CASE(B, V) \
  if (P.block == B && P.vpt == V)   \
    return launch_sampled<B, V>(P, pts, n, p, Lm, F, fshift, ngroups, ns, G1, wg_err, D, org, s, e0, e1);
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

// The binned reduce (p <= kBinPMax): per round k_bin over the round's points,
// k_bin_fold into S partial arrays, and between rounds k_bin_merge into the
// running L (array S) and the filter of the next round; in the second round
// k_bin_compact first keeps the points that filter cannot drop, and k_bin
// bins those.  e0 is recorded at
// the start of the first k_bin and e1 at the end of the last k_bin_fold.
static hipError_t launch_binned(const int32_t *pts, int64_t n, Extent p, int2 *part, uint16_t *F, char *bins,
                                int32_t *wg_err, ResetArgs R, int2 org, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
  const BinPlan B = bin_plan(n, p);
  const BinLayout Z = bin_layout(B);
  BinArgs A;
  A.pool = reinterpret_cast<uint32_t *>(bins + Z.pool);
  A.E = reinterpret_cast<int32_t *>(bins + Z.E);
  A.pg_off = reinterpret_cast<int32_t *>(bins + Z.pg_off);
  A.pg_list = reinterpret_cast<int32_t *>(bins + Z.pg_list);
  A.pwin = reinterpret_cast<int32_t *>(bins + Z.pwin);
  A.pages = B.pages;
  A.nw = B.nw;
  A.G = B.G;
  const int nf = (int)(((int64_t)p + (1 << kBinFilterShift) - 1) >> kBinFilterShift);
  // filter bounds in 8 bits: y - 1 < q in steps of 2^qs
  int qs = 0;
  while ((((int64_t)p.q - 1) >> qs) > 255) ++qs;
  if (B.nw > kBinNwMax || bin_lds_bytes(nf) > (size_t)device_info().lds_bytes || B.rounds * B.G > kMaxGrid)
    return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_bin, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             device_info().lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  int2 *cpts = reinterpret_cast<int2 *>(bins + Z.cpts);
  int64_t *ccount = reinterpret_cast<int64_t *>(bins + Z.ccount);
  int32_t *cover = reinterpret_cast<int32_t *>(bins + Z.cover);
  // the compaction's 32-column filter follows the 64-column one in the
  // filter region (8 bytes per 64 columns)
  const int nf32 = (int)(((int64_t)p + (1 << kCpFilterShift) - 1) >> kCpFilterShift);
  uint16_t *F32 = B.segcap > 0 ? F + ((nf + 7) & ~7) : nullptr;
  if (B.segcap > 0 && nf32 > kCpFilterMax) return hipErrorInvalidValue;
  for (int r = 0; r < B.rounds; ++r) {
    const int64_t a = r == 0 ? 0 : B.split, b = r == 0 ? B.split : n;
    ResetArgs Rr = R;
    if (r > 0) Rr.ctl = nullptr;
    const uint16_t *Fr = r > 0 ? F : nullptr;
    const uint32_t lds = (uint32_t)bin_lds_bytes(r > 0 ? nf : 0);
    const int32_t *pr = pts ? pts + 2 * a : pts;
    int32_t *err = wg_err + (size_t)r * B.G;
    const bool compact = r > 0 && B.segcap > 0;
    if (compact)   // the points the filter keeps, a segment per binning workgroup
      hipLaunchKernelGGL(k_bin_compact, dim3(B.G), dim3(kCpThreads), 0, s, pr, b - a, p, F32, nf32, qs, org, cpts,
                         B.segcap, ccount, cover);
    const int2 *cp = compact ? cpts : nullptr;
    if (r == 0 && e0)
      hipExtLaunchKernelGGL(k_bin, dim3(B.G), dim3(kBinThreads), lds, s, e0, nullptr, 0, pr, b - a, p, Fr, nf, qs, A,
                            err, org, Rr, cp, (const int64_t *)ccount, B.segcap, (const int32_t *)cover);
    else
      hipLaunchKernelGGL(k_bin, dim3(B.G), dim3(kBinThreads), lds, s, pr, b - a, p, Fr, nf, qs, A, err, org, Rr, cp,
                         (const int64_t *)ccount, B.segcap, (const int32_t *)cover);
    const int Sr = r == 0 ? B.S : B.S2;   // this round's partial arrays
    const dim3 gf((unsigned)(B.nw * Sr));
    if (r + 1 == B.rounds && e1)
      hipExtLaunchKernelGGL(k_bin_fold, gf, dim3(kBinFoldThreads), 0, s, nullptr, e1, 0, A, p, Sr, part);
    else
      hipLaunchKernelGGL(k_bin_fold, gf, dim3(kBinFoldThreads), 0, s, A, p, Sr, part);
    if (r + 1 < B.rounds)   // the running L goes to array S2, which the next round's fold leaves alone
      hipLaunchKernelGGL(k_bin_merge, dim3((unsigned)(((int64_t)p + 255) / 256)), dim3(256), 0, s, part, Sr,
                         r > 0 ? 1 : 0, B.S2, p, qs, F, F32, B.segcap > 0 ? cover : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Hull levels 2..nlev: a test launch and a compaction launch per level (the
// slab level ran in k_finish).  H must have its chain fields filled.
static void hull_buffers(HullArgs &H, const TreeShape &T, int64_t positions, char *w, const Layout &Y) {
  H.buf[0] = reinterpret_cast<int2 *>(w + Y.cand);
  H.buf[1] = H.buf[0] + 2 * (size_t)positions;
  H.keep = reinterpret_cast<uint8_t *>(w + Y.keep);
  H.keep_side = (int64_t)keep_side_bytes(positions);
  H.l2cnt = reinterpret_cast<int32_t *>(w + Y.l2cnt);
  H.ccount = reinterpret_cast<int32_t *>(w + Y.ccount);
  H.tree = T;
  H.positions = (int32_t)positions;
}

// Test workgroups per node level, about.  Each stages every sibling's hull,
// so more of them repeat that work: on the 2^20-column disc (256 nodes under
// 4 parents) 512 took the step 13 us below 1024, and 256 matched 512.
constexpr int kHullTestWgs = 512;
constexpr int kHullMaxSplit = 64;   // test workgroups per child, at most

static hipError_t launch_hull_levels(const TreeShape &T, int64_t positions, char *w, const Layout &Y,
                                     HullArgs H, bool small, hipStream_t s, bool l2path = false,
                                     bool l2_done = false) {
  if (T.nlev < 2) return hipSuccess;
  hull_buffers(H, T, positions, w, Y);
  int first = 2;
  if (l2_done) {
    // the level-2 nodes' hulls are in place (k_node_finish)
    first = 3;
    l2path = false;
  }
  if (l2path && T.nlev == 2) {
    // a single level-2 node: its test workgroups also write the hull (two
    // per slab, at least one per slab for the chain)
    H.split = std::min(kL2MaxParts, 2 * T.size[1]);
    if (small) hipLaunchKernelGGL((k_l2_root<true>), dim3(H.split), dim3(kHullBlock), 0, s, H);
    else hipLaunchKernelGGL((k_l2_root<false>), dim3(H.split), dim3(kHullBlock), 0, s, H);
    return hipGetLastError();
  }
  if (l2path) {
    // level 2 by the all-vertex test, which also writes the chain and the
    // totals (H carries the chain fields and the slab counts)
    // test workgroups per node: about kL2TargetWgs in all, 4 to kL2MaxParts per node
    H.split = std::max(4, std::min(kL2MaxParts, kL2TargetWgs / T.size[2]));
    const dim3 gt(T.size[2] * H.split), gc(T.size[2]);
    if (small) {
      hipLaunchKernelGGL((k_l2_test<true>), gt, dim3(kHullBlock), 0, s, H);
      hipLaunchKernelGGL((k_l2_compact<true>), gc, dim3(kHullBlock), 0, s, H);
    } else {
      hipLaunchKernelGGL((k_l2_test<false>), gt, dim3(kHullBlock), 0, s, H);
      hipLaunchKernelGGL((k_l2_compact<false>), gc, dim3(kHullBlock), 0, s, H);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    first = 3;
  }
  for (int lev = first; lev <= T.nlev; ++lev) {
    // slab children get kSplitSlab test workgroups each; node children
    // enough for about kHullTestWgs in all (each stages every sibling's hull)
    H.split = lev == 2 ? kSplitSlab
                       : std::max(1, std::min(kHullMaxSplit, kHullTestWgs / std::max(1, T.size[lev - 1])));
    const dim3 gt(T.size[lev - 1] * H.split), gc(T.size[lev]);
    if (small) {
      hipLaunchKernelGGL((k_hull_test<true>), gt, dim3(kHullBlock), 0, s, H, lev);
      hipLaunchKernelGGL((k_hull_compact<true>), gc, dim3(kHullBlock), 0, s, H, lev);
    } else {
      hipLaunchKernelGGL((k_hull_test<false>), gt, dim3(kHullBlock), 0, s, H, lev);
      hipLaunchKernelGGL((k_hull_compact<false>), gc, dim3(kHullBlock), 0, s, H, lev);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int hull_of_chain(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t positions,
                         int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, char *w, const Layout &Y,
                         const TreeShape &T, hipStream_t s, bool small);

// The node finish's LDS beyond the default limit, set once per process.
static bool node_lds_ready() {
  static int state = 0;
  if (state == 0) {
    const int bytes = (int)sizeof(NodeShared);
    const void *k[] = {(const void *)k_node_finish<kPrecSmall, false>, (const void *)k_node_finish<kPrecNode, false>,
                       (const void *)k_node_finish<kPrecSmall, true>, (const void *)k_node_finish<kPrecWide, true>};
    bool ok = true;
    for (const void *f : k) ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    state = ok ? 1 : 2;
  }
  return state == 1;
}

// The sparse path (HP_STRATEGY_SPARSE): work in the points and the occupied
// columns, plus ceil(p/64) words of M; L is written only as the export.
static int run_sparse(const int32_t *pts, int64_t n, Extent p, int32_t *lo, int32_t *hi, uint64_t *mask,
                      int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx, int32_t *hy,
                      int32_t hull_cap, int32_t *info, char *w, size_t ws_bytes, hipStream_t s, bool do_hull,
                      int2 org) {
  const SparseLayout Z = sparse_layout(n, p);
  if (ws_bytes < Z.total) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, Z.total);
  const int64_t W0 = ((int64_t)p + 63) / 64, W1 = (W0 + 63) / 64;
  uint64_t *L0 = mask ? mask : reinterpret_cast<uint64_t *>(w + Z.L0);
  uint64_t *L1 = reinterpret_cast<uint64_t *>(w + Z.L1);
  int32_t *cnt1 = reinterpret_cast<int32_t *>(w + Z.cnt1);
  int32_t *off1 = reinterpret_cast<int32_t *>(w + Z.off1);
  int32_t *wordbase = reinterpret_cast<int32_t *>(w + Z.wordbase);
  const int cus = device_info().cus;
  const int gw = (int)std::max<int64_t>(1, std::min<int64_t>(4 * cus, (W0 + kSparseBlock - 1) / kSparseBlock));
  const int gp = (int)std::max<int64_t>(1, std::min<int64_t>(8 * cus, (n + kSparseBlock - 1) / kSparseBlock));
  const int gs = (int)((W1 + kSparseBlock / kWave - 1) / (kSparseBlock / kWave));
  const int2 *P2 = reinterpret_cast<const int2 *>(pts);
  // the timed reduce runs from the clearing of M to the fold of the points
  hipEvent_t e0 = nullptr, e1 = nullptr;
  timing_slot(&e0, &e1);
  if (e0)
    hipExtLaunchKernelGGL(k_sp_clear, dim3(gw), dim3(kSparseBlock), 0, s, e0, nullptr, 0, L0, W0, L1, W1, info);
  else
    hipLaunchKernelGGL(k_sp_clear, dim3(gw), dim3(kSparseBlock), 0, s, L0, W0, L1, W1, info);
  if (n > 0) hipLaunchKernelGGL(k_sp_mark, dim3(gp), dim3(kSparseBlock), 0, s, P2, n, p, org, L0, L1, info);
  hipLaunchKernelGGL(k_sp_count, dim3(gs), dim3(kSparseBlock), 0, s, (const uint64_t *)L0, (const uint64_t *)L1,
                     W1, cnt1);
  hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(kSparseScan), 0, s, (const int32_t *)cnt1, W1, off1, chain_cap, info);
  hipLaunchKernelGGL(k_sp_write, dim3(gs), dim3(kSparseBlock), 0, s, (const uint64_t *)L0, (const uint64_t *)L1, W1,
                     (const int32_t *)off1, wordbase, cx, clo, chi, chain_cap, p.q);
  if (e1)   // with no points the fold is an empty grid-stride loop, kept for the stop event
    hipExtLaunchKernelGGL(k_sp_fold, dim3(gp), dim3(kSparseBlock), 0, s, nullptr, e1, 0, P2, n, p, org,
                          (const uint64_t *)L0, (const int32_t *)wordbase, clo, chi, chain_cap);
  else if (n > 0)
    hipLaunchKernelGGL(k_sp_fold, dim3(gp), dim3(kSparseBlock), 0, s, P2, n, p, org, (const uint64_t *)L0,
                       (const int32_t *)wordbase, clo, chi, chain_cap);
  if (lo) {
    const int gl = (int)std::max<int64_t>(1, std::min<int64_t>(8 * cus, ((int64_t)p + kSparseBlock - 1) / kSparseBlock));
    hipLaunchKernelGGL(k_sp_fill, dim3(gl), dim3(kSparseBlock), 0, s, lo, hi, p);
  }
  const int gk = (int)std::max<int64_t>(1, std::min<int64_t>(4 * cus, ((int64_t)Z.hpos + kSparseBlock - 1) / kSparseBlock));
  hipLaunchKernelGGL(k_sp_tail, dim3(gk), dim3(kSparseBlock), 0, s, (const int32_t *)cx, (const int32_t *)clo,
                     (const int32_t *)chi, chain_cap, lo, hi, info);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "sparse path launch: %s", hipGetErrorString(e));
  if (!do_hull) return HP_OK;
  // chain coordinates are at most max(p, q): below 2^15 the hull runs on 24-bit products
  return hull_of_chain(cx, clo, chi, Z.hpos, hx, hy, hull_cap, info, w, Z.Yh, Z.T, s,
                       std::max(p.p, p.q) < (1 << 15));
}

// Enqueue the whole single-cloud sequence.  Shared by hp_precondition,
// hp_run and the per-cloud baseline of the batched form.
int run_single(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi, uint64_t *mask,
               int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx, int32_t *hy,
               int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes, hipStream_t s,
               bool do_hull, int32_t ox, int32_t oy, int32_t q) {
  const int2 org = make_int2(ox, oy);
  if (q <= 0) q = p;
  const Extent E(p, q);   // p columns of L, q rows
  Plan1 P = choose(n, p, true, q);
  if (P.strategy == HP_STRATEGY_SPARSE)   // the callers have checked the arguments
    return run_sparse(pts, n, E, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info,
                      static_cast<char *>(ws), ws_bytes, s, do_hull, org);
  const TreeShape T = make_tree(p);
  if (P.strategy == HP_STRATEGY_BINNED &&
      ws_bytes < make_layout(p, p, part_pairs_for(P, n, p, q), T, bins_bytes_for(P, n, p)).total)
    P = choose(n, p, false, q);   // a workspace without room for the bins
  const bool binned = P.strategy == HP_STRATEGY_BINNED;
  const Layout Y = make_layout(p, p, part_pairs_for(P, n, p, q), T, bins_bytes_for(P, n, p));
  if (ws_bytes < Y.total) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, Y.total);
  char *w = static_cast<char *>(ws);
  int32_t *ctl = reinterpret_cast<int32_t *>(w + Y.ctl);
  int32_t *tree = reinterpret_cast<int32_t *>(w + Y.tree);
  int2 *part = reinterpret_cast<int2 *>(w + Y.part);
  int2 *Lm = reinterpret_cast<int2 *>(w + Y.Lm);
  const bool partial = partial_count(P, n, p) > 0;
  int32_t *wg_err = reinterpret_cast<int32_t *>(w + Y.wg_err);

  // The partial strategy writes every merged column itself, so only the
  // control words need clearing, which reduce workgroup 0 does; the atomic
  // strategies need the device L at the sentinel first.
  ResetArgs R;
  R.ctl = nullptr;
  R.tree_ctr = tree;
  R.nodes = T.nodes;
  R.info = info;
  hipError_t e;
  if (partial) {
    R.ctl = ctl;
  } else {
    const int ninit = (int)std::min<int64_t>(1024, std::max<int64_t>(1, ((int64_t)std::max<int64_t>(p, T.nodes) + 255) / 256));
    hipLaunchKernelGGL(k_init, dim3(ninit), dim3(256), 0, s, ctl, tree, T.nodes, info, 0, Lm, E);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_init launch: %s", hipGetErrorString(e));
  }
  // chunk sharing for the LDS and device-L strategies when every workgroup
  // has many chunks to stream: one counter serves about one grab per 10 ns,
  // which short runs would saturate
  DynArgs D;
  D.ctr = nullptr;
  D.wg_cnt = reinterpret_cast<int32_t *>(w + Y.wg_cnt);
  D.static_frac8 = dyn_static8();
  // the sampled filter: the sample is an even-length prefix (the rest keeps
  // the alignment of pts); 2^fshift columns per filter group, at least 64,
  // as few as LDS holds
  const bool sampled = P.strategy == HP_STRATEGY_SAMPLED;
  const int64_t ns = sampled ? (n / sample_div()) & ~(int64_t)1 : 0;
  int64_t n1 = 0;   // start of the pass that may share chunks
  const int nstages = sampled ? sampled_stages(ns, n, &n1) : 0;
  int fshift = 6, ngroups = 0, G1 = 0;
  if (sampled) {
    // LDS pairs left for the filter after the flag and grab words and the
    // per-wave queues of the filtered passes
    const int64_t pairs = device_info().lds_bytes / 8 - 2 - (int64_t)(P.block / kWave) * filt_queue_cap(P.vpt);
    if (pairs < 1) return set_error(HP_EINVAL, "launch shape leaves no LDS for the filter");
    while ((((int64_t)p + ((int64_t)1 << fshift) - 1) >> fshift) > pairs) ++fshift;
    ngroups = (int)(((int64_t)p + ((int64_t)1 << fshift) - 1) >> fshift);
    const int64_t per = (int64_t)P.block * P.vpt;
    G1 = (int)std::max<int64_t>(1, std::min<int64_t>(P.G, (ns / 2 + per - 1) / per));
    if (G1 + (int64_t)nstages * P.G > kMaxGrid) return set_error(HP_EINVAL, "reduce grid too large");
  }
  // the pass that may share chunks: all points, or the last filtered pass
  const int32_t *main_pts = pts ? pts + 2 * n1 : pts;
  const int64_t nchunks = dyn_chunks(n - n1, (uintptr_t)main_pts, (int64_t)P.block * P.vpt);
  if (D.static_frac8 >= 0 && P.strategy != HP_STRATEGY_WINDOW && !binned && nchunks >= kDynMinChunks * (int64_t)P.G)
    D.ctr = grab_counter();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  timing_slot(&e0, &e1);
  int n_wg_err = P.G;
  if (sampled) {
    e = dispatch_sampled(P, pts, n, E, Lm, reinterpret_cast<int2 *>(w + Y.filt), fshift, ngroups, ns, G1,
                         wg_err, D, org, s, e0, e1);
    n_wg_err = G1 + nstages * P.G;
  } else if (binned) {
    e = launch_binned(pts, n, E, part, reinterpret_cast<uint16_t *>(w + Y.filt), w + Y.bins, wg_err, R, org, s, e0,
                      e1);
    n_wg_err = bin_plan(n, p).rounds * bin_plan(n, p).G;
  } else
    e = dispatch_reduce(P, pts, n, E, Lm, part, wg_err, R, D, org, s, e0, e1);
  if (e != hipSuccess) return set_error(HP_EDEVICE, "reduce launch: %s", hipGetErrorString(e));

  FinishArgs A;
  memset(&A, 0, sizeof(A));
  A.part = partial ? part : Lm;
  A.G = partial ? partial_count(P, n, p) : 1;
  A.packed = partial && !binned && partial_packs(q) ? 1 : 0;
  A.positions = p;
  A.p = p;
  A.Lm = Lm;
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
  A.wg_err = wg_err;
  A.n_wg_err = n_wg_err;
  A.dyn_ctr = D.ctr;
  A.wg_cnt = D.wg_cnt;
  A.n_wg_cnt = P.G;
  A.dyn_expect = nchunks;
  // With the hull and more than one slab, level 2 is the all-vertex test,
  // which also writes the chain: from offsets it sums itself (up to
  // kL2MaxSlabs slabs, when it also writes the totals) or from the last
  // slab's scan.  Without the hull the last slab scans and writes the chain.
  const bool l2path = do_hull && T.nlev >= 2;
  const bool l2scan = l2path && T.size[1] > kL2MaxSlabs;
  const bool need_scan = !l2path || l2scan;
  // many slabs: the scan is a launch of its own instead of the last slab's
  const bool scan_launch = need_scan && T.size[1] > kScanRootMaxSlabs;
  A.scan_root = (need_scan && !scan_launch) ? 1 : 0;
  A.chain_inline = (!l2path && p <= kChainInline) ? 1 : 0;
  A.cx_out = cx;
  A.clo_out = clo;
  A.chi_out = chi;
  A.chain_cap = chain_cap;
  // coordinates of L are at most p: below 2^15 the hull runs on 24-bit products
  const bool small = std::max(p, q) < (1 << 15);
  HullArgs H;
  memset(&H, 0, sizeof(H));
  H.hx = hx;
  H.hy = hy;
  H.hull_cap = hull_cap;
  H.info = info;
  H.split = kSplit;
  H.slab_off = l2scan ? A.slab_off : nullptr;
  H.Lm = Lm;
  H.p = p;
  H.slab_k = A.slab_k;
  H.slab_s = A.slab_s;
  H.wg_err = wg_err;
  H.n_wg_err = n_wg_err;
  H.cx = cx;
  H.clo = clo;
  H.chi = chi;
  H.chain_cap = chain_cap;
  // more than one level-2 node: one launch finishes the columns, the chain
  // and the level-2 hulls
  if (do_hull && T.nlev >= 3 && !node_finish_off()) {
    HullArgs Hn = H;
    hull_buffers(Hn, T, p, w, Y);
    if (!node_lds_ready()) return set_error(HP_EDEVICE, "k_node_finish: %zu bytes of LDS not available", sizeof(NodeShared));
    if (small)
      hipLaunchKernelGGL((k_node_finish<kPrecSmall, false>), dim3(T.size[2]), dim3(kNodeBlock), sizeof(NodeShared), s,
                         A, Hn.buf[1], Hn.ccount);
    else
      hipLaunchKernelGGL((k_node_finish<kPrecNode, false>), dim3(T.size[2]), dim3(kNodeBlock), sizeof(NodeShared), s,
                         A, Hn.buf[1], Hn.ccount);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_node_finish launch: %s", hipGetErrorString(e));
    H.ctl = ctl;
    e = launch_hull_levels(T, p, w, Y, H, small, s, false, true);
    if (e != hipSuccess) return set_error(HP_EDEVICE, "hull level launch: %s", hipGetErrorString(e));
    return HP_OK;
  }
  // many slabs: 256-thread slab workgroups (the last-slab scan, which needs
  // 1024 threads, is then a launch of its own)
  const bool many = T.size[1] > kScanRootMaxSlabs;
  if (many && small)
    hipLaunchKernelGGL((k_finish<0, true, kFinBlockMany>), dim3(T.size[1]), dim3(kFinBlockMany), 0, s, A);
  else if (many)
    hipLaunchKernelGGL((k_finish<0, false, kFinBlockMany>), dim3(T.size[1]), dim3(kFinBlockMany), 0, s, A);
  else if (small)
    hipLaunchKernelGGL((k_finish<0, true>), dim3(T.size[1]), dim3(kFinBlock), 0, s, A);
  else
    hipLaunchKernelGGL((k_finish<0, false>), dim3(T.size[1]), dim3(kFinBlock), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_finish launch: %s", hipGetErrorString(e));
  if (scan_launch) {
    hipLaunchKernelGGL(k_slab_scan, dim3(1), dim3(kFinBlock), 0, s, A);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_slab_scan launch: %s", hipGetErrorString(e));
  }
  if (!l2path && !A.chain_inline) {
    const int nslab = T.size[1];
    hipLaunchKernelGGL(k_chain, dim3((nslab + 3) / 4), dim3(256), 0, s, Lm, p, A.slab_off, nslab, cx,
                       clo, chi, chain_cap, info);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_chain launch: %s", hipGetErrorString(e));
  }
  if (do_hull) {
    H.ctl = ctl;
    e = launch_hull_levels(T, p, w, Y, H, small, s, l2path);
    if (e != hipSuccess) return set_error(HP_EDEVICE, "hull level launch: %s", hipGetErrorString(e));
  }
  return HP_OK;
}

void tree_shape(int64_t positions, TreeShape *out) { *out = make_tree(positions); }

// Workspace of the single-cloud sequence inside batches and served requests:
// without the binned reduce's pages (their clouds fall back from it).
size_t single_ws_bytes(int64_t n, int32_t p) { return ws_bytes_for(n, p, false); }

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

extern "C" int hp_reduce_strategy(int64_t n, int32_t p, int32_t *strategy) {
  if (!strategy) return set_error(HP_EINVAL, "strategy is NULL");
  if (p < 1 || p > HP_P_MAX || n < 0) return set_error(HP_EINVAL, "bad n or p");
  *strategy = choose(n, p).strategy;
  return HP_OK;
}

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

namespace hp {

// Scratch memory of hp_run_noalloc: the hp_run workspace, held by the module
// itself for callers that cannot allocate (one copy per device the library
// runs on, kept until the process ends).  Host code never passes the name of
// the array to a kernel: that is only a host-side stand-in; the device address
// comes from hipGetSymbolAddress.
constexpr size_t kNoallocScratchBytes = HP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// This device's copy of `scratch`, looked up once per device with that device
// current (the first hp_run_noalloc call on it); null if the lookup fails.
static void *scratch_ptr() {
  static std::mutex mu;
  static void *base[64] = {};
  const int d = device_info().device;
  std::lock_guard<std::mutex> lk(mu);
  if (!base[d]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    base[d] = ptr;
  }
  return base[d];
}

}  // namespace hp

extern "C" int hp_run_noalloc(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi, uint64_t *mask,
                              int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx, int32_t *hy,
                              int32_t hull_cap, int32_t *info, void *stream) {
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  const size_t need = ws_bytes_for(n, p, false);
  if (need > kNoallocScratchBytes)
    return set_error(HP_ECAPACITY, "hp_run_noalloc: n = %lld, p = %d needs %zu bytes of scratch, the library holds %zu",
                     (long long)n, p, need, kNoallocScratchBytes);
  void *ws = scratch_ptr();
  if (!ws) return set_error(HP_EDEVICE, "hp_run_noalloc: no device address for the scratch array");
  return hp_run(pts, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, ws, kNoallocScratchBytes,
                stream);
}

extern "C" int hp_hull_workspace_bytes(int32_t chain_cap, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (chain_cap < 0 || chain_cap > HP_P_MAX) return set_error(HP_EINVAL, "chain_cap outside [0, %d]", HP_P_MAX);
  const TreeShape T = make_tree(chain_cap);
  *bytes = make_layout(chain_cap, 0, 0, T).total;
  return HP_OK;
}

namespace hp {

// Step 4 on a chain of `positions` entries whose length is read on the
// device: the slab finish from the chain, then the hull levels.
static int hull_of_chain(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t positions,
                         int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, char *w, const Layout &Y,
                         const TreeShape &T, hipStream_t s, bool small) {
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
  A.positions = positions;
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
  if (T.nlev >= 3 && !node_finish_off()) {
    // more than one level-2 node: the node finish on the chain's entries
    HullArgs Hn;
    memset(&Hn, 0, sizeof(Hn));
    hull_buffers(Hn, T, positions, w, Y);
    if (!node_lds_ready()) return set_error(HP_EDEVICE, "k_node_finish: %zu bytes of LDS not available", sizeof(NodeShared));
    if (small)
      hipLaunchKernelGGL((k_node_finish<kPrecSmall, true>), dim3(T.size[2]), dim3(kNodeBlock), sizeof(NodeShared), s,
                         A, Hn.buf[1], Hn.ccount);
    else
      hipLaunchKernelGGL((k_node_finish<kPrecWide, true>), dim3(T.size[2]), dim3(kNodeBlock), sizeof(NodeShared), s,
                         A, Hn.buf[1], Hn.ccount);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_node_finish launch: %s", hipGetErrorString(e));
    HullArgs H;
    memset(&H, 0, sizeof(H));
    H.hx = hx;
    H.hy = hy;
    H.hull_cap = hull_cap;
    H.info = info;
    e = launch_hull_levels(T, positions, w, Y, H, small, s, false, true);
    if (e != hipSuccess) return set_error(HP_EDEVICE, "hull level launch: %s", hipGetErrorString(e));
    return HP_OK;
  }
  // many slabs: 256-thread slab workgroups, so the grid stays below 2^32
  // work-items up to positions = HP_P_MAX
  if (T.size[1] > kScanRootMaxSlabs)
    hipLaunchKernelGGL((k_finish<1, false, kFinBlockMany>), dim3(T.size[1]), dim3(kFinBlockMany), 0, s, A);
  else
    hipLaunchKernelGGL((k_finish<1, false>), dim3(T.size[1]), dim3(kFinBlock), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_finish launch: %s", hipGetErrorString(e));
  HullArgs H;
  memset(&H, 0, sizeof(H));
  H.hx = hx;
  H.hy = hy;
  H.hull_cap = hull_cap;
  H.info = info;
  e = launch_hull_levels(T, positions, w, Y, H, false, s);
  if (e != hipSuccess) return set_error(HP_EDEVICE, "hull level launch: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp

extern "C" int hp_hull(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t chain_cap,
                       int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                       size_t ws_bytes, void *stream) {
  if (chain_cap < 0 || chain_cap > HP_P_MAX) return set_error(HP_EINVAL, "chain_cap outside [0, %d]", HP_P_MAX);
  if (chain_cap > 0 && (!cx || !clo || !chi)) return set_error(HP_EINVAL, "chain arrays must not be NULL");
  if (!hx || !hy || !info || !ws) return set_error(HP_EINVAL, "NULL output, info or workspace");
  if ((int64_t)hull_cap < 2 * (int64_t)chain_cap)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 chain_cap", hull_cap);
  const TreeShape T = make_tree(chain_cap);
  const Layout Y = make_layout(chain_cap, 0, 0, T);
  if (ws_bytes < Y.total) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, Y.total);
  // a chain from the caller may hold any int32 coordinates
  return hull_of_chain(cx, clo, chi, chain_cap, hx, hy, hull_cap, info, static_cast<char *>(ws), Y, T,
                       (hipStream_t)stream, false);
}

extern "C" int hp_bbox_workspace_bytes(size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  *bytes = sizeof(int4) * (size_t)kBoxMaxGrid;
  return HP_OK;
}

extern "C" int hp_bbox(const int32_t *pts, int64_t n, int32_t *box, void *ws, size_t ws_bytes, void *stream) {
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (n > 0 && !pts) return set_error(HP_EINVAL, "pts is NULL");
  if (pts && ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is not 8-byte aligned");
  if (!box) return set_error(HP_EINVAL, "box is NULL");
  if (!ws || ws_bytes < sizeof(int4) * (size_t)kBoxMaxGrid)
    return set_error(HP_ECAPACITY, "bounding-box workspace too small");
  const int64_t nv = (n + 1) / 2;
  const int64_t want = (nv + 4 * kBoxBlock - 1) / (4 * kBoxBlock);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kBoxMaxGrid, 4 * device_info().cus), want));
  hipStream_t s = (hipStream_t)stream;
  int4 *part = static_cast<int4 *>(ws);
  hipLaunchKernelGGL(k_bbox, dim3(grid), dim3(kBoxBlock), 0, s, pts, n, part);
  hipLaunchKernelGGL(k_bbox_fold, dim3(1), dim3(kBoxBlock), 0, s, (const int4 *)part, grid, box);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bbox launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_run_origin(const int32_t *pts, int64_t n, int32_t p, int32_t ox, int32_t oy, int32_t *lo,
                             int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                             int32_t chain_cap, int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info,
                             void *ws, size_t ws_bytes, void *stream) {
  const int rc = check_common(pts, n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc != HP_OK) return rc;
  if (!hx || !hy) return set_error(HP_EINVAL, "hull arrays must not be NULL");
  const int64_t need = 2 * std::min<int64_t>(n, p);
  if ((int64_t)hull_cap < need)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 min(n, p) = %lld", hull_cap, (long long)need);
  return run_single(pts, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, ws, ws_bytes,
                    (hipStream_t)stream, true, ox, oy);
}

extern "C" int hp_workspace_bytes_rect(int64_t n, int32_t p, int32_t q, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (p < 1 || p > HP_P_MAX || q < 1 || q > HP_P_MAX || n < 0) return set_error(HP_EINVAL, "bad n, p or q");
  *bytes = ws_bytes_for(n, p, true, q);
  return HP_OK;
}

extern "C" int hp_run_rect(const int32_t *pts, int64_t n, int32_t p, int32_t q, int32_t ox, int32_t oy,
                           int32_t *lo, int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                           int32_t chain_cap, int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                           size_t ws_bytes, void *stream) {
  if (q < 1 || q > HP_P_MAX) return set_error(HP_EINVAL, "q = %d outside [1, %d]", q, HP_P_MAX);
  const int rc = check_common(pts, n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc != HP_OK) return rc;
  if (!hx || !hy) return set_error(HP_EINVAL, "hull arrays must not be NULL");
  const int64_t need = 2 * std::min<int64_t>(n, p);
  if ((int64_t)hull_cap < need)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 min(n, p) = %lld", hull_cap, (long long)need);
  const size_t want = ws_bytes_for(n, p, true, q);
  if (ws_bytes < want && ws_bytes < ws_bytes_for(n, p, false, q))
    return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, want);
  return run_single(pts, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, ws, ws_bytes,
                    (hipStream_t)stream, true, ox, oy, q);
}

extern "C" int hp_bbox_f32(const float *pts, int64_t n, float *box, void *ws, size_t ws_bytes, void *stream) {
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (n > 0 && !pts) return set_error(HP_EINVAL, "pts is NULL");
  if (pts && ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is not 8-byte aligned");
  if (!box) return set_error(HP_EINVAL, "box is NULL");
  if (!ws || ws_bytes < sizeof(float4) * (size_t)kBoxMaxGrid)
    return set_error(HP_ECAPACITY, "bounding-box workspace too small");
  const int64_t want = ((n + 1) / 2 + 4 * kBoxBlock - 1) / (4 * kBoxBlock);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kBoxMaxGrid, 4 * device_info().cus), want));
  hipStream_t s = (hipStream_t)stream;
  float4 *part = static_cast<float4 *>(ws);
  hipLaunchKernelGGL(k_bbox_f32, dim3(grid), dim3(kBoxBlock), 0, s, reinterpret_cast<const float2 *>(pts), n, part);
  hipLaunchKernelGGL(k_bbox_fold_f32, dim3(1), dim3(kBoxBlock), 0, s, (const float4 *)part, grid, box);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bbox_f32 launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_quantize_f32(const float *pts, int64_t n, double ox, double oy, double scale, int32_t *out,
                               int32_t *info, void *stream) {
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (n > 0 && (!pts || !out)) return set_error(HP_EINVAL, "pts or out is NULL");
  if ((pts && ((uintptr_t)pts & 7)) || (out && ((uintptr_t)out & 7)))
    return set_error(HP_EINVAL, "pts or out is not 8-byte aligned");
  if (!info) return set_error(HP_EINVAL, "info is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_quantize_init, dim3(1), dim3(1), 0, s, info);
  if (n > 0) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8 * device_info().cus, (n + 255) / 256));
    hipLaunchKernelGGL(k_quantize_f32, dim3(grid), dim3(256), 0, s, reinterpret_cast<const float2 *>(pts), n, ox, oy,
                       scale, reinterpret_cast<int2 *>(out), info);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_quantize_f32 launch: %s", hipGetErrorString(e));
  return HP_OK;
}

// ---------------------------------------------------------------------------
// Steps 1-3 in one call: the box on the device, then the side, the origin
// (or the scale) and the sweep axis on the host after one synchronisation,
// then the path
// ---------------------------------------------------------------------------
__global__ void k_merge_status(const int32_t *__restrict__ from, int32_t *__restrict__ info) {
  if (threadIdx.x == 0 && from[0] != HP_OK) atomicMin(&info[HP_INFO_STATUS], from[0]);
}

namespace hp {

// Path workspace for every side up to p_cap.  The sizes grow with p
// between the points where a strategy's buffers drop out or change shape
// (the LDS and window limits, packed partials, the two binned rounds, every
// window count of the binned reduce), so the largest is at one of those
// points or at p_cap itself.
static size_t ws_bytes_any_q(int64_t n, int32_t c) {
  // for any number of rows: packed partials and bins (q = c), unpacked
  // partials with bins (q = 65535), neither (q = HP_P_MAX)
  return std::max({ws_bytes_for(n, c, true, c), ws_bytes_for(n, c, true, 65535), ws_bytes_for(n, c, true, HP_P_MAX)});
}

static size_t ws_bytes_upto(int64_t n, int32_t p_cap) {
  size_t m = ws_bytes_any_q(n, p_cap);
  const auto at = [&](int64_t q) {
    if (q >= 1 && q < p_cap) m = std::max(m, ws_bytes_any_q(n, (int32_t)q));
  };
  const int64_t lm = device_info().lds_max_p;
  at(lm);
  at((int64_t)kWinMax * lm);
  at(65534);
  at(n / kBinRoundsMinPerCol);
  for (int64_t q = kBinWc; q <= kBinPMax; q += kBinWc) at(q);
  return m;
}

struct AutoLayout {
  size_t parts, box, status, pts, path;
};

// Box partials, the box, a status word, a copy of the points (transposed or
// scaled; 8n bytes when `copy`), then the path's workspace.
static AutoLayout auto_layout(int64_t n, bool copy) {
  AutoLayout A;
  size_t o = 0;
  A.parts = o;  o = align_up(o + sizeof(int4) * (size_t)kBoxMaxGrid);
  A.box = o;    o = align_up(o + sizeof(int4));
  A.status = o; o = align_up(o + sizeof(int32_t));
  A.pts = o;    o = align_up(o + (copy ? (size_t)8 * (size_t)n : 0));
  A.path = o;
  return A;
}

static int check_hull_out(int64_t n, int32_t p, const int32_t *hx, const int32_t *hy, int32_t hull_cap) {
  if (!hx || !hy) return set_error(HP_EINVAL, "hull arrays must not be NULL");
  const int64_t need = 2 * std::min<int64_t>(n, p);
  if ((int64_t)hull_cap < need)
    return set_error(HP_ECAPACITY, "hull_cap %d < 2 min(n, p) = %lld", hull_cap, (long long)need);
  return HP_OK;
}

}  // namespace hp

extern "C" int hp_run_auto_workspace_bytes(int64_t n, int32_t axis, int32_t p_cap, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (n < 0 || axis < 0 || axis > 2 || p_cap < 0 || p_cap > HP_P_MAX)
    return set_error(HP_EINVAL, "bad n, axis or p_cap");
  *bytes = auto_layout(n, axis != 0 && p_cap > 0).path + (p_cap > 0 ? ws_bytes_upto(n, p_cap) : 0);
  return HP_OK;
}

extern "C" int hp_run_auto(const int32_t *pts, int64_t n, int32_t axis, int32_t p_cap, int64_t *plan,
                           int32_t *lo, int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                           int32_t chain_cap, int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                           size_t ws_bytes, void *stream) {
  if (n < 1) return set_error(HP_EINVAL, "n = %lld: the box of no points is undefined", (long long)n);
  if (!pts || ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is NULL or not 8-byte aligned");
  if (axis < 0 || axis > 2) return set_error(HP_EINVAL, "axis %d is not 0 (x), 1 (y) or 2 (shorter side)", axis);
  if (p_cap < 0 || p_cap > HP_P_MAX) return set_error(HP_EINVAL, "p_cap = %d outside [0, %d]", p_cap, HP_P_MAX);
  if (!plan || !ws) return set_error(HP_EINVAL, "plan or workspace is NULL");
  const AutoLayout A = auto_layout(n, axis != 0 && p_cap > 0);
  if (ws_bytes < A.path) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, A.path);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  // Step 1 on the device
  const int64_t want = ((n + 1) / 2 + 4 * kBoxBlock - 1) / (4 * kBoxBlock);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kBoxMaxGrid, 4 * device_info().cus), want));
  int4 *parts = reinterpret_cast<int4 *>(w + A.parts);
  int32_t *dbox = reinterpret_cast<int32_t *>(w + A.box);
  hipLaunchKernelGGL(k_bbox, dim3(grid), dim3(kBoxBlock), 0, s, pts, n, parts);
  hipLaunchKernelGGL(k_bbox_fold, dim3(1), dim3(kBoxBlock), 0, s, (const int4 *)parts, grid, dbox);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bbox launch: %s", hipGetErrorString(e));
  int32_t box[4];
  e = hipMemcpyAsync(box, dbox, sizeof(box), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(HP_EDEVICE, "reading the box: %s", hipGetErrorString(e));
  // Step 2 and the sweep axis: the p x q box that holds every point (p
  // columns along the sweep, q rows across it), the origin that moves the
  // smallest x and y to 1, and the axis of the shorter side (exchanging x
  // and y when the sweep runs along y), so that L has min(p, q) entries
  const int64_t ex = (int64_t)box[1] - box[0], ey = (int64_t)box[3] - box[2];
  const bool swap = axis == 1 || (axis == 2 && ey < ex);
  const int64_t bx0 = swap ? box[2] : box[0], bx1 = swap ? box[3] : box[1];
  const int64_t by0 = swap ? box[0] : box[2], by1 = swap ? box[1] : box[3];
  const int64_t cols = bx1 - bx0 + 1, rows = by1 - by0 + 1;
  plan[0] = bx0;
  plan[1] = bx1;
  plan[2] = by0;
  plan[3] = by1;
  plan[4] = cols;
  plan[5] = rows;
  plan[6] = bx0 - 1;
  plan[7] = by0 - 1;
  plan[8] = swap ? 1 : 0;
  if (cols > HP_P_MAX || rows > HP_P_MAX)
    return set_error(HP_EINVAL, "extent %lld x %lld exceeds HP_P_MAX", (long long)cols, (long long)rows);
  if (p_cap == 0) return HP_OK;   // the plan alone
  const int32_t p = (int32_t)cols, q = (int32_t)rows;
  if (p > p_cap) return set_error(HP_ECAPACITY, "p = %d columns > p_cap %d", p, p_cap);
  int rc = check_common(pts, n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc == HP_OK) rc = check_hull_out(n, p, hx, hy, hull_cap);
  if (rc != HP_OK) return rc;
  const size_t need = A.path + ws_bytes_for(n, p, true, q);
  if (ws_bytes < need) return set_error(HP_ECAPACITY, "workspace too small for p = %d: %zu < %zu bytes", p, ws_bytes, need);
  const int32_t *src = pts;
  if (swap) {
    int32_t *t = reinterpret_cast<int32_t *>(w + A.pts);
    rc = hp_transpose_points(pts, n, t, stream);
    if (rc != HP_OK) return rc;
    src = t;
  }
  // the origin is read modulo 2^32 by the reduce
  const int32_t ox = (int32_t)(uint32_t)(uint64_t)(bx0 - 1), oy = (int32_t)(uint32_t)(uint64_t)(by0 - 1);
  return run_single(src, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, w + A.path,
                    ws_bytes - A.path, s, true, ox, oy, q);
}

extern "C" int hp_run_auto_f32_workspace_bytes(int64_t n, int32_t p, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (n < 0 || p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "bad n or p");
  *bytes = auto_layout(n, true).path + ws_bytes_for(n, p);
  return HP_OK;
}

extern "C" int hp_run_auto_f32(const float *pts, int64_t n, int32_t p, double *plan, int32_t *qpts, int32_t *lo,
                               int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                               int32_t chain_cap, int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws,
                               size_t ws_bytes, void *stream) {
  if (n < 1) return set_error(HP_EINVAL, "n = %lld: the box of no points is undefined", (long long)n);
  if (!pts || ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is NULL or not 8-byte aligned");
  if (qpts && ((uintptr_t)qpts & 7)) return set_error(HP_EINVAL, "qpts is not 8-byte aligned");
  if (p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, HP_P_MAX);
  if (!plan || !ws) return set_error(HP_EINVAL, "plan or workspace is NULL");
  int rc = check_common(reinterpret_cast<const int32_t *>(pts), n, p, lo, hi, cx, clo, chi, chain_cap, info, ws);
  if (rc == HP_OK) rc = check_hull_out(n, p, hx, hy, hull_cap);
  if (rc != HP_OK) return rc;
  const AutoLayout A = auto_layout(n, true);
  const size_t need = A.path + ws_bytes_for(n, p);
  if (ws_bytes < need) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  const int64_t want = ((n + 1) / 2 + 4 * kBoxBlock - 1) / (4 * kBoxBlock);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kBoxMaxGrid, 4 * device_info().cus), want));
  float4 *parts = reinterpret_cast<float4 *>(w + A.parts);
  float *dbox = reinterpret_cast<float *>(w + A.box);
  hipLaunchKernelGGL(k_bbox_f32, dim3(grid), dim3(kBoxBlock), 0, s, reinterpret_cast<const float2 *>(pts), n, parts);
  hipLaunchKernelGGL(k_bbox_fold_f32, dim3(1), dim3(kBoxBlock), 0, s, (const float4 *)parts, grid, dbox);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_bbox_f32 launch: %s", hipGetErrorString(e));
  float box[4];
  e = hipMemcpyAsync(box, dbox, sizeof(box), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(HP_EDEVICE, "reading the box: %s", hipGetErrorString(e));
  // the scaling of floating-point input: origin (xmin, ymin) and scale
  // (p - 1) / (largest extent), in double precision (1 for a zero extent)
  for (int i = 0; i < 4; ++i) plan[i] = (double)box[i];
  if (!(box[0] <= box[1]) || !(box[2] <= box[3]) || !std::isfinite(box[0]) || !std::isfinite(box[1]) ||
      !std::isfinite(box[2]) || !std::isfinite(box[3]))
    return set_error(HP_EINVAL, "no finite points");
  const double ext = std::max((double)box[1] - (double)box[0], (double)box[3] - (double)box[2]);
  const double scale = ext > 0 ? (double)(p - 1) / ext : 1.0;
  plan[4] = scale;
  plan[5] = (double)box[0];
  plan[6] = (double)box[2];
  int32_t *q = qpts ? qpts : reinterpret_cast<int32_t *>(w + A.pts);
  int32_t *qstat = reinterpret_cast<int32_t *>(w + A.status);
  rc = hp_quantize_f32(pts, n, plan[5], plan[6], scale, q, qstat, stream);
  if (rc != HP_OK) return rc;
  rc = run_single(q, n, p, lo, hi, mask, cx, clo, chi, chain_cap, hx, hy, hull_cap, info, w + A.path,
                  ws_bytes - A.path, s, true);
  if (rc != HP_OK) return rc;
  // a coordinate that could not be scaled is reported in the path's status
  hipLaunchKernelGGL(k_merge_status, dim3(1), dim3(64), 0, s, (const int32_t *)qstat, info);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_merge_status launch: %s", hipGetErrorString(e));
  return HP_OK;
}

extern "C" int hp_rescan_y_workspace_bytes(int32_t k, int32_t p, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (k < 0 || p < 1 || p > HP_P_MAX) return set_error(HP_EINVAL, "bad k or p");
  *bytes = align_up(sizeof(int2) * 2 * (size_t)k) + ws_bytes_for(2 * (int64_t)k, p);
  return HP_OK;
}

extern "C" int hp_rescan_y(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t k, int32_t p,
                           int32_t *lo, int32_t *hi, uint64_t *mask, int32_t *ry, int32_t *rlo, int32_t *rhi,
                           int32_t chain_cap, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  if (k < 0) return set_error(HP_EINVAL, "k < 0");
  if (k > 0 && (!cx || !clo || !chi)) return set_error(HP_EINVAL, "chain arrays must not be NULL");
  if (!ws) return set_error(HP_EINVAL, "workspace is NULL");
  size_t need = 0;
  const int rq = hp_rescan_y_workspace_bytes(k, p, &need);
  if (rq != HP_OK) return rq;
  if (ws_bytes < need) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  int2 *rows = static_cast<int2 *>(ws);
  const size_t head = align_up(sizeof(int2) * 2 * (size_t)k);
  void *ws2 = static_cast<char *>(ws) + head;
  const int64_t n2 = 2 * (int64_t)k;
  const int rc = check_common(reinterpret_cast<const int32_t *>(rows), n2, p, lo, hi, ry, rlo, rhi, chain_cap, info,
                              ws2);
  if (rc != HP_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (k > 0) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4 * device_info().cus, (k + 255) / 256));
    hipLaunchKernelGGL(k_chain_transpose, dim3(grid), dim3(256), 0, s, cx, clo, chi, k, rows);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HP_EDEVICE, "k_chain_transpose launch: %s", hipGetErrorString(e));
  }
  return run_single(reinterpret_cast<const int32_t *>(rows), n2, p, lo, hi, mask, ry, rlo, rhi, chain_cap, nullptr,
                    nullptr, 0, info, ws2, ws_bytes - head, s, false);
}

extern "C" int hp_transpose_points(const int32_t *pts, int64_t n, int32_t *out, void *stream) {
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (n == 0) return HP_OK;
  if (!pts || !out) return set_error(HP_EINVAL, "pts or out is NULL");
  if (((uintptr_t)pts & 7) || ((uintptr_t)out & 7)) return set_error(HP_EINVAL, "pts or out is not 8-byte aligned");
  const uintptr_t a = (uintptr_t)pts, b = (uintptr_t)out, bytes = (uintptr_t)(8 * n);
  if (a < b + bytes && b < a + bytes) return set_error(HP_EINVAL, "pts and out overlap");
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8 * device_info().cus, ((n + 1) / 2 + 255) / 256));
  hipLaunchKernelGGL(k_points_transpose, dim3(grid), dim3(256), 0, (hipStream_t)stream, pts, n, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HP_EDEVICE, "k_points_transpose launch: %s", hipGetErrorString(e));
  return HP_OK;
}

