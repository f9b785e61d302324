// hp_output.h -- the two output writers shared by the single-cloud and the
// batched finish: the final hull from its two lower chains, and the chain
// of one slab at its scanned offset.
#pragma once

#include "hp_device.h"
#include "hullprep.h"

namespace hp {

// The final hull from the lower hull of (x, lo) and the lower hull of
// (x, -hi) (both left to right): lower chain, then the upper chain walked
// back, without the shared end points.  Returns h.
__device__ inline int assemble_hull(const int2 *low, int nl, const int2 *upn, int nu, int32_t *hx,
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

// Chain write of slabs [s0, s1) with the slab offsets already scanned: one
// wave per slab, ballot rank inside the slab (Lemma 1 order).
__device__ inline void write_chain_slab(const int2 *Lm, int32_t p, const int32_t *slab_off, int slab,
                                 int32_t *cx, int32_t *clo, int32_t *chi, int32_t cap,
                                 int32_t *info) {
  const int lane = threadIdx.x & (kWave - 1);
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

}  // namespace hp
