// hp_batched.hip -- plans and runs for batches of ragged point clouds.
//
// A plan fixes, once, everything that depends only on the cloud sizes: each
// cloud's reduce mode and chunks, its hull-tree shape, its workspace slots
// and its output offsets, plus the work tables of every launch.  A run is a
// fixed sequence of wide launches over all clouds (fill, one persistent
// reduce, slab tiles with their level-2 hulls, upper hull levels, per-cloud
// root, chain write), recorded once
// into a HIP graph and replayed; the graph is re-recorded only when the
// caller's buffers change.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "hp_host.h"
#include "hp_kernels.h"

namespace hp {

namespace {

// Points per reduce work item: at least 64 per column of the cloud, so the
// LDS init and the merge of a chunk's L stay small against its stream, and
// within [2^16, 2^20] so the persistent grid still balances.
constexpr int64_t kChunkMin = 1 << 16, kChunkMax = 1 << 20;
int64_t chunk_for(int32_t p) { return std::min(kChunkMax, std::max(kChunkMin, 64 * (int64_t)p)); }
constexpr int32_t kBatchPMax = 65536;    // largest p a batched cloud may have

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct CloudSlots {
  size_t ctl, slab_k, slab_s, slab_off, Lm, cand, keep, ccount;
};

}  // namespace

}  // namespace hp

struct hp_plan {
  int32_t B = 0;
  std::vector<int64_t> off;        // B+1
  std::vector<int32_t> p;          // B
  std::vector<hp::TreeShape> tree; // B
  std::vector<hp::CloudSlots> slot;
  std::vector<int64_t> chain_off, hull_off;  // B+1
  std::vector<uint8_t> needs_fill;
  std::vector<hp::BatchItem> items;
  int maxlev = 1;
  std::vector<int2> tiles;         // (cloud, tile of 64 slabs)
  std::vector<int4> nodes[2][hp::kMaxLevels + 1];  // [small?][level >= 3] (cloud, node, side, 0)
  std::vector<int2> chain_work;    // (cloud, slab)
  size_t ws_batched = 0, ws_single = 0;
  size_t lds_bytes = 0;
  int reduce_grid = 1;
  // device copies
  void *dmem = nullptr;
  hp::BatchItem *d_items = nullptr;
  uint8_t *d_needs_fill = nullptr;
  int32_t *d_counter = nullptr;
  hp::FinishArgs *d_fa = nullptr;
  hp::HullArgs *d_ha = nullptr;
  int2 *d_tiles = nullptr;
  int4 *d_nodes[2][hp::kMaxLevels + 1] = {};
  int2 *d_chain = nullptr;
  // graph state
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *bound[8] = {};
};

namespace hp {

namespace {

int fail_plan(hp_plan *P, int code) {
  hp_plan_destroy(P);
  return code;
}

// Fill the per-cloud argument blocks for the given buffers.
void build_args(const hp_plan *P, const int32_t *pts, int32_t *cx, int32_t *clo, int32_t *chi,
                int32_t *hx, int32_t *hy, int32_t *info, char *ws, std::vector<FinishArgs> &fa,
                std::vector<HullArgs> &ha) {
  (void)pts;
  fa.assign(P->B, FinishArgs());
  ha.assign(P->B, HullArgs());
  for (int b = 0; b < P->B; ++b) {
    const CloudSlots &S = P->slot[b];
    const int32_t p = P->p[b];
    const TreeShape &T = P->tree[b];
    FinishArgs A;
    memset(&A, 0, sizeof(A));
    int2 *Lm = reinterpret_cast<int2 *>(ws + S.Lm);
    A.part = Lm;
    A.G = 1;
    A.positions = p;
    A.p = p;
    A.Lm = Lm;
    A.slab_k = reinterpret_cast<int32_t *>(ws + S.slab_k);
    A.slab_s = reinterpret_cast<int32_t *>(ws + S.slab_s);
    A.slab_off = reinterpret_cast<int32_t *>(ws + S.slab_off);
    A.do_hull = 1;
    A.cand = reinterpret_cast<int2 *>(ws + S.cand);
    A.ccount = reinterpret_cast<int32_t *>(ws + S.ccount);
    A.tree = T;
    A.hx = hx + P->hull_off[b];
    A.hy = hy + P->hull_off[b];
    A.hull_cap = (int32_t)(P->hull_off[b + 1] - P->hull_off[b]);
    A.ctl = reinterpret_cast<int32_t *>(ws + S.ctl);
    A.info = info + (size_t)HP_INFO_WORDS * b;
    A.scan_root = T.nlev == 1 ? 1 : 0;
    A.chain_inline = 1;
    A.cx_out = cx + P->chain_off[b];
    A.clo_out = clo + P->chain_off[b];
    A.chi_out = chi + P->chain_off[b];
    A.chain_cap = (int32_t)(P->chain_off[b + 1] - P->chain_off[b]);
    fa[b] = A;

    HullArgs H;
    memset(&H, 0, sizeof(H));
    H.buf[0] = A.cand;
    H.buf[1] = A.cand + 2 * (size_t)p;
    H.keep = reinterpret_cast<uint8_t *>(ws + S.keep);
    H.ccount = A.ccount;
    H.tree = T;
    H.positions = p;
    H.hx = A.hx;
    H.hy = A.hy;
    H.hull_cap = A.hull_cap;
    H.info = A.info;
    H.chain_fused = T.nlev >= 2 ? 1 : 0;
    H.Lm = Lm;
    H.p = p;
    H.slab_k = A.slab_k;
    H.slab_s = A.slab_s;
    H.cx = A.cx_out;
    H.clo = A.clo_out;
    H.chi = A.chi_out;
    H.chain_cap = A.chain_cap;
    ha[b] = H;
  }
}

hipError_t enqueue_batched(const hp_plan *P, const int32_t *pts, hipStream_t s) {
  hipError_t e = launch_b_fill(P->B, P->d_fa, P->d_needs_fill, P->d_counter, s);
  if (e != hipSuccess) return e;
  if (!P->items.empty()) {
    e = launch_b_reduce(P->reduce_grid, P->lds_bytes, pts, P->d_items, (int32_t)P->items.size(),
                        P->d_counter, P->d_fa, s);
    if (e != hipSuccess) return e;
  }
  e = launch_b_tiles((int)P->tiles.size(), P->d_tiles, P->d_fa, s);
  if (e != hipSuccess) return e;
  for (int lev = 3; lev <= P->maxlev; ++lev)
    for (int sm = 0; sm < 2; ++sm) {
      e = launch_b_nodes(sm == 1, lev, (int)P->nodes[sm][lev].size(), P->d_nodes[sm][lev], P->d_ha, s);
      if (e != hipSuccess) return e;
    }
  e = launch_b_root(P->B, P->d_fa, P->d_ha, s);
  if (e != hipSuccess) return e;
  return launch_b_chain((int)P->chain_work.size(), P->d_chain, P->d_fa, s);
}

}  // namespace

}  // namespace hp

using namespace hp;

extern "C" void hp_plan_destroy(hp_plan *P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  if (P->dmem) (void)hipFree(P->dmem);
  delete P;
}

extern "C" int hp_plan_create(const int64_t *offsets, const int32_t *p, int32_t B, hp_plan **out) {
  if (!out) return set_error(HP_EINVAL, "plan pointer is NULL");
  *out = nullptr;
  if (B < 0) return set_error(HP_EINVAL, "B = %d < 0", B);
  if (B > 0 && (!offsets || !p)) return set_error(HP_EINVAL, "offsets or p is NULL");
  if (B > 0 && offsets[0] < 0) return set_error(HP_EINVAL, "offsets[0] < 0");
  for (int b = 0; b < B; ++b) {
    if (offsets[b + 1] < offsets[b]) return set_error(HP_EINVAL, "offsets decrease at cloud %d", b);
    if (p[b] < 1 || p[b] > kBatchPMax)
      return set_error(HP_EINVAL, "cloud %d: p = %d outside [1, %d]", b, p[b], kBatchPMax);
  }
  hp_plan *P = new (std::nothrow) hp_plan;
  if (!P) return set_error(HP_ENOMEM, "host allocation failed");
  P->B = B;
  P->off.assign(offsets, offsets + B + 1);
  if (B == 0) P->off.assign(1, 0);
  P->p.assign(p, p + B);
  P->tree.resize(B);
  P->slot.resize(B);
  P->chain_off.assign(B + 1, 0);
  P->hull_off.assign(B + 1, 0);
  P->needs_fill.assign(B, 1);

  const DeviceInfo &D = device_info();
  const int64_t lds_p_max = D.lds_max_p - 8;  // room for the reduce's own words
  int32_t pmax_lds = 1;
  size_t o = 0;
  size_t single_max = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = offsets[b + 1] - offsets[b];
    const int32_t pb = p[b];
    tree_shape(pb, &P->tree[b]);
    const TreeShape &T = P->tree[b];
    P->maxlev = std::max(P->maxlev, T.nlev);
    CloudSlots &S = P->slot[b];
    S.ctl = o;      o = align256(o + sizeof(int32_t) * kCtlWords);
    S.slab_k = o;   o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
    S.slab_s = o;   o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
    S.slab_off = o; o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
    S.Lm = o;       o = align256(o + sizeof(int2) * (size_t)pb);
    S.cand = o;     o = align256(o + sizeof(int2) * 4 * (size_t)pb);
    S.keep = o;     o = align256(o + 2 * (size_t)pb);
    S.ccount = o;   o = align256(o + sizeof(int32_t) * 2 * (size_t)T.nodes);
    const int64_t cap = std::min<int64_t>(n, pb);
    P->chain_off[b + 1] = P->chain_off[b] + cap;
    P->hull_off[b + 1] = P->hull_off[b] + 2 * cap;
    single_max = std::max(single_max, single_ws_bytes(n, pb));

    // reduce mode and chunks
    const bool dense = (int64_t)pb <= lds_p_max && n >= 4 * (int64_t)pb;
    if (n > 0) {
      const int64_t chunk = chunk_for(pb);
      if (dense && n <= chunk) {
        P->items.push_back(BatchItem{b, 0, offsets[b], n, 0});
        P->needs_fill[b] = 0;
      } else {
        for (int64_t s0 = 0; s0 < n; s0 += chunk)
          P->items.push_back(BatchItem{b, dense ? 1 : 2, offsets[b] + s0, std::min(chunk, n - s0), 0});
      }
      if (dense) pmax_lds = std::max(pmax_lds, pb);
    }
    // work tables
    const int sm = pb < (1 << 15) ? 1 : 0;
    for (int j = 0; j < T.size[1]; ++j) P->chain_work.push_back(make_int2(b, j));
    for (int j = 0; j * kFanIn < T.size[1]; ++j) P->tiles.push_back(make_int2(b, j));
    for (int lev = 3; lev <= T.nlev; ++lev)
      for (int q = 0; q < T.size[lev]; ++q)
        for (int side = 0; side < 2; ++side) P->nodes[sm][lev].push_back(make_int4(b, q, side, 0));
  }
  P->ws_batched = o;
  P->ws_single = single_max;
  // longest chunks first, so the persistent reduce ends evenly
  std::stable_sort(P->items.begin(), P->items.end(),
                   [](const BatchItem &a, const BatchItem &c) { return a.count > c.count; });
  P->lds_bytes = sizeof(int2) * ((size_t)pmax_lds + 1);
  const int per_cu = std::max<int>(1, std::min<int>(2, (int)((size_t)(D.lds_bytes - 64) / P->lds_bytes)));
  P->reduce_grid = D.cus * per_cu;

  // device tables: one allocation
  size_t dsz = 0;
  auto reserve = [&](size_t bytes) { size_t at = dsz; dsz = align256(dsz + std::max<size_t>(bytes, 1)); return at; };
  const size_t o_items = reserve(sizeof(BatchItem) * P->items.size());
  const size_t o_fill = reserve(P->needs_fill.size());
  const size_t o_counter = reserve(sizeof(int32_t));
  const size_t o_fa = reserve(sizeof(FinishArgs) * (size_t)std::max(1, B));
  const size_t o_ha = reserve(sizeof(HullArgs) * (size_t)std::max(1, B));
  size_t o_nodes[2][kMaxLevels + 1];
  const size_t o_chain = reserve(sizeof(int2) * P->chain_work.size());
  const size_t o_tiles = reserve(sizeof(int2) * P->tiles.size());
  for (int sm = 0; sm < 2; ++sm)
    for (int lev = 0; lev <= kMaxLevels; ++lev) o_nodes[sm][lev] = reserve(sizeof(int4) * P->nodes[sm][lev].size());
  if (hipMalloc(&P->dmem, dsz) != hipSuccess) return fail_plan(P, set_error(HP_ENOMEM, "device allocation of %zu bytes failed", dsz));
  char *dm = static_cast<char *>(P->dmem);
  P->d_items = reinterpret_cast<BatchItem *>(dm + o_items);
  P->d_needs_fill = reinterpret_cast<uint8_t *>(dm + o_fill);
  P->d_counter = reinterpret_cast<int32_t *>(dm + o_counter);
  P->d_fa = reinterpret_cast<FinishArgs *>(dm + o_fa);
  P->d_ha = reinterpret_cast<HullArgs *>(dm + o_ha);
  auto up = [&](size_t at, const void *src, size_t bytes) {
    return bytes == 0 || hipMemcpy(dm + at, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = up(o_items, P->items.data(), sizeof(BatchItem) * P->items.size()) &&
            up(o_fill, P->needs_fill.data(), P->needs_fill.size()) &&
            up(o_chain, P->chain_work.data(), sizeof(int2) * P->chain_work.size()) &&
            up(o_tiles, P->tiles.data(), sizeof(int2) * P->tiles.size());
  P->d_chain = reinterpret_cast<int2 *>(dm + o_chain);
  P->d_tiles = reinterpret_cast<int2 *>(dm + o_tiles);
  for (int sm = 0; sm < 2 && ok; ++sm)
    for (int lev = 0; lev <= kMaxLevels && ok; ++lev) {
      P->d_nodes[sm][lev] = reinterpret_cast<int4 *>(dm + o_nodes[sm][lev]);
      ok = up(o_nodes[sm][lev], P->nodes[sm][lev].data(), sizeof(int4) * P->nodes[sm][lev].size());
    }
  if (!ok) return fail_plan(P, set_error(HP_EDEVICE, "uploading plan tables failed"));
  if (prepare_b_reduce() != hipSuccess) return fail_plan(P, set_error(HP_EDEVICE, "reduce kernel setup failed"));
  if (hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess)
    return fail_plan(P, set_error(HP_EDEVICE, "stream creation failed"));
  *out = P;
  return HP_OK;
}

extern "C" int hp_plan_query(const hp_plan *P, int64_t *chain_total, int64_t *hull_total,
                             size_t *ws_bytes, int64_t *chain_off, int64_t *hull_off) {
  if (!P) return set_error(HP_EINVAL, "plan is NULL");
  if (chain_total) *chain_total = P->chain_off[P->B];
  if (hull_total) *hull_total = P->hull_off[P->B];
  if (ws_bytes) *ws_bytes = std::max(P->ws_batched, P->ws_single);
  if (chain_off) std::copy(P->chain_off.begin(), P->chain_off.end(), chain_off);
  if (hull_off) std::copy(P->hull_off.begin(), P->hull_off.end(), hull_off);
  return HP_OK;
}

static int check_run(const hp_plan *P, const int32_t *pts, int32_t *cx, int32_t *clo, int32_t *chi,
                     int32_t *hx, int32_t *hy, int32_t *info, void *ws, size_t ws_bytes, size_t need) {
  if (!P) return set_error(HP_EINVAL, "plan is NULL");
  if (P->off[P->B] > P->off[0] && !pts) return set_error(HP_EINVAL, "pts is NULL");
  if (pts && ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is not 8-byte aligned");
  if (P->B > 0 && (!cx || !clo || !chi || !hx || !hy || !info || !ws))
    return set_error(HP_EINVAL, "NULL output, info or workspace");
  if (ws_bytes < need) return set_error(HP_ECAPACITY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return HP_OK;
}

extern "C" int hp_batched_run(hp_plan *P, const int32_t *pts, int32_t *cx, int32_t *clo, int32_t *chi,
                              int32_t *hx, int32_t *hy, int32_t *info, void *ws, size_t ws_bytes,
                              void *stream) {
  const int rc = check_run(P, pts, cx, clo, chi, hx, hy, info, ws, ws_bytes, P ? P->ws_batched : 0);
  if (rc != HP_OK) return rc;
  if (P->B == 0) return HP_OK;
  hipStream_t s = (hipStream_t)stream;
  const void *now[8] = {pts, cx, clo, chi, hx, hy, info, ws};
  if (!P->exec || memcmp(now, P->bound, sizeof(now)) != 0) {
    // new buffers: rewrite the argument blocks and re-record the graph (the
    // caller's earlier runs on this plan must finish reading the old ones)
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(HP_EDEVICE, "stream synchronisation failed");
    std::vector<FinishArgs> fa;
    std::vector<HullArgs> ha;
    build_args(P, pts, cx, clo, chi, hx, hy, info, static_cast<char *>(ws), fa, ha);
    if (hipMemcpy(P->d_fa, fa.data(), sizeof(FinishArgs) * fa.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->d_ha, ha.data(), sizeof(HullArgs) * ha.size(), hipMemcpyHostToDevice) != hipSuccess)
      return set_error(HP_EDEVICE, "uploading argument blocks failed");
    if (P->exec) { (void)hipGraphExecDestroy(P->exec); P->exec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(HP_EDEVICE, "graph capture could not start");
    const hipError_t e = enqueue_batched(P, pts, P->cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(P->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return set_error(HP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    P->graph = g;
    if (hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) {
      P->exec = nullptr;
      return set_error(HP_EDEVICE, "graph instantiation failed");
    }
    memcpy(P->bound, now, sizeof(now));
  }
  if (hipGraphLaunch(P->exec, s) != hipSuccess) return set_error(HP_EDEVICE, "graph launch failed");
  return HP_OK;
}

extern "C" int hp_batched_run_percloud(hp_plan *P, const int32_t *pts, int32_t *cx, int32_t *clo,
                                       int32_t *chi, int32_t *hx, int32_t *hy, int32_t *info, void *ws,
                                       size_t ws_bytes, void *stream) {
  const int rc = check_run(P, pts, cx, clo, chi, hx, hy, info, ws, ws_bytes, P ? P->ws_single : 0);
  if (rc != HP_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int b = 0; b < P->B; ++b) {
    const int64_t n = P->off[b + 1] - P->off[b];
    const int32_t cap = (int32_t)(P->chain_off[b + 1] - P->chain_off[b]);
    const int r = run_single(pts ? pts + 2 * P->off[b] : nullptr, n, P->p[b], nullptr, nullptr, nullptr,
                             cx + P->chain_off[b], clo + P->chain_off[b], chi + P->chain_off[b], cap,
                             hx + P->hull_off[b], hy + P->hull_off[b], 2 * cap,
                             info + (size_t)HP_INFO_WORDS * b, ws, ws_bytes, s, true);
    if (r != HP_OK) return r;
  }
  return HP_OK;
}
