// hp_batched.hip -- batches of ragged point clouds: the shared work tables
// (hp_batch.h) and the recorded plan (hp_plan_*).
//
// A plan fixes, once, everything that depends only on the cloud sizes: each
// cloud's reduce mode and chunks, its hull-tree shape, its workspace slots
// and its output offsets, plus the work lists of every launch.  A run is a
// fixed sequence of wide launches over all clouds (fill, one persistent
// reduce, slab tiles with their level-2 hulls, upper node levels, per-cloud
// root, chain write), recorded once into a HIP graph and replayed; the
// graph is re-recorded only when the caller's buffers change.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "hp_batch.h"

namespace hp {

namespace {

// Points per reduce work item: at least 64 per column of the cloud, so the
// LDS init and the merge of a chunk's L stay small against its stream, and
// within [2^16, 2^20] so the persistent grid still balances.
constexpr int64_t kChunkMin = 1 << 16, kChunkMax = 1 << 20;
int64_t chunk_for(int32_t p) { return std::min(kChunkMax, std::max(kChunkMin, 64 * (int64_t)p)); }

}  // namespace

CloudSlots cloud_slots(int32_t p, const TreeShape &T) {
  CloudSlots S;
  size_t o = 0;
  S.slab_k = o;   o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
  S.slab_s = o;   o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
  S.slab_off = o; o = align256(o + sizeof(int32_t) * (size_t)T.size[1]);
  S.Lm = o;       o = align256(o + sizeof(int2) * (size_t)p);
  S.cand = o;     o = align256(o + sizeof(int2) * 4 * (size_t)p);
  S.ccount = o;   o = align256(o + sizeof(int32_t) * 2 * (size_t)T.nodes);
  S.total = o;
  return S;
}

BCloud make_bcloud(int32_t p, const TreeShape &T, char *base, const CloudSlots &S, const CloudOut &o) {
  BCloud c;
  memset(&c, 0, sizeof(c));
  c.p = p;
  c.tree = T;
  c.Lm = reinterpret_cast<int2 *>(base + S.Lm);
  c.mask = o.mask;
  c.slab_k = reinterpret_cast<int32_t *>(base + S.slab_k);
  c.slab_s = reinterpret_cast<int32_t *>(base + S.slab_s);
  c.slab_off = reinterpret_cast<int32_t *>(base + S.slab_off);
  c.cand = reinterpret_cast<int2 *>(base + S.cand);
  c.ccount = reinterpret_cast<int32_t *>(base + S.ccount);
  c.cx = o.cx;
  c.clo = o.clo;
  c.chi = o.chi;
  c.chain_cap = o.chain_cap;
  c.hx = o.hx;
  c.hy = o.hy;
  c.hull_cap = o.hull_cap;
  c.info = o.info;
  return c;
}

void BatchTables::clear() {
  B = 0;
  maxlev = 1;
  pmax_lds = 1;
  items.clear();
  needs_fill.clear();
  tiles.clear();
  chain.clear();
  for (auto &v : nodes)
    for (auto &w : v) w.clear();
}

void BatchTables::add_cloud(int64_t n, int32_t p, const TreeShape &T, int64_t lds_p_max) {
  const int32_t b = B++;
  maxlev = std::max(maxlev, T.nlev);
  // reduce: a cloud whose L fits in LDS goes through LDS when it is dense
  // (n >= 4p and the tuning table picks an LDS strategy for its (n, p)
  // regime), whole when it fits one item, else in chunks merged by atomics,
  // and also when it is sparse (n < 4p, always one item): a whole-cloud item
  // writes its L once, where folding straight into device memory would cost
  // a device-scope atomic for nearly every point.  Any other cloud folds
  // straight into its L in device memory.
  const int tuned = tuned_strategy(n, p);
  const bool lds_family = tuned == HP_STRATEGY_LDS || tuned == HP_STRATEGY_LDS_PARTIAL;
  const bool dense = (int64_t)p <= lds_p_max && (n >= 4 * (int64_t)p ? lds_family : n <= chunk_for(p));
  uint8_t fill = 1;
  if (n > 0) {
    const int64_t chunk = chunk_for(p);
    if (dense && n <= chunk) {
      items.push_back(HostItem{b, 0, 0, n});
      fill = 0;
    } else {
      for (int64_t s0 = 0; s0 < n; s0 += chunk)
        items.push_back(HostItem{b, dense ? 1 : 2, s0, std::min(chunk, n - s0)});
    }
    if (dense) pmax_lds = std::max(pmax_lds, p);
  }
  needs_fill.push_back(fill);
  const int sm = p < (1 << 15) ? 1 : 0;
  for (int j = 0; j < T.size[1]; ++j) chain.push_back(make_int2(b, j));
  for (int j = 0; j * kFanIn < T.size[1]; ++j) tiles.push_back(make_int2(b, j));
  for (int lev = 3; lev <= T.nlev; ++lev)
    for (int q = 0; q < T.size[lev]; ++q)
      for (int side = 0; side < 2; ++side) nodes[sm][lev].push_back(make_int4(b, q, side, 0));
}

size_t BatchTables::cloud_image_bound(int64_t n, int32_t p, const TreeShape &T) {
  const int64_t nitems = n / chunk_for(p) + 2;
  int64_t nnodes = 0;
  for (int lev = 3; lev <= T.nlev; ++lev) nnodes += 2 * (int64_t)T.size[lev];
  return sizeof(BCloud) + 1 + sizeof(BatchItem) * (size_t)nitems + sizeof(int2) * (size_t)T.size[1] * 2 +
         sizeof(int4) * (size_t)nnodes;
}

void BatchTables::sort_items() {
  std::stable_sort(items.begin(), items.end(),
                   [](const HostItem &a, const HostItem &c) { return a.count > c.count; });
}

namespace {

struct ImageLayout {
  size_t clouds, fill, counter, items, tiles, chain, nodes[2][kMaxLevels + 1], total;
};

ImageLayout image_layout(const BatchTables &t) {
  ImageLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + std::max<size_t>(bytes, 1)); return at; };
  L.clouds = take(sizeof(BCloud) * (size_t)t.B);
  L.fill = take(t.needs_fill.size());
  L.counter = take(sizeof(int32_t));
  L.items = take(sizeof(BatchItem) * t.items.size());
  L.tiles = take(sizeof(int2) * t.tiles.size());
  L.chain = take(sizeof(int2) * t.chain.size());
  for (int sm = 0; sm < 2; ++sm)
    for (int lev = 0; lev <= kMaxLevels; ++lev) L.nodes[sm][lev] = take(sizeof(int4) * t.nodes[sm][lev].size());
  L.total = o;
  return L;
}

}  // namespace

size_t batch_image_bytes(const BatchTables &t) { return image_layout(t).total; }

void batch_image(const BatchTables &t, const std::vector<BCloud> &clouds,
                 const std::vector<const int32_t *> &cloud_pts, char *host, char *dev, DeviceBatch &D) {
  const ImageLayout L = image_layout(t);
  memset(host, 0, L.total);
  memcpy(host + L.clouds, clouds.data(), sizeof(BCloud) * (size_t)t.B);
  memcpy(host + L.fill, t.needs_fill.data(), t.needs_fill.size());
  BatchItem *it = reinterpret_cast<BatchItem *>(host + L.items);
  for (size_t i = 0; i < t.items.size(); ++i) {
    const HostItem &h = t.items[i];
    it[i].pts = cloud_pts[h.cloud] + 2 * h.offset;
    it[i].count = h.count;
    it[i].cloud = h.cloud;
    it[i].mode = h.mode;
  }
  memcpy(host + L.tiles, t.tiles.data(), sizeof(int2) * t.tiles.size());
  memcpy(host + L.chain, t.chain.data(), sizeof(int2) * t.chain.size());
  D.B = t.B;
  D.clouds = reinterpret_cast<BCloud *>(dev + L.clouds);
  D.needs_fill = reinterpret_cast<uint8_t *>(dev + L.fill);
  D.counter = reinterpret_cast<int32_t *>(dev + L.counter);
  D.items = reinterpret_cast<BatchItem *>(dev + L.items);
  D.nitems = (int32_t)t.items.size();
  D.tiles = reinterpret_cast<int2 *>(dev + L.tiles);
  D.ntiles = (int32_t)t.tiles.size();
  D.chain = reinterpret_cast<int2 *>(dev + L.chain);
  D.nchain = (int32_t)t.chain.size();
  for (int sm = 0; sm < 2; ++sm)
    for (int lev = 0; lev <= kMaxLevels; ++lev) {
      memcpy(host + L.nodes[sm][lev], t.nodes[sm][lev].data(), sizeof(int4) * t.nodes[sm][lev].size());
      D.nodes[sm][lev] = reinterpret_cast<int4 *>(dev + L.nodes[sm][lev]);
      D.nnodes[sm][lev] = (int32_t)t.nodes[sm][lev].size();
    }
  D.maxlev = t.maxlev;
  const DeviceInfo &I = device_info();
  D.lds_bytes = sizeof(int2) * ((size_t)t.pmax_lds + 1);
  const int per_cu = std::max<int>(1, std::min<int>(2, (int)((size_t)(I.lds_bytes - 64) / D.lds_bytes)));
  D.reduce_grid = I.cus * per_cu;
}

hipError_t enqueue_batch(const DeviceBatch &D, hipStream_t s) {
  if (D.B == 0) return hipSuccess;
  hipError_t e = launch_b_fill(D.B, D.clouds, D.needs_fill, D.counter, s);
  if (e != hipSuccess) return e;
  e = launch_b_reduce(D.reduce_grid, D.lds_bytes, D.items, D.nitems, D.counter, D.clouds, s);
  if (e != hipSuccess) return e;
  e = launch_b_tiles(D.ntiles, D.tiles, D.clouds, s);
  if (e != hipSuccess) return e;
  for (int lev = 3; lev <= D.maxlev; ++lev)
    for (int sm = 0; sm < 2; ++sm) {
      e = launch_b_nodes(sm == 1, lev, D.nnodes[sm][lev], D.nodes[sm][lev], D.clouds, s);
      if (e != hipSuccess) return e;
    }
  e = launch_b_root(D.B, D.clouds, s);
  if (e != hipSuccess) return e;
  return launch_b_chain(D.nchain, D.chain, D.clouds, s);
}

}  // namespace hp

struct hp_plan {
  int32_t B = 0;
  std::vector<int64_t> off;          // B+1
  std::vector<int32_t> p;            // B
  std::vector<hp::TreeShape> tree;   // B
  std::vector<hp::CloudSlots> slot;  // B
  std::vector<size_t> slot_base;     // B: byte offset of each cloud's slots in the workspace
  std::vector<int64_t> chain_off, hull_off;  // B+1
  hp::BatchTables tables;
  size_t ws_batched = 0, ws_single = 0;
  // device image of the tables (rewritten when the buffers change)
  size_t image_bytes = 0;
  void *dimage = nullptr;
  std::vector<char> himage;
  hp::DeviceBatch dev;
  // graph state
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *bound[8] = {};
};

using namespace hp;

extern "C" void hp_plan_destroy(hp_plan *P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  if (P->dimage) (void)hipFree(P->dimage);
  delete P;
}

static int fail_plan(hp_plan *P, int code) {
  hp_plan_destroy(P);
  return code;
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
  P->slot_base.resize(B);
  P->chain_off.assign(B + 1, 0);
  P->hull_off.assign(B + 1, 0);

  const DeviceInfo &D = device_info();
  const int64_t lds_p_max = D.lds_max_p - 8;  // room for the reduce's own words
  size_t o = 0, single_max = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = offsets[b + 1] - offsets[b];
    tree_shape(p[b], &P->tree[b]);
    P->slot[b] = cloud_slots(p[b], P->tree[b]);
    P->slot_base[b] = o;
    o += P->slot[b].total;
    const int64_t cap = chain_cap_for(n, p[b]);
    P->chain_off[b + 1] = P->chain_off[b] + cap;
    P->hull_off[b + 1] = P->hull_off[b] + 2 * cap;
    single_max = std::max(single_max, single_ws_bytes(n, p[b]));
    P->tables.add_cloud(n, p[b], P->tree[b], lds_p_max);
  }
  P->tables.sort_items();
  P->ws_batched = o;
  P->ws_single = single_max;
  P->image_bytes = batch_image_bytes(P->tables);
  P->himage.resize(P->image_bytes);
  if (hipMalloc(&P->dimage, P->image_bytes) != hipSuccess)
    return fail_plan(P, set_error(HP_ENOMEM, "device allocation of %zu bytes failed", P->image_bytes));
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
    // new buffers: rewrite the device image and re-record the graph (the
    // caller's earlier runs on this plan must finish reading the old image)
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(HP_EDEVICE, "stream synchronisation failed");
    std::vector<BCloud> clouds(P->B);
    std::vector<const int32_t *> cpts(P->B);
    char *wsb = static_cast<char *>(ws);
    for (int b = 0; b < P->B; ++b) {
      CloudOut o;
      o.cx = cx + P->chain_off[b];
      o.clo = clo + P->chain_off[b];
      o.chi = chi + P->chain_off[b];
      o.chain_cap = (int32_t)(P->chain_off[b + 1] - P->chain_off[b]);
      o.hx = hx + P->hull_off[b];
      o.hy = hy + P->hull_off[b];
      o.hull_cap = (int32_t)(P->hull_off[b + 1] - P->hull_off[b]);
      o.info = info + (size_t)HP_INFO_WORDS * b;
      o.mask = nullptr;
      clouds[b] = make_bcloud(P->p[b], P->tree[b], wsb + P->slot_base[b], P->slot[b], o);
      cpts[b] = pts ? pts + 2 * P->off[b] : nullptr;
    }
    batch_image(P->tables, clouds, cpts, P->himage.data(), static_cast<char *>(P->dimage), P->dev);
    if (hipMemcpy(P->dimage, P->himage.data(), P->image_bytes, hipMemcpyHostToDevice) != hipSuccess)
      return set_error(HP_EDEVICE, "uploading the batch tables failed");
    if (P->exec) { (void)hipGraphExecDestroy(P->exec); P->exec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(HP_EDEVICE, "graph capture could not start");
    const hipError_t e = enqueue_batch(P->dev, P->cap);
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
