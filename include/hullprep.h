/*
 * hullprep.h -- C ABI of libhullprep.so, an MI355X (gfx950) implementation of
 * the sort-free convex-hull preconditioner of Cadenas & Megson, "An Empirical
 * Evaluation of Preconditioning Data for Accelerating Convex Hull
 * Computations" (arXiv 1505.00914), followed by an exact hull of the reduced
 * chain.
 *
 * The path, per point cloud:
 *   1. L init    -- every column of L starts as the empty sentinel (p+1, -1)
 *                   (Algorithm 1, initialisation of L);
 *   2. reduce    -- each point (x, y) lowers L[x].lo to y and raises L[x].hi
 *                   to y (Algorithm 1, the loop over P);
 *   3. compact   -- the columns that are not the sentinel, in ascending x,
 *                   become the chain (Lemma 1 and the "Building a polyline"
 *                   paragraph; extraction order of Table I);
 *   4. hull      -- the convex hull of the chain's points, listed CCW from the
 *                   lexicographic minimum, strictly convex vertices only (the
 *                   Appendix: collinear points are not hull vertices).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Points are interleaved int32 pairs (x, y) in DEVICE memory, 1 <= x, y <= p
 *   (the square of side p of the "Proposed heuristic" section).  Points
 *   outside that square are skipped and reported through the device status
 *   word (HP_ERANGE); the other outputs of that cloud are then unspecified.
 * - 1 <= p <= HP_P_MAX.  The paper only needs p + 1 to fit the coordinate
 *   type; the library's bound is lower because the compaction launches one
 *   256-thread workgroup per 64 columns and one dispatch holds fewer than
 *   2^32 work-items (ceil(HP_P_MAX / 64) * 256 = 2^32 - 256), which also
 *   keeps every count (k <= p, s <= 2p) inside int32.  n >= 0 is a 64-bit
 *   count.
 * - L is two int32 arrays lo[p], hi[p]; column x lives at index x-1.
 * - The bit array M uses 64-bit words: column i is bit (i-1)&63 of word
 *   (i-1)>>6 (Discussion, "Extraction using an array of bits", w = 64).
 * - A chain is three int32 arrays x[], lo[], hi[] over the valid columns in
 *   ascending x.  Its reduced point sequence is, per column, (x, lo) then
 *   (x, hi) when hi > lo (Lemma 1).
 * - A hull is two int32 arrays hx[], hy[]: counter-clockwise, starting at the
 *   lexicographically smallest vertex, no repeated closing vertex, collinear
 *   boundary points dropped.  0, 1 or 2 vertices for degenerate inputs.
 * - "info" is a DEVICE int32[4] per cloud: [HP_INFO_STATUS] = HP_OK or a
 *   negative data error, [HP_INFO_K] = valid columns k, [HP_INFO_S] = reduced
 *   points s, [HP_INFO_H] = hull vertices h.  It is written asynchronously;
 *   read it after synchronising the stream.
 * - Every data buffer is caller-owned device memory.  The library allocates
 *   nothing during hp_precondition / hp_hull / hp_run / hp_batched_run; the
 *   caller passes a workspace of at least the size the matching *_bytes /
 *   plan query returns.  The workspace needs no initialisation and must not
 *   be shared by calls that may overlap.
 * - All calls are asynchronous on `stream` (a hipStream_t, or NULL for the
 *   null stream).  A return value < 0 is a synchronous argument or launch
 *   error and nothing was enqueued; hp_last_error() then describes it (per
 *   thread).  Data errors never abort: they land in info[HP_INFO_STATUS].
 * - Calls on different streams with different workspaces may run
 *   concurrently.
 */
#ifndef HULLPREP_H
#define HULLPREP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HP_ABI_VERSION 1

#define HP_OK         0
#define HP_EINVAL    (-1)  /* bad argument: NULL pointer, p or n out of range  */
#define HP_ERANGE    (-2)  /* (device status) a coordinate outside [1, p]       */
#define HP_ECAPACITY (-3)  /* an output or workspace is smaller than required   */
#define HP_EDEVICE   (-4)  /* a HIP call failed                                  */
#define HP_ENOMEM    (-5)  /* host or device allocation failed (plans, servers)  */
#define HP_ETIMEOUT  (-6)  /* hp_server_wait: the request has not completed yet */

#define HP_P_MAX 1073741760  /* 2^30 - 64 */

#define HP_INFO_STATUS 0
#define HP_INFO_K      1
#define HP_INFO_S      2
#define HP_INFO_H      3
#define HP_INFO_WORDS  4

/* Reduction strategies for Algorithm 1 (all give identical results). */
#define HP_STRATEGY_AUTO         0  /* tuned choice per (n, p) regime             */
#define HP_STRATEGY_LDS          1  /* workgroup-private L in LDS, merged into the
                                       device L with filtered atomics            */
#define HP_STRATEGY_GLOBAL       2  /* one L in device memory, filtered atomics   */
#define HP_STRATEGY_LDS_PARTIAL  3  /* workgroup-private L in LDS, written out as
                                       partial arrays merged by the finish step  */
#define HP_STRATEGY_WINDOW       4  /* L split into column windows that fit LDS:
                                       the workgroups of one chunk of points, one
                                       per window, each fold the points of their
                                       window and write a partial array (for p
                                       above the LDS limit, up to 8 windows)     */
#define HP_STRATEGY_SAMPLED      5  /* one L in device memory: a sample of the
                                       points (a prefix, 1/8 of them) is folded
                                       first; per group of columns the sampled
                                       (max lo, min hi) then lets the passes over
                                       the rest skip every point that cannot
                                       change L, the filter being rebuilt once
                                       half-way (for large p, n >= 16 p)         */
#define HP_STRATEGY_BINNED       6  /* p <= 2^20: the points are binned by window
                                       of 4096 columns (32-bit entries written in
                                       128-byte blocks), then every window is
                                       folded in LDS into a partial array; from
                                       n >= 32 p the first quarter of the points
                                       builds a per-64-column filter that drops
                                       every later point that cannot change L.
                                       Needs the full hp_workspace_bytes(n, p)
                                       (about 4n bytes more); with less, the
                                       sampled or device-L strategy runs     */
#define HP_STRATEGY_SPARSE       7  /* n * 8 < p (the automatic choice): M and a
                                       summary bit per M word are built from
                                       the points, the occupied columns are
                                       listed through the summary and the
                                       points folded into their chain entries
                                       with device atomics; the work is in n,
                                       the occupied columns and p/64 words,
                                       and L is written only as the export   */

/* Steps 1 and 2 of the proposed heuristic (the bounding box, then the
 * translation that puts the points in [1, p]^2), on the device.
 *
 * hp_bbox: writes the bounding box of the n points to box[0..3] in device
 * memory as (xmin, xmax, ymin, ymax); for n = 0 it writes (INT32_MAX,
 * INT32_MIN, INT32_MAX, INT32_MIN).  One pass over the points (8n bytes).
 * ws is caller-owned device memory of hp_bbox_workspace_bytes() bytes.
 * Asynchronous on `stream`; errors as for hp_precondition.
 *
 * hp_run_origin: hp_run on the points translated by the origin (ox, oy):
 * every point is read as (x - ox, y - oy), computed modulo 2^32, with no
 * extra pass over the points.  All outputs (L, M, chain, hull) are those of
 * the translated points, i.e. equal to hp_run on a translated copy; add
 * (ox, oy) to map a vertex back.  With ox = xmin - 1, oy = ymin - 1 and
 * p = max(xmax - xmin, ymax - ymin) + 1 from hp_bbox every point is in
 * range; p must not exceed HP_P_MAX (the caller checks the extent). */
int hp_bbox_workspace_bytes(size_t *bytes);

/* Floating-point input (Conclusions: such data is brought to integers by a
 * suitable scaling).  Points are interleaved float32 pairs, 8-byte aligned.
 *
 * hp_bbox_f32: box[0..3] = (xmin, xmax, ymin, ymax) as float32 in device
 * memory, over the points without a NaN coordinate; (+inf, -inf, +inf, -inf)
 * when there is none.  Same workspace as hp_bbox.
 *
 * hp_quantize_f32: out (device int32 pairs, n of them) = (floor((x - ox) *
 * scale) + 1, floor((y - oy) * scale) + 1), evaluated in double precision
 * with one rounding per operation, so results are reproducible bit for bit.
 * A coordinate that is NaN or outside [1, 2^31 - 2] is written as 0 and sets
 * info[HP_INFO_STATUS] = HP_ERANGE (device int32[1] at least; HP_OK
 * otherwise).  With (ox, oy) = (xmin, ymin) from hp_bbox_f32 and scale =
 * (p - 1) / max(xmax - xmin, ymax - ymin), every point lands in [1, p]^2
 * and the output can go straight to hp_run with side p. */
/* Choice of sweep axis (Results: sweeping along the shorter side of the box
 * keeps fewer points): out (device, n int32 pairs) = the points with x and y
 * exchanged, so that the path on out sweeps along y.  One pass, 16n bytes.
 * pts and out are 8-byte aligned and must not overlap (HP_EINVAL). */
int hp_transpose_points(const int32_t *pts, int64_t n, int32_t *out, void *stream);

int hp_bbox_f32(const float *pts, int64_t n, float *box, void *ws, size_t ws_bytes, void *stream);
int hp_quantize_f32(const float *pts, int64_t n, double ox, double oy, double scale, int32_t *out,
                    int32_t *info, void *stream);
int hp_bbox(const int32_t *pts, int64_t n, int32_t *box, void *ws, size_t ws_bytes, void *stream);
int hp_run_origin(const int32_t *pts, int64_t n, int32_t p, int32_t ox, int32_t oy, int32_t *lo,
                  int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi,
                  int32_t chain_cap, int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info,
                  void *ws, size_t ws_bytes, void *stream);

/* The p x q box of Step 1 (Implementation of the proposed heuristic: Step 1
 * defines p and q; Lemma 1 works in that box): hp_run_origin with p columns
 * and q rows.  Every translated point must satisfy 1 <= x <= p and
 * 1 <= y <= q (HP_ERANGE otherwise); L has p entries and an empty column
 * holds (q + 1, -1); M, the chain and the hull are as for hp_run.  q = p is
 * hp_run_origin.  ws: hp_workspace_bytes_rect(n, p, q) bytes; 1 <= q <=
 * HP_P_MAX (HP_EINVAL otherwise). */
int hp_workspace_bytes_rect(int64_t n, int32_t p, int32_t q, size_t *bytes);
int hp_run_rect(const int32_t *pts, int64_t n, int32_t p, int32_t q, int32_t ox, int32_t oy, int32_t *lo,
                int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes,
                void *stream);

/* Steps 1 to 3 of the proposed heuristic in one call (Algorithm 1 preceded
 * by the bounding box, the p x q box of Step 1 and the translation into
 * [1, p] x [1, q]; the sweep along the shorter side of the box from
 * Results).
 *
 * hp_run_auto: the box of the n int32 points on the device, then, after one
 * synchronisation of `stream` (this call blocks until the box is known),
 * on the host: p = the extent along the sweep axis + 1 (the columns of L),
 * q = the extent across it + 1 (the rows), the origin (xmin - 1, ymin - 1)
 * and the sweep axis; then the path of hp_run_rect is enqueued on `stream`
 * and the call returns.
 *   axis   0: sweep along x (Algorithm 1 as written); 1: along y, i.e. the
 *          path runs on the points with x and y exchanged (one transposing
 *          pass into the workspace); 2: along y exactly when the y extent
 *          of the box is the smaller one, so that L has min(p, q) entries
 *   p_cap  capacity of lo, hi and mask in columns (they hold p_cap int32,
 *          p_cap int32 and ceil(p_cap / 64) uint64).  0 asks for the plan
 *          alone: nothing after the box is enqueued and the outputs other
 *          than plan may be NULL.  p > p_cap returns HP_ECAPACITY with the
 *          plan written
 *   plan   HOST int64[9]: xmin, xmax, ymin, ymax of the box, p, q, ox, oy
 *          and the axis taken (0 or 1).  With axis 1 the box and the origin
 *          are those of the exchanged points, and so are L, M, the chain and
 *          the hull
 *   other outputs as for hp_run_rect (chain_cap >= min(n, p), hull_cap >=
 *          2 min(n, p)); ws is caller-owned device memory of
 *          hp_run_auto_workspace_bytes(n, axis, p_cap) bytes (the path's
 *          workspace for every p <= p_cap and any q, plus the box and, for
 *          axis != 0, 8n bytes for the exchanged points)
 * n = 0 and an extent beyond HP_P_MAX return HP_EINVAL (the plan is written
 * in the second case).
 *
 * hp_run_auto_f32: the same for float32 points and a given side p (the
 * Conclusions' scaling of floating-point data): the float box on the
 * device, one synchronisation, then on the host the origin (xmin, ymin) and
 * scale = (p - 1) / max(xmax - xmin, ymax - ymin) in double precision (1
 * for a zero extent), then hp_quantize_f32 and hp_run with side p on the
 * scaled points.
 *   plan   HOST double[7]: the float box widened to double, scale, ox, oy
 *   qpts   DEVICE int32 pairs (n of them), 8-byte aligned: receives the
 *          scaled points; NULL keeps them in the workspace
 *   ws     hp_run_auto_f32_workspace_bytes(n, p) bytes
 * A coordinate that cannot be scaled into range sets info[HP_INFO_STATUS] =
 * HP_ERANGE once the path has completed.  No finite point returns
 * HP_EINVAL. */
int hp_run_auto_workspace_bytes(int64_t n, int32_t axis, int32_t p_cap, size_t *bytes);
int hp_run_auto(const int32_t *pts, int64_t n, int32_t axis, int32_t p_cap, int64_t *plan, int32_t *lo,
                int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes,
                void *stream);
int hp_run_auto_f32_workspace_bytes(int64_t n, int32_t p, size_t *bytes);
int hp_run_auto_f32(const float *pts, int64_t n, int32_t p, double *plan, int32_t *qpts, int32_t *lo,
                    int32_t *hi, uint64_t *mask, int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                    int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes,
                    void *stream);

/* The bit array M and its w-ary tree, w = 64 (Discussion, extraction by an
 * array of bits and by a tree structure).
 *
 * Storage is caller-owned DEVICE memory of hp_bitset_words(p, tree) uint64
 * words.  Level 0 is the array: column i (1-based) is bit (i-1) & 63 of word
 * (i-1) >> 6, the layout of the M that hp_precondition and hp_run write.
 * With tree != 0, level k+1 follows level k and holds one bit per word of
 * level k, set when that word is non-zero; the last level has one word.
 *
 * hp_bitset_clear: zero nwords words (a fill kernel, safe under graph
 * capture).  hp_bitset_insert: OR the columns cols[0..s) into zeroed (or
 * consistent) storage; with a tree the levels above are set as well.  info
 * is a DEVICE int32[2]: [HP_INFO_STATUS] = HP_OK, or HP_ERANGE when a column
 * lies outside [1, p] (such columns are skipped).  Duplicates are allowed.
 * hp_bitset_extract: the set columns, ascending, into cols[0..cap);
 * info[HP_INFO_K] = their count and info[HP_INFO_STATUS] = HP_ECAPACITY
 * when the count exceeds cap (the first cap columns are still written).
 * With a tree, a level-0 word whose level-1 bit is clear is not read.
 * Bits of level 0 beyond column p are ignored.  ws is caller-owned device
 * memory of hp_bitset_extract_workspace_bytes(p) bytes.  All of it is
 * asynchronous on `stream`; argument errors return synchronously. */
int hp_bitset_words(int32_t p, int32_t tree, int64_t *words);
int hp_bitset_clear(uint64_t *words, int64_t nwords, void *stream);
int hp_bitset_insert(const int32_t *cols, int64_t s, int32_t p, int32_t tree, uint64_t *words, int32_t *info,
                     void *stream);
int hp_bitset_extract_workspace_bytes(int32_t p, size_t *bytes);

/* hp_bitset_build: the same result as hp_bitset_insert (the columns ORed into
 * the storage, and with a tree every level above), built without device-
 * scope atomics on level 0: the columns are partitioned by window of
 * level-0 words, each window is assembled in LDS and stored once, and the
 * tree's upper levels are set from the finished words.  ws is caller-owned
 * device memory of hp_bitset_build_workspace_bytes(s, p) bytes (0 when the
 * shape is too small to partition, p < 2^18 or so: the call then performs
 * hp_bitset_insert).  info as for hp_bitset_insert. */
int hp_bitset_build_workspace_bytes(int64_t s, int32_t p, size_t *bytes);
int hp_bitset_build(const int32_t *cols, int64_t s, int32_t p, int32_t tree, uint64_t *words, int32_t *info,
                    void *ws, size_t ws_bytes, void *stream);
int hp_bitset_extract(const uint64_t *words, int32_t p, int32_t tree, int32_t *cols, int32_t cap, int32_t *info,
                      void *ws, size_t ws_bytes, void *stream);

/* Human-readable name of a status code (static string). */
const char *hp_status_string(int code);

/* Description of the last synchronous error on this host thread. */
const char *hp_last_error(void);

/* HP_ABI_VERSION of the loaded library. */
int hp_abi_version(void);

/* Largest p that the LDS strategy accepts on the current device. */
int32_t hp_lds_max_p(void);

/* Force a strategy for later calls on this process (HP_STRATEGY_*), e.g. for
 * tests; HP_STRATEGY_AUTO restores the tuned choice.  Also settable with the
 * environment variable HP_FORCE_STRATEGY=lds|global|lds_partial|window|sampled|binned|sparse.
 * Other environment variables, read once per process: HP_TUNING_FILE (a
 * tuning table to load instead of the one beside the library), HP_DYN_OFF=1
 * (no chunk sharing in the reduce), HP_DYN_STATIC8 (static share of a
 * shared-chunk reduce in eighths, 0..8, default 6) and HP_SAMPLE_DIV (the
 * sampled strategy folds the first n / HP_SAMPLE_DIV points exactly, 2..64,
 * default 8). */
int hp_set_strategy(int strategy);

/* The reduce strategy (HP_STRATEGY_*) that hp_run, hp_run_origin and
 * hp_precondition take for n points of side p, given the forced strategy and
 * the tuning table, when the workspace has hp_workspace_bytes(n, p) bytes. */
int hp_reduce_strategy(int64_t n, int32_t p, int32_t *strategy);

/* Launch-shape override for later calls in this process (used by the tuner):
 * strategy (HP_STRATEGY_*), reduce block size (256, 512 or 1024), 16-byte
 * vectors per lane per step (2, 4 or 8) and grid size; 0 leaves a field to
 * the tuning table.  hp_tune_set(0, 0, 0, 0) clears every override. */
int hp_tune_set(int32_t strategy, int32_t block, int32_t vpt, int32_t grid);

/* Load a tuning table written by the tuner: one line per regime
 * "log2n log2p strategy block vpt grid"; '#' starts a comment line.  A line
 * with a field the launch code cannot honour (strategy outside 1..6, block
 * not 256/512/1024, vpt not 2/4/8, grid outside 0..2^20) fails the load
 * with HP_EINVAL naming the line, and the table in use stays as it was. */
int hp_tune_load(const char *path);

/* Measurement hook.  While enabled, every reduce-kernel launch (the
 * n-proportional step, Algorithm 1) of hp_precondition / hp_run is bracketed
 * by a pair of HIP events recorded on the launch stream (up to 4096 pairs).
 * hp_timing_read synchronises those events, returns the number of timed
 * launches and their total / minimum / maximum duration in milliseconds, and
 * starts a new tally.  Off by default; enabling allocates the event pool. */
int hp_timing_enable(int on);
int hp_timing_read(int32_t *count, double *total_ms, double *min_ms, double *max_ms);

/* ------------------------------------------------------------------------
 * Single cloud
 * ---------------------------------------------------------------------- */

/* Workspace size (bytes) for hp_precondition and hp_run on n points with
 * side p.  Returns HP_OK and writes *bytes, or HP_EINVAL. */
int hp_workspace_bytes(int64_t n, int32_t p, size_t *bytes);

/* Steps 1-3 (L init, Algorithm 1, compaction into the Lemma 1 chain).
 *   pts        device, 2n int32, interleaved (x, y); may be NULL when n == 0
 *   lo, hi     device, p int32 each, or both NULL: receive L
 *   mask       device, ceil(p/64) uint64, or NULL: receives M
 *   cx, clo, chi  device, chain_cap int32 each: receive the chain
 *   chain_cap  must be >= min(n, p) (HP_ECAPACITY otherwise)
 *   info       device int32[4]: status, k, s (h is left as 0)
 *   ws         device workspace of ws_bytes >= hp_workspace_bytes(n, p)
 */
int hp_precondition(const int32_t *pts, int64_t n, int32_t p,
                    int32_t *lo, int32_t *hi, uint64_t *mask,
                    int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                    int32_t *info, void *ws, size_t ws_bytes, void *stream);

/* Workspace size (bytes) for hp_hull on a chain of capacity chain_cap. */
int hp_hull_workspace_bytes(int32_t chain_cap, size_t *bytes);

/* Step 4 alone: the hull of a chain produced by hp_precondition (or any
 * chain with strictly increasing x and lo <= hi).  The chain length k is
 * read on the device from info[HP_INFO_K]; info[HP_INFO_H] receives h.
 *   hx, hy     device, hull_cap int32 each; hull_cap >= 2 * chain_cap
 */
int hp_hull(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t chain_cap,
            int32_t *hx, int32_t *hy, int32_t hull_cap,
            int32_t *info, void *ws, size_t ws_bytes, void *stream);

/* Melkman's algorithm on the Lemma 1 polyline (Results, the linear hull of a
 * simple polyline): the same hull as hp_hull, in the same canonical form
 * (straight angles removed, counter-clockwise from the lexicographic
 * minimum), by one sequential pass with a deque.  A cross-check of hp_hull,
 * not a fast path: one lane runs it.  Arguments as for hp_hull (k is read
 * from info[HP_INFO_K], h written to info[HP_INFO_H]); hull_cap >=
 * max(2, 2 chain_cap).  The deque lives in LDS when chain_cap <= 5119, else
 * in ws, of hp_hull_melkman_workspace_bytes(chain_cap) bytes (ws may be
 * NULL in the LDS case).  A chain whose x is not strictly increasing or
 * with lo > hi sets info[HP_INFO_STATUS] = HP_EINVAL and h = 0. */
int hp_hull_melkman_workspace_bytes(int32_t chain_cap, size_t *bytes);
int hp_hull_melkman(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t chain_cap,
                    int32_t *hx, int32_t *hy, int32_t hull_cap, int32_t *info, void *ws, size_t ws_bytes,
                    void *stream);

/* The second sweep along y (Results: the rx -> rxy rescan): Algorithm 1 run
 * again on the reduced set of a chain with rows for columns, keeping per row
 * y the smallest and largest x, then compacted like hp_precondition.  The
 * hull of the result (read back as (x, y)) is the hull of the chain.
 *   cx, clo, chi  device chain of k columns (k: a HOST value, e.g. read from
 *                 info[HP_INFO_K] after the call that produced the chain)
 *   p             the side of the square (rows run over [1, p])
 *   lo, hi, mask  optional per-row extremes and row bit array, as in
 *                 hp_precondition (lo = smallest x, hi = largest x)
 *   ry, rlo, rhi  device, chain_cap >= min(2k, p) each: the rows in ascending y
 *   info          device int32[4]: status, rows k2, points s2 (rxy)
 *   ws            hp_rescan_y_workspace_bytes(k, p) bytes of device memory */
int hp_rescan_y_workspace_bytes(int32_t k, int32_t p, size_t *bytes);
int hp_rescan_y(const int32_t *cx, const int32_t *clo, const int32_t *chi, int32_t k, int32_t p, int32_t *lo,
                int32_t *hi, uint64_t *mask, int32_t *ry, int32_t *rlo, int32_t *rhi, int32_t chain_cap,
                int32_t *info, void *ws, size_t ws_bytes, void *stream);

/* Steps 1-4 fused: the chain and its hull in one call (the hull is built
 * from L directly, in parallel with the chain write).  Arguments as above;
 * hull_cap >= 2 * min(n, p).  Uses the hp_workspace_bytes(n, p) workspace. */
int hp_run(const int32_t *pts, int64_t n, int32_t p,
           int32_t *lo, int32_t *hi, uint64_t *mask,
           int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
           int32_t *hx, int32_t *hy, int32_t hull_cap,
           int32_t *info, void *ws, size_t ws_bytes, void *stream);

/* hp_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same outputs as hp_run, with the workspace taken from a scratch array of
 * HP_NOALLOC_SCRATCH_BYTES that the library itself holds on each device (no
 * hipMalloc, hipFree or other allocating call is made).  A call whose
 * hp_workspace_bytes(n, p) exceeds it returns HP_ECAPACITY before anything
 * is enqueued (on gfx950 every p up to about 3 million fits).  Every call
 * on one device shares that device's array and needs none of its previous
 * contents: calls that may overlap on one device (different streams or host
 * threads) race, so issue them on one stream. */
#define HP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int hp_run_noalloc(const int32_t *pts, int64_t n, int32_t p,
                   int32_t *lo, int32_t *hi, uint64_t *mask,
                   int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                   int32_t *hx, int32_t *hy, int32_t hull_cap,
                   int32_t *info, void *stream);

/* ------------------------------------------------------------------------
 * Batches of ragged clouds (one persistent launch, replayed from a HIP graph)
 * ---------------------------------------------------------------------- */

typedef struct hp_plan hp_plan;

/* Build a plan for B clouds.  offsets: HOST int64[B+1], non-decreasing, cloud
 * b owns points [offsets[b], offsets[b+1]) of the concatenated array;
 * p: HOST int32[B].  The plan copies both, picks a strategy and a work split
 * per cloud, and owns small device descriptor tables (allocated here, freed by
 * hp_plan_destroy).  Returns HP_OK and *plan, or an error. */
int hp_plan_create(const int64_t *offsets, const int32_t *p, int32_t B, hp_plan **plan);

/* Output and workspace sizes of a plan.  Cloud b's chain occupies
 * [chain_off[b], chain_off[b+1]) of the chain arrays (capacity min(n_b, p_b))
 * and its hull [hull_off[b], hull_off[b+1]) of the hull arrays (capacity
 * 2 min(n_b, p_b)).  Any pointer may be NULL; chain_off / hull_off are HOST
 * int64[B+1]. */
int hp_plan_query(const hp_plan *plan, int64_t *chain_total, int64_t *hull_total,
                  size_t *ws_bytes, int64_t *chain_off, int64_t *hull_off);

/* Run a plan: every cloud's chain, hull and info (device int32[B][4]).
 * The first call on a given (stream, buffers) captures a HIP graph of the
 * launch sequence; later calls with the same buffers replay it. */
int hp_batched_run(hp_plan *plan, const int32_t *pts,
                   int32_t *cx, int32_t *clo, int32_t *chi,
                   int32_t *hx, int32_t *hy, int32_t *info,
                   void *ws, size_t ws_bytes, void *stream);

/* Baseline of the batched form: the same outputs computed by one plain
 * hp_run-style launch sequence per cloud, cloud after cloud, on `stream`.
 * Uses the same workspace size as hp_batched_run. */
int hp_batched_run_percloud(hp_plan *plan, const int32_t *pts,
                            int32_t *cx, int32_t *clo, int32_t *chi,
                            int32_t *hx, int32_t *hy, int32_t *info,
                            void *ws, size_t ws_bytes, void *stream);

/* Free a plan (NULL is accepted).  The caller must have synchronised every
 * stream the plan ran on. */
void hp_plan_destroy(hp_plan *plan);

/* ------------------------------------------------------------------------
 * Served form: independent requests joined into batches by the library's
 * scheduler thread (continuous batching)
 * ---------------------------------------------------------------------- */

typedef struct hp_server hp_server;

/* Start a server on the current device.  device_budget_bytes is allocated
 * once, here, as the arena from which every request in flight takes one
 * block (its points when they come from host memory, its workspace, its
 * device outputs): a request is admitted, in arrival order, only when its
 * block fits.  max_batch bounds the requests joined into one launch
 * sequence.  Up to four batches are in flight, each on a stream of its own
 * that carries its points in, its kernels and its outputs back, so batches
 * (and the copies of one with the kernels of another) run concurrently; a
 * request that arrives while others are in flight starts on the next free
 * stream; a request that finds the server idle is issued by the thread
 * that submits it.  The scheduler thread polls for 2 ms after its last work
 * before it sleeps. */
int hp_server_create(size_t device_budget_bytes, int32_t max_batch, hp_server **server);

/* Device bytes of the arena block a request of n points with side p needs
 * (on_device: the points are already in device memory and are not copied). */
int hp_server_request_bytes(int64_t n, int32_t p, int32_t on_device, size_t *bytes);

/* Queue one request (one cloud, 1 <= p <= 65536).
 *   pts        n interleaved (x, y) int32: HOST memory, copied by the server
 *              (page-locked memory keeps the copy asynchronous), or DEVICE
 *              memory when on_device != 0; either way it must stay valid
 *              until the request completes
 *   cx, clo, chi  HOST int32[chain_cap] each: the chain (Lemma 1 order)
 *   hx, hy     HOST int32[2 * chain_cap] each: the hull
 *   chain_cap  >= min(n, p)
 *   info       HOST int32[HP_INFO_WORDS]: status, k, s, h
 * Outputs are written before the request completes (page-locked memory
 * keeps those copies asynchronous too).  When the six output arrays lie
 * back to back in one host buffer with c = min(n, p) entries per chain
 * array (cx at b, clo at b + c, chi at b + 2c, hx at b + 3c, hy at b + 5c,
 * info at b + 7c), they come back in a single copy; otherwise one copy
 * each.  Returns HP_OK and *ticket;
 * HP_ECAPACITY when the request alone exceeds the budget; HP_EINVAL for bad
 * arguments.  Data errors (a point outside [1, p]) go to info[0]. */
int hp_server_submit(hp_server *server, const int32_t *pts, int64_t n, int32_t p, int32_t on_device,
                     int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap,
                     int32_t *hx, int32_t *hy, int32_t *info, int64_t *ticket);

/* Wait for a request to complete (timeout_us < 0: without limit).  On
 * HP_OK the outputs are in place, *done_ns (may be NULL) holds the time the
 * server saw it complete (hp_clock_ns clock) and the ticket is retired;
 * HP_ETIMEOUT leaves it pending. */
int hp_server_wait(hp_server *server, int64_t ticket, int64_t timeout_us, int64_t *done_ns);

/* Counters: stats[0] batches issued, [1] requests completed, [2] requests
 * issued in batches, [3] peak arena bytes in use, [4] requests waiting,
 * [5] arena bytes. */
int hp_server_stats(hp_server *server, int64_t *stats);

/* Drain every queued request, stop the scheduler and free the server. */
int hp_server_destroy(hp_server *server);

/* Monotonic clock of the completion times, in nanoseconds. */
int64_t hp_clock_ns(void);

#ifdef __cplusplus
}
#endif
#endif /* HULLPREP_H */
