/*
 * oracle.h -- CPU oracle for the integer convex-hull preconditioner of
 * Cadenas & Megson, "An Empirical Evaluation of Preconditioning Data for
 * Accelerating Convex Hull Computations" (arXiv 1505.00914).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct statement of what the GPU path computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library, and the GPU
 * library never calls it.
 *
 * Everything here is exact integer arithmetic: the method never rounds.
 *
 * Conventions (readings of the paper, all written out in the design notes):
 *   - points are interleaved int32 pairs (x, y), 1 <= x, y <= p;
 *   - L is held as two int32 arrays lo[p], hi[p]; column x lives at index x-1;
 *   - an empty column holds the sentinel (p+1, -1) (Algorithm 1 initialisation);
 *   - the bit array M uses 64-bit words: column i is bit (i-1)&63 of word
 *     (i-1)>>6 (Discussion, "Extraction using an array of bits", with w = 64);
 *   - the hull is listed counter-clockwise starting at the lexicographic
 *     minimum (smallest x, then smallest y), without repeating the first
 *     vertex, keeping strictly convex vertices only (collinear points are
 *     dropped, as the Appendix argues they cannot be hull vertices).
 *
 * Pins: every function below is checked by the CPU test-suite against the
 * paper's worked example, its gap example and Table I, closed forms,
 * brute force on tiny inputs, exhaustive enumeration for p <= 3 and an
 * independent library hull (Qhull).  No function is "parity unpinned".
 */
#ifndef PAPER_1505_00914_ORACLE_H
#define PAPER_1505_00914_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK      0
#define OR_EINVAL (-1)   /* bad argument (p out of [1, 2^31-2], n < 0, NULL) */
#define OR_ERANGE (-2)   /* a coordinate lies outside [1, p]                 */
#define OR_EORDER (-3)   /* hull_chain input is not strictly x-increasing    */

/* Algorithm 1 (Proposed heuristic): lo/hi receive p entries each.  Every
 * point is checked for 1 <= x, y <= p first; on failure nothing is written
 * and OR_ERANGE is returned.  Then L starts at (p+1, -1) everywhere and the
 * points are folded in, in input order, by per-column min/max. */
int or_reduce(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi);

/* Algorithm 1 on the p x q box of Step 1: lo/hi receive p entries, points
 * must satisfy 1 <= x <= p and 1 <= y <= q, and an empty column holds
 * (q+1, -1).  or_reduce is the case q = p; or_mask_rect and or_chain_rect
 * read L with that sentinel, or_translate_rect gives the p x q box of the
 * points (p columns along x, q rows along y). */
int or_reduce_rect(const int32_t *pts, int64_t n, int32_t p, int32_t q, int32_t *lo, int32_t *hi);
int64_t or_mask_rect(const int32_t *lo, const int32_t *hi, int32_t p, int32_t q, uint64_t *M);
int32_t or_chain_rect(const int32_t *lo, const int32_t *hi, int32_t p, int32_t q,
                      int32_t *x, int32_t *clo, int32_t *chi);
int or_translate_rect(const int32_t *pts, int64_t n, const int32_t *box, int32_t *out, int32_t *p, int32_t *q);

/* Bit array M (Discussion, "Extraction using an array of bits"): word
 * (i-1)>>6, bit (i-1)&63 is set iff column i holds a valid entry.  M must
 * have ceil(p/64) words.  Returns the number of set bits. */
int64_t or_mask(const int32_t *lo, const int32_t *hi, int32_t p, uint64_t *M);

/* Table I: set-bit positions of one word by the count-trailing-zeros loop,
 * ascending.  Returns the count written to pos (at most 64). */
int32_t or_ctz_positions(uint64_t word, int32_t *pos);

/* Extraction of the valid columns from M, word by word with the Table I
 * loop, ascending.  cols receives 1-based column numbers; returns count. */
int32_t or_extract(const uint64_t *M, int32_t p, int32_t *cols);

/* Lemma 1 chain as a structure of arrays: the valid columns of L in
 * ascending x.  x, clo, chi need room for p entries.  Returns k. */
int32_t or_chain(const int32_t *lo, const int32_t *hi, int32_t p,
                 int32_t *x, int32_t *clo, int32_t *chi);

/* The reduced point sequence R walked along the Lemma 1 chain: for each
 * chain column (x, lo), then (x, hi) when hi > lo.  rx, ry need 2k entries.
 * Returns s = |R|. */
int64_t or_reduced(const int32_t *x, const int32_t *clo, const int32_t *chi,
                   int32_t k, int32_t *rx, int32_t *ry);

/* Convex hull of the chain (Andrew's monotone chain over R, which is already
 * in lexicographic order, so no sort).  vx, vy need 2k entries.  Returns the
 * vertex count h >= 0, or OR_EORDER if x is not strictly increasing. */
int32_t or_hull_chain(const int32_t *x, const int32_t *clo, const int32_t *chi,
                      int32_t k, int32_t *vx, int32_t *vy);

/* Convex hull of all n input points (Andrew's monotone chain after sorting
 * and de-duplicating a copy), the independent side of the Appendix claim
 * hull(reduced) == hull(input).  vx, vy need n entries.  Returns h, or
 * OR_EINVAL on allocation failure. */
int64_t or_hull_full(const int32_t *pts, int64_t n, int32_t *vx, int32_t *vy);

/* Step 1 (Proposed heuristic): box = (xmin, xmax, ymin, ymax) over the n >= 1
 * points.  OR_EINVAL for n < 1 or NULL arguments. */
int or_bbox(const int32_t *pts, int64_t n, int32_t *box);

/* Step 2 (Proposed heuristic): out[j] = (x - xmin + 1, y - ymin + 1) for the
 * box of step 1, and *p = max(xmax - xmin, ymax - ymin) + 1, the side of the
 * square Algorithm 1 then runs on.  OR_EINVAL if that side exceeds
 * 2^31 - 2.  out needs 2n entries. */
int or_translate(const int32_t *pts, int64_t n, const int32_t *box, int32_t *out, int32_t *p);

/* Bit array and w-ary tree (Discussion, extraction by an array of bits and
 * by a tree structure; w = 64).  or_tree_levels writes the word offset of
 * each level (level 0 = M) and the total word count at offset[levels] (offset
 * needs room for 8 entries) and returns the level count.  The inserts OR the
 * 1-based columns cols[0..s) into zeroed storage (M: ceil(p/64) words; T:
 * offset[levels] words); OR_ERANGE, with nothing written, if any column lies
 * outside [1, p].  or_tree_extract walks the tree from its top word and
 * writes the set columns in ascending order; returns their count. */
int32_t or_tree_levels(int32_t p, int64_t *offset);
int or_array_insert(int32_t p, const int32_t *cols, int64_t s, uint64_t *M);
int or_tree_insert(int32_t p, const int32_t *cols, int64_t s, uint64_t *T);
int32_t or_tree_extract(const uint64_t *T, int32_t p, int32_t *cols);

/* Melkman's algorithm on the Lemma 1 polyline (the reduced sequence walked
 * column by column), in the canonical form of or_hull_chain: straight angles
 * removed, counter-clockwise from the lexicographic minimum.  Inputs and
 * errors as for or_hull_chain; vx, vy need 2k entries. */
int32_t or_hull_melkman(const int32_t *x, const int32_t *clo, const int32_t *chi,
                        int32_t k, int32_t *vx, int32_t *vy);

/* Floating-point input (Conclusions).  or_bbox_f32: (xmin, xmax, ymin, ymax)
 * over the points, skipping any point with a NaN coordinate; OR_ERANGE when
 * none is left.  or_quantize_f32: out = (floor((x - ox) * s) + 1,
 * floor((y - oy) * s) + 1), in double precision, one rounding per operation;
 * a coordinate that is NaN or falls outside [1, 2^31 - 2] is written as 0
 * and makes the call return OR_ERANGE (the others are still written). */
int or_bbox_f32(const float *pts, int64_t n, float *box);
int or_quantize_f32(const float *pts, int64_t n, double ox, double oy, double s, int32_t *out);

#ifdef __cplusplus
}
#endif
#endif
