/*
 * oracle.c -- plain C statement of the preconditioner and hull (arXiv
 * 1505.00914).  TEST INFRASTRUCTURE ONLY: see oracle.h for who may use it.
 *
 * Written for a reader checking it against the paper by eye: no blocking,
 * no fusion, no reordering beyond what the definitions state.  Single thread.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Largest admissible p: p+1 (the empty-column sentinel) must fit in int32. */
#define OR_PMAX 2147483646

/* ---------------------------------------------------------------------------
 * Algorithm 1 (Proposed heuristic, "Reduction of Points"), on the p x q box
 * of Step 1 ("define p, q"): one (lo, hi) pair per column x in 1..p, all
 * starting at the empty value (q+1, -1), one past either end of the y range
 * 1..q.  A point only ever lowers the lo and raises the hi of its own column,
 * so after all n points a column holds the smallest and the largest y among
 * its points, or is still empty.  The square of side p is the case q = p.
 * A point outside the box is reported instead of folded in.
 * ------------------------------------------------------------------------- */
int or_reduce_rect(const int32_t *pts, int64_t n, int32_t p, int32_t q, int32_t *lo, int32_t *hi)
{
    if (p < 1 || p > OR_PMAX || q < 1 || q > OR_PMAX || n < 0) return OR_EINVAL;
    if (n > 0 && pts == NULL) return OR_EINVAL;
    if (lo == NULL || hi == NULL) return OR_EINVAL;

    for (int64_t j = 0; j < n; ++j) {
        const int32_t x = pts[2 * j], y = pts[2 * j + 1];
        if (x < 1 || x > p || y < 1 || y > q) return OR_ERANGE;
    }
    for (int32_t c = 0; c < p; ++c) {
        lo[c] = q + 1;
        hi[c] = -1;
    }
    for (int64_t j = 0; j < n; ++j) {
        const int32_t c = pts[2 * j] - 1, y = pts[2 * j + 1];
        if (y < lo[c]) lo[c] = y;
        if (y > hi[c]) hi[c] = y;
    }
    return OR_OK;
}

int or_reduce(const int32_t *pts, int64_t n, int32_t p, int32_t *lo, int32_t *hi)
{
    return or_reduce_rect(pts, n, p, p, lo, hi);
}

/* A column of L is occupied when it no longer holds the empty value
 * (q+1, -1): after Algorithm 1 it then holds 1 <= lo <= hi <= q. */
static int or_valid(int32_t lo, int32_t hi, int32_t q)
{
    return !(lo == q + 1 && hi == -1);
}

/* ---------------------------------------------------------------------------
 * Bit array M (Discussion, "Extraction using an array of bits").  M[i] = 1
 * exactly for the valid columns i; with w-bit words, column i is bit
 * (i-1) & (w-1) of word (i-1) >> log2(w).  Here w = 64.
 * ------------------------------------------------------------------------- */
int64_t or_mask_rect(const int32_t *lo, const int32_t *hi, int32_t p, int32_t q, uint64_t *M)
{
    if (p < 1 || p > OR_PMAX || q < 1 || q > OR_PMAX || lo == NULL || hi == NULL || M == NULL) return OR_EINVAL;
    const int64_t words = ((int64_t)p + 63) / 64;
    memset(M, 0, (size_t)words * sizeof(uint64_t));
    int64_t set = 0;
    for (int64_t c = 0; c < p; ++c) {
        if (!or_valid(lo[c], hi[c], q)) continue;
        M[c / 64] |= (uint64_t)1 << (c % 64);
        ++set;
    }
    return set;
}

int64_t or_mask(const int32_t *lo, const int32_t *hi, int32_t p, uint64_t *M)
{
    return or_mask_rect(lo, hi, p, p, M);
}

/* Count of trailing zero bits of a non-zero word, by plain shifting (the
 * hardware instruction the paper relies on is only a faster way to get the
 * same number). */
static int32_t or_ctz64(uint64_t x)
{
    int32_t c = 0;
    while ((x & 1u) == 0) {
        x >>= 1;
        ++c;
    }
    return c;
}

/* Table I: the set bits of a word in ascending order, by counting the
 * trailing zeros of what is left and then dropping its lowest set bit
 * (w & (w - 1) clears exactly that bit). */
int32_t or_ctz_positions(uint64_t word, int32_t *pos)
{
    int32_t c = 0;
    for (uint64_t w = word; w != 0; w &= w - 1) pos[c++] = or_ctz64(w);
    return c;
}

/* Extraction over all words of M: column i = b*w + pb + 1. */
int32_t or_extract(const uint64_t *M, int32_t p, int32_t *cols)
{
    if (p < 1 || p > OR_PMAX || M == NULL || cols == NULL) return OR_EINVAL;
    int64_t words = ((int64_t)p + 63) / 64;
    int32_t k = 0;
    int32_t pos[64];
    for (int64_t b = 0; b < words; ++b) {
        int32_t c = or_ctz_positions(M[b], pos);
        for (int32_t t = 0; t < c; ++t) cols[k++] = (int32_t)(b * 64 + pos[t] + 1);
    }
    return k;
}

/* ---------------------------------------------------------------------------
 * Lemma 1 (Building a polyline): scanning L along x and skipping the
 * entries that still hold the sentinel gives the valid columns in ascending
 * x.  The chain is stored as (x, lo, hi) per valid column.
 * ------------------------------------------------------------------------- */
int32_t or_chain_rect(const int32_t *lo, const int32_t *hi, int32_t p, int32_t q,
                      int32_t *x, int32_t *clo, int32_t *chi)
{
    if (p < 1 || p > OR_PMAX || q < 1 || q > OR_PMAX || lo == NULL || hi == NULL) return OR_EINVAL;
    int32_t k = 0;
    for (int32_t c = 0; c < p; ++c) {
        if (!or_valid(lo[c], hi[c], q)) continue;
        x[k] = c + 1;
        clo[k] = lo[c];
        chi[k] = hi[c];
        ++k;
    }
    return k;
}

int32_t or_chain(const int32_t *lo, const int32_t *hi, int32_t p,
                 int32_t *x, int32_t *clo, int32_t *chi)
{
    return or_chain_rect(lo, hi, p, p, x, clo, chi);
}

/* The points the chain joins, in the order Lemma 1 walks them: within a
 * column from (x, ly) up to (x, hy), then on to the next valid column.  A
 * column with ly = hy contributes its single point once. */
int64_t or_reduced(const int32_t *x, const int32_t *clo, const int32_t *chi,
                   int32_t k, int32_t *rx, int32_t *ry)
{
    int64_t s = 0;
    for (int32_t t = 0; t < k; ++t) {
        rx[s] = x[t];
        ry[s] = clo[t];
        ++s;
        if (chi[t] > clo[t]) {
            rx[s] = x[t];
            ry[s] = chi[t];
            ++s;
        }
    }
    return s;
}

/* ---------------------------------------------------------------------------
 * Andrew's monotone chain over a lexicographically sorted sequence of
 * distinct points.
 *
 * cross(o, a, b) = (a - o) x (b - o), evaluated in int64.  Every coordinate
 * difference is below 2^31 in magnitude, so each product is below 2^62 and
 * the difference of two products below 2^63: exact.
 *
 * lower: walk the points left to right; before pushing q, pop while the last
 *        two stacked points and q fail to make a strict left turn
 *        (cross <= 0, which also removes collinear points);
 * upper: the same walk right to left;
 * hull : lower without its last point, then upper without its last point.
 * A sequence of 0 or 1 points is its own hull.
 * ------------------------------------------------------------------------- */
static int64_t or_cross(int64_t ox, int64_t oy, int64_t ax, int64_t ay,
                        int64_t bx, int64_t by)
{
    return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);
}

static int64_t or_andrew(const int32_t *px, const int32_t *py, int64_t m,
                         int32_t *vx, int32_t *vy)
{
    if (m <= 1) {
        for (int64_t i = 0; i < m; ++i) {
            vx[i] = px[i];
            vy[i] = py[i];
        }
        return m;
    }
    /* The stack for one chain holds at most m points. */
    int32_t *sx = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    int32_t *sy = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    if (sx == NULL || sy == NULL) {
        free(sx);
        free(sy);
        return OR_EINVAL;
    }
    int64_t h = 0;

    /* lower chain */
    int64_t t = 0;
    for (int64_t i = 0; i < m; ++i) {
        while (t >= 2 && or_cross(sx[t - 2], sy[t - 2], sx[t - 1], sy[t - 1], px[i], py[i]) <= 0) --t;
        sx[t] = px[i];
        sy[t] = py[i];
        ++t;
    }
    for (int64_t i = 0; i + 1 < t; ++i) {
        vx[h] = sx[i];
        vy[h] = sy[i];
        ++h;
    }

    /* upper chain */
    t = 0;
    for (int64_t i = m - 1; i >= 0; --i) {
        while (t >= 2 && or_cross(sx[t - 2], sy[t - 2], sx[t - 1], sy[t - 1], px[i], py[i]) <= 0) --t;
        sx[t] = px[i];
        sy[t] = py[i];
        ++t;
    }
    for (int64_t i = 0; i + 1 < t; ++i) {
        vx[h] = sx[i];
        vy[h] = sy[i];
        ++h;
    }

    free(sx);
    free(sy);
    return h;
}

int32_t or_hull_chain(const int32_t *x, const int32_t *clo, const int32_t *chi,
                      int32_t k, int32_t *vx, int32_t *vy)
{
    if (k < 0) return OR_EINVAL;
    for (int32_t t = 0; t + 1 < k; ++t)
        if (!(x[t] < x[t + 1])) return OR_EORDER;
    for (int32_t t = 0; t < k; ++t)
        if (chi[t] < clo[t]) return OR_EORDER;
    if (k == 0) return 0;

    int32_t *rx = (int32_t *)malloc((size_t)2 * (size_t)k * sizeof(int32_t));
    int32_t *ry = (int32_t *)malloc((size_t)2 * (size_t)k * sizeof(int32_t));
    if (rx == NULL || ry == NULL) {
        free(rx);
        free(ry);
        return OR_EINVAL;
    }
    /* R is strictly increasing in (x, y) order: x grows from column to column
     * and lo < hi inside a column, so Andrew's scan needs no sort here. */
    int64_t s = or_reduced(x, clo, chi, k, rx, ry);
    int64_t h = or_andrew(rx, ry, s, vx, vy);
    free(rx);
    free(ry);
    return (int32_t)h;
}

static int or_lex_cmp(const void *a, const void *b)
{
    const int32_t *u = (const int32_t *)a, *v = (const int32_t *)b;
    if (u[0] != v[0]) return u[0] < v[0] ? -1 : 1;
    if (u[1] != v[1]) return u[1] < v[1] ? -1 : 1;
    return 0;
}

int64_t or_hull_full(const int32_t *pts, int64_t n, int32_t *vx, int32_t *vy)
{
    if (n < 0) return OR_EINVAL;
    if (n == 0) return 0;
    int32_t *q = (int32_t *)malloc((size_t)n * 2 * sizeof(int32_t));
    if (q == NULL) return OR_EINVAL;
    memcpy(q, pts, (size_t)n * 2 * sizeof(int32_t));
    qsort(q, (size_t)n, 2 * sizeof(int32_t), or_lex_cmp);

    /* keep one copy of each distinct point */
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (m > 0 && q[2 * (m - 1)] == q[2 * i] && q[2 * (m - 1) + 1] == q[2 * i + 1]) continue;
        q[2 * m] = q[2 * i];
        q[2 * m + 1] = q[2 * i + 1];
        ++m;
    }
    int32_t *px = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    int32_t *py = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    if (px == NULL || py == NULL) {
        free(q);
        free(px);
        free(py);
        return OR_EINVAL;
    }
    for (int64_t i = 0; i < m; ++i) {
        px[i] = q[2 * i];
        py[i] = q[2 * i + 1];
    }
    int64_t h = or_andrew(px, py, m, vx, vy);
    free(q);
    free(px);
    free(py);
    return h;
}

/* ---------------------------------------------------------------------------
 * Steps 1 and 2 of the proposed heuristic.
 *
 * Step 1 finds the extremes of x and y over P.  Step 2 moves P so that the
 * smallest x and the smallest y both become 1: x' = x - xmin + 1 and
 * y' = y - ymin + 1.  Algorithm 1 then runs on P' with one side p for both
 * coordinates, the larger of the two extents (xmax - xmin + 1 and
 * ymax - ymin + 1), so that every translated point lies in [1, p]^2.
 * ------------------------------------------------------------------------- */
int or_bbox(const int32_t *pts, int64_t n, int32_t *box)
{
    if (n < 1 || pts == NULL || box == NULL) return OR_EINVAL;
    int32_t xmin = pts[0], xmax = pts[0], ymin = pts[1], ymax = pts[1];
    for (int64_t j = 1; j < n; ++j) {
        int32_t x = pts[2 * j], y = pts[2 * j + 1];
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    box[0] = xmin;
    box[1] = xmax;
    box[2] = ymin;
    box[3] = ymax;
    return OR_OK;
}

/* Step 2 on the p x q box: the same translation, with p = xmax - xmin + 1
 * columns and q = ymax - ymin + 1 rows. */
int or_translate_rect(const int32_t *pts, int64_t n, const int32_t *box, int32_t *out, int32_t *p, int32_t *q)
{
    if (n < 1 || pts == NULL || box == NULL || out == NULL || p == NULL || q == NULL) return OR_EINVAL;
    const int64_t ex = (int64_t)box[1] - box[0] + 1, ey = (int64_t)box[3] - box[2] + 1;
    if (ex > OR_PMAX || ey > OR_PMAX) return OR_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        out[2 * j] = (int32_t)((int64_t)pts[2 * j] - box[0] + 1);
        out[2 * j + 1] = (int32_t)((int64_t)pts[2 * j + 1] - box[2] + 1);
    }
    *p = (int32_t)ex;
    *q = (int32_t)ey;
    return OR_OK;
}

int or_translate(const int32_t *pts, int64_t n, const int32_t *box, int32_t *out, int32_t *p)
{
    if (n < 1 || pts == NULL || box == NULL || out == NULL || p == NULL) return OR_EINVAL;
    int64_t ex = (int64_t)box[1] - box[0] + 1, ey = (int64_t)box[3] - box[2] + 1;
    int64_t side = ex > ey ? ex : ey;
    if (side > OR_PMAX) return OR_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        out[2 * j] = (int32_t)((int64_t)pts[2 * j] - box[0] + 1);
        out[2 * j + 1] = (int32_t)((int64_t)pts[2 * j + 1] - box[2] + 1);
    }
    *p = (int32_t)side;
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Discussion, "Extraction using an array of bits" and "Extraction using a
 * tree structure", with w = 64.
 *
 * Array: setting column i is M[(i-1) >> 6] |= 1 << ((i-1) & 63), and
 * extraction is or_extract above.
 *
 * Tree: level 0 is the array M.  A word of level k+1 holds one bit per word
 * of level k, set when that word is non-zero, so a group of 64 words of one
 * level maps to one word of the next.  Levels are added until a level holds
 * a single word (for p = 2^24: 262144, 4096, 64 and 1 words, 266305 in all).
 * The levels are stored one after another, level 0 first.  An insert sets the
 * bit of the column at every level (the h + 1 steps of the text); extraction
 * walks down from the top word, visiting the set bits of each word in
 * ascending order with the Table I loop, so the columns come out ascending
 * and empty words are never visited.
 * ------------------------------------------------------------------------- */
int32_t or_tree_levels(int32_t p, int64_t *offset)
{
    if (p < 1 || p > OR_PMAX) return OR_EINVAL;
    int32_t levels = 0;
    int64_t words = ((int64_t)p + 63) / 64, at = 0;
    for (;;) {
        if (offset != NULL) offset[levels] = at;
        at += words;
        ++levels;
        if (words == 1) break;
        words = (words + 63) / 64;
    }
    if (offset != NULL) offset[levels] = at;
    return levels;
}

int or_array_insert(int32_t p, const int32_t *cols, int64_t s, uint64_t *M)
{
    if (p < 1 || p > OR_PMAX || s < 0 || M == NULL || (s > 0 && cols == NULL)) return OR_EINVAL;
    for (int64_t j = 0; j < s; ++j)
        if (cols[j] < 1 || cols[j] > p) return OR_ERANGE;
    for (int64_t j = 0; j < s; ++j) {
        int64_t i = cols[j];
        M[(i - 1) >> 6] |= (uint64_t)1 << ((i - 1) & 63);
    }
    return OR_OK;
}

int or_tree_insert(int32_t p, const int32_t *cols, int64_t s, uint64_t *T)
{
    int64_t offset[8];
    int32_t levels = or_tree_levels(p, offset);
    if (levels < 0 || s < 0 || T == NULL || (s > 0 && cols == NULL)) return OR_EINVAL;
    for (int64_t j = 0; j < s; ++j)
        if (cols[j] < 1 || cols[j] > p) return OR_ERANGE;
    for (int64_t j = 0; j < s; ++j) {
        int64_t bit = cols[j] - 1;              /* bit index within level 0 */
        for (int32_t k = 0; k < levels; ++k) {
            T[offset[k] + (bit >> 6)] |= (uint64_t)1 << (bit & 63);
            bit >>= 6;                          /* the word index becomes the bit index above */
        }
    }
    return OR_OK;
}

static int32_t or_tree_visit(const uint64_t *T, const int64_t *offset, int32_t level, int64_t word,
                             int32_t *cols, int32_t k)
{
    int32_t pos[64];
    int32_t c = or_ctz_positions(T[offset[level] + word], pos);
    for (int32_t t = 0; t < c; ++t) {
        int64_t child = word * 64 + pos[t];
        if (level == 0)
            cols[k++] = (int32_t)(child + 1);
        else
            k = or_tree_visit(T, offset, level - 1, child, cols, k);
    }
    return k;
}

int32_t or_tree_extract(const uint64_t *T, int32_t p, int32_t *cols)
{
    int64_t offset[8];
    int32_t levels = or_tree_levels(p, offset);
    if (levels < 0 || T == NULL || cols == NULL) return OR_EINVAL;
    return or_tree_visit(T, offset, levels - 1, 0, cols, 0);
}

/* ---------------------------------------------------------------------------
 * Melkman's algorithm on the Lemma 1 polyline (Results, the linear hull of a
 * simple polyline; Conclusions).
 *
 * The reduced sequence R, walked column by column as (x, lo) then (x, hi),
 * is a simple polyline (Lemma 1), so Melkman's deque algorithm finds its hull
 * in one pass.  The deque holds the current hull counter-clockwise from
 * bottom to top, with the newest hull point at both ends.  A new point that
 * lies strictly left of both end edges is inside and skipped; otherwise the
 * top is popped while the point is not strictly left of the top edge, the
 * point is pushed on top, and the same is done at the bottom.  The result is
 * then put in the canonical form of the other hulls: vertices with a
 * straight angle removed, starting at the lexicographic minimum.
 *
 * The orientation test is written out here again on purpose, so that this
 * hull shares no arithmetic with the monotone-chain one it is checked
 * against.
 * ------------------------------------------------------------------------- */
static int64_t or_orient(const int32_t *a, const int32_t *b, const int32_t *c)
{
    /* twice the signed area of (a, b, c): > 0 when c is left of a -> b */
    int64_t abx = (int64_t)b[0] - a[0], aby = (int64_t)b[1] - a[1];
    int64_t acx = (int64_t)c[0] - a[0], acy = (int64_t)c[1] - a[1];
    return abx * acy - aby * acx;
}

int32_t or_hull_melkman(const int32_t *x, const int32_t *clo, const int32_t *chi,
                        int32_t k, int32_t *vx, int32_t *vy)
{
    if (k < 0) return OR_EINVAL;
    for (int32_t t = 0; t + 1 < k; ++t)
        if (!(x[t] < x[t + 1])) return OR_EORDER;
    for (int32_t t = 0; t < k; ++t)
        if (chi[t] < clo[t]) return OR_EORDER;

    /* R as interleaved (x, y) pairs */
    int64_t s = 0;
    int32_t *R = (int32_t *)malloc((size_t)(4 * (int64_t)k + 2) * sizeof(int32_t));
    int32_t *D = (int32_t *)malloc((size_t)(2 * (4 * (int64_t)k + 1) + 2) * sizeof(int32_t));
    if (R == NULL || D == NULL) {
        free(R);
        free(D);
        return OR_EINVAL;
    }
    for (int32_t t = 0; t < k; ++t) {
        R[2 * s] = x[t];
        R[2 * s + 1] = clo[t];
        ++s;
        if (chi[t] > clo[t]) {
            R[2 * s] = x[t];
            R[2 * s + 1] = chi[t];
            ++s;
        }
    }
    int64_t h = 0;
    if (s <= 2) {
        for (int64_t i = 0; i < s; ++i) {
            vx[i] = R[2 * i];
            vy[i] = R[2 * i + 1];
        }
        h = s;
        goto done;
    }
    {
        /* a, b: the first two points; points collinear with them move b along
         * the line (the walk is x-monotone, so the newest is the far end) */
        const int32_t *a = &R[0], *b = &R[2];
        int64_t j = 2;
        while (j < s && or_orient(a, b, &R[2 * j]) == 0) b = &R[2 * j++];
        if (j == s) {
            vx[0] = a[0];
            vy[0] = a[1];
            vx[1] = b[0];
            vy[1] = b[1];
            h = 2;
            goto done;
        }
        const int32_t *c = &R[2 * j];
        /* deque of points D[bot..top] (2 ints each), room for 2s + 1 */
        int64_t bot = s, top = s + 3;
        const int32_t *first = or_orient(a, b, c) > 0 ? a : b;
        const int32_t *second = first == a ? b : a;
#define DQ(i) (&D[2 * (i)])
        DQ(bot)[0] = c[0], DQ(bot)[1] = c[1];
        DQ(bot + 1)[0] = first[0], DQ(bot + 1)[1] = first[1];
        DQ(bot + 2)[0] = second[0], DQ(bot + 2)[1] = second[1];
        DQ(top)[0] = c[0], DQ(top)[1] = c[1];
        for (int64_t i = j + 1; i < s; ++i) {
            const int32_t *v = &R[2 * i];
            if (or_orient(DQ(top - 1), DQ(top), v) > 0 && or_orient(DQ(bot), DQ(bot + 1), v) > 0) continue;
            while (top - bot >= 2 && or_orient(DQ(top - 1), DQ(top), v) <= 0) --top;
            ++top;
            DQ(top)[0] = v[0], DQ(top)[1] = v[1];
            while (top - bot >= 2 && or_orient(DQ(bot), DQ(bot + 1), v) <= 0) ++bot;
            --bot;
            DQ(bot)[0] = v[0], DQ(bot)[1] = v[1];
        }
        /* the hull, counter-clockwise: D[bot..top-1] (D[top] repeats D[bot]) */
        int64_t m = top - bot;
        int32_t *H = &D[2 * bot];
        /* drop vertices with a straight angle until none is left */
        int changed = 1;
        while (changed && m > 2) {
            changed = 0;
            for (int64_t i = 0; i < m && m > 2; ++i) {
                const int32_t *pv = &H[2 * ((i + m - 1) % m)], *cv = &H[2 * i], *nv = &H[2 * ((i + 1) % m)];
                if (or_orient(pv, cv, nv) == 0) {
                    memmove(&H[2 * i], &H[2 * i + 2], (size_t)(m - i - 1) * 2 * sizeof(int32_t));
                    --m;
                    changed = 1;
                    --i;
                }
            }
        }
        /* start at the lexicographic minimum */
        int64_t lo = 0;
        for (int64_t i = 1; i < m; ++i)
            if (H[2 * i] < H[2 * lo] || (H[2 * i] == H[2 * lo] && H[2 * i + 1] < H[2 * lo + 1])) lo = i;
        for (int64_t i = 0; i < m; ++i) {
            vx[i] = H[2 * ((lo + i) % m)];
            vy[i] = H[2 * ((lo + i) % m) + 1];
        }
        h = m;
#undef DQ
    }
done:
    free(R);
    free(D);
    return (int32_t)h;
}

/* ---------------------------------------------------------------------------
 * Floating-point input (Conclusions: data with floating-point coordinates is
 * brought to integers by a suitable scaling).
 *
 * Step 1 on float points: the extremes of x and y, NaN coordinates skipped.
 * The scaling: X = floor((x - ox) * s) + 1 and Y = floor((y - oy) * s) + 1,
 * evaluated in double precision as written (the float widened exactly, one
 * subtraction, one multiplication, each rounded to nearest).  A coordinate
 * whose result is NaN or outside [1, 2^31 - 2] is reported (OR_ERANGE) and
 * written as 0.  With ox = xmin, oy = ymin and s = (p - 1) / max extent
 * every point lands in [1, p]^2.
 * ------------------------------------------------------------------------- */
int or_bbox_f32(const float *pts, int64_t n, float *box)
{
    if (n < 0 || box == NULL || (n > 0 && pts == NULL)) return OR_EINVAL;
    int any = 0;
    for (int64_t j = 0; j < n; ++j) {
        float x = pts[2 * j], y = pts[2 * j + 1];
        if (x != x || y != y) continue;             /* a NaN coordinate */
        if (!any || x < box[0]) box[0] = x;
        if (!any || x > box[1]) box[1] = x;
        if (!any || y < box[2]) box[2] = y;
        if (!any || y > box[3]) box[3] = y;
        any = 1;
    }
    return any ? OR_OK : OR_ERANGE;
}

static int32_t or_scale_one(float v, double o, double s, int *bad)
{
    double t = floor(((double)v - o) * s);
    if (!(t >= 0.0 && t <= (double)(OR_PMAX - 1))) {   /* also catches NaN */
        *bad = 1;
        return 0;
    }
    return (int32_t)t + 1;
}

int or_quantize_f32(const float *pts, int64_t n, double ox, double oy, double s, int32_t *out)
{
    if (n < 0 || out == NULL || (n > 0 && pts == NULL)) return OR_EINVAL;
    int bad = 0;
    for (int64_t j = 0; j < n; ++j) {
        out[2 * j] = or_scale_one(pts[2 * j], ox, s, &bad);
        out[2 * j + 1] = or_scale_one(pts[2 * j + 1], oy, s, &bad);
    }
    return bad ? OR_ERANGE : OR_OK;
}

