/*
 * CPU grid self-join: the host-core baseline that the GPU path is reported
 * against, beside the brute-force oracle.
 *
 * TEST AND BASELINE INFRASTRUCTURE ONLY. Nothing in the product path may
 * call, link or load this file. It shares no code, header or constant with
 * the HIP implementation.
 *
 * The method of Section IV on the host, written plainly: cells of width
 * w >= eps (Section IV-B), points sorted by linearised cell id so each
 * non-empty cell is one run of the sorted order (Section IV-C), and for each
 * non-empty cell the 3^d adjacent cells looked up by binary search among the
 * non-empty cell ids (Algorithm 1's lookup; every point of a cell has the
 * same adjacent cells) and their points scanned for each point of the cell.
 * The coordinates are read from a copy in the sorted order, so a cell's
 * points are contiguous in memory; the pair test is the oracle's: squared
 * distance in binary64, dimension order 0..d-1, no fused multiply-add
 * (-ffp-contract=off), accepted iff d2 <= fl(eps * eps). Every row's
 * neighbours are sorted ascending, so the pairs come out sorted by (i, j),
 * the same result as sjo_fill_rows.
 *
 * Cells are processed in parallel with OpenMP; the result does not depend
 * on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SJG_MAX_DIM 8

typedef struct {
    uint64_t key;
    uint32_t id;
} sjg_item;

static int sjg_cmp_item(const void *a, const void *b)
{
    const sjg_item *x = (const sjg_item *)a, *y = (const sjg_item *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

static int sjg_cmp_u32(const void *a, const void *b)
{
    const uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y);
}

static int sjg_within(const double *a, const double *b, int d, double eps2)
{
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        double sq = t * t;
        acc = acc + sq;
    }
    return acc <= eps2;
}

typedef struct {
    int d;
    double lo[SJG_MAX_DIM], w;
    uint64_t dims[SJG_MAX_DIM], stride[SJG_MAX_DIM];
    uint64_t ncells;     /* non-empty cells */
    uint64_t *cell_key;  /* ascending */
    uint64_t *cell_start;/* ncells + 1 */
    uint32_t *order;     /* point ids in cell order */
    uint32_t *coord;     /* n x d cell coordinates of each point */
    double *xs;          /* n x d coordinates in cell order: xs[r] = x[order[r]] */
} sjg_grid;

static uint64_t sjg_coord(double v, double lo, double w, uint64_t dim)
{
    double t = floor((v - lo) / w);
    if (!(t > 0.0)) return 0;
    if (t >= (double)(dim - 1)) return dim - 1;
    return (uint64_t)t;
}

static int sjg_build(const double *x, int64_t n, int d, double eps, sjg_grid *g)
{
    memset(g, 0, sizeof(*g));
    g->d = d;
    double hi[SJG_MAX_DIM];
    for (int k = 0; k < d; ++k) {
        g->lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            double v = x[i * d + k];
            if (v < g->lo[k]) g->lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    /* any width >= eps is correct; widen until the cell count fits 62 bits */
    g->w = eps * (1.0 + 1.0 / 65536.0);
    for (;;) {
        double prod = 1.0;
        for (int k = 0; k < d; ++k) {
            g->dims[k] = (uint64_t)floor((hi[k] - g->lo[k]) / g->w) + 1;
            prod *= (double)g->dims[k];
        }
        if (prod < 4.0e18) break;
        g->w *= 2.0;
    }
    uint64_t s = 1;
    for (int k = 0; k < d; ++k) {
        g->stride[k] = s;
        s *= g->dims[k];
    }
    sjg_item *items = (sjg_item *)malloc((size_t)n * sizeof(sjg_item));
    g->coord = (uint32_t *)malloc((size_t)n * (size_t)d * sizeof(uint32_t));
    if (!items || !g->coord) {
        free(items);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t key = 0;
        for (int k = 0; k < d; ++k) {
            uint64_t c = sjg_coord(x[i * d + k], g->lo[k], g->w, g->dims[k]);
            g->coord[i * d + k] = (uint32_t)c;
            key += c * g->stride[k];
        }
        items[i].key = key;
        items[i].id = (uint32_t)i;
    }
    qsort(items, (size_t)n, sizeof(sjg_item), sjg_cmp_item);
    g->order = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    g->cell_key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    g->cell_start = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!g->order || !g->cell_key || !g->cell_start) {
        free(items);
        return -1;
    }
    uint64_t nc = 0;
    for (int64_t r = 0; r < n; ++r) {
        g->order[r] = items[r].id;
        if (r == 0 || items[r].key != items[r - 1].key) {
            g->cell_key[nc] = items[r].key;
            g->cell_start[nc] = (uint64_t)r;
            ++nc;
        }
    }
    g->cell_start[nc] = (uint64_t)n;
    g->ncells = nc;
    free(items);
    g->xs = (double *)malloc((size_t)n * (size_t)d * sizeof(double));
    if (!g->xs) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r)
        for (int k = 0; k < d; ++k) g->xs[r * d + k] = x[(int64_t)g->order[r] * d + k];
    return 0;
}

static void sjg_free(sjg_grid *g)
{
    free(g->cell_key);
    free(g->cell_start);
    free(g->order);
    free(g->coord);
    free(g->xs);
}

/* position of key among the non-empty cells, or -1 */
static int64_t sjg_find(const sjg_grid *g, uint64_t key)
{
    uint64_t lo = 0, hi = g->ncells;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (g->cell_key[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < g->ncells && g->cell_key[lo] == key) ? (int64_t)lo : -1;
}

/*
 * Point ranges [lo, hi) of the sorted order covering the non-empty cells
 * among the 3^d cells adjacent to cell h (h itself included); returns their
 * number (at most 3^d, the capacity of rng).
 */
static int sjg_adjacent(const sjg_grid *g, uint64_t h, uint64_t *rng)
{
    const int d = g->d;
    const uint32_t *c0 = g->coord + (int64_t)g->order[g->cell_start[h]] * d;
    int off[SJG_MAX_DIM];
    for (int k = 0; k < d; ++k) off[k] = -1;
    int m = 0;
    for (;;) {
        int inside = 1;
        uint64_t key = 0;
        for (int k = 0; k < d; ++k) {
            int64_t v = (int64_t)c0[k] + off[k];
            if (v < 0 || v >= (int64_t)g->dims[k]) {
                inside = 0;
                break;
            }
            key += (uint64_t)v * g->stride[k];
        }
        if (inside) {
            int64_t a = sjg_find(g, key);
            if (a >= 0) {
                rng[2 * m] = g->cell_start[a];
                rng[2 * m + 1] = g->cell_start[a + 1];
                ++m;
            }
        }
        int k = 0;
        while (k < d && off[k] == 1) off[k++] = -1;
        if (k == d) break;
        ++off[k];
    }
    return m;
}

/*
 * Neighbours of the point at sorted position p into buf (capacity cap),
 * scanning the ranges of its cell's adjacent cells; returns the row length
 * (which may exceed cap: then only the count is valid).
 */
static uint64_t sjg_row(const sjg_grid *g, uint64_t p, const uint64_t *rng, int m, double eps2, uint32_t *buf,
                        uint64_t cap)
{
    const int d = g->d;
    const double *a = g->xs + (int64_t)p * d;
    uint64_t len = 0;
    for (int e = 0; e < m; ++e)
        for (uint64_t r = rng[2 * e]; r < rng[2 * e + 1]; ++r)
            if (sjg_within(a, g->xs + (int64_t)r * d, d, eps2)) {
                if (len < cap) buf[len] = g->order[r];
                ++len;
            }
    return len;
}

/*
 * Grid self-join. counts (n entries) receives every row length. If pairs is
 * not NULL it receives the interleaved (i, j) pairs sorted by (i, j) and
 * must hold the total. Returns the number of pairs, or -1 if out of memory.
 */
int64_t sjg_grid_join(const double *x, int64_t n, int64_t d, double eps, int64_t *counts, int32_t *pairs)
{
    if (n <= 0) return 0;
    if (d < 1 || d > SJG_MAX_DIM) return -1;
    sjg_grid g;
    if (sjg_build(x, n, (int)d, eps, &g) != 0) {
        sjg_free(&g);
        return -1;
    }
    int adj = 1;
    for (int k = 0; k < d; ++k) adj *= 3;
    const double eps2 = eps * eps;
    int64_t total = 0;
    int fail = 0;
#pragma omp parallel reduction(+ : total)
    {
        uint64_t *rng = (uint64_t *)malloc((size_t)adj * 2 * sizeof(uint64_t));
        if (!rng) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t h = 0; h < (int64_t)g.ncells; ++h) {
            if (!rng) continue;
            const int m = sjg_adjacent(&g, (uint64_t)h, rng);
            for (uint64_t p = g.cell_start[h]; p < g.cell_start[h + 1]; ++p) {
                const int64_t c = (int64_t)sjg_row(&g, p, rng, m, eps2, NULL, 0);
                counts[g.order[p]] = c;
                total += c;
            }
        }
        free(rng);
    }
    if (fail) {
        sjg_free(&g);
        return -1;
    }
    if (pairs) {
        int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
        if (!off) {
            sjg_free(&g);
            return -1;
        }
        off[0] = 0;
        for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + counts[i];
#pragma omp parallel
        {
            uint64_t cap = 1024;
            uint32_t *buf = (uint32_t *)malloc(cap * sizeof(uint32_t));
            uint64_t *rng = (uint64_t *)malloc((size_t)adj * 2 * sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
            for (int64_t h = 0; h < (int64_t)g.ncells; ++h) {
                const int m = sjg_adjacent(&g, (uint64_t)h, rng);
                for (uint64_t p = g.cell_start[h]; p < g.cell_start[h + 1]; ++p) {
                    const uint32_t i = g.order[p];
                    if ((uint64_t)counts[i] > cap) {
                        cap = (uint64_t)counts[i];
                        free(buf);
                        buf = (uint32_t *)malloc(cap * sizeof(uint32_t));
                    }
                    const uint64_t len = sjg_row(&g, p, rng, m, eps2, buf, cap);
                    qsort(buf, (size_t)len, sizeof(uint32_t), sjg_cmp_u32);
                    for (uint64_t k = 0; k < len; ++k) {
                        pairs[2 * (off[i] + (int64_t)k)] = (int32_t)i;
                        pairs[2 * (off[i] + (int64_t)k) + 1] = (int32_t)buf[k];
                    }
                }
            }
            free(buf);
            free(rng);
        }
        free(off);
    }
    sjg_free(&g);
    return total;
}
