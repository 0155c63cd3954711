/*
 * Brute-force CPU oracle for the Euclidean epsilon-distance self-join.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header or constant with
 * the HIP implementation.
 *
 * What it computes (Section III, problem statement): every ordered pair
 * (i, j) of rows of the n x d point array with dist(p_i, p_j) <= eps, where
 * dist is the Euclidean distance. As documented with the oracle, the
 * comparison is made on squared distances:
 *
 *     d2(i, j) = (...((t_0*t_0) + t_1*t_1) + ...) + t_{d-1}*t_{d-1},
 *     t_k = x[i][k] - x[j][k],
 *
 * evaluated in IEEE binary64 in dimension order 0..d-1 with every operation
 * rounded separately (the build passes -ffp-contract=off and no -march flag,
 * so no fused multiply-add is ever formed), and the pair is in the result
 * iff d2(i, j) <= fl(eps * eps). Every (i, i) is in the result (d2 = 0) and
 * both orders of every pair are reported (Section V-B reports (p, q) and
 * (q, p)). The output of sjo_fill_rows lists, per query row, its neighbours
 * in ascending j, so concatenating rows in ascending i gives the pairs
 * sorted by (i, j).
 *
 * O(n^2) work; rows are processed in parallel with OpenMP, each row scans
 * all n candidates in order, so the result does not depend on the thread
 * count.
 */
#include <stdint.h>
#include <stddef.h>

static int within(const double *a, const double *b, int d, double eps2)
{
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        double sq = t * t;
        acc = acc + sq;
    }
    return acc <= eps2;
}

/* Squared distance, same evaluation order as within(). */
double sjo_d2(const double *x, int64_t d, int64_t i, int64_t j)
{
    double acc = 0.0;
    for (int64_t k = 0; k < d; ++k) {
        double t = x[i * d + k] - x[j * d + k];
        double sq = t * t;
        acc = acc + sq;
    }
    return acc;
}

/*
 * Neighbour count of each query row (rows == NULL means rows 0..n-1).
 * counts[r] receives the number of j in [0, n) within eps of row rows[r].
 * Returns the sum of the counts.
 */
int64_t sjo_count_rows(const double *x, int64_t n, int64_t d, double eps,
                       const int64_t *rows, int64_t nrows, int64_t *counts)
{
    const double eps2 = eps * eps;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        const double *a = x + i * d;
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            c += within(a, x + j * d, (int)d, eps2);
        counts[r] = c;
        total += c;
    }
    return total;
}

/*
 * Neighbour lists of the query rows: for query r, the ascending j within eps
 * of row rows[r] are written to out_j[row_off[r] ...]. row_off must come from
 * the counts of sjo_count_rows for the same rows and eps.
 */
void sjo_fill_rows(const double *x, int64_t n, int64_t d, double eps,
                   const int64_t *rows, int64_t nrows, const int64_t *row_off,
                   uint32_t *out_j)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        const double *a = x + i * d;
        int64_t pos = row_off[r];
        for (int64_t j = 0; j < n; ++j)
            if (within(a, x + j * d, (int)d, eps2))
                out_j[pos++] = (uint32_t)j;
    }
}

/*
 * Neighbour counts of the query rows for several radii at once (used to
 * choose eps for a target neighbour count). eps_sorted must be ascending;
 * counts[r * neps + e] receives the number of j within eps_sorted[e] of row
 * rows[r].
 */
void sjo_count_rows_multi(const double *x, int64_t n, int64_t d,
                          const double *eps_sorted, int64_t neps,
                          const int64_t *rows, int64_t nrows, int64_t *counts)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        int64_t *c = counts + r * neps;
        for (int64_t e = 0; e < neps; ++e)
            c[e] = 0;
        const double big2 = eps_sorted[neps - 1] * eps_sorted[neps - 1];
        for (int64_t j = 0; j < n; ++j) {
            const double s = sjo_d2(x, d, i, j);
            if (!(s <= big2))
                continue;
            /* first radius whose square admits s */
            int64_t lo = 0, hi = neps - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (s <= eps_sorted[mid] * eps_sorted[mid])
                    hi = mid;
                else
                    lo = mid + 1;
            }
            c[lo] += 1;
        }
        for (int64_t e = 1; e < neps; ++e)
            c[e] += c[e - 1];
    }
}
