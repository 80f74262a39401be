/*
 * Baryon-block oracle: plain, slow complex128 CPU loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP
 * library.
 *
 * What it computes (paper, Sec. 2, eq. (3) written with the reconstructed
 * quark fields, i.e. with spin and noise labels fixed by the caller as the
 * paper states right after eq. (1)):
 *
 *   B[p][d1][d2][d3] = sum_x exp(-i p.x) sum_{a,b,c} eps_abc
 *                      q1[x][a][d1] q2[x][b][d2] q3[x][c][d3]
 *
 * Readings of points the paper leaves open:
 *   - momenta are integer vectors n with p = 2 pi n / L; the phase is formed
 *     from the exact integer reduction k = (n . x) mod L, so
 *     exp(-i p.x) = cos(2 pi k / L) - i sin(2 pi k / L);
 *   - site index x = ix + L*(iy + L*iz), origin at site 0;
 *   - eps_012 = +1 (Levi-Civita symbol);
 *   - dilution indices are 0-based; output is [p][d1][d2][d3].
 *
 * The sum over x runs serially in site order for every output entry.  The
 * epsilon sum is evaluated once per (x, d1, d2, d3) and then multiplied by the
 * phase of every momentum: a hoisting of a common factor, no reordering of the
 * sum over sites.
 *
 * Inputs are complex128 interleaved (re, im): q_i has layout [V][3][n_i].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Levi-Civita symbol on {0,1,2}: +1 for even permutations of (0,1,2), -1 for
 * odd ones, 0 when two indices coincide.  (a-b)(b-c)(c-a)/2 is exactly that
 * on this index set. */
static int levi_civita(int a, int b, int c)
{
    return ((a - b) * (b - c) * (c - a)) / 2;
}

/* exp(-i 2 pi k / L) for the reduced integer phase index k in [0, L). */
static double complex phase_of_index(int64_t k, int L)
{
    const double ang = 2.0 * M_PI * (double)k / (double)L;
    return cos(ang) - I * sin(ang);
}

static int64_t mod_nonneg(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/*
 * Rows variant: computes B for a list of (d1, d2) pairs, all d3, all momenta.
 *   rows : [n_rows][2] int32 (d1, d2)
 *   out  : [n_mom][n_rows][n3] complex128 interleaved
 * The full block is the special case rows = all (d1, d2) in row-major order,
 * which makes out equal to B[p][d1][d2][d3].
 * Returns 0 on success, -1 on invalid arguments.
 */
int oracle_bblock_rows(int L, int n1, int n2, int n3,
                       const double *q1, const double *q2, const double *q3,
                       int n_mom, const int32_t *mom,
                       int n_rows, const int32_t *rows,
                       double *out)
{
    if (L <= 0 || n1 <= 0 || n2 <= 0 || n3 <= 0 || n_mom <= 0 || n_rows < 0)
        return -1;
    if (!q1 || !q2 || !q3 || !mom || !out || (n_rows > 0 && !rows))
        return -1;
    for (int r = 0; r < n_rows; ++r)
        if (rows[2 * r] < 0 || rows[2 * r] >= n1 || rows[2 * r + 1] < 0 || rows[2 * r + 1] >= n2)
            return -1;

    const int64_t V = (int64_t)L * L * L;
    const double complex *Q1 = (const double complex *)q1;
    const double complex *Q2 = (const double complex *)q2;
    const double complex *Q3 = (const double complex *)q3;
    double complex *OUT = (double complex *)out;

#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rows; ++r) {
        const int d1 = rows[2 * r], d2 = rows[2 * r + 1];
        double complex *acc = (double complex *)calloc((size_t)n_mom * n3, sizeof(double complex));
        double complex *ph = (double complex *)malloc((size_t)n_mom * sizeof(double complex));
        for (int64_t x = 0; x < V; ++x) {
            const int64_t ix = x % L, iy = (x / L) % L, iz = x / ((int64_t)L * L);
            for (int p = 0; p < n_mom; ++p) {
                const int64_t nx = mom[3 * p], ny = mom[3 * p + 1], nz = mom[3 * p + 2];
                ph[p] = phase_of_index(mod_nonneg(nx * ix + ny * iy + nz * iz, L), L);
            }
            for (int d3 = 0; d3 < n3; ++d3) {
                double complex s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        for (int c = 0; c < 3; ++c) {
                            const int e = levi_civita(a, b, c);
                            if (e == 0) continue;
                            s += (double)e * Q1[(x * 3 + a) * n1 + d1]
                                           * Q2[(x * 3 + b) * n2 + d2]
                                           * Q3[(x * 3 + c) * n3 + d3];
                        }
                for (int p = 0; p < n_mom; ++p)
                    acc[(size_t)p * n3 + d3] += ph[p] * s;
            }
        }
        for (int p = 0; p < n_mom; ++p)
            for (int d3 = 0; d3 < n3; ++d3)
                OUT[((size_t)p * n_rows + r) * n3 + d3] = acc[(size_t)p * n3 + d3];
        free(ph);
        free(acc);
    }
    return 0;
}

/*
 * Entries variant: B[p][d1][d2][d3] for a list of (d1, d2, d3) index triples
 * and every momentum, each entry summed over sites exactly as in the rows
 * variant (serial in x, the epsilon sum per site, then the phase).  For
 * sampled checks of large blocks where even whole rows are expensive.
 *   entries : [n_ent][3] int32 (d1, d2, d3)
 *   out     : [n_mom][n_ent] complex128 interleaved
 * Returns 0 on success, -1 on invalid arguments.
 */
int oracle_bblock_entries(int L, int n1, int n2, int n3,
                          const double *q1, const double *q2, const double *q3,
                          int n_mom, const int32_t *mom,
                          int n_ent, const int32_t *entries,
                          double *out)
{
    if (L <= 0 || n1 <= 0 || n2 <= 0 || n3 <= 0 || n_mom <= 0 || n_ent < 0)
        return -1;
    if (!q1 || !q2 || !q3 || !mom || !out || (n_ent > 0 && !entries))
        return -1;
    for (int e = 0; e < n_ent; ++e)
        if (entries[3 * e] < 0 || entries[3 * e] >= n1 || entries[3 * e + 1] < 0 || entries[3 * e + 1] >= n2 ||
            entries[3 * e + 2] < 0 || entries[3 * e + 2] >= n3)
            return -1;

    const int64_t V = (int64_t)L * L * L;
    const double complex *Q1 = (const double complex *)q1;
    const double complex *Q2 = (const double complex *)q2;
    const double complex *Q3 = (const double complex *)q3;
    double complex *OUT = (double complex *)out;
    /* The L phases exp(-2 pi i k / L), tabulated once (the same values the
     * rows variant forms per site). */
    double complex *root = (double complex *)malloc((size_t)L * sizeof(double complex));
    if (!root) return -1;
    for (int k = 0; k < L; ++k) root[k] = phase_of_index(k, L);

#pragma omp parallel for schedule(dynamic, 1)
    for (int e = 0; e < n_ent; ++e) {
        const int d1 = entries[3 * e], d2 = entries[3 * e + 1], d3 = entries[3 * e + 2];
        double complex *acc = (double complex *)calloc((size_t)n_mom, sizeof(double complex));
        for (int64_t x = 0; x < V; ++x) {
            const int64_t ix = x % L, iy = (x / L) % L, iz = x / ((int64_t)L * L);
            double complex s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    for (int c = 0; c < 3; ++c) {
                        const int eps = levi_civita(a, b, c);
                        if (eps == 0) continue;
                        s += (double)eps * Q1[(x * 3 + a) * n1 + d1]
                                         * Q2[(x * 3 + b) * n2 + d2]
                                         * Q3[(x * 3 + c) * n3 + d3];
                    }
            for (int p = 0; p < n_mom; ++p) {
                const int64_t nx = mom[3 * p], ny = mom[3 * p + 1], nz = mom[3 * p + 2];
                acc[p] += root[mod_nonneg(nx * ix + ny * iy + nz * iz, L)] * s;
            }
        }
        for (int p = 0; p < n_mom; ++p)
            OUT[(size_t)p * n_ent + e] = acc[p];
        free(acc);
    }
    free(root);
    return 0;
}

/* Full block B[p][d1][d2][d3] (eq. (3)); out is [n_mom][n1][n2][n3] complex128. */
int oracle_bblock(int L, int n1, int n2, int n3,
                  const double *q1, const double *q2, const double *q3,
                  int n_mom, const int32_t *mom, double *out)
{
    if (n1 <= 0 || n2 <= 0) return -1;
    const int n_rows = n1 * n2;
    int32_t *rows = (int32_t *)malloc((size_t)n_rows * 2 * sizeof(int32_t));
    if (!rows) return -1;
    for (int d1 = 0; d1 < n1; ++d1)
        for (int d2 = 0; d2 < n2; ++d2) {
            rows[2 * (d1 * n2 + d2)] = d1;
            rows[2 * (d1 * n2 + d2) + 1] = d2;
        }
    const int rc = oracle_bblock_rows(L, n1, n2, n3, q1, q2, q3, n_mom, mom, n_rows, rows, out);
    free(rows);
    return rc;
}

/* Sets the OpenMP thread count of later calls (the CPU baseline times the
 * oracle on one thread and on all of them); returns the count now in force. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Threads the OpenMP runtime will use (reported beside CPU timings). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
