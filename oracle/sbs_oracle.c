/*
 * Oracle for batched solves against one shared tridiagonal or pentadiagonal
 * matrix (Gloster, Carroll, Bustamante, O Naraigh, "Efficient Interleaved
 * Batch Matrix Solvers for CUDA", arXiv:1909.04539).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Arithmetic: IEEE binary64, round to nearest even, true division (no
 * reciprocal multiply), no fused multiply-add (build with -ffp-contract=off),
 * subnormals kept.  Every expression is evaluated left to right exactly as
 * written in the comments.
 *
 * Storage (Section 2 of the paper): the right-hand sides are interleaved, so
 * unknown i of system j lives at d[i*ld + j].  For the plain batch ld == m;
 * other strides let the same routine walk one contiguous row (ld == 1, m == 1).
 *
 * Band convention (rows are 0-based here, the paper counts from 1):
 *   tridiagonal row i reads  a_i x_{i-1} + b_i x_i + c_i x_{i+1}
 *   pentadiagonal row i reads a_i x_{i-2} + b_i x_{i-1} + c_i x_i
 *                             + d_i x_{i+1} + e_i x_{i+2}
 * Coefficients that fall outside the matrix (tri: a_0, c_{n-1}; penta: a_0,
 * a_1, b_0, d_{n-1}, e_{n-2}, e_{n-1}) are never read; they count as zero.
 *
 * Return convention: -1 on success, otherwise the 0-based row whose pivot is
 * zero or not finite (the paper has no pivoting and no failure rule; a zero
 * or non-finite pivot is reported, never divided by).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int bad_pivot(double p) { return !(isfinite(p) && p != 0.0); }

/* ---------------------------------------------------------------------------
 * Tridiagonal pre-factorisation, Section 3.1 (the equations for c-hat).
 *   chat_0 = c_0 / b_0
 *   chat_i = c_i / (b_i - a_i chat_{i-1}),  i = 1..n-1
 * The denominator b_i - a_i chat_{i-1} depends only on the matrix; the
 * forward sweep divides by the same quantity, so it is kept as den_i
 * (den_0 = b_0).  c_{n-1} lies outside the matrix, so chat_{n-1} = 0.
 */
int64_t oracle_tri_factor(int64_t n, const double *a, const double *b,
                          const double *c, double *den, double *chat)
{
    if (n < 1) return 0;
    den[0] = b[0];
    if (bad_pivot(den[0])) return 0;
    chat[0] = (n > 1) ? c[0] / den[0] : 0.0;
    for (int64_t i = 1; i < n; ++i) {
        den[i] = b[i] - a[i] * chat[i - 1];
        if (bad_pivot(den[i])) return i;
        chat[i] = (i < n - 1) ? c[i] / den[i] : 0.0;
    }
    return -1;
}

/* Tridiagonal forward and backward sweeps, Section 3.1, applied to m
 * interleaved systems in place.
 *   forward:  dhat_0 = d_0 / b_0,  dhat_i = (d_i - a_i dhat_{i-1}) / den_i
 *   backward: x_{n-1} = dhat_{n-1}, x_i = dhat_i - chat_i x_{i+1}
 * (The paper's printed back-substitution omits x_{i+1}; the standard Thomas
 * step used here is the one that solves the system.)
 * Loop order: row i outer, system j inner, so each row is one contiguous
 * pass over the interleaved array. */
void oracle_tri_apply(int64_t n, int64_t m, int64_t ld, const double *a,
                      const double *den, const double *chat, double *d)
{
    for (int64_t j = 0; j < m; ++j) d[j] = d[j] / den[0];
    for (int64_t i = 1; i < n; ++i) {
        double *row = d + i * ld;
        const double *prev = d + (i - 1) * ld;
        for (int64_t j = 0; j < m; ++j) row[j] = (row[j] - a[i] * prev[j]) / den[i];
    }
    for (int64_t i = n - 2; i >= 0; --i) {
        double *row = d + i * ld;
        const double *next = d + (i + 1) * ld;
        for (int64_t j = 0; j < m; ++j) row[j] = row[j] - chat[i] * next[j];
    }
}

int64_t oracle_tri_solve(int64_t n, int64_t m, int64_t ld, const double *a,
                         const double *b, const double *c, double *d)
{
    if (n < 1) return 0;
    double *den = (double *)malloc(sizeof(double) * (size_t)n);
    double *chat = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t bad = oracle_tri_factor(n, a, b, c, den, chat);
    if (bad < 0) oracle_tri_apply(n, m, ld, a, den, chat, d);
    free(den);
    free(chat);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Pentadiagonal factorisation A = L R, Section 4.1.  L is lower triangular
 * with diagonal alpha_i and sub-diagonals beta_i (one below) and epsilon_i
 * (two below); R is unit upper triangular with super-diagonals gamma_i and
 * delta_i.  Matching the entries of L R against A row by row gives
 *   beta_i  = b_i - a_i gamma_{i-2}
 *   alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1}
 *   gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i
 *   delta_i = e_i / alpha_i
 *   epsilon_i = a_i
 * The paper writes the first two rows and the last two rows out separately
 * because their neighbours fall outside the matrix.  Here one loop covers all
 * rows: every coefficient and every gamma/delta with an index outside the
 * matrix is taken as 0, which turns the general step into exactly those
 * special rows (alpha_0 = c_0, beta_1 = b_1, and delta_{n-2}, gamma_{n-1},
 * delta_{n-1} come out as zero, the entries R does not have).
 */
int64_t oracle_penta_factor(int64_t n, const double *a, const double *b,
                            const double *c, const double *d, const double *e,
                            double *alpha, double *beta, double *gamma,
                            double *delta, double *eps)
{
    for (int64_t i = 0; i < n; ++i) {
        double ai = (i >= 2) ? a[i] : 0.0;
        double bi = (i >= 1) ? b[i] : 0.0;
        double di = (i <= n - 2) ? d[i] : 0.0;
        double ei = (i <= n - 3) ? e[i] : 0.0;
        double gm2 = (i >= 2) ? gamma[i - 2] : 0.0;
        double gm1 = (i >= 1) ? gamma[i - 1] : 0.0;
        double dm2 = (i >= 2) ? delta[i - 2] : 0.0;
        double dm1 = (i >= 1) ? delta[i - 1] : 0.0;
        beta[i] = bi - ai * gm2;
        alpha[i] = c[i] - ai * dm2 - beta[i] * gm1;
        if (bad_pivot(alpha[i])) return i;
        gamma[i] = (di - beta[i] * dm1) / alpha[i];
        delta[i] = ei / alpha[i];
        eps[i] = ai;
    }
    return -1;
}

/* Pentadiagonal solve of m interleaved systems in place, Section 4.1.
 *   L g = f:  g_i = (f_i - epsilon_i g_{i-2} - beta_i g_{i-1}) / alpha_i
 *   R x = g:  x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}
 * with g and x outside the matrix equal to 0. */
void oracle_penta_apply(int64_t n, int64_t m, int64_t ld, const double *alpha,
                        const double *beta, const double *gamma,
                        const double *delta, const double *eps, double *f)
{
    for (int64_t i = 0; i < n; ++i) {
        double *row = f + i * ld;
        const double *p1 = (i >= 1) ? f + (i - 1) * ld : NULL;
        const double *p2 = (i >= 2) ? f + (i - 2) * ld : NULL;
        for (int64_t j = 0; j < m; ++j) {
            double g2 = p2 ? p2[j] : 0.0;
            double g1 = p1 ? p1[j] : 0.0;
            row[j] = (row[j] - eps[i] * g2 - beta[i] * g1) / alpha[i];
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double *row = f + i * ld;
        const double *n1 = (i + 1 < n) ? f + (i + 1) * ld : NULL;
        const double *n2 = (i + 2 < n) ? f + (i + 2) * ld : NULL;
        for (int64_t j = 0; j < m; ++j) {
            double x1 = n1 ? n1[j] : 0.0;
            double x2 = n2 ? n2[j] : 0.0;
            row[j] = row[j] - gamma[i] * x1 - delta[i] * x2;
        }
    }
}

int64_t oracle_penta_solve(int64_t n, int64_t m, int64_t ld, const double *a,
                           const double *b, const double *c, const double *d,
                           const double *e, double *f)
{
    if (n < 1) return 0;
    double *w = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    double *alpha = w, *beta = w + n, *gamma = w + 2 * n, *delta = w + 3 * n,
           *eps = w + 4 * n;
    int64_t bad = oracle_penta_factor(n, a, b, c, d, e, alpha, beta, gamma, delta, eps);
    if (bad < 0) oracle_penta_apply(n, m, ld, alpha, beta, gamma, delta, eps, f);
    free(w);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Periodic tridiagonal systems, Section 3.3 (Sherman-Morrison).
 * Row i reads a_i x_{(i-1) mod n} + b_i x_i + c_i x_{(i+1) mod n}: besides
 * the three bands the matrix has a_0 in its top-right corner and c_{n-1} in
 * its bottom-left corner.  It is split as A = A' + u v^T with
 *   u = (-b_0, 0, ..., 0, c_{n-1})^T,   v = (1, 0, ..., 0, -a_0 / b_0)^T.
 * u v^T puts -b_0 at (0,0), a_0 at (0,n-1), c_{n-1} at (n-1,0) and
 * -a_0 c_{n-1} / b_0 at (n-1,n-1), so A' is tridiagonal with the same bands
 * except A'_00 = 2 b_0 and A'_{n-1,n-1} = b_{n-1} + a_0 c_{n-1} / b_0; its
 * corners are zero (the paper's display of A' still shows them, which would
 * make A' + u v^T differ from A).  Then
 *   A' y = d,   A' z = u,   x = y - ((v.y) / (1 + v.z)) z,
 * with v.w = w_0 + v_{n-1} w_{n-1}, v_{n-1} = -a_0 / b_0.
 * Needs n >= 3 (for smaller n the corner entries fall on the bands).
 * Returns -1, or the row of a bad pivot of A', or n when 1 + v.z is zero or
 * not finite.  The interleaved layout and loop order are as above.
 */
int64_t oracle_tri_periodic_solve(int64_t n, int64_t m, int64_t ld,
                                  const double *a, const double *b,
                                  const double *c, double *d)
{
    if (n < 3) return 0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(4 * n));
    double *bp = w, *den = w + n, *chat = w + 2 * n, *z = w + 3 * n;
    const double vlast = -a[0] / b[0];
    for (int64_t i = 0; i < n; ++i) bp[i] = b[i];
    bp[0] = b[0] + b[0];
    bp[n - 1] = b[n - 1] + a[0] * c[n - 1] / b[0];
    int64_t bad = oracle_tri_factor(n, a, bp, c, den, chat);
    if (bad < 0) {
        for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
        z[0] = -b[0];
        z[n - 1] = c[n - 1];
        oracle_tri_apply(n, 1, 1, a, den, chat, z);
        const double vz1 = 1.0 + (z[0] + vlast * z[n - 1]);
        if (bad_pivot(vz1)) {
            bad = n;
        } else {
            oracle_tri_apply(n, m, ld, a, den, chat, d);
            for (int64_t j = 0; j < m; ++j) {
                const double s = (d[j] + vlast * d[(n - 1) * ld + j]) / vz1;
                for (int64_t i = 0; i < n; ++i) d[i * ld + j] = d[i * ld + j] - s * z[i];
            }
        }
    }
    free(w);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Crank-Nicolson time steps, Sections 3.2 and 4.2.  Both benchmark schemes
 * have the form A C^{n+1} = f with the explicit half f = (2I - A) C^n: for
 * diffusion A = (-s, 1 + 2s, -s) and f_i = s C_{i-1} + (1 - 2s) C_i
 * + s C_{i+1}; for hyperdiffusion A = (s, -4s, 1 + 6s, -4s, s) and f_i =
 * -s C_{i-2} + 4s C_{i-1} + (1 - 6s) C_i + 4s C_{i+1} - s C_{i+2}.  With
 * per-row bands the same operator is written with the matrix's own entries:
 *   f_i = 2 C_i - (A C)_i,
 * (A C)_i summed over the bands left to right, a term outside the matrix
 * being zero (or wrapping round for kind 13, the periodic tridiagonal).
 * Each step forms f from C, then solves A C = f with the routines above.
 * kind: 3, 5 or 13; bands as for the solves.  Returns -1, or the bad row.
 */
int64_t oracle_cn_steps(int kind, int64_t n, int64_t m, const double *bands,
                        double *C, int steps)
{
    const int nb = (kind == 13) ? 3 : kind;
    const int h = nb / 2;
    const double *a = bands, *b = bands + n, *c = bands + 2 * n;
    const double *d = bands + 3 * n, *e = bands + 4 * n;
    double *f = (double *)malloc(sizeof(double) * (size_t)(n * m));
    int64_t bad = -1;
    for (int s = 0; s < steps && bad < 0; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) {
                double ac = 0.0;
                for (int k = 0; k < nb; ++k) {
                    int64_t col = i + k - h;
                    if (kind == 13) col = (col + n) % n;
                    else if (col < 0 || col >= n) continue;
                    ac = ac + bands[k * n + i] * C[col * m + j];
                }
                f[i * m + j] = 2.0 * C[i * m + j] - ac;
            }
        for (int64_t t = 0; t < n * m; ++t) C[t] = f[t];
        if (kind == 3) bad = oracle_tri_solve(n, m, m, a, b, c, C);
        else if (kind == 5) bad = oracle_penta_solve(n, m, m, a, b, c, d, e, C);
        else bad = oracle_tri_periodic_solve(n, m, m, a, b, c, C);
    }
    free(f);
    return bad;
}

/* ---------------------------------------------------------------------------
 * One alternating-direction step on an ny x nx grid stored row-major,
 * grid[y*nx + x] (the 2-D use of batched solvers named in the introduction).
 * First every column is solved along y with the y-matrix: the columns are
 * already interleaved (unknown y of system x at y*nx + x).  Then every row is
 * solved along x with the x-matrix, walking the row directly (stride 1): no
 * transpose is involved on this side.
 */
int64_t oracle_adi_step(int64_t ny, int64_t nx, const double *ay,
                        const double *by, const double *cy, const double *ax,
                        const double *bx, const double *cx, double *grid)
{
    int64_t bad = oracle_tri_solve(ny, nx, nx, ay, by, cy, grid);
    if (bad >= 0) return bad;
    double *den = (double *)malloc(sizeof(double) * (size_t)nx);
    double *chat = (double *)malloc(sizeof(double) * (size_t)nx);
    bad = oracle_tri_factor(nx, ax, bx, cx, den, chat);
    if (bad < 0)
        for (int64_t y = 0; y < ny; ++y)
            oracle_tri_apply(nx, 1, 1, ax, den, chat, grid + y * nx);
    free(den);
    free(chat);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Multi-threaded drivers for the CPU baseline: the column range is cut into
 * one contiguous block per thread and each block runs the plain routines
 * above unchanged (same operations per system, so the result is identical
 * to the single-threaded call).  nthreads <= 0 uses the OpenMP default.
 */
static int64_t run_blocks(int kind, int64_t n, int64_t m, const double *a,
                          const double *b, const double *c, const double *d,
                          const double *e, double *rhs, int nthreads)
{
    int64_t bad = -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int64_t nb = nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t t = 0; t < nb; ++t) {
        int64_t j0 = m * t / nb, j1 = m * (t + 1) / nb;
        if (j1 <= j0) continue;
        int64_t r = (kind == 3)
                        ? oracle_tri_solve(n, j1 - j0, m, a, b, c, rhs + j0)
                        : oracle_penta_solve(n, j1 - j0, m, a, b, c, d, e, rhs + j0);
        if (r >= 0) {
#pragma omp critical
            bad = r;
        }
    }
    return bad;
}

int64_t oracle_tri_solve_mt(int64_t n, int64_t m, const double *a,
                            const double *b, const double *c, double *rhs,
                            int nthreads)
{
    return run_blocks(3, n, m, a, b, c, NULL, NULL, rhs, nthreads);
}

int64_t oracle_penta_solve_mt(int64_t n, int64_t m, const double *a,
                              const double *b, const double *c, const double *d,
                              const double *e, double *rhs, int nthreads)
{
    return run_blocks(5, n, m, a, b, c, d, e, rhs, nthreads);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
