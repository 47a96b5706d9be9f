/*
 * sko.c -- FP64 CPU oracle for the PDE signature kernel.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: it exists so that tests/, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct solver.  It shares no code, header or table with the
 * HIP kernels.
 *
 * Paper: Salvi, Cass, Foster, Lyons, Yang, "The Signature Kernel is the
 * solution of a Goursat PDE" (arXiv 2006.14794).
 *
 * What is computed (all in IEEE double, round to nearest):
 *   - Section 3.1, piecewise-linear paths: on each coarse cell D_pq the PDE
 *     coefficient is the constant <x_{p+1}-x_p, y_{q+1}-y_q>.
 *   - Definition "fintite_diff" (dyadic grid P_lambda): each coarse interval is
 *     split into 2^lambda equal parts.
 *   - Remark after eq. (explicit_finite_diff): on P_lambda the increment inner
 *     product of a fine cell is 2^{-2 lambda} times that of its coarse cell.
 *   - Eq. (explicit_finite_diff): the explicit scheme with boundary values 1,
 *     evaluated cell by cell in row-major order, literally
 *         K[i+1][j+1] = K[i+1][j] + K[i][j+1] - K[i][j]
 *                       + 0.5 * inc[i][j] * (K[i+1][j] + K[i][j+1]).
 *   - The gradient of the discrete solution with respect to the path points,
 *     obtained by reverse accumulation through the same loop (the paper does
 *     not give one; the discrete adjoint is the derivative of what the scheme
 *     computes, so it is pinned by finite differences of the forward solve).
 *
 * Indexing conventions (the paper swaps the grid ranges in the definition of
 * the scheme; here rows follow x and columns follow y): x has lx points and
 * m = lx-1 increments, y has ly points and n = ly-1 increments, the fine grid
 * has nodes (i,j) in [0, 2^lambda m] x [0, 2^lambda n].
 *
 * Points are row-major [len][d] doubles (the caller converts the float32
 * inputs exactly to double).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Coarse increment Gram (Section 3.1): G0[p][q] = sum_c dx_p[c] * dy_q[c],
 * with dx_p = x_{p+1} - x_p and dy_q = y_{q+1} - y_q; channels summed in order. */
void sko_increment_gram(const double *x, int64_t lx, const double *y, int64_t ly,
                        int32_t d, double *g0)
{
    int64_t m = lx - 1, n = ly - 1;
    for (int64_t p = 0; p < m; ++p) {
        for (int64_t q = 0; q < n; ++q) {
            double s = 0.0;
            for (int32_t c = 0; c < d; ++c) {
                double dx = x[(p + 1) * d + c] - x[p * d + c];
                double dy = y[(q + 1) * d + c] - y[q * d + c];
                s += dx * dy;
            }
            g0[p * n + q] = s;
        }
    }
}

/* Explicit scheme of eq. (explicit_finite_diff) on P_lambda.  Returns the
 * terminal value K[M][N].  If grid != NULL it receives all (M+1)*(N+1) nodes
 * row-major.  A path with a single point has no increments: the grid is the
 * boundary only and the value is 1 (boundary condition of eq. (PDE)). */
double sko_solve(const double *x, int64_t lx, const double *y, int64_t ly,
                 int32_t d, int32_t lam, double *grid)
{
    int64_t m = lx - 1, n = ly - 1;
    int64_t M = m << lam, N = n << lam;
    if (m <= 0 || n <= 0) {
        if (grid)
            for (int64_t k = 0; k < (M + 1) * (N + 1); ++k) grid[k] = 1.0;
        return 1.0;
    }
    double *g0 = (double *)malloc((size_t)(m * n) * sizeof(double));
    sko_increment_gram(x, lx, y, ly, d, g0);
    /* refined increment inner product: 2^{-2 lambda} of the coarse one */
    double refine = ldexp(1.0, -2 * lam);

    int own = (grid == NULL);
    double *prev, *cur;
    double *rows = NULL;
    if (own) {
        rows = (double *)malloc((size_t)(2 * (N + 1)) * sizeof(double));
        prev = rows;
        cur = rows + (N + 1);
    } else {
        prev = grid;
        cur = grid + (N + 1);
    }
    for (int64_t j = 0; j <= N; ++j) prev[j] = 1.0;    /* K(s_0, .) = 1 */
    for (int64_t i = 0; i < M; ++i) {
        cur[0] = 1.0;                                     /* K(., t_0) = 1 */
        const double *g0row = g0 + (i >> lam) * n;
        for (int64_t j = 0; j < N; ++j) {
            double inc = g0row[j >> lam] * refine;
            double A = cur[j], B = prev[j + 1], C = prev[j];
            cur[j + 1] = A + B - C + 0.5 * inc * (A + B);
        }
        if (own) {
            double *t = prev;
            prev = cur;
            cur = t;
        } else {
            prev = cur;
            cur = cur + (N + 1);
        }
    }
    double result = prev[N];
    free(rows);
    free(g0);
    return result;
}

/* The implicit scheme of the remark after eq. (explicit_finite_diff): the
 * double integral over a cell is estimated with all four corner values,
 *     K11 = K10 + K01 - K00 + (1/4) inc (K00 + K10 + K01 + K11),
 * which is linear in the unknown corner K11; solved for it cell by cell in the
 * same row-major order, on the same refined grid and coefficients as
 * sko_solve.  (A cell with inc = 4 has no solution: the division gives
 * +-inf or NaN, which then propagates.) */
double sko_solve_implicit(const double *x, int64_t lx, const double *y, int64_t ly,
                          int32_t d, int32_t lam, double *grid)
{
    int64_t m = lx - 1, n = ly - 1;
    int64_t M = m << lam, N = n << lam;
    if (m <= 0 || n <= 0) {
        if (grid)
            for (int64_t k = 0; k < (M + 1) * (N + 1); ++k) grid[k] = 1.0;
        return 1.0;
    }
    double *g0 = (double *)malloc((size_t)(m * n) * sizeof(double));
    sko_increment_gram(x, lx, y, ly, d, g0);
    double refine = ldexp(1.0, -2 * lam);
    double *all = (double *)malloc((size_t)((M + 1) * (N + 1)) * sizeof(double));
    for (int64_t j = 0; j <= N; ++j) all[j] = 1.0;
    for (int64_t i = 0; i < M; ++i) {
        double *prev = all + i * (N + 1), *cur = prev + (N + 1);
        cur[0] = 1.0;
        const double *g0row = g0 + (i >> lam) * n;
        for (int64_t j = 0; j < N; ++j) {
            double inc = g0row[j >> lam] * refine;
            double K10 = cur[j], K01 = prev[j + 1], K00 = prev[j];
            cur[j + 1] = (K10 + K01 - K00 + 0.25 * inc * (K00 + K10 + K01)) / (1.0 - 0.25 * inc);
        }
    }
    double result = all[M * (N + 1) + N];
    if (grid) memcpy(grid, all, (size_t)((M + 1) * (N + 1)) * sizeof(double));
    free(all);
    free(g0);
    return result;
}

/* Value and gradient of K[M][N] with respect to every point of x and y.
 * Reverse accumulation through the row-major loop of sko_solve: cells are
 * visited in exactly the reverse order, and each cell pushes the adjoint of
 * its output node to its three input nodes and to its coefficient.  dx, dy
 * (either may be NULL) receive [lx][d] and [ly][d] gradients (overwritten). */
double sko_solve_grad(const double *x, int64_t lx, const double *y, int64_t ly,
                      int32_t d, int32_t lam, double *dx, double *dy)
{
    int64_t m = lx - 1, n = ly - 1;
    if (dx) memset(dx, 0, (size_t)(lx * d) * sizeof(double));
    if (dy) memset(dy, 0, (size_t)(ly * d) * sizeof(double));
    if (m <= 0 || n <= 0) return 1.0;
    int64_t M = m << lam, N = n << lam;
    int64_t W = N + 1;
    double *K = (double *)malloc((size_t)((M + 1) * W) * sizeof(double));
    double *Kb = (double *)calloc((size_t)((M + 1) * W), sizeof(double));
    double *g0 = (double *)malloc((size_t)(m * n) * sizeof(double));
    double *g0b = (double *)calloc((size_t)(m * n), sizeof(double));
    double value = sko_solve(x, lx, y, ly, d, lam, K);
    sko_increment_gram(x, lx, y, ly, d, g0);
    double refine = ldexp(1.0, -2 * lam);

    Kb[M * W + N] = 1.0;
    for (int64_t i = M - 1; i >= 0; --i) {
        for (int64_t j = N - 1; j >= 0; --j) {
            double a = Kb[(i + 1) * W + (j + 1)];
            if (a == 0.0) continue;
            int64_t p = i >> lam, q = j >> lam;
            double inc = g0[p * n + q] * refine;
            double A = K[(i + 1) * W + j], B = K[i * W + (j + 1)];
            /* d out / dA = d out / dB = 1 + inc/2, d out / dC = -1 */
            Kb[(i + 1) * W + j] += a + a * 0.5 * inc;
            Kb[i * W + (j + 1)] += a + a * 0.5 * inc;
            Kb[i * W + j] -= a;
            /* d out / d G0[p][q] = 0.5 * 2^{-2 lambda} * (A + B) */
            g0b[p * n + q] += a * 0.5 * refine * (A + B);
        }
    }
    /* G0[p][q] = <dx_p, dy_q>: chain rule into the increments, then into the
     * points through dx_p = x_{p+1} - x_p. */
    for (int64_t p = 0; p < m; ++p) {
        for (int64_t q = 0; q < n; ++q) {
            double gb = g0b[p * n + q];
            for (int32_t c = 0; c < d; ++c) {
                double ix = x[(p + 1) * d + c] - x[p * d + c];
                double iy = y[(q + 1) * d + c] - y[q * d + c];
                if (dx) {
                    dx[(p + 1) * d + c] += gb * iy;
                    dx[p * d + c] -= gb * iy;
                }
                if (dy) {
                    dy[(q + 1) * d + c] += gb * ix;
                    dy[q * d + c] -= gb * ix;
                }
            }
        }
    }
    free(K);
    free(Kb);
    free(g0);
    free(g0b);
    return value;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    return nthreads;
#else
    (void)nthreads;
    return 1;
#endif
}

/* Independent pairs: out[k] = k(x_k, y_k).  Paths are ragged: path k of xs
 * spans points [xoff[k], xoff[k+1]). */
void sko_pairs(const double *xs, const int64_t *xoff, const double *ys,
               const int64_t *yoff, int64_t npairs, int32_t d, int32_t lam,
               double *out, int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t k = 0; k < npairs; ++k) {
        out[k] = sko_solve(xs + xoff[k] * d, xoff[k + 1] - xoff[k],
                           ys + yoff[k] * d, yoff[k + 1] - yoff[k], d, lam, NULL);
    }
}

/* Independent pairs with the implicit scheme. */
void sko_pairs_implicit(const double *xs, const int64_t *xoff, const double *ys,
                        const int64_t *yoff, int64_t npairs, int32_t d, int32_t lam,
                        double *out, int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t k = 0; k < npairs; ++k) {
        out[k] = sko_solve_implicit(xs + xoff[k] * d, xoff[k + 1] - xoff[k],
                                    ys + yoff[k] * d, yoff[k + 1] - yoff[k], d, lam, NULL);
    }
}

/* Gram matrix: K[a*ny + b] = k(X_a, Y_b). */
void sko_gram(const double *X, const int64_t *xoff, int64_t nx, const double *Y,
              const int64_t *yoff, int64_t ny, int32_t d, int32_t lam, double *K,
              int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t ab = 0; ab < nx * ny; ++ab) {
        int64_t a = ab / ny, b = ab % ny;
        K[ab] = sko_solve(X + xoff[a] * d, xoff[a + 1] - xoff[a], Y + yoff[b] * d,
                          yoff[b + 1] - yoff[b], d, lam, NULL);
    }
}

/* Backward of the Gram matrix for an upstream weight dK[a][b]:
 *   dX[a] = sum_b dK[a][b] * grad_{X_a} k(X_a, Y_b),
 *   dY[b] = sum_a dK[a][b] * grad_{Y_b} k(X_a, Y_b).
 * dX / dY are ragged like X / Y ([total points][d]); either may be NULL. */
void sko_gram_backward(const double *X, const int64_t *xoff, int64_t nx,
                       const double *Y, const int64_t *yoff, int64_t ny, int32_t d,
                       int32_t lam, const double *dK, double *dX, double *dY,
                       int nthreads)
{
    int nt = set_threads(nthreads);
    int64_t totx = xoff[nx], toty = yoff[ny];
    int64_t maxlx = 1, maxly = 1;
    for (int64_t a = 0; a < nx; ++a)
        if (xoff[a + 1] - xoff[a] > maxlx) maxlx = xoff[a + 1] - xoff[a];
    for (int64_t b = 0; b < ny; ++b)
        if (yoff[b + 1] - yoff[b] > maxly) maxly = yoff[b + 1] - yoff[b];
    if (dX) memset(dX, 0, (size_t)(totx * d) * sizeof(double));
    if (dY) memset(dY, 0, (size_t)(toty * d) * sizeof(double));
    /* one private dY accumulator per thread, reduced at the end */
    double *dYp = NULL;
    if (dY) dYp = (double *)calloc((size_t)(nt * toty * d), sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gx = (double *)malloc((size_t)(maxlx * d) * sizeof(double));
        double *gy = (double *)malloc((size_t)(maxly * d) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t a = 0; a < nx; ++a) {
            int64_t lx = xoff[a + 1] - xoff[a];
            for (int64_t b = 0; b < ny; ++b) {
                double w = dK[a * ny + b];
                if (w == 0.0) continue;
                int64_t ly = yoff[b + 1] - yoff[b];
                sko_solve_grad(X + xoff[a] * d, lx, Y + yoff[b] * d, ly, d, lam,
                               dX ? gx : NULL, dY ? gy : NULL);
                if (dX)
                    for (int64_t k = 0; k < lx * d; ++k) dX[xoff[a] * d + k] += w * gx[k];
                if (dY) {
                    double *acc = dYp + (int64_t)tid * toty * d + yoff[b] * d;
                    for (int64_t k = 0; k < ly * d; ++k) acc[k] += w * gy[k];
                }
            }
        }
        free(gx);
        free(gy);
    }
    if (dY) {
        for (int t = 0; t < nt; ++t)
            for (int64_t k = 0; k < toty * d; ++k) dY[k] += dYp[(int64_t)t * toty * d + k];
        free(dYp);
    }
}

/* ------------------------------------------------------------------------
 * Static-kernel lift (Section "The signature PDE kernel from static kernels on
 * the ambient space", eq. (PDE_lifted) and the finite-difference form that
 * follows it).  The lifted paths X = phi(x), Y = psi(y) have, on the coarse
 * cell between nodes p, p+1 of x and q, q+1 of y, the constant coefficient
 *     (X_{p+1} - X_p, Y_{q+1} - Y_q)
 *       = kappa(x_{p+1}, y_{q+1}) - kappa(x_p, y_{q+1})
 *         - kappa(x_{p+1}, y_q) + kappa(x_p, y_q),
 * a second difference of the static-kernel matrix kappa(x_i, y_j).  (The
 * printed formula has kappa(x_{s-1}, x_t) in its second term; by bilinearity
 * of the pairing the term is kappa(x_{s-1}, y_t).)  The explicit or implicit
 * scheme then runs on P_lambda exactly as for the plain kernel, with this
 * coefficient in place of <dx_p, dy_q>.
 * ---------------------------------------------------------------------- */

/* kmat[i][j] = exp(-|x_i - y_j|^2 / (2 sigma^2)), the Gaussian (RBF) static
 * kernel with bandwidth sigma; channel differences summed in order. */
void sko_static_rbf(const double *x, int64_t lx, const double *y, int64_t ly, int32_t d,
                    double sigma, double *kmat)
{
    double inv = 1.0 / (2.0 * sigma * sigma);
    for (int64_t i = 0; i < lx; ++i) {
        for (int64_t j = 0; j < ly; ++j) {
            double r = 0.0;
            for (int32_t c = 0; c < d; ++c) {
                double t = x[i * d + c] - y[j * d + c];
                r += t * t;
            }
            kmat[i * ly + j] = exp(-r * inv);
        }
    }
}

/* kmat[i][j] = <x_i, y_j>, the linear static kernel (its lift is the path
 * itself, so its lifted kernel is the plain one). */
void sko_static_linear(const double *x, int64_t lx, const double *y, int64_t ly, int32_t d,
                       double *kmat)
{
    for (int64_t i = 0; i < lx; ++i) {
        for (int64_t j = 0; j < ly; ++j) {
            double s = 0.0;
            for (int32_t c = 0; c < d; ++c) s += x[i * d + c] * y[j * d + c];
            kmat[i * ly + j] = s;
        }
    }
}

/* coef[p][q] = second difference of kmat ([lx][ly]) over the cell (p, q). */
void sko_lifted_coefficients(const double *kmat, int64_t lx, int64_t ly, double *coef)
{
    int64_t m = lx - 1, n = ly - 1;
    for (int64_t p = 0; p < m; ++p)
        for (int64_t q = 0; q < n; ++q)
            coef[p * n + q] = kmat[(p + 1) * ly + (q + 1)] - kmat[p * ly + (q + 1)]
                              - kmat[(p + 1) * ly + q] + kmat[p * ly + q];
}

/* The scheme of eq. (explicit_finite_diff) (implicit == 0) or of the remark
 * after it (implicit != 0) on P_lambda, driven by a given coarse coefficient
 * matrix coef [m][n] in place of the increment Gram; each fine cell takes
 * 2^{-2 lambda} of its coarse cell's coefficient.  Returns K[M][N]; grid, if
 * not NULL, receives all (M+1)*(N+1) nodes row-major. */
double sko_solve_coef(const double *coef, int64_t m, int64_t n, int32_t lam, int32_t implicit,
                      double *grid)
{
    int64_t M = m << lam, N = n << lam;
    if (m <= 0 || n <= 0) {
        if (grid)
            for (int64_t k = 0; k < (M + 1) * (N + 1); ++k) grid[k] = 1.0;
        return 1.0;
    }
    double refine = ldexp(1.0, -2 * lam);
    double *all = (double *)malloc((size_t)((M + 1) * (N + 1)) * sizeof(double));
    for (int64_t j = 0; j <= N; ++j) all[j] = 1.0;
    for (int64_t i = 0; i < M; ++i) {
        double *prev = all + i * (N + 1), *cur = prev + (N + 1);
        cur[0] = 1.0;
        const double *row = coef + (i >> lam) * n;
        for (int64_t j = 0; j < N; ++j) {
            double inc = row[j >> lam] * refine;
            double K10 = cur[j], K01 = prev[j + 1], K00 = prev[j];
            if (implicit)
                cur[j + 1] = (K10 + K01 - K00 + 0.25 * inc * (K00 + K10 + K01))
                             / (1.0 - 0.25 * inc);
            else
                cur[j + 1] = K10 + K01 - K00 + 0.5 * inc * (K10 + K01);
        }
    }
    double result = all[M * (N + 1) + N];
    if (grid) memcpy(grid, all, (size_t)((M + 1) * (N + 1)) * sizeof(double));
    free(all);
    return result;
}

/* The RBF-lifted kernel of one pair: static matrix, second difference, scheme. */
double sko_solve_rbf(const double *x, int64_t lx, const double *y, int64_t ly, int32_t d,
                     double sigma, int32_t lam, int32_t implicit)
{
    if (lx <= 1 || ly <= 1) return 1.0;
    double *kmat = (double *)malloc((size_t)(lx * ly) * sizeof(double));
    double *coef = (double *)malloc((size_t)((lx - 1) * (ly - 1)) * sizeof(double));
    sko_static_rbf(x, lx, y, ly, d, sigma, kmat);
    sko_lifted_coefficients(kmat, lx, ly, coef);
    double v = sko_solve_coef(coef, lx - 1, ly - 1, lam, implicit, NULL);
    free(coef);
    free(kmat);
    return v;
}

/* RBF-lifted kernels of independent pairs (gram == 0: out[k] = k(x_k, y_k))
 * or of a Gram matrix (gram != 0: out[a*ny + b] = k(X_a, Y_b)). */
void sko_lifted_rbf_batch(const double *X, const int64_t *xoff, int64_t nx, const double *Y,
                          const int64_t *yoff, int64_t ny, int32_t d, int32_t lam,
                          double sigma, int32_t implicit, int32_t gram, double *out,
                          int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
    int64_t total = gram ? nx * ny : nx;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t k = 0; k < total; ++k) {
        int64_t a = gram ? k / ny : k, b = gram ? k % ny : k;
        out[k] = sko_solve_rbf(X + xoff[a] * d, xoff[a + 1] - xoff[a], Y + yoff[b] * d,
                               yoff[b + 1] - yoff[b], d, sigma, lam, implicit);
    }
}

int sko_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
