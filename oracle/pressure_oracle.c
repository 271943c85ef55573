/*
 * Plain FP64 CPU oracle for the direct FFT pressure solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU path is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links, loads or calls it, and it shares no code,
 * header or table with the GPU sources.
 *
 * What it computes (paper, Section 2.1 "Direct FFT"): a forward Fourier
 * transform of every horizontal level turns the 3D Poisson-like problem
 * into one independent vertical ODE per horizontal wavenumber, each ODE is
 * solved with a tridiagonal solver that walks up and down its column, and a
 * backward transform returns the pressure.  Because the method is direct it
 * reaches the exact solution of the discrete system (Section 3, first
 * paragraph), so this oracle is that exact solution written out:
 *
 *   A = dxx + dyy + V     on a grid i<nx, j<ny, k<nz, array b[k][j][i]
 *   dxx, dyy : periodic 3-point second differences (lateral periodicity,
 *              Section 2.2 notes the FFT solver imposes it)
 *   (V p)_k  = [ f_{k+1/2}(p_{k+1}-p_k) - f_{k-1/2}(p_k-p_{k-1}) ] / D_k
 *              f_{k+1/2} = rho_{k+1/2} / h_{k+1/2},  rho_{k+1/2} the mean of
 *              the two adjacent rho, h_{k+1/2} the mean of the two adjacent
 *              cell thicknesses, D_k = rho_k dz_k, zero flux at bottom/top.
 *   p solves the bordered system [[A,1],[1^T,0]] [p;mu] = [b;0]:
 *   A p = b - mu*1 with mu the D-weighted mean of b, and sum(p) = 0.
 *
 * The discretisation details (finite-difference eigenvalues, cell-centred
 * stretched levels, face density, Neumann ends, the gauge of the singular
 * mean mode) are readings of a paper that only names the equation; each is
 * listed with its reason in the design notes.
 *
 * Steps, in the paper's order (Section 2.1):
 *   1. compatibility projection of b (mean mode),
 *   2. forward DFT of every level, x then y ("one dimension for all data,
 *      then the next"), by direct summation with exactly reduced angles,
 *   3. one tridiagonal solve per wavenumber column (kx,ky) != (0,0), and the
 *      singular (0,0) column by two prefix sums plus the zero-mean gauge
 *      (formed from the level sums in extended precision, see
 *      mean_column_ext),
 *   4. backward DFT with 1/(nx*ny), Hermitian completion, real part.
 * Adjoint and density-gradient routines follow the same definitions.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 3

/* ---------------------------------------------------------------- tables */

/* Vertical coefficients: f[0] = f_{-1/2} = 0, f[k] = f_{k-1/2} for
 * 1 <= k <= nz-1, f[nz] = f_{nz-1/2} = 0; D[k] = rho_k dz_k. */
static void vertical_coefficients(int nz, const double *dz, const double *rho,
                                  double *f, double *D)
{
    f[0] = 0.0;
    f[nz] = 0.0;
    for (int k = 0; k + 1 < nz; ++k) {
        double h = 0.5 * (dz[k] + dz[k + 1]);
        double rf = 0.5 * (rho[k] + rho[k + 1]);
        f[k + 1] = rf / h;
    }
    for (int k = 0; k < nz; ++k)
        D[k] = rho[k] * dz[k];
}

/* Eigenvalue magnitude of the periodic 3-point second difference for
 * wavenumber m on n points with spacing d: 4 sin^2(pi m / n) / d^2. */
static double lateral_eigen(int m, int n, double d)
{
    int mm = m % n;
    if (mm > n - mm)
        mm = n - mm;
    double sn = sin(M_PI * (double)mm / (double)n);
    return 4.0 * sn * sn / (d * d);
}

/* cos/sin of 2 pi m / n for m in [0, n); the caller reduces the integer
 * product index*wavenumber modulo n before the lookup, so no large angle is
 * ever formed. */
static int unit_roots(int n, double **c, double **s)
{
    *c = (double *)malloc(sizeof(double) * (size_t)n);
    *s = (double *)malloc(sizeof(double) * (size_t)n);
    if (!*c || !*s) {
        free(*c);
        free(*s);
        return OR_ENOMEM;
    }
    for (int m = 0; m < n; ++m) {
        double a = 2.0 * M_PI * (double)m / (double)n;
        (*c)[m] = cos(a);
        (*s)[m] = sin(a);
    }
    return OR_OK;
}

static int check_grid(int nx, int ny, int nz, double dx, double dy,
                      const double *dz, const double *rho)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(dy > 0) || !dz || !rho)
        return OR_EINVAL;
    for (int k = 0; k < nz; ++k)
        if (!(dz[k] > 0) || !(rho[k] > 0))
            return OR_EINVAL;
    return OR_OK;
}

/* -------------------------------------------------------------- the DFTs */

/* Forward 2D DFT of every level, unnormalised:
 *   out[k][ky][kx] = sum_{j,i} in[k][j][i] exp(-2 pi i (kx i/nx + ky j/ny))
 * for kx in [0, nx/2] (the half spectrum of a real field) and ky in [0,ny).
 * Separable: x first, then y.  out is complex interleaved (re, im),
 * shape [nz][ny][nx/2+1][2]. */
int oracle_dft2_forward(int nx, int ny, int nz, const double *in, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out)
        return OR_EINVAL;
    const int hx = nx / 2 + 1;
    double *cx, *sx, *cy, *sy;
    if (unit_roots(nx, &cx, &sx))
        return OR_ENOMEM;
    if (unit_roots(ny, &cy, &sy)) {
        free(cx);
        free(sx);
        return OR_ENOMEM;
    }
    double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)nz * ny * hx);
    if (!tmp) {
        free(cx); free(sx); free(cy); free(sy);
        return OR_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        /* x direction: every row of the level */
        for (int j = 0; j < ny; ++j) {
            const double *row = in + ((size_t)k * ny + j) * nx;
            double *t = tmp + 2 * ((size_t)k * ny + j) * hx;
            for (int kx = 0; kx < hx; ++kx) {
                double re = 0.0, im = 0.0;
                for (int i = 0; i < nx; ++i) {
                    int m = (int)(((long long)i * kx) % nx);
                    re += row[i] * cx[m];
                    im -= row[i] * sx[m];
                }
                t[2 * kx] = re;
                t[2 * kx + 1] = im;
            }
        }
        /* y direction: every half-spectrum column of the level */
        for (int kx = 0; kx < hx; ++kx) {
            for (int ky = 0; ky < ny; ++ky) {
                double re = 0.0, im = 0.0;
                for (int j = 0; j < ny; ++j) {
                    int m = (int)(((long long)j * ky) % ny);
                    const double *t = tmp + 2 * (((size_t)k * ny + j) * hx + kx);
                    /* (tr + i ti)(c - i s) */
                    re += t[0] * cy[m] + t[1] * sy[m];
                    im += t[1] * cy[m] - t[0] * sy[m];
                }
                double *o = out + 2 * (((size_t)k * ny + ky) * hx + kx);
                o[0] = re;
                o[1] = im;
            }
        }
    }
    free(tmp);
    free(cx); free(sx); free(cy); free(sy);
    return OR_OK;
}

/* Backward 2D DFT with the 1/(nx*ny) factor.  in is a half spectrum
 * [nz][ny][nx/2+1][2]; the missing half is completed from Hermitian
 * symmetry, X(nx-kx, ky) = conj(X(kx, (ny-ky) mod ny)), and the real part of
 * the result is returned in out[nz][ny][nx]. */
int oracle_dft2_inverse(int nx, int ny, int nz, const double *in, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !in || !out)
        return OR_EINVAL;
    const int hx = nx / 2 + 1;
    double *cx, *sx, *cy, *sy;
    if (unit_roots(nx, &cx, &sx))
        return OR_ENOMEM;
    if (unit_roots(ny, &cy, &sy)) {
        free(cx); free(sx);
        return OR_ENOMEM;
    }
    double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)nz * ny * hx);
    if (!tmp) {
        free(cx); free(sx); free(cy); free(sy);
        return OR_ENOMEM;
    }
    const double scale = 1.0 / ((double)nx * (double)ny);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        /* y direction first (backward): q[j][kx] = sum_ky X[ky][kx] e^{+} */
        for (int kx = 0; kx < hx; ++kx) {
            for (int j = 0; j < ny; ++j) {
                double re = 0.0, im = 0.0;
                for (int ky = 0; ky < ny; ++ky) {
                    int m = (int)(((long long)j * ky) % ny);
                    const double *x = in + 2 * (((size_t)k * ny + ky) * hx + kx);
                    /* (xr + i xi)(c + i s) */
                    re += x[0] * cy[m] - x[1] * sy[m];
                    im += x[1] * cy[m] + x[0] * sy[m];
                }
                double *t = tmp + 2 * (((size_t)k * ny + j) * hx + kx);
                t[0] = re;
                t[1] = im;
            }
        }
        /* x direction over the full, Hermitian-completed row */
        for (int j = 0; j < ny; ++j) {
            const double *t = tmp + 2 * ((size_t)k * ny + j) * hx;
            double *row = out + ((size_t)k * ny + j) * nx;
            for (int i = 0; i < nx; ++i) {
                double re = 0.0;
                for (int kx = 0; kx < nx; ++kx) {
                    double qr, qi;
                    if (kx < hx) {
                        qr = t[2 * kx];
                        qi = t[2 * kx + 1];
                    } else {
                        qr = t[2 * (nx - kx)];
                        qi = -t[2 * (nx - kx) + 1];
                    }
                    int m = (int)(((long long)i * kx) % nx);
                    re += qr * cx[m] - qi * sx[m];
                }
                row[i] = re * scale;
            }
        }
    }
    free(tmp);
    free(cx); free(sx); free(cy); free(sy);
    return OR_OK;
}

/* ------------------------------------------------------ the column solves */

/* One vertical ODE of the transformed problem (Section 2.1: after the
 * forward transform each column is an independent tridiagonal system).
 * Solves T x = r with T = -s I + V for one column with lateral eigenvalue
 * magnitude s > 0.  Multiplying by -D makes the matrix
 *   tridiag(-f_{k-1/2},  f_{k-1/2} + f_{k+1/2} + s D_k,  -f_{k+1/2}),
 * symmetric and diagonally dominant, with right-hand side -D_k r_k.
 * Thomas elimination is written in dominance-excess form: the pivot is
 * u_k = e_k + f_{k+1/2} with e_0 = s D_0 and
 * e_k = s D_k + f_{k-1/2} e_{k-1} / u_{k-1}, so every pivot is built from
 * positive terms only.  Real and imaginary parts share the pivots.
 * rhs_is_scaled != 0 means r already carries the -D_k factor.
 * work must hold 2*nz doubles. */
static void column_solve(int nz, const double *f, const double *D, double s,
                         const double *r_re, const double *r_im,
                         int rhs_is_scaled, double *x_re, double *x_im,
                         double *work)
{
    double *u = work;
    double *y_re = x_re, *y_im = x_im; /* forward values stored in place */
    double e_prev = 0.0, u_prev = 1.0;
    for (int k = 0; k < nz; ++k) {
        double e = s * D[k] + (k > 0 ? f[k] * e_prev / u_prev : 0.0);
        double uk = e + f[k + 1];
        double sc = rhs_is_scaled ? 1.0 : -D[k];
        double yr = sc * r_re[k], yi = sc * r_im[k];
        if (k > 0) {
            double c = f[k] / u_prev;
            yr += c * y_re[k - 1];
            yi += c * y_im[k - 1];
        }
        y_re[k] = yr;
        y_im[k] = yi;
        u[k] = uk;
        e_prev = e;
        u_prev = uk;
    }
    for (int k = nz - 1; k >= 0; --k) {
        double nr = y_re[k], ni = y_im[k];
        if (k + 1 < nz) {
            nr += f[k + 1] * x_re[k + 1];
            ni += f[k + 1] * x_im[k + 1];
        }
        x_re[k] = nr / u[k];
        x_im[k] = ni / u[k];
    }
}

/* Exposed for stage tests: solve one column as above, r not yet scaled. */
int oracle_column_solve(int nz, const double *dz, const double *rho, double s,
                        const double *r_re, const double *r_im,
                        double *x_re, double *x_im)
{
    if (nz < 1 || !(s > 0) || !dz || !rho || !r_re || !r_im || !x_re || !x_im)
        return OR_EINVAL;
    double *f = (double *)malloc(sizeof(double) * (size_t)(3 * nz + 1));
    double *work = (double *)malloc(sizeof(double) * 2 * (size_t)nz);
    if (!f || !work) {
        free(f); free(work);
        return OR_ENOMEM;
    }
    double *D = f + nz + 1;
    vertical_coefficients(nz, dz, rho, f, D);
    column_solve(nz, f, D, s, r_re, r_im, 0, x_re, x_im, work);
    free(f);
    free(work);
    return OR_OK;
}

/* The singular (0,0) column: V x = c, where sum_k D_k c_k = 0 after the
 * compatibility projection.  Zero flux at the bottom fixes every face
 * flux as a prefix sum, F_{k+1/2} = sum_{j<=k} D_j c_j, and each level
 * difference follows as x_{k+1} - x_k = F_{k+1/2} / f_{k+1/2}.  The result
 * is defined up to a constant; the caller applies the gauge. */
static void mean_column(int nz, const double *f, const double *D,
                        const double *c_re, const double *c_im,
                        double *x_re, double *x_im)
{
    double Fr = 0.0, Fi = 0.0;
    x_re[0] = 0.0;
    x_im[0] = 0.0;
    for (int k = 0; k + 1 < nz; ++k) {
        Fr += D[k] * c_re[k];
        Fi += D[k] * c_im[k];
        x_re[k + 1] = x_re[k] + Fr / f[k + 1];
        x_im[k + 1] = x_im[k] + Fi / f[k + 1];
    }
}

/* The (0,0) column from the level sums of the input, in extended precision
 * (long double), written over spec[k][0][0].  The (0,0) coefficient of
 * level k of the projected right-hand side is S_k - N m, N = nx ny, with
 * S_k the level sum and m the projection's mean (forward: the D-weighted
 * mean of b; adjoint: the plain mean of w).  Forward: V x = that column by
 * the flux prefix sums of mean_column, zero plain mean over levels.
 * Adjoint: V z = D^{-1} (that column), sum_k D_k z_k = 0, output D_k z_k.
 * The prefix sums are divided by f_{k+1/2}, which is small near the top of
 * a tall stretched grid, so rounding in them is amplified there; carried in
 * extended precision, the oracle's own error stays far below the parity
 * bars.  Same steps as the FP64 path for the other columns. */
static int mean_column_ext(int nx, int ny, int nz, const double *f, const double *D,
                           const double *in, int adjoint, double *spec)
{
    const int hx = nx / 2 + 1;
    const size_t nxy = (size_t)nx * ny;
    long double *S = (long double *)malloc(sizeof(long double) * 2 * (size_t)nz);
    if (!S)
        return OR_ENOMEM;
    long double *x = S + nz;
    long double num = 0.0L, den = 0.0L, tot = 0.0L;
    for (int k = 0; k < nz; ++k) {
        long double acc = 0.0L;
        const double *lv = in + (size_t)k * nxy;
        for (size_t q = 0; q < nxy; ++q)
            acc += (long double)lv[q];
        S[k] = acc;
        num += (long double)D[k] * acc;
        den += (long double)D[k];
        tot += acc;
    }
    const long double N = (long double)nxy;
    const long double m = adjoint ? tot / (N * (long double)nz) : num / (N * den);
    long double F = 0.0L;
    x[0] = 0.0L;
    for (int k = 0; k + 1 < nz; ++k) {
        long double c = S[k] - N * m;
        if (adjoint)
            c /= (long double)D[k];
        F += (long double)D[k] * c;
        x[k + 1] = x[k] + F / (long double)f[k + 1];
    }
    long double g = 0.0L, w = 0.0L;
    for (int k = 0; k < nz; ++k) {
        long double wk = adjoint ? (long double)D[k] : 1.0L;
        g += wk * x[k];
        w += wk;
    }
    for (int k = 0; k < nz; ++k) {
        long double v = x[k] - g / w;
        if (adjoint)
            v *= (long double)D[k];
        double *e = spec + 2 * (((size_t)k * ny) * hx);
        e[0] = (double)v;
        e[1] = 0.0;
    }
    free(S);
    return OR_OK;
}

/* Shared driver for forward and adjoint spectral solves over the half
 * spectrum spec[nz][ny][hx][2], in place.  Forward (adjoint == 0):
 * x = T^{-1} b-hat per column, mean column by prefix sums, gauge: zero plain
 * mean over levels.  Adjoint (adjoint != 0): column systems with right-hand
 * side -w-hat (no D factor) and output multiplied by D_k; mean column by the
 * same prefix sums with the D-weighted gauge, then multiplied by D_k. */
static int spectral_solve(int nx, int ny, int nz, double dx, double dy,
                          const double *f, const double *D, double *spec,
                          int adjoint)
{
    const int hx = nx / 2 + 1;
    int err = OR_OK;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 8 * (size_t)nz);
        if (!buf) {
#pragma omp atomic write
            err = OR_ENOMEM;
        } else {
            double *rr = buf, *ri = buf + nz, *xr = buf + 2 * nz,
                   *xi = buf + 3 * nz, *work = buf + 4 * nz;
#pragma omp for schedule(dynamic, 16)
            for (int col = 0; col < ny * hx; ++col) {
                int ky = col / hx, kx = col % hx;
                for (int k = 0; k < nz; ++k) {
                    const double *v = spec + 2 * (((size_t)k * ny + ky) * hx + kx);
                    rr[k] = v[0];
                    ri[k] = v[1];
                }
                if (kx == 0 && ky == 0) {
                    if (adjoint) { /* V z = D^{-1} w-hat on the mean column */
                        for (int k = 0; k < nz; ++k) {
                            rr[k] /= D[k];
                            ri[k] /= D[k];
                        }
                    }
                    mean_column(nz, f, D, rr, ri, xr, xi);
                    double gr = 0.0, gi = 0.0, w = 0.0;
                    for (int k = 0; k < nz; ++k) {
                        double wk = adjoint ? D[k] : 1.0;
                        gr += wk * xr[k];
                        gi += wk * xi[k];
                        w += wk;
                    }
                    for (int k = 0; k < nz; ++k) {
                        xr[k] -= gr / w;
                        xi[k] -= gi / w;
                    }
                } else {
                    double s = lateral_eigen(kx, nx, dx) + lateral_eigen(ky, ny, dy);
                    if (adjoint) {
                        for (int k = 0; k < nz; ++k) {
                            rr[k] = -rr[k];
                            ri[k] = -ri[k];
                        }
                    }
                    column_solve(nz, f, D, s, rr, ri, adjoint, xr, xi, work);
                }
                for (int k = 0; k < nz; ++k) {
                    double m = adjoint ? D[k] : 1.0;
                    double *v = spec + 2 * (((size_t)k * ny + ky) * hx + kx);
                    v[0] = m * xr[k];
                    v[1] = m * xi[k];
                }
            }
            free(buf);
        }
    }
    return err;
}

/* ----------------------------------------------------------- public API */

/* Forward solve: p = S b, the p-block of [[A,1],[1^T,0]][p;mu] = [b;0].
 * All arrays [nz][ny][nx], host memory, FP64. */
int oracle_solve(int nx, int ny, int nz, double dx, double dy,
                 const double *dz, const double *rho, const double *b,
                 double *p)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !b || !p)
        return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    const int hx = nx / 2 + 1;
    double *f = (double *)malloc(sizeof(double) * (size_t)(2 * nz + 1));
    double *bp = (double *)malloc(sizeof(double) * n);
    double *spec = (double *)malloc(sizeof(double) * 2 * (size_t)nz * ny * hx);
    if (!f || !bp || !spec) {
        free(f); free(bp); free(spec);
        return OR_ENOMEM;
    }
    double *D = f + nz + 1;
    vertical_coefficients(nz, dz, rho, f, D);

    /* 1. compatibility: mu = sum_k D_k S_k / (nx ny sum_k D_k) */
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nz; ++k) {
        double S = 0.0;
        const double *lv = b + (size_t)k * nx * ny;
        for (size_t q = 0; q < (size_t)nx * ny; ++q)
            S += lv[q];
        num += D[k] * S;
        den += D[k];
    }
    double mu = num / ((double)nx * (double)ny * den);
    for (size_t q = 0; q < n; ++q)
        bp[q] = b[q] - mu;

    /* 2-4. transform, column solves, back-transform */
    err = oracle_dft2_forward(nx, ny, nz, bp, spec);
    if (!err)
        err = spectral_solve(nx, ny, nz, dx, dy, f, D, spec, 0);
    if (!err)
        err = mean_column_ext(nx, ny, nz, f, D, b, 0, spec);
    if (!err)
        err = oracle_dft2_inverse(nx, ny, nz, spec, p);
    free(f); free(bp); free(spec);
    return err;
}

/* Adjoint solve: lam = S^T w, the lambda-block of
 * [[A^T,1],[1^T,0]][lam;nu] = [w;0].  Since D A is symmetric,
 * A^T = D A D^{-1}: lam = D z with A z = D^{-1}(w - mean(w)) and
 * sum_k D_k zbar_k = 0 on the level means. */
int oracle_solve_adjoint(int nx, int ny, int nz, double dx, double dy,
                         const double *dz, const double *rho, const double *w,
                         double *lam)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !w || !lam)
        return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    const int hx = nx / 2 + 1;
    double *f = (double *)malloc(sizeof(double) * (size_t)(2 * nz + 1));
    double *wp = (double *)malloc(sizeof(double) * n);
    double *spec = (double *)malloc(sizeof(double) * 2 * (size_t)nz * ny * hx);
    if (!f || !wp || !spec) {
        free(f); free(wp); free(spec);
        return OR_ENOMEM;
    }
    double *D = f + nz + 1;
    vertical_coefficients(nz, dz, rho, f, D);
    double mean = 0.0;
    for (size_t q = 0; q < n; ++q)
        mean += w[q];
    mean /= (double)n;
    for (size_t q = 0; q < n; ++q)
        wp[q] = w[q] - mean;
    err = oracle_dft2_forward(nx, ny, nz, wp, spec);
    if (!err)
        err = spectral_solve(nx, ny, nz, dx, dy, f, D, spec, 1);
    if (!err)
        err = mean_column_ext(nx, ny, nz, f, D, w, 1, spec);
    if (!err)
        err = oracle_dft2_inverse(nx, ny, nz, spec, lam);
    free(f); free(wp); free(spec);
    return err;
}

/* The two dynamical-core steps either side of the solve (Section 1: the
 * source terms feed the pressure solve, whose result corrects the flow).
 * Velocities on the staggered (C) grid, arrays [nz][ny][nx]: u[k][j][i] at
 * the x-face between cells i-1 and i, v[k][j][i] at the y-face between rows
 * j-1 and j, w[k][j][i] at the face between levels k-1 and k (w of level 0
 * is the bottom boundary face, zero flux, never used).
 * Divergence (anelastic form, whose composition with the gradient below is
 * the operator A of the solve):
 *   div_ijk = (u_{i+1} - u_i)/dx + (v_{j+1} - v_j)/dy
 *           + (rho_{k+1/2} w_{k+1} - rho_{k-1/2} w_k) / (rho_k dz_k),
 * periodic in x and y, with no flux through the bottom and top faces.
 * Gradient: (p_i - p_{i-1})/dx on u faces, (p_j - p_{j-1})/dy on v faces,
 * (p_k - p_{k-1})/h_{k-1/2} on the w faces of levels k >= 1 (0 at k = 0). */
int oracle_divergence(int nx, int ny, int nz, double dx, double dy,
                      const double *dz, const double *rho, const double *u,
                      const double *v, const double *w, double *div)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !u || !v || !w || !div)
        return OR_EINVAL;
    for (int k = 0; k < nz; ++k) {
        const double Dk = rho[k] * dz[k];
        const double rup = k + 1 < nz ? 0.5 * (rho[k] + rho[k + 1]) : 0.0;
        const double rdn = k > 0 ? 0.5 * (rho[k - 1] + rho[k]) : 0.0;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = ((size_t)k * ny + j) * nx + i;
                const size_t ie = ((size_t)k * ny + j) * nx + (i + 1) % nx;
                const size_t jn = ((size_t)k * ny + (j + 1) % ny) * nx + i;
                double d = (u[ie] - u[c]) / dx + (v[jn] - v[c]) / dy;
                double flux = 0.0;
                if (k + 1 < nz)
                    flux += rup * w[c + (size_t)nx * ny];
                if (k > 0)
                    flux -= rdn * w[c];
                div[c] = d + flux / Dk;
            }
    }
    return OR_OK;
}

int oracle_gradient(int nx, int ny, int nz, double dx, double dy,
                    const double *dz, const double *rho, const double *p,
                    double *gu, double *gv, double *gw)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !p || !gu || !gv || !gw)
        return OR_EINVAL;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = ((size_t)k * ny + j) * nx + i;
                const size_t iw = ((size_t)k * ny + j) * nx + (i + nx - 1) % nx;
                const size_t js = ((size_t)k * ny + (j + ny - 1) % ny) * nx + i;
                gu[c] = (p[c] - p[iw]) / dx;
                gv[c] = (p[c] - p[js]) / dy;
                gw[c] = k > 0 ? (p[c] - p[c - (size_t)nx * ny]) / (0.5 * (dz[k - 1] + dz[k]))
                              : 0.0;
            }
    return OR_OK;
}

/* Explicit 7-point operator, A p, by direct stencil application. */
int oracle_apply(int nx, int ny, int nz, double dx, double dy,
                 const double *dz, const double *rho, const double *p,
                 double *Ap)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !p || !Ap)
        return OR_EINVAL;
    double *f = (double *)malloc(sizeof(double) * (size_t)(2 * nz + 1));
    if (!f)
        return OR_ENOMEM;
    double *D = f + nz + 1;
    vertical_coefficients(nz, dz, rho, f, D);
    const double ix2 = 1.0 / (dx * dx), iy2 = 1.0 / (dy * dy);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = ((size_t)k * ny + j) * nx + i;
                const double pc = p[c];
                const double *lv = p + (size_t)k * nx * ny;
                double pxm = lv[(size_t)j * nx + (i + nx - 1) % nx];
                double pxp = lv[(size_t)j * nx + (i + 1) % nx];
                double pym = lv[(size_t)((j + ny - 1) % ny) * nx + i];
                double pyp = lv[(size_t)((j + 1) % ny) * nx + i];
                double v = (pxp - 2.0 * pc + pxm) * ix2 + (pyp - 2.0 * pc + pym) * iy2;
                double flux = 0.0;
                if (k + 1 < nz)
                    flux += f[k + 1] * (p[c + (size_t)nx * ny] - pc);
                if (k > 0)
                    flux -= f[k] * (pc - p[c - (size_t)nx * ny]);
                Ap[c] = v + flux / D[k];
            }
    free(f);
    return OR_OK;
}

/* Gradient of L = <w, p> with respect to the per-level densities rho_k,
 * given lam = S^T w and the solution p:  g_k = -lam^T (dA/drho_k) p.
 * The border of the bordered system does not depend on rho, so no
 * projection term appears.  Only V depends on rho; differentiating its
 * three ingredients (the 1/D_k factor of row k and the two face densities
 * adjacent to level k) gives, with gamma_{k+1/2} = (p_{k+1}-p_k)/h_{k+1/2},
 *   lam^T dA/drho_k p = sum_ij [ -lam_k (V p)_k / rho_k
 *        + 1/2 gamma_{k+1/2} (lam_k/D_k - lam_{k+1}/D_{k+1})
 *        + 1/2 gamma_{k-1/2} (lam_{k-1}/D_{k-1} - lam_k/D_k) ],
 * faces outside the column omitted. */
int oracle_grad_rho(int nx, int ny, int nz, double dx, double dy,
                    const double *dz, const double *rho, const double *lam,
                    const double *p, double *g)
{
    int err = check_grid(nx, ny, nz, dx, dy, dz, rho);
    if (err || !lam || !p || !g)
        return OR_EINVAL;
    double *f = (double *)malloc(sizeof(double) * (size_t)(2 * nz + 1));
    if (!f)
        return OR_ENOMEM;
    double *D = f + nz + 1;
    vertical_coefficients(nz, dz, rho, f, D);
    const size_t lv = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double acc = 0.0;
        for (size_t q = 0; q < lv; ++q) {
            size_t c = (size_t)k * lv + q;
            double pc = p[c], lc = lam[c];
            double Vp = 0.0;
            if (k + 1 < nz)
                Vp += f[k + 1] * (p[c + lv] - pc);
            if (k > 0)
                Vp -= f[k] * (pc - p[c - lv]);
            Vp /= D[k];
            double t = -lc * Vp / rho[k];
            if (k + 1 < nz) {
                double h = 0.5 * (dz[k] + dz[k + 1]);
                double gam = (p[c + lv] - pc) / h;
                t += 0.5 * gam * (lc / D[k] - lam[c + lv] / D[k + 1]);
            }
            if (k > 0) {
                double h = 0.5 * (dz[k - 1] + dz[k]);
                double gam = (pc - p[c - lv]) / h;
                t += 0.5 * gam * (lam[c - lv] / D[k - 1] - lc / D[k]);
            }
            acc += t;
        }
        g[k] = -acc;
    }
    free(f);
    return OR_OK;
}

/* Vertical tables, exposed so tests can pin them against their own
 * independent assembly. f has nz+1 entries, D has nz. */
int oracle_vertical_coefficients(int nz, const double *dz, const double *rho,
                                 double *f, double *D)
{
    if (nz < 1 || !dz || !rho || !f || !D)
        return OR_EINVAL;
    vertical_coefficients(nz, dz, rho, f, D);
    return OR_OK;
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
