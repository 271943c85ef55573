// Matrix-free preconditioned conjugate gradients on the same discrete
// operator as the direct solve: the paper's iterative alternative (Section
// 2.2, the bespoke matrix-free CG with its hard-coded operator, several
// inner products reduced together, and termination on the relative
// residual; Table 1 compares its accuracy and cost with the FFT solve).
//
// A = dxx + dyy + V is not symmetric when the levels are stretched, but
// M = -D A (D_k = rho_k dz_k on level k) is symmetric positive semi-definite
// with the constants as its null space:
//   (M x)_ijk = D_k [ (2x - x_{i+1} - x_{i-1})/dx^2 + (2x - x_{j+1} - x_{j-1})/dy^2 ]
//             + f_{k+1/2} (x - x_{k+1}) + f_{k-1/2} (x - x_{k-1}),
// periodic in x and y, f_{-1/2} = f_{nz-1/2} = 0.  The right-hand side is
// projected first (b' = b - mu, mu the D-weighted mean, as in the direct
// solve), so M x = -D b' is consistent and CG converges to a solution; the
// result is shifted to zero mean at the end, the gauge of the direct solve.
// Preconditioner: none, or Jacobi (the diagonal of M).
//
// Each iteration is five launches: q = M p with the partial sums of p.q;
// alpha; x += alpha p, r -= alpha q with the partial sums of r.z and r.r
// (z = r / diag, not stored); beta and the convergence test; p = z + beta p.
// The scalars live on the device, so iterations are enqueued without host
// round trips; once the relative residual |r| / |M-rhs| reaches the
// tolerance a device flag makes every later launch return at once, and the
// host reads the status only every few iterations.  All sums are per-block
// partials in a fixed order, reduced in a fixed order: results do not depend
// on scheduling.
//
// BiCGStab (van der Vorst's stabilised bi-conjugate gradients), the paper's
// other bespoke Krylov solver, runs on A itself -- it needs no symmetric
// operator -- with the projected right-hand side b' = b - mu, and is
// post-conditioned as the paper's is (right preconditioning: it solves
// A K^-1 y = b' and x = K^-1 y, K the diagonal of A or the identity, so the
// residual it tracks is that of A x = b' itself).  An iteration is nine
// launches: p = r + beta (p - omega v); v = A K^-1 p with the partials of
// rh.v; alpha; x += alpha K^-1 p, s = r - alpha v with the partials of s.s;
// the test on |s| (a half step can end the solve); t = A K^-1 s with the
// partials of t.s and t.t; omega; x += omega K^-1 s, r = s - omega t with the
// partials of rh.r and r.r; rho, beta and the test on |r|.  K^-1 multiplies
// each value as it is loaded (a per-level factor), so neither K^-1 p nor
// K^-1 s is stored.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ps_internal.h"
#include "../../include/pressure_solve.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;
constexpr int kChunk = 16; // iterations enqueued between two status reads

// Device scalars of one solve.
struct CgState {
    double mu;      // projection mean
    double rz;      // r.z of the current residual
    double pq;      // p.q
    double alpha, beta;
    double rr;      // r.r
    double rhs2;    // |M-rhs|^2 = |D b'|^2
    double tol2;    // rtol^2 |M-rhs|^2
    double xmean;   // mean of x for the gauge
    double rho;     // BiCGStab: rh.r of the current residual
    double omega;   // BiCGStab: the stabilising step
    int done;       // 1 once converged (or max_iter reached, or a breakdown)
    int iters;      // completed iterations
    int max_iter;
    int pad;
};

struct Geo {
    int nx, ny, nz;
    unsigned n;        // nx ny nz < 2^31
    double idx2, idy2; // 1/dx^2, 1/dy^2
};

__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = ps::wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return s;
}

// (M x) at point c = (k, j, i); 32-bit index arithmetic (n < 2^31).
__device__ __forceinline__ double apply_m(const double *__restrict__ x, const Geo &g,
                                          const double *__restrict__ f,
                                          const double *__restrict__ D, unsigned c)
{
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const unsigned k = c / nxy, rem = c - k * nxy;
    const unsigned j = rem / (unsigned)g.nx, i = rem - j * (unsigned)g.nx;
    const double xc = x[c];
    const unsigned row = c - i, lev = k * nxy;
    const double xe = x[row + (i + 1 == (unsigned)g.nx ? 0u : i + 1)];
    const double xw = x[row + (i == 0 ? (unsigned)g.nx - 1 : i - 1)];
    const double xn = x[lev + (j + 1 == (unsigned)g.ny ? 0u : j + 1) * (unsigned)g.nx + i];
    const double xs = x[lev + (j == 0 ? (unsigned)g.ny - 1 : j - 1) * (unsigned)g.nx + i];
    const double fu = f[k + 1], fd = f[k];
    const double xu = k + 1 < (unsigned)g.nz ? x[c + nxy] : xc;
    const double xd = k > 0 ? x[c - nxy] : xc;
    const double lat = ((xc - xe) + (xc - xw)) * g.idx2 + ((xc - xn) + (xc - xs)) * g.idy2;
    return D[k] * lat + fu * (xc - xu) + fd * (xc - xd);
}

__device__ __forceinline__ double diag_inv(const Geo &g, const double *__restrict__ f,
                                           const double *__restrict__ D, int k, int precond)
{
    if (!precond) return 1.0;
    return 1.0 / (D[k] * (2.0 * g.idx2 + 2.0 * g.idy2) + f[k] + f[k + 1]);
}

// (A y) at point c with y = K^-1 x (per-level factor kinv, 1 without a
// preconditioner): the lateral second differences plus the vertical
// operator, whose coefficients f_{k+1/2}/D_k and f_{k-1/2}/D_k are tabled
// (au, ad; zero at the top and bottom faces).
__device__ __forceinline__ double apply_ak(const double *__restrict__ x, const Geo &g,
                                           const double *__restrict__ au,
                                           const double *__restrict__ ad,
                                           const double *__restrict__ kinv, unsigned c)
{
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const unsigned k = c / nxy, rem = c - k * nxy;
    const unsigned j = rem / (unsigned)g.nx, i = rem - j * (unsigned)g.nx;
    const double sk = kinv[k];
    const unsigned row = c - i, lev = k * nxy;
    const double xc = x[c] * sk;
    const double xe = x[row + (i + 1 == (unsigned)g.nx ? 0u : i + 1)] * sk;
    const double xw = x[row + (i == 0 ? (unsigned)g.nx - 1 : i - 1)] * sk;
    const double xn = x[lev + (j + 1 == (unsigned)g.ny ? 0u : j + 1) * (unsigned)g.nx + i] * sk;
    const double xs = x[lev + (j == 0 ? (unsigned)g.ny - 1 : j - 1) * (unsigned)g.nx + i] * sk;
    const double xu = k + 1 < (unsigned)g.nz ? x[c + nxy] * kinv[k + 1] : xc;
    const double xd = k > 0 ? x[c - nxy] * kinv[k - 1] : xc;
    const double lat = ((xe - xc) + (xw - xc)) * g.idx2 + ((xn - xc) + (xs - xc)) * g.idy2;
    return lat + au[k] * (xu - xc) + ad[k] * (xd - xc);
}

// Level sums of b, one block per level (fixed order).
__global__ __launch_bounds__(kThreads) void k_cg_levelsum(const double *__restrict__ b, Geo g,
                                                          double *__restrict__ S)
{
    __shared__ double red[4];
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double *lv = b + (size_t)blockIdx.x * nxy;
    double s = 0.0;
    for (unsigned q = threadIdx.x; q < nxy; q += blockDim.x) s += lv[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) S[blockIdx.x] = s;
}

// mu (D-weighted mean of b) and the state's initial values.
__global__ void k_cg_setup(const double *__restrict__ S, const double *__restrict__ D, Geo g,
                           CgState *st, int max_iter)
{
    double num = 0.0, den = 0.0;
    for (int k = 0; k < g.nz; ++k) {
        num += D[k] * S[k];
        den += D[k];
    }
    st->mu = num / (den * (double)g.nx * (double)g.ny);
    st->done = 0;
    st->iters = 0;
    st->max_iter = max_iter;
}

// r = -D (b - mu) - M x0, p = z = r / diag; partials of r.z, r.r, |D b'|^2.
__global__ __launch_bounds__(kThreads) void k_cg_start(const double *__restrict__ b,
                                                       const double *__restrict__ x, Geo g,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ D,
                                                       double *__restrict__ r,
                                                       double *__restrict__ p,
                                                       const CgState *__restrict__ st,
                                                       double *__restrict__ part, int precond)
{
    __shared__ double red[4];
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double mu = st->mu;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const int k = (int)(c / nxy);
        const double rhs = -D[k] * (b[c] - mu);
        const double rc = rhs - apply_m(x, g, f, D, c);
        const double z = rc * diag_inv(g, f, D, k, precond);
        r[c] = rc;
        p[c] = z;
        rz += rc * z;
        rr += rc * rc;
        bb += rhs * rhs;
    }
    const double a = block_sum(rz, red), b2 = block_sum(rr, red), c2 = block_sum(bb, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b2;
        part[2 * gridDim.x + blockIdx.x] = c2;
    }
}

// Fixed-order sum of nsum groups of nb partials: out[s] = sum_b part[s nb + b].
__device__ void reduce_groups(const double *__restrict__ part, int nb, int nsum, double *out)
{
    __shared__ double red[4];
    for (int s = 0; s < nsum; ++s) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[(size_t)s * nb + b];
        v = block_sum(v, red);
        if (threadIdx.x == 0) out[s] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_cg_start_scalars(const double *__restrict__ part,
                                                               int nb, CgState *st, double rtol)
{
    __shared__ double v[3];
    reduce_groups(part, nb, 3, v);
    if (threadIdx.x == 0) {
        st->rz = v[0];
        st->rr = v[1];
        st->rhs2 = v[2];
        st->tol2 = rtol * rtol * v[2];
        if (v[1] <= st->tol2 || st->max_iter <= 0) st->done = 1;
    }
}

// q = M p; partials of p.q.
__global__ __launch_bounds__(kThreads) void k_cg_apply(const double *__restrict__ p, Geo g,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ D,
                                                       double *__restrict__ q,
                                                       const CgState *__restrict__ st,
                                                       double *__restrict__ part)
{
    if (st->done) return;
    __shared__ double red[4];
    double pq = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const double v = apply_m(p, g, f, D, c);
        q[c] = v;
        pq += p[c] * v;
    }
    const double s = block_sum(pq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_cg_alpha(const double *__restrict__ part, int nb,
                                                       CgState *st)
{
    if (st->done) return;
    __shared__ double v[1];
    reduce_groups(part, nb, 1, v);
    if (threadIdx.x == 0) {
        st->pq = v[0];
        st->alpha = st->rz / v[0];
    }
}

// x += alpha p, r -= alpha q; partials of r.z (z = r / diag) and r.r.
__global__ __launch_bounds__(kThreads) void k_cg_update(double *__restrict__ x,
                                                        const double *__restrict__ p,
                                                        double *__restrict__ r,
                                                        const double *__restrict__ q, Geo g,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ D,
                                                        const CgState *__restrict__ st,
                                                        double *__restrict__ part, int precond)
{
    if (st->done) return;
    __shared__ double red[4];
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double alpha = st->alpha;
    double rz = 0.0, rr = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        x[c] += alpha * p[c];
        const double rc = r[c] - alpha * q[c];
        r[c] = rc;
        const int k = (int)(c / nxy);
        rz += rc * (rc * diag_inv(g, f, D, k, precond));
        rr += rc * rc;
    }
    const double a = block_sum(rz, red), b = block_sum(rr, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kThreads) void k_cg_beta(const double *__restrict__ part, int nb,
                                                      CgState *st)
{
    if (st->done) return;
    __shared__ double v[2];
    reduce_groups(part, nb, 2, v);
    if (threadIdx.x == 0) {
        st->beta = v[0] / st->rz;
        st->rz = v[0];
        st->rr = v[1];
        st->iters += 1;
        if (v[1] <= st->tol2 || st->iters >= st->max_iter) st->done = 1;
    }
}

// p = z + beta p.
__global__ __launch_bounds__(kThreads) void k_cg_dir(double *__restrict__ p,
                                                     const double *__restrict__ r, Geo g,
                                                     const double *__restrict__ f,
                                                     const double *__restrict__ D,
                                                     const CgState *__restrict__ st, int precond)
{
    if (st->done) return;
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double beta = st->beta;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const int k = (int)(c / nxy);
        p[c] = r[c] * diag_inv(g, f, D, k, precond) + beta * p[c];
    }
}

// Partials of sum(x), then the shift to zero mean.
__global__ __launch_bounds__(kThreads) void k_cg_xsum(const double *__restrict__ x, Geo g,
                                                      double *__restrict__ part)
{
    __shared__ double red[4];
    double s = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x)
        s += x[c];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_cg_xmean(const double *__restrict__ part, int nb,
                                                       Geo g, CgState *st)
{
    __shared__ double v[1];
    reduce_groups(part, nb, 1, v);
    if (threadIdx.x == 0) st->xmean = v[0] / (double)g.n;
}

__global__ __launch_bounds__(kThreads) void k_cg_shift(double *__restrict__ x, Geo g,
                                                       const CgState *__restrict__ st)
{
    const double m = st->xmean;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x)
        x[c] -= m;
}

// ------------------------------------------------------------- BiCGStab
// Tables of the BiCGStab kernels: au, ad and kinv, nz values each.
struct BiTab {
    const double *au, *ad, *kinv;
};

// r = rh = b' - A x0 (b' = b - mu), p = v = 0; partials of r.r and b'.b'.
__global__ __launch_bounds__(kThreads) void k_bi_start(const double *__restrict__ b,
                                                       const double *__restrict__ x, Geo g,
                                                       BiTab tb, const double *__restrict__ one,
                                                       double *__restrict__ r,
                                                       double *__restrict__ rh,
                                                       double *__restrict__ p,
                                                       double *__restrict__ v,
                                                       const CgState *__restrict__ st,
                                                       double *__restrict__ part)
{
    __shared__ double red[4];
    const double mu = st->mu;
    double rr = 0.0, bb = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const double rhs = b[c] - mu;
        const double rc = rhs - apply_ak(x, g, tb.au, tb.ad, one, c);
        r[c] = rc;
        rh[c] = rc;
        p[c] = 0.0;
        v[c] = 0.0;
        rr += rc * rc;
        bb += rhs * rhs;
    }
    const double a = block_sum(rr, red), c2 = block_sum(bb, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = c2;
    }
}

// rho = rh.r = r.r, beta = 0 (so the first direction is r), alpha = omega = 1.
__global__ __launch_bounds__(kThreads) void k_bi_start_scalars(const double *__restrict__ part,
                                                               int nb, CgState *st, double rtol)
{
    __shared__ double v[2];
    reduce_groups(part, nb, 2, v);
    if (threadIdx.x == 0) {
        st->rho = v[0];
        st->rr = v[0];
        st->rhs2 = v[1];
        st->tol2 = rtol * rtol * v[1];
        st->beta = 0.0;
        st->alpha = 1.0;
        st->omega = 1.0;
        if (v[0] <= st->tol2 || st->max_iter <= 0) st->done = 1;
    }
}

// p = r + beta (p - omega v).
__global__ __launch_bounds__(kThreads) void k_bi_dir(double *__restrict__ p,
                                                     const double *__restrict__ r,
                                                     const double *__restrict__ v, Geo g,
                                                     const CgState *__restrict__ st)
{
    if (st->done) return;
    const double beta = st->beta, omega = st->omega;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x)
        p[c] = r[c] + beta * (p[c] - omega * v[c]);
}

// out = A K^-1 in; partials of w1.out (and, with w2, of w2.out and out.out).
__global__ __launch_bounds__(kThreads) void k_bi_apply(const double *__restrict__ in, Geo g,
                                                       BiTab tb, double *__restrict__ out,
                                                       const double *__restrict__ w1,
                                                       int second,
                                                       const CgState *__restrict__ st,
                                                       double *__restrict__ part)
{
    if (st->done) return;
    __shared__ double red[4];
    double d1 = 0.0, d2 = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const double o = apply_ak(in, g, tb.au, tb.ad, tb.kinv, c);
        out[c] = o;
        d1 += w1[c] * o;
        d2 += o * o;
    }
    const double a = block_sum(d1, red);
    const double b = second ? block_sum(d2, red) : 0.0;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        if (second) part[gridDim.x + blockIdx.x] = b;
    }
}

// alpha = rho / rh.v (a zero rh.v is a breakdown: the solve stops).
__global__ __launch_bounds__(kThreads) void k_bi_alpha(const double *__restrict__ part, int nb,
                                                       CgState *st)
{
    if (st->done) return;
    __shared__ double v[1];
    reduce_groups(part, nb, 1, v);
    if (threadIdx.x == 0) {
        if (v[0] == 0.0 || !isfinite(v[0])) {
            st->done = 1;
            return;
        }
        st->alpha = st->rho / v[0];
    }
}

// x += alpha K^-1 p, r := s = r - alpha v; partials of s.s.
__global__ __launch_bounds__(kThreads) void k_bi_half(double *__restrict__ x,
                                                      const double *__restrict__ p,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ v, Geo g,
                                                      BiTab tb, const CgState *__restrict__ st,
                                                      double *__restrict__ part)
{
    if (st->done) return;
    __shared__ double red[4];
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double alpha = st->alpha;
    double ss = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        x[c] += alpha * (p[c] * tb.kinv[c / nxy]);
        const double sc = r[c] - alpha * v[c];
        r[c] = sc;
        ss += sc * sc;
    }
    const double a = block_sum(ss, red);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// The half-step test: |s| small ends the solve with x as it stands.
__global__ __launch_bounds__(kThreads) void k_bi_half_test(const double *__restrict__ part,
                                                           int nb, CgState *st)
{
    if (st->done) return;
    __shared__ double v[1];
    reduce_groups(part, nb, 1, v);
    if (threadIdx.x == 0 && v[0] <= st->tol2) {
        st->rr = v[0];
        st->iters += 1;
        st->done = 1;
    }
}

// omega = t.s / t.t (a zero t.t is a breakdown: the solve stops).
__global__ __launch_bounds__(kThreads) void k_bi_omega(const double *__restrict__ part, int nb,
                                                       CgState *st)
{
    if (st->done) return;
    __shared__ double v[2];
    reduce_groups(part, nb, 2, v);
    if (threadIdx.x == 0) {
        if (v[1] == 0.0 || !isfinite(v[1])) {
            st->done = 1;
            return;
        }
        st->omega = v[0] / v[1];
    }
}

// x += omega K^-1 s, r = s - omega t; partials of rh.r and r.r.
__global__ __launch_bounds__(kThreads) void k_bi_update(double *__restrict__ x,
                                                        double *__restrict__ r,
                                                        const double *__restrict__ t,
                                                        const double *__restrict__ rh, Geo g,
                                                        BiTab tb,
                                                        const CgState *__restrict__ st,
                                                        double *__restrict__ part)
{
    if (st->done) return;
    __shared__ double red[4];
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const double omega = st->omega;
    double rhr = 0.0, rr = 0.0;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n;
         c += gridDim.x * blockDim.x) {
        const double sc = r[c];
        x[c] += omega * (sc * tb.kinv[c / nxy]);
        const double rc = sc - omega * t[c];
        r[c] = rc;
        rhr += rh[c] * rc;
        rr += rc * rc;
    }
    const double a = block_sum(rhr, red), b = block_sum(rr, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}

// rho, beta = (rho_new / rho) (alpha / omega), the iteration count and the
// test on |r| (a zero rho_new is a breakdown: the solve stops).
__global__ __launch_bounds__(kThreads) void k_bi_rho(const double *__restrict__ part, int nb,
                                                     CgState *st)
{
    if (st->done) return;
    __shared__ double v[2];
    reduce_groups(part, nb, 2, v);
    if (threadIdx.x == 0) {
        st->rr = v[1];
        st->iters += 1;
        if (v[1] <= st->tol2 || st->iters >= st->max_iter || v[0] == 0.0 || st->omega == 0.0) {
            st->done = 1;
            return;
        }
        st->beta = (v[0] / st->rho) * (st->alpha / st->omega);
        st->rho = v[0];
    }
}

} // namespace

struct ps_cg {
    Geo g{};
    int precond = 0;
    int method = PS_KRYLOV_CG;
    hipStream_t stream = nullptr;
    int nblk = 1;
    double *f = nullptr; // [f (nz+1) | D (nz) | au (nz) | ad (nz) | kinv (nz) | ones (nz)]
    double *S = nullptr, *part = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr;
    double *rh = nullptr, *t = nullptr; // BiCGStab only (allocated when selected)
    CgState *st = nullptr;
    CgState *host = nullptr; // pinned copy of the state
    size_t bytes = 0;
};

static int cfail(int code, const std::string &msg) { return ps::set_error(code, msg); }

#define PS_CHIP_EARLY(call)                                                                        \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return cfail(PS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

static void free_cg(ps_cg *c)
{
    for (void *q : {(void *)c->f, (void *)c->S, (void *)c->part, (void *)c->r, (void *)c->p,
                    (void *)c->q, (void *)c->rh, (void *)c->t, (void *)c->st})
        if (q) (void)hipFree(q);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

extern "C" int ps_cg_create(ps_cg **out, int nx, int ny, int nz, double dx, double dy,
                            const double *dz, const double *rho, int precond, void *stream)
{
    if (!out) return cfail(PS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!dz || !rho) return cfail(PS_EINVAL, "dz and rho must not be NULL");
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz >= (1LL << 31))
        return cfail(PS_EUNSUPPORTED, "grid sizes must be >= 1, fewer than 2^31 points");
    if (!(std::isfinite(dx) && dx > 0) || !(std::isfinite(dy) && dy > 0))
        return cfail(PS_EINVAL, "dx and dy must be finite and > 0");
    if (precond != PS_CG_NONE && precond != PS_CG_JACOBI)
        return cfail(PS_EINVAL, "precond must be PS_CG_NONE or PS_CG_JACOBI");
    for (int k = 0; k < nz; ++k)
        if (!(std::isfinite(dz[k]) && dz[k] > 0) || !(std::isfinite(rho[k]) && rho[k] > 0))
            return cfail(PS_EINVAL, "dz and rho values must be finite and > 0");
    ps_cg *c = new ps_cg();
    c->g = Geo{nx, ny, nz, (unsigned)((long long)nx * ny * nz), 1.0 / (dx * dx), 1.0 / (dy * dy)};
    c->precond = precond;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->nblk = (int)std::min<long long>(kMaxBlocks, ((long long)c->g.n + kThreads - 1) / kThreads);
    // [f (nz+1) | D (nz) | au (nz) | ad (nz) | kinv (nz) | ones (nz)]
    std::vector<double> fd(6 * (size_t)nz + 1, 0.0);
    for (int k = 0; k + 1 < nz; ++k)
        fd[k + 1] = 0.5 * (rho[k] + rho[k + 1]) / (0.5 * (dz[k] + dz[k + 1]));
    for (int k = 0; k < nz; ++k) {
        const double D = rho[k] * dz[k];
        fd[nz + 1 + k] = D;
        fd[2 * nz + 1 + k] = fd[k + 1] / D;
        fd[3 * nz + 1 + k] = fd[k] / D;
        // the diagonal of A: -(2/dx^2 + 2/dy^2) - (f_{k-1/2} + f_{k+1/2}) / D_k
        const double diag = -(2.0 / (dx * dx) + 2.0 / (dy * dy)) - (fd[k] + fd[k + 1]) / D;
        fd[4 * nz + 1 + k] = precond == PS_CG_JACOBI ? 1.0 / diag : 1.0;
        fd[5 * nz + 1 + k] = 1.0;
    }
    auto alloc = [&](double **ptr, size_t n) {
        void *q = nullptr;
        if (hipMalloc(&q, n * sizeof(double)) != hipSuccess) return false;
        *ptr = reinterpret_cast<double *>(q);
        c->bytes += n * sizeof(double);
        return true;
    };
    void *stp = nullptr;
    if (!alloc(&c->f, fd.size()) || !alloc(&c->S, nz) || !alloc(&c->part, 3 * kMaxBlocks) ||
        !alloc(&c->r, c->g.n) || !alloc(&c->p, c->g.n) || !alloc(&c->q, c->g.n) ||
        hipMalloc(&stp, sizeof(CgState)) != hipSuccess) {
        free_cg(c);
        return cfail(PS_ENOMEM, "hipMalloc of the CG workspace failed");
    }
    c->st = reinterpret_cast<CgState *>(stp);
    if (hipHostMalloc((void **)&c->host, sizeof(CgState), hipHostMallocDefault) != hipSuccess) {
        free_cg(c);
        return cfail(PS_ENOMEM, "pinned status buffer");
    }
    if (hipMemcpy(c->f, fd.data(), fd.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess) {
        free_cg(c);
        return cfail(PS_EHIP, "uploading the CG coefficient tables failed");
    }
    *out = c;
    return PS_OK;
}

extern "C" int ps_cg_destroy(ps_cg *c)
{
    if (!c) return PS_OK;
    (void)hipStreamSynchronize(c->stream);
    free_cg(c);
    return PS_OK;
}

extern "C" int ps_cg_set_method(ps_cg *c, int method)
{
    if (!c) return cfail(PS_EINVAL, "cg is NULL");
    if (method != PS_KRYLOV_CG && method != PS_KRYLOV_BICGSTAB)
        return cfail(PS_EINVAL, "method must be PS_KRYLOV_CG or PS_KRYLOV_BICGSTAB");
    if (method == PS_KRYLOV_BICGSTAB && !c->rh) {
        PS_CHIP_EARLY(hipStreamSynchronize(c->stream));
        void *a = nullptr, *b = nullptr;
        const size_t n = (size_t)c->g.n * sizeof(double);
        if (hipMalloc(&a, n) != hipSuccess || hipMalloc(&b, n) != hipSuccess) {
            if (a) (void)hipFree(a);
            return cfail(PS_ENOMEM, "hipMalloc of the BiCGStab vectors failed");
        }
        c->rh = reinterpret_cast<double *>(a);
        c->t = reinterpret_cast<double *>(b);
        c->bytes += 2 * n;
    }
    c->method = method;
    return PS_OK;
}

extern "C" int ps_cg_set_stream(ps_cg *c, void *stream)
{
    if (!c) return cfail(PS_EINVAL, "cg is NULL");
    c->stream = reinterpret_cast<hipStream_t>(stream);
    return PS_OK;
}

#define PS_CHIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return cfail(PS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define PS_CLAUNCH(...)                                                                            \
    do {                                                                                           \
        hipLaunchKernelGGL(__VA_ARGS__);                                                           \
        hipError_t e_ = hipGetLastError();                                                         \
        if (e_ != hipSuccess)                                                                      \
            return cfail(PS_EHIP, std::string("launch: ") + hipGetErrorString(e_));                \
    } while (0)

extern "C" int ps_cg_solve(ps_cg *c, const double *rhs, double *x, double rtol, int max_iter,
                           int *iters, double *rel_res)
{
    if (!c || !rhs || !x) return cfail(PS_EINVAL, "cg, rhs and x must not be NULL");
    if (rhs == x) return cfail(PS_EINVAL, "rhs and x must not alias");
    if (!(rtol >= 0.0) || !std::isfinite(rtol)) return cfail(PS_EINVAL, "rtol must be >= 0");
    if (max_iter < 0) return cfail(PS_EINVAL, "max_iter must be >= 0");
    const Geo g = c->g;
    const double *f = c->f, *D = c->f + g.nz + 1;
    const BiTab tb{c->f + 2 * g.nz + 1, c->f + 3 * g.nz + 1, c->f + 4 * g.nz + 1};
    const double *ones = c->f + 5 * g.nz + 1;
    const int nb = c->nblk, pc = c->precond;
    const bool bi = c->method == PS_KRYLOV_BICGSTAB;
    hipStream_t s = c->stream;
    PS_CLAUNCH(k_cg_levelsum, dim3(g.nz), dim3(kThreads), 0, s, rhs, g, c->S);
    PS_CLAUNCH(k_cg_setup, dim3(1), dim3(1), 0, s, c->S, D, g, c->st, max_iter);
    if (bi) {
        PS_CLAUNCH(k_bi_start, dim3(nb), dim3(kThreads), 0, s, rhs, x, g, tb, ones, c->r, c->rh,
                   c->p, c->q, c->st, c->part);
        PS_CLAUNCH(k_bi_start_scalars, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st, rtol);
    } else {
        PS_CLAUNCH(k_cg_start, dim3(nb), dim3(kThreads), 0, s, rhs, x, g, f, D, c->r, c->p,
                   c->st, c->part, pc);
        PS_CLAUNCH(k_cg_start_scalars, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st, rtol);
    }
    for (int it = 0;;) {
        const int n = std::min(kChunk, std::max(1, max_iter - it));
        for (int i = 0; i < n; ++i) {
            if (bi) {
                // v = c->q; s overwrites r in place
                PS_CLAUNCH(k_bi_dir, dim3(nb), dim3(kThreads), 0, s, c->p, c->r, c->q, g, c->st);
                PS_CLAUNCH(k_bi_apply, dim3(nb), dim3(kThreads), 0, s, c->p, g, tb, c->q, c->rh,
                           0, c->st, c->part);
                PS_CLAUNCH(k_bi_alpha, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
                PS_CLAUNCH(k_bi_half, dim3(nb), dim3(kThreads), 0, s, x, c->p, c->r, c->q, g, tb,
                           c->st, c->part);
                PS_CLAUNCH(k_bi_half_test, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
                PS_CLAUNCH(k_bi_apply, dim3(nb), dim3(kThreads), 0, s, c->r, g, tb, c->t, c->r, 1,
                           c->st, c->part);
                PS_CLAUNCH(k_bi_omega, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
                PS_CLAUNCH(k_bi_update, dim3(nb), dim3(kThreads), 0, s, x, c->r, c->t, c->rh, g,
                           tb, c->st, c->part);
                PS_CLAUNCH(k_bi_rho, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
                continue;
            }
            PS_CLAUNCH(k_cg_apply, dim3(nb), dim3(kThreads), 0, s, c->p, g, f, D, c->q, c->st,
                       c->part);
            PS_CLAUNCH(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
            PS_CLAUNCH(k_cg_update, dim3(nb), dim3(kThreads), 0, s, x, c->p, c->r, c->q, g, f, D,
                       c->st, c->part, pc);
            PS_CLAUNCH(k_cg_beta, dim3(1), dim3(kThreads), 0, s, c->part, nb, c->st);
            PS_CLAUNCH(k_cg_dir, dim3(nb), dim3(kThreads), 0, s, c->p, c->r, g, f, D, c->st, pc);
        }
        it += n;
        PS_CHIP(hipMemcpyAsync(c->host, c->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        PS_CHIP(hipStreamSynchronize(s));
        if (c->host->done || it >= max_iter) break;
    }
    PS_CLAUNCH(k_cg_xsum, dim3(nb), dim3(kThreads), 0, s, x, g, c->part);
    PS_CLAUNCH(k_cg_xmean, dim3(1), dim3(kThreads), 0, s, c->part, nb, g, c->st);
    PS_CLAUNCH(k_cg_shift, dim3(nb), dim3(kThreads), 0, s, x, g, c->st);
    PS_CHIP(hipMemcpyAsync(c->host, c->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    PS_CHIP(hipStreamSynchronize(s));
    if (iters) *iters = c->host->iters;
    if (rel_res) *rel_res = c->host->rhs2 > 0 ? std::sqrt(c->host->rr / c->host->rhs2) : 0.0;
    return PS_OK;
}

extern "C" size_t ps_cg_workspace_bytes(const ps_cg *c) { return c ? c->bytes : 0; }
