// The dynamical-core steps on either side of the pressure solve (paper
// Section 1: the dynamical core produces the source terms that feed the
// solve, and the pressure it returns corrects the flow): the divergence of
// the provisional C-grid velocity, formed inside the forward x pass so that
// no right-hand-side field is written or read, and the pressure-gradient
// correction that makes the corrected velocity divergence-free.
//
// Velocities are [nz][ny][nx] fields: u[k][j][i] on the x-face between
// cells i-1 and i, v[k][j][i] on the y-face between rows j-1 and j,
// w[k][j][i] on the face between levels k-1 and k (level 0's w is the
// bottom boundary face: no flux, neither read nor written).
//   div = (u_{i+1} - u_i)/dx + (v_{j+1} - v_j)/dy
//       + (rho_{k+1/2} w_{k+1} - rho_{k-1/2} w_k) / (rho_k dz_k)
//   G p = ((p_i - p_{i-1})/dx, (p_j - p_{j-1})/dy, (p_k - p_{k-1})/h_{k-1/2})
// so that div(G p) = A p, the operator of the solve.
#include "ps_internal.h"
#include "ps_tiles.h"

namespace ps {

// Generic forward x pass of scale * div (any 2^a 3^b length): the rows'
// divergence is formed in FP64 from the loads, rounded once, staged in LDS
// and transformed as in fwd_x_tile.  With pres, the transformed rows are the
// residual scale * div - A pres of the refinement step instead (the 7-point
// operator with the forward vertical coefficients rc, 3 per level:
// f_{k+1/2}/D_k, f_{k-1/2}/D_k and their sum; idx2 = 1/dx^2, idy2 = 1/dy^2),
// all in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_x_div(
    const T *__restrict__ u, const T *__restrict__ v, const T *__restrict__ w, double scale,
    cx_t<T> *__restrict__ spec, double *__restrict__ rowsum, int nx, int ny, int nz, int rows,
    double idx, double idy, const double *__restrict__ dc, StagePlan sp,
    const cx_t<T> *__restrict__ twx, const cx_t<T> *__restrict__ tws,
    const T *__restrict__ pres, const double *__restrict__ rc)
{
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = nx >> 1;
    const int nrows_total = ny * nz;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * L;
    C *stw = b + rows * L;
    C *sws = stw + L;
    const int row0 = blockIdx.x * rows;
    const int nr = min(rows, nrows_total - row0);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        stw[t] = twx[t];
        sws[t] = tws[t];
    }
    const size_t lvl = (size_t)nx * ny;
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int r = t / L, n = t - r * L;
        const int g = row0 + r;
        const int lev = g / ny, j = g - lev * ny;
        const size_t rowoff = (size_t)g * nx;
        const size_t north = (size_t)lev * lvl + (size_t)((j + 1) % ny) * nx;
        const double au = dc[3 * lev], ad = dc[3 * lev + 1];
        double d[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * n + h;
            double x = ((double)u[rowoff + (i + 1) % nx] - (double)u[rowoff + i]) * idx +
                       ((double)v[north + i] - (double)v[rowoff + i]) * idy;
            if (lev + 1 < nz) x += au * (double)w[rowoff + lvl + i];
            if (lev > 0) x -= ad * (double)w[rowoff + i];
            x *= scale;
            if (pres) {
                const size_t south = (size_t)lev * lvl + (size_t)((j + ny - 1) % ny) * nx;
                const double pc = (double)pres[rowoff + i];
                double ap = ((double)pres[rowoff + (i + 1) % nx] - 2.0 * pc +
                             (double)pres[rowoff + (i + nx - 1) % nx]) * (idx * idx) +
                            ((double)pres[north + i] - 2.0 * pc + (double)pres[south + i]) *
                                (idy * idy) -
                            rc[3 * lev + 2] * pc;
                if (lev + 1 < nz) ap += rc[3 * lev] * (double)pres[rowoff + lvl + i];
                if (lev > 0) ap += rc[3 * lev + 1] * (double)pres[rowoff - lvl + i];
                x -= ap;
            }
            d[h] = x;
        }
        a[t] = C{(T)d[0], (T)d[1]};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r = wv; r < nr; r += nw) {
        double s = 0.0;
        for (int n = lane; n < L; n += 64) {
            const C z = a[r * L + n];
            s += (double)z.x + (double)z.y;
        }
        s = wave_sum(s);
        if (lane == 0) rowsum[row0 + r] = s;
    }
    C *Z = stockham_rows<-1>(a, b, nr, L, sp, stw);
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int kx = t / nr, r = t - kx * nr;
        const C *zr = Z + r * L;
        C X;
        if (kx == 0) {
            const C z0 = zr[0];
            X = C{z0.x + z0.y, z0.x - z0.y};
        } else {
            const C zk = zr[kx], zc = cconj(zr[L - kx]);
            const C e = C{T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
            const C dd = csub(zk, zc);
            const C o = C{T(0.5) * dd.y, T(-0.5) * dd.x};
            X = cadd(e, cmul(o, sws[kx]));
        }
        const int g = row0 + r;
        const int lev = g / ny, j = g - lev * ny;
        spec[((size_t)lev * L + kx) * ny + j] = X;
    }
}

// u -= dt Gx p, v -= dt Gy p, w -= dt Gz p (w of level 0 untouched), one
// thread per point along x (a block per row), FP64 differences.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_correct(T *__restrict__ u, T *__restrict__ v,
                                                      T *__restrict__ w,
                                                      const T *__restrict__ p, double dt,
                                                      int nx, int ny, int nz, double idx,
                                                      double idy, const double *__restrict__ dc)
{
    const int row = blockIdx.x; // k ny + j
    const int k = row / ny, j = row - k * ny;
    const size_t lvl = (size_t)nx * ny, off = (size_t)row * nx;
    const size_t south = (size_t)k * lvl + (size_t)(j == 0 ? ny - 1 : j - 1) * nx;
    const double ih = dc[3 * k + 2];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double pc = (double)p[off + i];
        const double pw = (double)p[off + (i == 0 ? nx - 1 : i - 1)];
        const double ps = (double)p[south + i];
        u[off + i] = (T)((double)u[off + i] - dt * (pc - pw) * idx);
        v[off + i] = (T)((double)v[off + i] - dt * (pc - ps) * idy);
        if (k > 0) {
            const double pd = (double)p[off - lvl + i];
            w[off + i] = (T)((double)w[off + i] - dt * (pc - pd) * ih);
        }
    }
}

template <typename T>
hipError_t launch_fwd_x_div(const T *u, const T *v, const T *w, double scale, cx_t<T> *spec,
                            double *rowsum, int nx, int ny, int nz, double dx, double dy,
                            const double *dc, const FftGeom &g, const StagePlan &spx,
                            const Tables<T> &tb, hipStream_t st, const T *pres,
                            const double *rc)
{
    const int total = ny * nz, L = nx / 2;
    const int grid = (total + g.rows_x - 1) / g.rows_x;
    const size_t lds = (size_t)(2 * g.rows_x * L + 2 * L) * sizeof(cx_t<T>);
    hipLaunchKernelGGL(k_fwd_x_div<T>, dim3(grid), dim3(256), lds, st, u, v, w, scale, spec,
                       rowsum, nx, ny, nz, g.rows_x, 1.0 / dx, 1.0 / dy, dc, spx, tb.tw_x,
                       tb.tw_s, pres, rc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_correct(T *u, T *v, T *w, const T *p, double dt, int nx, int ny, int nz,
                               double dx, double dy, const double *dc, hipStream_t st)
{
    const int threads = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
    hipLaunchKernelGGL(k_grad_correct<T>, dim3(ny * nz), dim3(threads), 0, st, u, v, w, p, dt, nx,
                       ny, nz, 1.0 / dx, 1.0 / dy, dc);
    return hipGetLastError();
}

template hipError_t launch_fwd_x_div<float>(const float *, const float *, const float *, double,
                                            cx_t<float> *, double *, int, int, int, double,
                                            double, const double *, const FftGeom &,
                                            const StagePlan &, const Tables<float> &,
                                            hipStream_t, const float *, const double *);
template hipError_t launch_fwd_x_div<double>(const double *, const double *, const double *,
                                             double, cx_t<double> *, double *, int, int, int,
                                             double, double, const double *, const FftGeom &,
                                             const StagePlan &, const Tables<double> &,
                                             hipStream_t, const double *, const double *);
template hipError_t launch_grad_correct<float>(float *, float *, float *, const float *, double,
                                               int, int, int, double, double, const double *,
                                               hipStream_t);
template hipError_t launch_grad_correct<double>(double *, double *, double *, const double *,
                                                double, int, int, int, double, double,
                                                const double *, hipStream_t);

} // namespace ps
