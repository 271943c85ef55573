// Horizontal transforms of the pressure solve (paper Section 2.1: a forward
// Fourier transform of each level, one dimension for all data then the
// next, and the matching backward transform).
//
// Spectral layout (packed, transposed): spec[k][kx][ky], kx in [0, nx/2),
// ky in [0, ny), complex.  The x pass reads contiguous real rows and writes
// each block's rows transposed, so the y pass and the column solves both
// read contiguous memory.  The real-to-complex x transform is computed as an
// nx/2-point complex FFT of z_n = x_{2n} + i x_{2n+1} followed by the
// even/odd split; the two real coefficients X_0 and X_{nx/2} share slot
// kx = 0 as X_0 + i X_{nx/2}.
#include "ps_internal.h"
#include "ps_tiles.h"

namespace ps {

// x forward of the residual r = b - A p (adjoint: r = b - A^T p with
// A^T = D A D^{-1}, which changes only the vertical term), formed with FP64
// arithmetic from the stored b and p (7-point operator, periodic x/y,
// zero-flux ends).
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_x_residual(
    const T *__restrict__ bsrc, const T *__restrict__ p, cx_t<T> *__restrict__ spec,
    double *__restrict__ rowsum, int nx, int ny, int nz, int rows, double idx2, double idy2,
    const double *__restrict__ f, const double *__restrict__ D, int adjoint, StagePlan sp,
    const cx_t<T> *__restrict__ twx, const cx_t<T> *__restrict__ tws)
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
        const size_t up = (size_t)((j + 1) % ny) * nx + (size_t)lev * lvl;
        const size_t dn = (size_t)((j + ny - 1) % ny) * nx + (size_t)lev * lvl;
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * n + h;
            const double pc = (double)p[rowoff + i];
            double lap = ((double)p[rowoff + (i + 1) % nx] - 2.0 * pc +
                          (double)p[rowoff + (i + nx - 1) % nx]) * idx2 +
                         ((double)p[up + i] - 2.0 * pc + (double)p[dn + i]) * idy2;
            double vert;
            if (!adjoint) {
                double fl = 0.0;
                if (lev + 1 < nz) fl += f[lev + 1] * ((double)p[rowoff + lvl + i] - pc);
                if (lev > 0) fl -= f[lev] * (pc - (double)p[rowoff - lvl + i]);
                vert = fl / D[lev];
            } else {
                const double zc = pc / D[lev];
                vert = 0.0;
                if (lev + 1 < nz) vert += f[lev + 1] * ((double)p[rowoff + lvl + i] / D[lev + 1] - zc);
                if (lev > 0) vert -= f[lev] * (zc - (double)p[rowoff - lvl + i] / D[lev - 1]);
            }
            v[h] = (double)bsrc[rowoff + i] - (lap + vert);
        }
        a[t] = C{(T)v[0], (T)v[1]};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r = wv; r < nr; r += nw) {
        double s = 0.0;
        for (int n = lane; n < L; n += 64) {
            C z = a[r * L + n];
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
            C z0 = zr[0];
            X = C{z0.x + z0.y, z0.x - z0.y};
        } else {
            C zk = zr[kx], zc = cconj(zr[L - kx]);
            C e = C{T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
            C d = csub(zk, zc);
            C o = C{T(0.5) * d.y, T(-0.5) * d.x};
            X = cadd(e, cmul(o, sws[kx]));
        }
        const int g = row0 + r;
        const int lev = g / ny, j = g - lev * ny;
        spec[((size_t)lev * L + kx) * ny + j] = X;
    }
}

// ---------------------------------------------------------------- kernels
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_x(const T *__restrict__ in, cx_t<T> *__restrict__ spec,
                                               double *__restrict__ rowsum, int nx, int ny,
                                               int nrows_total, int rows, StagePlan sp,
                                               const cx_t<T> *__restrict__ twx,
                                               const cx_t<T> *__restrict__ tws)
{
    extern __shared__ __align__(16) unsigned char smem[];
    fwd_x_tile<T>(in, spec, rowsum, nx, ny, nrows_total, rows, blockIdx.x * rows, sp, twx, tws,
                  smem);
}

template <typename T, int DIR>
__global__ __launch_bounds__(256) void k_fft_y(cx_t<T> *__restrict__ spec, int nrows_total, int ny,
                                               int rows, StagePlan sp,
                                               const cx_t<T> *__restrict__ twy, int L, int kxlo,
                                               int kxcnt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    fft_y_tile<T, DIR>(spec, nrows_total, ny, rows, blockIdx.x * rows, sp, twy, L, kxlo, kxcnt,
                       smem);
}

template <typename T>
__global__ __launch_bounds__(256) void k_inv_x(const cx_t<T> *__restrict__ spec, T *__restrict__ out,
                                               int nx, int ny, int nrows_total, int rows,
                                               int accumulate, StagePlan sp,
                                               const cx_t<T> *__restrict__ twx,
                                               const cx_t<T> *__restrict__ tws)
{
    extern __shared__ __align__(16) unsigned char smem[];
    inv_x_tile<T>(spec, out, nx, ny, nrows_total, rows, blockIdx.x * rows, accumulate, sp, twx,
                  tws, smem);
}

// ---------------------------------------------------------------- launchers
static inline size_t lds_x(int rows, int L, size_t csz) { return (size_t)(2 * rows * L + 2 * L) * csz; }
static inline size_t lds_y(int rows, int ny, size_t csz) { return (size_t)(2 * rows * ny + ny) * csz; }

template <typename T>
hipError_t launch_fwd_x(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                        const FftGeom &g, const StagePlan &spx, const Tables<T> &tb, hipStream_t st)
{
    const int total = ny * nz, L = nx / 2;
    const int grid = (total + g.rows_x - 1) / g.rows_x;
    hipLaunchKernelGGL(k_fwd_x<T>, dim3(grid), dim3(256), lds_x(g.rows_x, L, sizeof(cx_t<T>)), st,
                       in, spec, rowsum, nx, ny, total, g.rows_x, spx, tb.tw_x, tb.tw_s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fwd_x_residual(const T *b, const T *p, cx_t<T> *spec, double *rowsum, int nx,
                                 int ny, int nz, double idx2, double idy2, const double *f,
                                 const double *D, int adjoint, const FftGeom &g,
                                 const StagePlan &spx, const Tables<T> &tb, hipStream_t st)
{
    const int total = ny * nz, L = nx / 2;
    const int grid = (total + g.rows_x - 1) / g.rows_x;
    hipLaunchKernelGGL(k_fwd_x_residual<T>, dim3(grid), dim3(256),
                       lds_x(g.rows_x, L, sizeof(cx_t<T>)), st, b, p, spec, rowsum, nx, ny, nz,
                       g.rows_x, idx2, idy2, f, D, adjoint, spx, tb.tw_x, tb.tw_s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y(cx_t<T> *spec, int nz, int L, int kxlo, int kxcnt, int ny, int dir,
                        const FftGeom &g, const StagePlan &spy, const Tables<T> &tb,
                        hipStream_t st)
{
    const int nrows = nz * kxcnt;
    if (nrows <= 0) return hipSuccess;
    const int grid = (nrows + g.rows_y - 1) / g.rows_y;
    const size_t lds = lds_y(g.rows_y, ny, sizeof(cx_t<T>));
    if (dir < 0)
        hipLaunchKernelGGL((k_fft_y<T, -1>), dim3(grid), dim3(256), lds, st, spec, nrows, ny,
                           g.rows_y, spy, tb.tw_y, L, kxlo, kxcnt);
    else
        hipLaunchKernelGGL((k_fft_y<T, 1>), dim3(grid), dim3(256), lds, st, spec, nrows, ny,
                           g.rows_y, spy, tb.tw_y, L, kxlo, kxcnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_inv_x(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int accumulate,
                        const FftGeom &g, const StagePlan &spx, const Tables<T> &tb,
                        hipStream_t st)
{
    const int total = ny * nz, L = nx / 2;
    const int grid = (total + g.rows_x - 1) / g.rows_x;
    hipLaunchKernelGGL(k_inv_x<T>, dim3(grid), dim3(256), lds_x(g.rows_x, L, sizeof(cx_t<T>)), st,
                       spec, out, nx, ny, total, g.rows_x, accumulate, spx, tb.tw_x, tb.tw_s);
    return hipGetLastError();
}

#define PS_INST(T)                                                                                 \
    template hipError_t launch_fwd_x<T>(const T *, cx_t<T> *, double *, int, int, int,           \
                                        const FftGeom &, const StagePlan &, const Tables<T> &,    \
                                        hipStream_t);                                             \
    template hipError_t launch_fwd_x_residual<T>(const T *, const T *, cx_t<T> *, double *, int,  \
                                                 int, int, double, double, const double *,       \
                                                 const double *, int, const FftGeom &,           \
                                                 const StagePlan &, const Tables<T> &,           \
                                                 hipStream_t);                                    \
    template hipError_t launch_fft_y<T>(cx_t<T> *, int, int, int, int, int, int,                 \
                                        const FftGeom &, const StagePlan &, const Tables<T> &,    \
                                        hipStream_t);                                             \
    template hipError_t launch_inv_x<T>(const cx_t<T> *, T *, int, int, int, int, const FftGeom &, \
                                        const StagePlan &, const Tables<T> &, hipStream_t);
PS_INST(float)
PS_INST(double)
#undef PS_INST

} // namespace ps
