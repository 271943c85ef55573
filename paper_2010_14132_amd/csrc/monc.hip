// x passes for fields in MONC's own layout, p%data(z,y,x): Fortran order
// with z fastest (whole columns contiguous, the layout the paper's solver
// receives its source term in and returns the pressure in, Section 2.2), so
// element (i, j, k) sits at (i ny + j) nz + k.
//
// The forward pass reads such a field and writes the same packed,
// transposed spectrum spec[k][kx][ky] as the level-major x pass (so the y
// passes and the column solves are shared), and the backward pass reads the
// spectrum and writes the field back in the z-fastest layout: the
// transposes between the column layout and the transform rows happen in LDS
// inside the x passes, with no pass of their own (the paper's closing remark
// about not going back to a column decomposition through extra transposes).
//
// A block takes a tile of rows (k, j), k in [k0, k0 + KC), j in [j0, j0 + JC):
// its loads run along z (KC consecutive values per (i, j)), its spectrum
// stores along ky (JC consecutive values per (k, kx)).  Tiles with the same
// j and neighbouring k are consecutive in the tile order, and with the
// XCD-contiguous map they meet in one L2, so a cache line of the z-fastest
// field is fetched once for the few tiles that share it.
#include <algorithm>

#include "ps_internal.h"
#include "ps_tiles.h"

namespace ps {

template <typename T>
__global__ __launch_bounds__(256) void k_fwd_x_zyx(const T *__restrict__ in,
                                                   cx_t<T> *__restrict__ spec,
                                                   double *__restrict__ rowsum, int nx, int ny,
                                                   int nz, int KC, int JC, int nkc,
                                                   StagePlan sp, const cx_t<T> *__restrict__ twx,
                                                   const cx_t<T> *__restrict__ tws)
{
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = nx >> 1;
    const int rows = KC * JC;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * L;
    C *stw = b + rows * L;
    C *sws = stw + L;
    const int tile = tile_of(blockIdx.x, gridDim.x, 1);
    const int kc = tile % nkc, jc = tile / nkc;
    const int k0 = kc * KC, j0 = jc * JC;
    const int nk = min(KC, nz - k0), nj = min(JC, ny - j0), nr = nk * nj;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        stw[t] = twx[t];
        sws[t] = tws[t];
    }
    // row r = jj nk + kk holds x of level k0 + kk, row j0 + jj, as L complex
    // pairs (x_{2n}, x_{2n+1}); loads run along z
    T *ar = reinterpret_cast<T *>(a);
    const int nload = nx * nr;
    for (int t = threadIdx.x; t < nload; t += blockDim.x) {
        const int kk = t % nk, rest = t / nk;
        const int jj = rest % nj, i = rest / nj;
        ar[(jj * nk + kk) * nx + i] = in[((size_t)i * ny + (j0 + jj)) * nz + (k0 + kk)];
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
        const int jj = r / nk, kk = r - jj * nk;
        if (lane == 0) rowsum[(size_t)(k0 + kk) * ny + (j0 + jj)] = s;
    }
    C *Z = stockham_rows<-1>(a, b, nr, L, sp, stw);
    // even/odd split (slot 0: X_0 + i X_{nx/2}); stores run along ky
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int jj = t % nj, rest = t / nj;
        const int kk = rest % nk, kx = rest / nk;
        const C *zr = Z + (jj * nk + kk) * L;
        C X;
        if (kx == 0) {
            const C z0 = zr[0];
            X = C{z0.x + z0.y, z0.x - z0.y};
        } else {
            const C zk = zr[kx], zc = cconj(zr[L - kx]);
            const C e = C{T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
            const C d = csub(zk, zc);
            const C o = C{T(0.5) * d.y, T(-0.5) * d.x};
            X = cadd(e, cmul(o, sws[kx]));
        }
        spec[((size_t)(k0 + kk) * L + kx) * ny + (j0 + jj)] = X;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_inv_x_zyx(const cx_t<T> *__restrict__ spec,
                                                   T *__restrict__ out, int nx, int ny, int nz,
                                                   int KC, int JC, int nkc, StagePlan sp,
                                                   const cx_t<T> *__restrict__ twx,
                                                   const cx_t<T> *__restrict__ tws,
                                                   int accumulate)
{
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = nx >> 1;
    const int rows = KC * JC;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * L;
    C *stw = b + rows * L;
    C *sws = stw + L;
    const int tile = tile_of(blockIdx.x, gridDim.x, 1);
    const int kc = tile % nkc, jc = tile / nkc;
    const int k0 = kc * KC, j0 = jc * JC;
    const int nk = min(KC, nz - k0), nj = min(JC, ny - j0), nr = nk * nj;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        stw[t] = twx[t];
        sws[t] = tws[t];
    }
    // gather the rows from the spectrum (loads run along ky)
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int jj = t % nj, rest = t / nj;
        const int kk = rest % nk, kx = rest / nk;
        a[(jj * nk + kk) * L + kx] = spec[((size_t)(k0 + kk) * L + kx) * ny + (j0 + jj)];
    }
    __syncthreads();
    // undo the packing: Z_k = (X_k + conj X_{L-k}) + i W_nx^{-k} (X_k - conj X_{L-k})
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int r = t / L, k = t - r * L;
        const C *xr = a + r * L;
        C Zv;
        if (k == 0) {
            const T x0 = xr[0].x, xl = xr[0].y;
            Zv = C{x0 + xl, x0 - xl};
        } else {
            const C xk = xr[k], xc = cconj(xr[L - k]);
            const C s = cadd(xk, xc);
            const C dw = cmul(csub(xk, xc), cconj(sws[k]));
            Zv = C{s.x - dw.y, s.y + dw.x};
        }
        b[t] = Zv;
    }
    __syncthreads();
    const C *R = stockham_rows<1>(b, a, nr, L, sp, stw);
    const T *rr = reinterpret_cast<const T *>(R);
    // stores (or accumulations) run along z
    const int nst = nx * nr;
    for (int t = threadIdx.x; t < nst; t += blockDim.x) {
        const int kk = t % nk, rest = t / nk;
        const int jj = rest % nj, i = rest / nj;
        T *o = out + ((size_t)i * ny + (j0 + jj)) * nz + (k0 + kk);
        const T val = rr[(jj * nk + kk) * nx + i];
        *o = accumulate ? *o + val : val;
    }
}

// r = b - A p at every point of z-fastest fields, one thread per point in
// storage order (loads along k): the 7-point operator with periodic x and y
// neighbours and the vertical coefficients rc (3 per level: upper, lower,
// centre; zero at the top and bottom faces, where the missing neighbour is
// read as the point itself), FP64 accumulation in the same order as the
// level-major residual transform, rounded once.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_zyx(const T *__restrict__ b,
                                                      const T *__restrict__ p, T *__restrict__ r,
                                                      int nx, int ny, int nz, double idx2,
                                                      double idy2, const double *__restrict__ rc)
{
    const unsigned n = (unsigned)nx * (unsigned)ny * (unsigned)nz; // < 2^31
    const unsigned jstride = (unsigned)nz, istride = (unsigned)ny * (unsigned)nz;
    for (unsigned c = blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += gridDim.x * blockDim.x) {
        const unsigned k = c % (unsigned)nz, rest = c / (unsigned)nz;
        const unsigned j = rest % (unsigned)ny, i = rest / (unsigned)ny;
        const double pc = (double)p[c];
        const double pe = (double)p[i + 1 == (unsigned)nx ? c - i * istride : c + istride];
        const double pw = (double)p[i == 0 ? c + ((unsigned)nx - 1) * istride : c - istride];
        const double pn = (double)p[j + 1 == (unsigned)ny ? c - j * jstride : c + jstride];
        const double ps = (double)p[j == 0 ? c + ((unsigned)ny - 1) * jstride : c - jstride];
        const double pu = k + 1 < (unsigned)nz ? (double)p[c + 1] : pc;
        const double pd = k > 0 ? (double)p[c - 1] : pc;
        const double lap = ((pe - 2.0 * pc + pw) * idx2 + (pn - 2.0 * pc + ps) * idy2 +
                            rc[3 * k] * pu + rc[3 * k + 1] * pd - rc[3 * k + 2] * pc);
        r[c] = (T)((double)b[c] - lap);
    }
}

static inline size_t lds_rows(int rows, int L, size_t csz) { return (size_t)(2 * rows * L + 2 * L) * csz; }

// Rows per tile split as KC levels x JC rows for a tile of `rows` rows.
static inline void zyx_tile(int rows, int kc_pref, int nz, int *KC, int *JC)
{
    int kc = std::max(1, std::min(std::min(kc_pref, rows), nz));
    *KC = kc;
    *JC = std::max(1, rows / kc);
}

template <typename T>
hipError_t launch_fwd_x_zyx(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                            int rows, int kc_pref, const StagePlan &spx, const Tables<T> &tb,
                            hipStream_t st)
{
    int KC, JC;
    zyx_tile(rows, kc_pref, nz, &KC, &JC);
    const int nkc = (nz + KC - 1) / KC, njc = (ny + JC - 1) / JC;
    hipLaunchKernelGGL(k_fwd_x_zyx<T>, dim3(nkc * njc), dim3(256),
                       lds_rows(KC * JC, nx / 2, sizeof(cx_t<T>)), st, in, spec, rowsum, nx, ny,
                       nz, KC, JC, nkc, spx, tb.tw_x, tb.tw_s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_inv_x_zyx(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int rows,
                            int kc_pref, const StagePlan &spx, const Tables<T> &tb,
                            hipStream_t st, int accumulate)
{
    int KC, JC;
    zyx_tile(rows, kc_pref, nz, &KC, &JC);
    const int nkc = (nz + KC - 1) / KC, njc = (ny + JC - 1) / JC;
    hipLaunchKernelGGL(k_inv_x_zyx<T>, dim3(nkc * njc), dim3(256),
                       lds_rows(KC * JC, nx / 2, sizeof(cx_t<T>)), st, spec, out, nx, ny, nz, KC,
                       JC, nkc, spx, tb.tw_x, tb.tw_s, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual_zyx(const T *b, const T *p, T *r, int nx, int ny, int nz, double idx2,
                               double idy2, const double *rc, hipStream_t st)
{
    const long n = (long)nx * ny * nz;
    const int grid = (int)std::min<long>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_residual_zyx<T>, dim3(grid), dim3(256), 0, st, b, p, r, nx, ny, nz, idx2,
                       idy2, rc);
    return hipGetLastError();
}

template hipError_t launch_fwd_x_zyx<float>(const float *, cx_t<float> *, double *, int, int, int,
                                            int, int, const StagePlan &, const Tables<float> &,
                                            hipStream_t);
template hipError_t launch_fwd_x_zyx<double>(const double *, cx_t<double> *, double *, int, int,
                                             int, int, int, const StagePlan &,
                                             const Tables<double> &, hipStream_t);
template hipError_t launch_inv_x_zyx<float>(const cx_t<float> *, float *, int, int, int, int, int,
                                            const StagePlan &, const Tables<float> &, hipStream_t,
                                            int);
template hipError_t launch_inv_x_zyx<double>(const cx_t<double> *, double *, int, int, int, int,
                                             int, const StagePlan &, const Tables<double> &,
                                             hipStream_t, int);
template hipError_t launch_residual_zyx<float>(const float *, const float *, float *, int, int,
                                               int, double, double, const double *, hipStream_t);
template hipError_t launch_residual_zyx<double>(const double *, const double *, double *, int,
                                                int, int, double, double, const double *,
                                                hipStream_t);

} // namespace ps
