// Column solves of the pressure solve (paper Section 2.1: after the forward
// transform every horizontal wavenumber carries an independent vertical
// tridiagonal system, solved up and down its column), the singular mean
// column, and the density gradient.
//
// Per wavenumber (kx, ky) != (0, 0), with s = ax[kx] + ay[ky] > 0, the
// scaled system is M x = r with
//   M = tridiag(-f_{k-1/2}, s D_k + f_{k-1/2} + f_{k+1/2}, -f_{k+1/2}),
//   r_k = rs_k * spectrum_k  (rs_k = -D_k/(nx ny) forward, -1/(nx ny) adjoint),
// and the spectrum is overwritten by os_k * x_k (os_k = 1 forward, D_k adjoint).
// M is a symmetric, diagonally dominant M-matrix.  It is eliminated from both
// ends towards the middle row m = nz/2 (a "twisted" factorisation), each half
// in dominance-excess form (pivot u = e + f_next with
// e_i = s D_i + f_prev e_{i-1}/u_{i-1}, built from positive terms only).
#include <algorithm>

#include "ps_internal.h"
#include "ps_tiles.h"
#include "../../include/pressure_solve.h"

namespace ps {

// ----------------------------------------------------------- twisted sweep
// v holds the thread's half of the right-hand side in elimination order
// (low half: levels 0..m-1; high half: levels nz-1 down to m+1); on return
// it holds the solution for those levels.  rm is the middle row's
// right-hand side.  Both lanes of a column pair (lane and lane ^ 32) return
// the same x_m.  Pivots are recomputed block by block (CH rows) in the
// backward pass from checkpoints of the recursion state instead of being
// kept in registers.
template <typename T, int NH, int CH>
__device__ __forceinline__ T twisted_solve(T (&v)[NH], int n, int half, int m, int nz, T s,
                                           const T *sf, const T *sD, T rm)
{
    constexpr int NB = (NH + CH - 1) / CH;
    T qck[NB];
    T q = T(0), g = T(0), y = T(0);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i % CH == 0) qck[i / CH] = q;
        if (i < n) {
            const int k = half ? nz - 1 - i : i;
            const T fp = half ? sf[k + 1] : sf[k];
            const T fn = half ? sf[k] : sf[k + 1];
            const T e = s * sD[k] + fp * q;
            const T gi = T(1) / (e + fn);
            y = v[i] + (fp * g) * y;
            v[i] = y;
            q = e * gi;
            g = gi;
        }
    }
    T ma = T(0), mb = T(0);
    if (n > 0) {
        const int kl = half ? nz - n : n - 1;
        const T fn = half ? sf[kl] : sf[kl + 1];
        ma = fn * q;
        mb = (fn * g) * y;
    }
    const T pa = __shfl_xor(ma, 32, 64), pb = __shfl_xor(mb, 32, 64);
    const T la = half ? pa : ma, lb = half ? pb : mb;
    const T ha = half ? ma : pa, hb = half ? mb : pb;
    const T xm = ((rm + lb) + hb) / ((s * sD[m] + la) + ha);

    T xn = xm;
#pragma unroll
    for (int bb = NB - 1; bb >= 0; --bb) {
        if (bb * CH < n) {
            T gb[CH];
            T qq = qck[bb];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = bb * CH + c;
                if (i < n && i < NH) {
                    const int k = half ? nz - 1 - i : i;
                    const T fp = half ? sf[k + 1] : sf[k];
                    const T fn = half ? sf[k] : sf[k + 1];
                    const T e = s * sD[k] + fp * qq;
                    const T gi = T(1) / (e + fn);
                    gb[c] = gi;
                    qq = e * gi;
                }
            }
#pragma unroll
            for (int c = CH - 1; c >= 0; --c) {
                const int i = bb * CH + c;
                if (i < n && i < NH) {
                    const int k = half ? nz - 1 - i : i;
                    const T fn = half ? sf[k] : sf[k + 1];
                    xn = gb[c] * (v[i] + fn * xn);
                    v[i] = xn;
                }
            }
        }
    }
    return xm;
}

// ----------------------------------------------------------- main columns
// Four lanes per column: lane = half*32 + 2*c + comp (comp: real/imaginary,
// half: low/high part of the column).  A wavefront covers 16 consecutive
// columns (consecutive ky), so each level's load is two contiguous 128-byte
// runs (FP32).  Columns kx = 0 are left to k_special.  Columns flagged in
// maskcnt (min(ky, ny-ky) < maskcnt[kx]) are computed but not stored: they
// are solved in FP64 by k_special.
// REFINE: one refinement of M x = r with the residual formed in FP64 from the
// FP64 coefficients (ax64/ay64/f64/D64), solved with the same FP32 sweep.
template <typename T, int NH, int CH, bool REFINE>
__global__ __launch_bounds__(256) void k_columns(cx_t<T> *__restrict__ spec, int L, int ny, int nz,
                                                 const T *__restrict__ ax, const T *__restrict__ ay,
                                                 const T *__restrict__ fg, const T *__restrict__ Dg,
                                                 const T *__restrict__ rsg,
                                                 const T *__restrict__ osg,
                                                 const int *__restrict__ maskcnt,
                                                 const double *__restrict__ ax64,
                                                 const double *__restrict__ ay64,
                                                 const double *__restrict__ f64,
                                                 const double *__restrict__ D64,
                                                 const double *__restrict__ rs64, long c0,
                                                 long c1)
{
    __shared__ T sf[PS_MAX_NZ + 1], sD[PS_MAX_NZ], srs[PS_MAX_NZ], sos[PS_MAX_NZ];
    __shared__ double df[REFINE ? PS_MAX_NZ + 1 : 1], dD[REFINE ? PS_MAX_NZ : 1],
        drs[REFINE ? PS_MAX_NZ : 1];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) {
        sf[t] = fg[t];
        if (REFINE) df[t] = f64[t];
        if (t < nz) {
            sD[t] = Dg[t];
            srs[t] = rsg[t];
            sos[t] = osg ? osg[t] : T(1);
            if (REFINE) {
                dD[t] = D64[t];
                drs[t] = rs64[t];
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, comp = lane & 1, cl = (lane & 31) >> 1;
    const long col = c0 + ((long)blockIdx.x * 4 + wave) * 16 + cl;
    const bool valid = col < c1;
    const int kx = valid ? (int)((unsigned)col / (unsigned)ny) : 1; // col < 2^31
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const T s = ax[kx] + ay[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    const size_t ls = (size_t)2 * L * ny;
    T *cp = reinterpret_cast<T *>(spec) + 2 * (valid ? col : 0) + comp;
    const int m = nz >> 1;
    const int n = half ? nz - 1 - m : m;

    T raw[REFINE ? NH : 1];
    T v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i < n) {
            const int k = half ? nz - 1 - i : i;
            const T x = valid ? cp[(size_t)k * ls] : T(0);
            if (REFINE) raw[i] = x;
            v[i] = x * srs[k];
        }
    }
    const T rawm = valid ? cp[(size_t)m * ls] : T(0);
    T xm = twisted_solve<T, NH, CH>(v, n, half, m, nz, s, sf, sD, rawm * srs[m]);

    if constexpr (REFINE) {
        // residual rho = r - M x in FP64, r = rs * spectrum formed in FP64
        const double s64 = ax64[kx] + ay64[ky];
        T mylast = T(0); // v[n-1], selected without dynamic indexing
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (i == n - 1) mylast = v[i];
        const T other = __shfl_xor(mylast, 32, 64);
        const double xlo = half ? (double)other : (double)mylast; // x_{m-1}
        const double xhi = half ? (double)mylast : (double)other; // x_{m+1}
        // the residual overwrites the stored right-hand side in place
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            if (i < n) {
                const int k = half ? nz - 1 - i : i;
                const double fp = half ? df[k + 1] : df[k];
                const double fn = half ? df[k] : df[k + 1];
                const double xp = i > 0 ? (double)v[i - 1] : 0.0;
                const double xnx = i + 1 < n ? (double)v[i + 1] : (double)xm;
                const double diag = s64 * dD[k] + df[k] + df[k + 1];
                const double r = drs[k] * (double)raw[i];
                raw[i] = (T)(r - (diag * (double)v[i] - fp * xp - fn * xnx));
            }
        }
        const double diagm = s64 * dD[m] + df[m] + df[m + 1];
        const double rmid = drs[m] * (double)rawm;
        const T dm = (T)(rmid - (diagm * (double)xm - df[m] * xlo - df[m + 1] * xhi));
        const T em = twisted_solve<T, NH, CH>(raw, n, half, m, nz, s, sf, sD, dm);
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (i < n) v[i] += raw[i];
        xm += em;
    }

    if (store) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            if (i < n) {
                const int k = half ? nz - 1 - i : i;
                cp[(size_t)k * ls] = v[i] * sos[k];
            }
        }
        if (half) cp[(size_t)m * ls] = xm * sos[m];
    }
}

// ----------------------------------------------------------- complex sweep
// Same two-ended elimination as twisted_solve, with one lane per half column
// carrying the complex right-hand side (real and imaginary parts share the
// real pivots, so each pivot is computed once per lane).  KEEPG keeps the
// reciprocal pivots in registers for the backward pass instead of recomputing
// them from checkpoints.
template <typename T, int NH, int CH, bool KEEPG>
__device__ __forceinline__ cx_t<T> twisted_solve_c(cx_t<T> (&v)[NH], int n, int half, int m,
                                                   int nz, T s, const T *sf, const T *sD,
                                                   cx_t<T> rm)
{
    using C = cx_t<T>;
    constexpr int NB = (NH + CH - 1) / CH;
    T qck[KEEPG ? 1 : NB];
    T gk[KEEPG ? NH : 1];
    T q = T(0), g = T(0);
    C y = C{T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (!KEEPG && i % CH == 0) qck[i / CH] = q;
        if (i < n) {
            const int k = half ? nz - 1 - i : i;
            const T fp = half ? sf[k + 1] : sf[k];
            const T fn = half ? sf[k] : sf[k + 1];
            const T e = s * sD[k] + fp * q;
            const T gi = T(1) / (e + fn);
            const T c = fp * g;
            y = C{v[i].x + c * y.x, v[i].y + c * y.y};
            v[i] = y;
            q = e * gi;
            g = gi;
            if (KEEPG) gk[i] = gi;
        }
    }
    T ma = T(0);
    C mb = C{T(0), T(0)};
    if (n > 0) {
        const int kl = half ? nz - n : n - 1;
        const T fn = half ? sf[kl] : sf[kl + 1];
        ma = fn * q;
        mb = C{(fn * g) * y.x, (fn * g) * y.y};
    }
    const T pa = __shfl_xor(ma, 32, 64);
    const C pb = C{__shfl_xor(mb.x, 32, 64), __shfl_xor(mb.y, 32, 64)};
    const T la = half ? pa : ma, ha = half ? ma : pa;
    const C lb = half ? pb : mb, hb = half ? mb : pb;
    const T den = (s * sD[m] + la) + ha;
    const C xm = C{((rm.x + lb.x) + hb.x) / den, ((rm.y + lb.y) + hb.y) / den};

    C xn = xm;
    if constexpr (KEEPG) {
#pragma unroll
        for (int i = NH - 1; i >= 0; --i) {
            if (i < n) {
                const int k = half ? nz - 1 - i : i;
                const T fn = half ? sf[k] : sf[k + 1];
                xn = C{gk[i] * (v[i].x + fn * xn.x), gk[i] * (v[i].y + fn * xn.y)};
                v[i] = xn;
            }
        }
    } else {
#pragma unroll
        for (int bb = NB - 1; bb >= 0; --bb) {
            if (bb * CH < n) {
                T gb[CH];
                T qq = qck[bb];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int i = bb * CH + c;
                    if (i < n && i < NH) {
                        const int k = half ? nz - 1 - i : i;
                        const T fp = half ? sf[k + 1] : sf[k];
                        const T fn = half ? sf[k] : sf[k + 1];
                        const T e = s * sD[k] + fp * qq;
                        const T gi = T(1) / (e + fn);
                        gb[c] = gi;
                        qq = e * gi;
                    }
                }
#pragma unroll
                for (int c = CH - 1; c >= 0; --c) {
                    const int i = bb * CH + c;
                    if (i < n && i < NH) {
                        const int k = half ? nz - 1 - i : i;
                        const T fn = half ? sf[k] : sf[k + 1];
                        xn = C{gb[c] * (v[i].x + fn * xn.x), gb[c] * (v[i].y + fn * xn.y)};
                        v[i] = xn;
                    }
                }
            }
        }
    }
    return xm;
}

// Two lanes per column (lane = half * 32 + c): a wavefront covers 32
// consecutive columns, so each level's load is two contiguous 256-byte runs
// (FP32 complex).  Otherwise as k_columns (no in-register refinement).
template <typename T, int NH, int CH, bool KEEPG>
__global__ __launch_bounds__(256) void k_columns2(cx_t<T> *__restrict__ spec, int L, int ny, int nz,
                                                  const T *__restrict__ ax,
                                                  const T *__restrict__ ay,
                                                  const T *__restrict__ fg,
                                                  const T *__restrict__ Dg,
                                                  const T *__restrict__ rsg,
                                                  const T *__restrict__ osg,
                                                  const int *__restrict__ maskcnt, long c0,
                                                  long c1)
{
    using C = cx_t<T>;
    __shared__ T sf[PS_MAX_NZ + 1], sD[PS_MAX_NZ], srs[PS_MAX_NZ], sos[PS_MAX_NZ];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) {
        sf[t] = fg[t];
        if (t < nz) {
            sD[t] = Dg[t];
            srs[t] = rsg[t];
            sos[t] = osg ? osg[t] : T(1);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, cl = lane & 31;
    const long col = c0 + ((long)blockIdx.x * 4 + wave) * 32 + cl;
    const bool valid = col < c1;
    const int kx = valid ? (int)((unsigned)col / (unsigned)ny) : 1; // col < 2^31
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const T s = ax[kx] + ay[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    const size_t ls = (size_t)L * ny;
    C *cp = spec + (valid ? col : 0);
    const int m = nz >> 1;
    const int n = half ? nz - 1 - m : m;
    C v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i < n) {
            const int k = half ? nz - 1 - i : i;
            const C x = valid ? cp[(size_t)k * ls] : C{T(0), T(0)};
            v[i] = C{x.x * srs[k], x.y * srs[k]};
        }
    }
    const C xr = valid ? cp[(size_t)m * ls] : C{T(0), T(0)};
    const C xm = twisted_solve_c<T, NH, CH, KEEPG>(v, n, half, m, nz, s, sf, sD,
                                                   C{xr.x * srs[m], xr.y * srs[m]});
    if (store) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            if (i < n) {
                const int k = half ? nz - 1 - i : i;
                cp[(size_t)k * ls] = C{v[i].x * sos[k], v[i].y * sos[k]};
            }
        }
        if (half) cp[(size_t)m * ls] = C{xm.x * sos[m], xm.y * sos[m]};
    }
}

// ----------------------------------------------------------- tile kernels
// The uniform-half column sweep and the compact FP64 column tasks (the
// device code is in ps_tiles.h, shared with the batched persistent kernel).
template <typename T, int NH, bool KEEPG>
__global__ __launch_bounds__(256) void k_columns3(cx_t<T> *__restrict__ spec, int L, int ny,
                                                  const T *__restrict__ ax,
                                                  const T *__restrict__ ay,
                                                  const LevelCoef<T> *__restrict__ coef,
                                                  const int *__restrict__ maskcnt, long c0,
                                                  long c1)
{
    __shared__ T xa[2][2][64];
    __shared__ cx_t<T> xb[2][2][64];
    columns3_tile<T, NH, KEEPG>(spec, L, ny, ax, ay, coef, maskcnt, c0, c1, blockIdx.x, xa, xb);
}

template <int NH>
__global__ __launch_bounds__(256) void k_columns3r(float2 *__restrict__ spec, int L, int ny,
                                                   const float *__restrict__ ax,
                                                   const float *__restrict__ ay,
                                                   const LevelCoef<float> *__restrict__ coef,
                                                   const LevelCoef<double> *__restrict__ coef64,
                                                   const double *__restrict__ ax64,
                                                   const double *__restrict__ ay64,
                                                   const int *__restrict__ maskcnt, long c0,
                                                   long c1)
{
    __shared__ float xa[2][2][64];
    __shared__ float2 xb[2][2][64], xe[2][2][64];
    columns3r_tile<NH>(spec, L, ny, ax, ay, coef, coef64, ax64, ay64, maskcnt, c0, c1, blockIdx.x,
                       xa, xb, xe);
}

template <typename T, int NH, bool REFINE, bool SHG, int PPB>
__global__ __launch_bounds__(128 * PPB) void k_columns3s(cx_t<T> *__restrict__ spec, int L, int ny,
                                                   const T *__restrict__ ax,
                                                   const T *__restrict__ ay,
                                                   const LevelCoef<T> *__restrict__ coef,
                                                   const LevelCoef<double> *__restrict__ coef64,
                                                   const double *__restrict__ ax64,
                                                   const double *__restrict__ ay64,
                                                   const int *__restrict__ maskcnt, long c0,
                                                   long c1, int swz)
{
    __shared__ T xa[2][2][64], xb[2][2][64], xe[REFINE ? 2 : 1][2][64];
    __shared__ T gsh[SHG ? 2 * PPB * NH * 32 : 1];
    columns3s_tile<T, NH, REFINE, SHG, PPB>(spec, L, ny, ax, ay, coef, coef64, ax64, ay64, maskcnt,
                                            c0, c1, tile_of(blockIdx.x, gridDim.x, swz), xa, xb,
                                            xe, gsh);
}

// These few waves carry long dependent chains and usually share their SIMDs
// with the main column kernel: they are issued first (wave priority).
template <typename T, int U>
__global__ __launch_bounds__(64) void k_special_seq(
    cx_t<T> *__restrict__ spec, int nx, int ny, int nz, int adjoint, const int *__restrict__ mlist,
    int nmask, const double *__restrict__ S, double *__restrict__ ws,
    const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ fg,
    const double *__restrict__ Dg, const double *__restrict__ rsg, const double *__restrict__ osg)
{
    __builtin_amdgcn_s_setprio(3);
    __shared__ double f[PS_MAX_NZ + 1], D[PS_MAX_NZ], rs[PS_MAX_NZ], os[PS_MAX_NZ],
        sS[PS_MAX_NZ];
    for (int i = threadIdx.x; i <= nz; i += blockDim.x) {
        f[i] = fg[i];
        if (i < nz) {
            D[i] = Dg[i];
            rs[i] = rsg[i];
            os[i] = osg ? osg[i] : 1.0;
            sS[i] = S[i];
        }
    }
    __syncthreads();
    special_seq_tile<T, U>(spec, nx, ny, nz, adjoint, mlist, nmask, ws, ax, ay, f, D, rs, os, sS,
                           blockIdx.x * blockDim.x + threadIdx.x);
}

// LDS-staged form of the FP64 column tasks.  A block takes G consecutive
// tasks: it loads every level of their columns into LDS in one batch, solves
// the same systems as special_seq_tile (the A and B systems of a packed-row
// pair, a near-singular column's one system) with the eliminated values and
// reciprocal pivots kept in LDS instead of the HBM workspace, and stores
// every level in one batch.  The sweeps are latency-bound -- a few lanes per
// block, one dependent chain per system, one wave per SIMD issuing -- so the
// work on the chain is cut to the recurrence itself:
//  - each system is eliminated from both ends toward its middle level m by
//    two lanes (the chain is about nz/2 levels);
//  - a parallel pass over all threads first forms every system's
//    right-hand side and s D_k, and writes them into one row per (system,
//    half) in step order, so consecutive steps of a lane sit at constant
//    offsets (no address arithmetic per level), with the faces toward the end
//    and toward the middle of each half's steps in a shared row;
//  - both halves run the same number of steps, a whole number of chunks:
//    each half starts with inert dummy steps at its far end (faces 0, s D
//    = 1, right-hand side 0: y stays 0 and the first real step, a boundary
//    level whose outer face is 0, starts afresh), so no step is guarded;
//  - the next chunk of steps is read into registers (two buffers in turn)
//    before the current chunk is eliminated;
//  - each reciprocal pivot is a refined hardware estimate (fp64_rcp).
// The results agree with special_seq_tile's one-ended sweep to rounding.
constexpr int kSpecialChunk = 8;
struct SpecialLds {
    int NSTEP; // steps per half: m = nz/2 rounded up to whole chunks
    int NS;    // row length: NSTEP + one chunk of read-ahead, odd
    int f, D, rs, os, sS, ff, mc, y, gv, bm, xm, ss, zin, scol, total; // offsets in doubles
};
// LDS of k_special_lds for nz levels, G tasks and complex elements of csize
// bytes, in doubles; every part starts 16-byte aligned.
//   f (nz+1), D, rs, os, sS (nz each)   FP64 tables
//   ff [2][NS] double2                  per half and step: (f toward the
//                                       end, f toward the middle); zero for
//                                       the dummy steps and the read-ahead
//   mc [nz] double2                     the mean column
//   y  [G][2][2][NS] double2            per (task, system, half) row: the
//                                       right-hand side, then y, then x
//   gv [G][2][2][NS] double             s D_k, then the reciprocal pivot
//   bm, xm [G][2] double2               the middle level's right-hand side
//                                       and solution
//   ss [G][2] double                    s of each system
//   zin [nz][2][G] complex T            the loaded columns
//   scol [2][G] int                     the columns (index 0: Z_ky / the
//                                       column, 1: Z_-ky / the column)
// ff, y and gv are preceded by two chunks of padding, so the read-ahead of a
// row's first or last chunk stays inside the allocation.
__host__ __device__ inline SpecialLds special_lds_layout(int nz, int G, int csize)
{
    SpecialLds l{};
    l.NSTEP = ((nz >> 1) + kSpecialChunk - 1) / kSpecialChunk * kSpecialChunk;
    int ns = l.NSTEP + kSpecialChunk;
    if (!(ns & 1)) ++ns;
    l.NS = ns;
    int o = 0;
    auto take = [&o](int n) {
        const int r = o;
        o += (n + 1) & ~1;
        return r;
    };
    const int pad2 = 2 * 2 * kSpecialChunk; // two chunks of double2
    l.f = take(nz + 1);
    l.D = take(nz);
    l.rs = take(nz);
    l.os = take(nz);
    l.sS = take(nz);
    l.ff = take(pad2 + 2 * ns * 2) + pad2;
    l.mc = take(2 * nz);
    l.y = take(pad2 + 4 * G * ns * 2) + pad2;
    l.gv = take(2 * kSpecialChunk + 4 * G * ns) + 2 * kSpecialChunk;
    l.bm = take(2 * G * 2);
    l.xm = take(2 * G * 2);
    l.ss = take(2 * G);
    l.zin = take((nz * 2 * G * csize + 7) / 8);
    l.scol = take((2 * G + 1) / 2);
    l.total = o;
    return l;
}

template <typename T>
__global__ __launch_bounds__(256) void k_special_lds(
    cx_t<T> *__restrict__ spec, int nx, int ny, int nz, int adjoint, const int *__restrict__ mlist,
    int nmask, const double *__restrict__ S, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ fg, const double *__restrict__ Dg,
    const double *__restrict__ rsg, const double *__restrict__ osg, int G)
{
    using C = cx_t<T>;
    constexpr int CH = kSpecialChunk;
    __builtin_amdgcn_s_setprio(3);
    extern __shared__ __align__(16) double sm[];
    const int L = nx / 2, npair = ny / 2 + 1, ntask = npair + nmask;
    const size_t lvl = (size_t)L * ny;
    const SpecialLds ly = special_lds_layout(nz, G, (int)sizeof(C));
    const int NS = ly.NS, m = nz >> 1;
    double *f = sm + ly.f, *D = sm + ly.D, *rs = sm + ly.rs, *os = sm + ly.os, *sS = sm + ly.sS;
    double2 *FF = reinterpret_cast<double2 *>(sm + ly.ff);
    double2 *MC = reinterpret_cast<double2 *>(sm + ly.mc);
    double2 *Y = reinterpret_cast<double2 *>(sm + ly.y);
    double *GV = sm + ly.gv;
    double2 *BM = reinterpret_cast<double2 *>(sm + ly.bm);
    double2 *XM = reinterpret_cast<double2 *>(sm + ly.xm);
    double *SS = sm + ly.ss;
    C *zin = reinterpret_cast<C *>(sm + ly.zin);
    int *scol = reinterpret_cast<int *>(sm + ly.scol);
    const int t0 = blockIdx.x * G;

    for (int i = threadIdx.x; i <= nz; i += blockDim.x) {
        f[i] = fg[i];
        if (i < nz) {
            D[i] = Dg[i];
            rs[i] = rsg[i];
            os[i] = osg ? osg[i] : 1.0;
            sS[i] = S[i];
        }
    }
    if (threadIdx.x < 2 * G) {
        const int g = threadIdx.x % G, which = threadIdx.x / G;
        const int t = min(t0 + g, ntask - 1);
        scol[threadIdx.x] = t < npair ? (which ? (ny - t) % ny : t) : mlist[t - npair];
    }
    __syncthreads();

    // faces of each half's steps (the real steps of half h are the last
    // nreal_h of the NSTEP); s of each system
    const int NSTEP = ly.NSTEP;
    for (int i = threadIdx.x; i < 2 * NS; i += blockDim.x) {
        const int h = i / NS, st = i - h * NS;
        const int j = st - (NSTEP - (h ? nz - 1 - m : m)); // real step index
        double2 v = double2{0.0, 0.0};
        if (j >= 0 && st < NSTEP) {
            const int k = h ? nz - 1 - j : j;
            v = h ? double2{f[k + 1], f[k]} : double2{f[k], f[k + 1]};
        }
        FF[i] = v;
    }
    if (threadIdx.x < 2 * G) {
        const int g = threadIdx.x >> 1, sys = threadIdx.x & 1, t = t0 + g;
        double sv = 0.0;
        if (t < npair) {
            sv = sys ? ax[L] + ay[t] : ay[t];
        } else if (t < ntask) {
            const int c = scol[g], kx = c / ny, ky = c - kx * ny;
            sv = ax[kx] + ay[ky];
        }
        SS[threadIdx.x] = sv;
    }
    // one batch of loads: UNR per thread in flight before the first is used;
    // indices past the end are clamped (their values are never used)
    constexpr int UNR = 8;
    const int nload = nz * 2 * G;
    for (int base = 0; base < nload; base += UNR * (int)blockDim.x) {
        C v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int i = min(base + u * (int)blockDim.x + (int)threadIdx.x, nload - 1);
            const int g = i % G, r = i / G;
            v[u] = spec[(size_t)(r >> 1) * lvl + scol[(r & 1) * G + g]];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int i = base + u * (int)blockDim.x + (int)threadIdx.x;
            if (i < nload) zin[i] = v[u];
        }
    }
    __syncthreads();

    // every system's right-hand side rs_k (A or B of a pair, A = (Z +
    // conj Zm)/2, B = (Z - conj Zm)/(2i); or the column) and s D_k, into
    // the sweep rows (the middle level apart)
    for (int i = threadIdx.x; i < nload; i += blockDim.x) {
        const int g = i % G, r = i / G, sys = r & 1, k = r >> 1, t = t0 + g;
        const C z0 = zin[(k * 2) * G + g], z1 = zin[(k * 2 + 1) * G + g];
        double ar, ai;
        if (t < npair) {
            const double zr = z0.x, zi = z0.y, mr = z1.x, mi = -(double)z1.y;
            if (sys == 0) {
                ar = 0.5 * (zr + mr);
                ai = 0.5 * (zi + mi);
            } else {
                ar = 0.5 * (zi - mi);
                ai = -0.5 * (zr - mr);
            }
        } else {
            ar = z0.x;
            ai = z0.y;
        }
        const double2 b = double2{rs[k] * ar, rs[k] * ai};
        if (k == m) {
            BM[g * 2 + sys] = b;
        } else {
            const int h = k > m ? 1 : 0;
            const int st = (h ? nz - 1 - k : k) + NSTEP - (h ? nz - 1 - m : m);
            const int row = (g * 2 + sys) * 2 + h;
            Y[row * NS + st] = b;
            GV[row * NS + st] = SS[g * 2 + sys] * D[k];
        }
    }
    // the dummy steps
    for (int i = threadIdx.x; i < 4 * G * CH; i += blockDim.x) {
        const int row = i / CH, st = i - row * CH;
        if (st < NSTEP - ((row & 1) ? nz - 1 - m : m)) {
            Y[row * NS + st] = double2{0.0, 0.0};
            GV[row * NS + st] = 1.0;
        }
    }
    __syncthreads();

    // the sweeps: lanes [0, 4G), four per task -- (system, half), the
    // system A or B of a packed-row pair (a near-singular column has only A)
    // and the half the low levels 0..m-1 or the high levels nz-1..m+1 --
    // eliminated toward the middle level m from both ends at once.  The two
    // halves of a system sit in adjacent lanes and exchange their messages to
    // the middle row with one shuffle.  The mean column (task 0's A) is
    // computed by the block's last wave with scans (4G <= 192, so that wave
    // does no sweep).
    {
        const int lane4 = threadIdx.x;
        const int g = lane4 >> 2, sys = (lane4 >> 1) & 1, half = lane4 & 1, t = t0 + g;
        const bool pair = t < npair;
        const bool active = lane4 < 4 * G && t < ntask && (sys == 0 || pair) &&
                            !(pair && t == 0 && sys == 0);
        const int row = active ? (g * 2 + sys) * 2 + half : 0;
        double2 *Yr = Y + row * NS;
        double *Gr = GV + row * NS;
        const double2 *Fh = FF + half * NS;
        // forward elimination (dominance-excess pivots e_k, reciprocal
        // pivots g_k = 1 / (e_k + fn_k); fp, fn the faces toward the end and
        // toward the middle): e_k = s D_k + fp_k e_{k-1} g_{k-1}, with
        // fp_k = fn_{k-1}
        double e = 0.0, gp = 0.0, fpe = 0.0, yr = 0.0, yi = 0.0;
        auto fw_load = [&](int i0, double2 (&b)[CH], double (&sd)[CH], double2 (&fc)[CH]) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                b[c] = Yr[i0 + c];
                sd[c] = Gr[i0 + c];
                fc[c] = Fh[i0 + c];
            }
        };
        auto fw_step = [&](int i0, const double2 (&b)[CH], const double (&sd)[CH],
                           const double2 (&fc)[CH]) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                e = __builtin_fma(fpe, gp, sd[c]);
                const double gi = fp64_rcp(e + fc[c].y);
                const double cc = fc[c].x * gp;
                yr = __builtin_fma(cc, yr, b[c].x);
                yi = __builtin_fma(cc, yi, b[c].y);
                Yr[i0 + c] = double2{yr, yi};
                Gr[i0 + c] = gi;
                fpe = fc[c].y * e;
                gp = gi;
            }
        };
        if (active && NSTEP > 0) {
            double2 b0[CH], f0[CH], b1[CH], f1[CH];
            double s0[CH], s1[CH];
            fw_load(0, b0, s0, f0);
            for (int i0 = 0; i0 < NSTEP; i0 += 2 * CH) {
                fw_load(i0 + CH, b1, s1, f1);
                fw_step(i0, b0, s0, f0);
                if (i0 + CH < NSTEP) {
                    fw_load(i0 + 2 * CH, b0, s0, f0);
                    fw_step(i0 + CH, b1, s1, f1);
                }
            }
        }
        // messages to the middle row: fn q and fn g y of this half's last
        // step (q = e g; fn = 0 for a half of dummy steps only)
        const double fnl = NSTEP > 0 ? Fh[NSTEP - 1].y : 0.0;
        const double ma = active ? fnl * (e * gp) : 0.0;
        const double mbr = active ? (fnl * gp) * yr : 0.0, mbi = active ? (fnl * gp) * yi : 0.0;
        const double pa = __shfl_xor(ma, 1, 64);
        const double pbr = __shfl_xor(mbr, 1, 64), pbi = __shfl_xor(mbi, 1, 64);
        if (active) {
            const double la = half ? pa : ma, ha = half ? ma : pa;
            const double lbr = half ? pbr : mbr, hbr = half ? mbr : pbr;
            const double lbi = half ? pbi : mbi, hbi = half ? mbi : pbi;
            const double2 bm = BM[g * 2 + sys];
            const double den = (SS[g * 2 + sys] * D[m] + la) + ha;
            double xr = ((bm.x + lbr) + hbr) / den, xi = ((bm.y + lbi) + hbi) / den;
            if (half == 0) XM[g * 2 + sys] = double2{xr, xi};
            // backward substitution from the middle outward, in place (the
            // dummy steps get x = 0)
            auto bw_load = [&](int top, double2 (&y)[CH], double (&gv)[CH], double (&fn)[CH]) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    y[c] = Yr[top - c];
                    gv[c] = Gr[top - c];
                    fn[c] = Fh[top - c].y;
                }
            };
            auto bw_step = [&](int top, const double2 (&y)[CH], const double (&gv)[CH],
                               const double (&fn)[CH]) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    xr = gv[c] * __builtin_fma(fn[c], xr, y[c].x);
                    xi = gv[c] * __builtin_fma(fn[c], xi, y[c].y);
                    Yr[top - c] = double2{xr, xi};
                }
            };
            if (NSTEP > 0) {
                double2 y0[CH], y1[CH];
                double g0[CH], g1[CH], n0[CH], n1[CH];
                bw_load(NSTEP - 1, y0, g0, n0);
                for (int top = NSTEP - 1; top >= 0; top -= 2 * CH) {
                    bw_load(top - CH, y1, g1, n1);
                    bw_step(top, y0, g0, n0);
                    if (top - CH >= 0) {
                        bw_load(top - 2 * CH, y0, g0, n0);
                        bw_step(top - CH, y1, g1, n1);
                    }
                }
            }
        }
    }
    if (t0 == 0 && threadIdx.x >= blockDim.x - 64) {
        double *base = reinterpret_cast<double *>(MC);
        mean_column_wave(nz, nx, ny, adjoint, f, D, sS, base, base + 1, 2);
    }
    __syncthreads();

    // one batch of stores: repack a pair, Z'_ky = A' + i B',
    // Z'_-ky = conj A' + i conj B'; a near-singular column as it is
    const int nst = nz * G;
    for (int i = threadIdx.x; i < nst; i += blockDim.x) {
        const int g = i % G, k = i / G, t = t0 + g;
        if (t >= ntask) continue;
        const int h = k > m ? 1 : 0;
        const int st = (h ? nz - 1 - k : k) + NSTEP - (h ? nz - 1 - m : m);
        auto x_of = [&](int sys) {
            return k == m ? XM[g * 2 + sys] : Y[((g * 2 + sys) * 2 + h) * NS + st];
        };
        const double o = os[k];
        const double2 A = t == 0 ? MC[k] : x_of(0);
        const size_t base = (size_t)k * lvl;
        if (t < npair) {
            const double2 B = x_of(1);
            const double Ar = o * A.x, Ai = o * A.y, Br = o * B.x, Bi = o * B.y;
            const int i0 = scol[g], i1 = scol[G + g];
            spec[base + i0] = C{(T)(Ar - Bi), (T)(Ai + Br)};
            if (i1 != i0) spec[base + i1] = C{(T)(Ar + Bi), (T)(Br - Ai)};
        } else {
            spec[base + scol[g]] = C{(T)(o * A.x), (T)(o * A.y)};
        }
    }
}

// Tasks per block of k_special_lds: as many as fit in 64 KiB of LDS (at most
// 48: four sweeping lanes per task, and the last wave kept free for the mean
// column), and the block's LDS bytes for them.
template <typename T> static int special_lds_tasks(int nz, size_t *bytes)
{
    int G = 48;
    while (G > 1 && (size_t)special_lds_layout(nz, G, sizeof(cx_t<T>)).total * 8 > 65536) --G;
    *bytes = (size_t)special_lds_layout(nz, G, sizeof(cx_t<T>)).total * 8;
    return G;
}

// ----------------------------------------------------------- level sums
__global__ __launch_bounds__(256) void k_level_sums(const double *__restrict__ rowsum,
                                                    double *__restrict__ S, int ny)
{
    __shared__ double part[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < ny; j += blockDim.x) s += rowsum[(size_t)k * ny + j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) S[k] = part[0];
}

hipError_t launch_level_sums(const double *rowsum, double *S, int ny, int nz, hipStream_t st)
{
    hipLaunchKernelGGL(k_level_sums, dim3(nz), dim3(256), 0, st, rowsum, S, ny);
    return hipGetLastError();
}

// ----------------------------------------------------------- launchers
template <typename T, int NH, bool REFINE>
static hipError_t columns_nh(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                             const int *maskcnt, const Tables<T> &tb, const double *ax64,
                             const double *ay64, const double *f64, const double *D64,
                             const double *rs64, long c0, long c1, hipStream_t st)
{
    constexpr int CH = NH < 8 ? NH : 8;
    const long ncols = c1 - c0;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 63) / 64;
    hipLaunchKernelGGL((k_columns<T, NH, CH, REFINE>), dim3((unsigned)grid), dim3(256), 0, st, spec,
                       L, ny, nz, tb.ax, tb.ay, tb.f, tb.D, rs, os, maskcnt, ax64, ay64, f64, D64,
                       rs64, c0, c1);
    return hipGetLastError();
}

template <typename T, int NH, bool KEEPG>
static hipError_t columns2_nh(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                              const int *maskcnt, const Tables<T> &tb, long c0, long c1,
                              hipStream_t st)
{
    constexpr int CH = NH < 8 ? NH : 8;
    const long ncols = c1 - c0;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 127) / 128;
    hipLaunchKernelGGL((k_columns2<T, NH, CH, KEEPG>), dim3((unsigned)grid), dim3(256), 0, st,
                       spec, L, ny, nz, tb.ax, tb.ay, tb.f, tb.D, rs, os, maskcnt, c0, c1);
    return hipGetLastError();
}

template <typename T, bool KEEPG>
static hipError_t columns2_dispatch(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                                    const int *maskcnt, const Tables<T> &tb, long c0, long c1,
                                    hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N)                                                                                 \
        return columns2_nh<T, N, KEEPG>(spec, L, ny, nz, rs, os, maskcnt, tb, c0, c1, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <typename T, int NH, bool KEEPG>
static hipError_t columns3_nh(cx_t<T> *spec, int L, int ny, int nz, int adjoint,
                              const int *maskcnt, const Tables<T> &tb, long c0, long c1,
                              hipStream_t st)
{
    (void)nz;
    const long ncols = c1 - c0;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 127) / 128;
    const LevelCoef<T> *ct = reinterpret_cast<const LevelCoef<T> *>(
        adjoint ? tb.coef_adj : tb.coef_fwd);
    hipLaunchKernelGGL((k_columns3<T, NH, KEEPG>), dim3((unsigned)grid), dim3(256), 0, st, spec, L,
                       ny, tb.ax, tb.ay, ct, maskcnt, c0, c1);
    return hipGetLastError();
}

template <typename T, bool KEEPG>
static hipError_t columns3_dispatch(cx_t<T> *spec, int L, int ny, int nz, int adjoint,
                                    const int *maskcnt, const Tables<T> &tb, long c0, long c1,
                                    hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N)                                                                                 \
        return columns3_nh<T, N, KEEPG>(spec, L, ny, nz, adjoint, maskcnt, tb, c0, c1, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <int NH>
static hipError_t columns3r_nh(float2 *spec, int L, int ny, int adjoint, const int *maskcnt,
                               const Tables<float> &tb, const Tables<double> &t64, long c0,
                               long c1, hipStream_t st)
{
    const long ncols = c1 - c0;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 127) / 128;
    const auto *ct = reinterpret_cast<const LevelCoef<float> *>(adjoint ? tb.coef_adj : tb.coef_fwd);
    const auto *c64 =
        reinterpret_cast<const LevelCoef<double> *>(adjoint ? t64.coef_adj : t64.coef_fwd);
    hipLaunchKernelGGL((k_columns3r<NH>), dim3((unsigned)grid), dim3(256), 0, st, spec, L, ny,
                       tb.ax, tb.ay, ct, c64, t64.ax, t64.ay, maskcnt, c0, c1);
    return hipGetLastError();
}

static hipError_t columns3r_dispatch(float2 *spec, int L, int ny, int nz, int adjoint,
                                     const int *maskcnt, const Tables<float> &tb,
                                     const Tables<double> &t64, long c0, long c1, hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N) return columns3r_nh<N>(spec, L, ny, adjoint, maskcnt, tb, t64, c0, c1, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <typename T, int NH, bool REFINE, bool SHG, int PPB>
static hipError_t columns3s_nh(cx_t<T> *spec, int L, int ny, int adjoint, const int *maskcnt,
                               const Tables<T> &tb, const Tables<double> &t64, long c0, long c1,
                               int swz, hipStream_t st)
{
    const long ncols = c1 - c0;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 32 * PPB - 1) / (32 * PPB);
    const auto *ct = reinterpret_cast<const LevelCoef<T> *>(adjoint ? tb.coef_adj : tb.coef_fwd);
    const auto *c64 =
        reinterpret_cast<const LevelCoef<double> *>(adjoint ? t64.coef_adj : t64.coef_fwd);
    hipLaunchKernelGGL((k_columns3s<T, NH, REFINE, SHG, PPB>), dim3((unsigned)grid),
                       dim3(128 * PPB), 0, st, spec, L, ny, tb.ax, tb.ay, ct, c64, t64.ax, t64.ay,
                       maskcnt, c0, c1, swz);
    return hipGetLastError();
}

// SHG (pivots kept in LDS, 2 PPB NH 32 sizeof(T) bytes per block) up to
// NH = 64; beyond, the pivots are recomputed.  PPB wave pairs per block.
template <typename T, bool REFINE, bool SHG, int PPB = 2>
static hipError_t columns3s_dispatch(cx_t<T> *spec, int L, int ny, int nz, int adjoint,
                                     const int *maskcnt, const Tables<T> &tb,
                                     const Tables<double> &t64, long c0, long c1, hipStream_t st,
                                     int swz = 0)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N)                                                                                 \
        return columns3s_nh<T, N, REFINE, SHG && (N <= 64), PPB>(spec, L, ny, adjoint, maskcnt,   \
                                                                 tb, t64, c0, c1, swz, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <typename T, bool REFINE>
static hipError_t columns_dispatch(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                                   const int *maskcnt, const Tables<T> &tb, const double *ax64,
                                   const double *ay64, const double *f64, const double *D64,
                                   const double *rs64, long c0, long c1, hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N)                                                                                 \
        return columns_nh<T, N, REFINE>(spec, L, ny, nz, rs, os, maskcnt, tb, ax64, ay64, f64,     \
                                        D64, rs64, c0, c1, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

// variant: 0 = four lanes per column (re/im split, pivots recomputed),
// 1 = two lanes per column, pivots recomputed, 2 = two lanes, pivots kept,
// 3 = halves in separate waves with scalar coefficient tables, pivots
// recomputed, 4 = as 3 with pivots kept.
// 5 = as 3 with the real and imaginary parts in two lanes, 6 = as 5 with
// the pivots of the first sweep kept in LDS, 7 = as 6 with one wave pair
// (32 columns) per block, 8 = as 7 with XCD-contiguous column groups.
// The in-register refinement (FP32 only) uses variant 0's refining kernel
// for variants 0-2, the refining uniform-half kernel for 3-4 and the
// refining split-lane kernel for 5-8.
template <typename T>
hipError_t launch_columns_impl(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, int refine,
                               const int *maskcnt, const Tables<T> &tb, const Tables<double> *t64,
                               hipStream_t st, int variant, int kxlo, int kxhi)
{
    const int L = nx / 2;
    if (kxlo < 1) kxlo = 1;
    if (kxhi > L) kxhi = L;
    if (kxhi <= kxlo) return hipSuccess;
    const long c0 = (long)kxlo * ny, c1 = (long)kxhi * ny;
    const T *rs = adjoint ? tb.rs_adj : tb.rs_fwd;
    const T *os = adjoint ? tb.os_adj : nullptr;
    if constexpr (std::is_same<T, float>::value) {
        if (refine && variant == 5)
            return columns3s_dispatch<float, true, false>(spec, L, ny, nz, adjoint, maskcnt, tb,
                                                          *t64, c0, c1, st);
        if (refine && variant == 6)
            return columns3s_dispatch<float, true, true>(spec, L, ny, nz, adjoint, maskcnt, tb,
                                                         *t64, c0, c1, st);
        if (refine && (variant == 7 || variant == 8))
            return columns3s_dispatch<float, true, true, 1>(spec, L, ny, nz, adjoint, maskcnt, tb,
                                                            *t64, c0, c1, st, variant == 8);
        if (refine && variant >= 3)
            return columns3r_dispatch(spec, L, ny, nz, adjoint, maskcnt, tb, *t64, c0, c1, st);
        if (refine) {
            const double *rs64 = adjoint ? t64->rs_adj : t64->rs_fwd;
            return columns_dispatch<float, true>(spec, L, ny, nz, rs, os, maskcnt, tb, t64->ax,
                                                 t64->ay, t64->f, t64->D, rs64, c0, c1, st);
        }
    }
    if (variant == 1)
        return columns2_dispatch<T, false>(spec, L, ny, nz, rs, os, maskcnt, tb, c0, c1, st);
    if (variant == 2)
        return columns2_dispatch<T, true>(spec, L, ny, nz, rs, os, maskcnt, tb, c0, c1, st);
    if (variant == 3)
        return columns3_dispatch<T, false>(spec, L, ny, nz, adjoint, maskcnt, tb, c0, c1, st);
    if (variant == 4)
        return columns3_dispatch<T, true>(spec, L, ny, nz, adjoint, maskcnt, tb, c0, c1, st);
    if (variant == 5)
        return columns3s_dispatch<T, false, false>(spec, L, ny, nz, adjoint, maskcnt, tb, *t64, c0,
                                                   c1, st);
    if (variant == 6)
        return columns3s_dispatch<T, false, true>(spec, L, ny, nz, adjoint, maskcnt, tb, *t64, c0,
                                                  c1, st);
    if (variant == 7 || variant == 8)
        return columns3s_dispatch<T, false, true, 1>(spec, L, ny, nz, adjoint, maskcnt, tb, *t64,
                                                     c0, c1, st, variant == 8);
    return columns_dispatch<T, false>(spec, L, ny, nz, rs, os, maskcnt, tb, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, c0, c1, st);
}

template hipError_t launch_columns_impl<float>(cx_t<float> *, int, int, int, int, int, const int *,
                                               const Tables<float> &, const Tables<double> *,
                                               hipStream_t, int, int, int);
template hipError_t launch_columns_impl<double>(cx_t<double> *, int, int, int, int, int,
                                                const int *, const Tables<double> &,
                                                const Tables<double> *, hipStream_t, int, int,
                                                int);

// FP64 columns: the packed kx = 0 row, the mean column and the near-singular
// columns; parallel = 0: one lane per task through the HBM workspace
// (k_special_seq), else staged in LDS (k_special_lds).
template <typename T>
hipError_t launch_special(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, const int *mlist,
                          int nmask, const double *S, double *ws, const Tables<double> &tb64,
                          hipStream_t st, int parallel)
{
    const int ntask = ny / 2 + 1 + nmask;
    const double *rs = adjoint ? tb64.rs_adj : tb64.rs_fwd;
    const double *os = adjoint ? tb64.os_adj : nullptr;
    if (parallel) {
        size_t bytes = 0;
        const int G = special_lds_tasks<T>(nz, &bytes);
        hipLaunchKernelGGL(k_special_lds<T>, dim3((ntask + G - 1) / G), dim3(256), bytes, st,
                           spec, nx, ny, nz, adjoint, mlist, nmask, S, tb64.ax, tb64.ay, tb64.f,
                           tb64.D, rs, os, G);
        return hipGetLastError();
    }
    const int grid = (ntask + 63) / 64;
    hipLaunchKernelGGL((k_special_seq<T, 16>), dim3(grid), dim3(64), 0, st, spec, nx, ny, nz,
                       adjoint, mlist, nmask, S, ws, tb64.ax, tb64.ay, tb64.f, tb64.D, rs, os);
    return hipGetLastError();
}

template hipError_t launch_special<float>(cx_t<float> *, int, int, int, int, const int *, int,
                                          const double *, double *, const Tables<double> &,
                                          hipStream_t, int);
template hipError_t launch_special<double>(cx_t<double> *, int, int, int, int, const int *, int,
                                           const double *, double *, const Tables<double> &,
                                           hipStream_t, int);

// ----------------------------------------------------------- density gradient
// g_k = -sum_ij [ -lam_k (V p)_k / rho_k
//                 + 1/2 gam_{k+1/2} (lam_k/D_k - lam_{k+1}/D_{k+1})
//                 + 1/2 gam_{k-1/2} (lam_{k-1}/D_{k-1} - lam_k/D_k) ],
// gam_{k+1/2} = (p_{k+1} - p_k) / h_{k+1/2}: the derivative of the vertical
// operator's three rho-dependent ingredients (1/D_k of row k and the face
// densities on either side of level k).  A block row handles a chunk of GK
// levels; each thread walks a fixed set of horizontal points (grid stride)
// and sums its terms per level in registers, so that the wave reduction runs
// once per thread, not once per point.  Per-level block sums are written in
// fixed order and reduced by k_grad_reduce (no atomics): the result is the
// same on every run.
// gk = [f (nz+1) | D (nz) | rho (nz) | 1/h (nz+1, same indexing as f) |
//       1/D (nz) | 1/rho (nz)].
constexpr int GK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_grad_rho(const T *__restrict__ lam, const T *__restrict__ p,
                                                  int nxy, int nz, const double *__restrict__ gk,
                                                  double *__restrict__ partial, int nblk)
{
    __shared__ double red[4][GK];
    const double *f = gk, *D = gk + nz + 1, *rho = D + nz, *ih = rho + nz;
    const double *iD = ih + nz + 1, *irho = iD + nz;
    (void)D;
    (void)rho;
    const int k0 = blockIdx.y * GK;
    double acc[GK];
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) acc[kk] = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nxy; c += gridDim.x * blockDim.x) {
        // All GK + 2 levels of the chunk are loaded up front from clamped
        // indices, so that every load is issued before the first is waited
        // for; a clamped value only enters terms that the k > 0 and
        // k + 1 < nz conditions below leave out.
        T pv[GK + 2], lv[GK + 2];
#pragma unroll
        for (int j = 0; j < GK + 2; ++j) {
            const int k = min(max(k0 - 1 + j, 0), nz - 1);
            pv[j] = p[(size_t)k * nxy + c];
            lv[j] = lam[(size_t)k * nxy + c];
        }
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            const int k = k0 + kk;
            if (k < nz) { // uniform: the last chunk may hold fewer levels
                const double pm = pv[kk], pc = pv[kk + 1], pp = pv[kk + 2];
                const double lm = lv[kk], lc = lv[kk + 1], lp = lv[kk + 2];
                const double up = k + 1 < nz ? f[k + 1] * (pp - pc) : 0.0;
                const double dn = k > 0 ? f[k] * (pc - pm) : 0.0;
                const double Vp = (up - dn) * iD[k];
                double t = -lc * Vp * irho[k];
                if (k + 1 < nz) t += 0.5 * (pp - pc) * ih[k + 1] * (lc * iD[k] - lp * iD[k + 1]);
                if (k > 0) t += 0.5 * (pc - pm) * ih[k] * (lm * iD[k - 1] - lc * iD[k]);
                acc[kk] += t;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
        const double t = wave_sum(acc[kk]);
        if (lane == 0) red[wv][kk] = t;
    }
    __syncthreads();
    if (threadIdx.x < GK && k0 + (int)threadIdx.x < nz) {
        const int kk = threadIdx.x;
        partial[(size_t)(k0 + kk) * nblk + blockIdx.x] =
            ((red[0][kk] + red[1][kk]) + red[2][kk]) + red[3][kk];
    }
}

// One block per level: a fixed-order strided sum of the block partials per
// thread, then a fixed tree over the block.
__global__ __launch_bounds__(256) void k_grad_reduce(const double *__restrict__ partial, int nblk,
                                                     int nz, double *__restrict__ g)
{
    __shared__ double s[256];
    const int k = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += partial[(size_t)k * nblk + b];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && k < nz) g[k] = -s[0];
}

// Blocks per level chunk: one thread per point up to 1024 blocks, beyond
// which threads take several points.
int grad_blocks(int nx, int ny) { return std::min((nx * ny + 255) / 256, 1024); }

template <typename T>
hipError_t launch_grad_rho(const T *lam, const T *p, int nx, int ny, int nz, const double *gk,
                           double *partial, int nblk, double *grho, hipStream_t st)
{
    dim3 grid(nblk, (nz + GK - 1) / GK);
    hipLaunchKernelGGL(k_grad_rho<T>, grid, dim3(256), 0, st, lam, p, nx * ny, nz, gk, partial,
                       nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_reduce, dim3(nz), dim3(256), 0, st, partial, nblk, nz, grho);
    return hipGetLastError();
}

template hipError_t launch_grad_rho<float>(const float *, const float *, int, int, int,
                                           const double *, double *, int, double *, hipStream_t);
template hipError_t launch_grad_rho<double>(const double *, const double *, int, int, int,
                                            const double *, double *, int, double *, hipStream_t);

} // namespace ps
