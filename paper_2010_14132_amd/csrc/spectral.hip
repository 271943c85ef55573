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
#include "ps_internal.h"
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
                                                 const double *__restrict__ rs64)
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
    const long ncol = (long)L * ny;
    const long col = (long)ny + ((long)blockIdx.x * 4 + wave) * 16 + cl;
    const bool valid = col < ncol;
    const int kx = valid ? (int)(col / ny) : 1;
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
                                                  const int *__restrict__ maskcnt)
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
    const long ncol = (long)L * ny;
    const long col = (long)ny + ((long)blockIdx.x * 4 + wave) * 32 + cl;
    const bool valid = col < ncol;
    const int kx = valid ? (int)(col / ny) : 1;
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

// ----------------------------------------------------------- uniform-half sweep
// Reciprocal of a pivot u > 0 in the normal range.  FP32: the hardware
// reciprocal refined by one Newton step (within one ulp of the IEEE
// quotient); FP64: IEEE division.
__device__ __forceinline__ float pivot_rcp(float u)
{
    const float r = __builtin_amdgcn_rcpf(u);
    const float e = __builtin_fmaf(-u, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}
__device__ __forceinline__ double pivot_rcp(double u) { return 1.0 / u; }

// Per-slot coefficients in each half's elimination order (built by the plan):
// slot [half][i], i in [0, NH), for level k = i (low half) or k = nz - 1 - i
// (high half), with the half's real levels in the LAST n slots and dummy
// slots in front (f_prev = f_next = 0, D = 1, rs = 0, off -> middle row).  A
// dummy row never influences a real one: the first real row of each half is
// a boundary row (f_prev = 0).  Slot [2 NH] is the middle row m.  rs/os are
// the forward or adjoint right-hand-side and output factors.  `off` is the
// byte offset of the level in the spectrum.  Wave-uniform, so they are read
// through the scalar cache.
// Two waves per group of 64 columns: the low-half wave eliminates levels
// 0..m-1 and the high-half wave levels nz-1..m+1, one column per lane
// (complex values, real pivots); they exchange their messages to the middle
// row through LDS.  KEEPG keeps the reciprocal pivots in registers instead
// of recomputing them in the backward pass.
template <typename T, int NH, bool KEEPG>
__global__ __launch_bounds__(256) void k_columns3(cx_t<T> *__restrict__ spec, int L, int ny,
                                                  const T *__restrict__ ax,
                                                  const T *__restrict__ ay,
                                                  const LevelCoef<T> *__restrict__ coef,
                                                  const int *__restrict__ maskcnt)
{
    using C = cx_t<T>;
    constexpr int CH = NH < 8 ? NH : 8;
    constexpr int NB = (NH + CH - 1) / CH;
    __shared__ T xa[2][2][64];
    __shared__ C xb[2][2][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pair = w >> 1, half = w & 1;
    const long ncol = (long)L * ny;
    const long col = (long)ny + ((long)blockIdx.x * 2 + pair) * 64 + lane;
    const bool valid = col < ncol;
    const int kx = valid ? (int)(col / ny) : 1;
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const T s = ax[kx] + ay[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    char *base = reinterpret_cast<char *>(spec + (valid ? col : 0));
    const LevelCoef<T> *ct = coef + half * NH;

    C v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const C x = *reinterpret_cast<const C *>(base + (ct[i].off < 0 ? coef[2 * NH].off : ct[i].off));
        v[i] = C{x.x * ct[i].rs, x.y * ct[i].rs};
    }
    const LevelCoef<T> cm = coef[2 * NH];
    C rmv = *reinterpret_cast<const C *>(base + cm.off);
    rmv = C{rmv.x * cm.rs, rmv.y * cm.rs};

    T qck[KEEPG ? 1 : NB];
    T gk[KEEPG ? NH : 1];
    T q = T(0), g = T(0);
    C y = C{T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (!KEEPG && i % CH == 0) qck[i / CH] = q;
        const T e = s * ct[i].D + ct[i].fp * q;
        const T gi = pivot_rcp(e + ct[i].fn);
        const T c = ct[i].fp * g;
        y = C{v[i].x + c * y.x, v[i].y + c * y.y};
        v[i] = y;
        q = e * gi;
        g = gi;
        if (KEEPG) gk[i] = gi;
    }
    const T fl = ct[NH - 1].fn;
    xa[pair][half][lane] = fl * q;
    xb[pair][half][lane] = C{(fl * g) * y.x, (fl * g) * y.y};
    __syncthreads();
    const T la = xa[pair][0][lane], ha = xa[pair][1][lane];
    const C lb = xb[pair][0][lane], hb = xb[pair][1][lane];
    const T den = (s * cm.D + la) + ha;
    const C xm = C{((rmv.x + lb.x) + hb.x) / den, ((rmv.y + lb.y) + hb.y) / den};

    C xn = xm;
    if constexpr (KEEPG) {
#pragma unroll
        for (int i = NH - 1; i >= 0; --i) {
            const T fn = ct[i].fn;
            xn = C{gk[i] * (v[i].x + fn * xn.x), gk[i] * (v[i].y + fn * xn.y)};
            v[i] = xn;
        }
    } else {
#pragma unroll
        for (int bb = NB - 1; bb >= 0; --bb) {
            T gb[CH];
            T qq = qck[bb];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = bb * CH + c;
                const T e = s * ct[i].D + ct[i].fp * qq;
                const T gi = pivot_rcp(e + ct[i].fn);
                gb[c] = gi;
                qq = e * gi;
            }
#pragma unroll
            for (int c = CH - 1; c >= 0; --c) {
                const int i = bb * CH + c;
                const T fn = ct[i].fn;
                xn = C{gb[c] * (v[i].x + fn * xn.x), gb[c] * (v[i].y + fn * xn.y)};
                v[i] = xn;
            }
        }
    }
    if (store) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const long long off = ct[i].off;
            if (off >= 0)
                *reinterpret_cast<C *>(base + off) = C{v[i].x * ct[i].os, v[i].y * ct[i].os};
        }
        if (half) *reinterpret_cast<C *>(base + cm.off) = C{xm.x * cm.os, xm.y * cm.os};
    }
}

// ----------------------------------------------------------- FP64 columns
// One thread per task, FP64 throughout, column temporaries in the
// workspace laid out [quantity][level][task] (consecutive tasks contiguous).
__device__ void seq_column(int nz, double s, const double *f, const double *D, double *yr,
                           double *yi, double *gg, size_t st)
{
    double q = 0.0, g = 0.0, pr = 0.0, pi = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double fp = f[k], fn = f[k + 1];
        const double e = s * D[k] + fp * q;
        const double gi = 1.0 / (e + fn);
        const double r = yr[k * st] + (fp * g) * pr;
        const double i = yi[k * st] + (fp * g) * pi;
        yr[k * st] = r;
        yi[k * st] = i;
        gg[k * st] = gi;
        q = e * gi;
        g = gi;
        pr = r;
        pi = i;
    }
    double xr = 0.0, xi = 0.0;
    for (int k = nz - 1; k >= 0; --k) {
        const double fn = f[k + 1];
        xr = gg[k * st] * (yr[k * st] + fn * xr);
        xi = gg[k * st] * (yi[k * st] + fn * xi);
        yr[k * st] = xr;
        yi[k * st] = xi;
    }
}

// Tasks t in [0, ny/2]: the packed kx = 0 row.  Slot (kx=0, ky) holds
// Z = A + i B with A = DFT_y of the x-DC coefficients (modes (0, ky)) and
// B = DFT_y of the x-Nyquist coefficients (modes (nx/2, ky)); both come from
// real sequences, so A_ky = (Z_ky + conj Z_{-ky})/2 and
// B_ky = (Z_ky - conj Z_{-ky})/(2i).  The task solves A and B for ky and
// repacks ky and -ky.  Mode (0,0) is the singular mean column: it is taken
// from the FP64 level sums S_k instead of the transform (see below).
// Tasks t > ny/2: near-singular columns kx >= 1 from mlist, in FP64.
template <typename T>
__global__ __launch_bounds__(64) void k_special(cx_t<T> *__restrict__ spec, int nx, int ny, int nz,
                                                int adjoint, const int *__restrict__ mlist,
                                                int nmask, const double *__restrict__ S,
                                                double *__restrict__ ws, const double *__restrict__ ax,
                                                const double *__restrict__ ay,
                                                const double *__restrict__ fg,
                                                const double *__restrict__ Dg,
                                                const double *__restrict__ rs,
                                                const double *__restrict__ os)
{
    __shared__ double f[PS_MAX_NZ + 1], D[PS_MAX_NZ];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) {
        f[t] = fg[t];
        if (t < nz) D[t] = Dg[t];
    }
    __syncthreads();
    const int L = nx / 2;
    const int npair = ny / 2 + 1;
    const int ntask = npair + nmask;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    const size_t st = (size_t)ntask;
    double *Ar = ws + (0 * (size_t)nz) * st + t, *Ai = ws + (1 * (size_t)nz) * st + t;
    double *Br = ws + (2 * (size_t)nz) * st + t, *Bi = ws + (3 * (size_t)nz) * st + t;
    double *G = ws + (4 * (size_t)nz) * st + t;
    const size_t lvl = (size_t)L * ny;
    const double on = 1.0 / ((double)nx * (double)ny);

    if (t < npair) {
        const int ky = t, kp = (ny - t) % ny;
        for (int k = 0; k < nz; ++k) {
            const cx_t<T> z = spec[(size_t)k * lvl + ky];
            const cx_t<T> w = spec[(size_t)k * lvl + kp];
            const double zr = z.x, zi = z.y, wr = w.x, wi = -(double)w.y; // w = conj Z_{-ky}
            Ar[k * st] = rs[k] * 0.5 * (zr + wr);
            Ai[k * st] = rs[k] * 0.5 * (zi + wi);
            Br[k * st] = rs[k] * 0.5 * (zi - wi);
            Bi[k * st] = rs[k] * -0.5 * (zr - wr);
        }
        if (ky == 0) {
            // Mean column from the FP64 level sums.  Forward: level means of
            // b minus mu (the D-weighted mean); V x = c by flux prefix sums
            // F_{k+1/2} = sum_{j<=k} D_j c_j, x_{k+1} = x_k + F/f_{k+1/2};
            // gauge: zero mean over levels.  Adjoint: level means of w minus
            // the plain mean; V z = c / D; gauge sum D z = 0; output D z.
            double num = 0.0, den = 0.0, tot = 0.0;
            for (int k = 0; k < nz; ++k) {
                num += D[k] * S[k];
                den += D[k];
                tot += S[k];
            }
            const double mu = adjoint ? tot * on / (double)nz : num * on / den;
            double F = 0.0, x = 0.0, acc = 0.0, wsum = 0.0;
            Ar[0] = 0.0;
            for (int k = 0; k + 1 < nz; ++k) {
                const double c = S[k] * on - mu;
                F += adjoint ? c : D[k] * c;
                x += F / f[k + 1];
                Ar[(k + 1) * st] = x;
            }
            for (int k = 0; k < nz; ++k) {
                const double wk = adjoint ? D[k] : 1.0;
                acc += wk * Ar[k * st];
                wsum += wk;
            }
            const double shift = acc / wsum;
            for (int k = 0; k < nz; ++k) {
                Ar[k * st] -= shift;
                Ai[k * st] = 0.0;
            }
        } else {
            seq_column(nz, ay[ky], f, D, Ar, Ai, G, st);
        }
        seq_column(nz, ax[L] + ay[ky], f, D, Br, Bi, G, st);
        for (int k = 0; k < nz; ++k) {
            const double o = os ? os[k] : 1.0;
            const double ar = o * Ar[k * st], ai = o * Ai[k * st];
            const double br = o * Br[k * st], bi = o * Bi[k * st];
            spec[(size_t)k * lvl + ky] = cx_t<T>{(T)(ar - bi), (T)(ai + br)};
            if (kp != ky) spec[(size_t)k * lvl + kp] = cx_t<T>{(T)(ar + bi), (T)(br - ai)};
        }
    } else {
        const int c = mlist[t - npair];
        const int kx = c / ny, ky = c - kx * ny;
        for (int k = 0; k < nz; ++k) {
            const cx_t<T> z = spec[(size_t)k * lvl + c];
            Ar[k * st] = rs[k] * (double)z.x;
            Ai[k * st] = rs[k] * (double)z.y;
        }
        seq_column(nz, ax[kx] + ay[ky], f, D, Ar, Ai, G, st);
        for (int k = 0; k < nz; ++k) {
            const double o = os ? os[k] : 1.0;
            spec[(size_t)k * lvl + c] = cx_t<T>{(T)(o * Ar[k * st]), (T)(o * Ai[k * st])};
        }
    }
}

// ----------------------------------------------------------- FP64 columns, parallel
// The same FP64 work as k_special, with the register-resident two-ended
// sweep (4 lanes per column).  Waves [0, npw): the packed kx = 0 row, eight
// ky values per wave; lane = half*32 + 4*j + 2*which + comp, where which = 0
// solves A (modes (0, ky), s = ay[ky]) and which = 1 solves B (modes
// (nx/2, ky), s = ax[nx/2] + ay[ky]).  Each lane forms its component of A or
// B from Z_ky and Z_{-ky}; after the solve the (A, re) and (A, im) lanes
// repack Z'_ky = A' + i B' and Z'_{-ky} = conj A' + i conj B' with one
// shuffle.  The (A, ky = 0) lanes hold the singular mean column, computed
// from the FP64 level sums by flux prefix sums.  Waves [npw, npw + nmw):
// near-singular columns kx >= 1 from mlist, 16 per wave.
template <typename T, int NH>
__global__ __launch_bounds__(256) void k_special_par(
    cx_t<T> *__restrict__ spec, int nx, int ny, int nz, int adjoint, const int *__restrict__ mlist,
    int nmask, const double *__restrict__ S, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ fg, const double *__restrict__ Dg,
    const double *__restrict__ rsg, const double *__restrict__ osg)
{
    constexpr int CH = NH < 8 ? NH : 8;
    __shared__ double sf[PS_MAX_NZ + 1], sD[PS_MAX_NZ], srs[PS_MAX_NZ], sos[PS_MAX_NZ],
        sS[PS_MAX_NZ];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) {
        sf[t] = fg[t];
        if (t < nz) {
            sD[t] = Dg[t];
            srs[t] = rsg[t];
            sos[t] = osg ? osg[t] : 1.0;
            sS[t] = S[t];
        }
    }
    __syncthreads();
    const int L = nx / 2;
    const int npair = ny / 2 + 1;
    const int npw = (npair + 7) / 8;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int half = lane >> 5, comp = lane & 1;
    const size_t ls = (size_t)2 * L * ny; // level stride in T units
    const T *sp = reinterpret_cast<const T *>(spec);
    T *dp = reinterpret_cast<T *>(spec);
    const int m = nz >> 1;
    const int n = half ? nz - 1 - m : m;

    bool pair = wave < npw;
    int ky = 0, kp = 0, which = 0, col = 0;
    bool valid;
    double s;
    if (pair) {
        const int j = (lane & 31) >> 2;
        which = (lane >> 1) & 1;
        ky = wave * 8 + j;
        valid = ky < npair;
        if (!valid) ky = 0;
        kp = (ny - ky) % ny;
        s = which ? ax[L] + ay[ky] : ay[ky];
    } else {
        const int c = (wave - npw) * 16 + ((lane & 31) >> 1);
        valid = c < nmask;
        col = valid ? mlist[c] : ny; // column kx >= 1
        const int kx = col / ny, kyy = col - kx * ny;
        s = ax[kx] + ay[kyy];
    }
    const bool mean = pair && which == 0 && ky == 0;
    if (!(s > 0.0)) s = 1.0; // the mean column is not swept

    // value of this lane's component at level k
    auto load = [&](int k) -> double {
        if (!valid) return 0.0;
        const size_t b = (size_t)k * ls;
        if (!pair) return (double)sp[b + 2 * (size_t)col + comp];
        const int c1 = which ? 1 - comp : comp;
        const double zk = (double)sp[b + 2 * (size_t)ky + c1];
        const double zm = (double)sp[b + 2 * (size_t)kp + c1];
        // A.re = (zk.re+zm.re)/2, A.im = (zk.im-zm.im)/2,
        // B.re = (zk.im+zm.im)/2, B.im = (zm.re-zk.re)/2
        if (!which) return comp ? 0.5 * (zk - zm) : 0.5 * (zk + zm);
        return comp ? 0.5 * (zm - zk) : 0.5 * (zk + zm);
    };
    double v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i)
        if (i < n) {
            const int k = half ? nz - 1 - i : i;
            v[i] = load(k) * srs[k];
        }
    const double rm = load(m) * srs[m];
    double xm = twisted_solve<double, NH, CH>(v, n, half, m, nz, s, sf, sD, rm);

    if (mean) {
        // Forward: c_k = level mean of b - mu (D-weighted mean); V x = c by
        // F_{k+1/2} = sum_{j<=k} D_j c_j, x_{k+1} = x_k + F/f_{k+1/2}; gauge:
        // zero plain mean.  Adjoint: c_k = level mean of w - plain mean;
        // V z = c / D; gauge sum_k D_k z_k = 0.  Imaginary part zero.
        const double on = 1.0 / ((double)nx * (double)ny);
        double num = 0.0, den = 0.0, tot = 0.0;
        for (int k = 0; k < nz; ++k) {
            num += sD[k] * sS[k];
            den += sD[k];
            tot += sS[k];
        }
        const double mu = adjoint ? tot * on / (double)nz : num * on / den;
        double F = 0.0, x = 0.0, acc = 0.0, wsum = 0.0;
        for (int k = 0; k < nz; ++k) {
            if (k > 0) {
                const double c = sS[k - 1] * on - mu;
                F += adjoint ? c : sD[k - 1] * c;
                x += F / sf[k];
            }
            const double wk = adjoint ? sD[k] : 1.0;
            acc += wk * x;
            wsum += wk;
        }
        const double shift = acc / wsum;
        F = 0.0;
        x = 0.0;
        for (int k = 0; k < nz; ++k) {
            if (k > 0) {
                const double c = sS[k - 1] * on - mu;
                F += adjoint ? c : sD[k - 1] * c;
                x += F / sf[k];
            }
            const double val = comp ? 0.0 : x - shift;
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int ki = half ? nz - 1 - i : i;
                if (i < n && ki == k) v[i] = val;
            }
            if (k == m) xm = val;
        }
    }

    if (pair) {
        // (A, re) lanes: Z'_ky.re = A'.re - B'.im, Z'_-ky.re = A'.re + B'.im
        // (A, im) lanes: Z'_ky.im = A'.im + B'.re, Z'_-ky.im = B'.re - A'.im
        // the partner component sits in lane ^ 3.
        // every lane of the wave takes part in each shuffle; `st` gates the store
        auto emit = [&](int k, double x, bool st) {
            const double o = x * sos[k];
            const double other = __shfl_xor(o, 3, 64);
            if (st && valid && which == 0) {
                const size_t b = (size_t)k * ls;
                const double zy = comp ? o + other : o - other;
                const double zp = comp ? other - o : o + other;
                dp[b + 2 * (size_t)ky + comp] = (T)zy;
                if (kp != ky) dp[b + 2 * (size_t)kp + comp] = (T)zp;
            }
        };
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const bool act = i < n;
            const int k = act ? (half ? nz - 1 - i : i) : 0;
            emit(k, act ? v[i] : 0.0, act);
        }
        emit(m, xm, half == 1); // the middle row is stored by the high half
    } else if (valid) {
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (i < n) {
                const int k = half ? nz - 1 - i : i;
                dp[(size_t)k * ls + 2 * (size_t)col + comp] = (T)(v[i] * sos[k]);
            }
        if (half) dp[(size_t)m * ls + 2 * (size_t)col + comp] = (T)(xm * sos[m]);
    }
}

// ----------------------------------------------------------- FP64 columns, compact
// One lane per task, FP64, with short code: the level loop is unrolled by U
// only, the next U levels' loads are issued before the current U levels are
// eliminated, and the eliminated values and reciprocal pivots go to the
// workspace laid out [quantity][level][task] (consecutive tasks contiguous).
// Tasks [0, ny/2]: the packed kx = 0 row -- the lane forms A (modes
// (0, ky)) and B (modes (nx/2, ky)) from Z_ky and Z_{-ky}, runs both
// eliminations interleaved and repacks Z'_ky = A' + i B',
// Z'_{-ky} = conj A' + i conj B'.  Task 0's A is the singular mean column,
// from the FP64 level sums.  Tasks beyond: near-singular columns kx >= 1.
template <typename T, int U>
__global__ __launch_bounds__(64) void k_special_seq(
    cx_t<T> *__restrict__ spec, int nx, int ny, int nz, int adjoint, const int *__restrict__ mlist,
    int nmask, const double *__restrict__ S, double *__restrict__ ws,
    const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ fg,
    const double *__restrict__ Dg, const double *__restrict__ rsg, const double *__restrict__ osg)
{
    // These few waves carry long dependent chains and usually share their
    // SIMDs with the main column kernel: issue them first.
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
    const int L = nx / 2;
    const int npair = ny / 2 + 1;
    const int ntask = npair + nmask;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    const size_t st = (size_t)ntask, lz = (size_t)nz * st;
    double *yar = ws + 0 * lz + t, *yai = ws + 1 * lz + t;
    double *ybr = ws + 2 * lz + t, *ybi = ws + 3 * lz + t;
    double *ga = ws + 4 * lz + t, *gb = ws + 5 * lz + t;
    const size_t lvl = (size_t)L * ny;
    const bool pair = t < npair;
    int i0, i1; // spectrum indices within a level: Z_ky, Z_{-ky} (pair) or the column
    double sa, sb = 1.0;
    if (pair) {
        i0 = t;
        i1 = (ny - t) % ny;
        sa = ay[t];
        sb = ax[L] + ay[t];
    } else {
        const int c = mlist[t - npair];
        const int kx = c / ny, ky = c - kx * ny;
        i0 = i1 = c;
        sa = ax[kx] + ay[ky];
    }
    const bool mean = pair && t == 0;
    if (mean) sa = 1.0; // not used: the mean column is not eliminated

    // ---- forward elimination, A and B interleaved
    double qa = 0.0, gpa = 0.0, yra = 0.0, yia = 0.0;
    double qb = 0.0, gpb = 0.0, yrb = 0.0, yib = 0.0;
    cx_t<T> z0[U], z1[U];
    auto fetch = [&](int k0, cx_t<T> *a, cx_t<T> *b) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u < nz ? k0 + u : nz - 1;
            a[u] = spec[(size_t)k * lvl + i0];
            b[u] = spec[(size_t)k * lvl + i1];
        }
    };
    fetch(0, z0, z1);
    for (int k0 = 0; k0 < nz; k0 += U) {
        cx_t<T> n0[U], n1[U];
        fetch(k0 + U < nz ? k0 + U : k0, n0, n1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            if (k < nz) {
                double ar, ai, br = 0.0, bi = 0.0;
                if (pair) { // A = (Z + conj Zm)/2, B = (Z - conj Zm)/(2i)
                    const double zr = z0[u].x, zi = z0[u].y, mr = z1[u].x, mi = -(double)z1[u].y;
                    ar = 0.5 * (zr + mr);
                    ai = 0.5 * (zi + mi);
                    br = 0.5 * (zi - mi);
                    bi = -0.5 * (zr - mr);
                } else {
                    ar = z0[u].x;
                    ai = z0[u].y;
                }
                const double fp = f[k], fn = f[k + 1], r = rs[k];
                const double ea = sa * D[k] + fp * qa;
                const double gi_a = 1.0 / (ea + fn);
                const double ca = fp * gpa;
                yra = r * ar + ca * yra;
                yia = r * ai + ca * yia;
                yar[k * st] = yra;
                yai[k * st] = yia;
                ga[k * st] = gi_a;
                qa = ea * gi_a;
                gpa = gi_a;
                if (pair) {
                    const double eb = sb * D[k] + fp * qb;
                    const double gi_b = 1.0 / (eb + fn);
                    const double cb = fp * gpb;
                    yrb = r * br + cb * yrb;
                    yib = r * bi + cb * yib;
                    ybr[k * st] = yrb;
                    ybi[k * st] = yib;
                    gb[k * st] = gi_b;
                    qb = eb * gi_b;
                    gpb = gi_b;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            z0[u] = n0[u];
            z1[u] = n1[u];
        }
    }

    // ---- the mean column: level means minus mu (forward: D-weighted mean;
    // adjoint: plain mean), V x = c by flux prefix sums, then the gauge
    // (forward: zero plain mean; adjoint: sum_k D_k x_k = 0).  Stored into the
    // A workspace as final values.
    if (mean) {
        const double on = 1.0 / ((double)nx * (double)ny);
        double num = 0.0, den = 0.0, tot = 0.0;
        for (int k = 0; k < nz; ++k) {
            num += D[k] * sS[k];
            den += D[k];
            tot += sS[k];
        }
        const double mu = adjoint ? tot * on / (double)nz : num * on / den;
        double F = 0.0, x = 0.0, acc = 0.0, wsum = 0.0;
        for (int k = 0; k < nz; ++k) {
            if (k > 0) {
                const double c = sS[k - 1] * on - mu;
                F += adjoint ? c : D[k - 1] * c;
                x += F / f[k];
            }
            yar[k * st] = x;
            const double wk = adjoint ? D[k] : 1.0;
            acc += wk * x;
            wsum += wk;
        }
        const double shift = acc / wsum;
        for (int k = 0; k < nz; ++k) {
            yar[k * st] -= shift;
            yai[k * st] = 0.0;
        }
    }

    // ---- backward substitution (loads of the next U levels prefetched)
    double xra = 0.0, xia = 0.0, xrb = 0.0, xib = 0.0;
    for (int k1 = nz - 1; k1 >= 0; k1 -= U) {
        double lyar[U], lyai[U], lga[U], lybr[U], lybi[U], lgb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k1 - u >= 0 ? k1 - u : 0;
            lyar[u] = yar[k * st];
            lyai[u] = yai[k * st];
            lga[u] = ga[k * st];
            if (pair) {
                lybr[u] = ybr[k * st];
                lybi[u] = ybi[k * st];
                lgb[u] = gb[k * st];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k1 - u;
            if (k >= 0) {
                const double fn = f[k + 1], o = os[k];
                if (mean) {
                    xra = lyar[u];
                    xia = 0.0;
                } else {
                    xra = lga[u] * (lyar[u] + fn * xra);
                    xia = lga[u] * (lyai[u] + fn * xia);
                }
                if (pair) {
                    xrb = lgb[u] * (lybr[u] + fn * xrb);
                    xib = lgb[u] * (lybi[u] + fn * xib);
                    const double Ar = o * xra, Ai = o * xia, Br = o * xrb, Bi = o * xib;
                    spec[(size_t)k * lvl + i0] = cx_t<T>{(T)(Ar - Bi), (T)(Ai + Br)};
                    if (i1 != i0) spec[(size_t)k * lvl + i1] = cx_t<T>{(T)(Ar + Bi), (T)(Br - Ai)};
                } else {
                    spec[(size_t)k * lvl + i0] = cx_t<T>{(T)(o * xra), (T)(o * xia)};
                }
            }
        }
    }
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
                             const double *rs64, hipStream_t st)
{
    constexpr int CH = NH < 8 ? NH : 8;
    const long ncols = (long)(L - 1) * ny;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 63) / 64;
    hipLaunchKernelGGL((k_columns<T, NH, CH, REFINE>), dim3((unsigned)grid), dim3(256), 0, st, spec,
                       L, ny, nz, tb.ax, tb.ay, tb.f, tb.D, rs, os, maskcnt, ax64, ay64, f64, D64,
                       rs64);
    return hipGetLastError();
}

template <typename T, int NH, bool KEEPG>
static hipError_t columns2_nh(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                              const int *maskcnt, const Tables<T> &tb, hipStream_t st)
{
    constexpr int CH = NH < 8 ? NH : 8;
    const long ncols = (long)(L - 1) * ny;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 127) / 128;
    hipLaunchKernelGGL((k_columns2<T, NH, CH, KEEPG>), dim3((unsigned)grid), dim3(256), 0, st,
                       spec, L, ny, nz, tb.ax, tb.ay, tb.f, tb.D, rs, os, maskcnt);
    return hipGetLastError();
}

template <typename T, bool KEEPG>
static hipError_t columns2_dispatch(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                                    const int *maskcnt, const Tables<T> &tb, hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N) return columns2_nh<T, N, KEEPG>(spec, L, ny, nz, rs, os, maskcnt, tb, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <typename T, int NH, bool KEEPG>
static hipError_t columns3_nh(cx_t<T> *spec, int L, int ny, int nz, int adjoint,
                              const int *maskcnt, const Tables<T> &tb, hipStream_t st)
{
    (void)nz;
    const long ncols = (long)(L - 1) * ny;
    if (ncols <= 0) return hipSuccess;
    const long grid = (ncols + 127) / 128;
    const LevelCoef<T> *ct = reinterpret_cast<const LevelCoef<T> *>(
        adjoint ? tb.coef_adj : tb.coef_fwd);
    hipLaunchKernelGGL((k_columns3<T, NH, KEEPG>), dim3((unsigned)grid), dim3(256), 0, st, spec, L,
                       ny, tb.ax, tb.ay, ct, maskcnt);
    return hipGetLastError();
}

template <typename T, bool KEEPG>
static hipError_t columns3_dispatch(cx_t<T> *spec, int L, int ny, int nz, int adjoint,
                                    const int *maskcnt, const Tables<T> &tb, hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N) return columns3_nh<T, N, KEEPG>(spec, L, ny, nz, adjoint, maskcnt, tb, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

template <typename T, bool REFINE>
static hipError_t columns_dispatch(cx_t<T> *spec, int L, int ny, int nz, const T *rs, const T *os,
                                   const int *maskcnt, const Tables<T> &tb, const double *ax64,
                                   const double *ay64, const double *f64, const double *D64,
                                   const double *rs64, hipStream_t st)
{
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N)                                                                                 \
        return columns_nh<T, N, REFINE>(spec, L, ny, nz, rs, os, maskcnt, tb, ax64, ay64, f64,     \
                                        D64, rs64, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
}

// variant: 0 = four lanes per column (re/im split, pivots recomputed),
// 1 = two lanes per column, pivots recomputed, 2 = two lanes, pivots kept,
// 3 = halves in separate waves with scalar coefficient tables, pivots
// recomputed, 4 = as 3 with pivots kept.
// The in-register refinement always uses variant 0.
template <typename T>
hipError_t launch_columns_impl(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, int refine,
                               const int *maskcnt, const Tables<T> &tb, const Tables<double> *t64,
                               hipStream_t st, int variant)
{
    const int L = nx / 2;
    const T *rs = adjoint ? tb.rs_adj : tb.rs_fwd;
    const T *os = adjoint ? tb.os_adj : nullptr;
    if constexpr (std::is_same<T, float>::value) {
        if (refine) {
            const double *rs64 = adjoint ? t64->rs_adj : t64->rs_fwd;
            return columns_dispatch<float, true>(spec, L, ny, nz, rs, os, maskcnt, tb, t64->ax,
                                                 t64->ay, t64->f, t64->D, rs64, st);
        }
    }
    if (variant == 1)
        return columns2_dispatch<T, false>(spec, L, ny, nz, rs, os, maskcnt, tb, st);
    if (variant == 2)
        return columns2_dispatch<T, true>(spec, L, ny, nz, rs, os, maskcnt, tb, st);
    if (variant == 3)
        return columns3_dispatch<T, false>(spec, L, ny, nz, adjoint, maskcnt, tb, st);
    if (variant == 4)
        return columns3_dispatch<T, true>(spec, L, ny, nz, adjoint, maskcnt, tb, st);
    return columns_dispatch<T, false>(spec, L, ny, nz, rs, os, maskcnt, tb, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, st);
}

template hipError_t launch_columns_impl<float>(cx_t<float> *, int, int, int, int, int, const int *,
                                               const Tables<float> &, const Tables<double> *,
                                               hipStream_t, int);
template hipError_t launch_columns_impl<double>(cx_t<double> *, int, int, int, int, int,
                                                const int *, const Tables<double> &,
                                                const Tables<double> *, hipStream_t, int);

template <typename T, int NH>
static hipError_t special_nh(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, const int *mlist,
                             int nmask, const double *S, const Tables<double> &tb64, hipStream_t st)
{
    const int npw = (ny / 2 + 1 + 7) / 8;
    const int nmw = (nmask + 15) / 16;
    const int grid = (npw + nmw + 3) / 4;
    hipLaunchKernelGGL((k_special_par<T, NH>), dim3(grid), dim3(256), 0, st, spec, nx, ny, nz,
                       adjoint, mlist, nmask, S, tb64.ax, tb64.ay, tb64.f, tb64.D,
                       adjoint ? tb64.rs_adj : tb64.rs_fwd, adjoint ? tb64.os_adj : nullptr);
    return hipGetLastError();
}

// FP64 columns: the packed kx = 0 row, the mean column and the near-singular
// columns.  parallel != 0 selects the register-resident sweep (k_special_par);
// otherwise one thread per task walks its column through the workspace.
template <typename T>
hipError_t launch_special(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, const int *mlist,
                          int nmask, const double *S, double *ws, const Tables<double> &tb64,
                          hipStream_t st, int parallel)
{
    if (parallel == 2) {
        const int ntask = ny / 2 + 1 + nmask;
        const int grid = (ntask + 63) / 64;
        hipLaunchKernelGGL((k_special_seq<T, 16>), dim3(grid), dim3(64), 0, st, spec, nx, ny, nz,
                           adjoint, mlist, nmask, S, ws, tb64.ax, tb64.ay, tb64.f, tb64.D,
                           adjoint ? tb64.rs_adj : tb64.rs_fwd, adjoint ? tb64.os_adj : nullptr);
        return hipGetLastError();
    }
    if (!parallel) {
        const int ntask = ny / 2 + 1 + nmask;
        const int grid = (ntask + 63) / 64;
        hipLaunchKernelGGL(k_special<T>, dim3(grid), dim3(64), 0, st, spec, nx, ny, nz, adjoint,
                           mlist, nmask, S, ws, tb64.ax, tb64.ay, tb64.f, tb64.D,
                           adjoint ? tb64.rs_adj : tb64.rs_fwd, adjoint ? tb64.os_adj : nullptr);
        return hipGetLastError();
    }
    const int need = nz / 2;
#define PS_NH(N)                                                                                   \
    if (need <= N) return special_nh<T, N>(spec, nx, ny, nz, adjoint, mlist, nmask, S, tb64, st);
    PS_NH(1) PS_NH(2) PS_NH(4) PS_NH(8) PS_NH(16) PS_NH(32) PS_NH(64) PS_NH(128)
#undef PS_NH
    return hipErrorInvalidValue;
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
// densities on either side of level k).  Thread per horizontal point, a
// chunk of GK levels per block row; per-level block sums are written in
// fixed order and reduced by k_grad_reduce (no atomics).
// gk = [f (nz+1) | D (nz) | rho (nz) | 1/h (nz+1, same indexing as f)].
constexpr int GK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_grad_rho(const T *__restrict__ lam, const T *__restrict__ p,
                                                  int nxy, int nz, const double *__restrict__ gk,
                                                  double *__restrict__ partial, int nblk)
{
    __shared__ double red[4][GK];
    const double *f = gk, *D = gk + nz + 1, *rho = D + nz, *ih = rho + nz;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = blockIdx.y * GK;
    const bool ok = c < nxy;
    auto P = [&](int k) { return ok && k >= 0 && k < nz ? (double)p[(size_t)k * nxy + c] : 0.0; };
    auto Lm = [&](int k) { return ok && k >= 0 && k < nz ? (double)lam[(size_t)k * nxy + c] : 0.0; };
    double pm = P(k0 - 1), pc = P(k0), lm = Lm(k0 - 1), lc = Lm(k0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int kk = 0; kk < GK; ++kk) {
        const int k = k0 + kk;
        if (k >= nz) break;
        const double pp = P(k + 1), lp = Lm(k + 1);
        double Vp = 0.0, t = 0.0;
        if (k + 1 < nz) Vp += f[k + 1] * (pp - pc);
        if (k > 0) Vp -= f[k] * (pc - pm);
        Vp /= D[k];
        t = -lc * Vp / rho[k];
        if (k + 1 < nz) t += 0.5 * (pp - pc) * ih[k + 1] * (lc / D[k] - lp / D[k + 1]);
        if (k > 0) t += 0.5 * (pc - pm) * ih[k] * (lm / D[k - 1] - lc / D[k]);
        t = wave_sum(ok ? t : 0.0);
        if (lane == 0) red[wv][kk] = t;
        pm = pc;
        pc = pp;
        lm = lc;
        lc = lp;
    }
    __syncthreads();
    if (threadIdx.x < GK && k0 + (int)threadIdx.x < nz) {
        const int kk = threadIdx.x;
        partial[(size_t)(k0 + kk) * nblk + blockIdx.x] =
            ((red[0][kk] + red[1][kk]) + red[2][kk]) + red[3][kk];
    }
}

__global__ void k_grad_reduce(const double *__restrict__ partial, int nblk, int nz,
                              double *__restrict__ g)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(size_t)k * nblk + b];
    g[k] = -s;
}

int grad_blocks(int nx, int ny) { return (nx * ny + 255) / 256; }

template <typename T>
hipError_t launch_grad_rho(const T *lam, const T *p, int nx, int ny, int nz, const double *gk,
                           double *partial, int nblk, double *grho, hipStream_t st)
{
    dim3 grid(nblk, (nz + GK - 1) / GK);
    hipLaunchKernelGGL(k_grad_rho<T>, grid, dim3(256), 0, st, lam, p, nx * ny, nz, gk, partial,
                       nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_reduce, dim3((nz + 63) / 64), dim3(64), 0, st, partial, nblk, nz,
                       grho);
    return hipGetLastError();
}

template hipError_t launch_grad_rho<float>(const float *, const float *, int, int, int,
                                           const double *, double *, int, double *, hipStream_t);
template hipError_t launch_grad_rho<double>(const double *, const double *, int, int, int,
                                            const double *, double *, int, double *, hipStream_t);

} // namespace ps
