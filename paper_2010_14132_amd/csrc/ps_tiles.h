// Device-side work tiles shared by the standalone kernels and the batched
// persistent kernel: the Stockham transform tiles (x forward with FP64 row
// sums, y pass, x backward), the uniform-half column sweep over 128 columns
// and the compact FP64 column task.  Each is executed by one 256-thread
// block (the FP64 task by one lane).
#pragma once
#include <type_traits>
#include "ps_internal.h"
#include "../../include/pressure_solve.h"

namespace ps {

// ---------------------------------------------------------------- x forward
// Block: `rows` consecutive rows (row g = level * ny + j).  Also records the
// FP64 sum of every input row (for the mean column).
template <typename T>
__device__ void fwd_x_tile(const T *__restrict__ in, cx_t<T> *__restrict__ spec,
                           double *__restrict__ rowsum, int nx, int ny, int nrows_total, int rows,
                           int row0, const StagePlan &sp, const cx_t<T> *__restrict__ twx,
                           const cx_t<T> *__restrict__ tws, unsigned char *smem)
{
    using C = cx_t<T>;
    const int L = nx >> 1;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * L;
    C *stw = b + rows * L;
    C *sws = stw + L;
    const int nr = min(rows, nrows_total - row0);

    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        stw[t] = twx[t];
        sws[t] = tws[t];
    }
    // The block's rows are one contiguous run of nr * L complex pairs.
    const C *src = reinterpret_cast<const C *>(in) + (size_t)row0 * L;
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) a[t] = src[t];
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

    // Even/odd split, X_k = E_k + W_nx^k O_k with E_k = (Z_k + conj Z_{L-k})/2
    // and O_k = (Z_k - conj Z_{L-k})/(2i); slot 0 holds X_0 + i X_{L}.
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

// ---------------------------------------------------------------- y pass
// In-place complex transform of contiguous rows of length ny.  The rows
// transformed are (level, kx) for kx in [kxlo, kxlo + kxcnt) of a spectrum
// with L rows per level: row r maps to (r / kxcnt) L + kxlo + r % kxcnt.
template <typename T, int DIR>
__device__ void fft_y_tile(cx_t<T> *__restrict__ spec, int nrows_total, int ny, int rows, int row0,
                           const StagePlan &sp, const cx_t<T> *__restrict__ twy, int L, int kxlo,
                           int kxcnt, unsigned char *smem)
{
    using C = cx_t<T>;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * ny;
    C *stw = b + rows * ny;
    const int nr = min(rows, nrows_total - row0);
    for (int t = threadIdx.x; t < ny; t += blockDim.x) stw[t] = twy[t];
    for (int t = threadIdx.x; t < nr * ny; t += blockDim.x) {
        const int rr = row0 + t / ny, e = t - (t / ny) * ny;
        const long row = (long)(rr / kxcnt) * L + kxlo + rr % kxcnt;
        a[t] = spec[row * ny + e];
    }
    __syncthreads();
    C *Z = stockham_rows<DIR>(a, b, nr, ny, sp, stw);
    for (int t = threadIdx.x; t < nr * ny; t += blockDim.x) {
        const int rr = row0 + t / ny, e = t - (t / ny) * ny;
        const long row = (long)(rr / kxcnt) * L + kxlo + rr % kxcnt;
        spec[row * ny + e] = Z[t];
    }
}

// ---------------------------------------------------------------- x backward
// Gathers a block of rows from the transposed spectrum, undoes the packing
// (Z_k = (X_k + conj X_{L-k}) + i W_nx^{-k} (X_k - conj X_{L-k})), runs the
// nx/2-point backward transform and writes real rows (optionally added to
// what out already holds).
template <typename T>
__device__ void inv_x_tile(const cx_t<T> *__restrict__ spec, T *__restrict__ out, int nx, int ny,
                           int nrows_total, int rows, int row0, int accumulate,
                           const StagePlan &sp, const cx_t<T> *__restrict__ twx,
                           const cx_t<T> *__restrict__ tws, unsigned char *smem)
{
    using C = cx_t<T>;
    const int L = nx >> 1;
    C *a = reinterpret_cast<C *>(smem);
    C *b = a + rows * L;
    C *stw = b + rows * L;
    C *sws = stw + L;
    const int nr = min(rows, nrows_total - row0);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        stw[t] = twx[t];
        sws[t] = tws[t];
    }
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int kx = t / nr, r = t - kx * nr;
        const int g = row0 + r;
        const int lev = g / ny, j = g - lev * ny;
        a[r * L + kx] = spec[((size_t)lev * L + kx) * ny + j];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        const int r = t / L, k = t - r * L;
        const C *xr = a + r * L;
        C Z;
        if (k == 0) {
            const T x0 = xr[0].x, xl = xr[0].y;
            Z = C{x0 + xl, x0 - xl};
        } else {
            C xk = xr[k], xc = cconj(xr[L - k]);
            C s = cadd(xk, xc);
            C dw = cmul(csub(xk, xc), cconj(sws[k]));
            Z = C{s.x - dw.y, s.y + dw.x};
        }
        b[t] = Z;
    }
    __syncthreads();
    C *R = stockham_rows<1>(b, a, nr, L, sp, stw);
    C *dst = reinterpret_cast<C *>(out) + (size_t)row0 * L;
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) {
        C v = R[t];
        if (accumulate) v = cadd(v, dst[t]);
        dst[t] = v;
    }
}

// ----------------------------------------------------------- uniform-half sweep
// Reciprocal of a pivot u > 0 in the normal range.  FP32: the hardware
// reciprocal refined by one Newton step (within one ulp of the IEEE
// quotient); FP64: IEEE division.
// Column access of the uniform-half kernels through a buffer resource over
// the spectrum: the level's byte offset (wave-uniform, from the scalar
// table) is the instruction's scalar offset and the column's lane part its
// 32-bit vector offset, so no 64-bit address arithmetic runs per access.
// Both offsets stay below 2^32: the spectrum of the supported sizes is at
// most 2 GiB.  Raw (untyped) 32-bit data format, no range clamp.  Loads and
// stores are non-temporal: the kernel overwrites what it reads, and its
// stores, written through rather than left dirty in the caches, no longer
// cost the next pass their write-back.
constexpr int kNonTemporal = 2; // buffer instruction cache policy: nt
struct ColBuf {
    __amdgpu_buffer_rsrc_t r;
    unsigned lane_off;
};
__device__ __forceinline__ ColBuf col_buf(const void *spec, unsigned lane_off)
{
    return ColBuf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(spec), 0, 0xffffffffu,
                                                    0x00020000),
                  lane_off};
}
template <typename V> __device__ __forceinline__ V col_load(const ColBuf &b, long long off)
{
    static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "element size");
    if constexpr (sizeof(V) == 4)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(b.r, b.lane_off, (int)off, kNonTemporal));
    else if constexpr (sizeof(V) == 8)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(b.r, b.lane_off, (int)off, kNonTemporal));
    else
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(b.r, b.lane_off, (int)off, kNonTemporal));
}
template <typename V> __device__ __forceinline__ void col_store(const ColBuf &b, long long off, V v)
{
    if constexpr (sizeof(V) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, b.lane_off,
                                              (int)off, kNonTemporal);
    else if constexpr (sizeof(V) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), b.r, b.lane_off,
            (int)off, kNonTemporal);
    else
        __builtin_amdgcn_raw_buffer_store_b128(
            __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), b.r, b.lane_off,
            (int)off, kNonTemporal);
}

__device__ __forceinline__ float pivot_rcp(float u)
{
    const float r = __builtin_amdgcn_rcpf(u);
    const float e = __builtin_fmaf(-u, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}
__device__ __forceinline__ double pivot_rcp(double u) { return 1.0 / u; }
// FP64 reciprocal of u > 0 in the normal range, for the latency-bound FP64
// column sweeps: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - u r) (each step squares the relative error), a shorter
// dependent chain than IEEE division; within a few ulp of 1/u, not always
// the correctly rounded quotient.
__device__ __forceinline__ double fp64_rcp(double u)
{
    double r = __builtin_amdgcn_rcp(u);
    double e = __builtin_fma(-u, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-u, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Per-slot coefficients in each half's elimination order (built by the plan):
// slot [half][i], i in [0, NH), for level k = i (low half) or k = nz - 1 - i
// (high half), with the half's real levels in the LAST n slots and dummy
// slots in front (f_prev = f_next = 0, D = 1, rs = 0, real = 0; they read
// the middle row and are never stored).  A dummy row never influences a
// real one: the first real row of each half is a boundary row (f_prev = 0).
// Slot [2 NH] is the middle row m.  rs/os are the forward or adjoint
// right-hand-side and output factors.  `off` is the byte offset of the level
// in the spectrum.  Wave-uniform, so they are read through the scalar cache.
// Two waves per group of 64 columns: the low-half wave eliminates levels
// 0..m-1 and the high-half wave levels nz-1..m+1, one column per lane
// (complex values, real pivots); they exchange their messages to the middle
// row through LDS.  KEEPG keeps the reciprocal pivots in registers instead
// of recomputing them in the backward pass.
// `group` selects 128 consecutive columns of the range [c0, c1) (column
// index kx * ny + ky; c0 >= ny, every kx >= 1); xa / xb
// are LDS scratch of 2 * 2 * 64 values each (the block's 256 threads call
// this together).
template <typename T, int NH, bool KEEPG>
__device__ void columns3_tile(cx_t<T> *__restrict__ spec, int L, int ny, const T *__restrict__ ax,
                              const T *__restrict__ ay, const LevelCoef<T> *__restrict__ coef,
                              const int *__restrict__ maskcnt, long c0, long c1, long group, T (*xa)[2][64],
                              cx_t<T> (*xb)[2][64])
{
    using C = cx_t<T>;
    constexpr int CH = NH < 8 ? NH : 8;
    constexpr int NB = (NH + CH - 1) / CH;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pair = w >> 1, half = w & 1;
    const long col = c0 + (group * 2 + pair) * 64 + lane;
    const bool valid = col < c1;
    const int kx = valid ? (int)((unsigned)col / (unsigned)ny) : 1; // col < 2^31
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const T s = ax[kx] + ay[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    const ColBuf cb = col_buf(spec, (unsigned)((valid ? col : 0) * sizeof(C)));
    const LevelCoef<T> *ct = coef + half * NH;

    C v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const C x = col_load<C>(cb, ct[i].off);
        v[i] = C{x.x * ct[i].rs, x.y * ct[i].rs};
    }
    const LevelCoef<T> cm = coef[2 * NH];
    C rmv = col_load<C>(cb, cm.off);
    rmv = C{rmv.x * cm.rs, rmv.y * cm.rs};

    T qck[KEEPG ? 1 : NB];
    T gk[KEEPG ? NH : 1];
    T q = T(0), g = T(0);
    C y = C{T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i % CH == 0) __asm__ volatile("" ::: "memory"); // keep table loads near their use
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
            __asm__ volatile("" ::: "memory");
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
            if (ct[i].real) col_store<C>(cb, ct[i].off, C{v[i].x * ct[i].os, v[i].y * ct[i].os});
        }
        if (half) col_store<C>(cb, cm.off, C{xm.x * cm.os, xm.y * cm.os});
    }
}

// ----------------------------------------------------------- refined sweep (FP32)
// columns3_tile followed by one refinement: the residual rho = r - M x of
// every column is formed in FP64 from the FP64 coefficient table (same slot
// layout; s from the FP64 wavenumber tables) and the FP32 solution, rounded
// to FP32, and M d = rho is solved with the same FP32 elimination; x + d is
// stored.  The elimination of the correction has the same pivots, so only
// the right-hand-side part of the middle-row message is exchanged again.
// Pivots are recomputed from checkpoints in both backward passes.  xe is LDS
// scratch of 2 * 2 * 64 complex values (the halves' last solution values,
// which the middle row's residual needs).
template <int NH>
__device__ void columns3r_tile(float2 *__restrict__ spec, int L, int ny, const float *__restrict__ ax,
                               const float *__restrict__ ay,
                               const LevelCoef<float> *__restrict__ coef,
                               const LevelCoef<double> *__restrict__ coef64,
                               const double *__restrict__ ax64, const double *__restrict__ ay64,
                               const int *__restrict__ maskcnt, long c0, long c1, long group, float (*xa)[2][64],
                               float2 (*xb)[2][64], float2 (*xe)[2][64])
{
    using C = float2;
    constexpr int CH = NH < 8 ? NH : 8;
    constexpr int NB = (NH + CH - 1) / CH;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pair = w >> 1, half = w & 1;
    const long col = c0 + (group * 2 + pair) * 64 + lane;
    const bool valid = col < c1;
    const int kx = valid ? (int)((unsigned)col / (unsigned)ny) : 1; // col < 2^31
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const float s = ax[kx] + ay[ky];
    const double s64 = ax64[kx] + ay64[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    const ColBuf cb = col_buf(spec, (unsigned)((valid ? col : 0) * sizeof(C)));
    const LevelCoef<float> *ct = coef + half * NH;
    const LevelCoef<double> *ct64 = coef64 + half * NH;
    const LevelCoef<float> cm = coef[2 * NH];
    const LevelCoef<double> cm64 = coef64[2 * NH];

    C raw[NH], v[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        raw[i] = col_load<C>(cb, ct[i].off);
        v[i] = C{raw[i].x * ct[i].rs, raw[i].y * ct[i].rs};
    }
    const C rawm = col_load<C>(cb, cm.off);

    // ---- solve M x = r
    float qck[NB];
    float q = 0.f, g = 0.f;
    C y = C{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i % CH == 0) {
            qck[i / CH] = q;
            __asm__ volatile("" ::: "memory"); // keep table loads near their use
        }
        const float e = s * ct[i].D + ct[i].fp * q;
        const float gi = pivot_rcp(e + ct[i].fn);
        const float c = ct[i].fp * g;
        y = C{v[i].x + c * y.x, v[i].y + c * y.y};
        v[i] = y;
        q = e * gi;
        g = gi;
    }
    const float fl = ct[NH - 1].fn;
    const float gl = fl * g;
    xa[pair][half][lane] = fl * q;
    xb[pair][half][lane] = C{gl * y.x, gl * y.y};
    __syncthreads();
    const float den = (s * cm.D + xa[pair][0][lane]) + xa[pair][1][lane];
    C lb = xb[pair][0][lane], hb = xb[pair][1][lane];
    C xm = C{((rawm.x * cm.rs + lb.x) + hb.x) / den, ((rawm.y * cm.rs + lb.y) + hb.y) / den};
    auto backward = [&](C(&a)[NH], C xn) {
#pragma unroll
        for (int bb = NB - 1; bb >= 0; --bb) {
            float gb[CH];
            float qq = qck[bb];
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = bb * CH + c;
                const float e = s * ct[i].D + ct[i].fp * qq;
                const float gi = pivot_rcp(e + ct[i].fn);
                gb[c] = gi;
                qq = e * gi;
            }
#pragma unroll
            for (int c = CH - 1; c >= 0; --c) {
                const int i = bb * CH + c;
                const float fn = ct[i].fn;
                xn = C{gb[c] * (a[i].x + fn * xn.x), gb[c] * (a[i].y + fn * xn.y)};
                a[i] = xn;
            }
        }
    };
    backward(v, xm);

    // ---- residual in FP64 (dummy slots give 0: rs = fp = fn = 0, x = 0)
    xe[pair][half][lane] = v[NH - 1];
    __syncthreads(); // also: every wave has read xb above
    const C xlo = xe[pair][0][lane], xhi = xe[pair][1][lane];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const double fp = ct64[i].fp, fn = ct64[i].fn, r = ct64[i].rs;
        const double diag = s64 * ct64[i].D + fp + fn;
        const C xp = i > 0 ? v[i - 1] : C{0.f, 0.f};
        const C xn = i + 1 < NH ? v[i + 1] : xm;
        const double rr = r * (double)raw[i].x -
                          (diag * (double)v[i].x - fp * (double)xp.x - fn * (double)xn.x);
        const double ri = r * (double)raw[i].y -
                          (diag * (double)v[i].y - fp * (double)xp.y - fn * (double)xn.y);
        raw[i] = C{(float)rr, (float)ri};
    }
    const double diagm = s64 * cm64.D + cm64.fp + cm64.fn;
    const C rhom = C{(float)(cm64.rs * (double)rawm.x -
                             (diagm * (double)xm.x - cm64.fp * (double)xlo.x -
                              cm64.fn * (double)xhi.x)),
                     (float)(cm64.rs * (double)rawm.y -
                             (diagm * (double)xm.y - cm64.fp * (double)xlo.y -
                              cm64.fn * (double)xhi.y))};

    // ---- correction: same elimination on the residual
    q = 0.f;
    g = 0.f;
    y = C{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i % CH == 0) __asm__ volatile("" ::: "memory");
        const float e = s * ct[i].D + ct[i].fp * q;
        const float gi = pivot_rcp(e + ct[i].fn);
        const float c = ct[i].fp * g;
        y = C{raw[i].x + c * y.x, raw[i].y + c * y.y};
        raw[i] = y;
        q = e * gi;
        g = gi;
    }
    xb[pair][half][lane] = C{gl * y.x, gl * y.y};
    __syncthreads();
    lb = xb[pair][0][lane];
    hb = xb[pair][1][lane];
    const C dm = C{((rhom.x + lb.x) + hb.x) / den, ((rhom.y + lb.y) + hb.y) / den};
    backward(raw, dm);
    xm = C{xm.x + dm.x, xm.y + dm.y};

    if (store) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            if (ct[i].real)
                col_store<C>(cb, ct[i].off,
                             C{(v[i].x + raw[i].x) * ct[i].os, (v[i].y + raw[i].y) * ct[i].os});
        }
        if (half) col_store<C>(cb, cm.off, C{xm.x * cm.os, xm.y * cm.os});
    }
}

// ----------------------------------------------------------- split-lane sweep
// As columns3_tile, with the real and imaginary parts of a column half in
// two adjacent lanes (lane 2c + comp, comp 0: real, 1: imaginary): a wave
// pair covers 32 columns, each lane holds NH real values, and both lanes of
// a column compute the (real) pivots.  Half the registers per lane of the
// complex form, for FP64 and for the refining FP32 form.  REFINE (FP32 only)
// adds the refinement of columns3r_tile: FP64 residual from the FP64 table,
// FP32 correction with the same elimination.  xa, xb, xe: LDS scratch of
// 2 * 2 * 64 values each.  SHG: the reciprocal pivots of the first forward
// sweep are kept in LDS (gsh, 4 waves x NH x 32 values: one per column and
// level, written by both lanes of the column with the same value) and read
// back by the later sweeps instead of being recomputed from checkpoints.
// PPB: wave pairs per block (2: 256 threads and 64 columns, 1: 128 threads
// and 32 columns).
template <typename T, int NH, bool REFINE, bool SHG = false, int PPB = 2>
__device__ void columns3s_tile(cx_t<T> *__restrict__ spec, int L, int ny, const T *__restrict__ ax,
                               const T *__restrict__ ay, const LevelCoef<T> *__restrict__ coef,
                               const LevelCoef<double> *__restrict__ coef64,
                               const double *__restrict__ ax64, const double *__restrict__ ay64,
                               const int *__restrict__ maskcnt, long c0, long c1, long group, T (*xa)[2][64],
                               T (*xb)[2][64], T (*xe)[2][64], T *gsh = nullptr)
{
    constexpr int CH = NH < 8 ? NH : 8;
    constexpr int NB = (NH + CH - 1) / CH;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pair = w >> 1, half = w & 1;
    // this lane's pivot of slot i: gw[i * 32]
    T *gw = SHG ? gsh + (size_t)w * NH * 32 + (lane >> 1) : nullptr;
    // Pivot loads of the later sweeps: one chunk of GC levels is fetched
    // while the previous chunk is computed.  The fences take the sweep's
    // running value as an operand, so that a chunk's loads cannot be issued
    // before the chunk two steps back has been computed (otherwise all NH
    // loads are hoisted to the start of the sweep, NH registers live).
    // The array's address also goes into an asm statement: an LDS array
    // whose address never escapes is taken to be untouched by the fences,
    // and the pivots stored by the first sweep are then forwarded in
    // registers to the later sweeps.
    if constexpr (SHG) __asm__ volatile("" ::"s"(gsh) : "memory");
    constexpr int GC = NH < 4 ? NH : 4; // levels per pivot chunk
    constexpr int NG = NH / GC;
    auto gload = [&](T(&gd)[GC], int bb) {
#pragma unroll
        for (int c = 0; c < GC; ++c) gd[c] = gw[(bb * GC + c) * 32];
    };
    const long col = c0 + (group * PPB + pair) * 32 + (lane >> 1);
    const bool valid = col < c1;
    const int kx = valid ? (int)((unsigned)col / (unsigned)ny) : 1; // col < 2^31
    const int ky = valid ? (int)(col - (long)kx * ny) : 0;
    const T s = ax[kx] + ay[ky];
    bool store = valid;
    if (maskcnt && valid) {
        const int d = min(ky, ny - ky);
        if (d < maskcnt[kx]) store = false;
    }
    const ColBuf cb =
        col_buf(spec, (unsigned)((valid ? col : 0) * sizeof(cx_t<T>) + (lane & 1) * sizeof(T)));
    const LevelCoef<T> *ct = coef + half * NH;
    const LevelCoef<T> cm = coef[2 * NH];

    T v[NH];
    T raw[REFINE ? NH : 1];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const T x = col_load<T>(cb, ct[i].off);
        if constexpr (REFINE) raw[i] = x;
        v[i] = x * ct[i].rs;
    }
    const T rawm = col_load<T>(cb, cm.off);

    T qck[SHG ? 1 : NB];
    T q = T(0), g = T(0), y = T(0);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i % CH == 0) {
            if constexpr (!SHG) qck[i / CH] = q;
            __asm__ volatile("" ::: "memory"); // keep the table loads near their use
        }
        const T e = s * ct[i].D + ct[i].fp * q;
        const T gi = pivot_rcp(e + ct[i].fn);
        y = v[i] + (ct[i].fp * g) * y;
        v[i] = y;
        q = e * gi;
        g = gi;
        if constexpr (SHG) gw[i * 32] = gi;
    }
    const T gl = ct[NH - 1].fn * g;
    xa[pair][half][lane] = ct[NH - 1].fn * q;
    xb[pair][half][lane] = gl * y;
    __syncthreads();
    const T den = (s * cm.D + xa[pair][0][lane]) + xa[pair][1][lane];
    T xm = ((rawm * cm.rs + xb[pair][0][lane]) + xb[pair][1][lane]) / den;
    // FIN (SHG only): the last backward sweep, which stores each level's
    // result as soon as it is final (a is the correction when REFINE), so
    // that the stores spread over the sweep instead of leaving in one burst.
    auto backward = [&](T(&a)[NH], T xn, auto fin) {
        if constexpr (SHG) {
            T gc[GC], gn[GC];
            gload(gc, NG - 1);
#pragma unroll
            for (int bb = NG - 1; bb >= 0; --bb) {
                __asm__ volatile("" : "+v"(xn)::"memory");
                if (bb > 0) gload(gn, bb - 1);
#pragma unroll
                for (int c = GC - 1; c >= 0; --c) {
                    const int i = bb * GC + c;
                    xn = gc[c] * (a[i] + ct[i].fn * xn);
                    a[i] = xn;
                    if constexpr (decltype(fin)::value)
                        if (ct[i].real)
                            col_store<T>(cb, ct[i].off, (REFINE ? v[i] + xn : xn) * ct[i].os);
                }
#pragma unroll
                for (int c = 0; c < GC; ++c) gc[c] = gn[c];
            }
            return;
        }
#pragma unroll
        for (int bb = NB - 1; bb >= 0; --bb) {
            T gb[CH];
            T qq = qck[SHG ? 0 : bb];
            __asm__ volatile("" ::: "memory");
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
                xn = gb[c] * (a[i] + ct[i].fn * xn);
                a[i] = xn;
            }
        }
    };
    if constexpr (SHG && !REFINE) {
        if (store) backward(v, xm, std::true_type{});
    } else {
        backward(v, xm, std::false_type{});
    }

    if constexpr (REFINE) {
        const LevelCoef<double> *ct64 = coef64 + half * NH;
        const LevelCoef<double> cm64 = coef64[2 * NH];
        const double s64 = ax64[kx] + ay64[ky];
        xe[pair][half][lane] = v[NH - 1];
        __syncthreads(); // also: every wave has read xb above
        const double xlo = xe[pair][0][lane], xhi = xe[pair][1][lane];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const double fp = ct64[i].fp, fn = ct64[i].fn;
            const double diag = s64 * ct64[i].D + fp + fn;
            const double xp = i > 0 ? (double)v[i - 1] : 0.0;
            const double xn = i + 1 < NH ? (double)v[i + 1] : (double)xm;
            raw[i] = (T)(ct64[i].rs * (double)raw[i] - (diag * (double)v[i] - fp * xp - fn * xn));
            // (SHG) the scheduler otherwise converts most of raw to FP64 at once
            if (SHG && i % CH == CH - 1) __builtin_amdgcn_sched_barrier(0);
        }
        const double diagm = s64 * cm64.D + cm64.fp + cm64.fn;
        const T rhom = (T)(cm64.rs * (double)rawm -
                           (diagm * (double)xm - cm64.fp * xlo - cm64.fn * xhi));
        q = T(0);
        g = T(0);
        y = T(0);
        if constexpr (SHG) {
            T gc[GC], gn[GC];
            gload(gc, 0);
#pragma unroll
            for (int bb = 0; bb < NG; ++bb) {
                __asm__ volatile("" : "+v"(y)::"memory");
                if (bb + 1 < NG) gload(gn, bb + 1);
#pragma unroll
                for (int c = 0; c < GC; ++c) {
                    const int i = bb * GC + c;
                    y = raw[i] + (ct[i].fp * g) * y;
                    raw[i] = y;
                    g = gc[c];
                }
#pragma unroll
                for (int c = 0; c < GC; ++c) gc[c] = gn[c];
            }
        } else {
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                if (i % CH == 0) __asm__ volatile("" ::: "memory");
                const T e = s * ct[i].D + ct[i].fp * q;
                const T gi = pivot_rcp(e + ct[i].fn);
                y = raw[i] + (ct[i].fp * g) * y;
                raw[i] = y;
                q = e * gi;
                g = gi;
            }
        }
        xb[pair][half][lane] = gl * y;
        __syncthreads();
        const T dm = ((rhom + xb[pair][0][lane]) + xb[pair][1][lane]) / den;
        if constexpr (SHG) {
            if (store) backward(raw, dm, std::true_type{});
        } else {
            backward(raw, dm, std::false_type{});
#pragma unroll
            for (int i = 0; i < NH; ++i) v[i] += raw[i];
        }
        xm += dm;
    }

    if (store) {
        if constexpr (!SHG) {
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                if (ct[i].real) col_store<T>(cb, ct[i].off, v[i] * ct[i].os);
            }
        }
        if (half) col_store<T>(cb, cm.off, xm * cm.os);
    }
}

// ----------------------------------------------------------- the mean column
// The singular (0,0) column (FP64) from the level sums sS (unnormalised
// level sums of the input), written as final values to xr[k * stride]
// (xi[k * stride], used as scratch, ends zero).  The projection removes the
// mean M of the level sums (forward: D-weighted, adjoint: plain), so the
// column's right-hand side is c_k = (S_k - M)/(nx ny).  The face fluxes
// F_{k+1/2} = sum_{j<=k} t_j (t_j = D_j c_j forward, c_j adjoint) are zero at
// both ends (the projection makes the terms sum to zero), so each face's
// flux is taken from whichever end carries less weight: the bottom-up sum,
// or minus the top-down sum of the levels above.  Equal in exact
// arithmetic; in FP64 it keeps the rounding of the long sums out of the
// faces near the top, where the level differences F / f_{k+1/2} amplify it
// (f is small there on stretched grids with decaying density).  Then
// x_{k+1} = x_k + F_{k+1/2} / f_{k+1/2}, x_0 = 0, and the gauge (forward:
// zero plain mean over levels; adjoint: sum_k D_k x_k = 0).
__device__ inline void mean_column_fp64(int nz, int nx, int ny, int adjoint,
                                        const double *f, const double *D, const double *sS,
                                        double *xr, double *xi, int stride)
{
    const double on = 1.0 / ((double)nx * (double)ny);
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double w = adjoint ? 1.0 : D[k];
        num += w * sS[k];
        den += w;
    }
    const double M = num / den;
    double a = 0.0;
    for (int k = nz - 1; k >= 0; --k) {
        xi[(size_t)k * stride] = a; // sum of the terms above level k
        const double c = (sS[k] - M) * on;
        a += adjoint ? c : D[k] * c;
    }
    double P = 0.0, wlo = 0.0, x = 0.0;
    xr[0] = 0.0;
    for (int k = 0; k + 1 < nz; ++k) {
        const double c = (sS[k] - M) * on;
        P += adjoint ? c : D[k] * c;
        wlo += adjoint ? 1.0 : D[k];
        const double F = wlo <= den - wlo ? P : -xi[(size_t)k * stride];
        x += F / f[k + 1];
        xr[(size_t)(k + 1) * stride] = x;
    }
    double acc = 0.0, wsum = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double wk = adjoint ? D[k] : 1.0;
        acc += wk * xr[(size_t)k * stride];
        wsum += wk;
    }
    const double shift = acc / wsum;
    for (int k = 0; k < nz; ++k) {
        xr[(size_t)k * stride] -= shift;
        xi[(size_t)k * stride] = 0.0;
    }
}

// The same mean column computed by one whole wave (64 lanes; nz <= 256, so
// lane l takes levels 4l .. 4l+3): the sums are lane partials combined in a
// fixed butterfly, the bottom-up and top-down flux sums and the level
// differences are prefix / suffix sums (lane-local runs plus a scan of the
// lane totals).  The same definitions as mean_column_fp64 (including each
// face's choice between the two flux sums), summed in another order.
__device__ inline double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}
__device__ inline double wave_incl_scan_rev(double v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_down(v, o, 64);
        if (lane + o < 64) v += u;
    }
    return v;
}
__device__ inline void mean_column_wave(int nz, int nx, int ny, int adjoint, const double *f,
                                        const double *D, const double *sS, double *xr,
                                        double *xi, int stride)
{
    constexpr int P = 4;
    const int lane = threadIdx.x & 63;
    const int k0 = lane * P;
    const double on = 1.0 / ((double)nx * (double)ny);
    double w[P], t[P];
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = k0 + q;
        w[q] = k < nz ? (adjoint ? 1.0 : D[k]) : 0.0;
        num += k < nz ? w[q] * sS[k] : 0.0;
        den += w[q];
    }
    num = wave_sum(num);
    den = wave_sum(den);
    const double M = num / den;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = k0 + q;
        t[q] = k < nz ? w[q] * ((sS[k] - M) * on) : 0.0;
    }
    // bottom-up sums P_k and weights W_k (inclusive), top-down sums of the
    // levels above k (exclusive)
    double lt = 0.0, lw = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        lt += t[q];
        lw += w[q];
    }
    const double pt = wave_incl_scan(lt, lane) - lt, pw = wave_incl_scan(lw, lane) - lw;
    const double st = wave_incl_scan_rev(lt, lane) - lt;
    double up[P], wl[P], dn[P];
    double a = pt, b = pw;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        a += t[q];
        b += w[q];
        up[q] = a;
        wl[q] = b;
    }
    double c = st;
#pragma unroll
    for (int q = P - 1; q >= 0; --q) {
        dn[q] = c;
        c += t[q];
    }
    // level differences d_k = F_{k+1/2} / f_{k+1/2} (k < nz - 1), then
    // x_{k+1} = sum_{j <= k} d_j, x_0 = 0
    double d[P], ld = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = k0 + q;
        const double F = wl[q] <= den - wl[q] ? up[q] : -dn[q];
        d[q] = k + 1 < nz ? F / f[k + 1] : 0.0;
        ld += d[q];
    }
    const double pd = wave_incl_scan(ld, lane) - ld;
    double x[P];
    double e = pd;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        x[q] = e; // x_k = sum_{j < k} d_j
        e += d[q];
    }
    double acc = 0.0, wsum = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = k0 + q;
        const double wk = k < nz ? (adjoint ? D[k] : 1.0) : 0.0;
        acc += wk * x[q];
        wsum += wk;
    }
    acc = wave_sum(acc);
    wsum = wave_sum(wsum);
    const double shift = acc / wsum;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = k0 + q;
        if (k < nz) {
            xr[(size_t)k * stride] = x[q] - shift;
            xi[(size_t)k * stride] = 0.0;
        }
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
// The calling block stages the FP64 tables in LDS first: f (nz + 1 values),
// D, rs, os and the level sums sS (nz values each).  t is the task index
// (tasks >= ntask return at once).
template <typename T, int U>
__device__ void special_seq_tile(cx_t<T> *__restrict__ spec, int nx, int ny, int nz, int adjoint,
                                 const int *__restrict__ mlist, int nmask, double *__restrict__ ws,
                                 const double *__restrict__ ax, const double *__restrict__ ay,
                                 const double *f, const double *D, const double *rs,
                                 const double *os, const double *sS, int t)
{
    const int L = nx / 2;
    const int npair = ny / 2 + 1;
    const int ntask = npair + nmask;
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

    // ---- the mean column, stored into the A workspace as final values
    if (mean) mean_column_fp64(nz, nx, ny, adjoint, f, D, sS, yar, yai, (int)st);

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

} // namespace ps
