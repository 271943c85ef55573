// Register-resident transform kernels for power-of-two lengths L = R1 R2
// (R1 divides R2): same layouts and results as the Stockham kernels in
// fft.hip, with each row held by R1 lanes in registers (four_step), global
// loads and stores straight to and from registers, and LDS used only for the
// one transposition inside the row transform and, in the x passes, for the
// [row][kx] <-> [kx][row] transposition of the spectral layout.
#include "ps_internal.h"
#include "../../include/pressure_solve.h"

namespace ps {

// LDS slot of element (kx, rr) of the x passes' [kx][row] staging (ROWS rows
// of L values): rows XOR-swizzled per kx so that both the column-wise writes
// (R1 consecutive kx of each row) and the row-wise reads (ROWS consecutive
// rows of each kx) hit distinct banks.
template <int R1, int ROWS> __device__ __forceinline__ int stage_idx(int kx, int rr)
{
    constexpr int KB = R1 / ROWS > 1 ? R1 / ROWS : 1;
    constexpr int KM = ROWS / R1 > 1 ? ROWS / R1 : 1;
    return kx * ROWS + (rr ^ (((kx / KB) * KM) & (ROWS - 1)));
}

// Non-temporal loads and stores: of data that the solve does not touch
// again (the right-hand side in the forward x pass and in the residual
// transform, the spectrum, the result and the accumulated old values in the
// backward x pass), and the forward y pass's stores.
template <typename T> __device__ __forceinline__ cx_t<T> nt_load(const cx_t<T> *p)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 r = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return cx_t<T>{r.x, r.y};
}
template <typename T> __device__ __forceinline__ void nt_store(cx_t<T> v, cx_t<T> *p)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 r = {v.x, v.y};
    __builtin_nontemporal_store(r, reinterpret_cast<v2 *>(p));
}

// ---------------------------------------------------------------- y pass
// In place over contiguous rows of length L (= ny); NT threads = NT / R1
// rows.  Row r of the launch is spectrum row (r / kxcnt) nkx + kxlo +
// r % kxcnt (nkx rows per level).
template <typename T, int R1, int R2, int DIR, int NT>
__global__ __launch_bounds__(NT) void k_fft_y_fast(cx_t<T> *__restrict__ spec, int nrows,
                                                   const cx_t<T> *__restrict__ tw4, int nkx,
                                                   int kxlo, int kxcnt, int swz, int keep)
{
    using C = cx_t<T>;
    constexpr int L = R1 * R2, RB = NT / R1, S = four_step_stride<R1, R2, T>();
    __shared__ T lds[RB * S];
    const int r = threadIdx.x / R1, t = threadIdx.x - r * R1;
    const long rr = (long)tile_of(blockIdx.x, gridDim.x, swz) * RB + r;
    const bool ok = rr < nrows;
    const unsigned ur = ok ? (unsigned)rr : 0u; // rows < 2^31
    const long row = ok ? (long)(ur / (unsigned)kxcnt) * nkx + kxlo + ur % (unsigned)kxcnt : 0;
    C *base = spec + row * (long)L;
    C v[R2], w[R2];
#pragma unroll
    for (int q = 0; q < R2; ++q) v[q] = base[t + R1 * q]; // past the end: row 0, not stored
    four_step<R1, R2, DIR>(v, w, t, lds + r * S, tw4);
    if (ok) {
        // the forward pass stores non-temporally: its rows are read next by
        // the column kernel, which then does not pay for writing back this
        // pass's dirty lines (measured; the backward pass measured better
        // with plain stores).  keep (the kx ranges of a chunked pipeline,
        // small enough to stay in the last-level cache until the column
        // kernel reads them): plain stores.
        if (DIR < 0 && !keep) {
#pragma unroll
            for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1)
                    nt_store<T>(w[j * R1 + k1], &base[(t + R1 * j) + R2 * k1]);
        } else {
#pragma unroll
            for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) base[(t + R1 * j) + R2 * k1] = w[j * R1 + k1];
        }
    }
}

// y passes of the z-fastest solve, between the [kx][j][k] layout (k
// fastest; written and read by the z-fastest x passes) and the spectrum
// spec[k][kx][ky].  A block takes RB = NT / R1 consecutive levels of one kx
// (tiles level-chunk fastest, XCD-contiguous).  Forward: the rows are
// gathered into an LDS staging by loads along k, transformed, and stored
// into the spectrum along ky.  Backward: spectrum rows are loaded along ky,
// transformed, staged in LDS and stored along k.  Levels past the last one read
// level nz - 1 and are never stored.  The row transform is k_fft_y_fast's.
template <typename T, int R1, int R2, int DIR, int NT>
__global__ __launch_bounds__(NT) void k_fft_y_zyx(const cx_t<T> *__restrict__ src,
                                                  cx_t<T> *__restrict__ dst, int nz, int nkx,
                                                  const cx_t<T> *__restrict__ tw4)
{
    using C = cx_t<T>;
    constexpr int L = R1 * R2, RB = NT / R1, S = four_step_stride<R1, R2, T>();
    constexpr int SW = L + 2; // complex values per staged row
    constexpr int SA = RB * S, SB = 2 * RB * SW;
    __shared__ T lds[SA > SB ? SA : SB];
    C *stg = reinterpret_cast<C *>(lds);
    const int r = threadIdx.x / R1, t = threadIdx.x - r * R1;
    const int nkc = (nz + RB - 1) / RB;
    const int tile = tile_of(blockIdx.x, gridDim.x, 1);
    const int kx = tile / nkc, k0 = (tile % nkc) * RB, k = k0 + r;
    C v[R2], w[R2];
    constexpr int IT = RB * L / NT; // staged values per thread: level kk, rows jj0 + (NT / RB) it
    const int kk = threadIdx.x % RB, jj0 = threadIdx.x / RB;
    if constexpr (DIR < 0) {
        const C *col = src + (long)kx * L * nz + (k0 + kk < nz ? k0 + kk : nz - 1);
        C ld[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) ld[it] = col[(long)(jj0 + (NT / RB) * it) * nz];
#pragma unroll
        for (int it = 0; it < IT; ++it) stg[kk * SW + jj0 + (NT / RB) * it] = ld[it];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R2; ++q) v[q] = stg[r * SW + t + R1 * q];
        __syncthreads(); // the staging is read before the transform reuses it
    } else {
        const C *row = src + ((long)(k < nz ? k : nz - 1) * nkx + kx) * L;
#pragma unroll
        for (int q = 0; q < R2; ++q) v[q] = row[t + R1 * q];
    }
    four_step<R1, R2, DIR>(v, w, t, lds + r * S, tw4);
    if constexpr (DIR < 0) {
        if (k < nz) {
            C *row = dst + ((long)k * nkx + kx) * L;
#pragma unroll
            for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1)
                    nt_store<T>(w[j * R1 + k1], &row[(t + R1 * j) + R2 * k1]);
        }
    } else {
        __syncthreads(); // the transform's last LDS reads are done
#pragma unroll
        for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) stg[r * SW + (t + R1 * j) + R2 * k1] = w[j * R1 + k1];
        __syncthreads();
        if (k0 + kk < nz) {
            C *col = dst + (long)kx * L * nz + k0 + kk;
#pragma unroll
            for (int it = 0; it < IT; ++it)
                col[(long)(jj0 + (NT / RB) * it) * nz] = stg[kk * SW + jj0 + (NT / RB) * it];
        }
    }
}

// ---------------------------------------------------------------- x forward
// ROWS rows per block, R1 lanes per row.  Loads z_n = x_{2n} + i x_{2n+1},
// records FP64 row sums, transforms, applies the even/odd split with one
// shuffle per value (the partner of slot (t, j, k1), index L - k, sits in lane
// R1 - t of the same row, or in lane 0's own registers for t = 0), and stores
// the block's rows transposed through LDS (one real component at a time).
// korder (requires ny % ROWS == 0): tiles are taken level-fastest -- tile
// t covers rows j in [(t / nz) ROWS, +ROWS) of level t % nz -- so that, with
// XCD-contiguous tiles, the blocks of levels k-1, k, k+1 of one row range run
// together on one XCD and the residual's vertical neighbours come from L2.
// RES: the transformed row is the residual r = b - A p (b = in) formed with
// FP64 arithmetic from the stored b and p, rounded once to T.  The vertical
// term of row k is a_up p_{k+1} + a_dn p_{k-1} - a_c p_k with per-level
// coefficients rc[3k..3k+2] (forward: f_{k+1/2}/D_k, f_{k-1/2}/D_k,
// (f_{k+1/2}+f_{k-1/2})/D_k; adjoint, A^T = D A D^{-1}: f_{k+1/2}/D_{k+1},
// f_{k-1/2}/D_{k-1}, (f_{k+1/2}+f_{k-1/2})/D_k); zero at the ends.  The x
// neighbours x_{2n-1} and x_{2n+2} of the pair z_n = (x_{2n}, x_{2n+1}) come
// from the neighbouring lanes of the row.
// DIV: the transformed row is scale times the divergence of C-grid
// velocities (in = u on the x-faces i-1/2, pres = v on the y-faces j-1/2,
// wz = w on the faces k-1/2), formed in FP64 and rounded once to T:
// idx2 (u_{i+1} - u_i) + idy2 (v_{j+1} - v_i) + a_up w_{k+1} - a_dn w_k, with
// idx2 = 1/dx, idy2 = 1/dy and per-level rc[3k] = rho_{k+1/2}/D_k,
// rc[3k+1] = rho_{k-1/2}/D_k (zero at the top and bottom faces).  u_{2n+2}
// comes from the neighbouring lane as in RES.
// PAIR (R1 = 2 R2): the row transform is four_step_pair, whose output slot
// kk of lane t = 2m + h is X[m + R2 kk + R2^2 h].
// ZYX: the input is a field in the z-fastest layout ([nx][ny][nz]) and the
// output the [kx][j][k] layout (k fastest) that the z-fastest y pass reads:
// a block's rows are ROWS consecutive levels k of one row j (tiles level-
// chunk fastest, so that neighbouring level chunks of a row meet in one L2),
// its loads run along k into an LDS staging of the rows, and its stores run
// along k (ROWS values per (kx, j)).  The row transform is unchanged.
template <int R1, int R2, bool PAIR> __device__ __forceinline__ int out_index(int t, int i)
{
    if constexpr (PAIR)
        return (t >> 1) + R2 * i + R2 * R2 * (t & 1);
    else
        return (t + R1 * (i / R1)) + R2 * (i % R1);
}
template <int R1, int R2, typename T, bool PAIR> constexpr int row_stride()
{
    if constexpr (PAIR)
        return R2 * (R1 + 2);
    else
        return four_step_stride<R1, R2, T>();
}

template <int R1, int R2, int ROWS, typename T, bool PAIR, bool ZYX> constexpr int r2c_lds()
{
    constexpr int A = ROWS * row_stride<R1, R2, T, PAIR>(), B = R1 * R2 * ROWS;
    constexpr int Z = ZYX ? ROWS * (2 * R1 * R2 + 2) : 0;
    return A > B ? (A > Z ? A : Z) : (B > Z ? B : Z);
}

template <typename T, int R1, int R2, int ROWS, bool RES, bool PAIR = false, bool DIV = false,
          bool ZYX = false>
__global__ __launch_bounds__(ROWS *R1) void k_r2c_fast(const T *__restrict__ in,
                                                      cx_t<T> *__restrict__ spec,
                                                      double *__restrict__ rowsum, int ny,
                                                      int nrows, const cx_t<T> *__restrict__ tw4,
                                                      const cx_t<T> *__restrict__ tws,
                                                      const T *__restrict__ pres, int nz,
                                                      double idx2, double idy2,
                                                      const double *__restrict__ rc, int swz,
                                                      int korder, const T *__restrict__ wz,
                                                      double scale)
{
    using C = cx_t<T>;
    static_assert(!ZYX || (!RES && !DIV), "the z-fastest pass has no fused residual");
    constexpr int L = R1 * R2, NT = ROWS * R1, S = row_stride<R1, R2, T, PAIR>();
    __shared__ T lds[r2c_lds<R1, R2, ROWS, T, PAIR, ZYX>()];
    const int r = threadIdx.x / R1, t = threadIdx.x - r * R1;
    const long tile = tile_of(blockIdx.x, gridDim.x, swz);
    // ZYX: tile = (level chunk kc, row j), kc fastest
    const int nkc = ZYX ? (nz + ROWS - 1) / ROWS : 1;
    const int zj = ZYX ? (int)(tile / nkc) : 0, zk0 = ZYX ? (int)(tile % nkc) * ROWS : 0;
    const long g0 = korder ? (tile % nz) * (long)ny + (tile / nz) * ROWS : tile * ROWS;
    const long g = ZYX ? (long)(zk0 + r) * ny + zj : g0 + r;
    const bool ok = ZYX ? zk0 + r < nz : g < nrows;
    const C *src = reinterpret_cast<const C *>(in) + (ok && !ZYX ? g : 0) * (long)L;
    C v[R2], w[PAIR ? 1 : R2];
    double s = 0.0;
    if constexpr (ZYX) {
        // rows past the last level read level nz - 1: transformed, never stored
        constexpr int SW = 2 * L + 2;
        const long istride = (long)ny * nz;
        // thread: level kk of the chunk, points i = i0 + (NT / ROWS) it
        constexpr int IT = 2 * L * ROWS / NT;
        static_assert(NT % ROWS == 0 && (2 * L * ROWS) % NT == 0, "staging split");
        const int kk = threadIdx.x % ROWS, i0 = threadIdx.x / ROWS;
        const int kq = zk0 + kk < nz ? zk0 + kk : nz - 1;
        const T *col = in + (long)zj * nz + kq;
        T ld[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) ld[it] = col[(long)(i0 + (NT / ROWS) * it) * istride];
#pragma unroll
        for (int it = 0; it < IT; ++it) lds[kk * SW + i0 + (NT / ROWS) * it] = ld[it];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            const int n = t + R1 * q;
            v[q] = C{lds[r * SW + 2 * n], lds[r * SW + 2 * n + 1]};
            s += (double)v[q].x + (double)v[q].y;
        }
        __syncthreads(); // the staging is read before the transform reuses it
    } else if constexpr (DIV) {
        const long gg = ok ? g : 0;
        const int lev = (int)((unsigned)gg / (unsigned)ny), j = (int)(gg - (long)lev * ny);
        const double au = rc[3 * lev], ad = rc[3 * lev + 1];
        const C *V = reinterpret_cast<const C *>(pres);
        const C *W = reinterpret_cast<const C *>(wz);
        const C *vc_row = V + gg * L;
        const C *vn_row = V + ((long)lev * ny + (j + 1 == ny ? 0 : j + 1)) * L;
        const C *wc_row = W + gg * L;
        // the top level's upper face carries no flux: its row pointer is this
        // row and au is exactly zero (no branch around the load)
        const C *wu_row = wc_row + (lev + 1 < nz ? (long)ny * L : 0);
        C uc[R2];
#pragma unroll
        for (int q = 0; q < R2; ++q) uc[q] = nt_load<T>(&src[t + R1 * q]);
        const int lane = threadIdx.x & 63, base = lane - t;
        const int right = base + (t == R1 - 1 ? 0 : t + 1);
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            const int n = t + R1 * q;
            // u_{2n+2}: lane t+1 slot q, or for t = R1-1 lane 0 slot q+1 (mod R2)
            const T er_a = __shfl(uc[q].x, right, 64);
            const T er_b = __shfl(uc[(q + 1) % R2].x, right, 64);
            const T ue = t == R1 - 1 ? er_b : er_a;
            const C vc = vc_row[n], vn = vn_row[n], wc = wc_row[n], wu = wu_row[n];
            const double d0 = ((double)uc[q].y - (double)uc[q].x) * idx2 +
                              ((double)vn.x - (double)vc.x) * idy2 + au * (double)wu.x -
                              ad * (double)wc.x;
            const double d1 = ((double)ue - (double)uc[q].y) * idx2 +
                              ((double)vn.y - (double)vc.y) * idy2 + au * (double)wu.y -
                              ad * (double)wc.y;
            v[q] = C{(T)(scale * d0), (T)(scale * d1)};
            s += ok ? (double)v[q].x + (double)v[q].y : 0.0;
        }
    } else if constexpr (RES) {
        const long gg = ok ? g : 0;
        const int lev = (int)((unsigned)gg / (unsigned)ny), j = (int)(gg - (long)lev * ny);
        const double au = rc[3 * lev], ad = rc[3 * lev + 1], ac = rc[3 * lev + 2];
        const C *P = reinterpret_cast<const C *>(pres);
        const C *pc_row = P + gg * L;
        const C *pn_row = P + ((long)lev * ny + (j + 1 == ny ? 0 : j + 1)) * L;
        const C *ps_row = P + ((long)lev * ny + (j == 0 ? ny - 1 : j - 1)) * L;
        const bool has_up = lev + 1 < nz, has_dn = lev > 0;
        const C *pu_row = pc_row + (has_up ? (long)ny * L : 0);
        const C *pd_row = pc_row - (has_dn ? (long)ny * L : 0);
        C pc[R2];
#pragma unroll
        for (int q = 0; q < R2; ++q) pc[q] = pc_row[t + R1 * q];
        const int lane = threadIdx.x & 63, base = lane - t;
        const int left = base + (t == 0 ? R1 - 1 : t - 1);
        const int right = base + (t == R1 - 1 ? 0 : t + 1);
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            const int n = t + R1 * q;
            // x_{2n-1}: lane t-1 slot q, or for t = 0 lane R1-1 slot q-1 (mod R2)
            const T wl_a = __shfl(pc[q].y, left, 64);
            const T wl_b = __shfl(pc[(q + R2 - 1) % R2].y, left, 64);
            const T xw = t == 0 ? wl_b : wl_a;
            // x_{2n+2}: lane t+1 slot q, or for t = R1-1 lane 0 slot q+1 (mod R2)
            const T er_a = __shfl(pc[q].x, right, 64);
            const T er_b = __shfl(pc[(q + 1) % R2].x, right, 64);
            const T xe = t == R1 - 1 ? er_b : er_a;
            const C bv = nt_load<T>(&src[n]), pn = pn_row[n], psd = ps_row[n];
            // unconditional: at the top and bottom levels the row pointer is
            // this row and its coefficient (au or ad) is exactly zero, so no
            // branch (and no wait for the load inside it) is needed
            const C pu = pu_row[n];
            const C pd = pd_row[n];
            const double c0 = pc[q].x, c1 = pc[q].y;
            const double lap0 = ((double)c1 - 2.0 * c0 + (double)xw) * idx2 +
                                ((double)pn.x - 2.0 * c0 + (double)psd.x) * idy2 +
                                au * (double)pu.x + ad * (double)pd.x - ac * c0;
            const double lap1 = ((double)xe - 2.0 * c1 + c0) * idx2 +
                                ((double)pn.y - 2.0 * c1 + (double)psd.y) * idy2 +
                                au * (double)pu.y + ad * (double)pd.y - ac * c1;
            // (a row past the end reads row 0 and is transformed but never
            // stored; no select, so that the loads need no branch)
            v[q] = C{(T)((double)bv.x - lap0), (T)((double)bv.y - lap1)};
            s += ok ? (double)v[q].x + (double)v[q].y : 0.0;
        }
    } else {
        // a row past the end reads row 0: transformed, never stored
#pragma unroll
        for (int q = 0; q < R2; ++q) {
            v[q] = nt_load<T>(&src[t + R1 * q]);
            s += (double)v[q].x + (double)v[q].y;
        }
    }
#pragma unroll
    for (int o = R1 / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (ok && t == 0) rowsum[g] = s;

    if constexpr (PAIR)
        four_step_pair<R1, R2, -1>(v, t, lds + r * S, tw4);
    else
        four_step<R1, R2, -1>(v, w, t, lds + r * S, tw4);
    C *Z = PAIR ? v : w;

    // split: X_k = (Z_k + Zc)/2 + W_nx^k (Z_k - Zc)/(2i), Zc = conj Z_{L-k};
    // the real parts go straight to the [kx][row] staging in LDS, the
    // imaginary parts wait in registers for the second staging round.
    // Z_{L-k} of slot i sits in lane src_lane, slot R2 - 1 - i (PAIR: lane
    // R1 + 1 - t; the lanes of pair 0 take lane t ^ 1, slot R2 - i); for
    // t = 0 of the plain form in this lane's own registers.
    const int lane = threadIdx.x & 63;
    const int src_lane = PAIR ? lane - t + ((R1 + 1 - t) & (R1 - 1))
                              : lane - t + ((R1 - t) & (R1 - 1));
    T Xi[R2];
    T outr[R2], outi[R2];
    __syncthreads(); // the transform's last LDS reads are done
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        C zp;
        if constexpr (PAIR) {
            zp.x = __shfl(Z[R2 - 1 - i].x, src_lane, 64);
            zp.y = __shfl(Z[R2 - 1 - i].y, src_lane, 64);
            C zq;
            zq.x = __shfl_xor(Z[(R2 - i) & (R2 - 1)].x, 1, 64);
            zq.y = __shfl_xor(Z[(R2 - i) & (R2 - 1)].y, 1, 64);
            if (t < 2) zp = i == 0 ? Z[0] : zq;
        } else {
            constexpr int J = R2 / R1;
            const int j = i / R1, k1 = i % R1;
            const int other = (J - 1 - j) * R1 + (R1 - 1 - k1);
            const int own = j == 0 ? ((R1 - k1) & (R1 - 1)) : (J - j) * R1 + (R1 - 1 - k1);
            zp.x = __shfl(Z[other].x, src_lane, 64);
            zp.y = __shfl(Z[other].y, src_lane, 64);
            if (t == 0) zp = Z[own];
        }
        const C zk = Z[i];
        const int k = out_index<R1, R2, PAIR>(t, i);
        const C zc = cconj(zp);
        C X;
        if (k == 0) {
            X = C{zk.x + zk.y, zk.x - zk.y};
        } else {
            const C e = C{T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
            const C d = csub(zk, zc);
            const C o = C{T(0.5) * d.y, T(-0.5) * d.x};
            X = cadd(e, cmul(o, tws[k]));
        }
        lds[stage_idx<R1, ROWS>(k, r)] = X.x;
        Xi[i] = X.y;
    }

    // transposed store: [row][kx] -> spec[level][kx][j]
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int e = threadIdx.x + NT * i;
        outr[i] = lds[stage_idx<R1, ROWS>(e / ROWS, e % ROWS)];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R2; ++i) lds[stage_idx<R1, ROWS>(out_index<R1, R2, PAIR>(t, i), r)] = Xi[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int e = threadIdx.x + NT * i;
        outi[i] = lds[stage_idx<R1, ROWS>(e / ROWS, e % ROWS)];
    }
    // as in k_c2r_fast: this thread's row rr is the same for every i
    static_assert(NT % ROWS == 0, "rows per block must divide the block");
    if constexpr (ZYX) {
        const int kz = zk0 + threadIdx.x % ROWS;
        if (kz < nz) {
            C *dst = spec + (long)zj * nz + kz; // [kx][j][k]
            const long kstride = (long)ny * nz;
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int kx = threadIdx.x / ROWS + (NT / ROWS) * i;
                dst[(long)kx * kstride] = C{outr[i], outi[i]};
            }
        }
        return;
    }
    const long g2 = g0 + threadIdx.x % ROWS;
    if (g2 < nrows) {
        const long lev = (unsigned)g2 / (unsigned)ny, jj = g2 - lev * ny; // rows < 2^31
        C *dst = spec + lev * L * (long)ny + jj;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int kx = threadIdx.x / ROWS + (NT / ROWS) * i;
            dst[(long)kx * ny] = C{outr[i], outi[i]};
        }
    }
}

// ---------------------------------------------------------------- x backward
// Gathers ROWS rows of the transposed spectrum through LDS, undoes the
// packing, Z_k = (X_k + conj X_{L-k}) + i W_nx^{-k} (X_k - conj X_{L-k}),
// transforms backwards and stores real rows (optionally accumulated).
// ZYX (nz > 0): the rows are ROWS consecutive levels of one row j read from
// the [kx][j][k] layout (along k), and the result is staged in LDS and
// stored (or accumulated) along k into a z-fastest field ([nx][ny][nz]).
template <typename T, int R1, int R2, int ROWS, bool PAIR = false, bool ZYX = false>
__global__ __launch_bounds__(ROWS *R1) void k_c2r_fast(const cx_t<T> *__restrict__ spec,
                                                      T *__restrict__ out, int ny, int nrows,
                                                      int accumulate,
                                                      const cx_t<T> *__restrict__ tw4,
                                                      const cx_t<T> *__restrict__ tws, int swz,
                                                      int nz = 0)
{
    using C = cx_t<T>;
    constexpr int L = R1 * R2, NT = ROWS * R1, S = row_stride<R1, R2, T, PAIR>();
    __shared__ T lds[r2c_lds<R1, R2, ROWS, T, PAIR, ZYX>()];
    const int r = threadIdx.x / R1, t = threadIdx.x - r * R1;
    const long tile = tile_of(blockIdx.x, gridDim.x, swz);
    const int nkc = ZYX ? (nz + ROWS - 1) / ROWS : 1;
    const int zj = ZYX ? (int)(tile / nkc) : 0, zk0 = ZYX ? (int)(tile % nkc) * ROWS : 0;
    const long g = tile * ROWS + r;
    const bool ok = g < nrows;

    // Element i of this thread is (kx, rr) = (e / ROWS, e % ROWS) with
    // e = threadIdx.x + NT i; NT is a multiple of ROWS, so rr (and with it
    // the spectrum row's level and j) is the same for every i and is
    // computed once.  A row past the end reads row 0: it is transformed but
    // never stored.
    static_assert(NT % ROWS == 0, "rows per block must divide the block");
    T inr[R2], ini[R2];
    if constexpr (ZYX) {
        // levels past the last read level nz - 1: transformed, never stored
        const int kz = zk0 + threadIdx.x % ROWS;
        const C *src = spec + (long)zj * nz + (kz < nz ? kz : nz - 1);
        const long kstride = (long)ny * nz;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int kx = threadIdx.x / ROWS + (NT / ROWS) * i;
            const C x = nt_load<T>(&src[(long)kx * kstride]);
            inr[i] = x.x;
            ini[i] = x.y;
        }
    } else {
        const int rr = threadIdx.x % ROWS;
        const long g2 = tile * ROWS + rr < nrows ? tile * ROWS + rr : 0;
        const long lev = (unsigned)g2 / (unsigned)ny, jj = g2 - lev * ny; // rows < 2^31
        const C *src = spec + lev * L * (long)ny + jj;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int kx = threadIdx.x / ROWS + (NT / ROWS) * i;
            const C x = nt_load<T>(&src[(long)kx * ny]);
            inr[i] = x.x;
            ini[i] = x.y;
        }
    }
    C xa[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int e = threadIdx.x + NT * i;
        lds[stage_idx<R1, ROWS>(e / ROWS, e % ROWS)] = inr[i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R2; ++q) xa[q].x = lds[stage_idx<R1, ROWS>(t + R1 * q, r)];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int e = threadIdx.x + NT * i;
        lds[stage_idx<R1, ROWS>(e / ROWS, e % ROWS)] = ini[i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R2; ++q) xa[q].y = lds[stage_idx<R1, ROWS>(t + R1 * q, r)];
    // X_{L-k} for k = t + R1 q: lane R1 - t of the row, slot R2 - 1 - q (for
    // t = 0: this lane, slot (R2 - q) mod R2)
    const int lane = threadIdx.x & 63;
    const int src_lane = lane - t + ((R1 - t) & (R1 - 1));
    C v[R2], w[PAIR ? 1 : R2];
#pragma unroll
    for (int q = 0; q < R2; ++q) {
        const int k = t + R1 * q;
        C xb;
        xb.x = __shfl(xa[R2 - 1 - q].x, src_lane, 64);
        xb.y = __shfl(xa[R2 - 1 - q].y, src_lane, 64);
        if (t == 0) xb = xa[(R2 - q) % R2];
        if (k == 0) {
            const T x0 = xa[q].x, xl = xa[q].y;
            v[q] = C{x0 + xl, x0 - xl};
        } else {
            const C xc = cconj(xb);
            const C sm = cadd(xa[q], xc);
            const C dw = cmul(csub(xa[q], xc), cconj(tws[k]));
            v[q] = C{sm.x - dw.y, sm.y + dw.x};
        }
    }
    __syncthreads();
    if constexpr (PAIR)
        four_step_pair<R1, R2, 1>(v, t, lds + r * S, tw4);
    else
        four_step<R1, R2, 1>(v, w, t, lds + r * S, tw4);
    C *Z = PAIR ? v : w;
    if constexpr (ZYX) {
        constexpr int SW = 2 * L + 2;
        __syncthreads(); // the transform's last LDS reads are done
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int c = out_index<R1, R2, PAIR>(t, i);
            lds[r * SW + 2 * c] = Z[i].x;
            lds[r * SW + 2 * c + 1] = Z[i].y;
        }
        __syncthreads();
        const long istride = (long)ny * nz;
        constexpr int IT = 2 * L * ROWS / NT;
        const int kk = threadIdx.x % ROWS, i0 = threadIdx.x / ROWS;
        if (zk0 + kk < nz) {
            T *col = out + (long)zj * nz + zk0 + kk;
            if (accumulate) {
#pragma unroll 8
                for (int it = 0; it < IT; ++it) {
                    T *o = col + (long)(i0 + (NT / ROWS) * it) * istride;
                    *o += lds[kk * SW + i0 + (NT / ROWS) * it];
                }
            } else {
#pragma unroll 8
                for (int it = 0; it < IT; ++it)
                    col[(long)(i0 + (NT / ROWS) * it) * istride] =
                        lds[kk * SW + i0 + (NT / ROWS) * it];
            }
        }
        return;
    }
    if (ok) {
        C *dst = reinterpret_cast<C *>(out) + g * (long)L;
        if (accumulate) {
            // the old values are read GA at a time, so that their loads are
            // waited on once per group rather than once per store
            constexpr int GA = R2 < 8 ? R2 : 8;
#pragma unroll
            for (int i0 = 0; i0 < R2; i0 += GA) {
                C old[GA];
#pragma unroll
                for (int c = 0; c < GA; ++c)
                    old[c] = nt_load<T>(&dst[out_index<R1, R2, PAIR>(t, i0 + c)]);
#pragma unroll
                for (int c = 0; c < GA; ++c)
                    nt_store<T>(cadd(Z[i0 + c], old[c]), &dst[out_index<R1, R2, PAIR>(t, i0 + c)]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < R2; ++i) nt_store<T>(Z[i], &dst[out_index<R1, R2, PAIR>(t, i)]);
        }
    }
}

// ---------------------------------------------------------------- launchers
// Rows per block of the x passes: 128-byte runs of the transposed layout
// (16 FP32 or 8 FP64 complex values), halved until the LDS buffer fits 64 KiB;
// WIDE: 256-byte runs within 128 KiB.
template <typename T, int R1, int R2, bool WIDE, bool PAIR = false> constexpr int x_rows()
{
    int rows = (sizeof(T) == 8 ? 8 : 16) * (WIDE ? 2 : 1);
    while (rows > 1) {
        const int a = rows * row_stride<R1, R2, T, PAIR>(), b = R1 * R2 * rows;
        if ((a > b ? a : b) * (int)sizeof(T) <= (WIDE ? 131072 : 65536)) break;
        rows /= 2;
    }
    return rows;
}

// Returns hipErrorNotSupported when L has no register-resident kernel.
template <typename T, int R1, int R2>
static hipError_t y_fast(cx_t<T> *spec, int nrows, int dir, const cx_t<T> *tw4, int nkx, int kxlo,
                         int kxcnt, int swz, hipStream_t st, int keep)
{
    constexpr int NT = sizeof(T) == 8 && R1 * R2 >= 512 ? 128 : 256;
    constexpr int RB = NT / R1;
    if (nrows <= 0) return hipSuccess;
    const int grid = (nrows + RB - 1) / RB;
    if (dir < 0)
        hipLaunchKernelGGL((k_fft_y_fast<T, R1, R2, -1, NT>), dim3(grid), dim3(NT), 0, st, spec,
                           nrows, tw4, nkx, kxlo, kxcnt, swz, keep);
    else
        hipLaunchKernelGGL((k_fft_y_fast<T, R1, R2, 1, NT>), dim3(grid), dim3(NT), 0, st, spec,
                           nrows, tw4, nkx, kxlo, kxcnt, swz, keep);
    return hipGetLastError();
}

// Powers of two from 16 to 1024, and 3 2^k from 24 to 192 (an R2 of 12 or 24
// points: a prime-factor DFT in registers); in FP32 also 384 (R2 = 48, whose
// FP64 registers would not fit).
bool fast_length(int L, bool fp64)
{
    return L == 16 || L == 32 || L == 64 || L == 128 || L == 256 || L == 512 || L == 1024 ||
           L == 24 || L == 48 || L == 96 || L == 192 || (!fp64 && L == 384);
}
int fast_r1(int L)
{
    switch (L) {
    case 24: return 2;
    case 48: return 4;
    case 96: return 4;
    case 192: return 8;
    case 384: return 8;
    default: return L <= 32 ? 4 : L <= 128 ? 8 : L <= 512 ? 16 : 32;
    }
}
bool pair_length(int L) { return L == 32 || L == 128 || L == 512; }

#define PS_FAST_SWITCH(L, F)                                                                       \
    switch (L) {                                                                                   \
    case 16: return F(4, 4);                                                                       \
    case 32: return F(4, 8);                                                                       \
    case 64: return F(8, 8);                                                                       \
    case 128: return F(8, 16);                                                                     \
    case 256: return F(16, 16);                                                                    \
    case 512: return F(16, 32);                                                                    \
    case 1024: return F(32, 32);                                                                   \
    case 24: return F(2, 12);                                                                      \
    case 48: return F(4, 12);                                                                      \
    case 96: return F(4, 24);                                                                      \
    case 192: return F(8, 24);                                                                     \
    case 384:                                                                                      \
        if constexpr (sizeof(T) == 4) return F(8, 48);                                             \
        else return hipErrorNotSupported;                                                          \
    default: return hipErrorNotSupported;                                                          \
    }

// variant: 1 = plain block order, 2 = XCD-contiguous tiles.
template <typename T>
hipError_t launch_fft_y_fast(cx_t<T> *spec, int nz, int nkx, int kxlo, int kxcnt, int ny, int dir,
                             const cx_t<T> *tw4, hipStream_t st, int variant, int keep)
{
    const int nrows = nz * kxcnt;
    const int swz = variant >= 2;
#define PS_Y(a, b) y_fast<T, a, b>(spec, nrows, dir, tw4, nkx, kxlo, kxcnt, swz, st, keep)
    PS_FAST_SWITCH(ny, PS_Y)
#undef PS_Y
}

template <typename T, int R1, int R2, bool WIDE>
static hipError_t r2c_fast_rows(const T *in, cx_t<T> *spec, double *rowsum, int ny, int nz,
                                const cx_t<T> *tw4, const cx_t<T> *tws, const T *pres,
                                double idx2, double idy2, const double *rc, int swz,
                                hipStream_t st, const T *wz, double scale)
{
    constexpr int ROWS = x_rows<T, R1, R2, WIDE>();
    const int nrows = ny * nz;
    const int grid = (nrows + ROWS - 1) / ROWS;
    // the level-fastest tile order of the residual and divergence forms,
    // where tiles do not straddle levels
    const int korder = pres && swz && ny % ROWS == 0;
    if (wz)
        hipLaunchKernelGGL((k_r2c_fast<T, R1, R2, ROWS, false, false, true>), dim3(grid),
                           dim3(ROWS * R1), 0, st, in, spec, rowsum, ny, nrows, tw4, tws, pres, nz,
                           idx2, idy2, rc, swz, korder, wz, scale);
    else if (pres)
        hipLaunchKernelGGL((k_r2c_fast<T, R1, R2, ROWS, true>), dim3(grid), dim3(ROWS * R1), 0, st,
                           in, spec, rowsum, ny, nrows, tw4, tws, pres, nz, idx2, idy2, rc, swz,
                           korder, (const T *)nullptr, 1.0);
    else
        hipLaunchKernelGGL((k_r2c_fast<T, R1, R2, ROWS, false>), dim3(grid), dim3(ROWS * R1), 0,
                           st, in, spec, rowsum, ny, nrows, tw4, tws, pres, nz, idx2, idy2, rc,
                           swz, 0, (const T *)nullptr, 1.0);
    return hipGetLastError();
}

// The row transform with twice the lanes (four_step_pair) for L = 2 s^2,
// whose plain split is (s, 2 s).
template <typename T, int R1, int R2>
static hipError_t r2c_pair(const T *in, cx_t<T> *spec, double *rowsum, int ny, int nz,
                           const cx_t<T> *tw4, const cx_t<T> *tws, const T *pres, double idx2,
                           double idy2, const double *rc, hipStream_t st, const T *wz,
                           double scale)
{
    constexpr int ROWS = x_rows<T, R2, R1, false, true>();
    const int nrows = ny * nz;
    const int grid = (nrows + ROWS - 1) / ROWS;
    const int korder = pres && ny % ROWS == 0;
    if (wz)
        hipLaunchKernelGGL((k_r2c_fast<T, R2, R1, ROWS, false, true, true>), dim3(grid),
                           dim3(ROWS * R2), 0, st, in, spec, rowsum, ny, nrows, tw4, tws, pres, nz,
                           idx2, idy2, rc, 1, korder, wz, scale);
    else if (pres)
        hipLaunchKernelGGL((k_r2c_fast<T, R2, R1, ROWS, true, true>), dim3(grid), dim3(ROWS * R2), 0,
                           st, in, spec, rowsum, ny, nrows, tw4, tws, pres, nz, idx2, idy2, rc, 1,
                           korder, (const T *)nullptr, 1.0);
    else
        hipLaunchKernelGGL((k_r2c_fast<T, R2, R1, ROWS, false, true>), dim3(grid), dim3(ROWS * R2),
                           0, st, in, spec, rowsum, ny, nrows, tw4, tws, pres, nz, idx2, idy2, rc,
                           1, 0, (const T *)nullptr, 1.0);
    return hipGetLastError();
}

// variant: 1 = plain block order, 2 = XCD-contiguous tiles, 3 = as 2 with
// twice the rows per block (256-byte runs of the transposed layout), 4 = as 2
// with the paired row transform where L = 2 s^2 (else as 2).
template <typename T, int R1, int R2>
static hipError_t r2c_fast(const T *in, cx_t<T> *spec, double *rowsum, int ny, int nz,
                           const cx_t<T> *tw4, const cx_t<T> *tws, const T *pres, double idx2,
                           double idy2, const double *rc, int variant, hipStream_t st,
                           const T *wz, double scale)
{
    if constexpr (R2 == 2 * R1)
        if (variant == 4)
            return r2c_pair<T, R1, R2>(in, spec, rowsum, ny, nz, tw4, tws, pres, idx2, idy2, rc,
                                       st, wz, scale);
    if (variant == 3)
        return r2c_fast_rows<T, R1, R2, true>(in, spec, rowsum, ny, nz, tw4, tws, pres, idx2,
                                              idy2, rc, 1, st, wz, scale);
    return r2c_fast_rows<T, R1, R2, false>(in, spec, rowsum, ny, nz, tw4, tws, pres, idx2, idy2,
                                           rc, variant >= 2, st, wz, scale);
}

template <typename T>
hipError_t launch_r2c_fast(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                           const cx_t<T> *tw4, const cx_t<T> *tws, hipStream_t st,
                           const T *pres, double idx2, double idy2, const double *rc, int variant,
                           const T *wz, double scale)
{
#define PS_X(a, b)                                                                                 \
    r2c_fast<T, a, b>(in, spec, rowsum, ny, nz, tw4, tws, pres, idx2, idy2, rc, variant, st, wz,   \
                      scale)
    PS_FAST_SWITCH(nx / 2, PS_X)
#undef PS_X
}

template <typename T, int R1, int R2, bool WIDE>
static hipError_t c2r_fast_rows(const cx_t<T> *spec, T *out, int ny, int nrows, int accumulate,
                                const cx_t<T> *tw4, const cx_t<T> *tws, int swz, hipStream_t st)
{
    constexpr int ROWS = x_rows<T, R1, R2, WIDE>();
    const int grid = (nrows + ROWS - 1) / ROWS;
    hipLaunchKernelGGL((k_c2r_fast<T, R1, R2, ROWS>), dim3(grid), dim3(ROWS * R1), 0, st, spec, out,
                       ny, nrows, accumulate, tw4, tws, swz);
    return hipGetLastError();
}

template <typename T, int R1, int R2>
static hipError_t c2r_fast(const cx_t<T> *spec, T *out, int ny, int nrows, int accumulate,
                           const cx_t<T> *tw4, const cx_t<T> *tws, int variant, hipStream_t st)
{
    if constexpr (R2 == 2 * R1) {
        if (variant == 4) {
            constexpr int ROWS = x_rows<T, R2, R1, false, true>();
            const int grid = (nrows + ROWS - 1) / ROWS;
            hipLaunchKernelGGL((k_c2r_fast<T, R2, R1, ROWS, true>), dim3(grid), dim3(ROWS * R2), 0,
                               st, spec, out, ny, nrows, accumulate, tw4, tws, 1);
            return hipGetLastError();
        }
    }
    if (variant == 3)
        return c2r_fast_rows<T, R1, R2, true>(spec, out, ny, nrows, accumulate, tw4, tws, 1, st);
    return c2r_fast_rows<T, R1, R2, false>(spec, out, ny, nrows, accumulate, tw4, tws,
                                           variant >= 2, st);
}

template <typename T>
hipError_t launch_c2r_fast(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int accumulate,
                           const cx_t<T> *tw4, const cx_t<T> *tws, hipStream_t st, int variant)
{
    const int nrows = ny * nz;
#define PS_X(a, b) c2r_fast<T, a, b>(spec, out, ny, nrows, accumulate, tw4, tws, variant, st)
    PS_FAST_SWITCH(nx / 2, PS_X)
#undef PS_X
}

// The z-fastest solve's passes (fast lengths only).
template <typename T, int R1, int R2>
static hipError_t y_zyx(const cx_t<T> *src, cx_t<T> *dst, int nz, int nkx, int dir,
                        const cx_t<T> *tw4, hipStream_t st)
{
    constexpr int NT = sizeof(T) == 8 && R1 * R2 >= 512 ? 128 : 256;
    constexpr int RB = NT / R1;
    const int grid = nkx * ((nz + RB - 1) / RB);
    if (dir < 0)
        hipLaunchKernelGGL((k_fft_y_zyx<T, R1, R2, -1, NT>), dim3(grid), dim3(NT), 0, st, src, dst,
                           nz, nkx, tw4);
    else
        hipLaunchKernelGGL((k_fft_y_zyx<T, R1, R2, 1, NT>), dim3(grid), dim3(NT), 0, st, src, dst,
                           nz, nkx, tw4);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_zyx(const cx_t<T> *src, cx_t<T> *dst, int nz, int nkx, int ny, int dir,
                            const cx_t<T> *tw4, hipStream_t st)
{
#define PS_Y(a, b) y_zyx<T, a, b>(src, dst, nz, nkx, dir, tw4, st)
    PS_FAST_SWITCH(ny, PS_Y)
#undef PS_Y
}

template <typename T, int R1, int R2, bool WIDE>
static hipError_t x_zyx(const T *in, cx_t<T> *tmp, double *rowsum, const cx_t<T> *tmp_in,
                        T *out, int ny, int nz, const cx_t<T> *tw4, const cx_t<T> *tws,
                        int pair, int accumulate, hipStream_t st)
{
    if constexpr (R2 == 2 * R1) {
        if (pair) {
            constexpr int ROWS = x_rows<T, R2, R1, WIDE, true>();
            const int grid = ny * ((nz + ROWS - 1) / ROWS);
            if (in)
                hipLaunchKernelGGL((k_r2c_fast<T, R2, R1, ROWS, false, true, false, true>),
                                   dim3(grid), dim3(ROWS * R2), 0, st, in, tmp, rowsum, ny,
                                   ny * nz, tw4, tws, (const T *)nullptr, nz, 0.0, 0.0,
                                   (const double *)nullptr, 1, 0, (const T *)nullptr, 1.0);
            else
                hipLaunchKernelGGL((k_c2r_fast<T, R2, R1, ROWS, true, true>), dim3(grid),
                                   dim3(ROWS * R2), 0, st, tmp_in, out, ny, ny * nz, accumulate,
                                   tw4, tws, 1, nz);
            return hipGetLastError();
        }
    }
    constexpr int ROWS = x_rows<T, R1, R2, WIDE>();
    const int grid = ny * ((nz + ROWS - 1) / ROWS);
    if (in)
        hipLaunchKernelGGL((k_r2c_fast<T, R1, R2, ROWS, false, false, false, true>), dim3(grid),
                           dim3(ROWS * R1), 0, st, in, tmp, rowsum, ny, ny * nz, tw4, tws,
                           (const T *)nullptr, nz, 0.0, 0.0, (const double *)nullptr, 1, 0,
                           (const T *)nullptr, 1.0);
    else
        hipLaunchKernelGGL((k_c2r_fast<T, R1, R2, ROWS, false, true>), dim3(grid),
                           dim3(ROWS * R1), 0, st, tmp_in, out, ny, ny * nz, accumulate, tw4, tws,
                           1, nz);
    return hipGetLastError();
}

// Forward (in != NULL: z-fastest field -> [kx][j][k], row sums) or backward
// (in == NULL: [kx][j][k] -> z-fastest field, added to it when accumulate)
// x pass; pair selects the paired row transform where nx/2 = 2 s^2; wide:
// twice the levels per block (256-byte runs along k in FP32, within 128 KiB
// of LDS).
template <typename T>
hipError_t launch_x_zyx_fast(const T *in, cx_t<T> *tmp, double *rowsum, const cx_t<T> *tmp_in,
                             T *out, int nx, int ny, int nz, const cx_t<T> *tw4,
                             const cx_t<T> *tws, int pair, int wide, int accumulate,
                             hipStream_t st)
{
#define PS_X(a, b)                                                                                 \
    (wide ? x_zyx<T, a, b, true>(in, tmp, rowsum, tmp_in, out, ny, nz, tw4, tws, pair, accumulate, \
                                 st)                                                              \
          : x_zyx<T, a, b, false>(in, tmp, rowsum, tmp_in, out, ny, nz, tw4, tws, pair,           \
                                  accumulate, st))
    PS_FAST_SWITCH(nx / 2, PS_X)
#undef PS_X
}

#define PS_INST(T)                                                                                 \
    template hipError_t launch_fft_y_zyx<T>(const cx_t<T> *, cx_t<T> *, int, int, int, int,      \
                                            const cx_t<T> *, hipStream_t);                        \
    template hipError_t launch_x_zyx_fast<T>(const T *, cx_t<T> *, double *, const cx_t<T> *,    \
                                             T *, int, int, int, const cx_t<T> *,                 \
                                             const cx_t<T> *, int, int, int, hipStream_t);        \
    template hipError_t launch_fft_y_fast<T>(cx_t<T> *, int, int, int, int, int, int,            \
                                             const cx_t<T> *, hipStream_t, int, int);             \
    template hipError_t launch_r2c_fast<T>(const T *, cx_t<T> *, double *, int, int, int,        \
                                           const cx_t<T> *, const cx_t<T> *, hipStream_t,         \
                                           const T *, double, double, const double *, int,        \
                                           const T *, double);                                    \
    template hipError_t launch_c2r_fast<T>(const cx_t<T> *, T *, int, int, int, int,             \
                                           const cx_t<T> *, const cx_t<T> *, hipStream_t, int);
PS_INST(float)
PS_INST(double)
#undef PS_INST

} // namespace ps
