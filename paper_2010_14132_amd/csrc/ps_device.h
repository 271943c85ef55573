// Device helpers for the gfx950 pressure-solve kernels: complex arithmetic,
// small in-register DFTs, and one radix pass of a Stockham (self-sorting)
// FFT over rows held in LDS.
#pragma once
#include <hip/hip_runtime.h>

namespace ps {

// Block -> tile map.  Blocks are handed to the eight XCDs in turn (block b
// to XCD b mod 8), each with its own L2; with swz set, XCD x takes one
// contiguous range of tiles instead of every eighth one, so neighbouring
// tiles (adjacent rows, adjacent 128-byte runs of the transposed layout,
// adjacent column groups) meet in the same L2.  A bijection of [0, nb) for
// any nb.
__device__ __forceinline__ int tile_of(int b, int nb, int swz)
{
    if (!swz) return b;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <typename T> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };
template <typename T> using cx_t = typename cx<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * (conj(b) if DIR > 0 else b): twiddle tables hold the forward roots.
template <int DIR, typename C> __device__ __forceinline__ C ctw(C a, C b)
{
    if (DIR > 0) b.y = -b.y;
    return cmul(a, b);
}
// a * (DIR * i)
template <int DIR, typename C> __device__ __forceinline__ C cmul_i(C a)
{
    return DIR < 0 ? C{a.y, -a.x} : C{-a.y, a.x};
}
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { return C{a.x * s, a.y * s}; }

// cos and sin of 2 pi m / 16, m = 1..3 (exact mathematical constants).
#define PS_C16_1 0.92387953251128675613
#define PS_S16_1 0.38268343236508977173
#define PS_R2_2 0.70710678118654752440
#define PS_S3_2 0.86602540378443864676

// ---- small DFTs, X_k = sum_n v_n exp(DIR 2 pi i n k / R), in place --------
template <int DIR, typename C> __device__ __forceinline__ void dft2(C &a, C &b)
{
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C *v)
{
    using T = decltype(v[0].x);
    C s = cadd(v[1], v[2]);
    C d = csub(v[1], v[2]);
    C t = C{v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    C u = cscale(cmul_i<DIR>(d), T(PS_S3_2));
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C *v)
{
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
}

// Radix-2 split of an 8-point DFT: even and odd 4-point DFTs, then
// X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k.
template <int DIR, typename C> __device__ __forceinline__ void dft8(C *v)
{
    using T = decltype(v[0].x);
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    const T r = T(PS_R2_2);
    C w1 = C{r, DIR * r}, w3 = C{-r, DIR * r};
    C o1 = cmul(o[1], w1), o2 = cmul_i<DIR>(o[2]), o3 = cmul(o[3], w3);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft16(C *v)
{
    using T = decltype(v[0].x);
    C e[8], o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        e[q] = v[2 * q];
        o[q] = v[2 * q + 1];
    }
    dft8<DIR>(e);
    dft8<DIR>(o);
    const T c1 = T(PS_C16_1), s1 = T(PS_S16_1), r2 = T(PS_R2_2);
    const C w[8] = {C{T(1), T(0)}, C{c1, DIR * s1}, C{r2, DIR * r2}, C{s1, DIR * c1},
                    C{T(0), T(DIR)}, C{-s1, DIR * c1}, C{-r2, DIR * r2}, C{-c1, DIR * s1}};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        C t = q == 0 ? o[0] : cmul(o[q], w[q]);
        v[q] = cadd(e[q], t);
        v[q + 8] = csub(e[q], t);
    }
}

// cos and sin of pi m / 16, m = 1..3.
#define PS_C32_1 0.98078528040323044913
#define PS_S32_1 0.19509032201612826785
#define PS_C32_3 0.83146961230254523708
#define PS_S32_3 0.55557023301960222474

template <int DIR, typename C> __device__ __forceinline__ void dft32(C *v)
{
    using T = decltype(v[0].x);
    C e[16], o[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        e[q] = v[2 * q];
        o[q] = v[2 * q + 1];
    }
    dft16<DIR>(e);
    dft16<DIR>(o);
    const T c1 = T(PS_C32_1), s1 = T(PS_S32_1), c2 = T(PS_C16_1), s2 = T(PS_S16_1);
    const T c3 = T(PS_C32_3), s3 = T(PS_S32_3), r = T(PS_R2_2);
    // W32^q = cos(pi q/16) + DIR i sin(pi q/16), q = 0..15
    const T wc[16] = {T(1), c1, c2, c3, r, s3, s2, s1, T(0), -s1, -s2, -s3, -r, -c3, -c2, -c1};
    const T ws[16] = {T(0), s1, s2, s3, r, c3, c2, c1, T(1), c1, c2, c3, r, s3, s2, s1};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        C t = q == 0 ? o[0] : cmul(o[q], C{wc[q], DIR * ws[q]});
        v[q] = cadd(e[q], t);
        v[q + 16] = csub(e[q], t);
    }
}

// a^{-1} mod m (a and m coprime, m >= 2).
constexpr int inv_mod(int a, int m)
{
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C *v);

// Prime-factor (Good-Thomas) DFT of N = 3 M points, M a power of two (so 3
// and M are coprime): element n1 M + 3 n2 (mod N) of the input is entry
// (n1, n2) of a 3 x M array, M-point DFTs run over n2, then 3-point DFTs over
// n1, with no twiddle factors between them, and entry (k1, k2) is output
// element M U k1 + 3 W k2 (mod N), U = M^{-1} mod 3, W = 3^{-1} mod M (the
// Chinese-remainder map).  In place; the index maps are compile-time.
template <int M, int DIR, typename C> __device__ __forceinline__ void dft_pfa3(C *v)
{
    constexpr int N = 3 * M, U = inv_mod(M % 3, 3), W = inv_mod(3 % M, M);
    C a[3][M];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1)
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) a[n1][n2] = v[(M * n1 + 3 * n2) % N];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) dft<M, DIR>(a[n1]);
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
        C b[3] = {a[0][k2], a[1][k2], a[2][k2]};
        dft3<DIR>(b);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) v[(M * U * k1 + 3 * W * k2) % N] = b[k1];
    }
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C *v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (R == 3) dft3<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 8) dft8<DIR>(v);
    else if constexpr (R == 16) dft16<DIR>(v);
    else if constexpr (R == 32) dft32<DIR>(v);
    else if constexpr (R == 6) dft_pfa3<2, DIR>(v);
    else if constexpr (R == 12) dft_pfa3<4, DIR>(v);
    else if constexpr (R == 24) dft_pfa3<8, DIR>(v);
    else if constexpr (R == 48) dft_pfa3<16, DIR>(v);
    else static_assert(R == 0, "no in-register DFT of this length");
}

// ---- four-step row transform in registers ----------------------------------
// A row of length L = R1 R2 (R1 divides R2) is held by R1 lanes of one
// wavefront (lane t in [0, R1)).  On entry v[q] = x[t + R1 q].  Step A: an
// R2-point DFT over q, then the twiddle W_L^{t k2}; the [t][k2] -> [k2][t]
// exchange goes through LDS one real component at a time (row stride R1 + 1
// words, so the transposed reads do not conflict); step B: R1-point DFTs.
// On exit w[j R1 + k1] = X[(t + R1 j) + R2 k1], j in [0, R2/R1).
// tw4[k2 R1 + t] = W_L^{t k2} (forward roots; conjugated for DIR > 0).
// lds is this row's scratch of R2 (R1 + 1) values; every thread of the block
// must call this together (it synchronises the block).  Consecutive rows'
// scratch areas are four_step_stride() values apart: the padding puts the
// rows that share a wavefront on disjoint LDS banks (32 banks of 4 bytes:
// a row stride congruent to R1 words modulo the bank count), so both the
// column writes and the row reads run at the conflict-free rate.
template <int R1, int R2, typename T> constexpr int four_step_stride()
{
    constexpr int base = R2 * (R1 + 1);
    return sizeof(T) == 8 ? base + (((R1 / 2 - base) % 16) + 16) % 16
                          : base + (((R1 - base) % 32) + 32) % 32;
}

template <int R1, int R2, int DIR, typename C, typename T>
__device__ __forceinline__ void four_step(C (&v)[R2], C (&w)[R2], int t, T *lds,
                                          const C *__restrict__ tw4)
{
    constexpr int P = R1 + 1;
    dft<R2, DIR>(v);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) v[k2] = ctw<DIR>(v[k2], tw4[k2 * R1 + t]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) lds[k2 * P + t] = v[k2].x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) w[j * R1 + n1].x = lds[(t + R1 * j) * P + n1];
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) lds[k2 * P + t] = v[k2].y;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R2 / R1; ++j)
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) w[j * R1 + n1].y = lds[(t + R1 * j) * P + n1];
#pragma unroll
    for (int j = 0; j < R2 / R1; ++j) dft<R1, DIR>(&w[j * R1]);
}

// The same transform of a row of L = R1 R2 points with R1 = 2 R2: twice the
// lanes, half the values per lane.  Lane t holds v[q] = x[t + R1 q] (q < R2)
// on entry.  Stage 1 is the length-R2 DFT over q and the twiddle W_L^{t k2};
// after the transposition through LDS the lane pair (2m, 2m + 1) holds
// Y[2u][m] and Y[2u + 1][m] (u < R2) and each lane transforms its half over
// u; a radix-2 butterfly between the two lanes (W_L^{kk R2} on the odd half)
// finishes the length-R1 DFTs.  On exit lane t = 2m + h holds
// v[kk] = X[m + R2 kk + R2^2 h].  Works in place (the real and imaginary
// parts go through LDS one after the other).  tw4 is the table of the
// (R2, R1) split, entry W_L^{a b} at b R2 + a for a < R2, b < R1.  lds is this
// row's scratch of R2 (R1 + 2) values (the +2 spreads the pair reads over
// the banks); every thread of the block calls this together.
template <int R1, int R2, int DIR, typename C, typename T>
__device__ __forceinline__ void four_step_pair(C (&v)[R2], int t, T *lds,
                                               const C *__restrict__ tw4)
{
    static_assert(R1 == 2 * R2, "paired four-step: R1 = 2 R2");
    constexpr int P = R1 + 2;
    const int m = t >> 1, h = t & 1;
    dft<R2, DIR>(v);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) v[k2] = ctw<DIR>(v[k2], tw4[t * R2 + k2]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) lds[k2 * P + t] = v[k2].x;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R2; ++u) v[u].x = lds[m * P + 2 * u + h];
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) lds[k2 * P + t] = v[k2].y;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R2; ++u) v[u].y = lds[m * P + 2 * u + h];
    dft<R2, DIR>(v);
#pragma unroll
    for (int kk = 0; kk < R2; ++kk) {
        C o;
        o.x = __shfl_xor(v[kk].x, 1, 64);
        o.y = __shfl_xor(v[kk].y, 1, 64);
        const C e = h ? o : v[kk];
        C od = h ? v[kk] : o;
        if (kk) od = ctw<DIR>(od, tw4[R2 * R2 + kk]);
        v[kk] = h ? csub(e, od) : cadd(e, od);
    }
}

// ---- Stockham radix pass ---------------------------------------------------
// Factorisation of a transform length L = r_0 r_1 ... ; ns[s] = r_0...r_{s-1}.
struct StagePlan {
    int n;        // number of passes
    int r[16];
    int ns[16];
};

// Butterfly j (0 <= j < L/R) of a pass with stride product Ns: reads the R
// inputs j + q L/R, twiddles input q by W_{Ns R}^{q (j mod Ns)}, applies the
// R-point DFT and writes output q to (j - j mod Ns) R + j mod Ns + q Ns.
// After all passes the row is in natural order.  tw holds the forward roots
// W_L^m = exp(-2 pi i m / L), m in [0, L).
template <int R, int DIR, typename C>
__device__ __forceinline__ void stockham_bfly(const C *src, C *dst, int j, int L, int Ns, const C *tw)
{
    const int nb = L / R;
    const int kk = j % Ns;
    C v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[j + q * nb];
    if (Ns > 1) {
        const int m = kk * (L / (Ns * R));
#pragma unroll
        for (int q = 1; q < R; ++q) v[q] = ctw<DIR>(v[q], tw[q * m]);
    }
    dft<R, DIR>(v);
    const int base = (j - kk) * R + kk;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[base + q * Ns] = v[q];
}

// All passes over nrows rows of length L stored contiguously in LDS at a;
// b is a second LDS buffer of the same size.  Returns the buffer holding the
// result.  Every thread of the block must call it.
template <int DIR, typename C>
__device__ C *stockham_rows(C *a, C *b, int nrows, int L, const StagePlan &sp, const C *tw)
{
    for (int s = 0; s < sp.n; ++s) {
        const int R = sp.r[s], Ns = sp.ns[s];
        const int nb = L / R;
        const int total = nrows * nb;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int row = t / nb;
            const int j = t - row * nb;
            const C *src = a + row * L;
            C *dst = b + row * L;
            switch (R) {
            case 2: stockham_bfly<2, DIR>(src, dst, j, L, Ns, tw); break;
            case 3: stockham_bfly<3, DIR>(src, dst, j, L, Ns, tw); break;
            case 4: stockham_bfly<4, DIR>(src, dst, j, L, Ns, tw); break;
            case 8: stockham_bfly<8, DIR>(src, dst, j, L, Ns, tw); break;
            default: stockham_bfly<16, DIR>(src, dst, j, L, Ns, tw); break;
            }
        }
        __syncthreads();
        C *t = a;
        a = b;
        b = t;
    }
    return a;
}

// Sum over the 64 lanes of a wavefront, fixed butterfly order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

} // namespace ps
