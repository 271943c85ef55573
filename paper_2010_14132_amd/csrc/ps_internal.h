// Internal host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <type_traits>
#include <string>
#include <vector>

#include "ps_device.h"

namespace ps {

// Flags of the events that order work between streams of one device (the
// side stream of the FP64 columns, the lanes of a batch).  Their consumers
// are kernels on the same device, so the default system-scope fence on
// record and wait (cache write-back and invalidation for the host and other
// devices) is left out; the device-scope release and acquire that order
// kernels remain.
constexpr unsigned kStreamEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;

// One slot of the uniform-half column kernel's coefficient table (see
// k_columns3): coupling to the previous and next row of the elimination,
// D_k, right-hand-side and output factors, whether the slot is a real level
// (0 for a dummy slot, whose value is read but never written) and the
// level's byte offset in the spectrum (a dummy slot reads the middle row).
template <typename T> struct LevelCoef {
    T fp, fn, D, rs, os;
    int real;
    long long off;
};

// Device tables of one precision T.
template <typename T> struct Tables {
    T *ax = nullptr;      // [L+1]  4 sin^2(pi kx/nx)/dx^2
    T *ay = nullptr;      // [ny]   4 sin^2(pi ky/ny)/dy^2
    T *f = nullptr;       // [nz+1] f[0]=f[nz]=0, f[k]=f_{k-1/2}
    T *D = nullptr;       // [nz]   rho_k dz_k
    T *rs_fwd = nullptr;  // [nz]   right-hand-side factor -D_k/(nx ny)
    T *rs_adj = nullptr;  // [nz]   -1/(nx ny)
    T *os_adj = nullptr;  // [nz]   D_k
    cx_t<T> *tw_x = nullptr;  // [L]   W_L^m
    cx_t<T> *tw_s = nullptr;  // [L]   W_nx^k (real-to-complex split)
    cx_t<T> *tw_y = nullptr;  // [ny]  W_ny^m
    cx_t<T> *tw4_x = nullptr; // [L]   four-step twiddles W_L^{t k2} at [k2 R1 + t]
    cx_t<T> *tw4_y = nullptr; // [ny]  same for the y length
    // per-slot coefficients in elimination order for the uniform-half column
    // kernel (forward and adjoint): [2 NH + 1] entries of LevelCoef<T>, NH =
    // column_capacity(nz)
    void *coef_fwd = nullptr;
    void *coef_adj = nullptr;
};

// Launch geometry of the transform kernels chosen at planning time.
struct FftGeom {
    int rows_x = 1;   // rows per block of the x passes
    int rows_y = 1;   // rows per block of the y passes
    int variant_x = 0;   // forward x pass
    int variant_xi = 0;  // backward x pass
    int variant_y = 0;
    int special_side = 1; // FP64 columns: 0 on the plan's stream before the main kernel;
                          // 1 on the side stream, which also transforms their rows
                          // (kx < kmask) in y; 2 on the side stream after the whole
                          // y pass
    int columns = 2;     // column-solve kernel variant (see launch_columns_impl)
    int chunks = 1;      // y forward / columns / y backward run in this many kx chunks
    int special_variant = 1; // FP64 columns: 0 one lane per task via the HBM workspace,
                             // 1 staged in LDS (k_special_lds)
    int zyx_kc = 64;     // z-fastest (MONC) x passes: levels per tile (capped by the tile
                         // rows); with the register-resident passes, >= 32 selects blocks
                         // of twice the standard levels (32 FP32, 16 FP64)
    int xy_chunks = 1;   // level ranges in which the forward x and y passes, and the
                         // backward y and x passes, run pairwise (register-resident
                         // passes)
};

struct Launch {
    hipStream_t stream;
};

// Enqueue functions (defined in fft.hip / spectral.hip).
template <typename T>
hipError_t launch_fwd_x(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                        const FftGeom &g, const StagePlan &spx, const Tables<T> &tb, hipStream_t st);
template <typename T>
hipError_t launch_fwd_x_residual(const T *b, const T *p, cx_t<T> *spec, double *rowsum, int nx,
                                 int ny, int nz, double idx2, double idy2, const double *f,
                                 const double *D, int adjoint, const FftGeom &g,
                                 const StagePlan &spx, const Tables<T> &tb, hipStream_t st);
// y transforms of the spectrum rows (level, kx), kx in [kxlo, kxlo + kxcnt),
// L rows per level.
template <typename T>
hipError_t launch_fft_y(cx_t<T> *spec, int nz, int L, int kxlo, int kxcnt, int ny, int dir,
                        const FftGeom &g, const StagePlan &spy, const Tables<T> &tb,
                        hipStream_t st);
template <typename T>
hipError_t launch_inv_x(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int accumulate,
                        const FftGeom &g, const StagePlan &spx, const Tables<T> &tb,
                        hipStream_t st);

bool fast_length(int L, bool fp64); // a register-resident transform of this length exists
bool pair_length(int L); // L = 2 s^2 among the fast lengths (32, 128, 512)
int fast_r1(int L); // lanes per row of the register-resident kernels
// variant (the plan's variant_x / variant_y >= 1): 1 = plain block order,
// 2 = XCD-contiguous tiles, 3 (x passes only) = as 2 with twice the rows per
// block, 4 (x passes only) = as 2 with the paired row transform when
// nx/2 = 2 s^2 (else as 2).
// keep: the forward pass stores with the normal cache policy (its rows are
// read again soon, in a chunked pipeline) instead of non-temporally.
template <typename T>
hipError_t launch_fft_y_fast(cx_t<T> *spec, int nz, int L, int kxlo, int kxcnt, int ny, int dir,
                             const cx_t<T> *tw4, hipStream_t st, int variant, int keep = 0);
// pres != nullptr: transform the residual in - A pres (or in - A^T pres),
// with the per-level vertical coefficients rc (see k_r2c_fast).  wz !=
// nullptr: transform scale times the divergence of (in, pres, wz) = (u, v, w)
// with idx2 = 1/dx, idy2 = 1/dy and the divergence coefficients rc.
template <typename T>
hipError_t launch_r2c_fast(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                           const cx_t<T> *tw4, const cx_t<T> *tws, hipStream_t st,
                           const T *pres, double idx2, double idy2, const double *rc,
                           int variant, const T *wz = nullptr, double scale = 1.0);
// Generic (any length) forward x pass of scale times the divergence, and the
// pressure-gradient correction u -= dt Gx p, v -= dt Gy p, w -= dt Gz p
// (dyncore.hip).  dc: per level k, rho_{k+1/2}/D_k, rho_{k-1/2}/D_k and
// 1/h_{k-1/2} (three values each, zero where a face is a boundary).
// pres != nullptr: the residual scale * div - A pres instead (forward
// vertical coefficients rc, the plan's residual table).
template <typename T>
hipError_t launch_fwd_x_div(const T *u, const T *v, const T *w, double scale, cx_t<T> *spec,
                            double *rowsum, int nx, int ny, int nz, double dx, double dy,
                            const double *dc, const FftGeom &g, const StagePlan &spx,
                            const Tables<T> &tb, hipStream_t st, const T *pres = nullptr,
                            const double *rc = nullptr);
template <typename T>
hipError_t launch_grad_correct(T *u, T *v, T *w, const T *p, double dt, int nx, int ny, int nz,
                               double dx, double dy, const double *dc, hipStream_t st);
template <typename T>
hipError_t launch_c2r_fast(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int accumulate,
                           const cx_t<T> *tw4, const cx_t<T> *tws, hipStream_t st, int variant);

hipError_t launch_level_sums(const double *rowsum, double *S, int ny, int nz, hipStream_t st);

// x passes for fields in the z-fastest layout (i ny + j) nz + k (monc.hip):
// tiles of `rows` rows, kc_pref levels each (capped by rows and nz).
template <typename T>
hipError_t launch_fwd_x_zyx(const T *in, cx_t<T> *spec, double *rowsum, int nx, int ny, int nz,
                            int rows, int kc_pref, const StagePlan &spx, const Tables<T> &tb,
                            hipStream_t st);
template <typename T>
hipError_t launch_inv_x_zyx(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int rows,
                            int kc_pref, const StagePlan &spx, const Tables<T> &tb,
                            hipStream_t st, int accumulate = 0);
// r = b - A p for z-fastest fields (the refinement's residual; FP64
// accumulation, rounded once), rc: 3 vertical coefficients per level as for
// the level-major residual transform.
template <typename T>
hipError_t launch_residual_zyx(const T *b, const T *p, T *r, int nx, int ny, int nz, double idx2,
                               double idy2, const double *rc, hipStream_t st);

// The z-fastest solve's passes for fast lengths (fft_fast.hip), through
// the [kx][j][k] layout (k fastest, tmp): forward x (in != NULL: field ->
// tmp, row sums) or backward x (in == NULL: tmp_in -> field out), pair: the
// paired row transform (nx/2 = 2 s^2), wide: twice the levels per block;
// y forward (dir < 0: tmp -> spectrum) or backward (dir > 0: spectrum ->
// tmp).
template <typename T>
hipError_t launch_x_zyx_fast(const T *in, cx_t<T> *tmp, double *rowsum, const cx_t<T> *tmp_in,
                             T *out, int nx, int ny, int nz, const cx_t<T> *tw4,
                             const cx_t<T> *tws, int pair, int wide, int accumulate,
                             hipStream_t st);
template <typename T>
hipError_t launch_fft_y_zyx(const cx_t<T> *src, cx_t<T> *dst, int nz, int nkx, int ny, int dir,
                            const cx_t<T> *tw4, hipStream_t st);

// Column solves of the rows kx in [kxlo, kxhi) (kx = 0 excluded: the FP64
// kernel's row).
template <typename T>
hipError_t launch_columns_impl(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, int refine,
                               const int *maskcnt, const Tables<T> &tb, const Tables<double> *t64,
                               hipStream_t st, int variant, int kxlo, int kxhi);

template <typename T>
hipError_t launch_special(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, const int *mlist,
                          int nmask, const double *S, double *ws, const Tables<double> &tb64,
                          hipStream_t st, int parallel);

template <typename T>
hipError_t launch_grad_rho(const T *lam, const T *p, int nx, int ny, int nz, const double *gk,
                           double *partial, int nblk, double *grho, hipStream_t st);

int grad_blocks(int nx, int ny);

StagePlan make_stage_plan(int L);
int set_error(int code, const std::string &msg); // records ps_last_error(), returns code
int column_capacity(int nz);
bool is_2a3b(int n);

} // namespace ps
