// Internal host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <type_traits>
#include <string>
#include <vector>

#include "ps_device.h"

namespace ps {

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
};

// Launch geometry of the transform kernels chosen at planning time.
struct FftGeom {
    int rows_x = 1;   // rows per block of the x passes
    int rows_y = 1;   // rows per block of the y passes
    int variant_x = 0;
    int variant_y = 0;
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
template <typename T>
hipError_t launch_fft_y(cx_t<T> *spec, int nrows, int ny, int dir, const FftGeom &g,
                        const StagePlan &spy, const Tables<T> &tb, hipStream_t st);
template <typename T>
hipError_t launch_inv_x(const cx_t<T> *spec, T *out, int nx, int ny, int nz, int accumulate,
                        const FftGeom &g, const StagePlan &spx, const Tables<T> &tb,
                        hipStream_t st);

hipError_t launch_level_sums(const double *rowsum, double *S, int ny, int nz, hipStream_t st);

template <typename T>
hipError_t launch_columns_impl(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, int refine,
                               const int *maskcnt, const Tables<T> &tb, const Tables<double> *t64,
                               hipStream_t st);

template <typename T>
hipError_t launch_special(cx_t<T> *spec, int nx, int ny, int nz, int adjoint, const int *mlist,
                          int nmask, const double *S, double *ws, const Tables<double> &tb64,
                          hipStream_t st);

template <typename T>
hipError_t launch_grad_rho(const T *lam, const T *p, int nx, int ny, int nz, const double *gk,
                           double *partial, int nblk, double *grho, hipStream_t st);

int grad_blocks(int nx, int ny);

StagePlan make_stage_plan(int L);
bool is_2a3b(int n);

} // namespace ps
