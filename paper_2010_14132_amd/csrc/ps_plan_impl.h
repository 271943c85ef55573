// The plan object behind the C ABI's opaque ps_plan handle (shared by the
// planning code and the batched solver).
#pragma once
#include <vector>

#include "ps_internal.h"
#include "../../include/pressure_solve.h"

using ps::FftGeom;
using ps::StagePlan;
using ps::Tables;

// Per-kernel event timing (see ps_plan_profile).
enum KernelId { K_FWD_X, K_FWD_X_RES, K_LEVEL_SUMS, K_FFT_Y_FWD, K_COLUMNS, K_SPECIAL, K_FFT_Y_INV,
                K_INV_X, K_GRAD, K_FWD_X_DIV, K_CORRECT, K_COUNT };
static const char *const kKernelNames[K_COUNT] = {
    "fwd_x", "fwd_x_residual", "level_sums", "fft_y_fwd", "columns", "special_fp64",
    "fft_y_inv", "inv_x", "grad_rho", "fwd_x_divergence", "grad_correct"};

struct Profiler {
    bool on = false;
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double total_ms[K_COUNT] = {};
    int launches[K_COUNT] = {};
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Profiler()
    {
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct ps_plan {
    Profiler prof;
    int nx = 0, ny = 0, nz = 0, L = 0, precision = 0;
    double dx = 0, dy = 0, tau = 0;
    std::vector<double> dz, rho;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;        // the FP64 column kernel runs here, beside the main one
    hipEvent_t fork = nullptr, join = nullptr, ydone = nullptr;
    int device = 0;
    std::vector<double> ax, ay, f, D;
    StagePlan spx{}, spy{};
    FftGeom geom;
    Tables<float> t32;
    Tables<double> t64;
    int *d_maskcnt = nullptr;
    int *d_mlist = nullptr;
    int nmask = 0;
    int kmask = 1; // rows kx < kmask hold every column solved in FP64
    void *d_spec = nullptr;
    double *d_rowsum = nullptr;
    double *d_S = nullptr;
    double *d_ws = nullptr;
    double *d_gk = nullptr;
    double *d_partial = nullptr;
    double *d_rc = nullptr; // residual vertical coefficients [fwd: 3 nz][adj: 3 nz]
    double *d_dc = nullptr; // divergence / gradient coefficients, 3 per level
    void *d_zyx = nullptr;  // [kx][j][k] buffer of the z-fastest solve (allocated on its first call)
    void *d_zyx_res = nullptr; // residual field of the z-fastest PS_FP32_R1 solve (idem)
    int nblk = 0;
    size_t bytes = 0;
    std::vector<void *> allocs;
    bool fp64() const { return precision == PS_FP64; }
    size_t elem() const { return fp64() ? sizeof(double) : sizeof(float); }
    size_t spec_elems() const { return (size_t)nz * L * ny; }
};

