// Host side of the pressure-solve library: planning (paper Section 2.1:
// describe the problem once, reuse the plan every timestep), argument
// validation, device tables and workspace, and the C ABI entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ps_internal.h"
#include "ps_plan_impl.h"
#include "../../include/pressure_solve.h"

using namespace ps;

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int ps::set_error(int code, const std::string &msg) { return fail(code, msg); }

#define PS_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(PS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

namespace ps {

// Register capacity (levels per half column) of the column kernels for nz.
int column_capacity(int nz)
{
    int nh = 1;
    while (nh < nz / 2) nh *= 2;
    return nh;
}

bool is_2a3b(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Radix passes for length L = 2^a 3^b: as many radix-8 passes as possible
// (a 16 or a 4 absorbing the remainder of a / 3), then radix-3 passes.
StagePlan make_stage_plan(int L)
{
    StagePlan sp{};
    int a = 0, b = 0, m = L;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    std::vector<int> r(a / 3, 8);
    if (a % 3 == 1) {
        if (!r.empty()) r.back() = 16;
        else r.push_back(2);
    } else if (a % 3 == 2) {
        r.push_back(4);
    }
    for (int i = 0; i < b; ++i) r.push_back(3);
    sp.n = (int)r.size();
    int ns = 1;
    for (int s = 0; s < sp.n; ++s) {
        sp.r[s] = r[s];
        sp.ns[s] = ns;
        ns *= r[s];
    }
    return sp;
}

} // namespace ps

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validation shared by plan creation and batch creation; no HIP calls.
static int validate_grid(int nx, int ny, int nz, double dx, double dy, const double *dz,
                         const double *rho, int precision)
{
    if (!dz || !rho) return fail(PS_EINVAL, "dz and rho must not be NULL");
    if (!finite_pos(dx) || !finite_pos(dy)) return fail(PS_EINVAL, "dx and dy must be finite and > 0");
    if (precision < PS_FP64 || precision > PS_FP32_R1)
        return fail(PS_EUNSUPPORTED, "unknown precision");
    if (nx < 2 || nx % 2 || nx > PS_MAX_NX || !is_2a3b(nx / 2))
        return fail(PS_EUNSUPPORTED, "nx must be even with nx/2 = 2^a 3^b and nx <= 2048");
    if (ny < 1 || ny > PS_MAX_NY || !is_2a3b(ny))
        return fail(PS_EUNSUPPORTED, "ny must be 2^a 3^b and <= 1024");
    if (nz < 1 || nz > PS_MAX_NZ) return fail(PS_EUNSUPPORTED, "nz must be in [1, 256]");
    for (int k = 0; k < nz; ++k) {
        if (!finite_pos(dz[k])) return fail(PS_EINVAL, "dz values must be finite and > 0");
        if (!finite_pos(rho[k])) return fail(PS_EINVAL, "rho values must be finite and > 0");
    }
    return PS_OK;
}

static double lateral(int m, int n, double d)
{
    int mm = m % n;
    if (mm > n - mm) mm = n - mm;
    const double s = std::sin(M_PI * (double)mm / (double)n);
    return 4.0 * s * s / (d * d);
}

// exp(-2 pi i m / n) with the angle formed from the exactly reduced ratio.
static void root(int m, int n, double &c, double &s)
{
    m %= n;
    const double a = 2.0 * M_PI * (double)m / (double)n;
    c = std::cos(a);
    s = -std::sin(a);
}

static void host_tables(ps_plan *p)
{
    const int nz = p->nz;
    p->f.assign(nz + 1, 0.0);
    p->D.assign(nz, 0.0);
    for (int k = 0; k + 1 < nz; ++k) {
        const double h = 0.5 * (p->dz[k] + p->dz[k + 1]);
        p->f[k + 1] = 0.5 * (p->rho[k] + p->rho[k + 1]) / h;
    }
    for (int k = 0; k < nz; ++k) p->D[k] = p->rho[k] * p->dz[k];
    p->ax.resize(p->L + 1);
    for (int kx = 0; kx <= p->L; ++kx) p->ax[kx] = lateral(kx, p->nx, p->dx);
    p->ay.resize(p->ny);
    for (int ky = 0; ky < p->ny; ++ky) p->ay[ky] = lateral(ky, p->ny, p->dy);
}

template <typename T> static int dev_alloc(ps_plan *p, T **ptr, size_t n)
{
    void *q = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return fail(PS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->allocs.push_back(q);
    p->bytes += n * sizeof(T);
    *ptr = reinterpret_cast<T *>(q);
    return PS_OK;
}

template <typename T, typename S> static int upload(T *dst, const std::vector<S> &src)
{
    std::vector<T> tmp(src.begin(), src.end());
    PS_HIP(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
    return PS_OK;
}

#define PS_TRY(x)                                                                                  \
    do {                                                                                           \
        int rc_ = (x);                                                                             \
        if (rc_) return rc_;                                                                       \
    } while (0)

template <typename T> static int alloc_tables(ps_plan *p, Tables<T> &t)
{
    PS_TRY(dev_alloc(p, &t.ax, p->L + 1));
    PS_TRY(dev_alloc(p, &t.ay, p->ny));
    PS_TRY(dev_alloc(p, &t.f, p->nz + 1));
    PS_TRY(dev_alloc(p, &t.D, p->nz));
    PS_TRY(dev_alloc(p, &t.rs_fwd, p->nz));
    PS_TRY(dev_alloc(p, &t.rs_adj, p->nz));
    PS_TRY(dev_alloc(p, &t.os_adj, p->nz));
    PS_TRY(dev_alloc(p, &t.tw_x, p->L));
    PS_TRY(dev_alloc(p, &t.tw_s, p->L));
    PS_TRY(dev_alloc(p, &t.tw_y, p->ny));
    PS_TRY(dev_alloc(p, &t.tw4_x, p->L));
    PS_TRY(dev_alloc(p, &t.tw4_y, p->ny));
    const int nh = column_capacity(p->nz);
    const size_t entry = sizeof(LevelCoef<T>);
    char *cf = nullptr, *ca = nullptr;
    PS_TRY(dev_alloc(p, &cf, entry * (size_t)(2 * nh + 1)));
    PS_TRY(dev_alloc(p, &ca, entry * (size_t)(2 * nh + 1)));
    t.coef_fwd = cf;
    t.coef_adj = ca;
    return PS_OK;
}

template <typename T> static int upload_coeff_tables(ps_plan *p, Tables<T> &t)
{
    const double on = 1.0 / ((double)p->nx * (double)p->ny);
    std::vector<double> rsf(p->nz), rsa(p->nz, -on);
    for (int k = 0; k < p->nz; ++k) rsf[k] = -p->D[k] * on;
    PS_TRY(upload(t.f, p->f));
    PS_TRY(upload(t.D, p->D));
    PS_TRY(upload(t.rs_fwd, rsf));
    PS_TRY(upload(t.rs_adj, rsa));
    PS_TRY(upload(t.os_adj, p->D));
    // Per-slot coefficients in elimination order for the uniform-half column
    // kernel: [low slots][high slots][middle]; each half's n real levels sit in
    // its last n slots, dummies in front.
    const int nz = p->nz, nh = column_capacity(nz), m = nz / 2;
    const long long lvl_bytes = (long long)p->L * p->ny * 2 * (long long)sizeof(T);
    using Coef = LevelCoef<T>;
    for (int adj = 0; adj < 2; ++adj) {
        std::vector<Coef> c(2 * (size_t)nh + 1);
        auto put = [&](int slot, int k, double fp, double fn) {
            Coef &e = c[slot];
            e.fp = (T)fp;
            e.fn = (T)fn;
            e.D = (T)p->D[k];
            e.rs = (T)(adj ? -on : rsf[k]);
            e.os = (T)(adj ? p->D[k] : 1.0);
            e.real = 1;
            e.off = (long long)k * lvl_bytes;
        };
        for (int i = 0; i < 2 * nh + 1; ++i) {
            c[i] = Coef{T(0), T(0), T(1), T(0), T(0), 0, (long long)m * lvl_bytes};
        }
        const int nlo = m, nhi = nz - 1 - m;
        for (int i = 0; i < nlo; ++i) put(nh - nlo + i, i, p->f[i], p->f[i + 1]);
        for (int i = 0; i < nhi; ++i) {
            const int k = nz - 1 - i;
            put(2 * nh - nhi + i, k, p->f[k + 1], p->f[k]);
        }
        put(2 * nh, m, p->f[m], p->f[m + 1]);
        void *dst = adj ? t.coef_adj : t.coef_fwd;
        PS_HIP(hipMemcpy(dst, c.data(), c.size() * sizeof(Coef), hipMemcpyHostToDevice));
    }
    return PS_OK;
}

template <typename T> static int upload_tables(ps_plan *p, Tables<T> &t)
{
    using C = cx_t<T>;
    PS_TRY(upload(t.ax, p->ax));
    PS_TRY(upload(t.ay, p->ay));
    PS_TRY(upload_coeff_tables(p, t));
    auto roots = [&](C *dst, int count, int n) -> int {
        std::vector<C> h(count);
        for (int m = 0; m < count; ++m) {
            double c, s;
            root(m, n, c, s);
            h[m] = C{(T)c, (T)s};
        }
        PS_HIP(hipMemcpy(dst, h.data(), h.size() * sizeof(C), hipMemcpyHostToDevice));
        return PS_OK;
    };
    PS_TRY(roots(t.tw_x, p->L, p->L));
    PS_TRY(roots(t.tw_s, p->L, p->nx));
    PS_TRY(roots(t.tw_y, p->ny, p->ny));
    // four-step twiddles W_n^{t k2} at [k2 R1 + t] for the register kernels
    auto four = [&](C *dst, int n) -> int {
        if (!fast_length(n, sizeof(T) == 8)) return PS_OK;
        const int r1 = fast_r1(n), r2 = n / r1;
        std::vector<C> h(n);
        for (int k2 = 0; k2 < r2; ++k2)
            for (int t = 0; t < r1; ++t) {
                double c, s;
                root(t * k2, n, c, s);
                h[k2 * r1 + t] = C{(T)c, (T)s};
            }
        PS_HIP(hipMemcpy(dst, h.data(), h.size() * sizeof(C), hipMemcpyHostToDevice));
        return PS_OK;
    };
    PS_TRY(four(t.tw4_x, p->L));
    PS_TRY(four(t.tw4_y, p->ny));
    return PS_OK;
}

// Vertical coefficients of the residual kernel: row k's vertical term is
// a_up p_{k+1} + a_dn p_{k-1} - a_c p_k; forward A, then adjoint A^T.
static int upload_residual_table(ps_plan *p)
{
    const int nz = p->nz;
    std::vector<double> rc(6 * (size_t)nz, 0.0);
    for (int k = 0; k < nz; ++k) {
        const double fu = p->f[k + 1], fd = p->f[k], Dk = p->D[k];
        rc[3 * k] = fu / Dk;
        rc[3 * k + 1] = fd / Dk;
        rc[3 * k + 2] = (fu + fd) / Dk;
        double *a = &rc[3 * (size_t)nz + 3 * k];
        a[0] = k + 1 < nz ? fu / p->D[k + 1] : 0.0;
        a[1] = k > 0 ? fd / p->D[k - 1] : 0.0;
        a[2] = (fu + fd) / Dk;
    }
    return upload(p->d_rc, rc);
}

// Divergence and gradient coefficients per level k: rho_{k+1/2}/D_k (0 at
// the top), rho_{k-1/2}/D_k (0 at the bottom), 1/h_{k-1/2} (0 at k = 0).
static int upload_div_table(ps_plan *p)
{
    const int nz = p->nz;
    std::vector<double> dc(3 * (size_t)nz, 0.0);
    for (int k = 0; k < nz; ++k) {
        if (k + 1 < nz) dc[3 * k] = 0.5 * (p->rho[k] + p->rho[k + 1]) / p->D[k];
        if (k > 0) {
            dc[3 * k + 1] = 0.5 * (p->rho[k - 1] + p->rho[k]) / p->D[k];
            dc[3 * k + 2] = 2.0 / (p->dz[k - 1] + p->dz[k]);
        }
    }
    return upload(p->d_dc, dc);
}

static int upload_grad_table(ps_plan *p)
{
    const int nz = p->nz;
    std::vector<double> gk(6 * (size_t)nz + 2, 0.0);
    for (int k = 0; k <= nz; ++k) gk[k] = p->f[k];
    for (int k = 0; k < nz; ++k) {
        gk[nz + 1 + k] = p->D[k];
        gk[2 * nz + 1 + k] = p->rho[k];
        gk[4 * nz + 2 + k] = 1.0 / p->D[k];
        gk[5 * nz + 2 + k] = 1.0 / p->rho[k];
    }
    for (int k = 1; k < nz; ++k) gk[3 * nz + 1 + k] = 2.0 / (p->dz[k - 1] + p->dz[k]);
    return upload(p->d_gk, gk);
}

// Launch geometry of the transform kernels: as many rows per block as fit in
// 64 KiB of LDS (two row buffers plus twiddles), at most 64.
static void choose_geometry(ps_plan *p)
{
    const size_t cs = 2 * p->elem();
    const size_t budget = 65536 / cs;
    int rx = (int)((budget - 2 * (size_t)p->L) / (2 * (size_t)p->L));
    int ry = (int)((budget - (size_t)p->ny) / (2 * (size_t)p->ny));
    rx = std::max(1, std::min(64, rx));
    ry = std::max(1, std::min(64, ry));
    p->geom.rows_x = std::min(rx, p->ny * p->nz);
    p->geom.rows_y = std::min(ry, p->nz * p->L);
    // register-resident kernels where the length has one: the paired row
    // transform forward where nx/2 = 2 s^2, XCD-contiguous tiles backward
    p->geom.variant_x = pair_length(p->L) ? 4 : fast_length(p->L, p->fp64()) ? 1 : 0;
    p->geom.variant_xi = fast_length(p->L, p->fp64()) ? 2 : 0;
    p->geom.variant_y = fast_length(p->ny, p->fp64()) ? 1 : 0;
    // uniform-half column kernels: split lanes with the pivots in LDS for
    // FP64 and the in-register refinement, one complex column per lane for
    // the other FP32 forms
    p->geom.columns = (p->fp64() || p->precision == PS_FP32_R2) ? 6 : 3;
}

// Near-singular columns of the FP32 forms: lateral eigenvalue
// s = ax + ay below tau * max_k (f_{k-1/2} + f_{k+1/2}) / D_k.  s grows with
// kx and with min(ky, ny - ky), so per kx the set is min(ky, ny-ky) < cnt[kx].
static void choose_mask(ps_plan *p, std::vector<int> &cnt, std::vector<int> &list)
{
    cnt.assign(p->L, 0);
    list.clear();
    if (p->fp64()) return;
    double vmax = 0.0;
    for (int k = 0; k < p->nz; ++k) vmax = std::max(vmax, (p->f[k] + p->f[k + 1]) / p->D[k]);
    const double thr = p->tau * vmax;
    for (int kx = 1; kx < p->L; ++kx) {
        int c = 0;
        while (c <= p->ny / 2 && p->ax[kx] + p->ay[c] < thr) ++c;
        cnt[kx] = c;
        for (int ky = 0; ky < p->ny; ++ky)
            if (std::min(ky, p->ny - ky) < c) list.push_back(kx * p->ny + ky);
    }
}

static void free_plan(ps_plan *p)
{
    for (void *q : p->allocs) (void)hipFree(q);
    p->allocs.clear();
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    if (p->ydone) (void)hipEventDestroy(p->ydone);
    if (p->side) (void)hipStreamDestroy(p->side);
    delete p;
}

extern "C" int ps_plan_create(ps_plan **out, int nx, int ny, int nz, double dx, double dy,
                              const double *dz, const double *rho, int precision, double tau,
                              void *stream)
{
    if (!out) return fail(PS_EINVAL, "out must not be NULL");
    *out = nullptr;
    PS_TRY(validate_grid(nx, ny, nz, dx, dy, dz, rho, precision));
    if (std::isnan(tau) || std::isinf(tau)) return fail(PS_EINVAL, "tau must be finite");
    ps_plan *p = new ps_plan();
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->L = nx / 2;
    p->precision = precision;
    p->dx = dx;
    p->dy = dy;
    p->tau = tau > 0 ? tau : 1e-3;
    p->dz.assign(dz, dz + nz);
    p->rho.assign(rho, rho + nz);
    p->stream = reinterpret_cast<hipStream_t>(stream);
    host_tables(p);
    p->spx = make_stage_plan(p->L);
    p->spy = make_stage_plan(ny);
    choose_geometry(p);
    std::vector<int> cnt, list;
    choose_mask(p, cnt, list);
    p->nmask = (int)list.size();
    for (int kx = 1; kx < p->L; ++kx)
        if (cnt[kx] > 0) p->kmask = kx + 1;
    p->nblk = grad_blocks(nx, ny);

    int rc = PS_OK;
    auto step = [&](int r) {
        if (rc == PS_OK) rc = r;
    };
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        free_plan(p);
        return fail(PS_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->fork, kStreamEventFlags) != hipSuccess ||
        hipEventCreateWithFlags(&p->join, kStreamEventFlags) != hipSuccess ||
        hipEventCreateWithFlags(&p->ydone, kStreamEventFlags) != hipSuccess) {
        free_plan(p);
        return fail(PS_EHIP, "stream or event creation failed");
    }
    step(alloc_tables(p, p->t64));
    if (!p->fp64()) step(alloc_tables(p, p->t32));
    const size_t ntask = (size_t)(ny / 2 + 1 + p->nmask);
    if (p->fp64()) {
        double *sp = nullptr;
        step(dev_alloc(p, &sp, 2 * p->spec_elems()));
        p->d_spec = sp;
    } else {
        float *sp = nullptr;
        step(dev_alloc(p, &sp, 2 * p->spec_elems()));
        p->d_spec = sp;
    }
    step(dev_alloc(p, &p->d_rowsum, (size_t)ny * nz));
    step(dev_alloc(p, &p->d_S, (size_t)nz));
    step(dev_alloc(p, &p->d_ws, 6 * (size_t)nz * ntask));
    step(dev_alloc(p, &p->d_gk, 6 * (size_t)nz + 2));
    step(dev_alloc(p, &p->d_partial, (size_t)nz * p->nblk));
    step(dev_alloc(p, &p->d_rc, 6 * (size_t)nz));
    step(dev_alloc(p, &p->d_dc, 3 * (size_t)nz));
    step(dev_alloc(p, &p->d_maskcnt, (size_t)p->L));
    step(dev_alloc(p, &p->d_mlist, list.size()));
    if (rc == PS_OK) step(upload_tables(p, p->t64));
    if (rc == PS_OK && !p->fp64()) step(upload_tables(p, p->t32));
    if (rc == PS_OK) step(upload(p->d_maskcnt, cnt));
    if (rc == PS_OK && !list.empty()) step(upload(p->d_mlist, list));
    if (rc == PS_OK) step(upload_grad_table(p));
    if (rc == PS_OK) step(upload_residual_table(p));
    if (rc == PS_OK) step(upload_div_table(p));
    if (rc != PS_OK) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return PS_OK;
}

extern "C" int ps_plan_destroy(ps_plan *p)
{
    if (!p) return PS_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->side);
    free_plan(p);
    if (e != hipSuccess) return fail(PS_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return PS_OK;
}

extern "C" int ps_plan_set_stream(ps_plan *p, void *stream)
{
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    p->stream = reinterpret_cast<hipStream_t>(stream);
    return PS_OK;
}

extern "C" int ps_plan_set_coeffs(ps_plan *p, const double *rho)
{
    if (!p || !rho) return fail(PS_EINVAL, "plan and rho must not be NULL");
    for (int k = 0; k < p->nz; ++k)
        if (!finite_pos(rho[k])) return fail(PS_EINVAL, "rho values must be finite and > 0");
    // Work enqueued earlier may still read the tables, and not necessarily on
    // the plan's current stream (the stream may have been changed since): wait
    // for the whole device before they are overwritten.
    PS_HIP(hipDeviceSynchronize());
    p->rho.assign(rho, rho + p->nz);
    host_tables(p);
    PS_TRY(upload_coeff_tables(p, p->t64));
    if (!p->fp64()) PS_TRY(upload_coeff_tables(p, p->t32));
    PS_TRY(upload_grad_table(p));
    PS_TRY(upload_residual_table(p));
    PS_TRY(upload_div_table(p));
    return PS_OK;
}

extern "C" size_t ps_workspace_bytes(const ps_plan *p) { return p ? p->bytes : 0; }

// Whether the forward and backward x / y passes run pairwise over level
// ranges (fwd_xy_chunked): the register-resident passes.
static bool xy_chunked(const ps_plan *p)
{
    return p->geom.xy_chunks > 1 && p->geom.variant_x >= 1 && p->geom.variant_xi >= 1 &&
           p->geom.variant_y >= 1;
}

extern "C" int ps_plan_query(const ps_plan *p, ps_plan_info *info)
{
    if (!p || !info) return fail(PS_EINVAL, "plan and info must not be NULL");
    info->nx = p->nx;
    info->ny = p->ny;
    info->nz = p->nz;
    info->precision = p->precision;
    info->fp64_columns = p->nmask;
    info->tau = p->fp64() ? 0.0 : p->tau;
    info->fft_variant_x = p->geom.variant_x;
    info->fft_variant_xi = p->geom.variant_xi;
    info->fft_variant_y = p->geom.variant_y;
    info->spectrum_elems = p->spec_elems();
    info->column_variant = p->geom.columns;
    info->chunks = p->geom.special_side == 1 ? p->geom.chunks : 1;
    info->special_variant = p->geom.special_variant;
    info->zyx_kc = p->geom.zyx_kc;
    info->fp64_beside = p->geom.special_side;
    info->xy_chunks = xy_chunked(p) ? p->geom.xy_chunks : 1;
    return PS_OK;
}

// ------------------------------------------------------------------ timing
// Brackets one enqueue with profiling events when profiling is on.
template <typename F> static hipError_t timed(ps_plan *p, int id, F &&launch,
                                              hipStream_t st = nullptr)
{
    if (!p->prof.on) return launch();
    if (!st) st = p->stream;
    hipEvent_t a = p->prof.get(), b = p->prof.get();
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    p->prof.recs.push_back({id, a, b});
    return e;
}

static int collect_profile(ps_plan *p)
{
    PS_HIP(hipStreamSynchronize(p->stream));
    PS_HIP(hipStreamSynchronize(p->side));
    for (auto &r : p->prof.recs) {
        float ms = 0.f;
        PS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        p->prof.total_ms[r.id] += ms;
        p->prof.launches[r.id] += 1;
        p->prof.pool.push_back(r.a);
        p->prof.pool.push_back(r.b);
    }
    p->prof.recs.clear();
    return PS_OK;
}

extern "C" int ps_plan_profile(ps_plan *p, int enable)
{
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    PS_TRY(collect_profile(p));
    if (enable) {
        for (int i = 0; i < K_COUNT; ++i) {
            p->prof.total_ms[i] = 0.0;
            p->prof.launches[i] = 0;
        }
    }
    p->prof.on = enable != 0;
    return PS_OK;
}

extern "C" int ps_plan_profile_report(ps_plan *p, int idx, const char **name, double *total_ms,
                                      int *launches)
{
    if (!p || idx < 0 || idx >= K_COUNT) return fail(PS_EINVAL, "bad plan or kernel index");
    PS_TRY(collect_profile(p));
    if (name) *name = kKernelNames[idx];
    if (total_ms) *total_ms = p->prof.total_ms[idx];
    if (launches) *launches = p->prof.launches[idx];
    return PS_OK;
}

// ------------------------------------------------------------------ stages
template <typename T> static Tables<T> &tables(ps_plan *p);
template <> Tables<float> &tables<float>(ps_plan *p) { return p->t32; }
template <> Tables<double> &tables<double>(ps_plan *p) { return p->t64; }

template <typename T>
static hipError_t y_pass(ps_plan *p, cx_t<T> *spec, int dir, int kxlo = 0, int kxcnt = -1,
                         hipStream_t st = nullptr, int keep = 0)
{
    const Tables<T> &tb = tables<T>(p);
    if (kxcnt < 0) kxcnt = p->L - kxlo;
    if (kxcnt <= 0) return hipSuccess;
    if (!st) st = p->stream;
    return timed(
        p, dir < 0 ? K_FFT_Y_FWD : K_FFT_Y_INV,
        [&] {
            if (p->geom.variant_y >= 1)
                return launch_fft_y_fast<T>(spec, p->nz, p->L, kxlo, kxcnt, p->ny, dir, tb.tw4_y,
                                            st, p->geom.variant_y, keep);
            return launch_fft_y<T>(spec, p->nz, p->L, kxlo, kxcnt, p->ny, dir, p->geom, p->spy,
                                   tb, st);
        },
        st);
}

// Forward x transform, recording the row sums (no y pass).
template <typename T> static int fwd_x(ps_plan *p, const T *rhs, cx_t<T> *spec)
{
    const Tables<T> &tb = tables<T>(p);
    PS_HIP(timed(p, K_FWD_X, [&] {
        if (p->geom.variant_x >= 1)
            return launch_r2c_fast<T>(rhs, spec, p->d_rowsum, p->nx, p->ny, p->nz, tb.tw4_x,
                                      tb.tw_s, p->stream, nullptr, 0.0, 0.0, nullptr,
                                      p->geom.variant_x);
        return launch_fwd_x<T>(rhs, spec, p->d_rowsum, p->nx, p->ny, p->nz, p->geom, p->spx, tb,
                               p->stream);
    }));
    return PS_OK;
}

template <typename T> static int fwd(ps_plan *p, const T *rhs, cx_t<T> *spec)
{
    PS_TRY(fwd_x<T>(p, rhs, spec));
    PS_HIP(y_pass<T>(p, spec, -1));
    return PS_OK;
}

template <typename T>
static int fwd_residual_x(ps_plan *p, const T *b, const T *x, cx_t<T> *spec, int adjoint)
{
    PS_HIP(timed(p, K_FWD_X_RES, [&] {
        if (p->geom.variant_x >= 1)
            return launch_r2c_fast<T>(b, spec, p->d_rowsum, p->nx, p->ny, p->nz,
                                      tables<T>(p).tw4_x, tables<T>(p).tw_s, p->stream, x,
                                      1.0 / (p->dx * p->dx), 1.0 / (p->dy * p->dy),
                                      p->d_rc + (adjoint ? 3 * (size_t)p->nz : 0),
                                      p->geom.variant_x);
        return launch_fwd_x_residual<T>(b, x, spec, p->d_rowsum, p->nx, p->ny, p->nz,
                                        1.0 / (p->dx * p->dx), 1.0 / (p->dy * p->dy), p->t64.f,
                                        p->t64.D, adjoint, p->geom, p->spx, tables<T>(p),
                                        p->stream);
    }));
    return PS_OK;
}

// Main column solves of the rows kx in [kxlo, kxhi) on the plan's stream.
template <typename T>
static hipError_t main_columns(ps_plan *p, cx_t<T> *spec, int adjoint, int refine, int kxlo,
                               int kxhi)
{
    const int *mc = p->fp64() ? nullptr : p->d_maskcnt;
    return timed(p, K_COLUMNS, [&] {
        return launch_columns_impl<T>(spec, p->nx, p->ny, p->nz, adjoint, refine, mc,
                                      tables<T>(p), &p->t64, p->stream, p->geom.columns, kxlo,
                                      kxhi);
    });
}

// The FP64 columns (packed kx = 0 row, mean column, near-singular columns)
// on stream st.  The level sums of the row sums that the forward x pass
// recorded feed only the mean column, so they are formed here, on the same
// stream, off the main stream's path.
template <typename T>
static hipError_t special_columns(ps_plan *p, cx_t<T> *spec, int adjoint, hipStream_t st)
{
    const hipError_t e = timed(
        p, K_LEVEL_SUMS,
        [&] { return launch_level_sums(p->d_rowsum, p->d_S, p->ny, p->nz, st); }, st);
    if (e != hipSuccess) return e;
    return timed(
        p, K_SPECIAL,
        [&] {
            return launch_special<T>(spec, p->nx, p->ny, p->nz, adjoint, p->d_mlist, p->nmask,
                                     p->d_S, p->d_ws, p->t64, st, p->geom.special_variant);
        },
        st);
}

// Forks the FP64 columns onto the side stream (after what the plan's stream
// has queued); the caller waits for p->join before touching those rows.
template <typename T> static int fork_special(ps_plan *p, cx_t<T> *spec, int adjoint)
{
    PS_HIP(hipEventRecord(p->fork, p->stream));
    PS_HIP(hipStreamWaitEvent(p->side, p->fork, 0));
    PS_HIP(special_columns<T>(p, spec, adjoint, p->side));
    PS_HIP(hipEventRecord(p->join, p->side));
    return PS_OK;
}

// Column solves only (the spectral stage on its own).  The FP64 columns and
// the main column kernel touch disjoint columns, so they may run side by side.
template <typename T> static int columns(ps_plan *p, cx_t<T> *spec, int adjoint, int refine)
{
    if (!p->geom.special_side) {
        PS_HIP(special_columns<T>(p, spec, adjoint, p->stream));
        PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, p->L));
        return PS_OK;
    }
    PS_TRY(fork_special<T>(p, spec, adjoint));
    PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, p->L));
    PS_HIP(hipStreamWaitEvent(p->stream, p->join, 0));
    return PS_OK;
}

// y forward, column solves and y backward.  With the FP64 kernel beside the
// main one, the rows kx < kmask (which hold every FP64 column) are
// transformed apart from the rest -- by the side stream itself when the rest
// is not chunked, else first, on the plan's stream, before the fork -- the
// FP64 kernel runs on the side stream, and the rest runs meanwhile; the
// streams join before those rows are transformed back.  With chunks > 1 the
// rows kx >= kmask are processed in that many
// ranges, each y forward -> columns -> y backward in turn, so that a range's
// spectrum (nz ny (range) values) can still be in the last-level cache (the
// 256 MB Infinity Cache) when the column kernel and the backward y pass read
// it back.
template <typename T> static int middle(ps_plan *p, cx_t<T> *spec, int adjoint, int refine)
{
    const int L = p->L;
    if (!p->geom.special_side) {
        PS_HIP(y_pass<T>(p, spec, -1));
        PS_HIP(special_columns<T>(p, spec, adjoint, p->stream));
        PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, L));
        PS_HIP(y_pass<T>(p, spec, 1));
        return PS_OK;
    }
    if (p->geom.special_side == 2) {
        // The whole y pass on the plan's stream, then the FP64 columns forked
        // beside the main column kernel: one cross-stream wait (the join)
        // on the plan's stream instead of two.
        PS_HIP(y_pass<T>(p, spec, -1));
        PS_TRY(columns<T>(p, spec, adjoint, refine));
        PS_HIP(y_pass<T>(p, spec, 1));
        return PS_OK;
    }
    const int km = std::min(p->kmask, L);
    const int nch = std::max(1, std::min(p->geom.chunks, L - km));
    if (nch <= 1) {
        // The side stream transforms the rows kx < km itself, then forms the
        // level sums and solves the FP64 columns; the main stream transforms
        // the other rows meanwhile (disjoint rows) and waits for the side
        // stream's y pass before its column kernel, which also covers the
        // ordinary columns of the rows kx < km.
        PS_HIP(hipEventRecord(p->fork, p->stream));
        PS_HIP(hipStreamWaitEvent(p->side, p->fork, 0));
        PS_HIP(y_pass<T>(p, spec, -1, 0, km, p->side));
        PS_HIP(hipEventRecord(p->ydone, p->side));
        PS_HIP(special_columns<T>(p, spec, adjoint, p->side));
        PS_HIP(hipEventRecord(p->join, p->side));
        PS_HIP(y_pass<T>(p, spec, -1, km));
        PS_HIP(hipStreamWaitEvent(p->stream, p->ydone, 0));
        PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, L));
        PS_HIP(hipStreamWaitEvent(p->stream, p->join, 0));
        PS_HIP(y_pass<T>(p, spec, 1));
        return PS_OK;
    }
    PS_HIP(y_pass<T>(p, spec, -1, 0, km));
    PS_TRY(fork_special<T>(p, spec, adjoint));
    PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, km));
    const long rest = L - km;
    for (int c = 0; c < nch; ++c) {
        const int a = km + (int)(rest * c / nch), b = km + (int)(rest * (c + 1) / nch);
        if (b <= a) continue;
        PS_HIP(y_pass<T>(p, spec, -1, a, b - a, nullptr, 1));
        PS_HIP(main_columns<T>(p, spec, adjoint, refine, a, b));
        PS_HIP(y_pass<T>(p, spec, 1, a, b - a));
    }
    PS_HIP(hipStreamWaitEvent(p->stream, p->join, 0));
    PS_HIP(y_pass<T>(p, spec, 1, 0, km));
    return PS_OK;
}

// Backward x pass only.
template <typename T> static int inv_x(ps_plan *p, cx_t<T> *spec, T *out, int accumulate)
{
    const Tables<T> &tb = tables<T>(p);
    PS_HIP(timed(p, K_INV_X, [&] {
        if (p->geom.variant_xi >= 1)
            return launch_c2r_fast<T>(spec, out, p->nx, p->ny, p->nz, accumulate, tb.tw4_x,
                                      tb.tw_s, p->stream, p->geom.variant_xi);
        return launch_inv_x<T>(spec, out, p->nx, p->ny, p->nz, accumulate, p->geom, p->spx, tb,
                               p->stream);
    }));
    return PS_OK;
}

// Backward y and x passes (the inverse-transform stage on its own).
template <typename T> static int inv(ps_plan *p, cx_t<T> *spec, T *out, int accumulate)
{
    PS_HIP(y_pass<T>(p, spec, 1));
    return inv_x<T>(p, spec, out, accumulate);
}

// The forward x and y passes taken pairwise over xy_chunks level ranges,
// and likewise the backward y and x passes: each y pass reads the range its
// x pass has just written (and each backward x pass the range its y pass has
// just written) while much of it is still in the last-level cache (the
// 256 MB Infinity Cache: about 2 ranges at 1024^2 x 128 FP32, 4 FP64).
// Every level is transformed by the same kernels as in the whole-field
// passes, so the result is the same bit for bit.
// With the FP64 columns on the side stream with their rows (placement 1),
// the side stream transforms the rows kx < kmask of each range in y as soon
// as the range's x pass is done (an event per range, recorded after it),
// then forms the level sums and solves the FP64 columns; the plan's stream
// transforms the other rows of each range meanwhile.
template <typename T>
static int fwd_xy_chunked(ps_plan *p, const T *in, cx_t<T> *spec, int adjoint)
{
    const Tables<T> &tb = tables<T>(p);
    const size_t lin = (size_t)p->nx * p->ny, lsp = (size_t)p->L * p->ny;
    const int nc = p->geom.xy_chunks;
    const bool beside = p->geom.special_side == 1;
    const int km = beside ? std::min(p->kmask, p->L) : 0;
    for (int c = 0; c < nc; ++c) {
        const int k0 = (int)((long)p->nz * c / nc), k1 = (int)((long)p->nz * (c + 1) / nc);
        if (k1 <= k0) continue;
        PS_HIP(timed(p, K_FWD_X, [&] {
            return launch_r2c_fast<T>(in + k0 * lin, spec + k0 * lsp,
                                      p->d_rowsum + (size_t)k0 * p->ny, p->nx, p->ny, k1 - k0,
                                      tb.tw4_x, tb.tw_s, p->stream, nullptr, 0.0, 0.0, nullptr,
                                      p->geom.variant_x);
        }));
        if (beside) {
            PS_HIP(hipEventRecord(p->fork, p->stream));
            PS_HIP(hipStreamWaitEvent(p->side, p->fork, 0));
        }
        if (beside && km > 0) {
            PS_HIP(timed(
                p, K_FFT_Y_FWD,
                [&] {
                    return launch_fft_y_fast<T>(spec + k0 * lsp, k1 - k0, p->L, 0, km, p->ny, -1,
                                                tb.tw4_y, p->side, p->geom.variant_y, 0);
                },
                p->side));
        }
        if (km < p->L)
            PS_HIP(timed(p, K_FFT_Y_FWD, [&] {
                return launch_fft_y_fast<T>(spec + k0 * lsp, k1 - k0, p->L, km, p->L - km, p->ny,
                                            -1, tb.tw4_y, p->stream, p->geom.variant_y, 0);
            }));
    }
    if (beside) {
        PS_HIP(hipEventRecord(p->ydone, p->side));
        PS_HIP(special_columns<T>(p, spec, adjoint, p->side));
        PS_HIP(hipEventRecord(p->join, p->side));
    }
    return PS_OK;
}

template <typename T> static int inv_yx_chunked(ps_plan *p, cx_t<T> *spec, T *out)
{
    const Tables<T> &tb = tables<T>(p);
    const size_t lin = (size_t)p->nx * p->ny, lsp = (size_t)p->L * p->ny;
    const int nc = p->geom.xy_chunks;
    for (int c = 0; c < nc; ++c) {
        const int k0 = (int)((long)p->nz * c / nc), k1 = (int)((long)p->nz * (c + 1) / nc);
        if (k1 <= k0) continue;
        PS_HIP(timed(p, K_FFT_Y_INV, [&] {
            return launch_fft_y_fast<T>(spec + k0 * lsp, k1 - k0, p->L, 0, p->L, p->ny, 1,
                                        tb.tw4_y, p->stream, p->geom.variant_y, 0);
        }));
        PS_HIP(timed(p, K_INV_X, [&] {
            return launch_c2r_fast<T>(spec + k0 * lsp, out + k0 * lin, p->nx, p->ny, k1 - k0, 0,
                                      tb.tw4_x, tb.tw_s, p->stream, p->geom.variant_xi);
        }));
    }
    return PS_OK;
}

template <typename T> static int run(ps_plan *p, const T *in, T *out, int adjoint)
{
    auto *spec = reinterpret_cast<cx_t<T> *>(p->d_spec);
    const int refine = p->precision == PS_FP32_R2;
    if (xy_chunked(p)) {
        PS_TRY(fwd_xy_chunked<T>(p, in, spec, adjoint));
        if (p->geom.special_side == 1) {
            // the side stream's y pass of the rows kx < kmask, then its FP64
            // columns (joined before the backward passes)
            PS_HIP(hipStreamWaitEvent(p->stream, p->ydone, 0));
            PS_HIP(main_columns<T>(p, spec, adjoint, refine, 1, p->L));
            PS_HIP(hipStreamWaitEvent(p->stream, p->join, 0));
        } else {
            PS_TRY(columns<T>(p, spec, adjoint, refine));
        }
        PS_TRY(inv_yx_chunked<T>(p, spec, out));
    } else {
        PS_TRY(fwd_x<T>(p, in, spec));
        PS_TRY(middle<T>(p, spec, adjoint, refine));
        PS_TRY(inv_x<T>(p, spec, out, 0));
    }
    // R1's second solve takes the whole-field passes: its fused residual
    // reads p at the neighbouring levels
    if (p->precision == PS_FP32_R1) {
        PS_TRY(fwd_residual_x<T>(p, in, out, spec, adjoint));
        PS_TRY(middle<T>(p, spec, adjoint, 0));
        PS_TRY(inv_x<T>(p, spec, out, 1));
    }
    return PS_OK;
}

// Whether the z-fastest solve takes the register-resident passes through
// the [kx][j][k] buffer (the plan's x and y passes are register-resident).
static bool zyx_fast(const ps_plan *p) { return p->geom.variant_x >= 1 && p->geom.variant_y >= 1; }

// The solve for fields in the z-fastest (MONC) layout.  Register-resident
// lengths: forward x (field -> [kx][j][k], loads and stores along k), y
// forward ([kx][j][k] -> spectrum), the column solves, y backward and
// backward x, the same bytes per point as the level-major solve.  Other
// lengths: x passes that transpose between columns and rows in LDS around
// the level-major y / column / y passes.
template <typename T>
static int run_zyx_pass(ps_plan *p, const T *in, T *out, int adjoint, int accumulate)
{
    auto *spec = reinterpret_cast<cx_t<T> *>(p->d_spec);
    const Tables<T> &tb = tables<T>(p);
    if (zyx_fast(p)) {
        if (!p->d_zyx) {
            cx_t<T> *buf = nullptr;
            PS_TRY(dev_alloc(p, &buf, p->spec_elems()));
            p->d_zyx = buf;
        }
        auto *tmp = reinterpret_cast<cx_t<T> *>(p->d_zyx);
        const int refine = p->precision == PS_FP32_R2;
        const int wide = p->geom.zyx_kc >= 32;
        PS_HIP(timed(p, K_FWD_X, [&] {
            return launch_x_zyx_fast<T>(in, tmp, p->d_rowsum, nullptr, nullptr, p->nx, p->ny,
                                        p->nz, tb.tw4_x, tb.tw_s,
                                        p->geom.variant_x == 4 && pair_length(p->L), wide, 0,
                                        p->stream);
        }));
        PS_HIP(timed(p, K_FFT_Y_FWD, [&] {
            return launch_fft_y_zyx<T>(tmp, spec, p->nz, p->L, p->ny, -1, tb.tw4_y, p->stream);
        }));
        PS_TRY(columns<T>(p, spec, adjoint, refine));
        PS_HIP(timed(p, K_FFT_Y_INV, [&] {
            return launch_fft_y_zyx<T>(spec, tmp, p->nz, p->L, p->ny, 1, tb.tw4_y, p->stream);
        }));
        PS_HIP(timed(p, K_INV_X, [&] {
            return launch_x_zyx_fast<T>(nullptr, nullptr, nullptr, tmp, out, p->nx, p->ny, p->nz,
                                        tb.tw4_x, tb.tw_s,
                                        p->geom.variant_xi == 4 && pair_length(p->L), wide,
                                        accumulate, p->stream);
        }));
        return PS_OK;
    }
    PS_HIP(timed(p, K_FWD_X, [&] {
        return launch_fwd_x_zyx<T>(in, spec, p->d_rowsum, p->nx, p->ny, p->nz, p->geom.rows_x,
                                   p->geom.zyx_kc, p->spx, tb, p->stream);
    }));
    PS_TRY(middle<T>(p, spec, adjoint, p->precision == PS_FP32_R2));
    PS_HIP(timed(p, K_INV_X, [&] {
        return launch_inv_x_zyx<T>(spec, out, p->nx, p->ny, p->nz, p->geom.rows_x,
                                   p->geom.zyx_kc, p->spx, tb, p->stream, accumulate);
    }));
    return PS_OK;
}

// The z-fastest solve; the PS_FP32_R1 form adds one refinement step: the
// residual of the first solution (FP64 accumulation, a pass of its own in
// this layout), its solve, and the correction accumulated by the last
// backward x pass.
template <typename T> static int run_zyx(ps_plan *p, const T *in, T *out, int adjoint)
{
    PS_TRY(run_zyx_pass<T>(p, in, out, adjoint, 0));
    if (p->precision != PS_FP32_R1) return PS_OK;
    if (!p->d_zyx_res) {
        T *buf = nullptr;
        PS_TRY(dev_alloc(p, &buf, (size_t)p->nx * p->ny * p->nz));
        p->d_zyx_res = buf;
    }
    T *res = reinterpret_cast<T *>(p->d_zyx_res);
    PS_HIP(timed(p, K_FWD_X_RES, [&] {
        return launch_residual_zyx<T>(in, out, res, p->nx, p->ny, p->nz, 1.0 / (p->dx * p->dx),
                                      1.0 / (p->dy * p->dy),
                                      p->d_rc + (adjoint ? 3 * (size_t)p->nz : 0), p->stream);
    }));
    return run_zyx_pass<T>(p, res, out, adjoint, 1);
}

static int solve_zyx_common(ps_plan *p, const void *in, void *out, int adjoint)
{
    if (!p || !in || !out) return fail(PS_EINVAL, "plan, input and output must not be NULL");
    if (p->precision == PS_FP32_R1 && in == out)
        return fail(PS_EINVAL, "the PS_FP32_R1 form needs input and output not to alias");
    if (p->fp64()) return run_zyx<double>(p, (const double *)in, (double *)out, adjoint != 0);
    return run_zyx<float>(p, (const float *)in, (float *)out, adjoint != 0);
}

extern "C" int ps_solve_zyx(ps_plan *p, const void *rhs, void *out, int adjoint)
{
    return solve_zyx_common(p, rhs, out, adjoint);
}

// One projection step: p = S(div(u, v, w) / dt) with the divergence formed
// inside the forward x pass, then optionally (u, v, w) -= dt G p.
template <typename T>
static int run_project(ps_plan *p, T *u, T *v, T *w, double dt, T *out, int correct)
{
    auto *spec = reinterpret_cast<cx_t<T> *>(p->d_spec);
    const Tables<T> &tb = tables<T>(p);
    PS_HIP(timed(p, K_FWD_X_DIV, [&] {
        if (p->geom.variant_x >= 1)
            return launch_r2c_fast<T>(u, spec, p->d_rowsum, p->nx, p->ny, p->nz, tb.tw4_x,
                                      tb.tw_s, p->stream, v, 1.0 / p->dx, 1.0 / p->dy, p->d_dc,
                                      p->geom.variant_x, w, 1.0 / dt);
        return launch_fwd_x_div<T>(u, v, w, 1.0 / dt, spec, p->d_rowsum, p->nx, p->ny, p->nz,
                                   p->dx, p->dy, p->d_dc, p->geom, p->spx, tb, p->stream);
    }));
    PS_TRY(middle<T>(p, spec, 0, p->precision == PS_FP32_R2));
    PS_TRY(inv_x<T>(p, spec, out, 0));
    if (p->precision == PS_FP32_R1) {
        // one refinement step: the residual of the divergence, formed again
        // inside the forward pass with FP64 accumulation, solved and added
        PS_HIP(timed(p, K_FWD_X_RES, [&] {
            return launch_fwd_x_div<T>(u, v, w, 1.0 / dt, spec, p->d_rowsum, p->nx, p->ny,
                                       p->nz, p->dx, p->dy, p->d_dc, p->geom, p->spx, tb,
                                       p->stream, out, p->d_rc);
        }));
        PS_TRY(middle<T>(p, spec, 0, 0));
        PS_TRY(inv_x<T>(p, spec, out, 1));
    }
    if (correct)
        PS_HIP(timed(p, K_CORRECT, [&] {
            return launch_grad_correct<T>(u, v, w, out, dt, p->nx, p->ny, p->nz, p->dx, p->dy,
                                          p->d_dc, p->stream);
        }));
    return PS_OK;
}

extern "C" int ps_project(ps_plan *p, void *u, void *v, void *w, double dt, void *out,
                          int correct)
{
    if (!p || !u || !v || !w || !out) return fail(PS_EINVAL, "arguments must not be NULL");
    if (!std::isfinite(dt) || dt <= 0.0) return fail(PS_EINVAL, "dt must be finite and > 0");
    if (out == u || out == v || out == w || u == v || u == w || v == w)
        return fail(PS_EINVAL, "u, v, w and p must be distinct fields");
    if (p->fp64())
        return run_project<double>(p, (double *)u, (double *)v, (double *)w, dt, (double *)out,
                                   correct);
    return run_project<float>(p, (float *)u, (float *)v, (float *)w, dt, (float *)out, correct);
}

static int solve_common(ps_plan *p, const void *in, void *out, int adjoint)
{
    if (!p || !in || !out) return fail(PS_EINVAL, "plan, input and output must not be NULL");
    if (p->precision == PS_FP32_R1 && in == out)
        return fail(PS_EINVAL, "the PS_FP32_R1 form needs input and output not to alias");
    if (p->fp64()) return run<double>(p, (const double *)in, (double *)out, adjoint);
    return run<float>(p, (const float *)in, (float *)out, adjoint);
}

extern "C" int ps_solve(ps_plan *p, const void *rhs, void *out) { return solve_common(p, rhs, out, 0); }

extern "C" int ps_solve_adjoint(ps_plan *p, const void *gp, void *grhs)
{
    return solve_common(p, gp, grhs, 1);
}

extern "C" int ps_grad_coeffs(ps_plan *p, const void *lam, const void *x, double *grho)
{
    if (!p || !lam || !x || !grho) return fail(PS_EINVAL, "arguments must not be NULL");
    PS_HIP(timed(p, K_GRAD, [&] {
        if (p->fp64())
            return launch_grad_rho<double>((const double *)lam, (const double *)x, p->nx, p->ny,
                                           p->nz, p->d_gk, p->d_partial, p->nblk, grho, p->stream);
        return launch_grad_rho<float>((const float *)lam, (const float *)x, p->nx, p->ny, p->nz,
                                      p->d_gk, p->d_partial, p->nblk, grho, p->stream);
    }));
    return PS_OK;
}

extern "C" int ps_forward_transform(ps_plan *p, const void *rhs, void *spectrum)
{
    if (!p || !rhs || !spectrum) return fail(PS_EINVAL, "arguments must not be NULL");
    if (p->fp64()) return fwd<double>(p, (const double *)rhs, (double2 *)spectrum);
    return fwd<float>(p, (const float *)rhs, (float2 *)spectrum);
}

extern "C" int ps_spectral_solve(ps_plan *p, void *spectrum, int adjoint)
{
    if (!p || !spectrum) return fail(PS_EINVAL, "arguments must not be NULL");
    const int refine = p->precision == PS_FP32_R2;
    if (p->fp64()) return columns<double>(p, (double2 *)spectrum, adjoint != 0, 0);
    return columns<float>(p, (float2 *)spectrum, adjoint != 0, refine);
}

extern "C" int ps_inverse_transform(ps_plan *p, const void *spectrum, void *out)
{
    if (!p || !spectrum || !out) return fail(PS_EINVAL, "arguments must not be NULL");
    // The backward y pass runs in place, so work on the plan's own buffer.
    const size_t bytes = p->spec_elems() * 2 * p->elem();
    if (spectrum != p->d_spec)
        PS_HIP(hipMemcpyAsync(p->d_spec, spectrum, bytes, hipMemcpyDeviceToDevice, p->stream));
    if (p->fp64()) return inv<double>(p, (double2 *)p->d_spec, (double *)out, 0);
    return inv<float>(p, (float2 *)p->d_spec, (float *)out, 0);
}

// ------------------------------------------------------------------ autotuning
// Planning chooses kernels from the sizes alone; ps_plan_autotune instead
// times the implemented variants on the device (the measured planning that
// FFTW offers, done here for this library's own kernels): coordinate descent
// over the x-transform kernel, the y-transform kernel and the column-solve
// variant, each candidate timed over `reps` solves with events on the plan's
// stream.  Choices are cached per (device architecture, nx, ny, nz,
// precision) for the life of the process and can be saved and loaded as text.
static std::mutex g_tune_mu;
static std::map<std::string, FftGeom> g_tune;

static std::string tune_key(const ps_plan *p)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << ' ' << p->nx << ' ' << p->ny << ' ' << p->nz << ' ' << p->precision;
    return k.str();
}

static int time_solves(ps_plan *p, const void *in, void *out, int reps, float *ms,
                       int (*solve)(ps_plan *, const void *, void *, int) = solve_common)
{
    hipEvent_t a, b;
    PS_HIP(hipEventCreate(&a));
    PS_HIP(hipEventCreate(&b));
    int rc = solve(p, in, out, 0); // warm-up
    if (rc == PS_OK && hipEventRecord(a, p->stream) != hipSuccess) rc = PS_EHIP;
    for (int i = 0; i < reps && rc == PS_OK; ++i) rc = solve(p, in, out, 0);
    if (rc == PS_OK && hipEventRecord(b, p->stream) != hipSuccess) rc = PS_EHIP;
    if (rc == PS_OK && hipEventSynchronize(b) != hipSuccess) rc = PS_EHIP;
    if (rc == PS_OK && hipEventElapsedTime(ms, a, b) != hipSuccess) rc = PS_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == PS_EHIP) g_last_error = "autotune timing failed";
    return rc;
}

extern "C" int ps_plan_autotune(ps_plan *p, int reps)
{
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    if (reps < 1) reps = 1;
    if (reps > 100) reps = 100;
    const std::string key = tune_key(p);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            // only the tuned knobs: the tile shapes follow from the plan
            p->geom.variant_x = fast_length(p->L, p->fp64()) ? it->second.variant_x : 0;
            p->geom.variant_xi = fast_length(p->L, p->fp64()) ? it->second.variant_xi : 0;
            p->geom.variant_y = fast_length(p->ny, p->fp64()) ? it->second.variant_y : 0;
            p->geom.columns = it->second.columns;
            p->geom.special_side = it->second.special_side;
            p->geom.chunks = it->second.chunks;
            p->geom.special_variant = it->second.special_variant;
            p->geom.zyx_kc = it->second.zyx_kc;
            p->geom.xy_chunks = it->second.xy_chunks;
            return PS_OK;
        }
    }
    const size_t bytes = (size_t)p->nx * p->ny * p->nz * p->elem();
    void *in = nullptr, *out = nullptr;
    PS_HIP(hipMalloc(&in, bytes));
    if (hipMalloc(&out, bytes) != hipSuccess) {
        (void)hipFree(in);
        return fail(PS_ENOMEM, "autotune buffers");
    }
    int rc = PS_OK;
    if (hipMemsetAsync(in, 0, bytes, p->stream) != hipSuccess) rc = fail(PS_EHIP, "memset");
    const bool prof = p->prof.on;
    p->prof.on = false;
    // Each option is timed in two interleaved rounds (A B C, A B C) and keeps
    // its faster time, so that a slow drift of the clock or a one-off stall
    // does not decide between options a few per cent apart.
    auto pick = [&](int FftGeom::*knob, const std::vector<int> &opts,
                    int (*solve)(ps_plan *, const void *, void *, int) = solve_common) {
        if (rc != PS_OK || opts.size() < 2) return;
        std::vector<float> best_of(opts.size(), 1e30f);
        for (int round = 0; round < 2; ++round) {
            for (size_t i = 0; i < opts.size(); ++i) {
                p->geom.*knob = opts[i];
                float ms = 0.f;
                rc = time_solves(p, in, out, reps, &ms, solve);
                if (rc != PS_OK) return;
                best_of[i] = std::min(best_of[i], ms);
            }
        }
        size_t best = 0;
        for (size_t i = 1; i < opts.size(); ++i)
            if (best_of[i] < best_of[best]) best = i;
        p->geom.*knob = opts[best];
    };
    std::vector<int> vx{0}, vy{0};
    if (fast_length(p->L, p->fp64())) vx.insert(vx.end(), {1, 2, 3});
    if (pair_length(p->L)) vx.push_back(4);
    if (fast_length(p->ny, p->fp64())) vy.insert(vy.end(), {1, 2});
    pick(&FftGeom::variant_x, vx);
    pick(&FftGeom::variant_xi, vx);
    pick(&FftGeom::variant_y, vy);
    if (p->precision != PS_FP32_R2)
        pick(&FftGeom::columns, {0, 1, 2, 3, 4, 5, 6, 7, 8});
    else
        pick(&FftGeom::columns, {0, 3, 5, 6, 7, 8});
    pick(&FftGeom::special_variant, {0, 1});
    pick(&FftGeom::special_side, {0, 1, 2});
    if (p->geom.special_side == 1) pick(&FftGeom::chunks, {1, 2, 4, 8});
    // The level-range passes with each FP64-column placement, against the
    // placement just chosen, in one search (the placement that wins with
    // whole-field passes need not win with ranges).
    if (rc == PS_OK && p->geom.variant_x >= 1 && p->geom.variant_xi >= 1 &&
        p->geom.variant_y >= 1 && p->nz >= 2) {
        std::vector<std::pair<int, int>> combos{{p->geom.special_side, 1}};
        for (int c : {2, 3, 4, 8})
            if (c <= p->nz)
                for (int side : {0, 1, 2}) combos.push_back({side, c});
        std::vector<float> best_of(combos.size(), 1e30f);
        for (int round = 0; round < 2 && rc == PS_OK; ++round) {
            for (size_t i = 0; i < combos.size() && rc == PS_OK; ++i) {
                p->geom.special_side = combos[i].first;
                p->geom.xy_chunks = combos[i].second;
                float ms = 0.f;
                rc = time_solves(p, in, out, reps, &ms, solve_common);
                best_of[i] = std::min(best_of[i], ms);
            }
        }
        size_t best = 0;
        for (size_t i = 1; i < combos.size(); ++i)
            if (best_of[i] < best_of[best]) best = i;
        p->geom.special_side = combos[best].first;
        p->geom.xy_chunks = combos[best].second;
        // the transform variants again, for launches over level ranges
        if (p->geom.xy_chunks > 1) {
            pick(&FftGeom::variant_x, vx);
            pick(&FftGeom::variant_xi, vx);
            pick(&FftGeom::variant_y, vy);
        }
    }
    if (zyx_fast(p))
        pick(&FftGeom::zyx_kc, {16, 64}, solve_zyx_common); // standard or wide blocks
    else
        pick(&FftGeom::zyx_kc, {1, 2, 4, 8, 64}, solve_zyx_common);
    p->prof.on = prof;
    (void)hipStreamSynchronize(p->stream);
    (void)hipFree(in);
    (void)hipFree(out);
    if (rc != PS_OK) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = p->geom;
    return PS_OK;
}

// Text format, one line per entry: arch nx ny nz precision variant_x
// variant_y columns special_side chunks variant_xi special_variant zyx_kc
// xy_chunks (the last six optional on reading; variant_xi defaults to
// variant_x, special_variant to 1, zyx_kc to 64, xy_chunks to 1)
extern "C" int ps_tune_cache_save(const char *path)
{
    if (!path) return fail(PS_EINVAL, "path is NULL");
    std::ofstream f(path);
    if (!f) return fail(PS_EINVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : g_tune)
        f << kv.first << ' ' << kv.second.variant_x << ' ' << kv.second.variant_y << ' '
          << kv.second.columns << ' ' << kv.second.special_side << ' ' << kv.second.chunks << ' '
          << kv.second.variant_xi << ' ' << kv.second.special_variant << ' '
          << kv.second.zyx_kc << ' ' << kv.second.xy_chunks << '\n';
    return f.good() ? PS_OK : fail(PS_EINVAL, "write failed");
}

extern "C" int ps_tune_cache_load(const char *path)
{
    if (!path) return fail(PS_EINVAL, "path is NULL");
    std::ifstream f(path);
    if (!f) return fail(PS_EINVAL, std::string("cannot read ") + path);
    std::string line;
    std::map<std::string, FftGeom> got;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string arch;
        int nx, ny, nz, prec, vx, vy, col, side = 1, chunks = 1, vxi = -1, spv = 1, zkc = 64,
            xyc = 1;
        if (!(is >> arch >> nx >> ny >> nz >> prec >> vx >> vy >> col)) continue;
        if (!(is >> side)) side = 1;
        if (!(is >> chunks)) chunks = 1;
        if (!(is >> vxi)) vxi = vx;
        if (!(is >> spv)) spv = 1;
        if (!(is >> zkc)) zkc = 64;
        if (!(is >> xyc)) xyc = 1;
        if (vx < 0 || vx > 4 || vy < 0 || vy > 2 || col < 0 || col > 8 || side < 0 || side > 2 ||
            chunks < 1 || chunks > 64 || vxi < 0 || vxi > 4 || spv < 0 || spv > 1 || zkc < 1 ||
            zkc > 256 || xyc < 1 || xyc > 64)
            continue;
        std::ostringstream k;
        k << arch << ' ' << nx << ' ' << ny << ' ' << nz << ' ' << prec;
        FftGeom g;
        g.variant_x = fast_length(nx / 2, prec == PS_FP64) ? vx : 0;
        g.variant_xi = fast_length(nx / 2, prec == PS_FP64) ? vxi : 0;
        g.variant_y = fast_length(ny, prec == PS_FP64) ? vy : 0;
        g.columns = col;
        g.special_side = side;
        g.chunks = chunks;
        g.special_variant = spv;
        g.zyx_kc = zkc;
        g.xy_chunks = xyc;
        got[k.str()] = g;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : got) g_tune[kv.first] = kv.second;
    return PS_OK;
}

extern "C" const char *ps_status_string(int s)
{
    switch (s) {
    case PS_OK: return "ok";
    case PS_EINVAL: return "invalid argument";
    case PS_EUNSUPPORTED: return "unsupported size or precision";
    case PS_ENOMEM: return "out of memory";
    case PS_EHIP: return "HIP runtime error";
    case PS_ESTATE: return "invalid state";
    default: return "unknown status";
    }
}

extern "C" const char *ps_last_error(void) { return g_last_error.c_str(); }
