// ps_grad_coeffs_noalloc: the density gradient with its per-block partial
// sums in a fixed device array of this library instead of the plan's
// buffer, for callers that may not allocate during the call.
//
// The array below is one per GPU the library runs on (each device holds its
// own copy, at its own address) and lives until the process ends.  Its
// device address is looked up once per device with hipGetSymbolAddress,
// with that device current; host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in, not a device
// address), always the looked-up pointer.  Every call on a device shares
// that device's array: calls that overlap on one device race.  Nothing in it
// needs clearing: the gradient kernel writes every partial it later reads.
#include <mutex>
#include <string>

#include "ps_internal.h"
#include "ps_plan_impl.h"
#include "../../include/pressure_solve.h"

namespace {

// nz (<= 256) levels times at most 1024 blocks per level, FP64
constexpr size_t kScratchBytes = (size_t)PS_MAX_NZ * 1024 * sizeof(double);
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

// The device address of `scratch` on device dev (looked up on first use).
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return ps::set_error(PS_EUNSUPPORTED, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        const hipError_t r = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess)
            return ps::set_error(PS_EHIP, std::string("hipGetSymbolAddress: ") +
                                              hipGetErrorString(e));
        if (r != hipSuccess)
            return ps::set_error(PS_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(r));
        if (!ptr) return ps::set_error(PS_EHIP, "hipGetSymbolAddress returned NULL");
        g_addr[dev] = ptr;
    }
    *out = g_addr[dev];
    return PS_OK;
}

} // namespace

extern "C" int ps_grad_coeffs_noalloc(ps_plan *p, const void *lam, const void *x, double *grho)
{
    if (!p || !lam || !x || !grho) return ps::set_error(PS_EINVAL, "arguments must not be NULL");
    const size_t need = (size_t)p->nz * (size_t)p->nblk * sizeof(double);
    if (need > kScratchBytes)
        return ps::set_error(PS_EUNSUPPORTED,
                             "the partial sums (" + std::to_string(need) +
                                 " bytes) exceed the fixed no-allocation array (" +
                                 std::to_string(kScratchBytes) + " bytes)");
    void *ptr = nullptr;
    const int rc = scratch_address(p->device, &ptr);
    if (rc != PS_OK) return rc;
    double *partial = static_cast<double *>(ptr);
    hipError_t e;
    if (p->fp64())
        e = ps::launch_grad_rho<double>((const double *)lam, (const double *)x, p->nx, p->ny, p->nz,
                                        p->d_gk, partial, p->nblk, grho, p->stream);
    else
        e = ps::launch_grad_rho<float>((const float *)lam, (const float *)x, p->nx, p->ny, p->nz,
                                       p->d_gk, partial, p->nblk, grho, p->stream);
    if (e != hipSuccess)
        return ps::set_error(PS_EHIP, std::string("launch_grad_rho: ") + hipGetErrorString(e));
    return PS_OK;
}
