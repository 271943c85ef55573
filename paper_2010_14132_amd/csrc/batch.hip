// Batched solves (placeholders until implemented).
#include "ps_internal.h"
#include "../../include/pressure_solve.h"

extern "C" int ps_batch_create(ps_batch **out, int count, const int *nx, const int *ny,
                               const int *nz, const double *dx, const double *dy,
                               const double *const *dz, const double *const *rho, int precision,
                               void *stream)
{
    (void)count; (void)nx; (void)ny; (void)nz; (void)dx; (void)dy; (void)dz; (void)rho;
    (void)precision; (void)stream;
    if (out) *out = nullptr;
    return PS_EUNSUPPORTED;
}
extern "C" int ps_batch_solve(ps_batch *batch, const void *const *rhs, void *const *p)
{
    (void)batch; (void)rhs; (void)p;
    return PS_EUNSUPPORTED;
}
extern "C" int ps_batch_destroy(ps_batch *batch)
{
    (void)batch;
    return PS_OK;
}
