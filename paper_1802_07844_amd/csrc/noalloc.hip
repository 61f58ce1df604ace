// Allocation-free evaluation: ewald_halfspace_noalloc.
//
// For callers that cannot allocate device memory during a call (serving
// loops with a fixed memory budget, harnesses that forbid hipMalloc).  Every
// buffer of the evaluation -- stage tables, truncated-kernel octants of one
// grid size, grids, cell lists, sort scratch -- comes from one file-scope
// device array, `scratch`, of EHS_NOALLOC_SCRATCH_BYTES.  Each device the
// library runs on holds its own copy of the array until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): at context creation, with the device
// current, hipGetSymbolAddress resolves the device address once per device,
// and only that pointer is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ehs.h"
#include "ctx.h"

static __device__ __align__(256) unsigned char scratch[EHS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    ehs::Fixed fx;        // region = the device's copy of `scratch`
    bool attached = false;
};

std::mutex g_attach_mu;
DeviceScratch g_dev[MAX_DEVICES];

}  // namespace

int ehs::noalloc_attach(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return EHS_EINVAL;
    std::lock_guard<std::mutex> lk(g_attach_mu);
    DeviceScratch& d = g_dev[device];
    if (d.attached) return EHS_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        hipGetLastError();
        return EHS_EHIP;
    }
    d.fx.base = static_cast<char*>(ptr);
    d.fx.bytes = EHS_NOALLOC_SCRATCH_BYTES;
    d.fx.tables.arena = d.fx.base;
    d.fx.tables.cap = FIXED_TABLE_BYTES;
    d.attached = true;
    return EHS_OK;
}

extern "C" int ewald_halfspace_noalloc(ehs_ctx* ctx, int family, const double* sources, const double* strengths,
                                       int64_t N, const double* targets, int64_t T, double xi, double r_c,
                                       double tol, double* u_out, void* stream, ehs_report* rep)
{
    if (!ctx || family < EHS_STOKESLET || family > EHS_ROTLET) return EHS_EINVAL;
    int dev = ctx->device;
    if (dev < 0 || dev >= MAX_DEVICES) return EHS_EINVAL;
    ehs::Fixed* fx = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_attach_mu);
        if (g_dev[dev].attached) fx = &g_dev[dev].fx;
    }
    if (!fx) return EHS_EHIP;  // the context's creation resolves the scratch address
    return ehs::evaluate_fixed(ctx, fx, family, sources, strengths, N, targets, T, xi, r_c, tol, u_out, stream, rep,
                               EHS_ETOOBIG);
}
