// mol_step_static: one step of a box-grid plan that allocates no device
// memory.  The step's workspace fields live in one file-scope device array
// (`scratch`, a fixed size), shared by every call on a GPU; each device holds
// its own copy of the array, whose address is looked up once per device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <new>

#include "../../include/molt.h"
#include "molt_internal.h"
#include "molt_program.h"

using namespace molt;

static constexpr size_t MOL_STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[MOL_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on the current device, looked up on
// the first call with that device current.  The array's name is a host-side
// stand-in: only this address reaches kernels.
mol_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_err(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES)
        return set_error(MOL_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return dev_err(e, "hipGetSymbolAddress of the scratch array");
        if (!p) return set_error(MOL_E_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MOL_OK;
}

// workspace fields a program uses: 1 + the largest workspace buffer id
int program_ws_fields(const Program &prog)
{
    int m = 0;
    auto see = [&](int b) {
        if (b >= B_WS0) m = std::max(m, b - B_WS0 + 1);
    };
    for (const ProgOp &po : prog) {
        for (int i = 0; i < po.op.nf; ++i) see(po.op.f[i]);
        for (int i = 0; i < po.op.no; ++i) see(po.op.o[i]);
        if (po.op.chain) see(po.op.ochain);
    }
    return m;
}

}  // namespace

extern "C" {

size_t mol_step_static_max_bytes(void) { return MOL_STATIC_SCRATCH_BYTES; }

mol_status mol_step_static(const mol_desc *desc, const void *u_prev, const void *u_curr, void *u_next,
                           void *stream)
{
    if (!desc || !u_prev || !u_curr || !u_next) return set_error(MOL_E_INVALID, "NULL argument");
    if (u_next == u_curr) return set_error(MOL_E_INVALID, "u_next must not overlap u_curr");
    if (desc->mask) return set_error(MOL_E_UNSUPPORTED, "mol_step_static takes box grids (no mask)");
    mol_plan_ *pl = new (std::nothrow) mol_plan_();
    if (!pl) return set_error(MOL_E_NOMEM, "host allocation failed");
    // the schedule and launch configurations of mol_plan_create's plan, with
    // no device allocation (box grids have no device tables)
    mol_status s = build_plan(desc, pl, false);
    if (s == MOL_OK) {
        const int nf = program_ws_fields(pl->step);
        const size_t field = ((size_t)pl->npts * pl->es + 255) / 256 * 256;
        const size_t aggb = (pl->agg_bytes + 255) / 256 * 256;
        const size_t need = (size_t)nf * field + aggb;
        void *base = nullptr;
        if (need > MOL_STATIC_SCRATCH_BYTES) {
            char buf[200];
            snprintf(buf, sizeof buf,
                     "mol_step_static: this step needs %zu bytes of workspace (%d fields and a "
                     "%zu-byte carry table), the static scratch holds %zu",
                     need, nf, aggb, MOL_STATIC_SCRATCH_BYTES);
            s = set_error(MOL_E_INVALID, buf);
        } else if ((s = scratch_address(&base)) == MOL_OK) {
            pl->ws.assign(pl->nws, nullptr);
            for (int i = 0; i < nf; ++i) pl->ws[i] = static_cast<unsigned char *>(base) + (size_t)i * field;
            // the aggregate table of exact strided sweeps after the fields
            if (aggb) pl->agg = static_cast<unsigned char *>(base) + (size_t)nf * field;
            (void)hipGetDevice(&pl->dev);
            const hipError_t e = run_program(pl, pl->step, u_prev, u_curr, u_next, nullptr, nullptr,
                                             (hipStream_t)stream);
            if (e != hipSuccess) s = dev_err(e, "mol_step_static");
        }
    }
    pl->ws.clear();            // the scratch array is not the plan's to free
    pl->agg = nullptr;
    free_plan(pl);
    return s;
}

}  // extern "C"
