// Chained strided-sweep kernels (two levels of the strided sweep in one strip
// walk), float, three fields per sub-tile; one argument set or a batched
// table of them (BatchTab).
#include "molt_sweep.h"

namespace molt {
namespace {
template <int S, int W, int NO>
hipError_t run_yy(const KArgs<float> &k, const BatchTab *bt, hipStream_t st)
{
    if (bt) {
        const KArgs<float> *tab = static_cast<const KArgs<float> *>(bt->tab);
        if (k.periodic)
            launch_k((k_sweep_yy_b<float, S, W, NO, true, 3>), dim3((unsigned)bt->blocks), dim3(64 * W),
                     0, st, tab, bt->first, bt->nent);
        else
            launch_k((k_sweep_yy_b<float, S, W, NO, false, 3>), dim3((unsigned)bt->blocks), dim3(64 * W),
                     0, st, tab, bt->first, bt->nent);
        return hipGetLastError();
    }
    if (k.periodic)
        launch_k((k_sweep_yy<float, S, W, NO, true, 3>), dim3((unsigned)k.nblocks), dim3(64 * W), 0,
                 st, k);
    else
        launch_k((k_sweep_yy<float, S, W, NO, false, 3>), dim3((unsigned)k.nblocks), dim3(64 * W), 0,
                 st, k);
    return hipGetLastError();
}

template <int NO>
hipError_t dispatch_yy(const KArgs<float> &k, int id, const BatchTab *bt, hipStream_t st)
{
    static_assert(NYCFG == 5, "chained configuration table and dispatch out of step");
    switch (id) {
    case 0: return run_yy<kYCfg[0].S, kYCfg[0].W, NO>(k, bt, st);
    case 1: return run_yy<kYCfg[1].S, kYCfg[1].W, NO>(k, bt, st);
    case 2: return run_yy<kYCfg[2].S, kYCfg[2].W, NO>(k, bt, st);
    case 3: return run_yy<kYCfg[3].S, kYCfg[3].W, NO>(k, bt, st);
    case 4: return run_yy<kYCfg[4].S, kYCfg[4].W, NO>(k, bt, st);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t dispatch_yy_f32(const KArgs<float> &k, int no, int id, const BatchTab *bt, hipStream_t st)
{
    switch (no) {
    case 1: return dispatch_yy<1>(k, id, bt, st);
    case 2: return dispatch_yy<2>(k, id, bt, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace molt
