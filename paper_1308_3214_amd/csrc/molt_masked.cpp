// Embedded-boundary (masked 2D) plans: line objects of Sec. 4.3.
#include <hip/hip_runtime.h>

#include <string>

#include "molt_program.h"

namespace molt {

mol_status masked_tables(mol_plan_ *pl, bool dry, std::string &err)
{
    (void)pl;
    (void)dry;
    err = "embedded boundaries are not built yet";
    return MOL_E_UNSUPPORTED;
}

void masked_free(mol_plan_ *pl) { (void)pl; }

bool build_rhs_masked(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo)
{
    (void)prog; (void)u; (void)fo;
    b.err = "embedded boundaries are not built yet";
    return false;
}

bool build_apply_masked(Builder &b, Program &prog, int op)
{
    (void)prog; (void)op;
    b.err = "embedded boundaries are not built yet";
    return false;
}

hipError_t launch_seg_op(const SweepOp &op, const mol_plan_ *pl, const void *const *fptr,
                         void *const *optr, hipStream_t st)
{
    (void)op; (void)pl; (void)fptr; (void)optr; (void)st;
    return hipErrorNotSupported;
}

}  // namespace molt
