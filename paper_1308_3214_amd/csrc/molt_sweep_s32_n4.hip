// strided-sweep kernels, float, field loop bound 4.
#define MOLT_NFMAX 4
#include "molt_sweep_s32.inc"
