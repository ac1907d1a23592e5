// strided-sweep kernels, float, field loop bound 16.
#define MOLT_NFMAX 16
#include "molt_sweep_s32.inc"
