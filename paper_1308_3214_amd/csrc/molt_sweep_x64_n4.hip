// x-sweep kernels, double, field loop bound 4.
#define MOLT_NFMAX 4
#include "molt_sweep_x64.inc"
