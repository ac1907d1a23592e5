// x-sweep kernels, double, field loop bound 16.
#define MOLT_NFMAX 16
#include "molt_sweep_x64.inc"
