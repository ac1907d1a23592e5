// Exact two-pass strided-sweep kernels, float, field loop bound 16.
#define MOLT_T float
#define MOLT_TAG f32
#define MOLT_NFMAX 16
#include "molt_sweep_e.inc"
