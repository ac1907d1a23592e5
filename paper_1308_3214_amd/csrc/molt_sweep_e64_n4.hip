// Exact two-pass strided-sweep kernels, double, field loop bound 4.
#define MOLT_T double
#define MOLT_TAG f64
#define MOLT_NFMAX 4
#include "molt_sweep_e.inc"
