// Pipelined strided-sweep kernels, double, 4 field(s) per sub-tile.
#define MOLT_T double
#define MOLT_TAG f64
#define MOLT_NFP 4
#include "molt_sweep_p.inc"
