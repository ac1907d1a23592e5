// Pipelined strided-sweep kernels, float, 1 field(s) per sub-tile.
#define MOLT_T float
#define MOLT_TAG f32
#define MOLT_NFP 1
#include "molt_sweep_p.inc"
