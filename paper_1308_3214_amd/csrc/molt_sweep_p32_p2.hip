// Pipelined strided-sweep kernels, float, 2 field(s) per sub-tile.
#define MOLT_T float
#define MOLT_TAG f32
#define MOLT_NFP 2
#include "molt_sweep_p.inc"
