// Pipelined strided-sweep kernels, float, 4 field(s) per sub-tile.
#define MOLT_T float
#define MOLT_TAG f32
#define MOLT_NFP 4
#include "molt_sweep_p.inc"
