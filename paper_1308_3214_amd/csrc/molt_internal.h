// Internal declarations shared by the plan builder, the C-ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace molt {

constexpr int MAXF = 16;  // fields loaded by one launch
constexpr int MAXS = 2;   // swept combinations per launch
constexpr int MAXO = 3;   // outputs per launch

// Per-direction constants of the uniform-cell quadrature (all FP64, from the plan).
//   d  = e^{-nu},  g = (1 - d)/(2 nu),  w2 = curvature weight
// so that with E = I - v/2 (I = I^L or I^R):
//   E^L_p = d E^L_{p-1} + w2 (v_{p+1} - 2 v_p + v_{p-1}) - g (v_p - v_{p-1})
//   E^R_p = d E^R_{p+1} + w2 (v_{p+1} - 2 v_p + v_{p-1}) + g (v_{p+1} - v_p)
//   D v_p = -(E^L_p + E^R_p + A d^p + B d^{M-p})
// and [A, B] = K [E^R_0, E^L_M] (Dirichlet or periodic closure).
struct DirCoef {
    double nu, d, g, w2;
    double K[2][2];
    int periodic;
    int64_t n;          // nodes on the line
    int halo;           // rows of halo needed for relative truncation <= tol
};

// One launch of a directional sweep with a linear prologue and epilogue:
//   s_k   = sum_f mS[k][f]  F_f                     (swept combinations)
//   out_o = sum_f mOF[o][f] F_f + sum_k mOD[o][k] D_dir(s_k)
struct SweepOp {
    int dir = 0;
    int nf = 0, ns = 0, no = 0;
    int f[MAXF] = {};
    int o[MAXO] = {};
    double mS[MAXS][MAXF] = {};
    double mOF[MAXO][MAXF] = {};
    double mOD[MAXO][MAXS] = {};
    int proj = 0;        // write 0 on every Dirichlet boundary node of the outputs
    int chain = 0;       // x sweeps: also write D_x(out_0) to buffer ochain
    int ochain = -1;
};

// Geometry of a full box grid (x fastest).
struct Geom {
    int ndim;
    int64_t n[3];
    int dirichlet[3];
};

// Launch one sweep.  ptrs: resolved device pointers for op.f / op.o (followed
// by the chained output when op.chain is set).
// Returns hipSuccess or the launch error.
hipError_t launch_sweep(const SweepOp &op, const Geom &g, const DirCoef &dc, bool fp64,
                        const void *const *fptr, void *const *optr, const int *cfg,
                        hipStream_t st);

// Per-direction launch configuration chosen by the plan: cfg[0] = variant id.
// Strided sweeps: ids below config_count_tiled() are the tile kernel, the
// rest the pipelined strip kernel.
int default_config(const Geom &g, const DirCoef &dc, int dir, bool fp64, int nf, int ns, int no,
                   int *cfg);
bool config_valid(const Geom &g, const DirCoef &dc, int dir, bool fp64, int nf, int ns, int no,
                  const int *cfg);
int config_count(int dir);

// Elementwise a*x + b*y -> z on n values (state conversion for the increment form).
hipError_t launch_axpby(bool fp64, int64_t n, double a, const void *x, double b, const void *y,
                        void *z, hipStream_t st);

// ---- embedded boundary (2D masked) line objects ----
struct SegTable {
    int64_t nseg = 0;
    int64_t *d_idx = nullptr;     // [nseg][4]: line, first inside node, count, pad
    double *d_coef = nullptr;     // [nseg][NSEGCOEF] FP64 per-segment constants
};
constexpr int NSEGCOEF = 16;

hipError_t launch_seg_sweep(const SweepOp &op, const Geom &g, int dir, const SegTable &tab,
                            const DirCoef &dc, bool fp64, const void *const *fptr,
                            void *const *optr, const unsigned char *d_mask, hipStream_t st);

}  // namespace molt
