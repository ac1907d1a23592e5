// Internal declarations shared by the plan builder, the C-ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace molt {

// Kernel-duration events of mol_profile_step: when set, the next box-sweep
// launch of this thread takes them as its dispatch's start / stop timestamps
// (and clears them), so a duration excludes launch gaps.
struct ProfEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local ProfEvents g_prof;

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
    double w0, w1;      // weights of the I recurrences: J^L_p = w0 v_p + w1 v_{p-1} + w2 (curvature)
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
    int kform[MAXS] = {};  // 1: combination k is swept for L^{-1} (the I recurrences), else D
    // x sweeps of 1D lines with boundary data, one combination.  Dirichlet
    // (bmode = 1): L^{-1} targets and data curvatures (times h^2) at the two
    // ends, and the values the projected outputs take at the end nodes.
    // Neumann (bmode = 2): bt = (S_a, -S_b) / alpha for the slopes S that
    // L^{-1} takes at the ends, bk = 2 h times the slopes of the input
    int bmode = 0;
    double bt[2] = {}, bk[2] = {}, bend[2] = {};
    int proj = 0;        // write 0 on every Dirichlet boundary node of the outputs
    int chain = 0;       // x sweeps: also write D_x(out_0) to buffer ochain
    int ochain = -1;
    // chained strided sweep (yy = 1): v1 = sum mE1 f + D(sum mS[0] f), y = D v1,
    // out_o = sum mOF[o] f + mV[o] v1 + mOD[o][0] y
    int yy = 0;
    double mE1[MAXF] = {};
    double mV[MAXO] = {};
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
// agg: the plan's aggregate table for exact two-pass strided sweeps (may be
// NULL for other configurations).
hipError_t launch_sweep(const SweepOp &op, const Geom &g, const DirCoef &dc, bool fp64,
                        const void *const *fptr, void *const *optr, const int *cfg,
                        hipStream_t st, void *agg = nullptr);
// Exact two-pass strided configurations: the smallest tile they use, whether
// cfg is one, and the bytes of the aggregate table a plan holds for sweeps
// along dir (0 for x).
constexpr int EXACT_MIN_TILE = 64;
bool config_exact(const SweepOp &op, const int *cfg);
size_t exact_agg_bytes(const Geom &g, int dir, bool fp64);

// Per-direction launch configuration chosen by the plan: cfg[0] = variant id.
// Strided sweeps: ids below NSCFG are the tile kernel, the
// rest the pipelined strip kernel.
// Chained strided sweeps have their own configuration ids.
int default_config(const Geom &g, const DirCoef &dc, const SweepOp &op, bool fp64, int *cfg);
bool config_valid(const Geom &g, const DirCoef &dc, const SweepOp &op, bool fp64, const int *cfg);
int config_count(const SweepOp &op);
// Nodes per lane times waves of x configuration id (line capacity / 64).
int uniform_x_capacity(int id);

// Kernel instantiation of one sweep launch: launches with equal keys may run
// as one batched launch over a table of their argument sets.
struct SweepKey {
    int fp64 = 0, cls = 0, cfg = 0, nsno = 0, nfb = 0, periodic = 0;
    bool operator<(const SweepKey &o) const
    {
        const int a[6] = {fp64, cls, cfg, nsno, nfb, periodic};
        const int b[6] = {o.fp64, o.cls, o.cfg, o.nsno, o.nfb, o.periodic};
        for (int i = 0; i < 6; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    }
    bool operator==(const SweepKey &o) const { return !(*this < o) && !(o < *this); }
};
// Bytes of one argument set (host and device layout are the same).
size_t sweep_args_bytes(bool fp64);
// Fills the argument set of one sweep into args (sweep_args_bytes(fp64)
// bytes), its key and its workgroup count; false when cfg is not valid.
bool sweep_prepare(const SweepOp &op, const Geom &g, const DirCoef &dc, bool fp64,
                   const void *const *fptr, void *const *optr, const int *cfg, void *args,
                   SweepKey &key, int64_t &blocks);
// One launch of nent argument sets sharing key: d_tab holds them in device
// memory, d_first their first workgroups (nent + 1 values, ascending from 0 to
// blocks).
hipError_t launch_sweep_batch(const SweepKey &key, const void *d_tab, const int64_t *d_first, int nent,
                              int64_t blocks, hipStream_t st);

// Elementwise a*x + b*y -> z on n values (state conversion for the increment form).
hipError_t launch_axpby(bool fp64, int64_t n, double a, const void *x, double b, const void *y,
                        void *z, hipStream_t st);

// ---- embedded boundary (2D masked) line objects (Sec. 4.3) ----
// One record per line object: the inside nodes base + j*pstride, j < m, of one
// grid line, closed by boundary points theta_lo*h before the first and
// theta_hi*h after the last inside node.  The FP64 constants give the forcing
// of the end cells (E = I - v/2 form), the end values I^R and I^L at the two
// boundary points, and the 2x2 closure:
//   first node   F^L = AL0 v0 + AL1 v1,  F^R = AR0 v0 + AR1 v1
//   last node    F^L = BL0 v_{m-2} + BL1 v_{m-1},  F^R = BR0 v_{m-2} + BR1 v_{m-1}
//   (m = 1: F^L = AL0 v0, F^R = AR0 v0)
//   I^R(a) = EA E^R_0 + QA v0,  I^L(b) = EB E^L_{m-1} + QB v_{m-1}
//   A = (-I^R(a) + MU I^L(b)) INV,  B = (-I^L(b) + MU I^R(a)) INV
//   D v_j = -(E^L_j + E^R_j + A EA d^j + B EB d^{m-1-j})
enum {
    SEG_AL0, SEG_AL1, SEG_AR0, SEG_AR1, SEG_EA, SEG_QA,
    SEG_BL0, SEG_BL1, SEG_BR0, SEG_BR1, SEG_EB, SEG_QB,
    SEG_MU, SEG_INV, NSEGC
};
struct SegRec {
    int64_t base;   // element offset of the first inside node
    int32_t m;      // inside nodes, >= 1
    int32_t cls;    // length class
    double c[NSEGC];
};
// length classes: one workgroup of 64*WPL lanes x S nodes per line object
constexpr int NSEGCLS = 6;
int seg_class_capacity(int cls);
struct SegTable {
    int64_t nseg = 0;
    int64_t pstride = 1;                  // element stride along the line
    int64_t cls_begin[NSEGCLS + 1] = {};  // records [cls_begin[c], cls_begin[c+1]) have class c
    SegRec *d_rec = nullptr;              // device copy
};

// All line objects of one direction (every class), one launch per class.
hipError_t launch_seg_sweep(const SweepOp &op, const SegTable &tab, const DirCoef &dc, bool fp64,
                            const void *const *fptr, void *const *optr, hipStream_t st);
// out = transpose of the R x C array in (C x R); with d_mask (of out's
// layout) the outside nodes of out are written as 0
hipError_t launch_transpose(bool fp64, const void *in, void *out, int64_t R, int64_t C,
                            const unsigned char *d_mask, hipStream_t st);
// the same for nt (1..4) pairs in[i] -> out[i] of one shape, in one launch
// where every array allows 16-byte accesses
hipError_t launch_transpose_n(bool fp64, int nt, const void *const *in, void *const *out, int64_t R,
                              int64_t C, const unsigned char *d_mask, hipStream_t st);
// out[i] = 0 where mask[i] == 0 (outside nodes of a user-visible output)
hipError_t launch_mask_zero(bool fp64, int64_t n, const unsigned char *d_mask, void *out,
                            hipStream_t st);

}  // namespace molt
