// Directional sweep kernels for gfx950 (templates; instantiated in molt_sweep_*.hip): the O(N) recursive convolution
// L_gamma^{-1} (Sec. 2: characteristic split I^L + I^R, each an exponential
// recurrence with decay e^{-alpha h}, local integrals over one cell against the
// quadratic through three nodes, then the boundary correction
// A e^{-alpha(x-a)} + B e^{-alpha(b-x)}) applied along x, y or z lines, with
// D_gamma = 1 - L_gamma^{-1} (Sec. 4, eq. LD_gam) emitted directly.
//
// Formulation used on the device.  With E = I - v/2 the recurrences are forced
// only by differences of the data,
//   E^L_p = d E^L_{p-1} + w2 (v_{p+1} - 2 v_p + v_{p-1}) - g (v_p - v_{p-1}),
//   E^R_p = d E^R_{p+1} + w2 (v_{p+1} - 2 v_p + v_{p-1}) + g (v_{p+1} - v_p),
//   D v_p = -(E^L_p + E^R_p + A d^p + B d^{M-p}),
// (d = e^{-nu}, g = (1-d)/(2 nu), nu = alpha h), which is the same discrete
// operator as I^L + I^R (exact in real arithmetic) but never forms v - L^{-1} v,
// so D keeps full relative precision in FP32.  At a Dirichlet end node the
// curvature term is dropped (the data's curvature there is 0 for homogeneous
// boundary values, Sec. 3.2).
//
// Each launch computes up to MAXS swept combinations s_k = sum_f mS[k][f] F_f
// of up to MAXF loaded fields and writes up to MAXO outputs
// out_o = sum_f mOF[o][f] F_f + sum_k mOD[o][k] D(s_k): the ADI compositions
// (eqs. C_def_ADI, D_def_ADI, ...) and the time update are fused this way.
//
// x lines (contiguous): one workgroup per line, the line staged through LDS
// (coalesced vector loads, padded to avoid bank conflicts), every lane runs
// the recurrences over S consecutive nodes, lane carries are combined by a
// wave-level scan of the linear recurrence (multiplier d^S) and waves through
// LDS: exact.
//
// y / z lines (strided): lanes own consecutive columns (coalesced rows), waves
// of a workgroup stack along the line, each lane runs S nodes, wave carries
// are scanned through LDS.  Lines longer than one tile of W*S nodes are split
// into tiles; the carry entering a tile is the truncated sum over a halo of
// K nodes with d^K below the dtype's rounding (the exponential decay of the
// Green's function), computed cooperatively by all waves of the tile.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>

#include "molt_internal.h"

namespace molt {

template <typename... A, typename F>
inline void launch_k(F fn, dim3 grid, dim3 block, size_t shmem, hipStream_t st, A... args)
{
    if (g_prof.start || g_prof.stop) {
        hipExtLaunchKernelGGL(fn, grid, block, (std::uint32_t)shmem, st, g_prof.start, g_prof.stop, 0u,
                              args...);
        g_prof = ProfEvents{};
    } else {
        hipLaunchKernelGGL(fn, grid, block, shmem, st, args...);
    }
}

template <typename T>
struct KArgs {
    const T *f[MAXF];
    T *o[MAXO];
    T mS[MAXS][MAXF];
    T mOF[MAXO][MAXF];
    T mOD[MAXO][MAXS];
    int nf;
    int proj;
    int chain;        // x: also write D_x(out_0) to ochain (next sweep of out_0)
    T *ochain;
    int64_t n;        // nodes per line
    int64_t nlines;   // x: lines; strided: columns (x extent)
    int64_t lineoff;  // x: element offset between lines
    int64_t ls;       // strided: stride between nodes of a line
    int64_t os;       // strided: stride of the outer index
    int64_t nouter;   // strided: outer extent
    int64_t nblocks;  // strided: total workgroups (XCD remap)
    int ntiles;       // strided: tiles per line
    int halo;         // strided: halo nodes per side
    int aligned;      // x: vector loads allowed
    int periodic;     // along the sweep
    T d, g, w2;
    T gw;             // g + w2
    T w0, w1;         // weights of the I recurrences (combinations swept for L^{-1})
    int kform[MAXS];  // 1: combination k is swept for L^{-1} (I recurrences), else D
    T dS;             // d^S
    T dBlk;           // x: d^{64 S} (one wave of lanes)
    T dpw[6];         // x: d^{S 2^i}, i < 6 (the lane scan's multipliers)
    double nu;
    double K00, K01, K10, K11;
    // projection: line index = (i1 in [0,pn1), i2 in [0,pn2)); Dirichlet flags
    int64_t pn1, pn2;
    int pd1, pd2;
    // chained strided sweeps: field terms of the first-level result v1, weight
    // of v1 in each output, rows of data next to a strip in its walk
    T mE1[MAXF];
    T mV[MAXO];
    int roll;
    // fold of output 0 into the second-level sums: ykv = mV[0] / mOD[0][0],
    // yk0 = 1 / mOD[0][0] (field terms of a single output), ykh = mV[1] -
    // mOD[1][0] mV[0] / mOD[0][0] (weight of v1 left in output 1)
    T ykv, yk0, ykh;
    // exact two-pass strided sweeps: per-tile aggregates (device table of
    // nouter x column groups x ntiles x MAXS x 3 x 64 values)
    T *agg;
    int tile_rows;    // exact sweeps: rows per tile (W S)
    // x sweeps of a line with boundary data.  bmode = 1 (Dirichlet): the
    // L^{-1} targets at the two ends, the data's curvature there times h^2,
    // and the values the outputs take at the end nodes when projected.
    // bmode = 2 (Neumann): bt = (S_a, -S_b) / alpha from the slopes S of
    // L^{-1} at the ends, bk = 2 h times the slopes of the input there
    int bmode;
    T bt[2], bk[2], bend[2];
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_remap(int64_t i, int64_t N)
{
    // Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
    // contiguous range of logical tiles so that neighbouring tiles of a line
    // (which read each other's halo) share one L2.
    const int64_t X = 8;
    int64_t x = i % X, local = i / X;
    int64_t per = N / X, rem = N % X;
    return x * per + (x < rem ? x : rem) + local;
}

// Batched launches: the workgroups of entry e of a table of argument sets are
// [first[e], first[e+1]); first[0] = 0, ascending.  Returns the entry of
// workgroup b (the last e with first[e] <= b; always in [0, nent)).
__device__ __forceinline__ int batch_entry(const int64_t *__restrict__ first, int nent, int64_t b)
{
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int C>
struct ic {
    static constexpr int value = C;
};

// Calls body(f0, ic<c>{}) over the fields [0, nf) in chunks of c <= CH fields
// (c static): each chunk issues all of its loads before it uses any of them.
template <int CH, int NFMAX, typename F>
__device__ __forceinline__ void field_chunks(int nf, F &&body)
{
    static_assert(CH >= 1 && CH <= 4, "chunk of 1..4 fields");
    if constexpr (NFMAX <= 4) {
#pragma unroll
        for (int f0 = 0; f0 < NFMAX; f0 += CH) {
            const int left = nf - f0;
            if (left <= 0) break;
            if constexpr (CH >= 4) { if (left >= 4) { body(f0, ic<4>{}); continue; } }
            if constexpr (CH >= 3) { if (left == 3) { body(f0, ic<3>{}); continue; } }
            if constexpr (CH >= 2) { if (left >= 2) { body(f0, ic<2>{}); continue; } }
            body(f0, ic<1>{});
        }
    } else {
        for (int f0 = 0; f0 < nf; f0 += CH) {
            const int left = nf - f0;
            if constexpr (CH >= 4) { if (left >= 4) { body(f0, ic<4>{}); continue; } }
            if constexpr (CH >= 3) { if (left == 3) { body(f0, ic<3>{}); continue; } }
            if constexpr (CH >= 2) { if (left >= 2) { body(f0, ic<2>{}); continue; } }
            body(f0, ic<1>{});
        }
    }
}

// Lane moves through DPP (data-parallel primitives on the VALU, no LDS):
// CTRL 0x111+n / 0x101+n = row shift right / left by n inside rows of 16
// lanes, 0x138 / 0x130 = whole-wave shift right / left by one, 0x142 / 0x143
// = lane 15 / lane 31 broadcast into the rows that ROWM enables.  Lanes
// without a source (and lanes of disabled rows) read 0.
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWM,
                                                                 0xf, false));
}
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ double dpp_mov(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWM, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWM, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float lane_read(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_read(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// A row of zeros in device memory.  Loads of nodes that read as 0 (outside a
// line, Dirichlet end rows of a halo) are pointed here instead of being
// predicated: every load is issued unconditionally, so a wave keeps all of its
// loads in flight at once.
__device__ double kZeroRow[64] = {};   // never written
template <typename T>
__device__ __forceinline__ const T *zero_row()
{
    return reinterpret_cast<const T *>(kZeroRow);
}

// Raw buffer access: a 128-bit resource (base, size in bytes) and a 32-bit
// per-lane byte offset.  The hardware range check on that offset returns 0 for
// reads beyond the resource (negative offsets included) and drops such writes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int voff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, 0, 0);
}
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, 0, 0);
}

// e^{-x} for x >= 0 in the kernel's precision: FP32 kernels use the hardware
// base-2 exponential (about 1 ulp), FP64 kernels the FP64 library exp.
template <typename T>
__device__ __forceinline__ T expneg(double x);
template <>
__device__ __forceinline__ float expneg<float>(double x)
{
    return exp2f((float)(-x * 1.4426950408889634));
}
template <>
__device__ __forceinline__ double expneg<double>(double x)
{
    return exp(-x);
}

// Weights of the lane scans below for a lane with multiplier m = d^S per lane:
// wA = m^(j+1) (from the last lane of the row above), wB = m^(l-31) for rows 2
// and 3 (from lane 31), wR = m^(16-j) (from the first lane of the row below);
// l = lane, j = l mod 16.  Each rounded once from FP64 arguments.
template <typename T>
struct LaneW {
    T wA, wB, wR;
};
template <typename T>
__device__ __forceinline__ LaneW<T> lane_weights(double nuS, int lane)
{
    const int j = lane & 15;
    LaneW<T> w;
    w.wA = expneg<T>(nuS * (double)(j + 1));
    w.wB = expneg<T>(nuS * (double)(lane >= 32 ? lane - 31 : j + 1));
    w.wR = expneg<T>(nuS * (double)(16 - j));
    return w;
}

// Weighted inclusive scans over the 64 lanes of a wave, in place:
// xl_l = sum_{k <= l} m^(l-k) x_k and xr_l = sum_{k >= l} m^(k-l) x_k, m = d^S;
// dpw[i] = m^(2^i).  Row shifts by 1, 2, 4, 8 scan each row of 16 lanes;
// forward, the row ends are then broadcast into the rows below; backward, the
// row heads are read into scalars and their carries formed there.
template <typename T>
__device__ __forceinline__ void lane_scans(T &xl, T &xr, const T *dpw, const LaneW<T> &w, int lane)
{
    xl += dpw[0] * dpp_mov<0x111>(xl);
    xr += dpw[0] * dpp_mov<0x101>(xr);
    xl += dpw[1] * dpp_mov<0x112>(xl);
    xr += dpw[1] * dpp_mov<0x102>(xr);
    xl += dpw[2] * dpp_mov<0x114>(xl);
    xr += dpw[2] * dpp_mov<0x104>(xr);
    xl += dpw[3] * dpp_mov<0x118>(xl);
    xr += dpw[3] * dpp_mov<0x108>(xr);
    xl += w.wA * dpp_mov<0x142, 0xa>(xl);       // rows 1, 3 from lanes 15, 47
    xl += w.wB * dpp_mov<0x143, 0xc>(xl);       // rows 2, 3 from lane 31
    const T m16 = dpw[4];
    const T q2 = lane_read(xr, 48);
    const T q1 = lane_read(xr, 32) + m16 * q2;
    const T q0 = lane_read(xr, 16) + m16 * q1;
    const int r = lane >> 4;
    const T q = (r == 0) ? q0 : (r == 1) ? q1 : (r == 2) ? q2 : T(0);
    xr += w.wR * q;
}

// Forcing of the two recurrences at node p from its neighbours vm, v0, vp
// (end and outside nodes already read as 0).  Dirichlet end nodes drop the
// curvature term; E^L starts at node 0 and E^R at node M.
template <typename T>
__device__ __forceinline__ T force_L(T vm, T v0, T vp, int p, int M, bool dir_end, T g, T w2)
{
    if (dir_end) {
        if (p <= 0 || p > M) return T(0);
        if (p == M) return -g * (v0 - vm);
    } else if (p > M) {
        return T(0);
    }
    return w2 * ((vp - v0) - (v0 - vm)) - g * (v0 - vm);
}
template <typename T>
__device__ __forceinline__ T force_R(T vm, T v0, T vp, int p, int M, bool dir_end, T g, T w2)
{
    if (dir_end) {
        if (p < 0 || p >= M) return T(0);
        if (p == 0) return g * (vp - v0);
    } else if (p > M) {
        return T(0);
    }
    return w2 * ((vp - v0) - (v0 - vm)) + g * (vp - v0);
}

// Local recurrences over S nodes p0..p0+S-1 from the values v[0..S+1] of
// nodes p0-1..p0+S.  sum[j] = local E^L + local E^R (zero carry-in at both
// segment ends); aL = local E^L at the last node, aR = local E^R at the first
// node, eLM = local E^L at node M if this segment holds it.
template <typename T, int S>
__device__ __forceinline__ void seg_recur(const T (&v)[S + 2], int p0, int M, bool dir_end, T d,
                                          T g, T w2, T (&sum)[S], T &aL, T &aR, T &eLM)
{
    T e = T(0);
    eLM = T(0);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        e = d * e + force_L(v[j], v[j + 1], v[j + 2], p, M, dir_end, g, w2);
        sum[j] = e;
        if (p == M) eLM = e;
    }
    aL = e;
    e = T(0);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        e = d * e + force_R(v[j], v[j + 1], v[j + 2], p0 + j, M, dir_end, g, w2);
        sum[j] += e;
    }
    aR = e;
}

// In place: sum[j] <- D_j = -(sum[j] + d^{j+1} cL + d^{S-j} cR + A d^p + B d^{M-p}),
// p = p0 + j; zero beyond the line and at Dirichlet end nodes.  A, B in FP64.
template <typename T, int S>
__device__ __forceinline__ void seg_close(T (&sum)[S], T cL, T cR, double A, double B, int p0,
                                          int M, double nu, T d, bool dir_end)
{
    const double dd = exp(-nu);
    double ta = (A != 0.0) ? A * exp(-nu * (double)p0) : 0.0;
    T ldec = d * cL;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        sum[j] += (T)ta + ldec;
        ta *= dd;
        ldec *= d;
    }
    const int rem = M - p0;
    const int jmax = (rem >= S - 1) ? (S - 1) : rem;
    double tb = (B != 0.0 && jmax >= 0) ? B * exp(-nu * (double)(rem - jmax)) : 0.0;
    T rdec = cR;
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        rdec *= d;
        sum[j] += rdec;
        if (j <= jmax) {
            sum[j] += (T)tb;
            tb *= dd;
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        sum[j] = (p > M || (dir_end && (p == 0 || p == M))) ? T(0) : -sum[j];
    }
}

// Branch-free recurrences for a segment whose nodes are all interior nodes of
// a Dirichlet line or of a periodic line (values outside the line read as 0).
// With dl_j = v_j - v_{j-1}:  F^L_j = w2 dl_{j+1} - (g + w2) dl_j,
// F^R_j = (g + w2) dl_{j+1} - w2 dl_j.
template <typename T, int S>
__device__ __forceinline__ void seg_recur_fast(const T (&v)[S + 2], T d, T gw, T w2, T (&sum)[S],
                                               T &aL, T &aR)
{
    T dl[S + 1];
#pragma unroll
    for (int j = 0; j <= S; ++j) dl[j] = v[j + 1] - v[j];
    T e = T(0);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        e = d * e + (w2 * dl[j + 1] - gw * dl[j]);
        sum[j] = e;
    }
    aL = e;
    e = T(0);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        e = d * e + (gw * dl[j + 1] - w2 * dl[j]);
        sum[j] += e;
    }
    aR = e;
}

// The recurrences of I^L and I^R themselves (a combination swept for
// L^{-1} = 1 - D, whose values are small where D is close to 1: formed from D
// they would lose the digits D and the data share).  Forcing by the local
// integrals J^L_j = w0 v_j + w1 v_{j-1} + w2 (v_{j+1} - 2 v_j + v_{j-1}) and
// J^R_j = w0 v_j + w1 v_{j+1} + w2 (...), w0 = 1/2 - g, w1 = g - d/2.  The
// Dirichlet end fix-ups of the D form apply unchanged (same curvature term),
// and the closure is the same linear map of the end values; the kernel
// returns -(sums + carries + closure), which the host's output weights negate.
template <typename T, int S>
__device__ __forceinline__ void seg_recur_fast_I(const T (&v)[S + 2], T d, T w0, T w1, T w2, T (&sum)[S],
                                                 T &aL, T &aR)
{
    T e = T(0);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const T cv = (v[j + 2] - v[j + 1]) - (v[j + 1] - v[j]);
        e = d * e + (w0 * v[j + 1] + w1 * v[j] + w2 * cv);
        sum[j] = e;
    }
    aL = e;
    e = T(0);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        const T cv = (v[j + 2] - v[j + 1]) - (v[j + 1] - v[j]);
        e = d * e + (w0 * v[j + 1] + w1 * v[j + 2] + w2 * cv);
        sum[j] += e;
    }
    aR = e;
}
// The same for a periodic segment that crosses the line end (nodes beyond M
// force nothing; values already wrapped).
template <typename T, int S>
__device__ __forceinline__ void seg_recur_I(const T (&v)[S + 2], int p0, int M, T d, T w0, T w1, T w2,
                                            T (&sum)[S], T &aL, T &aR, T &eLM)
{
    T e = T(0);
    eLM = T(0);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        const T cv = (v[j + 2] - v[j + 1]) - (v[j + 1] - v[j]);
        e = d * e + ((p > M) ? T(0) : (w0 * v[j + 1] + w1 * v[j] + w2 * cv));
        sum[j] = e;
        if (p == M) eLM = e;
    }
    aL = e;
    e = T(0);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        const int p = p0 + j;
        const T cv = (v[j + 2] - v[j + 1]) - (v[j + 1] - v[j]);
        e = d * e + ((p > M) ? T(0) : (w0 * v[j + 1] + w1 * v[j + 2] + w2 * cv));
        sum[j] += e;
    }
    aR = e;
}

// Dirichlet end nodes inside a segment handled by seg_recur_fast: at node 0 the
// forcing must be F^L = 0, F^R = g v_1 and at node M F^L = g v_{M-1}, F^R = 0
// (no curvature at a boundary node); the branch-free forcing is off by
// -w2 v_1 (node 0) and -w2 v_{M-1} (node M) in both directions.  The linear
// recurrences carry these corrections with powers of d.  v1 = value at node 1,
// vM1 = value at node M-1 (read by the caller).  Returns E^L_M (local) in eLM.
template <typename T, int S>
__device__ __forceinline__ void seg_fix_dirichlet(int p0, int M, T v1, T vM1, T d, T w2,
                                                  T (&sum)[S], T &aL, T &aR, T &eLM)
{
    if (p0 == 0) {
        const T c = -w2 * v1;
        T pw = c, last = c;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            sum[j] += pw;                 // forward: c d^j
            last = pw;
            pw *= d;
        }
        aL += last;                       // c d^{S-1}
        sum[0] += c;                      // backward: node 0 only
        aR += c;
    }
    const int jm = M - p0;
    if (jm >= 0 && jm < S) {
        const T c = -w2 * vM1;
        T pf = c, pb = c, lf = T(0), lb = T(0);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j >= jm) { sum[j] += pf; lf = pf; pf *= d; }
        }
#pragma unroll
        for (int j = S - 1; j >= 0; --j) {
            if (j <= jm) { sum[j] += pb; lb = pb; pb *= d; }
        }
        aL += lf;                         // c d^{S-1-jm}
        aR += lb;                         // c d^{jm}
        T em = T(0);
#pragma unroll
        for (int j = 0; j < S; ++j)
            if (j == jm) em = sum[j];     // E^R_M = 0 locally: sum = E^L_M
        eLM = em;
    }
}

// End nodes of a line with boundary data (end values v_0 = v(a), v_M = v(b) in
// the field; ka, kb the curvatures of the end cells' quadratics times h^2:
// the data's for Dirichlet ends, those the end slopes give for Neumann ends).
// The recurrences start at the end nodes, E^L_0 = -v_0/2 and E^R_M = -v_M/2,
// and the end cells take the quadratic through the end node and its inner
// neighbour with that curvature (the forcing of a node next to a ghost value
// 2 v_0 - v_1 + ka).  The branch-free forcing (values beyond the line read as 0) is
// corrected at nodes 0, M and M+1 by the differences below, propagated by
// powers of d; returns E^L_M (local) in eLM.
template <typename T, int S>
__device__ __forceinline__ void seg_fix_bdata(int p0, int M, T v0, T v1, T vM1, T vM, T ka, T kb, T d,
                                              T g, T w2, T (&sum)[S], T &aL, T &aR, T &eLM)
{
    const T gw2 = g + T(2) * w2;
    const int q[3] = {0, M, M + 1};
    const T cLq[3] = {-T(0.5) * v0 - w2 * v1 + gw2 * v0, w2 * (kb + T(2) * vM - vM1), -(g + w2) * vM};
    const T cRq[3] = {w2 * (ka - v1 + T(2) * v0), -T(0.5) * vM + gw2 * vM - w2 * vM1, -w2 * vM};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int jq = q[i] - p0;
        if (jq < 0 || jq >= S) continue;
        T pf = cLq[i], pb = cRq[i], lf = T(0), lb = T(0);
#pragma unroll
        for (int j = 0; j < S; ++j)
            if (j >= jq) { sum[j] += pf; lf = pf; pf *= d; }
#pragma unroll
        for (int j = S - 1; j >= 0; --j)
            if (j <= jq) { sum[j] += pb; lb = pb; pb *= d; }
        aL += lf;
        aR += lb;
    }
    // E^R_M is -v_M/2 locally (the forcing beyond M is removed)
    const int jm = M - p0;
    if (jm >= 0 && jm < S) {
        T em = T(0);
#pragma unroll
        for (int j = 0; j < S; ++j)
            if (j == jm) em = sum[j];
        eLM = em + T(0.5) * vM;
    }
}

// Closure for a segment: D_j = -(sum_j + d^{j+1} cL + d^{S-j} cR + A d^p + B d^{M-p}).
// Interior segments carry two decaying terms, advanced by repeated products with d;
// a segment holding node M (or nodes beyond it) adds the B term
// node by node and zeroes what lies beyond M; Dirichlet end nodes get D = 0.
// mwave (wave-uniform) = false: no lane of this wave holds node M or lies
// beyond it, so the per-lane end handling is skipped by a branch instead of
// being evaluated (and discarded) by every lane.
// ea = e^{-nu p0}, eb = e^{-nu (M - p0 - S + 1)}: the closure's decay factors
// at this segment (seg_close_fast forms them; a caller that closes several
// sweeps with the same segments passes them in)
template <typename T, int S>
__device__ __forceinline__ void seg_close_fast_w(T (&sum)[S], T cL, T cR, double A, double B, int p0,
                                                 int M, T ea, T eb, T d, bool dir_end, bool mwave = true)
{
    const int jm = M - p0;
    const bool holdsM = jm < S;
    const T lt = d * cL + ((A != 0.0) ? (T)A * ea : T(0));
    const T rt = d * cR + ((!holdsM && B != 0.0) ? (T)B * eb : T(0));
    T tl = lt, tr = rt;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        sum[j] += tl;                 // lt d^j
        tl *= d;
        sum[S - 1 - j] += tr;         // rt d^{S-1-j}
        tr *= d;
    }
#pragma unroll
    for (int j = 0; j < S; ++j) sum[j] = -sum[j];
    if (mwave && holdsM) {
        T pw = (T)B;
#pragma unroll
        for (int j = S - 1; j >= 0; --j) {
            if (j > jm) {
                sum[j] = T(0);
            } else {
                sum[j] -= pw;
                pw *= d;
            }
        }
        if (dir_end) {
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (j == jm) sum[j] = T(0);
        }
    }
    if (dir_end && p0 == 0) sum[0] = T(0);
}
template <typename T, int S>
__device__ __forceinline__ void seg_close_fast(T (&sum)[S], T cL, T cR, double A, double B, int p0,
                                               int M, double nu, T d, bool dir_end, bool mwave = true)
{
    const int jm = M - p0;
    const T ea = (A != 0.0) ? expneg<T>(nu * (double)p0) : T(0);
    const T eb = (jm >= S && B != 0.0) ? expneg<T>(nu * (double)(jm - (S - 1))) : T(0);
    seg_close_fast_w<T, S>(sum, cL, cR, A, B, p0, M, ea, eb, d, dir_end, mwave);
}

// ---------------------------------------------------------------------------
// x sweep: contiguous lines, one line per workgroup of NT = 64*WPL threads
// ---------------------------------------------------------------------------
// D_x of NSW combinations staged in LDS (sm + k*NPAD, padded slots); the D
// values replace the inputs in place.  Ends with a __syncthreads.
// XM: 0 = D sweeps, 1 = some combination swept for L^{-1}, 2 = a line with
// boundary data (Dirichlet or Neumann, one combination)
// Per-thread decay factors of an x sweep (the same for every sweep of the
// workgroup's line): the lane scans' weights, d^{S lane} and d^{S (63 - lane)}
// for the carries between waves, and the closure's factors at the thread's
// segment.  Formed once and shared by the chained sweeps.
template <typename T>
struct XW {
    LaneW<T> lw;
    T pl, pr, ea, eb;
};
template <typename T, int S>
__device__ __forceinline__ XW<T> x_weights(const KArgs<T> &a, int t, int n)
{
    const int lane = t & 63;
    const int p0 = t * S, jm = n - 1 - p0;
    XW<T> w;
    w.lw = lane_weights<T>(a.nu * (double)S, lane);
    w.pl = expneg<T>(a.nu * (double)S * (double)lane);
    w.pr = expneg<T>(a.nu * (double)S * (double)(63 - lane));
    w.ea = expneg<T>(a.nu * (double)p0);
    w.eb = (jm >= S) ? expneg<T>(a.nu * (double)(jm - (S - 1))) : T(0);
    return w;
}

template <typename T, int S, int WPL, int NSW, bool PER, int XM = 0>
__device__ __forceinline__ void x_line_sweep(const KArgs<T> &a, T *sm, T (*wtot)[MAXS][WPL],
                                             T (*ends)[MAXS], int t, int n, const XW<T> &xw)
{
    constexpr bool KF = (XM == 1), BD = (XM == 2);
    constexpr int NT = 64 * WPL;
    constexpr int NPAD = NT * (S + 1);
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int M = n - 1;
    const int p0 = t * S;
    const int jm = M - p0;
    // the wave whose lanes hold node M (n <= NT S): only waves 0 and waveM
    // take the Dirichlet end fix-ups, only waves from waveM on the closure's
    // end handling (wave-uniform branches; the other waves skip that code)
    const int waveM = (M / S) >> 6;
    constexpr bool dir_end = !PER;
    const bool slow = PER && (p0 + S - 1 > M);          // periodic lane crossing the end
    T sum[NSW][S];
    T aL[NSW], aR[NSW], eLM[NSW];
#pragma unroll
    for (int k = 0; k < NSW; ++k) {
        const T *sk = sm + k * NPAD;
        T v[S + 2];
#pragma unroll
        for (int j = 0; j < S; ++j) v[j + 1] = sk[t * (S + 1) + j];
        if (p0 == 0) v[0] = PER ? sk[(M / S) * (S + 1) + (M % S)] : T(0);
        else v[0] = sk[(t - 1) * (S + 1) + (S - 1)];
        v[S + 1] = (t + 1 < NT) ? sk[(t + 1) * (S + 1)] : T(0);
        if (PER && jm >= 0 && jm < S) v[jm + 2] = sk[0];          // wrap at node M
        if (PER && slow) {
            if (KF && a.kform[k]) seg_recur_I<T, S>(v, p0, M, a.d, a.w0, a.w1, a.w2, sum[k], aL[k], aR[k], eLM[k]);
            else seg_recur<T, S>(v, p0, M, false, a.d, a.g, a.w2, sum[k], aL[k], aR[k], eLM[k]);
        } else {
            if (KF && a.kform[k]) seg_recur_fast_I<T, S>(v, a.d, a.w0, a.w1, a.w2, sum[k], aL[k], aR[k]);
            else seg_recur_fast<T, S>(v, a.d, a.gw, a.w2, sum[k], aL[k], aR[k]);
            eLM[k] = aL[k];                            // periodic: node M ends its lane
            if (dir_end && (BD || wave == 0 || wave == waveM)) {
                const T v1 = (p0 == 0 && n > 1) ? sk[1] : T(0);
                const int q = M - 1;
                const T vM1 = (jm >= 0 && jm < S && q >= 0) ? sk[(q / S) * (S + 1) + (q % S)] : T(0);
                if (BD) {
                    // end-cell curvatures times h^2: the data's (bmode 1), or
                    // those of the quadratics through the end node and its
                    // neighbour with the given slopes, bk = 2 h slope (bmode 2)
                    const T v0 = sk[0];
                    const T vM = sk[(M / S) * (S + 1) + (M % S)];
                    const bool nm = a.bmode == 2;
                    const T ka = nm ? T(2) * (v1 - v0) - a.bk[0] : a.bk[0];
                    const T kb = nm ? T(2) * (vM1 - vM) + a.bk[1] : a.bk[1];
                    seg_fix_bdata<T, S>(p0, M, v0, v1, vM1, vM, ka, kb, a.d, a.g, a.w2, sum[k], aL[k], aR[k],
                                        eLM[k]);
                } else {
                    seg_fix_dirichlet<T, S>(p0, M, v1, vM1, a.d, a.w2, sum[k], aL[k], aR[k], eLM[k]);
                }
            }
        }
    }
    // lane scan (multiplier d^S per lane; multipliers d^(S off) rounded once
    // from FP64: repeated squaring in FP32 would compound its rounding), then
    // waves through LDS
    T cL[NSW], cR[NSW];
#pragma unroll
    for (int k = 0; k < NSW; ++k) {
        T xl = aL[k], xr = aR[k];
        lane_scans<T>(xl, xr, a.dpw, xw.lw, lane);
        cL[k] = dpp_mov<0x138>(xl);              // lane - 1 (0 at lane 0)
        cR[k] = dpp_mov<0x130>(xr);              // lane + 1 (0 at lane 63)
        if (WPL > 1) {
            if (lane == 63) wtot[0][k][wave] = xl;
            if (lane == 0) wtot[1][k][wave] = xr;
        }
    }
    if (WPL > 1) {
        __syncthreads();
        const T pl = xw.pl, pr = xw.pr;
#pragma unroll
        for (int k = 0; k < NSW; ++k) {
            T cw = T(0), cwr = T(0);
            for (int w = 0; w < wave; ++w) cw = a.dBlk * cw + wtot[0][k][w];
            for (int w = WPL - 1; w > wave; --w) cwr = a.dBlk * cwr + wtot[1][k][w];
            cL[k] += pl * cw;
            cR[k] += pr * cwr;
        }
    }
    // line ends: E^R_0 (lane holding node 0) and E^L_M (lane holding node M)
#pragma unroll
    for (int k = 0; k < NSW; ++k) {
        if (p0 == 0) ends[0][k] = aR[k] + a.dS * cR[k];
        if (jm >= 0 && jm < S) ends[1][k] = eLM[k] + expneg<T>(a.nu * (double)(jm + 1)) * cL[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NSW; ++k) {
        T *sk = sm + k * NPAD;
        double er0 = (double)ends[0][k], elm = (double)ends[1][k];
        if (BD) {
            // L^{-1} v takes the targets at the ends: the closure acts on
            // E^R_0 - (t_a - v_0/2) and E^L_M - (t_b - v_M/2)
            er0 -= (double)a.bt[0] - 0.5 * (double)sk[0];
            elm -= (double)a.bt[1] - 0.5 * (double)sk[(M / S) * (S + 1) + (M % S)];
            __syncthreads();     // every thread has read the end values before any D replaces them
        }
        const double A = a.K00 * er0 + a.K01 * elm;
        const double B = a.K10 * er0 + a.K11 * elm;
        if (PER && slow) seg_close<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, a.nu, a.d, false);
        else seg_close_fast_w<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, xw.ea, xw.eb, a.d, dir_end && !BD,
                                    wave >= waveM);
#pragma unroll
        for (int j = 0; j < S; ++j) sk[t * (S + 1) + j] = sum[k][j];
    }
    __syncthreads();
}

// FULL: the line fills the workgroup (n = 64 WPL S), a compile-time length,
// so that no bounds selects remain on the loads, the staging and the stores
template <typename T, int S, int WPL, int NS, int NO, int VW, bool PER, int NFMAX, int XM, bool FULL>
__device__ __forceinline__ void sweep_x_body_n(const KArgs<T> &a, const int64_t bid)
{
    constexpr bool BD = (XM == 2);
    constexpr int NT = 64 * WPL;
    constexpr int NPAD = NT * (S + 1);
    constexpr int NV = S / VW;
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);          // [NS][NPAD]
    __shared__ T wtot[2][MAXS][WPL];
    __shared__ T ends[2][MAXS];

    const int t = threadIdx.x;
    const int64_t line = bid;
    const int n = FULL ? NT * S : (int)a.n;
    const int M = n - 1;
    const int64_t base = line * a.lineoff;            // uniform per workgroup
    constexpr bool dir_end = !PER;

    bool bline = false;
    if (a.proj) {
        const int64_t i1 = line % a.pn1, i2 = line / a.pn1;
        bline = (a.pd1 && (i1 == 0 || i1 == a.pn1 - 1)) || (a.pd2 && (i2 == 0 || i2 == a.pn2 - 1));
    }

    // ---- phase 1: coalesced loads (all of one field at once), prologue ----
    T sv[NS][S], ev[NO][S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
#pragma unroll
        for (int k = 0; k < NS; ++k) sv[k][j] = T(0);
#pragma unroll
        for (int o = 0; o < NO; ++o) ev[o][j] = T(0);
    }
    // Loads are unconditional (clamped addresses, values beyond the line
    // zeroed afterwards) so that all of a field's loads are in flight at once;
    // vector loads need an aligned line whose length is a multiple of VW, so a
    // vector lies wholly inside or wholly beyond the line.
    auto accumulate = [&](int f, const T (&x)[S]) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
#pragma unroll
            for (int k = 0; k < NS; ++k) sv[k][j] += a.mS[k][f] * x[j];
#pragma unroll
            for (int o = 0; o < NO; ++o) ev[o][j] += a.mOF[o][f] * x[j];
        }
    };
    auto load_vec = [&](int f0, auto cc) {
        constexpr int C = decltype(cc)::value;
        T x[C][S];
#pragma unroll
        for (int c0 = 0; c0 < C; ++c0) {
            const T *src = a.f[f0 + c0] + base;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int e0 = (i * NT + t) * VW;
                const bool in = e0 < n;
                const vec_t vv = *reinterpret_cast<const vec_t *>(src + (in ? (unsigned)e0 : 0u));
#pragma unroll
                for (int c = 0; c < VW; ++c) x[c0][i * VW + c] = in ? vv[c] : T(0);
            }
        }
#pragma unroll
        for (int c0 = 0; c0 < C; ++c0) accumulate(f0 + c0, x[c0]);
    };
    auto load_scalar = [&](int f) {
        const T *src = a.f[f] + base;
        T x[S];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
#pragma unroll
            for (int c = 0; c < VW; ++c) {
                const int e = (i * NT + t) * VW + c;
                const T val = src[(unsigned)(e < n ? e : n - 1)];
                x[i * VW + c] = (e < n) ? val : T(0);
            }
        }
        accumulate(f, x);
    };
    if (a.aligned) {
        field_chunks<4, NFMAX>(a.nf, load_vec);
    } else {
        for (int f = 0; f < a.nf; ++f) load_scalar(f);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const int e = (i * NT + t) * VW + c;
            const int slot = (e / S) * (S + 1) + (e % S);
            // (a line with Dirichlet data keeps its end values)
            const bool zero = (e >= n) || (dir_end && !BD && (e == 0 || e == M));
#pragma unroll
            for (int k = 0; k < NS; ++k) sm[k * NPAD + slot] = zero ? T(0) : sv[k][i * VW + c];
        }
    }
    __syncthreads();

    // ---- phases 2-3: recurrences, scans, closure (D in LDS) ----
    const XW<T> xw = x_weights<T, S>(a, t, n);
    x_line_sweep<T, S, WPL, NS, PER, XM>(a, sm, wtot, ends, t, n, xw);

    // ---- phase 4: epilogue in the coalesced layout ----
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int e0 = (i * NT + t) * VW;
        T out[NO][VW];
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const int e = e0 + c;
            const int slot = (e / S) * (S + 1) + (e % S);
            T Dk[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) Dk[k] = sm[k * NPAD + slot];
            const bool z = a.proj && (bline || (dir_end && (e == 0 || e == M)));
            // projected end nodes of a line with Dirichlet data take the data
            const T zv = BD ? (e == 0 ? a.bend[0] : a.bend[1]) : T(0);
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                T r = ev[o][i * VW + c];
#pragma unroll
                for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * Dk[k];
                out[o][c] = z ? zv : r;
            }
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            T *dst = a.o[o] + base;
            if (a.aligned && e0 + VW <= n) {
                vec_t vv;
#pragma unroll
                for (int c = 0; c < VW; ++c) vv[c] = out[o][c];
                *reinterpret_cast<vec_t *>(dst + e0) = vv;
            } else {
#pragma unroll
                for (int c = 0; c < VW; ++c)
                    if (e0 + c < n) dst[e0 + c] = out[o][c];
            }
        }
        if (a.chain) {
            // the next x sweep of output 0 starts from these values (each
            // slot is read and rewritten by the same thread only)
#pragma unroll
            for (int c = 0; c < VW; ++c) {
                const int e = e0 + c;
                const int slot = (e / S) * (S + 1) + (e % S);
                const bool zero = (e >= n) || (dir_end && (e == 0 || e == M));
                sm[slot] = zero ? T(0) : out[0][c];
            }
        }
    }
    if (a.chain) {
        __syncthreads();
        x_line_sweep<T, S, WPL, 1, PER>(a, sm, wtot, ends, t, n, xw);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e0 = (i * NT + t) * VW;
            T out[VW];
#pragma unroll
            for (int c = 0; c < VW; ++c) {
                const int e = e0 + c;
                out[c] = sm[(e / S) * (S + 1) + (e % S)];
            }
            T *dst = a.ochain + base;
            if (a.aligned && e0 + VW <= n) {
                vec_t vv;
#pragma unroll
                for (int c = 0; c < VW; ++c) vv[c] = out[c];
                *reinterpret_cast<vec_t *>(dst + e0) = vv;
            } else {
#pragma unroll
                for (int c = 0; c < VW; ++c)
                    if (e0 + c < n) dst[e0 + c] = out[c];
            }
        }
    }
}
template <typename T, int S, int WPL, int NS, int NO, int VW, bool PER, int NFMAX, int XM = 0>
__device__ __forceinline__ void sweep_x_body(const KArgs<T> &a, const int64_t bid)
{
    if (a.n == (int64_t)64 * WPL * S) sweep_x_body_n<T, S, WPL, NS, NO, VW, PER, NFMAX, XM, true>(a, bid);
    else sweep_x_body_n<T, S, WPL, NS, NO, VW, PER, NFMAX, XM, false>(a, bid);
}
// XM = 1: some combination is swept for L^{-1} (the I recurrences); XM = 2: a
// line with Dirichlet data; XM = 0: D recurrences and homogeneous ends only
template <typename T, int S, int WPL, int NS, int NO, int VW, bool PER, int NFMAX, int XM = 0>
__global__ void __launch_bounds__(64 * WPL)
k_sweep_x(const KArgs<T> a)
{
    sweep_x_body<T, S, WPL, NS, NO, VW, PER, NFMAX, XM>(a, blockIdx.x);
}
template <typename T, int S, int WPL, int NS, int NO, int VW, bool PER, int NFMAX>
__global__ void __launch_bounds__(64 * WPL)
k_sweep_x_b(const KArgs<T> *__restrict__ tab, const int64_t *__restrict__ first, int nent)
{
    const int e = batch_entry(first, nent, blockIdx.x);
    sweep_x_body<T, S, WPL, NS, NO, VW, PER, NFMAX>(tab[e], (int64_t)blockIdx.x - first[e]);
}

// ---------------------------------------------------------------------------
// strided sweep (y or z): lanes = 64 consecutive columns, W waves x S nodes
// ---------------------------------------------------------------------------
template <typename T, int S, int W, int NS, int NO, bool PER, int NFMAX>
__device__ __forceinline__ void sweep_s_body(const KArgs<T> &a, const int64_t bid)
{
    constexpr int WS = W * S;
    __shared__ T red[2][NS][W][64];      // cooperative sums, then wave aggregates
    __shared__ T endv[2][NS][64];        // E^R_0 and E^L_M per column (one tile)

    const int lane = threadIdx.x & 63;
    // wave index as a scalar: row numbers, row pointers and every per-row
    // decision below are wave-uniform (scalar registers, one shared lane offset)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t L = xcd_remap(bid, a.nblocks);
    const int tile = (int)(L % a.ntiles);
    const int64_t rest = L / a.ntiles;
    const int64_t ncg = (a.nlines + 63) / 64;
    const int64_t cg = rest % ncg;
    const int64_t outer = rest / ncg;
    const int col = (int)(cg * 64) + lane;
    const bool active = col < a.nlines;
    const int n = (int)a.n, M = n - 1;
    const int ls = (int)a.ls;
    const int64_t blk = cg * 64 + outer * a.os;          // uniform per workgroup
    const int loff = active ? lane : 0;                  // per-lane column offset
    constexpr bool dir_end = !PER;
    constexpr bool per = PER;
    const T d = a.d, g = a.g, w2 = a.w2;
    const int oa = tile * WS;
    const int ob = (oa + WS < n) ? oa + WS : n;
    const bool split = a.ntiles > 1;
    const int K = a.halo;
    const int p0 = oa + wave * S;

    // this wave's share of the halo sums: kk in [k0, k1) (truncation length K)
    constexpr int QB = 2;                                // halo rows per wave in the batched path
    const int q = (K + W - 1) / W;
    const int k0 = wave * q;
    const int k1 = (k0 + q < K) ? k0 + q : K;
    const bool hb_top = split && (per || oa > 0);
    const bool hb_bot = split && (per || ob < n);
    const bool batched = (q <= QB);
    // row index as read: periodic wrap, or -1 when the node reads as 0
    auto rowidx = [&](int p) -> int {
        if (per) {
            p %= n;
            if (p < 0) p += n;
            return p;
        }
        return (p <= 0 || p >= M) ? -1 : p;
    };

    // ---- main nodes p0-1 .. p0+S and the halo rows: one batch of loads per field ----
    T ev[NO][S];
    T v[NS][S + 2];
    T ht[NS][QB + 2], hbv[NS][QB + 2];   // top rows oa-k0-i, bottom rows ob+k0-1+i
#pragma unroll
    for (int k = 0; k < NS; ++k) {
#pragma unroll
        for (int j = 0; j < S + 2; ++j) v[k][j] = T(0);
#pragma unroll
        for (int i = 0; i < QB + 2; ++i) { ht[k][i] = T(0); hbv[k][i] = T(0); }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
#pragma unroll
        for (int o = 0; o < NO; ++o) ev[o][j] = T(0);
    }
    const unsigned lo = (unsigned)loff;
    // row pointer of node p of this column group (wave-uniform), or the zero
    // row when the node reads as 0 (outside a Dirichlet line)
    auto rowptr = [&](const T *fb, int p) -> const T * {
        if (per) {
            if (p < 0) p += n;
            if (p >= n) p -= n;
        }
        return (p >= 0 && p <= M) ? fb + (int64_t)p * ls : zero_row<T>();
    };
    auto load_fields = [&](int f0, auto cc) {
        constexpr int C = decltype(cc)::value;
        T x[C][S + 2], xt[C][QB + 2], xb[C][QB + 2];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T *fb = a.f[f0 + c] + blk;
#pragma unroll
            for (int j = 0; j < S + 2; ++j) x[c][j] = rowptr(fb, p0 - 1 + j)[lo];
            if (batched) {
#pragma unroll
                for (int i = 0; i < QB + 2; ++i) {
                    const int rt = rowidx(oa - k0 - i);
                    const int rb = rowidx(ob + k0 - 1 + i);
                    xt[c][i] = (hb_top && rt >= 0 && rt <= M ? fb + (int64_t)rt * ls : zero_row<T>())[lo];
                    xb[c][i] = (hb_bot && rb >= 0 && rb <= M ? fb + (int64_t)rb * ls : zero_row<T>())[lo];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int f = f0 + c;
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
#pragma unroll
                for (int k = 0; k < NS; ++k) v[k][j] += a.mS[k][f] * x[c][j];
                if (j >= 1 && j <= S) {
#pragma unroll
                    for (int o = 0; o < NO; ++o) ev[o][j - 1] += a.mOF[o][f] * x[c][j];
                }
            }
            if (batched) {
#pragma unroll
                for (int i = 0; i < QB + 2; ++i) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        ht[k][i] += a.mS[k][f] * xt[c][i];
                        hbv[k][i] += a.mS[k][f] * xb[c][i];
                    }
                }
            }
        }
    };
    field_chunks<2, NFMAX>(a.nf, load_fields);
    if (dir_end) {
#pragma unroll
        for (int j = 0; j < S + 2; ++j) {
            const int p = p0 - 1 + j;
            if (p == 0 || p == M) {
#pragma unroll
                for (int k = 0; k < NS; ++k) v[k][j] = T(0);
            }
        }
    }

    // swept combination k at node p of this column (0 outside / at Dirichlet ends)
    auto sval = [&](int k, int p) -> T {
        const int r = rowidx(p);
        if (r < 0 || !active) return T(0);
        const int off = loff + r * ls;
        T s = T(0);
        for (int f = 0; f < a.nf; ++f) s += a.mS[k][f] * a.f[f][blk + off];
        return s;
    };
    // this wave's share of sum_{kk<K} d^kk F(r0 + sg*kk) by direct loads (long
    // halos only): sg = -1 sums the forcing of E^L moving up from r0, sg = +1
    // that of E^R moving down
    auto part = [&](int k, int r0, int sg) -> T {
        T acc = T(0);
        if (k0 >= k1) return acc;
        T pw = expneg<T>(a.nu * (double)k0);
        int r = r0 + sg * k0;
        T vb = sval(k, r - sg), v0 = sval(k, r);
        for (int kk = k0; kk < k1; ++kk, r += sg) {
            const T vn = sval(k, r + sg);
            const int rr = per ? ((r % n) + n) % n : r;
            const T fv = (sg < 0) ? force_L(vn, v0, vb, rr, M, dir_end, g, w2)
                                  : force_R(vb, v0, vn, rr, M, dir_end, g, w2);
            acc += pw * fv;
            pw *= d;
            vb = v0;
            v0 = vn;
        }
        return acc;
    };
    // the same sums from the batched halo rows
    auto part_batched = [&](int k, bool top) -> T {
        T acc = T(0);
        T pw = expneg<T>(a.nu * (double)k0);
#pragma unroll
        for (int i = 0; i < QB; ++i) {
            const int kk = k0 + i;
            if (kk < k1) {
                T fv;
                if (top) {
                    const int r = oa - 1 - kk;      // values at r+1, r, r-1 = ht[i], ht[i+1], ht[i+2]
                    const int rr = per ? ((r % n) + n) % n : r;
                    fv = force_L(ht[k][i + 2], ht[k][i + 1], ht[k][i], rr, M, dir_end, g, w2);
                } else {
                    const int r = ob + kk;          // values at r-1, r, r+1 = hbv[i], hbv[i+1], hbv[i+2]
                    const int rr = per ? ((r % n) + n) % n : r;
                    fv = force_R(hbv[k][i], hbv[k][i + 1], hbv[k][i + 2], rr, M, dir_end, g, w2);
                }
                acc += pw * fv;
                pw *= d;
            }
        }
        return acc;
    };
    // cooperative pair of sums over all waves (workgroup-uniform call)
    auto coop = [&](int r0a, int sga, bool usea, int r0b, int sgb, bool useb, bool fromregs,
                    T (&oa_)[NS], T (&ob_)[NS]) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            red[0][k][wave][lane] = !usea ? T(0) : fromregs ? part_batched(k, true) : part(k, r0a, sga);
            red[1][k][wave][lane] = !useb ? T(0) : fromregs ? part_batched(k, false) : part(k, r0b, sgb);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T x = T(0), y = T(0);
            for (int w = 0; w < W; ++w) {
                x += red[0][k][w][lane];
                y += red[1][k][w][lane];
            }
            oa_[k] = x;
            ob_[k] = y;
        }
        __syncthreads();
    };

    // ---- local recurrences of this wave's S nodes ----
    const int jm = M - p0;
    const bool slow = per && (p0 + S - 1 > M);          // periodic wave crossing the end
    T sum[NS][S];
    T aL[NS], aR[NS], eLM[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (PER && slow) {
            if (a.kform[k]) seg_recur_I<T, S>(v[k], p0, M, d, a.w0, a.w1, w2, sum[k], aL[k], aR[k], eLM[k]);
            else seg_recur<T, S>(v[k], p0, M, false, d, g, w2, sum[k], aL[k], aR[k], eLM[k]);
        } else {
            if (a.kform[k]) seg_recur_fast_I<T, S>(v[k], d, a.w0, a.w1, w2, sum[k], aL[k], aR[k]);
            else seg_recur_fast<T, S>(v[k], d, a.gw, w2, sum[k], aL[k], aR[k]);
            eLM[k] = aL[k];
            if (dir_end && (p0 == 0 || (jm >= 0 && jm < S))) {
                T vM1 = T(0);
#pragma unroll
                for (int j = 0; j < S + 2; ++j)
                    if (j == jm) vM1 = v[k][j];            // node M-1
                seg_fix_dirichlet<T, S>(p0, M, v[k][2], vM1, d, w2, sum[k], aL[k], aR[k], eLM[k]);
            }
        }
    }

    // ---- carries entering the tile, and line-end values for split lines ----
    T cTop[NS], cBot[NS], er0s[NS], elms[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        cTop[k] = T(0);
        cBot[k] = T(0);
        er0s[k] = T(0);
        elms[k] = T(0);
    }
    // a tile that does not hold a line end but lies within K nodes of it
    // needs that end's value (cooperative sums, rare)
    const bool needA = split && !per && oa > 0 && oa < K;
    const bool needB = split && !per && ob < n && n - ob < K;
    if (split) {
        coop(oa - 1, -1, hb_top, ob, +1, hb_bot, batched, cTop, cBot);
        if (needA || needB) coop(0, +1, needA, M, -1, needB, false, er0s, elms);
    }

#pragma unroll
    for (int k = 0; k < NS; ++k) {
        red[0][k][wave][lane] = aL[k];
        red[1][k][wave][lane] = aR[k];
    }
    __syncthreads();
    // In a short last tile of a split periodic line the bottom carry enters
    // at node n, inside a wave: it is applied through the closure instead.
    const bool botAsB = per && split && ob == n;
    T cL[NS], cR[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T c = cTop[k];
        for (int w = 0; w < wave; ++w) c = a.dS * c + red[0][k][w][lane];
        cL[k] = c;
        T cr = botAsB ? T(0) : cBot[k];
        for (int w = W - 1; w > wave; --w) cr = a.dS * cr + red[1][k][w][lane];
        cR[k] = cr;
    }
    const bool has0 = (oa == 0), hasM = (ob == n);
    if (!per || !split) {
        // exact line-end values from this tile's own scan
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (p0 == 0) endv[0][k][lane] = aR[k] + a.dS * cR[k];
            if (jm >= 0 && jm < S) endv[1][k][lane] = eLM[k] + expneg<T>(a.nu * (double)(jm + 1)) * cL[k];
        }
        __syncthreads();
    }

    // ---- closure and epilogue ----
    bool bline = false;
    if (a.proj)
        bline = (a.pd1 && (col == 0 || col == a.pn1 - 1)) ||
                (a.pd2 && (outer == 0 || outer == a.pn2 - 1));
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double A = 0.0, B = 0.0;
        if (!per || !split) {
            // a split Dirichlet line takes each end value from the tile holding
            // it, or from the cooperative sums within K nodes of it
            const double er0 = has0 ? (double)endv[0][k][lane] : (double)er0s[k];
            const double elm = hasM ? (double)endv[1][k][lane] : (double)elms[k];
            A = a.K00 * er0 + a.K01 * elm;
            B = a.K10 * er0 + a.K11 * elm;
        } else if (botAsB) {
            B = (double)d * (double)cBot[k];     // cBot d^{n-p} = (d cBot) d^{M-p}
        }
        if (PER && slow) seg_close<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, a.nu, d, false);
        else seg_close_fast<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, a.nu, d, dir_end);
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        if (p > M) break;
        const bool z = a.proj && (bline || (dir_end && (p == 0 || p == M)));
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            T r = ev[o][j];
#pragma unroll
            for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * sum[k][j];
            (a.o[o] + blk + (int64_t)p * ls)[lo] = z ? T(0) : r;
        }
    }
}
template <typename T, int S, int W, int NS, int NO, bool PER, int NFMAX>
__global__ void __launch_bounds__(64 * W)
k_sweep_s(const KArgs<T> a)
{
    sweep_s_body<T, S, W, NS, NO, PER, NFMAX>(a, blockIdx.x);
}
template <typename T, int S, int W, int NS, int NO, bool PER, int NFMAX>
__global__ void __launch_bounds__(64 * W)
k_sweep_s_b(const KArgs<T> *__restrict__ tab, const int64_t *__restrict__ first, int nent)
{
    const int e = batch_entry(first, nent, blockIdx.x);
    sweep_s_body<T, S, W, NS, NO, PER, NFMAX>(tab[e], (int64_t)blockIdx.x - first[e]);
}

// ---------------------------------------------------------------------------
// exact strided sweep in two passes (y or z lines of any length and any nu)
// ---------------------------------------------------------------------------
// The recurrences are linear, so the carry entering a tile is a sum over the
// tiles before it of their own aggregates, each damped by d per node.  Pass 1
// (MODE 1) sweeps every tile with zero carries in and writes, per column, its
// forward aggregate TL (E^L at its last row), its backward aggregate TR (E^R
// at its first row) and, for the tile holding node M, E^L at M (EM).  A small
// scan (k_exact_scan, one lane per column) folds the aggregates in place into
// the exact carries entering every tile, cTop = sum_{t'<t} d^{WS (t-1-t')} TL_t'
// and cBot = sum_{t'>t} d^{WS (t'-t-1)} TR_t', and into the line-end values
// E^R_0 = sum_t d^{WS t} TR_t and E^L_M = EM + d^{M - s_last + 1} cTop_last.
// Pass 2 (MODE 2) sweeps every tile again with those carries and forms the
// boundary correction (Dirichlet or periodic) as on a line held by one tile.  Nothing is truncated: the cost is one more read of
// the swept fields instead of halos that grow like 1/nu.
template <typename T, int S, int W, int NS, int NO, bool PER, int NFMAX, int MODE>
__device__ __forceinline__ void sweep_e_body(const KArgs<T> &a, const int64_t bid)
{
    constexpr int WS = W * S;
    __shared__ T red[2][NS][W][64];      // wave aggregates
    __shared__ T carry[4][NS][64];       // cTop, cBot, E^R_0, E^L_M of the tile's columns

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t L = xcd_remap(bid, a.nblocks);
    const int ntiles = a.ntiles;
    const int tile = (int)(L % ntiles);
    const int64_t rest = L / ntiles;
    const int64_t ncg = (a.nlines + 63) / 64;
    const int64_t cg = rest % ncg;
    const int64_t outer = rest / ncg;
    const int col = (int)(cg * 64) + lane;
    const bool active = col < a.nlines;
    const int n = (int)a.n, M = n - 1;
    const int ls = (int)a.ls;
    const int64_t blk = cg * 64 + outer * a.os;
    const int loff = active ? lane : 0;
    constexpr bool dir_end = !PER;
    const T d = a.d, g = a.g, w2 = a.w2;
    const int oa = tile * WS;
    const int p0 = oa + wave * S;
    // aggregate table of this column group: [tile][k][3][64]
    T *tab = a.agg + (size_t)(outer * ncg + cg) * (size_t)ntiles * (MAXS * 3 * 64);

    // ---- loads of nodes p0-1 .. p0+S and the prologue ----
    constexpr int NOE = (MODE == 2) ? NO : 1;
    T ev[NOE][S];
    T v[NS][S + 2];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int j = 0; j < S + 2; ++j) v[k][j] = T(0);
#pragma unroll
    for (int o = 0; o < NOE; ++o)
#pragma unroll
        for (int j = 0; j < S; ++j) ev[o][j] = T(0);
    const unsigned lo = (unsigned)loff;
    auto rowptr = [&](const T *fb, int p) -> const T * {
        if (PER) {
            if (p < 0) p += n;
            if (p >= n) p -= n;
        }
        return (p >= 0 && p <= M) ? fb + (int64_t)p * ls : zero_row<T>();
    };
    // rows p0-1 .. p0+S all inside the line (a wave-uniform test): plain row
    // addresses, no per-row choice of the zero row
    const bool rows_in = p0 >= 1 && p0 + S <= M;
    auto load_fields = [&](int f0, auto cc) {
        constexpr int C = decltype(cc)::value;
        T x[C][S + 2];
        if (rows_in) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T *fb = a.f[f0 + c] + blk + (int64_t)(p0 - 1) * ls + lo;
#pragma unroll
                for (int j = 0; j < S + 2; ++j) x[c][j] = fb[(int64_t)j * ls];
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T *fb = a.f[f0 + c] + blk;
#pragma unroll
                for (int j = 0; j < S + 2; ++j) x[c][j] = rowptr(fb, p0 - 1 + j)[lo];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int f = f0 + c;
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
#pragma unroll
                for (int k = 0; k < NS; ++k) v[k][j] += a.mS[k][f] * x[c][j];
                if (MODE == 2 && j >= 1 && j <= S) {
#pragma unroll
                    for (int o = 0; o < NOE; ++o) ev[o][j - 1] += a.mOF[o][f] * x[c][j];
                }
            }
        }
    };
    field_chunks<2, NFMAX>(a.nf, load_fields);
    // only waves whose rows p0-1 .. p0+S hold an end node take the per-row
    // end checks (a wave-uniform test)
    if (dir_end && !(p0 > 1 && p0 + S < M)) {
#pragma unroll
        for (int j = 0; j < S + 2; ++j) {
            const int p = p0 - 1 + j;
            if (p == 0 || p == M) {
#pragma unroll
                for (int k = 0; k < NS; ++k) v[k][j] = T(0);
            }
        }
    }

    // ---- local recurrences of this wave's S nodes (zero carries in) ----
    const int jm = M - p0;
    const bool slow = PER && (p0 + S - 1 > M);          // periodic wave crossing the end
    T sum[NS][S];
    T aL[NS], aR[NS], eLM[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (PER && slow) {
            if (a.kform[k]) seg_recur_I<T, S>(v[k], p0, M, d, a.w0, a.w1, w2, sum[k], aL[k], aR[k], eLM[k]);
            else seg_recur<T, S>(v[k], p0, M, false, d, g, w2, sum[k], aL[k], aR[k], eLM[k]);
        } else {
            if (a.kform[k]) seg_recur_fast_I<T, S>(v[k], d, a.w0, a.w1, w2, sum[k], aL[k], aR[k]);
            else seg_recur_fast<T, S>(v[k], d, a.gw, w2, sum[k], aL[k], aR[k]);
            eLM[k] = aL[k];
            if (dir_end && (p0 == 0 || (jm >= 0 && jm < S))) {
                T vM1 = T(0);
#pragma unroll
                for (int j = 0; j < S + 2; ++j)
                    if (j == jm) vM1 = v[k][j];            // node M-1
                seg_fix_dirichlet<T, S>(p0, M, v[k][2], vM1, d, w2, sum[k], aL[k], aR[k], eLM[k]);
            }
        }
        red[0][k][wave][lane] = aL[k];
        red[1][k][wave][lane] = aR[k];
    }
    __syncthreads();

    // sums across the waves of the tile (and, in the scan, across tiles) are
    // accumulated in FP64 and rounded once: with small nu they add up to
    // hundreds of terms of like size
    const double dS = exp(-a.nu * (double)S);
    if (MODE == 1) {
        // the tile's aggregates; E^L at node M from the wave holding it
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T *tk = tab + ((size_t)tile * MAXS + k) * (3 * 64);
            if (wave == 0) {
                double c = 0.0, cr = 0.0;
                for (int w = 0; w < W; ++w) c = dS * c + (double)red[0][k][w][lane];
                for (int w = W - 1; w >= 0; --w) cr = dS * cr + (double)red[1][k][w][lane];
                tk[lane] = (T)c;
                tk[64 + lane] = (T)cr;
            }
            if (jm >= 0 && jm < S) {
                double c = 0.0;
                for (int w = 0; w < wave; ++w) c = dS * c + (double)red[0][k][w][lane];
                tk[128 + lane] = (T)((double)eLM[k] + exp(-a.nu * (double)(jm + 1)) * c);
            }
        }
        return;
    }

    // ---- exact carries and line-end values (written by k_exact_scan) ----
    if (wave == 0) {
        const int last = ntiles - 1;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            carry[0][k][lane] = tab[((size_t)tile * MAXS + k) * (3 * 64) + lane];
            carry[1][k][lane] = tab[((size_t)tile * MAXS + k) * (3 * 64) + 64 + lane];
            carry[2][k][lane] = tab[(size_t)k * (3 * 64) + 128 + lane];
            carry[3][k][lane] = tab[((size_t)last * MAXS + k) * (3 * 64) + 128 + lane];
        }
    }
    __syncthreads();
    T cL[NS], cR[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double c = (double)carry[0][k][lane];
        for (int w = 0; w < wave; ++w) c = dS * c + (double)red[0][k][w][lane];
        cL[k] = (T)c;
        double cr = (double)carry[1][k][lane];
        for (int w = W - 1; w > wave; --w) cr = dS * cr + (double)red[1][k][w][lane];
        cR[k] = (T)cr;
    }

    // ---- closure and epilogue ----
    bool bline = false;
    if (a.proj)
        bline = (a.pd1 && (col == 0 || col == a.pn1 - 1)) ||
                (a.pd2 && (outer == 0 || outer == a.pn2 - 1));
    // the closure's decay factors at this wave's rows, skipped (wave-uniform
    // tests) where they fall below the smallest number of the type
    const double elim = sizeof(T) == 4 ? 104.0 : 745.0;
    T ea = T(0), eb = T(0);
    if (a.nu * (double)p0 < elim) ea = expneg<T>(a.nu * (double)p0);
    if (jm >= S && a.nu * (double)(jm - (S - 1)) < elim) eb = expneg<T>(a.nu * (double)(jm - (S - 1)));
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double er0 = (double)carry[2][k][lane], elm = (double)carry[3][k][lane];
        const double A = a.K00 * er0 + a.K01 * elm;
        const double B = a.K10 * er0 + a.K11 * elm;
        if (PER && slow) seg_close<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, a.nu, d, false);
        else seg_close_fast_w<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, ea, eb, d, dir_end);
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        if (p > M) break;
        const bool z = a.proj && (bline || (dir_end && (p == 0 || p == M)));
#pragma unroll
        for (int o = 0; o < NOE; ++o) {
            T r = ev[o][j];
#pragma unroll
            for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * sum[k][j];
            (a.o[o] + blk + (int64_t)p * ls)[lo] = z ? T(0) : r;
        }
    }
}
template <typename T, int S, int W, int NS, int NO, bool PER, int NFMAX, int MODE>
__global__ void __launch_bounds__(64 * W)
k_sweep_e(const KArgs<T> a)
{
    sweep_e_body<T, S, W, NS, NO, PER, NFMAX, MODE>(a, blockIdx.x);
}

// Between the two passes: one lane per column of one column group (blockIdx.x
// over outer x column groups) and one combination (blockIdx.y), the tiles
// split into 8 contiguous blocks, one per wave.  Each wave folds its block's
// aggregates into a block aggregate (both directions), the waves combine the
// block aggregates through LDS into the carries entering their blocks, and
// each wave then walks its block again writing the exact carries in place:
// TL_t <- cTop_t, TR_t <- cBot_t, slot 2 of tile 0 <- E^R_0, slot 2 of the last
// tile <- E^L_M (the host requires two tiles or more).  Sixteen tiles' loads
// are in flight at a time; sums in FP64, each stored value rounded once.
template <typename T>
__global__ void __launch_bounds__(512)
k_exact_scan(const KArgs<T> a)
{
    constexpr int NW = 8, U = 16;
    __shared__ double blkF[NW][64], blkB[NW][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = blockIdx.y;
    const int ntiles = a.ntiles, last = ntiles - 1;
    T *tab = a.agg + (size_t)blockIdx.x * (size_t)ntiles * (MAXS * 3 * 64) + (size_t)k * (3 * 64) + lane;
    const size_t tstride = (size_t)MAXS * 3 * 64;
    const double rows = (double)a.tile_rows;
    const double dT = exp(-a.nu * rows);
    const int per = (ntiles + NW - 1) / NW;
    auto bstart = [&](int w) { return min(w * per, ntiles); };
    const int b0 = bstart(wave), b1 = bstart(wave + 1);
    // block aggregates: forward sum_t dT^(b1-1-t) TL_t, backward sum_t dT^(t-b0) TR_t
    double fa = 0.0, ba = 0.0, bp = 1.0;
    for (int t0 = b0; t0 < b1; t0 += U) {
        T x[U], y[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const size_t tt = (size_t)min(t0 + i, b1 - 1);
            x[i] = tab[tt * tstride];
            y[i] = tab[tt * tstride + 64];
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (t0 + i < b1) {
                fa = dT * fa + (double)x[i];
                ba += bp * (double)y[i];
                bp *= dT;
            }
        }
    }
    blkF[wave][lane] = fa;
    blkB[wave][lane] = ba;
    __syncthreads();
    // carries entering this block: from the blocks before it (forward) and
    // after it (backward), each block's decay dT^(its tile count)
    double cf = 0.0, cb = 0.0;
    for (int w = 0; w < wave; ++w) cf = exp(-a.nu * rows * (double)(bstart(w + 1) - bstart(w))) * cf + blkF[w][lane];
    for (int w = NW - 1; w > wave; --w) cb = exp(-a.nu * rows * (double)(bstart(w + 1) - bstart(w))) * cb + blkB[w][lane];
    // forward walk of the block: the carry entering each tile; E^L at node M
    // from the carry entering the last tile
    for (int t0 = b0; t0 < b1; t0 += U) {
        T x[U];
#pragma unroll
        for (int i = 0; i < U; ++i) x[i] = tab[(size_t)min(t0 + i, b1 - 1) * tstride];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (t0 + i < b1) {
                tab[(size_t)(t0 + i) * tstride] = (T)cf;
                if (t0 + i == last) {
                    const int M = (int)a.n - 1;
                    const T em = tab[(size_t)last * tstride + 128];
                    tab[(size_t)last * tstride + 128] =
                        (T)((double)em + exp(-a.nu * (double)(M - last * a.tile_rows + 1)) * cf);
                }
                cf = dT * cf + (double)x[i];
            }
        }
    }
    // backward walk: the carry entering each tile from below; E^R_0 after tile 0
    for (int t0 = b1 - 1; t0 >= b0; t0 -= U) {
        T y[U];
#pragma unroll
        for (int i = 0; i < U; ++i) y[i] = tab[(size_t)max(t0 - i, b0) * tstride + 64];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (t0 - i >= b0) {
                tab[(size_t)(t0 - i) * tstride + 64] = (T)cb;
                cb = dT * cb + (double)y[i];
            }
        }
    }
    if (b0 == 0 && b1 > 0) tab[128] = (T)cb;
}

// ---------------------------------------------------------------------------
// pipelined strided sweep (y or z): a workgroup walks a strip of R sub-tiles
// of WS = W*S rows down 64 columns
// ---------------------------------------------------------------------------
// The forward carry entering a sub-tile is exact (the strip is walked in
// order).  The backward carry entering sub-tile t is the backward aggregate of
// sub-tile t+1, whose loads and local recurrences run one step ahead; what
// enters t+1 from below reaches t damped by d^WS <= d^K, below the rounding of
// the result (the host requires WS >= K).  Only the two strip ends take the
// decay-bounded halo sums.  The cross terms of the Dirichlet closure (weight
// e^{-nu(n-1)}) are dropped and the A (B) term is applied only within the
// first (last) sub-tiles: the host requires n >= 2 WS >= 2 K, where both are
// below the rounding as well.  NFP fields are loaded per sub-tile (op.nf <= NFP;
// missing fields read the zero row with zero coefficients).
template <typename T, int S, int NS, int NO>
struct SubTile {
    T sum[NS][S];
    T ev[NO][S];
    T aL[NS], aR[NS], eLM[NS];
};

template <typename T, int S, int W, int NS, int NO, bool PER, int NFP>
__device__ __forceinline__ void sweep_p_body(const KArgs<T> &a, const int64_t bid)
{
    static_assert(W >= 2, "the carry scans take waves 0 and 1");
    constexpr int WS = W * S;
    constexpr int HB = 4;                        // halo rows per wave and round
    __shared__ T agg[3][2][NS][W][64];           // aL, aR of every wave, 3 sub-tiles in flight
    __shared__ T endv[NS][64];                   // E^L_M of each column
    __shared__ T cLs[NS][W][64], cRs[NS][W][64]; // carries entering every wave of a sub-tile
    __shared__ T ctopS[NS][64], er0S[NS][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nstrips = a.ntiles;
    const int64_t L = bid;
    const int strip = (int)(L % nstrips);
    const int64_t rest = L / nstrips;
    const int64_t ncg = (a.nlines + 63) / 64;
    const int64_t cg = rest % ncg;
    const int64_t outer = rest / ncg;
    const int col = (int)(cg * 64) + lane;
    const bool active = col < a.nlines;
    const int n = (int)a.n, M = n - 1;
    const int64_t ls = a.ls;
    const int64_t blk = cg * 64 + outer * a.os;
    const unsigned lo = active ? (unsigned)lane : 0u;
    constexpr bool per = PER;
    constexpr bool dir_end = !PER;
    const T d = a.d, g = a.g, w2 = a.w2, gw = a.gw, dS = a.dS;
    const int K = a.halo;

    // sub-tiles [t0, t0 + R) of the line belong to this strip
    const int Tt = (n + WS - 1) / WS;
    const int base = Tt / nstrips, extra = Tt % nstrips;
    const int t0 = strip * base + (strip < extra ? strip : extra);
    const int R = base + (strip < extra ? 1 : 0);
    const int s0 = t0 * WS;
    const int s1 = ((t0 + R) * WS < n) ? (t0 + R) * WS : n;
    const bool hb_top = per || s0 > 0;
    const bool hb_bot = per || s1 < n;

    // Fields through buffer resources over the n rows of this column group
    // (the host keeps every row offset used here, n + 2 WS + 8 rows, below
    // 2^31 bytes): a row outside the line reads 0 from the range check, a
    // missing field (c >= nf) has an empty resource.
    const int rowb = (int)(ls * (int64_t)sizeof(T));
    const int lineb = n * rowb;
    const int vl = (int)lo * (int)sizeof(T);
    __amdgpu_buffer_rsrc_t rsf[NFP];
#pragma unroll
    for (int c = 0; c < NFP; ++c)
        rsf[c] = make_rsrc(c < a.nf ? a.f[c] + blk : a.f[0] + blk, c < a.nf ? lineb : 0);
    // node p as read: periodic lines wrap once (|p| stays below 2n)
    auto wrap = [&](int p) -> int {
        if (per) {
            if (p < 0) p += n;
            if (p >= n) p -= n;
        }
        return p;
    };

    // raw loads of the sub-tiles ahead (two buffers: loads run two sub-tiles
    // ahead of the finish): nodes p0-1 .. p0+S of this wave
    typedef T Raw[NFP][S + 2];
    Raw xa, xb;
    auto issue = [&](int t, Raw &xr) {
        const int p0 = s0 + t * WS + wave * S;
#pragma unroll
        for (int j = 0; j < S + 2; ++j) {
            const int off = vl + wrap(p0 - 1 + j) * rowb;
#pragma unroll
            for (int c = 0; c < NFP; ++c) xr[c][j] = buf_load<T>(rsf[c], off);
        }
    };
    // swept combinations, elementwise parts and local recurrences of sub-tile t
    auto combine = [&](int t, SubTile<T, S, NS, NO> &st, const Raw &xr) {
        const int p0 = s0 + t * WS + wave * S;
        T v[NS][S + 2];
#pragma unroll
        for (int j = 0; j < S + 2; ++j) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T x = T(0);
#pragma unroll
                for (int c = 0; c < NFP; ++c) x += a.mS[k][c] * xr[c][j];
                v[k][j] = x;
            }
            if (j >= 1 && j <= S) {
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    T x = T(0);
#pragma unroll
                    for (int c = 0; c < NFP; ++c) x += a.mOF[o][c] * xr[c][j];
                    st.ev[o][j - 1] = x;
                }
            }
        }
        // rows p0-1 .. p0+S hold no end node (a wave-uniform test) in all but
        // the end sub-tiles: only those take the per-row end checks
        if (dir_end && !(p0 > 1 && p0 + S < M)) {
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
                const int p = p0 - 1 + j;
                if (p == 0 || p == M) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) v[k][j] = T(0);
                }
            }
        }
        const int jm = M - p0;
        const bool slow = per && (p0 + S - 1 > M);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (PER && slow) {
                seg_recur<T, S>(v[k], p0, M, false, d, g, w2, st.sum[k], st.aL[k], st.aR[k], st.eLM[k]);
            } else {
                seg_recur_fast<T, S>(v[k], d, gw, w2, st.sum[k], st.aL[k], st.aR[k]);
                st.eLM[k] = st.aL[k];
                if (dir_end && (p0 == 0 || (jm >= 0 && jm < S))) {
                    T vM1 = T(0);
#pragma unroll
                    for (int j = 0; j < S + 2; ++j)
                        if (j == jm) vM1 = v[k][j];            // node M-1
                    seg_fix_dirichlet<T, S>(p0, M, v[k][2], vM1, d, w2, st.sum[k], st.aL[k], st.aR[k],
                                            st.eLM[k]);
                }
            }
            agg[t % 3][0][k][wave][lane] = st.aL[k];
            agg[t % 3][1][k][wave][lane] = st.aR[k];
        }
    };

    SubTile<T, S, NS, NO> cur, nxt;
    issue(0, xa);

    // ---- halo sums at the strip ends (cooperative over all waves) ----
    T ctop[NS], cbs[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        ctop[k] = T(0);
        cbs[k] = T(0);
    }
    if (hb_top || hb_bot) {
        const int q = (K + W - 1) / W;
        const int k0 = wave * q;
        const int k1 = (k0 + q < K) ? k0 + q : K;
        T st_[NS], sb_[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            st_[k] = T(0);
            sb_[k] = T(0);
        }
        T pw = expneg<T>(a.nu * (double)k0);
        for (int kb = k0; kb < k1; kb += HB) {
            // top: E^L forcing at rows s0-1-kk needs rows s0-kb-i, i = 0..HB+1;
            // bottom: E^R forcing at rows s1+kk needs rows s1+kb-1+i
            T xt[NFP][HB + 2], xb[NFP][HB + 2];
#pragma unroll
            for (int i = 0; i < HB + 2; ++i) {
                // a side without halo reads beyond the resource (0)
                const int ot = hb_top ? vl + wrap(s0 - kb - i) * rowb : -16;
                const int ob = hb_bot ? vl + wrap(s1 + kb - 1 + i) * rowb : -16;
#pragma unroll
                for (int c = 0; c < NFP; ++c) {
                    xt[c][i] = buf_load<T>(rsf[c], ot);
                    xb[c][i] = buf_load<T>(rsf[c], ob);
                }
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T ht[HB + 2], hv[HB + 2];
#pragma unroll
                for (int i = 0; i < HB + 2; ++i) {
                    T x = T(0), y = T(0);
#pragma unroll
                    for (int c = 0; c < NFP; ++c) {
                        x += a.mS[k][c] * xt[c][i];
                        y += a.mS[k][c] * xb[c][i];
                    }
                    // Dirichlet end rows read as 0
                    const int pt = s0 - kb - i, pb = s1 + kb - 1 + i;
                    ht[i] = (dir_end && (pt == 0 || pt == M)) ? T(0) : x;
                    hv[i] = (dir_end && (pb == 0 || pb == M)) ? T(0) : y;
                }
                T pk = pw;
#pragma unroll
                for (int i = 0; i < HB; ++i) {
                    const int kk = kb + i;
                    if (kk < k1) {
                        int rt = s0 - 1 - kk, rb = s1 + kk;
                        if (per) {
                            if (rt < 0) rt += n;
                            if (rb >= n) rb -= n;
                        }
                        st_[k] += pk * force_L(ht[i + 2], ht[i + 1], ht[i], rt, M, dir_end, g, w2);
                        sb_[k] += pk * force_R(hv[i], hv[i + 1], hv[i + 2], rb, M, dir_end, g, w2);
                    }
                    pk *= d;
                }
            }
#pragma unroll
            for (int i = 0; i < HB; ++i) pw *= d;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            agg[0][0][k][wave][lane] = st_[k];
            agg[0][1][k][wave][lane] = sb_[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T x = T(0), y = T(0);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                x += agg[0][0][k][w][lane];
                y += agg[0][1][k][w][lane];
            }
            ctop[k] = hb_top ? x : T(0);
            cbs[k] = hb_bot ? y : T(0);
        }
        __syncthreads();
    }

    combine(0, cur, xa);
    if (R > 1) issue(1, xa);
    if (R > 2) issue(2, xb);

    bool bline = false;
    if (a.proj)
        bline = (a.pd1 && (col == 0 || col == a.pn1 - 1)) ||
                (a.pd2 && (outer == 0 || outer == a.pn2 - 1));
    __amdgpu_buffer_rsrc_t rso[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) rso[o] = make_rsrc(a.o[o] + blk, lineb);

    // sub-tile t + 1 sits in buffer xa when t is even, xb when odd
    auto finish = [&](int t, Raw &xr) {
        const bool last = (t + 1 == R);
        if (!last) {
            combine(t + 1, nxt, xr);
            if (t + 3 < R) issue(t + 3, xr);
        }
        __syncthreads();

        // ---- finish sub-tile t ----
        const int st0 = s0 + t * WS;
        const int p0 = st0 + wave * S;
        const bool botAsB = per && last && s1 == n;
        // carries of every wave, computed once: wave 0 scans forward (and
        // keeps the carry into the next sub-tile), wave 1 the look-ahead
        // aggregate and backward
        if (wave == 0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T c = ctop[k];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    cLs[k][w][lane] = c;
                    c = dS * c + agg[t % 3][0][k][w][lane];
                }
                ctop[k] = c;
                ctopS[k][lane] = c;
            }
        } else if (wave == 1) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T cb;
                if (!last) {
                    T ag = T(0);
#pragma unroll
                    for (int w = W - 1; w >= 0; --w) ag = dS * ag + agg[(t + 1) % 3][1][k][w][lane];
                    if (t + 2 == R) ag += expneg<T>(a.nu * (double)(s1 - (st0 + WS))) * cbs[k];
                    cb = ag;
                } else {
                    cb = botAsB ? T(0) : cbs[k];
                }
                T cr = cb;
#pragma unroll
                for (int w = W - 1; w >= 0; --w) {
                    cRs[k][w][lane] = cr;
                    cr = dS * cr + agg[t % 3][1][k][w][lane];
                }
                er0S[k][lane] = cr;                  // E^R at node st0
            }
        }
        __syncthreads();
        T cL[NS], cR[NS], ctopn[NS], er0[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            cL[k] = cLs[k][wave][lane];
            cR[k] = cRs[k][wave][lane];
            ctopn[k] = ctopS[k][lane];
            er0[k] = er0S[k][lane];
        }
        double A[NS], B[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            A[k] = (dir_end && st0 == 0) ? a.K00 * (double)er0[k] : 0.0;
            B[k] = botAsB ? (double)d * (double)cbs[k] : 0.0;
        }
        // E^L_M when node M lies in this sub-tile or the next one
        const bool mhere = dir_end && M < st0 + WS;
        const bool mnext = dir_end && !last && M >= st0 + WS && M < st0 + 2 * WS;
        if (mhere || mnext) {
            if (mhere && wave == (M - st0) / S) {
                const int jmw = M - p0;
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    endv[k][lane] = cur.eLM[k] + expneg<T>(a.nu * (double)(jmw + 1)) * cL[k];
            }
            if (mnext && wave == (M - st0 - WS) / S) {
                const int jmw = M - (p0 + WS);
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    T c = ctopn[k];
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        if (w < wave) c = dS * c + agg[(t + 1) % 3][0][k][w][lane];
                    endv[k][lane] = nxt.eLM[k] + expneg<T>(a.nu * (double)(jmw + 1)) * c;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NS; ++k) B[k] = a.K11 * (double)endv[k][lane];
        }
        const bool slow = per && (p0 + S - 1 > M);
        // the closure's decay factors, formed only where A or B can be
        // nonzero (wave-uniform tests: the first sub-tile of a Dirichlet line,
        // the sub-tiles next to node M, the bottom of a split periodic strip)
        T ea = T(0), eb = T(0);
        if (dir_end && st0 == 0) ea = expneg<T>(a.nu * (double)p0);
        if ((botAsB || mhere || mnext) && M - p0 >= S) eb = expneg<T>(a.nu * (double)(M - p0 - (S - 1)));
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (PER && slow) seg_close<T, S>(cur.sum[k], cL[k], cR[k], A[k], B[k], p0, M, a.nu, d, false);
            else seg_close_fast_w<T, S>(cur.sum[k], cL[k], cR[k], A[k], B[k], p0, M, ea, eb, d, dir_end);
        }
        if (active) {
            // rows past node M lie beyond the output resources: the hardware
            // drops those stores
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int p = p0 + j;
                const bool z = a.proj && (bline || (dir_end && (p == 0 || p == M)));
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    T r = cur.ev[o][j];
#pragma unroll
                    for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * cur.sum[k][j];
                    buf_store<T>(z ? T(0) : r, rso[o], vl + p * rowb);
                }
            }
        }
        cur = nxt;
    };
    for (int t = 0; t < R; t += 2) {
        finish(t, xa);
        if (t + 1 < R) finish(t + 1, xb);
    }
}
template <typename T, int S, int W, int NS, int NO, bool PER, int NFP>
__global__ void __launch_bounds__(64 * W)
k_sweep_p(const KArgs<T> a)
{
    sweep_p_body<T, S, W, NS, NO, PER, NFP>(a, blockIdx.x);
}
template <typename T, int S, int W, int NS, int NO, bool PER, int NFP>
__global__ void __launch_bounds__(64 * W)
k_sweep_p_b(const KArgs<T> *__restrict__ tab, const int64_t *__restrict__ first, int nent)
{
    const int e = batch_entry(first, nent, blockIdx.x);
    sweep_p_body<T, S, W, NS, NO, PER, NFP>(tab[e], (int64_t)blockIdx.x - first[e]);
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// x lines longer than one workgroup: chunks of XC_C = 64 XC_WPL XC_S nodes,
// one workgroup per (line, chunk), exact across chunks (Dirichlet lines)
// ---------------------------------------------------------------------------
// Pass 1 (MODE 1) sweeps a chunk with zero carries at its ends and writes the
// chunk's forward aggregate (E^L at its last node), its backward aggregate
// (E^R at its first node) and, in the chunk holding node M, E^L at M, into
// the table the exact strided sweeps use, a line taking the place of a column:
// ((line/64 * nchunks + chunk) * MAXS + k) * 3 * 64 + slot * 64 + line % 64.
// k_exact_scan folds them into the carries entering every chunk and the two
// line ends; pass 2 (MODE 2) sweeps the chunk again with those carries, forms
// the closure from the line ends and writes the outputs.
constexpr int XC_S = 8, XC_WPL = 8, XC_C = 64 * XC_WPL * XC_S;
template <typename T, int NS, int NO, int NFMAX, int MODE>
__device__ __forceinline__ void sweep_xc_body(const KArgs<T> &a, const int64_t bid)
{
    constexpr int S = XC_S, WPL = XC_WPL, C = XC_C;
    constexpr int NT = 64 * WPL;
    constexpr int NPAD = NT * (S + 1);
    constexpr int NOE = (MODE == 2) ? NO : 1;
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);          // [NS][NPAD]
    __shared__ T wtot[2][MAXS][WPL];
    __shared__ T halo[2][MAXS];                       // combinations at nodes cs - 1 and cs + C

    const int t = threadIdx.x;
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nch = a.ntiles;
    const int64_t line = bid / nch;
    const int chunk = (int)(bid % nch);
    const int n = (int)a.n, M = n - 1;
    const int cs = chunk * C;                        // first node of the chunk
    const int cn = (n - cs < C) ? n - cs : C;        // nodes in the chunk
    const int64_t base = line * a.lineoff + cs;
    const T d = a.d, w2 = a.w2;
    T *tab = a.agg + (size_t)(line >> 6) * (size_t)nch * (MAXS * 3 * 64) + (int)(line & 63);

    // ---- loads of node cs + e, e = i*NT + t: combinations and field terms ----
    T sv[NS][S], ev[NOE][S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
#pragma unroll
        for (int k = 0; k < NS; ++k) sv[k][i] = T(0);
#pragma unroll
        for (int o = 0; o < NOE; ++o) ev[o][i] = T(0);
    }
    auto load_fields = [&](int f0, auto cc) {
        constexpr int CC = decltype(cc)::value;
        T x[CC][S];
#pragma unroll
        for (int c = 0; c < CC; ++c) {
            const T *src = a.f[f0 + c] + base;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const int e = i * NT + t;
                x[c][i] = src[e < cn ? e : 0];
            }
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) {
            const int f = f0 + c;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const T xv = (i * NT + t < cn) ? x[c][i] : T(0);
#pragma unroll
                for (int k = 0; k < NS; ++k) sv[k][i] += a.mS[k][f] * xv;
                if (MODE == 2) {
#pragma unroll
                    for (int o = 0; o < NOE; ++o) ev[o][i] += a.mOF[o][f] * xv;
                }
            }
        }
    };
    field_chunks<4, NFMAX>(a.nf, load_fields);
    // staging; the Dirichlet end nodes and nodes past the line read as 0
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const int e = i * NT + t;
        const int ge = cs + e;
        const int slot = (e / S) * (S + 1) + (e % S);
        const bool zero = (e >= cn) || ge == 0 || ge == M;
#pragma unroll
        for (int k = 0; k < NS; ++k) sm[k * NPAD + slot] = zero ? T(0) : sv[k][i];
    }
    // the combinations at the nodes just outside the chunk (0 at and past the
    // line ends), for the forcing of its first and last node
    if (t < 2) {
        const int gn = (t == 0) ? cs - 1 : cs + C;
        const bool in = gn >= 1 && gn < M;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T sk = T(0);
            if (in)
                for (int f = 0; f < a.nf; ++f) sk += a.mS[k][f] * a.f[f][line * a.lineoff + gn];
            halo[t][k] = sk;
        }
    }
    __syncthreads();

    // ---- recurrences over S consecutive nodes per lane (global node p0..) ----
    const int p0l = t * S, p0 = cs + p0l;
    const int jm = M - p0;
    T sum[NS][S], aL[NS], aR[NS], eLM[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const T *sk = sm + k * NPAD;
        T v[S + 2];
#pragma unroll
        for (int j = 0; j < S; ++j) v[j + 1] = sk[t * (S + 1) + j];
        v[0] = (t == 0) ? halo[0][k] : sk[(t - 1) * (S + 1) + (S - 1)];
        v[S + 1] = (t + 1 < NT) ? sk[(t + 1) * (S + 1)] : halo[1][k];
        seg_recur_fast<T, S>(v, d, a.gw, w2, sum[k], aL[k], aR[k]);
        eLM[k] = aL[k];
        if (p0 == 0 || (jm >= 0 && jm < S)) {
            const T v1 = (p0 == 0 && n > 1) ? sk[1] : T(0);
            T vM1 = T(0);
            if (jm >= 0 && jm < S) {
                const int q = M - 1 - cs;                // node M-1, local
                vM1 = (q >= 0) ? sk[(q / S) * (S + 1) + (q % S)] : halo[0][k];
            }
            seg_fix_dirichlet<T, S>(p0, M, v1, vM1, d, w2, sum[k], aL[k], aR[k], eLM[k]);
        }
    }
    // lane scan (multiplier d^S per lane), then waves through LDS
    T cL[NS], cR[NS];
    const LaneW<T> lw = lane_weights<T>(a.nu * (double)S, lane);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T xl = aL[k], xr = aR[k];
        lane_scans<T>(xl, xr, a.dpw, lw, lane);
        cL[k] = dpp_mov<0x138>(xl);              // lane - 1 (0 at lane 0)
        cR[k] = dpp_mov<0x130>(xr);              // lane + 1 (0 at lane 63)
        if (lane == 63) wtot[0][k][wave] = xl;
        if (lane == 0) wtot[1][k][wave] = xr;
    }
    __syncthreads();
    {
        const T pl = expneg<T>(a.nu * (double)S * (double)lane);
        const T pr = expneg<T>(a.nu * (double)S * (double)(63 - lane));
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T cw = T(0), cwr = T(0);
            for (int w = 0; w < wave; ++w) cw = a.dBlk * cw + wtot[0][k][w];
            for (int w = WPL - 1; w > wave; --w) cwr = a.dBlk * cwr + wtot[1][k][w];
            cL[k] += pl * cw;
            cR[k] += pr * cwr;
        }
    }
    if (MODE == 1) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            T *tk = tab + ((size_t)chunk * MAXS + k) * (3 * 64);
            if (t == 0) {
                T c = T(0), cr = T(0);
                for (int w = 0; w < WPL; ++w) c = a.dBlk * c + wtot[0][k][w];
                for (int w = WPL - 1; w >= 0; --w) cr = a.dBlk * cr + wtot[1][k][w];
                tk[0] = c;
                tk[64] = cr;
            }
            if (jm >= 0 && jm < S) tk[128] = eLM[k] + expneg<T>(a.nu * (double)(jm + 1)) * cL[k];
        }
        return;
    }

    // ---- pass 2: carries entering the chunk, line ends, closure ----
    const int last = nch - 1;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const T cinL = tab[((size_t)chunk * MAXS + k) * (3 * 64)];
        const T cinR = tab[((size_t)chunk * MAXS + k) * (3 * 64) + 64];
        cL[k] += expneg<T>(a.nu * (double)p0l) * cinL;
        cR[k] += expneg<T>(a.nu * (double)(C - p0l - S)) * cinR;
        const double er0 = (double)tab[(size_t)k * (3 * 64) + 128];
        const double elm = (double)tab[((size_t)last * MAXS + k) * (3 * 64) + 128];
        const double A = a.K00 * er0 + a.K01 * elm;
        const double B = a.K10 * er0 + a.K11 * elm;
        seg_close_fast<T, S>(sum[k], cL[k], cR[k], A, B, p0, M, a.nu, d, true);
    }
    __syncthreads();                                 // every read of the staged data is done
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T *sk = sm + k * NPAD;
#pragma unroll
        for (int j = 0; j < S; ++j) sk[t * (S + 1) + j] = sum[k][j];
    }
    __syncthreads();
    bool bline = false;
    if (a.proj) {
        const int64_t i1 = line % a.pn1, i2 = line / a.pn1;
        bline = (a.pd1 && (i1 == 0 || i1 == a.pn1 - 1)) || (a.pd2 && (i2 == 0 || i2 == a.pn2 - 1));
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const int e = i * NT + t;
        if (e < cn) {
            const int ge = cs + e;
            const int slot = (e / S) * (S + 1) + (e % S);
            T Dk[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) Dk[k] = sm[k * NPAD + slot];
            const bool z = a.proj && (bline || ge == 0 || ge == M);
#pragma unroll
            for (int o = 0; o < NOE; ++o) {
                T r = ev[o][i];
#pragma unroll
                for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * Dk[k];
                a.o[o][base + e] = z ? T(0) : r;
            }
        }
    }
}
template <typename T, int NS, int NO, int NFMAX, int MODE>
__global__ void __launch_bounds__(64 * XC_WPL)
k_sweep_xc(const KArgs<T> a)
{
    sweep_xc_body<T, NS, NO, NFMAX, MODE>(a, blockIdx.x);
}

// chained strided sweep: v1 = e1 + D s1 and y = D v1 along the same lines in
// one strip walk (2D: the two y sweeps of a step, stage 1 and stage 2)
// ---------------------------------------------------------------------------
// Level 1 is the strip recurrence above applied to s1 = sum_c mS[0][c] f_c; it
// yields v1 = sum_c mE1[c] f_c + D s1 one sub-tile at a time.  Level 2 runs the
// same recurrence on v1 two sub-tiles behind level 1 (its backward carry needs
// the next sub-tile's aggregate), so v1 never leaves the chip.  The outputs are
// out_o = fp_o + mV[o] v1 + mOD[o][0] y with fp_o = sum_c mOF[o][c] f_c (only the
// last output may have field terms).  Output 0 is folded into the level-2 sums
// (y' = y + (fp_0 +) mV[0] v1 / mOD[0][0], out_0 = mOD[0][0] y'), so a level-2
// sub-tile keeps two values per row.
//
// v1 one row below a sub-tile (needed by the forcing of its last row) is taken
// before that row's own sub-tile is finished: its forward carry is exact and
// its backward carry is the look-ahead aggregate, the same truncation
// (d^WS <= d^K) as the backward carries themselves.  A strip is walked with one
// sub-tile before and after it where it has neighbours; of those, only `roll`
// rows next to the strip hold data (the rest read 0), with zero carries at the
// walk's ends: level 1 is then exact to d^roll at the strip's first and last
// rows, level 2 to about roll * d^roll, both below the rounding (the host
// takes the smallest roll with (roll + 1) d^roll <= 2^-28).
// Periodic lines are walked as the periodic continuation (rows wrap on load);
// they have no end node.
template <typename T, int S, int NO>
struct YYLev1 {
    T sum[S];      // local sums less e1: the closure yields v1 directly
    T fp[S];       // field terms of the last output
    T aL, aR, eLM;
};
template <typename T, int S, int NO>
struct YYLev2 {
    T sum[S];      // local sums less the folded part of output 0
    T gH[S];       // output 1 without its y term (two outputs)
    T aL, aR, eLM;
};

template <typename T, int S, int W, int NO, bool PER, int NFP>
__device__ __forceinline__ void sweep_yy_body(const KArgs<T> &a, const int64_t bid)
{
    static_assert(W >= 4, "the carry scans take waves 0..3");
    constexpr int WS = W * S;
    __shared__ T agg1[3][2][W][64], agg2[3][2][W][64];   // aL, aR of every wave
    __shared__ T cLs1[W][64], cRs1[W][64], cLs2[W][64], cRs2[W][64];
    __shared__ T vfirst[W][64], vlast[W][64];     // v1 at the first / last row of every wave
    __shared__ T ctopS1[64], er0S1[64], agS1[64], ctopS2[64], er0S2[64];
    __shared__ T endv1[64], endv2[64], peekS[2][64];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nstrips = a.ntiles;
    const int64_t L = bid;
    const int strip = (int)(L % nstrips);
    const int64_t rest = L / nstrips;
    const int64_t ncg = (a.nlines + 63) / 64;
    const int64_t cg = rest % ncg;
    const int64_t outer = rest / ncg;
    const int col = (int)(cg * 64) + lane;
    const bool active = col < a.nlines;
    const int n = (int)a.n;
    constexpr bool dir_end = !PER;
    const int M = PER ? (1 << 30) : n - 1;     // no end node on a periodic line
    const int64_t ls = a.ls;
    const int64_t blk = cg * 64 + outer * a.os;
    const unsigned lo = active ? (unsigned)lane : 0u;
    const T d = a.d, w2 = a.w2, gw = a.gw, dS = a.dS;

    // output sub-tiles [t0, t0 + R) of this strip inside a walk of Rw sub-tiles
    const int Tt = (n + WS - 1) / WS;
    const int base = Tt / nstrips, extra = Tt % nstrips;
    const int t0 = strip * base + (strip < extra ? strip : extra);
    const int R = base + (strip < extra ? 1 : 0);
    const int s0 = t0 * WS, se = (t0 + R) * WS;
    const int pre = (PER || s0 > 0) ? 1 : 0;
    const int post = (PER || se < n) ? 1 : 0;
    const int Rw = pre + R + post;
    const int wst = s0 - pre * WS;               // first row of the walk
    const int rlo = pre ? s0 - a.roll : -(1 << 30);
    const int rhi = post ? se + a.roll : (1 << 30);

    // buffer resources over the n rows of this column group: rows outside the
    // line (Dirichlet) and rows outside [rlo, rhi) read 0; the host keeps every
    // offset formed here below 2^31 bytes
    const int rowb = (int)(ls * (int64_t)sizeof(T));
    const int lineb = n * rowb;
    const int vl = (int)lo * (int)sizeof(T);
    // Dirichlet lines: the load resources cover only the rows of the line
    // that hold data for this walk, [wlo, whi); rows before them (negative
    // offsets), after them, and every row past the walk fall outside and read
    // 0, so the loads need no per-row choice of resource.  Periodic lines wrap
    // rows and keep the choice below.
    const int wlo = PER ? 0 : (rlo > 0 ? rlo : 0);
    const int whi = PER ? n : (rhi < n ? rhi : n);
    __amdgpu_buffer_rsrc_t rsf[NFP];
#pragma unroll
    for (int c = 0; c < NFP; ++c)
        rsf[c] = make_rsrc((c < a.nf ? a.f[c] : a.f[0]) + blk + (int64_t)wlo * ls,
                           c < a.nf ? (whi - wlo) * rowb : 0);
    __amdgpu_buffer_rsrc_t rso[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) rso[o] = make_rsrc(a.o[o] + blk, lineb);
    // periodic lines wrap once (|p| < 2n); branch-free, so that no load sits
    // under a branch
    auto wrap = [&](int p) -> int {
        if (PER) p += n * ((int)(p < 0) - (int)(p >= n));
        return p;
    };

    typedef T Raw[NFP][S + 2];
    Raw xa, xb;
    // loads of sub-tile t (none beyond the walk, none outside [rlo, rhi)).
    // Issued without a branch or a per-lane select: a load under a branch makes
    // the compiler wait for every load in flight where the branch rejoins,
    // which would serialise the prefetch.  A row without data is read through
    // an empty resource (no memory access, value 0), chosen by a scalar select.
    const __amdgpu_buffer_rsrc_t rnone = make_rsrc(a.f[0] + blk, 0);
    auto issue = [&](int t, Raw &xr) {
        const int p0 = wst + t * WS + wave * S;
        if (PER) {
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
                const int r = p0 - 1 + j;
                const bool ok = t < Rw && r >= rlo && r < rhi;
                const int off = vl + wrap(r) * rowb;
#pragma unroll
                for (int c = 0; c < NFP; ++c) xr[c][j] = buf_load<T>(ok ? rsf[c] : rnone, off);
            }
        } else {
            // rows past the walk lie at or beyond whi: rhi <= the walk's end
            // when the strip has a successor, else whi = n
            const int off0 = vl + (p0 - 1 - wlo) * rowb;
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
#pragma unroll
                for (int c = 0; c < NFP; ++c) xr[c][j] = buf_load<T>(rsf[c], off0 + j * rowb);
            }
        }
    };

    // local recurrences of one wave's S rows from values v[0..S+1] of rows
    // p0-1 .. p0+S (Dirichlet end rows already read as 0)
    auto local = [&](const T (&v)[S + 2], int p0, T (&sum)[S], T &aL, T &aR, T &eLM) {
        seg_recur_fast<T, S>(v, d, gw, w2, sum, aL, aR);
        eLM = aL;
        const int jm = M - p0;
        if (dir_end && (p0 == 0 || (jm >= 0 && jm < S))) {
            T vM1 = T(0);
#pragma unroll
            for (int j = 0; j < S + 2; ++j)
                if (j == jm) vM1 = v[j];                  // node M-1
            seg_fix_dirichlet<T, S>(p0, M, v[2], vM1, d, w2, sum, aL, aR, eLM);
        }
    };

    // level 1, sub-tile t: combinations and local recurrences; wave 0 leaves
    // e1 - F^L at the sub-tile's first row for the look-ahead value of v1
    // rows p0-1 .. p0+S of a wave hold no end node of a Dirichlet line (the
    // usual case): a wave-uniform test that spares the per-row end checks
    auto inner_rows = [&](int p0) -> bool { return !dir_end || (p0 > 1 && p0 + S < M); };

    auto combine1 = [&](int t, YYLev1<T, S, NO> &st, const Raw &xr) {
        const int p0 = wst + t * WS + wave * S;
        T v[S + 2], e1[S];
        auto rows = [&](auto inner) {
#pragma unroll
            for (int j = 0; j < S + 2; ++j) {
                T x = T(0);
#pragma unroll
                for (int c = 0; c < NFP; ++c) x += a.mS[0][c] * xr[c][j];
                const int p = p0 - 1 + j;
                if constexpr (decltype(inner)::value) v[j] = x;
                else v[j] = (dir_end && (p == 0 || p == M)) ? T(0) : x;
                if (j >= 1 && j <= S) {
                    T e = T(0), f = T(0);
#pragma unroll
                    for (int c = 0; c < NFP; ++c) {
                        e += a.mE1[c] * xr[c][j];
                        f += a.mOF[NO - 1][c] * xr[c][j];
                    }
                    e1[j - 1] = e;
                    st.fp[j - 1] = f;
                }
            }
        };
        if (inner_rows(p0)) rows(ic<1>{});
        else rows(ic<0>{});
        local(v, p0, st.sum, st.aL, st.aR, st.eLM);
        // D = -(sum + carries + closure): subtracting e1 here makes the closure
        // return v1 = e1 + D (0 at Dirichlet end nodes, which level 2 reads as 0)
#pragma unroll
        for (int j = 0; j < S; ++j) st.sum[j] -= e1[j];
        agg1[t % 3][0][wave][lane] = st.aL;
        agg1[t % 3][1][wave][lane] = st.aR;
        if (wave == 0) peekS[t & 1][lane] = e1[0] - (w2 * (v[2] - v[1]) - gw * (v[1] - v[0]));
    };

    // carries entering every wave of sub-tile t, computed once: wave F scans
    // forward from the running carry ctop, wave F+1 backward from the
    // look-ahead aggregate of sub-tile t+1 (zero beyond the walk)
    T ctop1 = T(0), ctop2 = T(0);
    auto scan = [&](int t, T (&agg)[3][2][W][64], T (&cLs)[W][64], T (&cRs)[W][64], T &ctop,
                    T *ctopS, T *er0S, T *agS, int F) {
        if (wave == F) {
            T c = ctop;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                cLs[w][lane] = c;
                c = dS * c + agg[t % 3][0][w][lane];
            }
            ctop = c;
            ctopS[lane] = c;
        } else if (wave == F + 1) {
            T cb = T(0);
            if (t + 1 < Rw) {
#pragma unroll
                for (int w = W - 1; w >= 0; --w) cb = dS * cb + agg[(t + 1) % 3][1][w][lane];
            }
            if (agS) agS[lane] = cb;
            T cr = cb;
#pragma unroll
            for (int w = W - 1; w >= 0; --w) {
                cRs[w][lane] = cr;
                cr = dS * cr + agg[t % 3][1][w][lane];
            }
            er0S[lane] = cr;
        }
    };

    // closure of sub-tile t of one level (in place: sum <- D); returns the
    // line's B coefficient when node M lies in t + 1 (else 0).  A (B) is taken
    // only where node 0 (M) is a row of the walk that holds data; elsewhere its
    // weight on the strip's rows is below d^roll.
    auto close = [&](int t, T (&sum)[S], T eLMcur, T eLMnext, T (&agg)[3][2][W][64],
                     T (&cLs)[W][64], T (&cRs)[W][64], const T *ctopS, const T *er0S, T *endv) -> double {
        const int st0 = wst + t * WS;
        const int p0 = st0 + wave * S;
        const T cL = cLs[wave][lane], cR = cRs[wave][lane];
        // the closure's terms and their decay factors, formed only in the
        // sub-tiles that hold a line end (wave-uniform tests)
        const bool aon = dir_end && st0 == 0 && pre == 0;
        const double A = aon ? a.K00 * (double)er0S[lane] : 0.0;
        T ea = T(0), eb = T(0);
        if (aon) ea = expneg<T>(a.nu * (double)p0);
        double B = 0.0;
        const bool mhere = dir_end && M < rhi && M >= st0 && M < st0 + WS;
        const bool mnext = dir_end && M < rhi && t + 1 < Rw && M >= st0 + WS && M < st0 + 2 * WS;
        if (mhere || mnext) {
            if (mhere && wave == (M - st0) / S)
                endv[lane] = eLMcur + expneg<T>(a.nu * (double)(M - p0 + 1)) * cL;
            if (mnext && wave == (M - st0 - WS) / S) {
                T c = ctopS[lane];
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (w < wave) c = dS * c + agg[(t + 1) % 3][0][w][lane];
                endv[lane] = eLMnext + expneg<T>(a.nu * (double)(M - (p0 + WS) + 1)) * c;
            }
            __syncthreads();
            B = a.K11 * (double)endv[lane];
            if (M - p0 >= S) eb = expneg<T>(a.nu * (double)(M - p0 - (S - 1)));
        }
        seg_close_fast_w<T, S>(sum, cL, cR, A, B, p0, M, ea, eb, d, dir_end);
        return mnext ? B : 0.0;
    };

    // sub-tile states in two-slot rings indexed by the parity of the sub-tile
    // (static: the step loop is unrolled by two), so no state is copied
    YYLev1<T, S, NO> L1[2];         // level 1: sub-tiles t and t+1
    YYLev2<T, S, NO> L2[2];         // level 2: sub-tiles t-1 and t (t-2 until it retires)
    T prevlast = T(0);              // wave 0: v1 at the row above its sub-tile

    issue(0, xa);
    issue(1, xb);
    combine1(0, L1[0], xa);
    issue(2, xa);

    // step t: level 1 finishes sub-tile t, level 2 combines t and finishes t-2;
    // xr holds the loads of sub-tile t+1 and receives those of t+3 (loads run
    // two sub-tiles ahead)
    auto step = [&](int t, Raw &xr, auto parity) {
        constexpr int P0 = decltype(parity)::value, P1 = 1 - P0;   // parities of t and t+1
        YYLev1<T, S, NO> &c1 = L1[P0], &n1 = L1[P1];
        YYLev2<T, S, NO> &q0 = L2[P0], &q1 = L2[P1], &q2 = L2[P0];   // t-2, t-1, t
        if (t + 1 < Rw) combine1(t + 1, n1, xr);
        issue(t + 3, xr);
        __syncthreads();
        if (t < Rw) scan(t, agg1, cLs1, cRs1, ctop1, ctopS1, er0S1, agS1, 0);
        if (t >= 2 && t - 2 < Rw) scan(t - 2, agg2, cLs2, cRs2, ctop2, ctopS2, er0S2, nullptr, 2);
        __syncthreads();
        // level 2 retires sub-tile t-2 before level 1 hands over sub-tile t
        const int t2 = t - 2;
        if (t2 >= pre && t2 < pre + R) {
            (void)close(t2, q0.sum, q0.eLM, q1.eLM, agg2, cLs2, cRs2, ctopS2, er0S2, endv2);
            if (active) {
                // rows past the line end lie beyond the output resources:
                // the hardware drops those stores
                const int p0 = wst + t2 * WS + wave * S;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const int p = p0 + j;
                    buf_store<T>(a.mOD[0][0] * q0.sum[j], rso[0], vl + p * rowb);
                    if (NO == 2) buf_store<T>(q0.gH[j] + a.mOD[NO - 1][0] * q0.sum[j], rso[NO - 1], vl + p * rowb);
                }
            }
        }
        T pk = T(0);
        if (t < Rw) {
            const double Bn = close(t, c1.sum, c1.eLM, n1.eLM, agg1, cLs1, cRs1, ctopS1, er0S1, endv1);
            vfirst[wave][lane] = c1.sum[0];
            vlast[wave][lane] = c1.sum[S - 1];
            // v1 at the first row of sub-tile t+1 (0 beyond the walk, at M and beyond)
            const int ptop = wst + (t + 1) * WS;
            if (wave == W - 1 && t + 1 < Rw && !(dir_end && ptop >= M)) {
                pk = peekS[(t + 1) & 1][lane] - (d * ctopS1[lane] + agS1[lane]);
                if (Bn != 0.0) pk -= (T)(Bn * exp(-a.nu * (double)(M - ptop)));
            }
        }
        __syncthreads();
        if (t < Rw) {
            const int p0 = wst + t * WS + wave * S;
            T v[S + 2];
            v[0] = (wave == 0) ? prevlast : vlast[wave > 0 ? wave - 1 : 0][lane];
#pragma unroll
            for (int j = 0; j < S; ++j) v[j + 1] = c1.sum[j];            // v1
            v[S + 1] = (wave == W - 1) ? pk : vfirst[wave < W - 1 ? wave + 1 : W - 1][lane];
            if (!inner_rows(p0)) {
#pragma unroll
                for (int j = 0; j < S + 2; ++j) {
                    const int p = p0 - 1 + j;
                    if (p <= 0 || p >= M) v[j] = T(0);
                }
            }
            local(v, p0, q2.sum, q2.aL, q2.aR, q2.eLM);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const T v1 = c1.sum[j];
                if (NO == 2) {
                    q2.sum[j] -= a.ykv * v1;
                    q2.gH[j] = c1.fp[j] + a.ykh * v1;
                } else {
                    q2.sum[j] -= a.ykv * v1 + a.yk0 * c1.fp[j];
                }
            }
            agg2[t % 3][0][wave][lane] = q2.aL;
            agg2[t % 3][1][wave][lane] = q2.aR;
            if (wave == 0) prevlast = vlast[W - 1][lane];
        }
    };
    for (int t = 0; t < Rw + 2; t += 2) {
        step(t, xb, ic<0>{});
        step(t + 1, xa, ic<1>{});      // a step past the walk does nothing
    }
}
template <typename T, int S, int W, int NO, bool PER, int NFP>
__global__ void __launch_bounds__(64 * W)
k_sweep_yy(const KArgs<T> a)
{
    sweep_yy_body<T, S, W, NO, PER, NFP>(a, blockIdx.x);
}
template <typename T, int S, int W, int NO, bool PER, int NFP>
__global__ void __launch_bounds__(64 * W)
k_sweep_yy_b(const KArgs<T> *__restrict__ tab, const int64_t *__restrict__ first, int nent)
{
    const int e = batch_entry(first, nent, blockIdx.x);
    sweep_yy_body<T, S, W, NO, PER, NFP>(tab[e], (int64_t)blockIdx.x - first[e]);
}

// ---------------------------------------------------------------------------
// elementwise z = a x + b y
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *x, T b, const T *y, T *z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) z[k] = a * x[k] + b * y[k];
}

// ---------------------------------------------------------------------------
// host side: launch dispatch
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// launch configurations (cfg id -> template parameters)
// ---------------------------------------------------------------------------
struct XCfg { int S, WPL; };
struct SCfg { int S, W; };
constexpr XCfg kXCfg[] = {{2, 1}, {4, 1}, {8, 1}, {16, 1}, {16, 2}, {16, 4}, {8, 8}, {16, 8}, {8, 2}, {8, 4},
                          {16, 16}};
constexpr SCfg kSCfg[] = {{16, 16}, {16, 8}, {8, 16}, {8, 8}, {4, 16}, {16, 4}};
constexpr int NXCFG = sizeof(kXCfg) / sizeof(kXCfg[0]);
constexpr int NSCFG = sizeof(kSCfg) / sizeof(kSCfg[0]);
// pipelined strided configurations: S, W and the number of workgroups aimed at
// (strips per line = target / column groups, at least 2 sub-tiles per strip)
struct PCfg { int S, W, target; };
constexpr PCfg kPCfg[] = {{8, 16, 256}, {16, 8, 512}, {8, 8, 512}, {8, 16, 512}, {16, 8, 256}, {4, 16, 256}};
constexpr int NPCFG = sizeof(kPCfg) / sizeof(kPCfg[0]);
// exact two-pass strided configurations (tile shapes, S x W rows per tile)
constexpr SCfg kECfg[] = {{16, 16}, {8, 16}, {16, 8}, {8, 8}};
constexpr int NECFG = sizeof(kECfg) / sizeof(kECfg[0]);
// chained strided configurations (same fields as PCfg)
constexpr PCfg kYCfg[] = {{8, 8, 256}, {4, 16, 256}, {8, 8, 512}, {4, 16, 512}, {4, 8, 256}};
constexpr int NYCFG = sizeof(kYCfg) / sizeof(kYCfg[0]);

// A batched launch: entry e of the device table tab (KArgs<T>[nent]) runs on
// workgroups [first[e], first[e+1]) of a grid of `blocks` workgroups
// (first[0] = 0, first[nent] = blocks; device memory).  Every entry shares the
// kernel instantiation chosen by the dispatch arguments.
struct BatchTab {
    const void *tab;
    const int64_t *first;
    int nent;
    int64_t blocks;
};

// one per (dtype, direction class): launch a prepared KArgs with config id
// `id` and (swept, output) counts encoded as nsno = 10*ns + no, or a batched
// table (bt != nullptr; k then only selects the instantiation)
// _n4: field loop unrolled with static indices (op.nf <= 4); _n16: runtime loop
hipError_t dispatch_x_f32_n4(const KArgs<float> &k, int64_t nlines, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_x_f64_n4(const KArgs<double> &k, int64_t nlines, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_x_f32_n16(const KArgs<float> &k, int64_t nlines, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_x_f64_n16(const KArgs<double> &k, int64_t nlines, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_s_f32_n4(const KArgs<float> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_s_f64_n4(const KArgs<double> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_s_f32_n16(const KArgs<float> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_s_f64_n16(const KArgs<double> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
// pipelined strided kernels: _p<NFP>, fields loaded per sub-tile (op.nf <= NFP)
hipError_t dispatch_p_f32_p1(const KArgs<float> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_p_f32_p2(const KArgs<float> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_p_f32_p4(const KArgs<float> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_p_f64_p1(const KArgs<double> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_p_f64_p2(const KArgs<double> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
hipError_t dispatch_p_f64_p4(const KArgs<double> &k, int nsno, int id, const BatchTab *bt, hipStream_t st);
// exact two-pass strided kernels: both passes of one sweep (k.agg set)
hipError_t dispatch_e_f32_n4(const KArgs<float> &k, int nsno, int id, hipStream_t st);
hipError_t dispatch_e_f64_n4(const KArgs<double> &k, int nsno, int id, hipStream_t st);
hipError_t dispatch_e_f32_n16(const KArgs<float> &k, int nsno, int id, hipStream_t st);
hipError_t dispatch_e_f64_n16(const KArgs<double> &k, int nsno, int id, hipStream_t st);
// chunked exact x kernels (lines longer than one workgroup, k.agg set)
hipError_t dispatch_xc_f32_n4(const KArgs<float> &k, int nsno, hipStream_t st);
hipError_t dispatch_xc_f64_n4(const KArgs<double> &k, int nsno, hipStream_t st);
hipError_t dispatch_xc_f32_n16(const KArgs<float> &k, int nsno, hipStream_t st);
hipError_t dispatch_xc_f64_n16(const KArgs<double> &k, int nsno, hipStream_t st);
// chained strided kernels (FP32, op.nf <= 3, one or two outputs)
hipError_t dispatch_yy_f32(const KArgs<float> &k, int no, int id, const BatchTab *bt, hipStream_t st);

}  // namespace molt
