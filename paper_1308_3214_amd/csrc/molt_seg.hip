// Sweeps over the line objects of an embedded boundary (Sec. 4.3): every
// maximal run of inside nodes of a grid line, closed by the two boundary
// points where the line crosses the curve.  One workgroup per line object: the
// object's nodes are staged through LDS, every lane runs the E = I - v/2
// recurrences over S consecutive nodes (uniform cells inside, the end cells of
// widths theta*h through per-object FP64 forcing coefficients), lane and wave
// carries are scanned exactly (multiplier d^S), and the per-object 2x2 closure
// enforces L^{-1}v = 0 at the two boundary points.  Outputs follow the same
// linear prologue / epilogue as the box sweeps (SweepOp).
#include "molt_sweep.h"

namespace molt {
namespace {

template <typename T>
struct SegArgs {
    const T *f[MAXF];
    T *o[MAXO];
    T mS[MAXS][MAXF];
    T mOF[MAXO][MAXF];
    T mOD[MAXO][MAXS];
    int nf;
    const SegRec *rec;
    int64_t seg0;        // first record of this launch
    int64_t pstride;     // element stride along the line
    T d, g, w2, gw, dS, dBlk;
    T dpw[6];            // d^{S 2^i}, i < 6: the lane scan's multipliers
    double nu;
};

// Forcing of the two recurrences at node p of an object of m inside nodes
// (vm, v0, vp = values at p-1, p, p+1; outside the object 0).
template <typename T>
__device__ __forceinline__ T obj_force_L(T vm, T v0, T vp, int p, int m, const T *cf, T g, T w2)
{
    if (p >= m) return T(0);
    if (m == 1) return cf[SEG_AL0] * v0;
    if (p == 0) return cf[SEG_AL0] * v0 + cf[SEG_AL1] * vp;
    if (p == m - 1) return cf[SEG_BL0] * vm + cf[SEG_BL1] * v0;
    return w2 * ((vp - v0) - (v0 - vm)) - g * (v0 - vm);
}
template <typename T>
__device__ __forceinline__ T obj_force_R(T vm, T v0, T vp, int p, int m, const T *cf, T g, T w2)
{
    if (p >= m) return T(0);
    if (m == 1) return cf[SEG_AR0] * v0;
    if (p == 0) return cf[SEG_AR0] * v0 + cf[SEG_AR1] * vp;
    if (p == m - 1) return cf[SEG_BR0] * vm + cf[SEG_BR1] * v0;
    return w2 * ((vp - v0) - (v0 - vm)) + g * (vp - v0);
}

template <typename T, int S>
__device__ __forceinline__ void obj_recur(const T (&v)[S + 2], int p0, int m, const T *cf, T d, T g,
                                          T w2, T (&sum)[S], T &aL, T &aR, T &eLast)
{
    T e = T(0);
    eLast = T(0);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int p = p0 + j;
        e = d * e + obj_force_L(v[j], v[j + 1], v[j + 2], p, m, cf, g, w2);
        sum[j] = e;
        if (p == m - 1) eLast = e;
    }
    aL = e;
    e = T(0);
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
        e = d * e + obj_force_R(v[j], v[j + 1], v[j + 2], p0 + j, m, cf, g, w2);
        sum[j] += e;
    }
    aR = e;
}

template <typename T, int S, int WPL, int NS, int NO>
__global__ void __launch_bounds__(64 * WPL)
k_seg_sweep(const SegArgs<T> a)
{
    constexpr int NT = 64 * WPL;
    constexpr int NPAD = NT * (S + 1);
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);          // [NS][NPAD]
    __shared__ T wtot[2][MAXS][WPL];
    __shared__ T ends[2][MAXS];

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const SegRec &rec = a.rec[a.seg0 + blockIdx.x];
    const int m = rec.m;
    const int64_t base = rec.base;
    const int64_t ps = a.pstride;
    T cf[NSEGC];
#pragma unroll
    for (int i = 0; i < NSEGC; ++i) cf[i] = (T)rec.c[i];
    const T d = a.d, g = a.g, w2 = a.w2;

    // ---- loads: node e = i*NT + t (consecutive threads, consecutive nodes) ----
    T sv[NS][S], ev[NO][S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
#pragma unroll
        for (int k = 0; k < NS; ++k) sv[k][i] = T(0);
#pragma unroll
        for (int o = 0; o < NO; ++o) ev[o][i] = T(0);
    }
    // every load of a chunk of up to four fields is issued before any value
    // is used, so that a chunk costs one memory latency, not one per field.
    // Buffer loads over the object's nodes: 32-bit offsets, and nodes past
    // the object (offsets beyond the resource) read 0 in hardware.
    const int rbytes = (int)((int64_t)m * ps * (int64_t)sizeof(T));
    const int ostep = (int)(NT * ps * (int64_t)sizeof(T));      // bytes between a lane's nodes
    const int off0 = (int)(t * ps * (int64_t)sizeof(T));
    auto load_chunk = [&](int f0, auto cc) {
        constexpr int C = decltype(cc)::value;
        T x[C][S];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const __amdgpu_buffer_rsrc_t r = make_rsrc(a.f[f0 + c] + base, rbytes);
#pragma unroll
            for (int i = 0; i < S; ++i) x[c][i] = buf_load<T>(r, off0 + i * ostep);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int f = f0 + c;
#pragma unroll
            for (int i = 0; i < S; ++i) {
#pragma unroll
                for (int k = 0; k < NS; ++k) sv[k][i] += a.mS[k][f] * x[c][i];
#pragma unroll
                for (int o = 0; o < NO; ++o) ev[o][i] += a.mOF[o][f] * x[c][i];
            }
        }
    };
    field_chunks<4, MAXF>(a.nf, load_chunk);
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const int e = i * NT + t;
        const int slot = (e / S) * (S + 1) + (e % S);
#pragma unroll
        for (int k = 0; k < NS; ++k) sm[k * NPAD + slot] = sv[k][i];
    }
    __syncthreads();

    // ---- recurrences over S consecutive nodes per lane ----
    const int p0 = t * S;
    const int jm = m - 1 - p0;                       // position of the last node in this lane
    // lanes wholly past the object force nothing (their data read 0, and the
    // node before the first of them is zeroed below): the uniform recurrence;
    // the object's end cells only in the lanes holding node 0 or node m-1
    const bool beyond = p0 >= m;
    const bool interior = ((p0 >= 1) && (p0 + S - 1 <= m - 2)) || beyond;
    // a wave wholly past the object (wave-uniform) skips the recurrences
    const bool idle = __builtin_amdgcn_readfirstlane(wave) * 64 * S >= m;
    T sum[NS][S], aL[NS], aR[NS], eLast[NS], v0s[NS], vls[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const T *sk = sm + k * NPAD;
        T v[S + 2];
#pragma unroll
        for (int j = 0; j < S; ++j) v[j + 1] = sk[t * (S + 1) + j];
        v[0] = (t > 0 && !beyond) ? sk[(t - 1) * (S + 1) + (S - 1)] : T(0);
        v[S + 1] = (t + 1 < NT) ? sk[(t + 1) * (S + 1)] : T(0);
        if (idle) {
#pragma unroll
            for (int j = 0; j < S; ++j) sum[k][j] = T(0);
            aL[k] = aR[k] = eLast[k] = T(0);
        } else if (interior) {
            seg_recur_fast<T, S>(v, d, a.gw, w2, sum[k], aL[k], aR[k]);
            eLast[k] = T(0);
        } else {
            obj_recur<T, S>(v, p0, m, cf, d, g, w2, sum[k], aL[k], aR[k], eLast[k]);
        }
        // end values of the swept data, read before the D values replace them
        v0s[k] = sk[0];
        vls[k] = sk[((m - 1) / S) * (S + 1) + ((m - 1) % S)];
    }
    T cL[NS], cR[NS];
    const LaneW<T> lw = lane_weights<T>(a.nu * (double)S, lane);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T xl = aL[k], xr = aR[k];
        lane_scans<T>(xl, xr, a.dpw, lw, lane);  // multipliers d^(S off), rounded once from FP64
        cL[k] = dpp_mov<0x138>(xl);              // lane - 1 (0 at lane 0)
        cR[k] = dpp_mov<0x130>(xr);              // lane + 1 (0 at lane 63)
        if (WPL > 1) {
            if (lane == 63) wtot[0][k][wave] = xl;
            if (lane == 0) wtot[1][k][wave] = xr;
        }
    }
    if (WPL > 1) {
        __syncthreads();
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
    // E^R at the first and E^L at the last inside node
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (p0 == 0) ends[0][k] = aR[k] + a.dS * cR[k];
        if (jm >= 0 && jm < S) ends[1][k] = eLast[k] + expneg<T>(a.nu * (double)(jm + 1)) * cL[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double IRa = rec.c[SEG_EA] * (double)ends[0][k] + rec.c[SEG_QA] * (double)v0s[k];
        const double ILb = rec.c[SEG_EB] * (double)ends[1][k] + rec.c[SEG_QB] * (double)vls[k];
        const double A = (-IRa + rec.c[SEG_MU] * ILb) * rec.c[SEG_INV];
        const double B = (-ILb + rec.c[SEG_MU] * IRa) * rec.c[SEG_INV];
        seg_close_fast<T, S>(sum[k], cL[k], cR[k], A * rec.c[SEG_EA], B * rec.c[SEG_EB], p0, m - 1,
                             a.nu, d, false);
    }
    __syncthreads();                                 // every read of the swept data is done
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T *sk = sm + k * NPAD;
#pragma unroll
        for (int j = 0; j < S; ++j) sk[t * (S + 1) + j] = sum[k][j];
    }
    __syncthreads();

    // ---- epilogue in the load layout ----
    __amdgpu_buffer_rsrc_t ro[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) ro[o] = make_rsrc(a.o[o] + base, rbytes);
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const int e = i * NT + t;
        const int slot = (e / S) * (S + 1) + (e % S);
        T Dk[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) Dk[k] = sm[k * NPAD + slot];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            T r = ev[o][i];
#pragma unroll
            for (int k = 0; k < NS; ++k) r += a.mOD[o][k] * Dk[k];
            buf_store<T>(r, ro[o], off0 + i * ostep);         // nodes past the object: dropped
        }
    }
}

// out[c][r] = in[r][c] for an R x C array (64 x 64 tiles through LDS, both
// sides coalesced); with a mask (of out's layout), outside nodes become 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_transpose(const T *__restrict__ in, T *__restrict__ out, int R, int C, const unsigned char *mask)
{
    __shared__ T tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4 threads
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = r0 + ty + 4 * i, c = c0 + tx;
        if (r < R && c < C) tile[ty + 4 * i][tx] = in[(int64_t)r * C + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int c = c0 + ty + 4 * i, r = r0 + tx;           // out row c, column r
        if (r < R && c < C) {
            const int64_t o = (int64_t)c * R + r;
            const T v = tile[tx][ty + 4 * i];
            out[o] = (mask && !mask[o]) ? T(0) : v;
        }
    }
}

// The same with 16-byte accesses on both sides (R and C multiples of 4 and
// 16-byte aligned arrays): thread t reads rows t/16 + 16 i, four columns
// 4 (t % 16) .. + 3, of a 64 x 64 tile, and writes four consecutive entries
// of the transposed rows.  Up to four arrays of the same shape in one launch:
// grid slice z transposes pair z.
struct TPairs {
    const void *in[4];
    void *out[4];
};

template <typename T>
__global__ void __launch_bounds__(256)
k_transpose4(const TPairs pr, int R, int C, const unsigned char *mask)
{
    typedef T v4 __attribute__((ext_vector_type(4)));
    const T *__restrict__ in = static_cast<const T *>(pr.in[blockIdx.z]);
    T *__restrict__ out = static_cast<T *>(pr.out[blockIdx.z]);
    __shared__ T tile[64][65];
    const int t = threadIdx.x;
    const int tr = t >> 4, tc = (t & 15) * 4;
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + tr + 16 * i, c = c0 + tc;
        if (r < R && c < C) {
            const v4 x = *reinterpret_cast<const v4 *>(in + (int64_t)r * C + c);
            tile[tr + 16 * i][tc + 0] = x[0];
            tile[tr + 16 * i][tc + 1] = x[1];
            tile[tr + 16 * i][tc + 2] = x[2];
            tile[tr + 16 * i][tc + 3] = x[3];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = c0 + tr + 16 * i, r = r0 + tc;            // out row c, columns r .. r+3
        if (c < C && r < R) {
            const int64_t o = (int64_t)c * R + r;
            v4 y;
            y[0] = tile[tc + 0][tr + 16 * i];
            y[1] = tile[tc + 1][tr + 16 * i];
            y[2] = tile[tc + 2][tr + 16 * i];
            y[3] = tile[tc + 3][tr + 16 * i];
            if (mask) {
                const uchar4 mk = *reinterpret_cast<const uchar4 *>(mask + o);
                if (!mk.x) y[0] = T(0);
                if (!mk.y) y[1] = T(0);
                if (!mk.z) y[2] = T(0);
                if (!mk.w) y[3] = T(0);
            }
            *reinterpret_cast<v4 *>(out + o) = y;
        }
    }
}

template <typename T>
__global__ void k_mask_zero(int64_t n, const unsigned char *mask, T *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride)
        if (!mask[k]) out[k] = T(0);
}
// The same four nodes per thread (n a multiple of 4, mask 4-byte aligned):
// one mask load per four nodes; inside nodes are not touched
template <typename T>
__global__ void k_mask_zero4(int64_t n4, const unsigned char *mask, T *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n4; k += stride) {
        const uchar4 m = reinterpret_cast<const uchar4 *>(mask)[k];
        if (!m.x) out[4 * k + 0] = T(0);
        if (!m.y) out[4 * k + 1] = T(0);
        if (!m.z) out[4 * k + 2] = T(0);
        if (!m.w) out[4 * k + 3] = T(0);
    }
}

struct SegCfg { int S, WPL; };
constexpr SegCfg kSegCfg[NSEGCLS] = {{4, 1}, {8, 1}, {8, 2}, {8, 4}, {8, 8}, {16, 8}};

template <typename T, int S, int WPL, int NS, int NO>
hipError_t run_seg(const SegArgs<T> &k, int64_t count, hipStream_t st)
{
    const size_t lds = (size_t)NS * 64 * WPL * (S + 1) * sizeof(T);
    auto fn = k_seg_sweep<T, S, WPL, NS, NO>;
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)count), dim3(64 * WPL), lds, st, k);
    return hipGetLastError();
}

template <typename T, int NS, int NO>
hipError_t dispatch_seg(const SegArgs<T> &k, int cls, int64_t count, hipStream_t st)
{
    switch (cls) {
    case 0: return run_seg<T, kSegCfg[0].S, kSegCfg[0].WPL, NS, NO>(k, count, st);
    case 1: return run_seg<T, kSegCfg[1].S, kSegCfg[1].WPL, NS, NO>(k, count, st);
    case 2: return run_seg<T, kSegCfg[2].S, kSegCfg[2].WPL, NS, NO>(k, count, st);
    case 3: return run_seg<T, kSegCfg[3].S, kSegCfg[3].WPL, NS, NO>(k, count, st);
    case 4: return run_seg<T, kSegCfg[4].S, kSegCfg[4].WPL, NS, NO>(k, count, st);
    case 5: return run_seg<T, kSegCfg[5].S, kSegCfg[5].WPL, NS, NO>(k, count, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t seg_sweep_t(const SweepOp &op, const SegTable &tab, const DirCoef &dc,
                       const void *const *fptr, void *const *optr, hipStream_t st)
{
    SegArgs<T> k{};
    for (int i = 0; i < MAXF; ++i) k.f[i] = i < op.nf ? static_cast<const T *>(fptr[i]) : nullptr;
    for (int i = 0; i < MAXO; ++i) k.o[i] = i < op.no ? static_cast<T *>(optr[i]) : nullptr;
    for (int s = 0; s < MAXS; ++s)
        for (int f = 0; f < MAXF; ++f) k.mS[s][f] = (T)op.mS[s][f];
    for (int o = 0; o < MAXO; ++o) {
        for (int f = 0; f < MAXF; ++f) k.mOF[o][f] = (T)op.mOF[o][f];
        for (int s = 0; s < MAXS; ++s) k.mOD[o][s] = (T)op.mOD[o][s];
    }
    k.nf = op.nf;
    k.rec = tab.d_rec;
    k.pstride = tab.pstride;
    k.d = (T)dc.d;
    k.g = (T)dc.g;
    k.w2 = (T)dc.w2;
    k.gw = (T)(dc.g + dc.w2);
    k.nu = dc.nu;
    const int nsno = op.ns * 10 + op.no;
    for (int c = 0; c < NSEGCLS; ++c) {
        const int64_t count = tab.cls_begin[c + 1] - tab.cls_begin[c];
        if (count <= 0) continue;
        k.seg0 = tab.cls_begin[c];
        k.dS = (T)std::exp(-dc.nu * kSegCfg[c].S);
        k.dBlk = (T)std::exp(-dc.nu * kSegCfg[c].S * 64.0);
        for (int i = 0; i < 6; ++i) k.dpw[i] = (T)std::exp(-dc.nu * kSegCfg[c].S * (double)(1 << i));
        hipError_t e;
        switch (nsno) {
        case 11: e = dispatch_seg<T, 1, 1>(k, c, count, st); break;
        case 12: e = dispatch_seg<T, 1, 2>(k, c, count, st); break;
        case 22: e = dispatch_seg<T, 2, 2>(k, c, count, st); break;
        case 23: e = dispatch_seg<T, 2, 3>(k, c, count, st); break;
        default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int seg_class_capacity(int cls)
{
    return (cls >= 0 && cls < NSEGCLS) ? 64 * kSegCfg[cls].WPL * kSegCfg[cls].S : 0;
}

hipError_t launch_seg_sweep(const SweepOp &op, const SegTable &tab, const DirCoef &dc, bool fp64,
                            const void *const *fptr, void *const *optr, hipStream_t st)
{
    if (!((op.ns == 1 && (op.no == 1 || op.no == 2)) || (op.ns == 2 && (op.no == 2 || op.no == 3))))
        return hipErrorInvalidValue;
    return fp64 ? seg_sweep_t<double>(op, tab, dc, fptr, optr, st)
                : seg_sweep_t<float>(op, tab, dc, fptr, optr, st);
}

hipError_t launch_transpose_n(bool fp64, int nt, const void *const *in, void *const *out, int64_t R,
                              int64_t C, const unsigned char *d_mask, hipStream_t st)
{
    if (nt < 1 || nt > 4) return hipErrorInvalidValue;
    const size_t es = fp64 ? 8 : 4;
    bool v4 = (R % 4 == 0) && (C % 4 == 0) && (reinterpret_cast<uintptr_t>(d_mask) % 4 == 0);
    for (int i = 0; i < nt; ++i)
        v4 = v4 && (reinterpret_cast<uintptr_t>(in[i]) % (4 * es) == 0) &&
             (reinterpret_cast<uintptr_t>(out[i]) % (4 * es) == 0);
    if (v4) {
        TPairs pr{};
        for (int i = 0; i < nt; ++i) {
            pr.in[i] = in[i];
            pr.out[i] = out[i];
        }
        const dim3 grid((unsigned)((C + 63) / 64), (unsigned)((R + 63) / 64), (unsigned)nt);
        if (fp64)
            hipLaunchKernelGGL(k_transpose4<double>, grid, dim3(256), 0, st, pr, (int)R, (int)C, d_mask);
        else
            hipLaunchKernelGGL(k_transpose4<float>, grid, dim3(256), 0, st, pr, (int)R, (int)C, d_mask);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((C + 63) / 64), (unsigned)((R + 63) / 64));
    for (int i = 0; i < nt; ++i) {
        if (fp64)
            hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, st, static_cast<const double *>(in[i]),
                               static_cast<double *>(out[i]), (int)R, (int)C, d_mask);
        else
            hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, st, static_cast<const float *>(in[i]),
                               static_cast<float *>(out[i]), (int)R, (int)C, d_mask);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_transpose(bool fp64, const void *in, void *out, int64_t R, int64_t C,
                            const unsigned char *d_mask, hipStream_t st)
{
    return launch_transpose_n(fp64, 1, &in, &out, R, C, d_mask, st);
}

hipError_t launch_mask_zero(bool fp64, int64_t n, const unsigned char *d_mask, void *out,
                            hipStream_t st)
{
    const int bs = 256;
    if (n % 4 == 0 && reinterpret_cast<uintptr_t>(d_mask) % 4 == 0) {
        const int64_t n4 = n / 4;
        int64_t nb4 = (n4 + bs - 1) / bs;
        if (nb4 > 65536) nb4 = 65536;
        if (nb4 < 1) nb4 = 1;
        if (fp64)
            hipLaunchKernelGGL(k_mask_zero4<double>, dim3((unsigned)nb4), dim3(bs), 0, st, n4, d_mask,
                               static_cast<double *>(out));
        else
            hipLaunchKernelGGL(k_mask_zero4<float>, dim3((unsigned)nb4), dim3(bs), 0, st, n4, d_mask,
                               static_cast<float *>(out));
        return hipGetLastError();
    }
    int64_t nb = (n + bs - 1) / bs;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (fp64)
        hipLaunchKernelGGL(k_mask_zero<double>, dim3((unsigned)nb), dim3(bs), 0, st, n, d_mask,
                           static_cast<double *>(out));
    else
        hipLaunchKernelGGL(k_mask_zero<float>, dim3((unsigned)nb), dim3(bs), 0, st, n, d_mask,
                           static_cast<float *>(out));
    return hipGetLastError();
}

}  // namespace molt
