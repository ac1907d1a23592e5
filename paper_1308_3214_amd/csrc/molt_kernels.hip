// Host side of the directional sweeps: argument packing, launch-configuration
// choice and validation, dispatch to the instantiation units.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "molt_internal.h"
#include "molt_sweep.h"

namespace molt {

thread_local ProfEvents g_prof;


namespace {


int g_max_lds = -1;
int max_lds()
{
    if (g_max_lds < 0) {
        int dev = 0, v = 163840;          // gfx950: 160 KB per workgroup
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            g_max_lds = v;
        else
            g_max_lds = 163840;
    }
    return g_max_lds;
}

// strips per line: the configuration's workgroup target over the column
// groups, at least two sub-tiles per strip
int64_t strips_for(const PCfg &c, int64_t Tt, int64_t groups)
{
    int64_t ns = (c.target + groups - 1) / groups;
    if (ns > Tt / 2) ns = Tt / 2;
    if (ns < 1) ns = 1;
    return ns;
}

// rows of data next to a strip in a chained walk: the smallest r with
// (r + 1) d^r <= 2^-(24 + 4) (level 2 is exact to about roll d^roll at the
// strip's ends; FP32 rounding with four bits to spare), in whole waves
int yy_roll(const DirCoef &dc, int S)
{
    const double lim = std::ldexp(1.0, -28);
    int64_t r = 1;
    while (r < ((int64_t)1 << 20) && (double)(r + 1) * std::exp(-dc.nu * (double)r) > lim) ++r;
    r = (r + S - 1) / S * S;
    return (int)r;
}

template <typename T>
void fill_common(KArgs<T> &k, const SweepOp &op, const DirCoef &dc, const void *const *fptr,
                 void *const *optr)
{
    for (int i = 0; i < MAXF; ++i) k.f[i] = i < op.nf ? static_cast<const T *>(fptr[i]) : nullptr;
    for (int i = 0; i < MAXO; ++i) k.o[i] = i < op.no ? static_cast<T *>(optr[i]) : nullptr;
    for (int s = 0; s < MAXS; ++s)
        for (int f = 0; f < MAXF; ++f) k.mS[s][f] = (T)op.mS[s][f];
    // a combination swept for L^{-1} comes back as -(I^L + I^R + closure):
    // its output weights carry the sign
    for (int o = 0; o < MAXO; ++o) {
        for (int f = 0; f < MAXF; ++f) k.mOF[o][f] = (T)op.mOF[o][f];
        for (int s = 0; s < MAXS; ++s) k.mOD[o][s] = (T)(op.kform[s] ? -op.mOD[o][s] : op.mOD[o][s]);
        k.mV[o] = (T)op.mV[o];
    }
    for (int s = 0; s < MAXS; ++s) k.kform[s] = op.kform[s];
    k.bmode = op.bmode;
    for (int i = 0; i < 2; ++i) {
        k.bt[i] = (T)op.bt[i];
        k.bk[i] = (T)op.bk[i];
        k.bend[i] = (T)op.bend[i];
    }
    k.w0 = (T)dc.w0;
    k.w1 = (T)dc.w1;
    for (int f = 0; f < MAXF; ++f) k.mE1[f] = (T)op.mE1[f];
    k.nf = op.nf;
    k.proj = op.proj;
    k.n = dc.n;
    k.periodic = dc.periodic;
    k.d = (T)dc.d;
    k.g = (T)dc.g;
    k.w2 = (T)dc.w2;
    k.gw = (T)(dc.g + dc.w2);
    k.chain = op.chain;
    k.ochain = op.chain ? static_cast<T *>(optr[op.no]) : nullptr;
    k.nu = dc.nu;
    k.K00 = dc.K[0][0];
    k.K01 = dc.K[0][1];
    k.K10 = dc.K[1][0];
    k.K11 = dc.K[1][1];
}

// Argument set, instantiation key and workgroup count of one launch.
template <typename T>
void prep_t(const SweepOp &op, const Geom &g, const DirCoef &dc, const void *const *fptr,
            void *const *optr, const int *cfg, KArgs<T> &k, SweepKey &key, int64_t &blocks,
            void *agg = nullptr)
{
    k = KArgs<T>{};
    fill_common<T>(k, op, dc, fptr, optr);
    k.agg = static_cast<T *>(agg);
    const int dir = op.dir;
    key = SweepKey{};
    key.fp64 = sizeof(T) == 8 ? 1 : 0;
    key.cfg = cfg[0];
    key.nsno = op.ns * 10 + op.no;
    key.periodic = dc.periodic ? 1 : 0;
    if (dir == 0 && cfg[0] == NXCFG) {
        // chunked x lines (exact across chunks)
        const int64_t nlines = g.n[1] * g.n[2];
        k.nlines = nlines;
        k.lineoff = g.n[0];
        k.ntiles = (int)((g.n[0] + XC_C - 1) / XC_C);
        k.tile_rows = XC_C;
        k.nblocks = nlines * k.ntiles;
        k.dS = (T)exp(-dc.nu * XC_S);
        k.dBlk = (T)exp(-dc.nu * XC_S * 64.0);
        for (int i = 0; i < 6; ++i) k.dpw[i] = (T)exp(-dc.nu * XC_S * (double)(1 << i));
        k.pn1 = g.n[1];
        k.pn2 = g.n[2];
        k.pd1 = g.ndim > 1 ? g.dirichlet[1] : 0;
        k.pd2 = g.ndim > 2 ? g.dirichlet[2] : 0;
        key.cls = 5;
        key.cfg = 0;
        key.nfb = op.nf <= 4 ? 4 : 16;
        blocks = k.nblocks;
        return;
    }
    if (dir == 0) {
        const XCfg c = kXCfg[cfg[0]];
        const int64_t nlines = g.n[1] * g.n[2];
        k.nlines = nlines;
        k.lineoff = g.n[0];
        const int vw = (sizeof(T) == 4) ? (c.S >= 4 ? 4 : c.S) : (c.S >= 2 ? 2 : 1);
        k.aligned = (g.n[0] % vw == 0) ? 1 : 0;
        for (int i = 0; i < MAXF; ++i)
            if (i < op.nf && (reinterpret_cast<uintptr_t>(fptr[i]) % (vw * sizeof(T)))) k.aligned = 0;
        for (int i = 0; i < MAXO; ++i)
            if (i < op.no && (reinterpret_cast<uintptr_t>(optr[i]) % (vw * sizeof(T)))) k.aligned = 0;
        k.dS = (T)exp(-dc.nu * c.S);
        k.dBlk = (T)exp(-dc.nu * c.S * 64.0);
        for (int i = 0; i < 6; ++i) k.dpw[i] = (T)exp(-dc.nu * c.S * (double)(1 << i));
        k.pn1 = g.n[1];
        k.pn2 = g.n[2];
        k.pd1 = g.ndim > 1 ? g.dirichlet[1] : 0;
        k.pd2 = g.ndim > 2 ? g.dirichlet[2] : 0;
        if (op.chain && (reinterpret_cast<uintptr_t>(optr[op.no]) % (vw * sizeof(T)))) k.aligned = 0;
        key.cls = 0;
        key.nfb = op.nf <= 4 ? 4 : 16;
        blocks = nlines;
        return;
    }
    k.nlines = g.n[0];
    if (dir == 1) {
        k.ls = g.n[0];
        k.os = g.n[0] * g.n[1];
        k.nouter = g.n[2];
        k.pn1 = g.n[0];
        k.pn2 = g.n[2];
        k.pd1 = g.dirichlet[0];
        k.pd2 = g.ndim > 2 ? g.dirichlet[2] : 0;
    } else {
        k.ls = g.n[0] * g.n[1];
        k.os = g.n[0];
        k.nouter = g.n[1];
        k.pn1 = g.n[0];
        k.pn2 = g.n[1];
        k.pd1 = g.dirichlet[0];
        k.pd2 = g.dirichlet[1];
    }
    k.halo = dc.halo;
    const int64_t ncg = (g.n[0] + 63) / 64;
    if (op.yy) {
        const PCfg c = kYCfg[cfg[0]];
        const int64_t WS = (int64_t)c.S * c.W;
        const int64_t Tt = (dc.n + WS - 1) / WS;
        k.ntiles = (int)strips_for(c, Tt, ncg * k.nouter);
        k.nblocks = (int64_t)k.ntiles * ncg * k.nouter;
        k.dS = (T)exp(-dc.nu * c.S);
        k.dBlk = k.dS;
        k.roll = yy_roll(dc, c.S);
        const double m00 = op.mOD[0][0];
        k.ykv = (T)(op.mV[0] / m00);
        k.yk0 = (T)(1.0 / m00);
        k.ykh = op.no > 1 ? (T)(op.mV[1] - op.mOD[1][0] * op.mV[0] / m00) : T(0);
        key.cls = 3;
        key.nsno = op.no;
        key.nfb = 3;
        blocks = k.nblocks;
        return;
    }
    if (cfg[0] >= NSCFG + NPCFG) {
        // exact two-pass tiles
        const SCfg c = kECfg[cfg[0] - NSCFG - NPCFG];
        const int64_t WS = (int64_t)c.S * c.W;
        k.ntiles = (int)((dc.n + WS - 1) / WS);
        k.nblocks = (int64_t)k.ntiles * ncg * k.nouter;
        k.dS = (T)exp(-dc.nu * c.S);
        k.dBlk = k.dS;
        k.tile_rows = (int)WS;
        key.cls = 4;
        key.cfg = cfg[0] - NSCFG - NPCFG;
        key.nfb = op.nf <= 4 ? 4 : 16;
        blocks = k.nblocks;
        return;
    }
    if (cfg[0] >= NSCFG) {
        // pipelined strips
        const PCfg c = kPCfg[cfg[0] - NSCFG];
        const int64_t WS = (int64_t)c.S * c.W;
        const int64_t Tt = (dc.n + WS - 1) / WS;
        const int64_t ns_ = strips_for(c, Tt, ncg * k.nouter);
        k.ntiles = (int)ns_;
        k.nblocks = ns_ * ncg * k.nouter;
        k.dS = (T)exp(-dc.nu * c.S);
        k.dBlk = k.dS;
        key.cls = 2;
        key.cfg = cfg[0] - NSCFG;
        key.nfb = op.nf == 1 ? 1 : op.nf == 2 ? 2 : 4;
        blocks = k.nblocks;
        return;
    }
    const SCfg c = kSCfg[cfg[0]];
    const int WS = c.S * c.W;
    k.ntiles = (int)((dc.n + WS - 1) / WS);
    k.nblocks = (int64_t)k.ntiles * ncg * k.nouter;
    k.dS = (T)exp(-dc.nu * c.S);
    k.dBlk = k.dS;
    key.cls = 1;
    key.nfb = op.nf <= 4 ? 4 : 16;
    blocks = k.nblocks;
}

// Launch of one argument set (bt == nullptr) or of a batched table; k selects
// the instantiation (its periodic flag) together with the key.
template <typename T>
hipError_t dispatch_t(const KArgs<T> &k, const SweepKey &key, int64_t blocks, const BatchTab *bt,
                      hipStream_t st)
{
    const bool small = key.nfb <= 4;
    switch (key.cls) {
    case 0:
        if constexpr (sizeof(T) == 4)
            return small ? dispatch_x_f32_n4(k, blocks, key.nsno, key.cfg, bt, st)
                         : dispatch_x_f32_n16(k, blocks, key.nsno, key.cfg, bt, st);
        else
            return small ? dispatch_x_f64_n4(k, blocks, key.nsno, key.cfg, bt, st)
                         : dispatch_x_f64_n16(k, blocks, key.nsno, key.cfg, bt, st);
    case 1:
        if constexpr (sizeof(T) == 4)
            return small ? dispatch_s_f32_n4(k, key.nsno, key.cfg, bt, st)
                         : dispatch_s_f32_n16(k, key.nsno, key.cfg, bt, st);
        else
            return small ? dispatch_s_f64_n4(k, key.nsno, key.cfg, bt, st)
                         : dispatch_s_f64_n16(k, key.nsno, key.cfg, bt, st);
    case 2:
        if constexpr (sizeof(T) == 4) {
            if (key.nfb == 1) return dispatch_p_f32_p1(k, key.nsno, key.cfg, bt, st);
            if (key.nfb == 2) return dispatch_p_f32_p2(k, key.nsno, key.cfg, bt, st);
            return dispatch_p_f32_p4(k, key.nsno, key.cfg, bt, st);
        } else {
            if (key.nfb == 1) return dispatch_p_f64_p1(k, key.nsno, key.cfg, bt, st);
            if (key.nfb == 2) return dispatch_p_f64_p2(k, key.nsno, key.cfg, bt, st);
            return dispatch_p_f64_p4(k, key.nsno, key.cfg, bt, st);
        }
    case 3:
        if constexpr (sizeof(T) == 4) return dispatch_yy_f32(k, key.nsno, key.cfg, bt, st);
        else return hipErrorInvalidValue;
    case 4:
        // two launches of their own: no batched table
        if (bt) return hipErrorInvalidValue;
        if constexpr (sizeof(T) == 4)
            return small ? dispatch_e_f32_n4(k, key.nsno, key.cfg, st) : dispatch_e_f32_n16(k, key.nsno, key.cfg, st);
        else
            return small ? dispatch_e_f64_n4(k, key.nsno, key.cfg, st) : dispatch_e_f64_n16(k, key.nsno, key.cfg, st);
    case 5:
        // chunked x lines: three launches of their own, no batched table
        if (bt) return hipErrorInvalidValue;
        if constexpr (sizeof(T) == 4)
            return small ? dispatch_xc_f32_n4(k, key.nsno, st) : dispatch_xc_f32_n16(k, key.nsno, st);
        else
            return small ? dispatch_xc_f64_n4(k, key.nsno, st) : dispatch_xc_f64_n16(k, key.nsno, st);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_t(const SweepOp &op, const Geom &g, const DirCoef &dc,
                    const void *const *fptr, void *const *optr, const int *cfg, hipStream_t st,
                    void *agg)
{
    KArgs<T> k;
    SweepKey key;
    int64_t blocks = 0;
    prep_t<T>(op, g, dc, fptr, optr, cfg, k, key, blocks, agg);
    return dispatch_t<T>(k, key, blocks, nullptr, st);
}

}  // namespace

bool config_valid(const Geom &g, const DirCoef &dc, const SweepOp &op, bool fp64, const int *cfg)
{
    const int dir = op.dir, nf = op.nf, ns = op.ns, no = op.no;
    const size_t es = fp64 ? 8 : 4;
    const bool kf = op.kform[0] || op.kform[1];
    if (op.yy) {
        if (kf) return false;
        // chained strided sweeps (FP32): at most 3 fields, one swept
        // combination, field terms only in the last output, a walk whose
        // data rows next to a strip fit one sub-tile, lines of at least two
        // sub-tiles (periodic: rows formed stay within one wrap), 32-bit
        // buffer offsets over the rows walked
        if (fp64 || dir == 0 || op.proj || op.chain) return false;
        if (nf < 1 || nf > 3 || ns != 1 || no < 1 || no > 2) return false;
        if (op.mOD[0][0] == 0.0) return false;     // output 0 is folded into the y sums
        for (int o = 0; o + 1 < no; ++o)
            for (int f = 0; f < MAXF; ++f)
                if (op.mOF[o][f] != 0.0) return false;
        if (cfg[0] < 0 || cfg[0] >= NYCFG) return false;
        const PCfg c = kYCfg[cfg[0]];
        const int64_t WS = (int64_t)c.S * c.W;
        if (yy_roll(dc, c.S) > WS) return false;
        if (dc.n < 2 * WS + (dc.periodic ? 2 : 0)) return false;
        const int64_t ls = dir == 1 ? g.n[0] : g.n[0] * g.n[1];
        if ((dc.n + 3 * WS + 8) * ls * (int64_t)es + 64 * (int64_t)es >= ((int64_t)1 << 31)) return false;
        return true;
    }
    // (ns, no) in {(1, 1), (1, 2), (2, 1), (2, 2), (2, 3)}; (2, 1) not for the strip kernel
    if (!((ns == 1 && (no == 1 || no == 2)) || (ns == 2 && (no >= 1 && no <= 3)))) return false;
    if (dir == 0 && cfg[0] == NXCFG) {
        // chunked x lines: D sweeps of Dirichlet lines (no periodic wrap, no
        // L^{-1} or boundary-data sweeps, no chained second sweep)
        if (dc.periodic || kf || op.bmode || op.chain) return false;
        // lines of more than one chunk (the plan holds the chunk table then)
        if (g.n[0] <= XC_C) return false;
        const size_t lds = (size_t)ns * 64 * XC_WPL * (XC_S + 1) * es;
        return lds <= (size_t)max_lds();
    }
    if (dir == 0) {
        if (cfg[0] < 0 || cfg[0] >= NXCFG) return false;
        const XCfg c = kXCfg[cfg[0]];
        const int64_t cap = (int64_t)64 * c.WPL * c.S;
        if (g.n[0] > cap) return false;
        const size_t lds = (size_t)ns * 64 * c.WPL * (c.S + 1) * es;
        if (lds > (size_t)max_lds()) return false;
        return true;
    }
    if (cfg[0] < 0 || cfg[0] >= NSCFG + NPCFG + NECFG) return false;
    if (cfg[0] >= NSCFG + NPCFG) {
        // exact two-pass tiles: a line of at least two tiles (a shorter one is
        // exact in the tile kernel), at most ntiles_max(dc.n) tiles (the size
        // of the aggregate table a plan holds)
        const SCfg c = kECfg[cfg[0] - NSCFG - NPCFG];
        const int64_t WS = (int64_t)c.S * c.W;
        if (dc.n <= WS) return false;
        if (WS < EXACT_MIN_TILE) return false;
        return true;
    }
    if (cfg[0] < NSCFG && kf) {
        // tiles joined by halo sums carry the D recurrences only: a line
        // swept for L^{-1} fits one tile (else the exact two-pass sweep)
        const SCfg c = kSCfg[cfg[0]];
        if (dc.n > (int64_t)c.S * c.W) return false;
    }
    if (cfg[0] >= NSCFG) {
        // pipelined strips (D sweeps only): at most 4 fields, sub-tiles at
        // least as tall as the halo and lines of at least two sub-tiles per strip
        if (kf || (ns == 2 && no == 1)) return false;
        const PCfg c = kPCfg[cfg[0] - NSCFG];
        const int64_t WS = (int64_t)c.S * c.W;
        if (nf < 1 || nf > 4) return false;
        if (dc.halo > WS) return false;
        if (dc.n < 2 * WS) return false;
        // 32-bit buffer offsets over the rows of a column group
        const int64_t ls = dir == 1 ? g.n[0] : g.n[0] * g.n[1];
        if ((dc.n + 2 * WS + 8) * ls * (int64_t)es + 64 * (int64_t)es >= ((int64_t)1 << 31)) return false;
    }
    return true;
}

int default_config(const Geom &g, const DirCoef &dc, const SweepOp &op, bool fp64, int *cfg)
{
    const int dir = op.dir, nf = op.nf, ns = op.ns, no = op.no;
    (void)nf;
    (void)no;
    if (op.yy) {
        // the first valid configuration whose strips fill the chip (>= 256
        // workgroups), else the first valid one; 32-row sub-tiles of 8 waves
        // first (the fastest measured at 1024^2 and 4096^2 where the carry
        // length lets them in), then 64-row ones
        static const int order[] = {4, 0, 1, 2, 3};
        static_assert(NYCFG == 5, "chained configuration order out of step");
        const int64_t groups = ((g.n[0] + 63) / 64) * (dir == 1 ? g.n[2] : g.n[1]);
        int first = -1;
        for (int i : order) {
            cfg[0] = i;
            if (!config_valid(g, dc, op, fp64, cfg)) continue;
            if (first < 0) first = i;
            const PCfg c = kYCfg[i];
            const int64_t WS = (int64_t)c.S * c.W;
            const int64_t Tt = (dc.n + WS - 1) / WS;
            if (strips_for(c, Tt, groups) * groups >= 256) return 0;
        }
        if (first < 0) return -1;
        cfg[0] = first;
        return 0;
    }
    if (dir == 0) {
        const int64_t n = g.n[0];
        // smallest line capacity that holds the line, with 8 nodes per lane
        // and more waves where two capacities tie (the choice the tuner makes
        // on MI355X for FP32 and FP64 at 1024 and 4096 nodes; 16 nodes per
        // lane spill in FP64)
        static const int order[] = {0, 1, 2, 8, 9, 6, 7, 10};
        const int cnt = 8;
        for (int i = 0; i < cnt; ++i) {
            cfg[0] = order[i];
            const XCfg c = kXCfg[cfg[0]];
            if (64 * c.WPL * c.S >= n && config_valid(g, dc, op, fp64, cfg)) return 0;
        }
        // longer than any workgroup holds: chunks, exact across them
        cfg[0] = NXCFG;
        return config_valid(g, dc, op, fp64, cfg) ? 0 : -1;
    }
    // strided: the pipelined strip kernel for one swept combination, else
    // tall tiles (16 waves x 16 nodes) for FP32 single sweeps, shorter lanes
    // when more registers are live
    if (ns <= 2) {
        // only when the strips give enough workgroups to fill the chip
        cfg[0] = NSCFG + ((fp64 || ns == 2) ? 2 : 0);   // {8,16,256} FP32 one combo, else {8,8,512}
        const PCfg c = kPCfg[cfg[0] - NSCFG];
        const int64_t tiles = (dc.n + (int64_t)c.S * c.W - 1) / ((int64_t)c.S * c.W);
        const int64_t groups = ((g.n[0] + 63) / 64) * (dir == 1 ? g.n[2] : g.n[1]);
        if (groups * (tiles / 2) >= 256 && config_valid(g, dc, op, fp64, cfg)) return 0;
    }
    const int regs = (2 * ns + no) * (fp64 ? 2 : 1);
    const int tcfg = (regs <= 4) ? 0 : 2;   // {16,16} or {8,16}
    // exact two-pass tiles of 512 threads, so that two or more workgroups
    // share a CU and one's loads overlap another's recurrences and barriers:
    // {16,8} (128 rows) for one FP32 combination, else {8,8} (64 rows; the
    // fastest measured at 4096^2 for D-form FP64 and every K-form sweep)
    const int ecfg = NSCFG + NPCFG + ((regs <= 4) ? 2 : 3);
    if (op.kform[0] || op.kform[1]) {
        // L^{-1} sweeps: one tile, else the exact two-pass sweep
        cfg[0] = tcfg;
        if (config_valid(g, dc, op, fp64, cfg)) return 0;
        cfg[0] = 0;
        if (config_valid(g, dc, op, fp64, cfg)) return 0;
        cfg[0] = ecfg;
        if (config_valid(g, dc, op, fp64, cfg)) return 0;
        cfg[0] = NSCFG + NPCFG;
        return config_valid(g, dc, op, fp64, cfg) ? 0 : -1;
    }
    // carries longer than half a tile (small nu): the tile kernel's halo sums
    // would read more than the tile itself; the exact two-pass sweep reads
    // each tile twice, whatever the carry length
    const SCfg tc = kSCfg[tcfg];
    if (2 * (int64_t)dc.halo > (int64_t)tc.S * tc.W) {
        cfg[0] = ecfg;
        if (config_valid(g, dc, op, fp64, cfg)) return 0;
    }
    cfg[0] = tcfg;
    return config_valid(g, dc, op, fp64, cfg) ? 0 : -1;
}

int uniform_x_capacity(int id) { return (id >= 0 && id < NXCFG) ? kXCfg[id].S * kXCfg[id].WPL : 0; }

int config_count(const SweepOp &op)
{
    return op.yy ? NYCFG : op.dir == 0 ? NXCFG : NSCFG + NPCFG + NECFG;
}

bool config_exact(const SweepOp &op, const int *cfg)
{
    if (op.dir == 0) return !op.yy && cfg[0] == NXCFG;
    return !op.yy && cfg[0] >= NSCFG + NPCFG;
}

size_t exact_agg_bytes(const Geom &g, int dir, bool fp64)
{
    if (dir == 0) {
        // chunked x lines (only where a line exceeds one chunk)
        if (g.n[0] <= XC_C) return 0;
        const int64_t groups = (g.n[1] * g.n[2] + 63) / 64;
        const int64_t chunks = (g.n[0] + XC_C - 1) / XC_C;
        return (size_t)(groups * chunks) * MAXS * 3 * 64 * (fp64 ? 8 : 4);
    }
    if (dir < 1 || dir >= g.ndim) return 0;
    const int64_t ncg = (g.n[0] + 63) / 64;
    const int64_t nouter = dir == 1 ? g.n[2] : g.n[1];
    const int64_t ntiles = (g.n[dir] + EXACT_MIN_TILE - 1) / EXACT_MIN_TILE;
    return (size_t)(nouter * ncg * ntiles) * MAXS * 3 * 64 * (fp64 ? 8 : 4);
}

hipError_t launch_sweep(const SweepOp &op, const Geom &g, const DirCoef &dc, bool fp64,
                        const void *const *fptr, void *const *optr, const int *cfg,
                        hipStream_t st, void *agg)
{
    if (!config_valid(g, dc, op, fp64, cfg)) return hipErrorInvalidValue;
    if (config_exact(op, cfg) && !agg) return hipErrorInvalidValue;
    return fp64 ? launch_t<double>(op, g, dc, fptr, optr, cfg, st, agg)
                : launch_t<float>(op, g, dc, fptr, optr, cfg, st, agg);
}

size_t sweep_args_bytes(bool fp64) { return fp64 ? sizeof(KArgs<double>) : sizeof(KArgs<float>); }

bool sweep_prepare(const SweepOp &op, const Geom &g, const DirCoef &dc, bool fp64,
                   const void *const *fptr, void *const *optr, const int *cfg, void *args,
                   SweepKey &key, int64_t &blocks)
{
    // batched tables hold D sweeps of one launch each
    if (!config_valid(g, dc, op, fp64, cfg) || config_exact(op, cfg) || op.kform[0] || op.kform[1] ||
        op.bmode)
        return false;
    if (fp64) {
        KArgs<double> k;
        prep_t<double>(op, g, dc, fptr, optr, cfg, k, key, blocks);
        std::memcpy(args, &k, sizeof k);
    } else {
        KArgs<float> k;
        prep_t<float>(op, g, dc, fptr, optr, cfg, k, key, blocks);
        std::memcpy(args, &k, sizeof k);
    }
    return true;
}

hipError_t launch_sweep_batch(const SweepKey &key, const void *d_tab, const int64_t *d_first, int nent,
                              int64_t blocks, hipStream_t st)
{
    if (nent < 1 || blocks < 1 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    BatchTab bt{d_tab, d_first, nent, blocks};
    if (key.fp64) {
        KArgs<double> k{};
        k.periodic = key.periodic;
        return dispatch_t<double>(k, key, blocks, &bt, st);
    }
    KArgs<float> k{};
    k.periodic = key.periodic;
    return dispatch_t<float>(k, key, blocks, &bt, st);
}

hipError_t launch_axpby(bool fp64, int64_t n, double a, const void *x, double b, const void *y,
                        void *z, hipStream_t st)
{
    const int bs = 256;
    int64_t nb = (n + bs - 1) / bs;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (fp64)
        hipLaunchKernelGGL(k_axpby<double>, dim3((unsigned)nb), dim3(bs), 0, st, n, a,
                           static_cast<const double *>(x), b, static_cast<const double *>(y),
                           static_cast<double *>(z));
    else
        hipLaunchKernelGGL(k_axpby<float>, dim3((unsigned)nb), dim3(bs), 0, st, n, (float)a,
                           static_cast<const float *>(x), (float)b, static_cast<const float *>(y),
                           static_cast<float *>(z));
    return hipGetLastError();
}

}  // namespace molt
