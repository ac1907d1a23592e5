// Embedded-boundary (masked 2D) plans: the line objects of Sec. 4.3 and the
// non-commuting ADI compositions of Sec. 4 (eqs. C_def_ADI, D_def_ADI taken
// literally, since L_x^{-1} and L_y^{-1} do not commute on such a domain).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "molt_program.h"

namespace molt {
namespace {

// M_k(nu) = int_0^1 z^k e^{-nu z} dz, k = 0, 1, 2: power series for small nu
// (no cancellation), closed forms otherwise.
void moments(double nu, double M[3])
{
    if (nu < 1.0) {
        for (int k = 0; k < 3; ++k) {
            double term = 1.0, s = 0.0;       // term = (-nu)^n / n!
            for (int n = 0; n < 40; ++n) {
                s += term / (double)(n + k + 1);
                term *= -nu / (double)(n + 1);
            }
            M[k] = s;
        }
    } else {
        const double e = std::exp(-nu);
        M[0] = -std::expm1(-nu) / nu;
        M[1] = (1.0 - e * (1.0 + nu)) / (nu * nu);
        M[2] = (2.0 - e * (2.0 + 2.0 * nu + nu * nu)) / (nu * nu * nu);
    }
}

// Local integrals at a node with cells hl (left) and hr (right) against the
// quadratic through (-hl, vm), (0, v0), (hr, vp) (the reading of the local
// quadrature: the quadratic through the node and its two neighbours):
//   J^L = (alpha/2) int_{-hl}^0 e^{alpha t} q(t) dt,
//   J^R = (alpha/2) int_0^{hr} e^{-alpha t} q(t) dt.
struct Quad { double v0, b, c; };
Quad quad3(double vm, double v0, double vp, double hl, double hr)
{
    Quad q;
    q.v0 = v0;
    q.c = ((vp - v0) / hr - (v0 - vm) / hl) / (hl + hr);
    q.b = (vp - v0) / hr - q.c * hr;
    return q;
}
double jl(const Quad &q, double alpha, double hl)
{
    double M[3];
    const double nu = alpha * hl;
    moments(nu, M);
    return 0.5 * nu * (q.v0 * M[0] - q.b * hl * M[1] + q.c * hl * hl * M[2]);
}
double jr(const Quad &q, double alpha, double hr)
{
    double M[3];
    const double nu = alpha * hr;
    moments(nu, M);
    return 0.5 * nu * (q.v0 * M[0] + q.b * hr * M[1] + q.c * hr * hr * M[2]);
}

// FP64 constants of one line object (layout of SegRec::c).
void object_constants(int64_t m, double tlo, double thi, double h, double alpha, double *c)
{
    const double d = std::exp(-alpha * h);
    const double hlo = tlo * h, hhi = thi * h;
    for (int i = 0; i < NSEGC; ++i) c[i] = 0.0;
    if (m == 1) {
        // one inside node between the two boundary points (values 0)
        c[SEG_AL0] = jl(quad3(0, 1, 0, hlo, hhi), alpha, hlo) - 0.5;
        c[SEG_AR0] = jr(quad3(0, 1, 0, hlo, hhi), alpha, hhi) - 0.5;
    } else {
        // first node: left cell hlo (boundary point, value 0), right cell h
        c[SEG_AL0] = jl(quad3(0, 1, 0, hlo, h), alpha, hlo) - 0.5;
        c[SEG_AL1] = jl(quad3(0, 0, 1, hlo, h), alpha, hlo);
        c[SEG_AR0] = jr(quad3(0, 1, 0, hlo, h), alpha, h) - 0.5;
        c[SEG_AR1] = jr(quad3(0, 0, 1, hlo, h), alpha, h) + 0.5 * d;
        // last node: left cell h, right cell hhi (boundary point, value 0)
        c[SEG_BL0] = jl(quad3(1, 0, 0, h, hhi), alpha, h) + 0.5 * d;
        c[SEG_BL1] = jl(quad3(0, 1, 0, h, hhi), alpha, h) - 0.5;
        c[SEG_BR0] = jr(quad3(1, 0, 0, h, hhi), alpha, hhi);
        c[SEG_BR1] = jr(quad3(0, 1, 0, h, hhi), alpha, hhi) - 0.5;
    }
    // the boundary points: I^R(a) = e^{-alpha hlo} I^R_0 + J^R(a), with the
    // data linear on the end cell (curvature 0 at a homogeneous Dirichlet
    // point): J^R(a) = (alpha hlo / 2) M_1 v_0; I^R_0 = E^R_0 + v_0/2
    double M[3];
    const double ea = std::exp(-alpha * hlo), eb = std::exp(-alpha * hhi);
    moments(alpha * hlo, M);
    c[SEG_EA] = ea;
    c[SEG_QA] = 0.5 * ea + 0.5 * alpha * hlo * M[1];
    moments(alpha * hhi, M);
    c[SEG_EB] = eb;
    c[SEG_QB] = 0.5 * eb + 0.5 * alpha * hhi * M[1];
    // closure on [a, b], b - a = (m - 1 + tlo + thi) h
    const double L = alpha * ((double)(m - 1) * h + hlo + hhi);
    c[SEG_MU] = std::exp(-L);
    c[SEG_INV] = 1.0 / (-std::expm1(-2.0 * L));
}

int class_of(int64_t m)
{
    for (int c = 0; c < NSEGCLS; ++c)
        if (m <= seg_class_capacity(c)) return c;
    return -1;
}

}  // namespace

mol_status masked_tables(mol_plan_ *pl, bool dry, std::string &err)
{
    const int64_t nx = pl->geom.n[0], ny = pl->geom.n[1];
    const unsigned char *mk = pl->h_mask.data();
    for (int64_t i = 0; i < nx; ++i)
        if (mk[i] || mk[(ny - 1) * nx + i]) { err = "the outer ring of the mask must be 0"; return MOL_E_INVALID; }
    for (int64_t j = 0; j < ny; ++j)
        if (mk[j * nx] || mk[j * nx + nx - 1]) { err = "the outer ring of the mask must be 0"; return MOL_E_INVALID; }
    const bool hc = !pl->h_cross.empty();
    pl->table_bytes = (size_t)pl->npts;                   // device mask
    for (int dir = 0; dir < 2; ++dir) {
        const int64_t nl = dir == 0 ? ny : nx;            // lines
        const int64_t len = dir == 0 ? nx : ny;           // nodes per line
        const int64_t ls = dir == 0 ? nx : 1;             // line stride
        const int64_t ps = dir == 0 ? 1 : nx;             // node stride
        const double h = pl->desc.h[dir];
        std::vector<SegRec> recs;
        for (int64_t l = 0; l < nl; ++l) {
            int64_t i = 0;
            while (i < len) {
                if (!mk[l * ls + i * ps]) { ++i; continue; }
                int64_t j = i;
                while (j + 1 < len && mk[l * ls + (j + 1) * ps]) ++j;
                double tlo = 1.0, thi = 1.0;
                if (hc) {
                    const int64_t first = l * ls + i * ps, last = l * ls + j * ps;
                    tlo = pl->h_cross[(size_t)(2 * dir) * pl->npts + first];
                    thi = pl->h_cross[(size_t)(2 * dir + 1) * pl->npts + last];
                }
                if (!(tlo > 0.0 && tlo <= 1.0) || !(thi > 0.0 && thi <= 1.0)) {
                    err = "crossing offsets must lie in (0, 1] at every line-object end";
                    return MOL_E_INVALID;
                }
                SegRec r{};
                r.base = l * ls + i * ps;
                r.m = (int32_t)(j - i + 1);
                r.cls = class_of(r.m);
                if (r.cls < 0) {
                    err = "a line object is longer than the segment kernels support";
                    return MOL_E_UNSUPPORTED;
                }
                object_constants(r.m, tlo, thi, h, pl->alpha, r.c);
                recs.push_back(r);
                i = j + 1;
            }
        }
        // one launch per sweep: every object of the direction in the class of
        // the longest one, longest objects first
        int cmax = 0;
        for (const SegRec &r : recs) cmax = std::max(cmax, (int)r.cls);
        for (SegRec &r : recs) r.cls = cmax;
        std::stable_sort(recs.begin(), recs.end(),
                         [](const SegRec &a, const SegRec &b) { return a.m > b.m; });
        auto upload = [&](SegTable &t, const std::vector<SegRec> &rv, int64_t pstride) -> mol_status {
            t.nseg = (int64_t)rv.size();
            t.pstride = pstride;
            for (int c = 0; c <= NSEGCLS; ++c) t.cls_begin[c] = 0;
            for (const SegRec &r : rv) t.cls_begin[r.cls + 1] += 1;
            for (int c = 0; c < NSEGCLS; ++c) t.cls_begin[c + 1] += t.cls_begin[c];
            pl->table_bytes += rv.size() * sizeof(SegRec);
            if (dry || rv.empty()) return MOL_OK;
            if (hipMalloc(&t.d_rec, rv.size() * sizeof(SegRec)) != hipSuccess) {
                err = "hipMalloc of the line-object table failed";
                return MOL_E_NOMEM;
            }
            if (hipMemcpy(t.d_rec, rv.data(), rv.size() * sizeof(SegRec), hipMemcpyHostToDevice) !=
                hipSuccess) {
                err = "copy of the line-object table failed";
                return MOL_E_DEVICE;
            }
            return MOL_OK;
        };
        mol_status us = upload(pl->seg[dir], recs, ps);
        if (us != MOL_OK) return us;
        pl->nsegs[dir] = (int64_t)recs.size();
        if (dir == 1) {
            // the same objects on the transposed grid: column l, first row i at l*ny + i
            std::vector<SegRec> rt = recs;
            for (SegRec &r : rt) {
                const int64_t l = r.base % nx, i = r.base / nx;
                r.base = l * ny + i;
            }
            us = upload(pl->segT, rt, 1);
            if (us != MOL_OK) return us;
        }
    }
    // transposed copies of a y launch's fields
    pl->table_bytes += (size_t)mol_plan_::NTBUF * (size_t)pl->npts * pl->es;
    if (!dry) {
        for (int i = 0; i < mol_plan_::NTBUF; ++i) {
            if (hipMalloc(&pl->tbuf[i], (size_t)pl->npts * pl->es) != hipSuccess) {
                err = "hipMalloc of the transposed buffers failed";
                return MOL_E_NOMEM;
            }
            (void)hipMemset(pl->tbuf[i], 0, (size_t)pl->npts * pl->es);
        }
    }
    if (!dry) {
        if (hipMalloc(&pl->d_mask, (size_t)pl->npts) != hipSuccess) {
            err = "hipMalloc of the mask failed";
            return MOL_E_NOMEM;
        }
        if (hipMemcpy(pl->d_mask, mk, (size_t)pl->npts, hipMemcpyHostToDevice) != hipSuccess) {
            err = "copy of the mask failed";
            return MOL_E_DEVICE;
        }
    }
    return MOL_OK;
}

void masked_free(mol_plan_ *pl)
{
    for (int dir = 0; dir < 2; ++dir) {
        if (pl->seg[dir].d_rec) (void)hipFree(pl->seg[dir].d_rec);
        pl->seg[dir].d_rec = nullptr;
    }
    if (pl->segT.d_rec) (void)hipFree(pl->segT.d_rec);
    pl->segT.d_rec = nullptr;
    for (int i = 0; i < mol_plan_::NTBUF; ++i) {
        if (pl->tbuf[i]) (void)hipFree(pl->tbuf[i]);
        pl->tbuf[i] = nullptr;
    }
    if (pl->d_mask) (void)hipFree(pl->d_mask);
    pl->d_mask = nullptr;
}

hipError_t launch_seg_op(const SweepOp &op, const mol_plan_ *pl, const void *const *fptr,
                         void *const *optr, hipStream_t st)
{
    if (op.dir < 0 || op.dir > 1 || op.chain) return hipErrorInvalidValue;
    const int64_t nx = pl->geom.n[0], ny = pl->geom.n[1];
    if (op.dir == 1 && op.nf + op.no <= mol_plan_::NTBUF) {
        // y objects as rows of the transposed grid: coalesced sweeps; the
        // outputs come back with their outside nodes written as 0
        // (every input transposed in one launch, every output in one launch)
        const void *tf[MAXF];
        void *tin[MAXF];
        void *to[MAXO];
        const void *tout[MAXO];
        hipError_t e = hipSuccess;
        for (int f = 0; f < op.nf; ++f) tf[f] = tin[f] = pl->tbuf[f];
        for (int o = 0; o < op.no; ++o) tout[o] = to[o] = pl->tbuf[op.nf + o];
        if (op.nf > 0) e = launch_transpose_n(pl->fp64, op.nf, fptr, tin, ny, nx, nullptr, st);
        if (e == hipSuccess) e = launch_seg_sweep(op, pl->segT, pl->dc[1], pl->fp64, tf, to, st);
        if (e == hipSuccess && op.no > 0)
            e = launch_transpose_n(pl->fp64, op.no, tout, optr, nx, ny, pl->d_mask, st);
        return e;
    }
    hipError_t e = launch_seg_sweep(op, pl->seg[op.dir], pl->dc[op.dir], pl->fp64, fptr, optr, st);
    if (e != hipSuccess) return e;
    if (op.proj) {
        // user-visible outputs: every outside node written as 0
        for (int o = 0; o < op.no; ++o) {
            e = launch_mask_zero(pl->fp64, pl->npts, pl->d_mask, optr[o], st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// programs: the literal compositions on line objects
//   D w = w - L_x^{-1}(L_y^{-1} w):   t = w - D_y w;  D w = (w - t) + D_x t
//   C w = L_y^{-1}(D_x w) + L_x^{-1}(D_y w):
//         a = D_x w;  b = D_y w, la = a - D_y a;  C w = (la + b) - D_x b
// Each term of a stage is then  elem + s D_x(comb)  with (elem, comb, s).
// ---------------------------------------------------------------------------
namespace {

struct Term {
    Lin elem;      // elementwise part
    Lin comb;      // swept by the final x sweep
    double s;      // sign of that sweep
};

// the transverse work of C on the inputs cw and of D on dw (dw < 0: none);
// returns one Term per C input (in order) and then the D term.  With avg,
// D is the mean over the two orders of the directional inverses.
bool transverse(Builder &b, Program &prog, const std::vector<int> &cw, int dw,
                std::vector<Term> &terms, bool avg)
{
    // the averaged D of an input that C does not take needs that input's
    // D_x w, D_y w and L_y^{-1} D_x w too: sweep it with the C inputs
    std::vector<int> w = cw;
    if (avg && dw >= 0 && std::find(cw.begin(), cw.end(), dw) == cw.end()) w.push_back(dw);
    // x sweeps a_k = D_x w_k, two per launch
    std::vector<int> av(w.size());
    for (size_t k = 0; k < w.size(); k += 2) {
        std::vector<Lin> cmb;
        std::vector<OutSpec> outs;
        for (size_t j = k; j < std::min(w.size(), k + 2); ++j) {
            av[j] = b.new_ws();
            cmb.push_back(lin(w[j]));
            OutSpec o{};
            o.buf = av[j];
            o.dc[j - k] = 1.0;
            outs.push_back(o);
        }
        if (!b.emit(prog, 0, cmb, outs, 0)) return false;
    }
    // y sweeps: b_k = D_y w_k and la_k = a_k - D_y a_k = L_y^{-1} D_x w_k in
    // one launch per k
    std::vector<int> bv(w.size()), lv(w.size());
    for (size_t k = 0; k < w.size(); ++k) {
        const int bb = b.new_ws(), la = b.new_ws();
        bv[k] = bb;
        lv[k] = la;
        OutSpec o1{}, o2{};
        o1.buf = bb;
        o1.dc[0] = 1.0;
        o2.buf = la;
        o2.elem = lin(av[k]);
        o2.dc[1] = -1.0;
        if (!b.emit(prog, 1, {lin(w[k]), lin(av[k])}, {o1, o2}, 0)) return false;
        if (k < cw.size()) terms.push_back({lin(la) + lin(bb), lin(bb), -1.0});
    }
    if (dw >= 0) {
        // D w = w - L_x^{-1}(L_y^{-1} w) = D_y w + D_x(w - D_y w) with
        // L_y^{-1} w = w - D_y w: when w is also an input of C, its D_y w is
        // b_k above and no sweep is needed.  The other order,
        // w - L_y^{-1}(L_x^{-1} w) = D_y w + L_y^{-1} D_x w, needs no sweep
        // either, so the mean of the two is
        //   D_y w + (L_y^{-1} D_x w) / 2 + D_x(w - D_y w) / 2.
        for (size_t k = 0; k < w.size(); ++k) {
            if (w[k] != dw) continue;
            if (avg)
                terms.push_back({lin(bv[k]) + lin(lv[k], 0.5), lin(dw, 0.5) + lin(bv[k], -0.5), 1.0});
            else
                terms.push_back({lin(bv[k]), lin(dw) + lin(bv[k], -1.0), 1.0});
            return true;
        }
        const int tt = b.new_ws();
        OutSpec o{};
        o.buf = tt;
        o.elem = lin(dw);
        o.dc[0] = -1.0;
        if (!b.emit(prog, 1, {lin(dw)}, {o}, 0)) return false;
        terms.push_back({lin(dw) + lin(tt, -1.0), lin(tt), 1.0});
    }
    return true;
}

}  // namespace

// Stage schedule of Table 2 with the compositions above.
bool build_rhs_masked(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo)
{
    mol_plan_ &pl = b.pl;
    const int P = pl.desc.P;
    const double beta = pl.beta;
    const bool avg = (pl.desc.flags & MOL_SYMMETRIC_D) != 0;
    std::vector<int> v{u};
    int accbuf = -1;
    for (int p = 1; p <= P; ++p) {
        const int nin = (int)v.size();
        std::vector<Term> terms;
        // stage p: C on every input, D on the newest (p >= 2); term k carries
        // m = p - k factors of C (Table 2)
        if (!transverse(b, prog, v, p >= 2 ? v[nin - 1] : -1, terms, avg)) return false;
        const int nt = (int)terms.size();
        Lin acc_in;
        if (p == 2) acc_in = lin(v[0], b.coef(1, 1));
        else if (p >= 3) acc_in = lin(accbuf);
        if (p == P) {
            // one x sweep of the weighted sum of this stage's terms
            Lin es = acc_in, cs;
            for (int k = 0; k < nt; ++k) {
                const double c = b.coef(p, p - k);
                es = es + c * terms[k].elem;
                cs = cs + (c * terms[k].s) * terms[k].comb;
            }
            return b.emit(prog, 0, {cs}, finals(fo, es, 1.0), 1);
        }
        std::vector<int> nv(nt);
        for (int k = 0; k < nt; ++k) nv[k] = b.new_ws();
        const bool need_acc = (P >= 3);
        const int newacc = need_acc ? b.new_ws() : -1;
        Lin acc_done = acc_in;
        for (int k = 0; k < nt; k += 2) {
            const int k1 = std::min(nt, k + 2);
            std::vector<Lin> cmb;
            std::vector<OutSpec> outs;
            for (int j = k; j < k1; ++j) {
                cmb.push_back(terms[j].comb);
                OutSpec o{};
                o.buf = nv[j];
                o.elem = terms[j].elem;
                o.dc[j - k] = terms[j].s;
                outs.push_back(o);
            }
            if (k1 == nt && need_acc) {
                OutSpec o{};
                o.buf = newacc;
                o.elem = acc_done;
                for (int j = k; j < k1; ++j) {
                    const double c = b.coef(p, p - j);
                    o.elem = o.elem + c * terms[j].elem;
                    o.dc[j - k] = c * terms[j].s;
                }
                outs.push_back(o);
            }
            if (!b.emit(prog, 0, cmb, outs, 0)) return false;
            for (int j = k; j < k1; ++j) acc_done = acc_done + lin(nv[j], b.coef(p, p - j));
        }
        v = nv;
        accbuf = newacc;
    }
    return true;
}

bool build_apply_masked(Builder &b, Program &prog, int op)
{
    if (op <= MOL_OP_D_Y) {
        const int dir = op % 3;
        OutSpec o{};
        o.buf = B_OUT;
        o.dc[0] = (op <= MOL_OP_LINV_Z) ? -1.0 : 1.0;
        if (op <= MOL_OP_LINV_Z) o.elem = lin(B_IN);
        return b.emit(prog, dir, {lin(B_IN)}, {o}, 1);
    }
    if (op == MOL_OP_RHS) return build_rhs_masked(b, prog, B_IN, {{B_OUT, Lin{}, 1.0}});
    std::vector<Term> terms;
    const bool avg = (b.pl.desc.flags & MOL_SYMMETRIC_D) != 0;
    if (op == MOL_OP_C) {
        if (!transverse(b, prog, {B_IN}, -1, terms, avg)) return false;
    } else if (op == MOL_OP_D) {
        if (!transverse(b, prog, {}, B_IN, terms, avg)) return false;
    } else {
        b.err = "operator not available on a masked plan";
        return false;
    }
    OutSpec f{};
    f.buf = B_OUT;
    f.elem = terms[0].elem;
    f.dc[0] = terms[0].s;
    return b.emit(prog, 0, {terms[0].comb}, {f}, 1);
}

}  // namespace molt
