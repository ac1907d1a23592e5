// Plan builder and C-ABI of libmolt.
//
// A plan turns the problem statement (domain, c, dt, beta, order P, boundary
// types, optional embedded boundary) into
//   * FP64 scheme constants: beta_max(P) (Sec. 3.1, eq. Stab_cond),
//     alpha = beta/(c dt) (eq. L_def), the stage weights
//     c_{p,m} = (-1)^m 2 beta^{2m}/(2m)! binom(p-1, m-1) (eq. Full_2D);
//   * per-direction quadrature constants: d = e^{-nu}, g = (1-d)/(2 nu) via
//     expm1, the curvature weight w2 (series below nu = 1), the 2x2 closure
//     of the boundary correction (Dirichlet: e^{-alpha L} and 1/(1-e^{-2 alpha L});
//     periodic: 1/(1-e^{-alpha L})), and the halo length of split lines;
//   * a kernel program per entry point: the stage schedule of Table 2 with the
//     ADI compositions written through directional D's and fused into the
//     sweeps' prologues/epilogues, the time update fused into the last sweep.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/molt.h"
#include "molt_internal.h"
#include "molt_program.h"

using namespace molt;

namespace {

thread_local std::string g_err;

mol_status fail(mol_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

// ---------------------------------------------------------------------------
// scheme constants
// ---------------------------------------------------------------------------
double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

}  // namespace

// weight of C^m D^{p-m} in eq. Full_2D
double molt::stage_c(int p, int m, double beta)
{
    return ((m % 2) ? -2.0 : 2.0) * std::pow(beta, 2 * m) / fact(2 * m) * binom(p - 1, m - 1);
}

// Weight of C^m D^{p-m} in the odd part of the start (Sec. 3.2): the series
// sum_m beta^{2m} / (2m+1)! (laplacian / alpha^2)^m g with (laplacian /
// alpha^2)^m = (-1)^m C^m (1 - D)^{-m} expanded as for eq. Full_2D:
// b_{p,m} = (-1)^m beta^{2m} / (2m+1)! binom(p-1, m-1).
double molt::start_b(int p, int m, double beta)
{
    return ((m % 2) ? -1.0 : 1.0) * std::pow(beta, 2 * m) / fact(2 * m + 1) * binom(p - 1, m - 1);
}

// A_p = sum_m c_{p,m}: the 1D weights (eq. update_P)
double molt::A_p(int p, double beta)
{
    double s = 0.0;
    for (int m = 1; m <= p; ++m) s += stage_c(p, m, beta);
    return s;
}

namespace {

// S(beta, 1) = -sum_{p<=P} A_p(beta) (eq. Stab_sum at Dhat = 1)
double S1(int P, double beta)
{
    double s = 0.0;
    for (int p = 1; p <= P; ++p) s -= A_p(p, beta);
    return s;
}

double beta_max_of(int P)
{
    // S(beta, 1) grows from 0 at beta = 0; march to the first crossing of 4,
    // then refine by bisection.
    double lo = 0.0, hi = 0.0;
    const double step = 1.0 / 512.0;
    for (double b = step; b < 16.0; b += step) {
        if (S1(P, b) >= 4.0) {
            lo = b - step;
            hi = b;
            break;
        }
    }
    if (hi == 0.0) return -1.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (S1(P, mid) < 4.0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// curvature weight w2(nu) = (2(1-e^{-nu})/nu^2 - (1+e^{-nu})/nu)/4
double w2_of(double nu)
{
    if (nu < 1.0) {
        // -(nu/4) sum_{k>=0} (-nu)^k / (k! (k+2)(k+3))
        double s = 0.0, t = 1.0;
        for (int k = 0; k < 40; ++k) {
            s += t / ((k + 2.0) * (k + 3.0));
            t *= -nu / (k + 1.0);
        }
        return -0.25 * nu * s;
    }
    const double om = -std::expm1(-nu);
    const double d = std::exp(-nu);
    return 0.25 * (2.0 * om / (nu * nu) - (1.0 + d) / nu);
}

int halo_for(double nu, bool fp64)
{
    // d^K <= 2^-(mantissa bits) / 16: below the rounding of the result
    const double lnTol = fp64 ? (53.0 + 4.0) * std::log(2.0) : (24.0 + 4.0) * std::log(2.0);
    const double K = std::ceil(lnTol / nu) + 1.0;
    return K > 1e9 ? 1000000000 : (int)K;
}

// weights of the I recurrences, w0 = 1/2 - g and w1 = g - d/2 (g = (1 - d) /
// (2 nu)): series below nu = 1, where the differences cancel
//   w0 = (1/2) sum_{k>=1} (-1)^(k+1) nu^k / (k+1)!
//   w1 = (1/2) sum_{k>=1} (-1)^(k+1) k nu^k / (k+1)!
void w01_of(double nu, double &w0, double &w1)
{
    if (nu < 1.0) {
        double s0 = 0.0, s1 = 0.0, t = 1.0;   // t = nu^k / (k+1)!
        for (int k = 1; k < 40; ++k) {
            t *= nu / (double)(k + 1);
            const double sg = (k % 2) ? 1.0 : -1.0;
            s0 += sg * t;
            s1 += sg * (double)k * t;
        }
        w0 = 0.5 * s0;
        w1 = 0.5 * s1;
        return;
    }
    const double g = -std::expm1(-nu) / (2.0 * nu);
    w0 = 0.5 - g;
    w1 = g - 0.5 * std::exp(-nu);
}

DirCoef make_dircoef(double nu, int64_t n, bool periodic, bool fp64, bool neumann = false)
{
    DirCoef c{};
    c.nu = nu;
    c.d = std::exp(-nu);
    c.g = -std::expm1(-nu) / (2.0 * nu);
    c.w2 = w2_of(nu);
    w01_of(nu, c.w0, c.w1);
    c.periodic = periodic ? 1 : 0;
    c.n = n;
    c.halo = halo_for(nu, fp64);
    if (periodic) {
        const double f = c.d / (-std::expm1(-nu * (double)n));
        c.K[0][0] = 0.0; c.K[0][1] = f;
        c.K[1][0] = f;   c.K[1][1] = 0.0;
    } else if (neumann) {
        // slopes imposed: (-1, mu; -mu, 1) (A, B) = (-r0, r1) on the end
        // residuals the sweep forms (r0 = I^R(a) - S_a / alpha,
        // r1 = I^L(b) + S_b / alpha)
        const double L = nu * (double)(n - 1);
        const double mu = std::exp(-L);
        const double inv = 1.0 / (-std::expm1(-2.0 * L));
        c.K[0][0] = inv;       c.K[0][1] = mu * inv;
        c.K[1][0] = mu * inv;  c.K[1][1] = inv;
    } else {
        const double L = nu * (double)(n - 1);       // alpha * (b - a)
        const double mu = std::exp(-L);
        const double inv = 1.0 / (-std::expm1(-2.0 * L));
        c.K[0][0] = -inv;      c.K[0][1] = mu * inv;
        c.K[1][0] = mu * inv;  c.K[1][1] = -inv;
    }
    return c;
}

}  // namespace

namespace molt {

// MOL_UNIFORM_CONFIG: x sweeps take the smallest line capacity that holds
// max(n, 2048) nodes, strided sweeps the tall-tile kernel; a choice that is
// not valid for this op keeps the default.
void uniform_config(const mol_plan_ &pl, const SweepOp &op, int *cfg)
{
    const int dir = op.dir;
    int c[2] = {0, 0};
    if (dir == 0) {
        static const int order32[] = {0, 1, 2, 3, 4, 5, 7};
        static const int order64[] = {0, 1, 2, 8, 9, 6, 7};
        const int *ord = pl.fp64 ? order64 : order32;
        const int64_t need = std::max<int64_t>(pl.geom.n[0], 2048);
        for (int i = 0; i < 7; ++i) {
            c[0] = ord[i];
            const int cap = 64 * uniform_x_capacity(c[0]);
            if (cap >= need && config_valid(pl.geom, pl.dc[dir], op, pl.fp64, c)) {
                cfg[0] = c[0];
                return;
            }
        }
        return;
    }
    if (op.yy) return;
    const int regs = (2 * op.ns + op.no) * (pl.fp64 ? 2 : 1);
    c[0] = (regs <= 4) ? 0 : 2;
    if (config_valid(pl.geom, pl.dc[dir], op, pl.fp64, c)) cfg[0] = c[0];
}

bool Builder::emit(Program &prog, int dir, const std::vector<Lin> &combos,
                   const std::vector<OutSpec> &outs, int proj, int chain_buf,
                   const std::vector<int> &kf)
{

        const int ns = (int)combos.size(), no = (int)outs.size();
        if (ns < 1 || ns > MAXS || no < 1 || no > MAXO) {
            err = "internal: launch shape";
            return false;
        }
        if (chain_buf >= 0 && dir != 0) {
            err = "internal: chained sweeps are x sweeps";
            return false;
        }
        SweepOp op;
        op.dir = dir;
        op.ns = ns;
        op.no = no;
        op.proj = proj;
        op.chain = chain_buf >= 0 ? 1 : 0;
        op.ochain = chain_buf;
        for (int k = 0; k < ns && k < (int)kf.size(); ++k) op.kform[k] = kf[k] ? 1 : 0;
        if (op.chain && (op.kform[0] || op.kform[1])) {
            err = "internal: chained sweeps sweep for D";
            return false;
        }
        if (pl.neumann) {
            // the sweep closes each line by the slopes at its ends (zero
            // data here; mol_step_bdata sets them per step); every node is
            // an unknown, nothing is projected
            if (ns != 1 || op.kform[0] || op.chain) {
                err = "Neumann lines take one D sweep per launch";
                return false;
            }
            op.bmode = 2;
            op.proj = 0;
        }
        std::vector<int> fields;
        auto fid = [&](int b) -> int {
            for (size_t i = 0; i < fields.size(); ++i)
                if (fields[i] == b) return (int)i;
            fields.push_back(b);
            return (int)fields.size() - 1;
        };
        for (int k = 0; k < ns; ++k)
            for (auto &t : combos[k]) {
                const int i = fid(t.first);
                if (i < MAXF) op.mS[k][i] += t.second;
            }
        for (int o = 0; o < no; ++o) {
            op.o[o] = outs[o].buf;
            for (auto &t : outs[o].elem) {
                const int i = fid(t.first);
                if (i < MAXF) op.mOF[o][i] += t.second;
            }
            for (int k = 0; k < ns; ++k) op.mOD[o][k] = outs[o].dc[k];
        }
        if ((int)fields.size() > MAXF) {
            err = "schedule needs more fields per launch than supported (lower P)";
            return false;
        }
        op.nf = (int)fields.size();
        for (int i = 0; i < op.nf; ++i) op.f[i] = fields[i];

        // does a configuration exist? else split two combos into two launches
        int cfg[2] = {0, 0};
        if (!pl.masked && default_config(pl.geom, pl.dc[dir], op, pl.fp64, cfg) != 0) {
            if (ns == 2) {
                std::vector<OutSpec> o0, o1;
                for (const OutSpec &o : outs) {
                    const bool u0 = o.dc[0] != 0.0, u1 = o.dc[1] != 0.0;
                    if (u0 && u1) {
                        err = "internal: cannot split a launch whose output needs both sweeps";
                        return false;
                    }
                    OutSpec t = o;
                    if (u1) { t.dc[0] = t.dc[1]; t.dc[1] = 0; o1.push_back(t); }
                    else o0.push_back(t);
                }
                bool ok = true;
                if (!o0.empty()) ok = ok && emit(prog, dir, {combos[0]}, o0, proj, -1, {op.kform[0]});
                if (!o1.empty()) ok = ok && emit(prog, dir, {combos[1]}, o1, proj, -1, {op.kform[1]});
                return ok;
            }
            if (no > 1) {
                bool ok = true;
                for (const OutSpec &o : outs)
                    ok = ok && emit(prog, dir, combos, {o}, proj, -1, {op.kform[0], op.kform[1]});
                return ok;
            }
            err = "no kernel configuration fits this line length";
            return false;
        }
        if (!pl.masked && (pl.desc.flags & MOL_UNIFORM_CONFIG)) {
            uniform_config(pl, op, cfg);
        } else if (!pl.masked) {
            const std::string key = tune_op_key(op);
            for (const auto &t : pl.tuned) {
                int c[2] = {t.second, 0};
                if (t.first == key && config_valid(pl.geom, pl.dc[dir], op, pl.fp64, c))
                    cfg[0] = t.second;
            }
        }
        ProgOp po;
        po.op = op;
        po.cfg[0] = cfg[0];
        po.cfg[1] = cfg[1];
        prog.push_back(po);
        return true;
    }

bool Builder::yy_available(int dir, int nf, int no) const
{
    if (pl.masked) return false;
    SweepOp op;
    op.dir = dir;
    op.yy = 1;
    op.nf = nf;
    op.ns = 1;
    op.no = no;
    op.mOD[0][0] = 1.0;
    int cfg[2] = {0, 0};
    return default_config(pl.geom, pl.dc[dir], op, pl.fp64, cfg) == 0;
}

bool Builder::emit_yy(Program &prog, int dir, const Lin &s1, const Lin &e1,
                      const std::vector<std::pair<int, Lin>> &outs)
{
    SweepOp op;
    op.dir = dir;
    op.yy = 1;
    op.ns = 1;
    op.no = (int)outs.size();
    if (op.no < 1 || op.no > MAXO) {
        err = "internal: launch shape";
        return false;
    }
    std::vector<int> fields;
    auto fid = [&](int b) -> int {
        for (size_t i = 0; i < fields.size(); ++i)
            if (fields[i] == b) return (int)i;
        fields.push_back(b);
        return (int)fields.size() - 1;
    };
    for (auto &t : s1) {
        const int i = fid(t.first);
        if (i < MAXF) op.mS[0][i] += t.second;
    }
    for (auto &t : e1) {
        const int i = fid(t.first);
        if (i < MAXF) op.mE1[i] += t.second;
    }
    for (int o = 0; o < op.no; ++o) {
        op.o[o] = outs[o].first;
        for (auto &t : outs[o].second) {
            if (t.first == V1) {
                op.mV[o] += t.second;
            } else if (t.first == Y) {
                op.mOD[o][0] += t.second;
            } else {
                const int i = fid(t.first);
                if (i < MAXF) op.mOF[o][i] += t.second;
            }
        }
    }
    if ((int)fields.size() > MAXF) {
        err = "schedule needs more fields per launch than supported (lower P)";
        return false;
    }
    op.nf = (int)fields.size();
    for (int i = 0; i < op.nf; ++i) op.f[i] = fields[i];
    int cfg[2] = {0, 0};
    if (default_config(pl.geom, pl.dc[dir], op, pl.fp64, cfg) != 0) {
        err = "internal: no chained configuration";
        return false;
    }
    const std::string key = tune_op_key(op);
    for (const auto &t : pl.tuned) {
        int c[2] = {t.second, 0};
        if (t.first == key && config_valid(pl.geom, pl.dc[dir], op, pl.fp64, c)) cfg[0] = t.second;
    }
    ProgOp po;
    po.op = op;
    po.cfg[0] = cfg[0];
    po.cfg[1] = cfg[1];
    prog.push_back(po);
    return true;
}

std::vector<OutSpec> finals(const std::vector<FinalOut> &fo, const Lin &rhs_elem, double rhs_dcoef)
{
    std::vector<OutSpec> v;
    for (const FinalOut &f : fo) {
        OutSpec o{};
        o.buf = f.buf;
        o.elem = f.elem + f.r * rhs_elem;
        o.dc[0] = f.r * rhs_dcoef;
        o.dc[1] = 0.0;
        v.push_back(o);
    }
    return v;
}

// 1D: rhs = sum_p A_p D^p u, D^p by repeated sweeps (Sec. 3, eq. update_P).
bool build_rhs_1d(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo)
{
    mol_plan_ &pl = b.pl;
    const int P = pl.desc.P;
    std::vector<int> w(P, u);   // w[p] = D^p u, w[0] = u
    Lin acc;
    for (int p = 1; p < P; ++p) {
        w[p] = b.new_ws();
        OutSpec o{};
        o.buf = w[p];
        o.dc[0] = 1.0;
        if (!b.emit(prog, 0, {lin(w[p - 1])}, {o}, 0)) return false;
        acc = acc + lin(w[p], b.Ap(p));
    }
    return b.emit(prog, 0, {lin(w[P - 1])}, finals(fo, acc, b.Ap(P)), 1);
}

// 2D rectangles at small nu: the stage schedule of Table 2 with
//   C v = D_x(K_y v) + K_x(D_y v),   D v = D_x(K_y v) + D_y v   (K = L^{-1}),
// the same operators as eqs. C_def_ADI, D_def_ADI on a rectangle (the
// directional operators commute), written so that no term cancels: for data
// that varies on the grid scale L^{-1} is small where nu is small, and the
// D-form C v = D_x(v - 2 D_y v) + D_y v would be a difference of order-one
// terms.  One y launch per input sweeps it for D_y and for K_y; one x launch
// per new term sweeps K_y v for D_x and D_y v for K_x.
bool build_rhs_box_k(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo)
{
    const int P = b.pl.desc.P;
    std::vector<int> v{u};
    int accbuf = -1;
    for (int p = 1; p <= P; ++p) {
        const int nin = (int)v.size();
        std::vector<int> y(nin), k(nin);
        for (int j = 0; j < nin; ++j) {
            y[j] = b.new_ws();
            k[j] = b.new_ws();
            OutSpec oy{}, ok{};
            oy.buf = y[j];
            oy.dc[0] = 1.0;
            ok.buf = k[j];
            ok.dc[1] = 1.0;
            if (!b.emit(prog, 1, {lin(v[j]), lin(v[j])}, {oy, ok}, 0, -1, {0, 1})) return false;
        }
        // terms: D_x(g) + K_x(gk) + h
        struct KT { Lin g, gk, h; };
        std::vector<KT> t;
        for (int j = 0; j < nin; ++j) t.push_back({lin(k[j]), lin(y[j]), Lin{}});
        if (p >= 2) t.push_back({lin(k[nin - 1]), Lin{}, lin(y[nin - 1])});
        const int nt = (int)t.size();
        Lin acc_in;
        if (p == 2) acc_in = lin(v[0], b.coef(1, 1));
        else if (p >= 3) acc_in = lin(accbuf);
        if (p == P) {
            Lin gs, gks, hs = acc_in;
            for (int j = 0; j < nt; ++j) {
                const double c = b.coef(p, p - j);
                gs = gs + c * t[j].g;
                gks = gks + c * t[j].gk;
                hs = hs + c * t[j].h;
            }
            std::vector<OutSpec> outs;
            for (const FinalOut &f : fo) {
                OutSpec o{};
                o.buf = f.buf;
                o.elem = f.elem + f.r * hs;
                o.dc[0] = f.r;
                o.dc[1] = gks.empty() ? 0.0 : f.r;
                outs.push_back(o);
            }
            if (gks.empty()) return b.emit(prog, 0, {gs}, outs, 1);
            return b.emit(prog, 0, {gs, gks}, outs, 1, -1, {0, 1});
        }
        std::vector<int> nv(nt);
        const bool need_acc = (P >= 3);
        const int newacc = need_acc ? b.new_ws() : -1;
        Lin acc_done = acc_in;
        for (int j = 0; j < nt; ++j) {
            nv[j] = b.new_ws();
            const double c = b.coef(p, p - j);
            const bool two = !t[j].gk.empty();
            OutSpec o{};
            o.buf = nv[j];
            o.elem = t[j].h;
            o.dc[0] = 1.0;
            o.dc[1] = two ? 1.0 : 0.0;
            std::vector<OutSpec> outs{o};
            if (j + 1 == nt && need_acc) {
                OutSpec a{};
                a.buf = newacc;
                a.elem = acc_done + c * t[j].h;
                a.dc[0] = c;
                a.dc[1] = two ? c : 0.0;
                outs.push_back(a);
            }
            const bool okj = two ? b.emit(prog, 0, {t[j].g, t[j].gk}, outs, 0, -1, {0, 1})
                                 : b.emit(prog, 0, {t[j].g}, outs, 0);
            if (!okj) return false;
            acc_done = acc_done + lin(nv[j], c);
        }
        v = nv;
        accbuf = newacc;
    }
    return true;
}

// 2D / 3D rectangles and boxes: stage schedule of Table 2; each application of
// C or D composed from directional D's (operators commute on boxes):
//   2D: C v = D_x(v - 2y) + y,  D v = D_x(v - y) + y,  y = D_y v
//   3D: C v = D_x(v - 2y - 2z + 3yz) + (y + z - 2yz),
//       D v = D_x(v - y - z + yz) + (y + z - yz),  z = D_z v, y = D_y v, yz = D_y z
bool build_rhs_box(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo,
                   int chain_a = -1, int csrc = -1, double ksrc = 0.0)
{
    // csrc >= 0 (2D, no chaining, one output): the output also gets
    // ksrc C[csrc]; csrc is swept with u in the first y launch and
    // C csrc = D_x(csrc - 2 y_s) + y_s joins the last x sweep
    mol_plan_ &pl = b.pl;
    const int P = pl.desc.P;
    const int nd = pl.geom.ndim;
    const double beta = pl.beta;
    std::vector<int> v{u};      // inputs of the current stage
    int accbuf = -1;            // accumulated earlier-stage terms (stage >= 3)
    int pfirst = 1;
    int ys = -1;                // D_y csrc
    if (csrc >= 0 && (nd != 2 || chain_a >= 0 || fo.size() != 1 || P < 2)) {
        b.err = "internal: folded C term needs a 2D unchained program with P >= 2";
        return false;
    }
    if (chain_a >= 0 && P == 2 && nd == 2 && fo.size() == 1 &&
        !(pl.desc.flags & MOL_SPLIT_Y) && b.yy_available(1, 3, 2)) {
        // 2D, P = 2: both y sweeps of the step in one launch.  v1 = C u =
        // D_y(u - 2a) + a and y = D_y v1 stay on chip; the launch writes the
        // x sweep's combination G = c22 (v1 - 2y) + c21 (v1 - y) and its
        // elementwise part H = elem + r (c11 v1 + (c22 + c21) y).
        const int V1 = Builder::V1, Y = Builder::Y;
        const double c11 = b.coef(1, 1), c22 = b.coef(2, 2), c21 = b.coef(2, 1);
        const Lin gs = c22 * (lin(V1) + lin(Y, -2.0)) + c21 * (lin(V1) + lin(Y, -1.0));
        const Lin hs = lin(V1, c11) + c22 * lin(Y) + c21 * lin(Y);
        const int G = b.new_ws(), H = b.new_ws();
        // elementwise terms on caller fields other than u^n, u^{n-1} (a
        // separable source) go to the x sweep: the walk takes three fields
        Lin he, xe;
        for (const auto &t : fo[0].elem)
            (t.first == B_AUX0 || t.first == B_AUX1 ? xe : he).push_back(t);
        if (!b.emit_yy(prog, 1, lin(u) + lin(chain_a, -2.0), lin(chain_a),
                       {{G, gs}, {H, he + fo[0].r * hs}}))
            return false;
        OutSpec o{};
        o.buf = fo[0].buf;
        o.elem = lin(H) + xe;
        o.dc[0] = fo[0].r;
        return b.emit(prog, 0, {lin(G)}, {o}, 1, chain_a);
    }
    if (chain_a >= 0) {
        // 2D, P >= 2: stage 1 in the order x then y, with a = D_x u written by
        // the previous step's last sweep: C u = D_y(u - 2a) + a
        const int v1 = b.new_ws();
        OutSpec o{};
        o.buf = v1;
        o.elem = lin(chain_a);
        o.dc[0] = 1.0;
        if (!b.emit(prog, 1, {lin(u) + lin(chain_a, -2.0)}, {o}, 0)) return false;
        v = {v1};
        pfirst = 2;
    }
    for (int p = pfirst; p <= P; ++p) {
        const int nin = (int)v.size();     // p == 1: {u}; else v_1..v_{p-1}
        // ---- transverse sweeps ----
        std::vector<Lin> gC(nin), hC(nin);   // C v_k = D_x(gC) + hC
        Lin gD, hD;                           // D v_last = D_x(gD) + hD
        if (nd == 2) {
            std::vector<int> y(nin);
            for (int k = 0; k < nin; k += 2) {
                std::vector<Lin> cmb;
                std::vector<OutSpec> outs;
                for (int j = k; j < std::min(nin, k + 2); ++j) {
                    y[j] = b.new_ws();
                    cmb.push_back(lin(v[j]));
                    OutSpec o{};
                    o.buf = y[j];
                    o.dc[j - k] = 1.0;
                    outs.push_back(o);
                }
                if (p == 1 && csrc >= 0 && nin == 1) {
                    ys = b.new_ws();
                    cmb.push_back(lin(csrc));
                    OutSpec o{};
                    o.buf = ys;
                    o.dc[1] = 1.0;
                    outs.push_back(o);
                }
                if (!b.emit(prog, 1, cmb, outs, 0)) return false;
            }
            for (int k = 0; k < nin; ++k) {
                gC[k] = lin(v[k]) + lin(y[k], -2.0);
                hC[k] = lin(y[k]);
            }
            gD = lin(v[nin - 1]) + lin(y[nin - 1], -1.0);
            hD = lin(y[nin - 1]);
        } else {
            std::vector<int> z(nin), y(nin), yz(nin);
            for (int k = 0; k < nin; k += 2) {
                std::vector<Lin> cmb;
                std::vector<OutSpec> outs;
                for (int j = k; j < std::min(nin, k + 2); ++j) {
                    z[j] = b.new_ws();
                    cmb.push_back(lin(v[j]));
                    OutSpec o{};
                    o.buf = z[j];
                    o.dc[j - k] = 1.0;
                    outs.push_back(o);
                }
                if (!b.emit(prog, 2, cmb, outs, 0)) return false;
            }
            for (int k = 0; k < nin; ++k) {
                y[k] = b.new_ws();
                yz[k] = b.new_ws();
                OutSpec o1{}, o2{};
                o1.buf = y[k];
                o1.dc[0] = 1.0;
                o2.buf = yz[k];
                o2.dc[1] = 1.0;
                if (!b.emit(prog, 1, {lin(v[k]), lin(z[k])}, {o1, o2}, 0)) return false;
            }
            for (int k = 0; k < nin; ++k) {
                gC[k] = lin(v[k]) + lin(y[k], -2.0) + lin(z[k], -2.0) + lin(yz[k], 3.0);
                hC[k] = lin(y[k]) + lin(z[k]) + lin(yz[k], -2.0);
            }
            const int l = nin - 1;
            gD = lin(v[l]) + lin(y[l], -1.0) + lin(z[l], -1.0) + lin(yz[l]);
            hD = lin(y[l]) + lin(z[l]) + lin(yz[l], -1.0);
        }
        // ---- x sweeps: the new terms of stage p ----
        // stage p produces p terms: C v_k (k < nin) and D v_{nin-1} (p >= 2); for
        // p == 1 the single term C u.  Term k carries m = p - k factors of C.
        std::vector<Lin> g, h;
        for (int k = 0; k < nin; ++k) { g.push_back(gC[k]); h.push_back(hC[k]); }
        if (p >= 2) { g.push_back(gD); h.push_back(hD); }
        const int nt = (int)g.size();          // == p
        // earlier-stage terms carried into this stage
        Lin acc_in;
        if (p == 2) acc_in = lin(v[0], b.coef(1, 1));   // v_1 = C u
        else if (p >= 3) acc_in = lin(accbuf);
        if (p == P) {
            // one sweep of the weighted sum of this stage's terms
            Lin gs, hs = acc_in;
            for (int k = 0; k < nt; ++k) {
                const double c = b.coef(p, p - k);
                gs = gs + c * g[k];
                hs = hs + c * h[k];
            }
            if (csrc >= 0) {
                const double w = ksrc / fo[0].r;
                gs = gs + w * (lin(csrc) + lin(ys, -2.0));
                hs = hs + w * lin(ys);
            }
            return b.emit(prog, 0, {gs}, finals(fo, hs, 1.0), 1, chain_a);
        }
        // non-final stage: write the p new terms (and the accumulator if needed)
        std::vector<int> nv(nt);
        for (int k = 0; k < nt; ++k) nv[k] = b.new_ws();
        const bool need_acc = (P >= 3);
        const int newacc = need_acc ? b.new_ws() : -1;
        // launches of <= 2 sweeps; the last one also writes the accumulator
        Lin acc_done = acc_in;    // contributions of terms already written
        for (int k = 0; k < nt; k += 2) {
            const int k1 = std::min(nt, k + 2);
            std::vector<Lin> cmb;
            std::vector<OutSpec> outs;
            for (int j = k; j < k1; ++j) {
                cmb.push_back(g[j]);
                OutSpec o{};
                o.buf = nv[j];
                o.elem = h[j];
                o.dc[j - k] = 1.0;
                outs.push_back(o);
            }
            const bool last = (k1 == nt);
            if (last && need_acc) {
                OutSpec o{};
                o.buf = newacc;
                o.elem = acc_done;
                for (int j = k; j < k1; ++j) {
                    const double c = b.coef(p, p - j);
                    o.elem = o.elem + c * h[j];
                    o.dc[j - k] = c;
                }
                outs.push_back(o);
            }
            if (!b.emit(prog, 0, cmb, outs, 0)) return false;
            for (int j = k; j < k1; ++j) acc_done = acc_done + lin(nv[j], b.coef(p, p - j));
        }
        // stage p+1 inputs: terms in Table 2 order (m = p, p-1, ..., 1)
        v = nv;
        accbuf = newacc;
    }
    return true;
}

bool build_rhs(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo)
{
    if (b.pl.masked) {
        return build_rhs_masked(b, prog, u, fo);
    }
    if (b.pl.geom.ndim == 1) return build_rhs_1d(b, prog, u, fo);
    if (b.pl.kmode) return build_rhs_box_k(b, prog, u, fo);
    return build_rhs_box(b, prog, u, fo);
}

// single operators
bool emit_CD(Builder &b, Program &prog, bool isC, int in, int out);

bool build_apply(Builder &b, Program &prog, int op)
{
    mol_plan_ &pl = b.pl;
    const int nd = pl.geom.ndim;
    if (op <= MOL_OP_D_Z) {
        const int dir = op % 3;
        if (dir >= nd) {
            b.err = "operator direction not present";
            return false;
        }
        if (pl.masked) return build_apply_masked(b, prog, op);
        // L^{-1} by its own recurrences, D by the difference-driven ones;
        // on Neumann lines L^{-1} v = v - D v
        OutSpec o{};
        o.buf = B_OUT;
        o.dc[0] = 1.0;
        if (pl.neumann && op <= MOL_OP_LINV_Z) {
            o.elem = lin(B_IN);
            o.dc[0] = -1.0;
            return b.emit(prog, dir, {lin(B_IN)}, {o}, 1);
        }
        if (b.emit(prog, dir, {lin(B_IN)}, {o}, 1, -1, {op <= MOL_OP_LINV_Z ? 1 : 0})) return true;
        if (op > MOL_OP_LINV_Z) return false;
        // lines swept in chunks carry the D recurrences only: L^{-1} v = v - D v
        b.err.clear();
        o.elem = lin(B_IN);
        o.dc[0] = -1.0;
        return b.emit(prog, dir, {lin(B_IN)}, {o}, 1);
    }
    if (pl.masked) return build_apply_masked(b, prog, op);
    if (op == MOL_OP_RHS) return build_rhs(b, prog, B_IN, {{B_OUT, Lin{}, 1.0}});
    return emit_CD(b, prog, op == MOL_OP_C, B_IN, B_OUT);
}

// out = C in or D in on a box (eqs. C_def_ADI, D_def_ADI and their 3D forms).
bool emit_CD(Builder &b, Program &prog, bool isC, int in, int out)
{
    const int nd = b.pl.geom.ndim;
    if (nd == 1) {
        OutSpec o{};
        o.buf = out;
        o.dc[0] = 1.0;
        return b.emit(prog, 0, {lin(in)}, {o}, 1);
    }
    if (nd == 2 && b.pl.kmode) {
        // C = D_x(K_y in) + K_x(D_y in), D = D_x(K_y in) + D_y in
        const int y = b.new_ws(), k = b.new_ws();
        OutSpec oy{}, ok{};
        oy.buf = y;
        oy.dc[0] = 1.0;
        ok.buf = k;
        ok.dc[1] = 1.0;
        if (!b.emit(prog, 1, {lin(in), lin(in)}, {oy, ok}, 0, -1, {0, 1})) return false;
        OutSpec f{};
        f.buf = out;
        f.dc[0] = 1.0;
        if (isC) {
            f.dc[1] = 1.0;
            return b.emit(prog, 0, {lin(k), lin(y)}, {f}, 1, -1, {0, 1});
        }
        f.elem = lin(y);
        return b.emit(prog, 0, {lin(k)}, {f}, 1);
    }
    if (nd == 2) {
        const int y = b.new_ws();
        OutSpec o{};
        o.buf = y;
        o.dc[0] = 1.0;
        if (!b.emit(prog, 1, {lin(in)}, {o}, 0)) return false;
        OutSpec f{};
        f.buf = out;
        f.elem = lin(y);
        f.dc[0] = 1.0;
        return b.emit(prog, 0, {lin(in) + lin(y, isC ? -2.0 : -1.0)}, {f}, 1);
    }
    const int z = b.new_ws(), y = b.new_ws(), yz = b.new_ws();
    OutSpec oz{};
    oz.buf = z;
    oz.dc[0] = 1.0;
    if (!b.emit(prog, 2, {lin(in)}, {oz}, 0)) return false;
    OutSpec o1{}, o2{};
    o1.buf = y;
    o1.dc[0] = 1.0;
    o2.buf = yz;
    o2.dc[1] = 1.0;
    if (!b.emit(prog, 1, {lin(in), lin(z)}, {o1, o2}, 0)) return false;
    OutSpec f{};
    f.buf = out;
    f.dc[0] = 1.0;
    if (isC) {
        f.elem = lin(y) + lin(z) + lin(yz, -2.0);
        return b.emit(prog, 0, {lin(in) + lin(y, -2.0) + lin(z, -2.0) + lin(yz, 3.0)}, {f}, 1);
    }
    f.elem = lin(y) + lin(z) + lin(yz, -1.0);
    return b.emit(prog, 0, {lin(in) + lin(y, -1.0) + lin(z, -1.0) + lin(yz)}, {f}, 1);
}

// Step with a source term for u_tt / c^2 = laplacian(u) + S (Sec. 4, inclusion
// of source terms), (c dt)^2 = (beta / alpha)^2:
//   P = 1: u^{n+1} = 2 u^n - u^{n-1} + rhs(u^n) + (c dt)^2 S^n
//   P = 2: ... + (c dt)^2 / 12 (S^{n+1} + 10 S^n + S^{n-1}) - beta^2 (c dt)^2 / 12 C[S^n]
// The C[S^n] coefficient is the dt^4 c^4 laplacian(S) / 12 term of the Taylor
// expansion with the laplacian replaced by -alpha^2 C, as in the homogeneous
// part.  In 2D, S^n is swept with u^n in the step's first y launch and C[S^n]
// joins the step's last x sweep; in 1D and 3D C[S^n] goes to a workspace
// field first.  The other source terms join the elementwise part of the last
// sweep.
bool build_step_source(Builder &b, Program &prog)
{
    mol_plan_ &pl = b.pl;
    const double a2 = (pl.beta / pl.alpha) * (pl.beta / pl.alpha);
    Lin elem = lin(B_UCURR, 2.0) + lin(B_UPREV, -1.0);
    if (pl.desc.P == 1) {
        elem = elem + lin(B_IN, a2);
    } else {
        const double sg = a2 / 12.0;
        elem = elem + lin(B_AUX0, sg) + lin(B_IN, 10.0 * sg) + lin(B_AUX1, sg);
        if (pl.geom.ndim == 2 && !pl.kmode)
            // C[S^n] folded into the step's own sweeps
            return build_rhs_box(b, prog, B_UCURR, {{B_UNEXT, elem, 1.0}}, -1, B_IN,
                                 -pl.beta * pl.beta * sg);
        const int cs = b.new_ws();
        if (!emit_CD(b, prog, true, B_IN, cs)) return false;
        elem = elem + lin(cs, -pl.beta * pl.beta * sg);
    }
    return build_rhs(b, prog, B_UCURR, {{B_UNEXT, elem, 1.0}});
}

// Start with an initial velocity g (Sec. 3.2): the even terms of the Taylor
// series of u(dt) give u0 + rhs(u0)/2 as without g; the odd ones give
// dt sum_m beta^{2m} / (2m+1)! (laplacian / alpha^2)^m g, taken with Table 2's
// schedule and weights b_{p,m} (p <= P).  The odd part dt (g + rhs_b(g)) is
// written to u1 itself, whose last sweep for the even part then reads it
// elementwise: u1 = u0 + u1 + rhs(u0) / 2.  The two parts share workspace.
bool build_start_g(Builder &b, Program &prog)
{
    const double dt = b.pl.desc.dt;
    const int mark = b.pl.nws;
    b.series = 1;
    const bool ok = build_rhs(b, prog, B_AUX0, {{B_OUT, lin(B_AUX0, dt), dt}});
    b.series = 0;
    const int used = b.pl.nws;
    b.pl.nws = mark;
    const bool ok2 = ok && build_rhs(b, prog, B_IN, {{B_OUT, lin(B_IN) + lin(B_OUT), 0.5}});
    b.pl.nws = std::max(used, b.pl.nws);
    return ok2;
}

// Step for a separable source S = f(t) G(x) (Sec. 4, inclusion of source
// terms): the source part a_n G + b_n C[G] joins the last launch of the step
// as two elementwise fields, G (B_AUX0) and C[G] (B_AUX1, P = 2 only), with
// unit weights that mol_solve_source replaces every step.  Fused (chained) in
// 2D like mol_solve's own program.
bool build_solve_source(Builder &b, Program &prog, int chain_a)
{
    mol_plan_ &pl = b.pl;
    Lin elem = lin(B_UCURR, 2.0) + lin(B_UPREV, -1.0) + lin(B_AUX0, 1.0);
    if (pl.desc.P == 2) elem = elem + lin(B_AUX1, 1.0);
    const bool ok = chain_a >= 0
                        ? build_rhs_box(b, prog, B_UCURR, {{B_UNEXT, elem, 1.0}}, chain_a)
                        : build_rhs(b, prog, B_UCURR, {{B_UNEXT, elem, 1.0}});
    if (!ok || prog.empty()) return false;
    const SweepOp &last = prog.back().op;
    pl.src_fg = pl.src_fcg = -1;
    for (int i = 0; i < last.nf; ++i) {
        if (last.f[i] == B_AUX0) pl.src_fg = i;
        if (last.f[i] == B_AUX1) pl.src_fcg = i;
    }
    // every other launch must not read them
    for (size_t k = 0; k + 1 < prog.size(); ++k)
        for (int i = 0; i < prog[k].op.nf; ++i)
            if (prog[k].op.f[i] == B_AUX0 || prog[k].op.f[i] == B_AUX1) return false;
    return pl.src_fg >= 0 && (pl.desc.P == 1 || pl.src_fcg >= 0);
}

std::string tune_problem_key(const mol_plan_ *pl)
{
    std::ostringstream o;
    o << (pl->fp64 ? "f64" : "f32") << " nd" << pl->geom.ndim << " n" << pl->geom.n[0] << "x"
      << pl->geom.n[1] << "x" << pl->geom.n[2] << " bc" << pl->desc.bc[0] << pl->desc.bc[1]
      << pl->desc.bc[2] << " P" << pl->desc.P << (pl->masked ? " masked" : "");
    return o.str();
}

std::string tune_op_key(const SweepOp &op)
{
    std::ostringstream o;
    o << "dir" << op.dir << " nf" << op.nf << " ns" << op.ns << " no" << op.no << " ch" << op.chain;
    if (op.yy) o << " yy";
    if (op.kform[0] || op.kform[1]) o << " kf" << op.kform[0] << op.kform[1];
    return o.str();
}

// Tuning cache: lines "<problem key> | <op key> | <config id>".
// The tuning cache (tune_cache.txt beside the library, or the file named by
// MOLT_TUNE_CACHE) is parsed once per process and path.
void load_tune_cache(mol_plan_ *pl)
{
    std::string path;
    if (const char *e = std::getenv("MOLT_TUNE_CACHE")) {
        path = e;
    } else {
        Dl_info info;
        if (dladdr(reinterpret_cast<void *>(&load_tune_cache), &info) && info.dli_fname) {
            path = info.dli_fname;
            const size_t sl = path.rfind('/');
            path = (sl == std::string::npos ? std::string(".") : path.substr(0, sl)) + "/tune_cache.txt";
        }
    }
    if (path.empty()) return;
    // problem key -> (kernel key, config id)
    typedef std::vector<std::pair<std::string, std::pair<std::string, int>>> Entries;
    static std::mutex mu;
    static std::map<std::string, Entries> parsed;
    std::lock_guard<std::mutex> lk(mu);
    auto it = parsed.find(path);
    if (it == parsed.end()) {
        Entries ent;
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            const size_t a = line.find(" | "), b = line.rfind(" | ");
            if (a == std::string::npos || b == a) continue;
            ent.push_back({line.substr(0, a),
                           {line.substr(a + 3, b - a - 3), std::atoi(line.c_str() + b + 3)}});
        }
        it = parsed.emplace(path, std::move(ent)).first;
    }
    const std::string pk = tune_problem_key(pl);
    for (const auto &e : it->second)
        if (e.first == pk) pl->tuned.push_back(e.second);
}

mol_status validate(const mol_desc *d)
{
    if (!d) return fail(MOL_E_INVALID, "desc is NULL");
    if (d->ndim < 1 || d->ndim > 3) return fail(MOL_E_INVALID, "ndim must be 1, 2 or 3");
    for (int a = 0; a < 3; ++a) {
        if (a < d->ndim) {
            if (d->n[a] < 3) return fail(MOL_E_INVALID, "every axis needs at least 3 nodes");
            if (!(d->h[a] > 0.0)) return fail(MOL_E_INVALID, "h must be > 0");
            if (d->bc[a] != MOL_BC_DIRICHLET && d->bc[a] != MOL_BC_PERIODIC && d->bc[a] != MOL_BC_NEUMANN)
                return fail(MOL_E_INVALID, "unknown boundary type");
            if (d->bc[a] == MOL_BC_NEUMANN && d->ndim != 1)
                return fail(MOL_E_UNSUPPORTED, "Neumann ends are supported on 1D lines");
        } else if (d->n[a] != 1 && d->n[a] != 0) {
            return fail(MOL_E_INVALID, "unused axes must have n = 1");
        }
    }
    if (d->P < 1 || d->P > 5) return fail(MOL_E_INVALID, "P must be in 1..5 (Table 1)");
    if (!(d->c > 0.0) || !(d->dt > 0.0)) return fail(MOL_E_INVALID, "c and dt must be > 0");
    if (d->dtype != MOL_F64 && d->dtype != MOL_F32) return fail(MOL_E_INVALID, "unknown dtype");
    if (d->mask) {
        if (d->ndim != 2) return fail(MOL_E_UNSUPPORTED, "masks are supported in 2D only");
        if (d->bc[0] != MOL_BC_DIRICHLET || d->bc[1] != MOL_BC_DIRICHLET)
            return fail(MOL_E_INVALID, "a mask needs Dirichlet boundaries");
    } else if (d->cross) {
        return fail(MOL_E_INVALID, "cross given without mask");
    }
    int64_t npts = 1;
    for (int a = 0; a < d->ndim; ++a) {
        if (d->n[a] > (int64_t)1 << 31) return fail(MOL_E_UNSUPPORTED, "axis too long");
        npts *= d->n[a];
    }
    if (npts >= ((int64_t)1 << 31)) return fail(MOL_E_UNSUPPORTED, "fields of 2^31 nodes or more are not supported");
    return MOL_OK;
}

// Build everything except device allocations (dry = true) or including them.
mol_status build_plan(const mol_desc *d, mol_plan_ *pl, bool dry)
{
    mol_status s = validate(d);
    if (s != MOL_OK) return s;
    pl->desc = *d;
    pl->desc.mask = nullptr;
    pl->desc.cross = nullptr;
    pl->fp64 = (d->dtype == MOL_F64);
    pl->es = pl->fp64 ? 8 : 4;
    Geom &g = pl->geom;
    g.ndim = d->ndim;
    pl->npts = 1;
    pl->unknowns = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = (a < d->ndim) ? d->n[a] : 1;
        g.dirichlet[a] = (a < d->ndim && d->bc[a] == MOL_BC_DIRICHLET) ? 1 : 0;
        pl->npts *= g.n[a];
        pl->unknowns *= (a < d->ndim) ? (g.dirichlet[a] ? g.n[a] - 2 : g.n[a]) : 1;
    }
    pl->betamax = beta_max_of(d->P);
    pl->beta = (d->beta > 0.0) ? d->beta : pl->betamax;
    if (pl->beta > pl->betamax * (1.0 + 1e-12) && !(d->flags & MOL_ALLOW_UNSTABLE)) {
        char buf[160];
        snprintf(buf, sizeof buf, "beta = %.8g exceeds beta_max(%d) = %.8g", pl->beta, d->P,
                 pl->betamax);
        return fail(MOL_E_UNSTABLE, buf);
    }
    pl->alpha = pl->beta / (d->c * d->dt);
    for (int a = 0; a < d->ndim; ++a) {
        const double nu = pl->alpha * d->h[a];
        pl->dc[a] = make_dircoef(nu, g.n[a], d->bc[a] == MOL_BC_PERIODIC, pl->fp64,
                                 d->bc[a] == MOL_BC_NEUMANN);
    }
    pl->masked = (d->mask != nullptr);
    pl->neumann = d->ndim == 1 && d->bc[0] == MOL_BC_NEUMANN;
    pl->kmode = !pl->masked && g.ndim == 2 &&
                std::min(pl->dc[0].nu, pl->dc[1].nu) < KMODE_NU;
    if (!pl->masked)
        pl->agg_bytes = std::max(exact_agg_bytes(g, 0, pl->fp64),
                                 std::max(exact_agg_bytes(g, 1, pl->fp64), exact_agg_bytes(g, 2, pl->fp64)));
    if (pl->masked) {
        std::string err;
        pl->h_mask.assign(d->mask, d->mask + pl->npts);
        if (d->cross) pl->h_cross.assign(d->cross, d->cross + 4 * pl->npts);
        mol_status ms = masked_tables(pl, dry, err);
        if (ms != MOL_OK) return fail(ms, err);
        pl->unknowns = 0;
        for (int64_t i = 0; i < pl->npts; ++i) pl->unknowns += d->mask[i] ? 1 : 0;
    }
    if (!dry) load_tune_cache(pl);
    Builder b(*pl, dry);
    // step: u_next = 2 u - u_prev + rhs(u)
    bool ok = build_rhs(b, pl->step, B_UCURR, {{B_UNEXT, lin(B_UCURR, 2.0) + lin(B_UPREV, -1.0), 1.0}});
    // increment form: (u, du) -> (u + du + rhs, du + rhs), in place
    ok = ok && build_rhs(b, pl->inc_step, B_UCURR,
                         {{B_UCURR, lin(B_UCURR) + lin(B_UPREV), 1.0}, {B_UPREV, lin(B_UPREV), 1.0}});
    // fused solve programs (2D rectangles, P >= 2); where they cannot be
    // built (x lines longer than one workgroup: the chained x sweep needs the
    // whole line), mol_solve takes the step programs
    if (ok && !pl->masked && !pl->kmode && g.ndim == 2 && d->P >= 2) {
        const int n0 = pl->nws;
        pl->chain_a = b.new_ws();
        OutSpec o{};
        o.buf = pl->chain_a;
        o.dc[0] = 1.0;
        bool fused = b.emit(pl->solve_pro, 0, {lin(B_UCURR)}, {o}, 0);
        fused = fused && build_rhs_box(b, pl->solve_step, B_UCURR,
                                       {{B_UNEXT, lin(B_UCURR, 2.0) + lin(B_UPREV, -1.0), 1.0}},
                                       pl->chain_a);
        fused = fused && build_rhs_box(b, pl->solve_inc_step, B_UCURR,
                                       {{B_UCURR, lin(B_UCURR) + lin(B_UPREV), 1.0},
                                        {B_UPREV, lin(B_UPREV), 1.0}},
                                       pl->chain_a);
        if (!fused) {
            pl->solve_pro.clear();
            pl->solve_step.clear();
            pl->solve_inc_step.clear();
            pl->chain_a = -1;
            pl->nws = n0;
            b.err.clear();
        }
    }
    // step with a source term: its workspace ids start again from the first
    // field (the other programs keep nothing there between calls)
    if (ok && !pl->masked && d->P <= 2) {
        const int n0 = pl->nws;
        pl->nws = 0;
        pl->has_src = build_step_source(b, pl->step_src);
        if (!pl->has_src) pl->step_src.clear();
        pl->nws = std::max(n0, pl->nws);
    }
    if (ok && !pl->masked && d->P <= 2) {
        // shares the fused programs' chain field; nothing else kept
        const int n0 = pl->nws;
        pl->nws = 0;
        if (pl->chain_a >= 0) pl->nws = std::max(pl->nws, pl->chain_a - B_WS0 + 1);
        pl->has_solve_src = build_solve_source(b, pl->solve_src, pl->chain_a);
        if (!pl->has_solve_src) pl->solve_src.clear();
        pl->nws = std::max(n0, pl->nws);
    }
    if (ok) {
        const int n0 = pl->nws;
        pl->nws = 0;
        pl->has_start_g = build_start_g(b, pl->start_g);
        if (!pl->has_start_g) pl->start_g.clear();
        pl->nws = std::max(n0, pl->nws);
    }
    // start: u1 = u0 + rhs(u0)/2
    ok = ok && build_rhs(b, pl->start, B_IN, {{B_OUT, lin(B_IN), 0.5}});
    for (int op = 0; op <= MOL_OP_RHS && ok; ++op) {
        if (op <= MOL_OP_D_Z && (op % 3) >= d->ndim) continue;
        ok = build_apply(b, pl->apply[op], op);
    }
    if (!ok) return fail(MOL_E_UNSUPPORTED, b.err);
    // one more workspace field: scratch for the odd-step swap of mol_solve
    pl->nws += 1;
    return MOL_OK;
}

void resolve_op(const mol_plan_ *pl, const ProgOp &po, const void *uprev, const void *ucurr, void *unext,
                const void *in, void *out, const void **fp, void **op, const void *aux0,
                const void *aux1)
{
    auto res = [&](int b) -> void * {
        switch (b) {
        case B_UPREV: return const_cast<void *>(uprev);
        case B_UCURR: return const_cast<void *>(ucurr);
        case B_UNEXT: return unext;
        case B_IN: return const_cast<void *>(in);
        case B_OUT: return out;
        case B_AUX0: return const_cast<void *>(aux0);
        case B_AUX1: return const_cast<void *>(aux1);
        default: return pl->ws[b - B_WS0];
        }
    };
    for (int i = 0; i < po.op.nf; ++i) fp[i] = res(po.op.f[i]);
    for (int i = 0; i < po.op.no; ++i) op[i] = res(po.op.o[i]);
    if (po.op.chain) op[po.op.no] = res(po.op.ochain);
}

hipError_t run_program(mol_plan_ *pl, const Program &prog, const void *uprev, const void *ucurr,
                       void *unext, const void *in, void *out, hipStream_t st, const void *aux0,
                       const void *aux1)
{
    for (const ProgOp &po : prog) {
        const void *fp[MAXF];
        void *op[MAXO + 1];
        resolve_op(pl, po, uprev, ucurr, unext, in, out, fp, op, aux0, aux1);
        hipError_t e;
        if (pl->masked)
            e = launch_seg_op(po.op, pl, fp, op, st);
        else
            e = launch_sweep(po.op, pl->geom, pl->dc[po.op.dir], pl->fp64, fp, op, po.cfg, st, pl->agg);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

double program_bytes(const mol_plan_ *pl, const Program &prog)
{
    // fields read and written by every launch; a masked plan moves the
    // inside nodes only (plus the zero fill of its user-visible outputs)
    double b = 0, fill = 0;
    for (const ProgOp &po : prog) {
        b += (double)(po.op.nf + po.op.no + po.op.chain);
        if (pl->masked && po.op.proj) fill += (double)po.op.no;
    }
    if (pl->masked)
        return b * (double)pl->unknowns * (double)pl->es +
               fill * ((double)pl->npts + (double)(pl->npts - pl->unknowns) * (double)pl->es);
    return b * (double)pl->npts * (double)pl->es;
}

// drop the graphs captured by mol_solve
void drop_graphs(mol_plan_ *pl)
{
    if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->gtail) (void)hipGraphExecDestroy(pl->gtail);
    if (pl->gtailg) (void)hipGraphDestroy(pl->gtailg);
    pl->gexec = nullptr;
    pl->graph = nullptr;
    pl->gtail = nullptr;
    pl->gtailg = nullptr;
    pl->gtail_n = 0;
    pl->gA = pl->gB = nullptr;
    pl->ginc = -1;
}

void free_plan(mol_plan_ *pl, hipStream_t st)
{
    if (!pl) return;
    drop_graphs(pl);
    if (pl->async_ws) {
        if (pl->slab) (void)hipFreeAsync(pl->slab, st);
        pl->slab = nullptr;
        pl->ws.clear();
        pl->agg = nullptr;
    }
    for (void *p : pl->ws)
        if (p) (void)hipFree(p);
    if (pl->agg) {
        (void)hipFree(pl->agg);
        pl->agg = nullptr;
    }
    masked_free(pl);
    delete pl;
}

mol_status set_error(mol_status s, const std::string &msg) { return fail(s, msg); }

mol_status dev_err(hipError_t e, const char *what)
{
    std::string m = what;
    m += ": ";
    m += hipGetErrorString(e);
    return fail(MOL_E_DEVICE, m);
}

mol_status plan_create_async(const mol_desc *desc, hipStream_t st, mol_plan_ **out,
                             hipMemPool_t pool)
{
    if (!out) return fail(MOL_E_INVALID, "plan out-pointer is NULL");
    mol_plan_ *pl = new (std::nothrow) mol_plan_();
    if (!pl) return fail(MOL_E_NOMEM, "host allocation failed");
    mol_status s = build_plan(desc, pl, false);
    if (s != MOL_OK) {
        free_plan(pl);
        return s;
    }
    hipGetDevice(&pl->dev);
    pl->async_ws = true;
    // one block: the workspace fields (256-byte aligned), then the table;
    // a single allocation and a single clear per plan keep the host cost of
    // admitting a request low
    const size_t fb = ((size_t)pl->npts * pl->es + 255) & ~(size_t)255;
    const size_t total = fb * (size_t)pl->nws + pl->agg_bytes;
    pl->ws.assign(pl->nws, nullptr);
    if (total) {
        const hipError_t e = pool ? hipMallocFromPoolAsync(&pl->slab, total, pool, st)
                                  : hipMallocAsync(&pl->slab, total, st);
        if (e != hipSuccess) {
            pl->slab = nullptr;
            free_plan(pl, st);
            return fail(MOL_E_NOMEM, "stream-ordered allocation of the workspace failed");
        }
        unsigned char *base = static_cast<unsigned char *>(pl->slab);
        for (int i = 0; i < pl->nws; ++i) pl->ws[i] = base + (size_t)i * fb;
        if (pl->nws) (void)hipMemsetAsync(base, 0, fb * (size_t)pl->nws, st);
        if (pl->agg_bytes) pl->agg = base + fb * (size_t)pl->nws;
    }
    *out = pl;
    return MOL_OK;
}

void plan_destroy_async(mol_plan_ *pl, hipStream_t st) { free_plan(pl, st); }

}  // namespace molt

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

double mol_beta_max(int P)
{
    if (P < 1 || P > 8) return -1.0;
    return beta_max_of(P);
}

const char *mol_last_error(void) { return g_err.c_str(); }

size_t mol_workspace_bytes(const mol_desc *desc)
{
    mol_plan_ *pl = new (std::nothrow) mol_plan_();
    if (!pl) return 0;
    size_t r = 0;
    if (build_plan(desc, pl, true) == MOL_OK)
        r = (size_t)pl->nws * (size_t)pl->npts * pl->es + pl->table_bytes + pl->agg_bytes;
    masked_free(pl);
    delete pl;
    return r;
}

mol_status mol_plan_create(const mol_desc *desc, mol_plan **out)
{
    if (!out) return fail(MOL_E_INVALID, "plan out-pointer is NULL");
    mol_plan_ *pl = new (std::nothrow) mol_plan_();
    if (!pl) return fail(MOL_E_NOMEM, "host allocation failed");
    mol_status s = build_plan(desc, pl, false);
    if (s != MOL_OK) {
        free_plan(pl);
        return s;
    }
    hipGetDevice(&pl->dev);
    pl->ws.assign(pl->nws, nullptr);
    for (int i = 0; i < pl->nws; ++i) {
        hipError_t e = hipMalloc(&pl->ws[i], (size_t)pl->npts * pl->es);
        if (e != hipSuccess) {
            free_plan(pl);
            return fail(MOL_E_NOMEM, "hipMalloc of the workspace failed");
        }
        // workspace never holds stale non-finite values
        hipMemset(pl->ws[i], 0, (size_t)pl->npts * pl->es);
    }
    if (pl->agg_bytes && hipMalloc(&pl->agg, pl->agg_bytes) != hipSuccess) {
        pl->agg = nullptr;
        free_plan(pl);
        return fail(MOL_E_NOMEM, "hipMalloc of the aggregate table failed");
    }
    hipDeviceSynchronize();
    *out = pl;
    return MOL_OK;
}

mol_status mol_plan_destroy(mol_plan *pl)
{
    if (!pl) return MOL_OK;
    hipDeviceSynchronize();
    free_plan(pl);
    return MOL_OK;
}

mol_status mol_plan_get_info(const mol_plan *pl, mol_plan_info *info)
{
    if (!pl || !info) return fail(MOL_E_INVALID, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->beta = pl->beta;
    info->beta_max = pl->betamax;
    info->alpha = pl->alpha;
    for (int a = 0; a < pl->geom.ndim; ++a) info->nu[a] = pl->dc[a].nu;
    info->points = pl->npts;
    info->unknowns = pl->unknowns;
    info->segments[0] = pl->nsegs[0];
    info->segments[1] = pl->nsegs[1];
    // mol_solve runs the fused program when the plan has one
    const Program &sp = pl->solve_step.empty() ? pl->step : pl->solve_step;
    info->kernels_per_step = (int)sp.size();
    info->bytes_per_step = program_bytes(pl, sp);
    info->workspace_bytes = (size_t)pl->nws * (size_t)pl->npts * pl->es + pl->table_bytes + pl->agg_bytes;
    if (pl->has_src) {
        info->kernels_per_source_step = (int)pl->step_src.size();
        info->bytes_per_source_step = program_bytes(pl, pl->step_src);
    }
    return MOL_OK;
}

mol_status mol_start(mol_plan *pl, const void *u0, const void *g, void *u1, void *stream)
{
    if (!pl || !u0 || !u1) return fail(MOL_E_INVALID, "NULL argument");
    if (u0 == u1) return fail(MOL_E_INVALID, "u0 and u1 must not overlap");
    if (g && !pl->has_start_g) return fail(MOL_E_UNSUPPORTED, "initial velocity not available for this plan");
    if (g && g == u1) return fail(MOL_E_INVALID, "g and u1 must not overlap");
    hipError_t e = g ? run_program(pl, pl->start_g, nullptr, nullptr, nullptr, u0, u1, (hipStream_t)stream, g)
                     : run_program(pl, pl->start, nullptr, nullptr, nullptr, u0, u1, (hipStream_t)stream);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_start");
}

mol_status mol_step(mol_plan *pl, const void *u_prev, const void *u_curr, void *u_next, void *stream)
{
    if (!pl || !u_prev || !u_curr || !u_next) return fail(MOL_E_INVALID, "NULL argument");
    if (u_next == u_curr) return fail(MOL_E_INVALID, "u_next must not overlap u_curr");
    hipError_t e = run_program(pl, pl->step, u_prev, u_curr, u_next, nullptr, nullptr,
                               (hipStream_t)stream);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_step");
}

mol_status mol_step_source(mol_plan *pl, const void *u_prev, const void *u_curr, void *u_next,
                           const void *s_prev, const void *s_curr, const void *s_next, void *stream)
{
    if (!pl || !u_prev || !u_curr || !u_next || !s_curr) return fail(MOL_E_INVALID, "NULL argument");
    if (!pl->has_src)
        return fail(MOL_E_UNSUPPORTED, "source terms are given for box grids with P = 1 and 2");
    if (pl->desc.P == 2 && (!s_prev || !s_next))
        return fail(MOL_E_INVALID, "P = 2 needs the source at three time levels");
    if (u_next == u_curr) return fail(MOL_E_INVALID, "u_next must not overlap u_curr");
    if (u_next == s_curr || (pl->desc.P == 2 && (u_next == s_prev || u_next == s_next)))
        return fail(MOL_E_INVALID, "u_next must not overlap a source field");
    hipError_t e = run_program(pl, pl->step_src, u_prev, u_curr, u_next, s_curr, nullptr,
                               (hipStream_t)stream, s_prev, s_next);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_step_source");
}

}  // extern "C"

namespace {

double binom_or0(int m, int k) { return (m >= 0 && k >= 0 && m >= k) ? binom(m, k) : 0.0; }

// Data of application p (1..P) of D at one end of a line with boundary data,
// from U_j = (X^j q)(end), X = d_xx / alpha^2, j = 0..P, where q is u
// (Dirichlet: values) or u_x (Neumann: slopes): the end value of D^{p-1} q
// (val), the curvature of D^{p-1} u there (kap, Dirichlet only) and the end
// value of L^{-1} D^{p-1} q (tgt); D = -X (1 - X)^{-1} and L^{-1} = (1 - X)^{-1}
// as power series in X, truncated at X^P.
void ilw_pass(int p, int P, const double *U, double alpha, double &val, double &kap, double &tgt)
{
    const double s = (p % 2) ? 1.0 : -1.0;        // (-1)^(p-1)
    double v = 0.0, k = 0.0, t = 0.0;
    for (int j = 0; j <= P; ++j) {
        t += binom_or0(j, p - 1) * U[j];
        v += (p == 1) ? (j == 0 ? U[j] : 0.0) : binom_or0(j - 1, p - 2) * U[j];
        k += (p == 1) ? (j == 1 ? U[j] : 0.0) : binom_or0(j - 2, p - 2) * U[j];
    }
    val = s * v;
    kap = s * alpha * alpha * k;
    tgt = s * t;
}

}  // namespace

extern "C" {

mol_status mol_step_bdata(mol_plan *pl, const void *u_prev, const void *u_curr, void *u_next,
                          const double *bdata, void *stream)
{
    if (!pl || !u_prev || !u_curr || !u_next || !bdata) return fail(MOL_E_INVALID, "NULL argument");
    if (u_next == u_curr) return fail(MOL_E_INVALID, "u_next must not overlap u_curr");
    const bool dir = pl->geom.ndim == 1 && pl->geom.dirichlet[0] != 0;
    if (pl->masked || !(dir || pl->neumann))
        return fail(MOL_E_UNSUPPORTED, "boundary data are given for 1D Dirichlet or Neumann plans");
    const int P = pl->desc.P;
    Program prog = pl->step;
    if ((int)prog.size() != P) return fail(MOL_E_UNSUPPORTED, "internal: 1D step program shape");
    // U_j = (X^j u)(end) = (dt / beta)^{2j} d_t^{2j} (data): even space
    // derivatives of u (Dirichlet) or of u_x (Neumann) from the data (Sec. 3.2)
    const double r = 1.0 / ((pl->alpha * pl->desc.c) * (pl->alpha * pl->desc.c));
    double Ua[16], Ub[16];
    double rj = 1.0;
    for (int j = 0; j <= P; ++j) {
        Ua[j] = bdata[j] * rj;
        Ub[j] = bdata[P + 2 + j] * rj;
        rj *= r;
    }
    const double h = pl->desc.h[0];
    for (int p = 1; p <= P; ++p) {
        SweepOp &op = prog[p - 1].op;
        if (op.dir != 0 || op.ns != 1) return fail(MOL_E_UNSUPPORTED, "internal: 1D step program shape");
        double va, vb, ka, kb, ta, tb;
        ilw_pass(p, P, Ua, pl->alpha, va, ka, ta);
        ilw_pass(p, P, Ub, pl->alpha, vb, kb, tb);
        if (dir) {
            // curvature of D^{p-1} u in the end cells (times h^2) and the
            // values L^{-1} D^{p-1} u takes at the ends
            op.bmode = 1;
            op.bk[0] = ka * h * h;
            op.bk[1] = kb * h * h;
            op.bt[0] = ta;
            op.bt[1] = tb;
        } else {
            // slopes of D^{p-1} u at the ends (the end cells' quadratics) and
            // the slopes L^{-1} D^{p-1} u takes there, as the sweep's closure
            // reads them
            op.bmode = 2;
            op.bk[0] = 2.0 * h * va;
            op.bk[1] = 2.0 * h * vb;
            op.bt[0] = ta / pl->alpha;
            op.bt[1] = -tb / pl->alpha;
        }
    }
    if (dir) {
        prog.back().op.bend[0] = bdata[P + 1];
        prog.back().op.bend[1] = bdata[2 * P + 3];
    }
    hipError_t e = run_program(pl, prog, u_prev, u_curr, u_next, nullptr, nullptr, (hipStream_t)stream);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_step_bdata");
}

mol_status mol_apply(mol_plan *pl, int op, const void *in, void *out, void *stream)
{
    if (!pl || !in || !out) return fail(MOL_E_INVALID, "NULL argument");
    if (op < 0 || op > MOL_OP_RHS) return fail(MOL_E_INVALID, "unknown operator");
    if (in == out) return fail(MOL_E_INVALID, "in and out must not overlap");
    if (pl->apply[op].empty()) return fail(MOL_E_INVALID, "operator not available for this plan");
    hipError_t e = run_program(pl, pl->apply[op], nullptr, nullptr, nullptr, in, out,
                               (hipStream_t)stream);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_apply");
}

}  // extern "C"

namespace {

// one replay unit of mol_solve: UNIT_STEPS steps (three-level: in pairs, so
// that the fields return to their buffers), one graph launch per unit
constexpr int64_t UNIT_STEPS = 8;

// Pinned staging of mol_step_batch's argument tables: a ring of slots, each
// reused once the copy that last read it has completed (its event).
struct BatchStaging {
    static constexpr int NSLOT = 4;
    struct Slot {
        void *h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool used = false;
    };
    std::mutex mu;
    Slot slot[NSLOT];
    unsigned next = 0;
};
BatchStaging g_batch;

// count steps of the solve program on (A, B), launched directly; the
// three-level form alternates the roles of the two buffers
hipError_t solve_steps(mol_plan_ *pl, void *A, void *B, int64_t count, bool inc, hipStream_t s)
{
    const bool fused = !pl->solve_step.empty();
    const Program &stepP = fused ? pl->solve_step : pl->step;
    const Program &incP = fused ? pl->solve_inc_step : pl->inc_step;
    hipError_t r = hipSuccess;
    for (int64_t i = 0; i < count && r == hipSuccess; ++i) {
        if (inc) r = run_program(pl, incP, A, B, nullptr, nullptr, nullptr, s);
        else if (i % 2 == 0) r = run_program(pl, stepP, A, B, A, nullptr, nullptr, s);
        else r = run_program(pl, stepP, B, A, B, nullptr, nullptr, s);
    }
    return r;
}

// a graph of count steps on (A, B), captured on st and instantiated
mol_status capture_steps(mol_plan_ *pl, void *A, void *B, int64_t count, bool inc, hipStream_t st,
                         hipGraph_t *gout, hipGraphExec_t *eout)
{
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return dev_err(e, "hipStreamBeginCapture");
    const hipError_t eu = solve_steps(pl, A, B, count, inc, st);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(st, &gr);
    if (eu != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return dev_err(eu, "capture");
    }
    if (e != hipSuccess) return dev_err(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return dev_err(e, "hipGraphInstantiate");
    }
    *gout = gr;
    *eout = ge;
    return MOL_OK;
}

// Makes sure the graphs mol_solve(A, B, nsteps) replays exist: the unit
// (nsteps >= UNIT_STEPS) and the tail of the even part of the remainder.
// Graphs of other buffers are dropped first.
mol_status ensure_graphs(mol_plan_ *pl, void *A, void *B, int64_t nsteps, bool inc, hipStream_t st)
{
    if (pl->gA != A || pl->gB != B || pl->ginc != (int)inc) drop_graphs(pl);
    pl->gA = A;
    pl->gB = B;
    pl->ginc = (int)inc;
    if (nsteps >= UNIT_STEPS && !pl->gexec) {
        mol_status s = capture_steps(pl, A, B, UNIT_STEPS, inc, st, &pl->graph, &pl->gexec);
        if (s != MOL_OK) return s;
    }
    const int64_t rest = nsteps % UNIT_STEPS;
    const int64_t tail = inc ? rest : rest - rest % 2;
    if (tail > 0 && pl->gtail_n != tail) {
        if (pl->gtail) (void)hipGraphExecDestroy(pl->gtail);
        if (pl->gtailg) (void)hipGraphDestroy(pl->gtailg);
        pl->gtail = nullptr;
        pl->gtailg = nullptr;
        pl->gtail_n = 0;
        mol_status s = capture_steps(pl, A, B, tail, inc, st, &pl->gtailg, &pl->gtail);
        if (s != MOL_OK) return s;
        pl->gtail_n = tail;
    }
    return MOL_OK;
}

}  // namespace

extern "C" {

mol_status mol_solve_prepare(mol_plan *pl, void *A, void *B, int64_t nsteps, void *stream)
{
    if (!pl || !A || !B) return fail(MOL_E_INVALID, "NULL argument");
    if (A == B) return fail(MOL_E_INVALID, "u_prev and u_curr must differ");
    if (nsteps < 0) return fail(MOL_E_INVALID, "nsteps < 0");
    if ((pl->desc.flags & MOL_NO_GRAPH) || stream == nullptr) return MOL_OK;
    return ensure_graphs(pl, A, B, nsteps, (pl->desc.flags & MOL_INCREMENT_FORM) != 0,
                         (hipStream_t)stream);
}

mol_status mol_solve(mol_plan *pl, void *A, void *B, int64_t nsteps, void *stream)
{
    if (!pl || !A || !B) return fail(MOL_E_INVALID, "NULL argument");
    if (A == B) return fail(MOL_E_INVALID, "u_prev and u_curr must differ");
    if (nsteps < 0) return fail(MOL_E_INVALID, "nsteps < 0");
    if (nsteps == 0) return MOL_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool inc = (pl->desc.flags & MOL_INCREMENT_FORM) != 0;
    // graph capture needs a stream other than the legacy default stream
    const bool graph = !(pl->desc.flags & MOL_NO_GRAPH) && st != nullptr;
    const size_t bytes = (size_t)pl->npts * pl->es;
    hipError_t e;
    if (inc) {
        // A <- du = B - A, steps in place on (B, A), then A <- B - du
        e = launch_axpby(pl->fp64, pl->npts, 1.0, B, -1.0, A, A, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
    }
    const bool fused = !pl->solve_step.empty();
    const Program &stepP = fused ? pl->solve_step : pl->step;
    if (graph) {
        // captured before the prologue's launch below: capture records the
        // launches without running them
        mol_status s = ensure_graphs(pl, A, B, nsteps, inc, st);
        if (s != MOL_OK) return s;
    }
    if (fused) {
        // D_x of the current field for the first stage of the first step
        e = run_program(pl, pl->solve_pro, A, B, nullptr, nullptr, nullptr, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
    }
    const int64_t reps = nsteps / UNIT_STEPS;
    for (int64_t r = 0; r < reps; ++r) {
        e = graph ? hipGraphLaunch(pl->gexec, st) : solve_steps(pl, A, B, UNIT_STEPS, inc, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
    }
    // the steps beyond whole units: the even part (or all of them in the
    // increment form) as one more graph, then one odd step
    const int64_t rest = nsteps % UNIT_STEPS;
    const int64_t tail = inc ? rest : rest - rest % 2;
    if (tail > 0) {
        e = graph ? hipGraphLaunch(pl->gtail, st) : solve_steps(pl, A, B, tail, inc, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
    }
    if (!inc && (rest % 2)) {
        // odd count: one more step into A, then swap the contents of A and B
        e = run_program(pl, stepP, A, B, A, nullptr, nullptr, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
        if (pl->nws < 1) return fail(MOL_E_DEVICE, "no workspace for the swap");
        void *W = pl->ws[pl->nws - 1];
        e = hipMemcpyAsync(W, A, bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(A, B, bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(B, W, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve swap");
    }
    if (inc) {
        e = launch_axpby(pl->fp64, pl->npts, 1.0, B, -1.0, A, A, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve");
    }
    return MOL_OK;
}

mol_status mol_solve_source(mol_plan *pl, void *A, void *B, int64_t nsteps, const void *G,
                            const void *CG, const double *f, void *stream)
{
    if (!pl || !A || !B || !G) return fail(MOL_E_INVALID, "NULL argument");
    if (!pl->has_solve_src)
        return fail(MOL_E_UNSUPPORTED, "separable sources are given for box grids with P = 1 and 2");
    if (pl->desc.flags & MOL_INCREMENT_FORM)
        return fail(MOL_E_UNSUPPORTED, "separable sources step the three-level form only");
    if (pl->desc.P == 2 && !CG) return fail(MOL_E_INVALID, "P = 2 needs C[G]");
    if (A == B) return fail(MOL_E_INVALID, "u_prev and u_curr must differ");
    if (G == A || G == B || (CG && (CG == A || CG == B)))
        return fail(MOL_E_INVALID, "G and C[G] must not overlap the solution fields");
    if (nsteps < 0) return fail(MOL_E_INVALID, "nsteps < 0");
    if (nsteps == 0) return MOL_OK;
    if (!f) return fail(MOL_E_INVALID, "NULL f");
    hipStream_t st = (hipStream_t)stream;
    const double a2 = (pl->beta / pl->alpha) * (pl->beta / pl->alpha);
    const double sg = a2 / 12.0;
    const bool fused = pl->chain_a >= 0;
    hipError_t e = hipSuccess;
    if (fused) {
        e = run_program(pl, pl->solve_pro, A, B, nullptr, nullptr, nullptr, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve_source");
    }
    Program prog = pl->solve_src;
    SweepOp &last = prog.back().op;
    for (int64_t k = 0; k < nsteps; ++k) {
        // step k makes u^{n+k+1} from S at t_{n+k-1}, t_{n+k}, t_{n+k+1}
        if (pl->desc.P == 1) {
            last.mOF[0][pl->src_fg] = a2 * f[k + 1];
        } else {
            last.mOF[0][pl->src_fg] = sg * (f[k + 2] + 10.0 * f[k + 1] + f[k]);
            last.mOF[0][pl->src_fcg] = -pl->beta * pl->beta * sg * f[k + 1];
        }
        e = (k % 2 == 0) ? run_program(pl, prog, A, B, A, nullptr, nullptr, st, G, CG)
                         : run_program(pl, prog, B, A, B, nullptr, nullptr, st, G, CG);
        if (e != hipSuccess) return dev_err(e, "mol_solve_source");
    }
    if (nsteps % 2) {
        // the newest field is in A: swap the contents of A and B
        void *W = pl->ws[pl->nws - 1];
        const size_t bytes = (size_t)pl->npts * pl->es;
        e = hipMemcpyAsync(W, A, bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(A, B, bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(B, W, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return dev_err(e, "mol_solve_source swap");
    }
    return MOL_OK;
}

mol_status mol_profile_step(mol_plan *pl, const void *u_prev, const void *u_curr, void *u_next,
                            int reps, void *stream, int max, double *ms, double *bytes, int *dir,
                            int *nsweep, int *count)
{
    if (!pl || !u_prev || !u_curr || !u_next || reps < 1) return fail(MOL_E_INVALID, "bad arguments");
    // the program mol_solve replays (fused when the plan has one)
    const bool fused = !pl->solve_step.empty();
    const Program &sp = fused ? pl->solve_step : pl->step;
    const int nk = (int)sp.size();
    if (count) *count = nk;
    hipStream_t st = (hipStream_t)stream;
    std::vector<hipEvent_t> ev(2 * (size_t)nk * reps);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(MOL_E_DEVICE, "hipEventCreate failed");
    hipError_t e = hipSuccess;
    if (fused) e = run_program(pl, pl->solve_pro, u_prev, u_curr, u_next, nullptr, nullptr, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        for (int i = 0; i < nk && e == hipSuccess; ++i) {
            Program one(1, sp[i]);
            hipEvent_t e0 = ev[2 * ((size_t)r * nk + i)], e1 = ev[2 * ((size_t)r * nk + i) + 1];
            if (pl->masked) {
                // several launches per sweep: events around the group
                e = hipEventRecord(e0, st);
                if (e == hipSuccess) e = run_program(pl, one, u_prev, u_curr, u_next, nullptr, nullptr, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
            } else {
                // the launch records the kernel's own start and stop
                g_prof.start = e0;
                g_prof.stop = e1;
                e = run_program(pl, one, u_prev, u_curr, u_next, nullptr, nullptr, st);
                g_prof = ProfEvents{};
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int i = 0; i < nk && i < max && e == hipSuccess; ++i) {
        double tot = 0.0;
        for (int r = 0; r < reps; ++r) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[2 * ((size_t)r * nk + i)], ev[2 * ((size_t)r * nk + i) + 1]);
            tot += t;
        }
        const SweepOp &op = sp[i].op;
        if (ms) ms[i] = tot / reps;
        if (bytes) bytes[i] = (double)(op.nf + op.no + op.chain) * (double)pl->npts * (double)pl->es;
        if (dir) dir[i] = op.dir;
        if (nsweep) nsweep[i] = op.yy ? 2 : op.ns;
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_profile_step");
}

mol_status mol_plan_kernel_configs(const mol_plan *pl, int kernel, int *ids, int max, int *count,
                                   int *current)
{
    if (!pl) return fail(MOL_E_INVALID, "NULL plan");
    const Program &sp = pl->solve_step.empty() ? pl->step : pl->solve_step;
    if (kernel < 0 || kernel >= (int)sp.size()) return fail(MOL_E_INVALID, "kernel index out of range");
    const SweepOp &op = sp[kernel].op;
    int cnt = 0;
    if (!pl->masked) {
        for (int c = 0; c < config_count(op); ++c) {
            int cf[2] = {c, 0};
            if (!config_valid(pl->geom, pl->dc[op.dir], op, pl->fp64, cf))
                continue;
            if (ids && cnt < max) ids[cnt] = c;
            ++cnt;
        }
    }
    if (count) *count = cnt;
    if (current) *current = sp[kernel].cfg[0];
    return MOL_OK;
}

mol_status mol_plan_set_kernel_config(mol_plan *pl, int kernel, int config)
{
    if (!pl) return fail(MOL_E_INVALID, "NULL plan");
    if (pl->masked) return fail(MOL_E_UNSUPPORTED, "masked plans have a single configuration");
    Program &sp = pl->solve_step.empty() ? pl->step : pl->solve_step;
    if (kernel < 0 || kernel >= (int)sp.size()) return fail(MOL_E_INVALID, "kernel index out of range");
    const SweepOp ref = sp[kernel].op;
    int cf[2] = {config, 0};
    if (!config_valid(pl->geom, pl->dc[ref.dir], ref, pl->fp64, cf))
        return fail(MOL_E_INVALID, "configuration not valid for this kernel");
    const std::string key = tune_op_key(ref);
    for (Program *pr : {&pl->step, &pl->start, &pl->inc_step, &pl->solve_pro, &pl->solve_step,
                        &pl->solve_inc_step, &pl->step_src, &pl->start_g, &pl->solve_src}) {
        for (ProgOp &po : *pr)
            if (tune_op_key(po.op) == key) po.cfg[0] = config;
    }
    for (Program &pr : pl->apply)
        for (ProgOp &po : pr)
            if (tune_op_key(po.op) == key) po.cfg[0] = config;
    // the captured graphs hold the old launches
    drop_graphs(pl);
    return MOL_OK;
}

mol_status mol_plan_tune_key(const mol_plan *pl, int kernel, char *buf, int len)
{
    if (!pl || !buf || len < 1) return fail(MOL_E_INVALID, "bad arguments");
    const Program &sp = pl->solve_step.empty() ? pl->step : pl->solve_step;
    if (kernel < 0 || kernel >= (int)sp.size()) return fail(MOL_E_INVALID, "kernel index out of range");
    const std::string k = tune_problem_key(pl) + " | " + tune_op_key(sp[kernel].op);
    snprintf(buf, (size_t)len, "%s", k.c_str());
    return MOL_OK;
}

mol_status mol_step_batch(mol_plan *const *plans, const void *const *u_prev,
                          const void *const *u_curr, void *const *u_next, int count, void *stream)
{
    if (count < 0 || (count > 0 && (!plans || !u_prev || !u_curr || !u_next)))
        return fail(MOL_E_INVALID, "bad batch arguments");
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !u_prev[i] || !u_curr[i] || !u_next[i]) return fail(MOL_E_INVALID, "NULL argument");
        if (u_next[i] == u_curr[i]) return fail(MOL_E_INVALID, "u_next must not overlap u_curr");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(MOL_E_INVALID, "plans of a batch must be distinct");
    }
    if (count == 0) return MOL_OK;
    const hipStream_t st = (hipStream_t)stream;
    // argument sets of every plan's step: launches at the same position of
    // their steps that share a kernel instantiation form one group; launches
    // that cannot share one (line objects, exact two-pass sweeps, L^{-1} and
    // boundary-data sweeps) run by themselves at their position
    struct Ent {
        int64_t blocks;
        size_t off, bytes;        // in args
    };
    struct Direct {
        int k, i;
    };
    std::vector<unsigned char> args;
    std::map<std::pair<int, SweepKey>, std::vector<Ent>> groups;
    std::vector<Direct> direct;
    int maxk = 0;
    for (int i = 0; i < count; ++i) {
        mol_plan_ *pl = plans[i];
        const Program &prog = pl->step;
        maxk = std::max(maxk, (int)prog.size());
        const size_t asz = sweep_args_bytes(pl->fp64);
        for (int k = 0; k < (int)prog.size(); ++k) {
            if (pl->masked) {
                direct.push_back({k, i});
                continue;
            }
            const void *fp[MAXF];
            void *op[MAXO + 1];
            resolve_op(pl, prog[k], u_prev[i], u_curr[i], u_next[i], nullptr, nullptr, fp, op);
            const size_t off = args.size();
            args.resize(off + asz);
            SweepKey key;
            int64_t blocks = 0;
            if (!sweep_prepare(prog[k].op, pl->geom, pl->dc[prog[k].op.dir], pl->fp64, fp, op, prog[k].cfg,
                               args.data() + off, key, blocks)) {
                args.resize(off);
                direct.push_back({k, i});
                continue;
            }
            groups[{k, key}].push_back({blocks, off, asz});
        }
    }
    // one table per group: first[] (nent + 1 workgroup offsets), then the
    // argument sets; all tables in one stream-ordered device allocation,
    // copied from pinned staging
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t total = 0;
    for (auto &g : groups) {
        total += a256((g.second.size() + 1) * sizeof(int64_t));
        for (const Ent &e : g.second) total += e.bytes;
        total = a256(total);
    }
    struct Launch {
        int k;
        SweepKey key;
        size_t tab, first;
        int nent;
        int64_t blocks;
    };
    std::vector<Launch> ls;
    void *dtab = nullptr;
    if (total > 0) {
        std::unique_lock<std::mutex> lk(g_batch.mu);
        BatchStaging::Slot &sl = g_batch.slot[g_batch.next++ % BatchStaging::NSLOT];
        if (sl.used && hipEventSynchronize(sl.ev) != hipSuccess) return fail(MOL_E_DEVICE, "staging wait failed");
        if (total > sl.cap) {
            if (sl.h) (void)hipHostFree(sl.h);
            sl.h = nullptr;
            sl.cap = 0;
            const size_t cap = std::max(total * 2, (size_t)1 << 16);
            if (hipHostMalloc(&sl.h, cap, hipHostMallocDefault) != hipSuccess)
                return fail(MOL_E_NOMEM, "pinned staging allocation failed");
            sl.cap = cap;
        }
        if (!sl.ev && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
            return fail(MOL_E_DEVICE, "staging event failed");
        unsigned char *h = static_cast<unsigned char *>(sl.h);
        size_t pos = 0;
        for (auto &g : groups) {
            const size_t nent = g.second.size();
            int64_t *first = reinterpret_cast<int64_t *>(h + pos);
            const size_t fpos = pos;
            pos += a256((nent + 1) * sizeof(int64_t));
            const size_t tpos = pos;
            int64_t b = 0;
            for (size_t e = 0; e < nent; ++e) {
                first[e] = b;
                b += g.second[e].blocks;
                std::memcpy(h + pos, args.data() + g.second[e].off, g.second[e].bytes);
                pos += g.second[e].bytes;
            }
            first[nent] = b;
            pos = a256(pos);
            ls.push_back({g.first.first, g.first.second, tpos, fpos, (int)nent, b});
        }
        if (hipMallocAsync(&dtab, total, st) != hipSuccess) return fail(MOL_E_NOMEM, "table allocation failed");
        hipError_t e = hipMemcpyAsync(dtab, sl.h, total, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
        if (e != hipSuccess) {
            (void)hipFreeAsync(dtab, st);
            return dev_err(e, "mol_step_batch table copy");
        }
        sl.used = true;
    }
    // position k of every plan's step after position k - 1
    hipError_t e = hipSuccess;
    for (int k = 0; k < maxk && e == hipSuccess; ++k) {
        for (const Direct &dr : direct) {
            if (dr.k != k || e != hipSuccess) continue;
            mol_plan_ *pl = plans[dr.i];
            const Program one(1, pl->step[k]);
            e = run_program(pl, one, u_prev[dr.i], u_curr[dr.i], u_next[dr.i], nullptr, nullptr, st);
        }
        for (const Launch &l : ls) {
            if (l.k != k || e != hipSuccess) continue;
            unsigned char *d = static_cast<unsigned char *>(dtab);
            e = launch_sweep_batch(l.key, d + l.tab, reinterpret_cast<const int64_t *>(d + l.first), l.nent,
                                   l.blocks, st);
        }
    }
    if (dtab) {
        const hipError_t ef = hipFreeAsync(dtab, st);
        if (e == hipSuccess) e = ef;
    }
    return e == hipSuccess ? MOL_OK : dev_err(e, "mol_step_batch");
}

}  // extern "C"
