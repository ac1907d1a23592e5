// Plan state and the kernel-program builder shared by the plan sources.
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/molt.h"
#include "molt_internal.h"

namespace molt {

// buffer ids inside a program: caller fields, then plan workspace fields
// Buffers of a program: caller fields, then workspace fields from B_WS0.  Two
// more caller fields: the step with a source term reads S^n as B_IN and
// S^{n-1}, S^{n+1} as B_AUX0, B_AUX1; the start with an initial velocity reads
// g as B_AUX0.
enum { B_UPREV = 0, B_UCURR = 1, B_UNEXT = 2, B_IN = 3, B_OUT = 4, B_AUX0 = 5, B_AUX1 = 6, B_WS0 = 7 };

struct ProgOp {
    SweepOp op;
    int cfg[2];
};
typedef std::vector<ProgOp> Program;

}  // namespace molt

struct mol_plan_ {
    mol_desc desc{};
    molt::Geom geom{};
    bool fp64 = false;
    double beta = 0, betamax = 0, alpha = 0;
    molt::DirCoef dc[3]{};
    int64_t npts = 0, unknowns = 0;
    size_t es = 8;
    int nws = 0;                       // workspace fields
    std::vector<void *> ws;            // device workspace fields
    // aggregate table of the exact two-pass strided sweeps (box plans in 2D
    // and 3D; sized for the smallest tile along y and z)
    void *agg = nullptr;
    size_t agg_bytes = 0;
    molt::Program step, start, inc_step;
    // fused solve (2D rectangles, P >= 2): the last x sweep of a step also
    // writes D_x u^{n+1} into ws chain_a for the next step's first stage
    molt::Program solve_pro, solve_step, solve_inc_step;
    int chain_a = -1;
    molt::Program apply[9];
    // step with a source term (box plans, P <= 2; workspace shared with the
    // other programs: it holds nothing between calls)
    molt::Program step_src;
    bool has_src = false;
    // start with an initial velocity (workspace shared in the same way)
    molt::Program start_g;
    bool has_start_g = false;
    // steps with a separable source f(t) G(x): the step program (fused when
    // the plan has one) whose last launch also takes G (B_AUX0) and C[G]
    // (B_AUX1, P = 2) elementwise, their weights set per step
    molt::Program solve_src;
    bool has_solve_src = false;
    int src_fg = -1, src_fcg = -1;     // field slots of G and C[G] in its last launch
    int dev = 0;
    // graph cache for mol_solve: the unit of UNIT_STEPS steps and one tail of
    // an even number of steps (gtail_n), both for the buffers (gA, gB)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gtail = nullptr;
    hipGraph_t gtailg = nullptr;
    int64_t gtail_n = 0;
    const void *gA = nullptr, *gB = nullptr;
    int ginc = -1;
    // masked plans (embedded boundary)
    bool masked = false;
    // 1D line with Neumann ends: every x sweep runs in boundary-data mode
    // (zero data unless mol_step_bdata gives some), no projection
    bool neumann = false;
    molt::SegTable seg[2];
    // y line objects on the transposed grid (x <-> y), swept through
    // transposed copies of a launch's fields (coalesced rows)
    molt::SegTable segT;
    static constexpr int NTBUF = 4;
    void *tbuf[NTBUF] = {};
    unsigned char *d_mask = nullptr;
    int64_t nsegs[2] = {0, 0};
    size_t table_bytes = 0;
    std::vector<unsigned char> h_mask;  // kept for table construction
    std::vector<double> h_cross;
    // tuned launch configurations: key "dir nf ns no" -> config id
    std::vector<std::pair<std::string, int>> tuned;
    // workspace from the stream-ordered allocator (plans of the request
    // server): one block holding the workspace fields and the aggregate table
    bool async_ws = false;
    void *slab = nullptr;
    // 2D box plans at small nu: the ADI operator C composed as
    // D_x(L_y^-1 v) + L_x^-1(D_y v), with L^-1 swept by its own recurrences
    bool kmode = false;
};

namespace molt {

// 2D box plans whose smaller nu lies below this compose C from L^{-1} and D
// sweeps (D_x(L_y^-1 v) + L_x^-1(D_y v)) instead of D sweeps alone: the D-form
// C of data that varies on the grid scale cancels about 1 / (2 min K^) ~ 3 / nu
// (60 at this nu) of its leading digits
constexpr double KMODE_NU = 0.05;

// linear expression over buffers
typedef std::vector<std::pair<int, double>> Lin;

inline Lin lin(int b, double c = 1.0) { return Lin{{b, c}}; }
inline Lin operator+(Lin a, const Lin &b)
{
    a.insert(a.end(), b.begin(), b.end());
    return a;
}
inline Lin operator*(double s, Lin a)
{
    for (auto &t : a) t.second *= s;
    return a;
}

// weights of the schemes (eq. Full_2D, eq. update_P) and of the start's odd series
double stage_c(int p, int m, double beta);
double A_p(int p, double beta);
double start_b(int p, int m, double beta);

struct OutSpec {
    int buf;
    Lin elem;
    double dc[MAXS];
};

struct Builder {
    mol_plan_ &pl;
    bool dry;
    std::string err;
    // weights of the terms C^{m-1} D^{p-m} C of Table 2's schedule: the step's
    // c_{p,m} (series 0) or the odd series of the start, b_{p,m} (series 1)
    int series = 0;
    explicit Builder(mol_plan_ &p, bool d) : pl(p), dry(d) {}
    double coef(int p, int m) const { return series ? start_b(p, m, pl.beta) : stage_c(p, m, pl.beta); }
    double Ap(int p) const
    {
        double s = 0.0;
        for (int m = 1; m <= p; ++m) s += coef(p, m);
        return s;
    }

    int new_ws() { return B_WS0 + pl.nws++; }

    // one directional launch: combos = swept combinations, outs = outputs
    // kf[k] = 1: combination k is swept for L^{-1} (else D)
    bool emit(Program &prog, int dir, const std::vector<Lin> &combos,
              const std::vector<OutSpec> &outs, int proj, int chain_buf = -1,
              const std::vector<int> &kf = {});

    // chained strided launch: v1 = e1 + D s1, y = D v1 along direction dir;
    // output expressions may name the two results through the ids V1 and Y
    static constexpr int V1 = -2, Y = -3;
    bool yy_available(int dir, int nf, int no) const;
    bool emit_yy(Program &prog, int dir, const Lin &s1, const Lin &e1,
                 const std::vector<std::pair<int, Lin>> &outs);
};

// How the right-hand side sum_{p,m} c_{p,m} C^m D^{p-m} u is consumed: each
// final output = elem + r * rhs.
struct FinalOut {
    int buf;
    Lin elem;
    double r;
};

std::string tune_problem_key(const mol_plan_ *pl);
std::string tune_op_key(const SweepOp &op);

std::vector<OutSpec> finals(const std::vector<FinalOut> &fo, const Lin &rhs_elem, double rhs_dcoef);

// masked (embedded boundary) plans
bool build_rhs_masked(Builder &b, Program &prog, int u, const std::vector<FinalOut> &fo);
bool build_apply_masked(Builder &b, Program &prog, int op);
mol_status masked_tables(mol_plan_ *pl, bool dry, std::string &err);
void masked_free(mol_plan_ *pl);
hipError_t launch_seg_op(const SweepOp &op, const mol_plan_ *pl, const void *const *fptr,
                         void *const *optr, hipStream_t st);

// Device pointers of one launch of a program: fields (op.nf) and outputs
// (op.no, then the chained output) for the given caller fields.
void resolve_op(const mol_plan_ *pl, const ProgOp &po, const void *uprev, const void *ucurr, void *unext,
                const void *in, void *out, const void **fp, void **op, const void *aux0 = nullptr,
                const void *aux1 = nullptr);
// Run a program on st (one launch per op).
hipError_t run_program(mol_plan_ *pl, const Program &prog, const void *uprev, const void *ucurr,
                       void *unext, const void *in, void *out, hipStream_t st,
                       const void *aux0 = nullptr, const void *aux1 = nullptr);

// The plan of a descriptor without its workspace (dry: no device tables
// either), and its release (frees pl->ws entries; hipFreeAsync on st for
// plans of the request server).
mol_status build_plan(const mol_desc *d, mol_plan_ *pl, bool dry);
void free_plan(mol_plan_ *pl, hipStream_t st = nullptr);
// A failing status with the message mol_last_error() returns; dev_err adds
// the HIP error string.
mol_status set_error(mol_status s, const std::string &msg);
mol_status dev_err(hipError_t e, const char *what);

// plans whose workspace is allocated and freed in stream order on st (no
// device-wide synchronisation; used by the request server), as one block from
// pool (nullptr: the device's default pool)
mol_status plan_create_async(const mol_desc *desc, hipStream_t st, mol_plan_ **out,
                             hipMemPool_t pool = nullptr);
void plan_destroy_async(mol_plan_ *pl, hipStream_t st);

}  // namespace molt
