/*
 * Plain FP64 CPU oracle for the MOL^T recursive-convolution wave solver
 * (Causley & Christlieb, "Higher order A-stable schemes for the wave equation
 * using a recursive convolution approach").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares nothing with the
 * HIP library: no headers, no tables, no helpers.
 *
 * What it computes, in the paper's order and notation:
 *   - L^{-1} along one grid line (Sec. 2, eq. L_Inverse) as the characteristic
 *     split I^L + I^R, each obtained by its exponential recurrence (Sec. 2,
 *     the two recurrence identities), with the local integrals taken over one
 *     cell against the quadratic through the three nodes centred on the node
 *     the recurrence arrives at; then the homogeneous solutions
 *     A e^{-alpha(x-a)} + B e^{-alpha(b-x)} that enforce the boundary values
 *     (Sec. 2, "boundary corrections on a finite domain"; Sec. 3.2).
 *   - D = 1 - L^{-1} (Sec. 2, eq. D_def_1d), the directional operators
 *     L_gamma^{-1}, D_gamma (Sec. 4, eq. LD_gam), and the ADI operators
 *     C_xy, C_xyz (eqs. C_def_ADI, C_def_ADI_3) and D_xy, D_xyz
 *     (eqs. D_def_ADI, D_def_ADI_3) as the literal compositions printed.
 *   - The order-2P update sum_{p<=P} sum_{m<=p} c_{p,m} C^m D^{p-m} u
 *     (Sec. 4, eq. Full_2D; 1D: eq. update_P with C = D) built with the
 *     re-use schedule of Table 2, and the three-level time step.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes):
 *   - local quadrature: quadratic through (x_{j-1}, x_j, x_{j+1});
 *   - at a Dirichlet end node the missing neighbour is replaced by the
 *     boundary curvature (inverse Lax-Wendroff, Sec. 3.2), 0 for homogeneous
 *     data;
 *   - homogeneous Dirichlet: every application of L^{-1} returns 0 at the end
 *     nodes, and end-node inputs are read as 0;
 *   - periodic lines: the free-space convolution of the periodic extension
 *     (geometric sum over the images);
 *   - embedded boundaries (Sec. 4.3): each maximal run of inside nodes on a
 *     grid line is one line object, closed by two boundary points at the
 *     curve crossings.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* Real type of the arithmetic: double by default.  The same source is also
   built with OR_LONG_DOUBLE (x87 80-bit) for long multi-step references, where
   the literal D = v - L^{-1} v loses digits to cancellation on smooth data. */
#ifdef OR_LONG_DOUBLE
typedef long double real;
#define R_EXP expl
#define R_EXPM1 expm1l
#define R_FABS fabsl
#else
typedef double real;
#define R_EXP exp
#define R_EXPM1 expm1
#define R_FABS fabs
#endif

#define OR_OK 0
/* number of applications of C or D since the last reset (Table 2 count) */
static long or_napply = 0;
void or_count_reset(void) { or_napply = 0; }
long or_count_get(void) { return or_napply; }
#define OR_EINVAL 1
#define OR_ENOMEM 4

/* ------------------------------------------------------------------------ */
/* Moments M_k(nu) = int_0^1 z^k e^{-nu z} dz, k = 0, 1, 2.                  */
/* Power series below nu = 2 (no cancellation), closed form above.           */
/* ------------------------------------------------------------------------ */
static void or_moments(real nu, real M[3])
{
    if (nu < 2.0) {
        for (int k = 0; k < 3; ++k) {
            /* sum_{n>=0} (-nu)^n / (n! (n+k+1)) */
            real term = 1.0, s = 0.0;
            for (int n = 0; n < 80; ++n) {
                real c = term / (real)(n + k + 1);
                s += c;
                if (R_FABS(c) < 1e-300 || (n > 4 && R_FABS(c) < 1e-19 * R_FABS(s))) break;
                term *= -nu / (real)(n + 1);
            }
            M[k] = s;
        }
    } else {
        real e = R_EXP(-nu);
        M[0] = (1.0 - e) / nu;
        M[1] = (1.0 - e * (1.0 + nu)) / (nu * nu);
        M[2] = (2.0 - e * (2.0 + 2.0 * nu + nu * nu)) / (nu * nu * nu);
    }
}

/* Quadratic q(t) = v0 + b t + c t^2 around node x_j (t = y - x_j). */
typedef struct { real v0, b, c; } or_quad;

/* Through (-hl, vm), (0, v0), (hr, vp). */
static or_quad or_quad3(real vm, real v0, real vp, real hl, real hr)
{
    or_quad q;
    q.v0 = v0;
    q.c = ((vp - v0) / hr - (v0 - vm) / hl) / (hl + hr);
    q.b = (vp - v0) / hr - q.c * hr;
    return q;
}

/* Left end node: through (0, v0), (hr, vp) with prescribed curvature q'' = kap. */
static or_quad or_quad_left_end(real v0, real vp, real hr, real kap)
{
    or_quad q;
    q.v0 = v0;
    q.c = 0.5 * kap;
    q.b = (vp - v0) / hr - q.c * hr;
    return q;
}

/* Right end node: through (-hl, vm), (0, v0) with prescribed curvature kap. */
static or_quad or_quad_right_end(real vm, real v0, real hl, real kap)
{
    or_quad q;
    q.v0 = v0;
    q.c = 0.5 * kap;
    q.b = (v0 - vm) / hl + q.c * hl;
    return q;
}

/* J^L_j = (alpha/2) int_{x_j - hl}^{x_j} e^{-alpha (x_j - y)} q(y - x_j) dy  */
static real or_JL(or_quad q, real alpha, real hl)
{
    real nu = alpha * hl, M[3];
    or_moments(nu, M);
    return 0.5 * nu * (q.v0 * M[0] - q.b * hl * M[1] + q.c * hl * hl * M[2]);
}

/* J^R_j = (alpha/2) int_{x_j}^{x_j + hr} e^{-alpha (y - x_j)} q(y - x_j) dy  */
static real or_JR(or_quad q, real alpha, real hr)
{
    real nu = alpha * hr, M[3];
    or_moments(nu, M);
    return 0.5 * nu * (q.v0 * M[0] + q.b * hr * M[1] + q.c * hr * hr * M[2]);
}

/*
 * O1: L^{-1} on one bounded line object with nodes x[0] < ... < x[m] (m >= 1)
 * and values v[0..m].  bnd = {ta, tb, ka, kb}: target values of L^{-1}v at the
 * two ends and the curvature of the data at the two ends (all 0 for
 * homogeneous Dirichlet data).  Writes w[0..m] = L^{-1} v.
 */
int or_linv_line(long m, const real *x, const real *v, real alpha,
                 const real *bnd, real *w)
{
    if (m < 1 || alpha <= 0.0) return OR_EINVAL;
    real ta = bnd ? bnd[0] : 0.0, tb = bnd ? bnd[1] : 0.0;
    real ka = bnd ? bnd[2] : 0.0, kb = bnd ? bnd[3] : 0.0;
    real *IL = (real *)malloc(sizeof(real) * (size_t)(m + 1));
    real *IR = (real *)malloc(sizeof(real) * (size_t)(m + 1));
    if (!IL || !IR) { free(IL); free(IR); return OR_ENOMEM; }

    /* local quadratics, one per node */
    /* left-to-right recurrence: I^L_0 = 0, I^L_j = e^{-alpha h_j} I^L_{j-1} + J^L_j */
    IL[0] = 0.0;
    for (long j = 1; j <= m; ++j) {
        real hl = x[j] - x[j - 1];
        or_quad q = (j < m) ? or_quad3(v[j - 1], v[j], v[j + 1], hl, x[j + 1] - x[j])
                            : or_quad_right_end(v[j - 1], v[j], hl, kb);
        IL[j] = R_EXP(-alpha * hl) * IL[j - 1] + or_JL(q, alpha, hl);
    }
    /* right-to-left recurrence: I^R_m = 0, I^R_j = e^{-alpha h_{j+1}} I^R_{j+1} + J^R_j */
    IR[m] = 0.0;
    for (long j = m - 1; j >= 0; --j) {
        real hr = x[j + 1] - x[j];
        or_quad q = (j > 0) ? or_quad3(v[j - 1], v[j], v[j + 1], x[j] - x[j - 1], hr)
                            : or_quad_left_end(v[j], v[j + 1], hr, ka);
        IR[j] = R_EXP(-alpha * hr) * IR[j + 1] + or_JR(q, alpha, hr);
    }
    /* boundary correction: w = I^L + I^R + A e^{-alpha(x-a)} + B e^{-alpha(b-x)}
       with w(a) = ta, w(b) = tb */
    real len = x[m] - x[0];
    real mu = R_EXP(-alpha * len);
    real one_m_mu2 = -R_EXPM1(-2.0 * alpha * len);
    real ra = ta - IR[0];            /* I^L_0 = 0 */
    real rb = tb - IL[m];            /* I^R_m = 0 */
    real A = (ra - mu * rb) / one_m_mu2;
    real B = (rb - mu * ra) / one_m_mu2;
    for (long j = 0; j <= m; ++j)
        w[j] = IL[j] + IR[j] + A * R_EXP(-alpha * (x[j] - x[0])) + B * R_EXP(-alpha * (x[m] - x[j]));
    free(IL);
    free(IR);
    return OR_OK;
}

/*
 * L^{-1} on a periodic line of n uniformly spaced nodes (spacing h, period
 * n h).  The convolution of the periodic extension: contributions from the
 * earlier images form a geometric series with ratio e^{-alpha n h}.
 */
int or_linv_periodic_line(long n, real h, const real *v, real alpha, real *w)
{
    if (n < 3 || alpha <= 0.0 || h <= 0.0) return OR_EINVAL;
    real *JL = (real *)malloc(sizeof(real) * (size_t)n);
    real *JR = (real *)malloc(sizeof(real) * (size_t)n);
    real *IL = (real *)malloc(sizeof(real) * (size_t)n);
    real *IR = (real *)malloc(sizeof(real) * (size_t)n);
    if (!JL || !JR || !IL || !IR) { free(JL); free(JR); free(IL); free(IR); return OR_ENOMEM; }
    for (long j = 0; j < n; ++j) {
        or_quad q = or_quad3(v[(j - 1 + n) % n], v[j], v[(j + 1) % n], h, h);
        JL[j] = or_JL(q, alpha, h);
        JR[j] = or_JR(q, alpha, h);
    }
    real d = R_EXP(-alpha * h);
    real one_m_mu = -R_EXPM1(-alpha * h * (real)n);
    /* I^L at the last node: all images to the left, summed geometrically */
    real s = 0.0, dk = 1.0;
    for (long k = 0; k < n; ++k) { s += dk * JL[n - 1 - k]; dk *= d; }
    real prev = s / one_m_mu;
    for (long j = 0; j < n; ++j) { IL[j] = d * prev + JL[j]; prev = IL[j]; }
    /* I^R at the first node: all images to the right */
    s = 0.0; dk = 1.0;
    for (long k = 0; k < n; ++k) { s += dk * JR[k]; dk *= d; }
    prev = s / one_m_mu;
    for (long j = n - 1; j >= 0; --j) { IR[j] = d * prev + JR[j]; prev = IR[j]; }
    for (long j = 0; j < n; ++j) w[j] = IL[j] + IR[j];
    free(JL); free(JR); free(IL); free(IR);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid problems                                                             */
/* ------------------------------------------------------------------------ */

/*
 * Embedded line objects (Sec. 4.3): for direction d, seg_idx holds triples
 * (line, first inside node, last inside node) and seg_th pairs (theta_lo,
 * theta_hi): the boundary points sit theta_lo*h before the first and
 * theta_hi*h after the last inside node, 0 < theta <= 1.  A 2D line index is
 * the row (d = 0) or the column (d = 1).
 */
typedef struct or_problem {
    int ndim;               /* 1, 2 or 3 */
    long n[3];              /* points per axis, x fastest */
    double h[3];            /* grid spacing per axis */
    int bc[3];              /* 0 Dirichlet (homogeneous), 1 periodic */
    double alpha;           /* beta / (c dt) */
    long nseg[3];           /* > 0: embedded line objects for that axis (2D) */
    const long *seg_idx[3];
    const double *seg_th[3];
    const unsigned char *mask; /* nullable, 1 = inside; outside forced to 0 */
} or_problem;

static long or_npts(const or_problem *pb)
{
    long N = 1;
    for (int d = 0; d < pb->ndim; ++d) N *= pb->n[d];
    return N;
}

static long or_stride(const or_problem *pb, int dir)
{
    long s = 1;
    for (int d = 0; d < dir; ++d) s *= pb->n[d];
    return s;
}

/* L_gamma^{-1} along axis dir for every line of the grid. */
int or_apply_linv(const or_problem *pb, int dir, const real *in, real *out)
{
    if (!pb || dir < 0 || dir >= pb->ndim) return OR_EINVAL;
    long N = or_npts(pb), nl = pb->n[dir], st = or_stride(pb, dir);
    long nlines = N / nl;
    int rc = OR_OK;
    if (pb->nseg[dir] > 0) {
        /* embedded: only line objects carry values; everything else is 0 */
        memset(out, 0, sizeof(real) * (size_t)N);
        if (pb->ndim != 2) return OR_EINVAL;
        long other = 1 - dir;
        long so = or_stride(pb, (int)other);
        long nseg = pb->nseg[dir];
#pragma omp parallel for schedule(dynamic, 16) reduction(| : rc)
        for (long s = 0; s < nseg; ++s) {
            long line = pb->seg_idx[dir][3 * s], i0 = pb->seg_idx[dir][3 * s + 1];
            long i1 = pb->seg_idx[dir][3 * s + 2];
            real tl = (real)pb->seg_th[dir][2 * s], tr = (real)pb->seg_th[dir][2 * s + 1];
            long m = (i1 - i0) + 2; /* nodes: boundary, i0..i1, boundary */
            real *x = (real *)malloc(sizeof(real) * (size_t)(m + 1));
            real *v = (real *)malloc(sizeof(real) * (size_t)(m + 1));
            real *w = (real *)malloc(sizeof(real) * (size_t)(m + 1));
            if (!x || !v || !w) { free(x); free(v); free(w); rc |= OR_ENOMEM; continue; }
            real hh = pb->h[dir];
            x[0] = ((real)i0 - tl) * hh; v[0] = 0.0;
            for (long i = i0; i <= i1; ++i) {
                x[i - i0 + 1] = (real)i * hh;
                v[i - i0 + 1] = in[line * so + i * st];
            }
            x[m] = ((real)i1 + tr) * hh; v[m] = 0.0;
            rc |= or_linv_line(m, x, v, pb->alpha, NULL, w);
            for (long i = i0; i <= i1; ++i) out[line * so + i * st] = w[i - i0 + 1];
            free(x); free(v); free(w);
        }
        return rc;
    }
#pragma omp parallel for schedule(static) reduction(| : rc)
    for (long L = 0; L < nlines; ++L) {
        /* base offset of line L: index with axis dir removed */
        long lo = L % st, hi = L / st;
        long base = hi * st * nl + lo;
        real *x = (real *)malloc(sizeof(real) * (size_t)nl);
        real *v = (real *)malloc(sizeof(real) * (size_t)nl);
        real *w = (real *)malloc(sizeof(real) * (size_t)nl);
        if (!x || !v || !w) { free(x); free(v); free(w); rc |= OR_ENOMEM; continue; }
        for (long i = 0; i < nl; ++i) {
            x[i] = (real)i * pb->h[dir];
            v[i] = in[base + i * st];
        }
        if (pb->bc[dir] == 1) {
            rc |= or_linv_periodic_line(nl, pb->h[dir], v, pb->alpha, w);
        } else {
            v[0] = 0.0; v[nl - 1] = 0.0;      /* homogeneous Dirichlet end nodes */
            rc |= or_linv_line(nl - 1, x, v, pb->alpha, NULL, w);
        }
        for (long i = 0; i < nl; ++i) out[base + i * st] = w[i];
        free(x); free(v); free(w);
    }
    return rc;
}

/* Zero every node that is not an unknown: Dirichlet end nodes, outside nodes. */
static void or_project(const or_problem *pb, real *f)
{
    long N = or_npts(pb);
    if (pb->mask) {
        for (long i = 0; i < N; ++i) if (!pb->mask[i]) f[i] = 0.0;
    }
    for (int d = 0; d < pb->ndim; ++d) {
        if (pb->bc[d] == 1 || pb->nseg[d] > 0) continue;
        long nl = pb->n[d], st = or_stride(pb, d);
        for (long i = 0; i < N; ++i) {
            long k = (i / st) % nl;
            if (k == 0 || k == nl - 1) f[i] = 0.0;
        }
    }
}

/* D_gamma v = v - L_gamma^{-1} v (eq. LD_gam) */
int or_apply_Dg(const or_problem *pb, int dir, const real *in, real *out)
{
    long N = or_npts(pb);
    real *t = (real *)malloc(sizeof(real) * (size_t)N);
    if (!t) return OR_ENOMEM;
    memcpy(t, in, sizeof(real) * (size_t)N);
    or_project(pb, t);
    int rc = or_apply_linv(pb, dir, t, out);
    for (long i = 0; i < N; ++i) out[i] = t[i] - out[i];
    free(t);
    return rc;
}

/*
 * C: 1D: C = D.  2D: C_xy = L_y^{-1} D_x + L_x^{-1} D_y  (eq. C_def_ADI).
 * 3D: C_xyz = L_y^{-1}L_z^{-1} D_x + L_z^{-1}L_x^{-1} D_y + L_x^{-1}L_y^{-1} D_z
 * (eq. C_def_ADI_3).  The rightmost operator of each product acts first.
 */
int or_apply_C(const or_problem *pb, const real *in, real *out)
{
    long N = or_npts(pb);
    int rc = OR_OK;
    ++or_napply;
    if (pb->ndim == 1) return or_apply_Dg(pb, 0, in, out);
    real *a = (real *)malloc(sizeof(real) * (size_t)N);
    real *b = (real *)malloc(sizeof(real) * (size_t)N);
    if (!a || !b) { free(a); free(b); return OR_ENOMEM; }
    if (pb->ndim == 2) {
        rc |= or_apply_Dg(pb, 0, in, a);     /* D_x v */
        rc |= or_apply_linv(pb, 1, a, out);  /* L_y^{-1} D_x v */
        rc |= or_apply_Dg(pb, 1, in, a);     /* D_y v */
        rc |= or_apply_linv(pb, 0, a, b);    /* L_x^{-1} D_y v */
        for (long i = 0; i < N; ++i) out[i] += b[i];
    } else {
        memset(out, 0, sizeof(real) * (size_t)N);
        /* term gamma: L_{g2}^{-1} L_{g1}^{-1} D_gamma with (gamma, g1, g2) =
           (x, z, y), (y, x, z), (z, y, x) following the printed products */
        const int g[3][3] = {{0, 2, 1}, {1, 0, 2}, {2, 1, 0}};
        for (int t = 0; t < 3; ++t) {
            rc |= or_apply_Dg(pb, g[t][0], in, a);
            rc |= or_apply_linv(pb, g[t][1], a, b);
            rc |= or_apply_linv(pb, g[t][2], b, a);
            for (long i = 0; i < N; ++i) out[i] += a[i];
        }
    }
    free(a); free(b);
    return rc;
}

/* D: 1D: D.  2D: D_xy = 1 - L_x^{-1} L_y^{-1} (eq. D_def_ADI).
   3D: D_xyz = 1 - L_x^{-1} L_y^{-1} L_z^{-1} (eq. D_def_ADI_3). */
int or_apply_D(const or_problem *pb, const real *in, real *out)
{
    long N = or_npts(pb);
    int rc = OR_OK;
    ++or_napply;
    if (pb->ndim == 1) return or_apply_Dg(pb, 0, in, out);
    real *t = (real *)malloc(sizeof(real) * (size_t)N);
    real *a = (real *)malloc(sizeof(real) * (size_t)N);
    if (!t || !a) { free(t); free(a); return OR_ENOMEM; }
    memcpy(t, in, sizeof(real) * (size_t)N);
    or_project(pb, t);
    if (pb->ndim == 2) {
        rc |= or_apply_linv(pb, 1, t, a);
        rc |= or_apply_linv(pb, 0, a, out);
    } else {
        rc |= or_apply_linv(pb, 2, t, a);
        rc |= or_apply_linv(pb, 1, a, out);
        rc |= or_apply_linv(pb, 0, out, a);
        memcpy(out, a, sizeof(real) * (size_t)N);
    }
    for (long i = 0; i < N; ++i) out[i] = t[i] - out[i];
    free(t); free(a);
    return rc;
}

/*
 * Right-hand side of the order-2P scheme (eq. Full_2D truncated at P; 1D
 * eq. update_P), assembled with the re-use schedule of Table 2:
 *   stage 1:  v_1 := C[u]
 *   stage p:  v_p := D[v_{p-1}], then v_k := C[v_k] for k = p-1, ..., 1.
 * After stage p, v_k holds the term with m = p + 1 - k factors of C and it is
 * weighted by c_{p,m} = (-1)^m 2 beta^{2m}/(2m)! binom(p-1, m-1).
 * coef[(p-1)*P + (m-1)] = c_{p,m}, supplied by the caller.
 */
int or_rhs(const or_problem *pb, int P, const real *coef, const real *u, real *rhs)
{
    if (P < 1) return OR_EINVAL;
    long N = or_npts(pb);
    int rc = OR_OK;
    real **v = (real **)calloc((size_t)P, sizeof(real *));
    real *t = (real *)malloc(sizeof(real) * (size_t)N);
    if (!v || !t) { free(v); free(t); return OR_ENOMEM; }
    for (int k = 0; k < P; ++k) {
        v[k] = (real *)malloc(sizeof(real) * (size_t)N);
        if (!v[k]) rc = OR_ENOMEM;
    }
    if (rc) goto done;
    rc |= or_apply_C(pb, u, v[0]);
    for (long i = 0; i < N; ++i) rhs[i] = coef[0] * v[0][i];
    for (int p = 2; p <= P; ++p) {
        rc |= or_apply_D(pb, v[p - 2], v[p - 1]);
        for (int k = p - 1; k >= 1; --k) {
            rc |= or_apply_C(pb, v[k - 1], t);
            memcpy(v[k - 1], t, sizeof(real) * (size_t)N);
        }
        for (int k = 1; k <= p; ++k) {
            real c = coef[(p - 1) * P + (p + 1 - k) - 1];
            for (long i = 0; i < N; ++i) rhs[i] += c * v[k - 1][i];
        }
    }
done:
    for (int k = 0; k < P; ++k) free(v[k]);
    free(v); free(t);
    return rc;
}

/* u^{n+1} = 2u^n - u^{n-1} + rhs(u^n)   (eq. Full_2D, left-hand side) */
int or_step(const or_problem *pb, int P, const real *coef, const real *u_prev,
            const real *u_curr, real *u_next)
{
    long N = or_npts(pb);
    real *r = (real *)malloc(sizeof(real) * (size_t)N);
    if (!r) return OR_ENOMEM;
    int rc = or_rhs(pb, P, coef, u_curr, r);
    for (long i = 0; i < N; ++i) u_next[i] = 2.0 * u_curr[i] - u_prev[i] + r[i];
    or_project(pb, u_next);
    free(r);
    return rc;
}

/* Starting value for zero initial velocity (Sec. 3.2): u^1 = u^0 + rhs(u^0)/2,
   the even Taylor terms up to order 2P with the spatial derivatives built from
   the same convolution operators. */
int or_start(const or_problem *pb, int P, const real *coef, const real *u0, real *u1)
{
    long N = or_npts(pb);
    real *r = (real *)malloc(sizeof(real) * (size_t)N);
    if (!r) return OR_ENOMEM;
    int rc = or_rhs(pb, P, coef, u0, r);
    for (long i = 0; i < N; ++i) u1[i] = u0[i] + 0.5 * r[i];
    or_project(pb, u1);
    free(r);
    return rc;
}

/* nsteps of the three-level scheme; on return u_prev/u_curr hold
   (u^{n+nsteps-1}, u^{n+nsteps}). */
int or_run(const or_problem *pb, int P, const real *coef, real *u_prev, real *u_curr,
           long nsteps)
{
    long N = or_npts(pb);
    real *nx = (real *)malloc(sizeof(real) * (size_t)N);
    if (!nx) return OR_ENOMEM;
    int rc = OR_OK;
    for (long s = 0; s < nsteps && rc == OR_OK; ++s) {
        rc = or_step(pb, P, coef, u_prev, u_curr, nx);
        memcpy(u_prev, u_curr, sizeof(real) * (size_t)N);
        memcpy(u_curr, nx, sizeof(real) * (size_t)N);
    }
    free(nx);
    return rc;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
