/*
 * molt.h -- C-ABI of the MI355X MOL^T wave solver library (libmolt.so).
 *
 * The library advances the wave equation u_tt = c^2 (u_xx + u_yy + u_zz) with
 * the A-stable order-2P schemes of Causley & Christlieb built from recursive
 * applications of the convolution operator L^{-1} = (1 - alpha^{-2} d^2)^{-1}
 * (Sec. 2, eqs. L_def, L_Inverse), D = 1 - L^{-1} (eq. D_def_1d), the
 * univariate operators L_gamma, D_gamma (Sec. 4, eq. LD_gam) and the ADI
 * operators C and D (eqs. C_def_ADI, C_def_ADI_3, D_def_ADI, D_def_ADI_3):
 *
 *     u^{n+1} - 2 u^n + u^{n-1} = sum_{p=1}^{P} sum_{m=1}^{p}
 *         (-1)^m 2 beta^{2m}/(2m)! binom(p-1, m-1) C^m D^{p-m} [u^n]
 *
 * (eq. Full_2D; in 1D C = D and this is eq. update_P), with
 * alpha = beta / (c dt), 0 < beta <= beta_max(P) (Sec. 3.1, eq. Stab_cond).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Fields are dense arrays of n[0]*n[1]*n[2] values (1D: n[1] = n[2] = 1) in
 * C order with x fastest: element (i, j, k) at i + n[0]*(j + n[1]*k).  Field
 * pointers are DEVICE pointers owned by the caller (e.g. torch tensors); their
 * element type is the plan's dtype.  Every call is asynchronous on the given
 * stream (a hipStream_t passed as void*, NULL = the default stream) and
 * returns after enqueueing; nothing synchronises unless stated.  Errors are
 * reported as a mol_status; mol_last_error() returns a message for the last
 * failing call of the calling thread.  No call throws.
 *
 * Boundary data (Sec. 3.2): homogeneous.  On a Dirichlet axis the first and
 * last node of every line are boundary nodes: the library reads them as 0 and
 * writes 0 there.  With a mask (2D only) every node outside the domain is read
 * as 0 and written as 0, and the x and y convolutions act on line objects
 * (Sec. 4.3): the inside nodes between two crossings of the boundary curve
 * plus the two boundary points at the crossings.
 */
#ifndef MOLT_H
#define MOLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MOL_OK = 0,
    MOL_E_INVALID = 1,     /* bad argument (descriptor, pointer, size) */
    MOL_E_UNSUPPORTED = 2, /* valid but not provided (e.g. g != NULL, mask in 3D) */
    MOL_E_UNSTABLE = 3,    /* beta > beta_max(P) without MOL_ALLOW_UNSTABLE */
    MOL_E_NOMEM = 4,       /* device or host allocation failed */
    MOL_E_DEVICE = 5       /* a HIP call or kernel launch failed */
} mol_status;

/* Boundary type of an axis.  MOL_BC_NEUMANN (1D plans only): the end nodes
 * are unknowns, the slope u_x is prescribed there (zero with mol_step, data
 * with mol_step_bdata); Sec. 3.2, boundary data of the recursive
 * convolutions. */
typedef enum { MOL_BC_DIRICHLET = 0, MOL_BC_PERIODIC = 1, MOL_BC_NEUMANN = 2 } mol_bc;
typedef enum { MOL_F64 = 0, MOL_F32 = 1 } mol_dtype;

enum {
    MOL_ALLOW_UNSTABLE = 1,   /* accept beta > beta_max(P) */
    MOL_INCREMENT_FORM = 2,   /* mol_solve carries du = u^n - u^{n-1} instead of u^{n-1} */
    MOL_NO_GRAPH = 4,         /* mol_solve launches kernels directly instead of a hipGraph */
    MOL_SPLIT_Y = 8,          /* mol_solve (2D, P = 2) sweeps y twice in two launches instead of
                                 one chained launch (same operator; for comparisons) */
    MOL_UNIFORM_CONFIG = 16,  /* launch configurations that do not depend on the grid size where
                                 the size allows (x: one line capacity up to 2048 nodes; y/z:
                                 the tile kernel), so that plans of different sizes share
                                 kernels; no tuning-cache entries (used by the batched server) */
    MOL_SYMMETRIC_D = 32      /* masked plans: D = 1 - (L_x^-1 L_y^-1 + L_y^-1 L_x^-1) / 2, the
                                 mean over both orders of the directional inverses, in place of
                                 1 - L_x^-1 L_y^-1 (averaging the sweep orders against the
                                 anisotropy of ADI, Sec. 4, operation count); no extra sweep.
                                 A mask symmetric under x <-> y then gives solutions that are.
                                 Box plans: no effect (the directional operators commute). */
};

/* Problem descriptor (Sec. 2: domain, c, dt, beta; Sec. 3: order P;
 * Sec. 3.2: boundary type; Sec. 4.3: embedded boundary). */
typedef struct mol_desc {
    int ndim;               /* 1, 2 or 3 */
    int64_t n[3];           /* nodes per axis (x, y, z); unused axes = 1 */
    double h[3];            /* node spacing per axis */
    int bc[3];              /* mol_bc per axis */
    const uint8_t *mask;    /* HOST pointer or NULL (2D only): n[1] x n[0] bytes,
                               1 = inside; the outer ring of nodes must be 0 */
    const double *cross;    /* HOST pointer or NULL: 4 x n[1] x n[0] doubles; at an
                               inside node next to an outside node, the distance to
                               the boundary crossing in units of h toward -x, +x,
                               -y, +y, in (0, 1]; NULL puts the crossing on the
                               outside node (distance 1) */
    int P;                  /* order 2P, 1 <= P <= 5 (Table 1) */
    double c;               /* wave speed > 0 */
    double dt;              /* time step > 0 */
    double beta;            /* <= 0 selects beta_max(P) (Table 1) */
    int dtype;              /* mol_dtype of every field */
    int flags;              /* MOL_ALLOW_UNSTABLE | MOL_INCREMENT_FORM | MOL_NO_GRAPH */
} mol_desc;

typedef struct mol_plan_ mol_plan;

/* Scalars derived by the plan (for reporting). */
typedef struct mol_plan_info {
    double beta;            /* beta used */
    double beta_max;        /* beta_max(P) */
    double alpha;           /* beta / (c dt) (eq. L_def) */
    double nu[3];           /* alpha * h per axis */
    int64_t points;         /* nodes per field */
    int64_t unknowns;       /* nodes that are not boundary / outside nodes */
    int64_t segments[2];    /* line objects per axis (masked plans), else 0 */
    int kernels_per_step;   /* kernel launches in one mol_step */
    double bytes_per_step;  /* algorithmic HBM bytes of one step (fields read + written) */
    size_t workspace_bytes; /* device workspace held by the plan */
    int kernels_per_source_step;   /* launches of one mol_step_source, 0 if unsupported */
    double bytes_per_source_step;  /* its algorithmic HBM bytes */
} mol_plan_info;

/* beta_max(P): first positive root of -sum_{p<=P} A_p(beta) = 4
 * (Theorem of Sec. 3.1, eq. Stab_cond); returns -1 for P outside 1..8. */
double mol_beta_max(int P);

/* Size limits: fewer than 2^31 nodes per field; any length along y and z; an
 * x line of up to 16384 nodes is one workgroup (8192 in FP64 for launches that
 * sweep two combinations); longer x lines of homogeneous Dirichlet type are
 * swept in chunks of 4096 nodes, exact across them (a carry table and scan
 * between two passes; L^{-1} applied as v - D v there), while periodic,
 * Neumann and K-form (small nu) x lines must fit one workgroup, and the line
 * objects of a mask at most 8192 nodes; beyond them MOL_E_UNSUPPORTED.
 * Validates the descriptor, derives alpha, the quadrature weights and the
 * stage coefficients in FP64, builds the kernel schedule (and for a mask the
 * line-object tables), and allocates the device workspace on the current
 * device.  *plan is set only on MOL_OK.  The plan is bound to that device. */
mol_status mol_plan_create(const mol_desc *desc, mol_plan **plan);

/* Frees the plan and its device memory (synchronises the device first). */
mol_status mol_plan_destroy(mol_plan *plan);

mol_status mol_plan_get_info(const mol_plan *plan, mol_plan_info *info);

/* Device bytes mol_plan_create would allocate for this descriptor (workspace
 * plus tables), not counting the caller's fields; 0 if the descriptor is
 * invalid.  For admission by footprint. */
size_t mol_workspace_bytes(const mol_desc *desc);

/* Starting value u1 = u(dt) (Sec. 3.2) from u0 = u(0) and g = u_t(0): the
 * Taylor series of u(dt) with every time derivative turned into powers of the
 * laplacian.  The even terms give u0 + rhs(u0)/2 (the step's weights); the odd
 * terms give dt sum_m beta^{2m} / (2m+1)! (laplacian / alpha^2)^m g, taken with
 * the same schedule and weights b_{p,m} = (-1)^m beta^{2m} / (2m+1)!
 * binom(p-1, m-1) for p <= P:  u1 = u0 + rhs(u0)/2 + dt (g + rhs_b(g)).
 * g == NULL: zero initial velocity.  g is a device field like u0 (read only);
 * u1 is 0 on Dirichlet and outside nodes.  u0 and u1 must not overlap, nor g
 * and u1. */
mol_status mol_start(mol_plan *plan, const void *u0, const void *g, void *u1, void *stream);

/* One step of the three-level scheme: u_next = 2 u_curr - u_prev + rhs(u_curr).
 * u_next may alias u_prev (it is written after u_prev is read); it must not
 * overlap u_curr. */
mol_status mol_step(mol_plan *plan, const void *u_prev, const void *u_curr, void *u_next,
                    void *stream);

/* One step with a source term (Sec. 4, inclusion of source terms) for
 * u_tt / c^2 = laplacian(u) + S, with (c dt)^2 = (beta / alpha)^2:
 *   P = 1: u_next = 2 u_curr - u_prev + rhs(u_curr) + (c dt)^2 s_curr
 *   P = 2: u_next = 2 u_curr - u_prev + rhs(u_curr)
 *                   + (c dt)^2 / 12 (s_next + 10 s_curr + s_prev)
 *                   - beta^2 (c dt)^2 / 12 C[s_curr]
 * s_prev, s_curr, s_next: device fields of S at t_{n-1}, t_n, t_{n+1}, the
 * plan's dtype and shape (read only; S in the units of laplacian(u)).  The
 * C[S^n] coefficient is the dt^4 c^4 laplacian(S) / 12 term of the Taylor
 * expansion with the laplacian replaced by -alpha^2 C; the coefficient as
 * printed is not dimensionally consistent and gives a second-order scheme.
 * Dirichlet boundary nodes of u_next are 0 whatever S is there.  Full order
 * needs S = 0 on Dirichlet boundaries: the end cells of every sweep take the
 * curvature of homogeneous data (u_xx = 0), while a source makes it -S there
 * (a source nonzero on the boundary measured order 2.4-2.9 at P = 2 in 1D).
 * A source that depends on u (S^{n+1} through u^{n+1}) needs the caller's
 * iteration.
 * s_prev and s_next are not read for P = 1 (may be NULL).  Box plans with
 * P = 1 or 2 only, else MOL_E_UNSUPPORTED.  Aliasing as mol_step; u_next must
 * not overlap a source field.  Asynchronous on stream. */
mol_status mol_step_source(mol_plan *plan, const void *u_prev, const void *u_curr, void *u_next,
                           const void *s_prev, const void *s_curr, const void *s_next,
                           void *stream);

/* One step of the 1D scheme (eq. update_P) with time-dependent boundary data
 * (Sec. 3.2, boundary conditions for the recursive convolutions).  Each
 * application of D within D^p needs at each end the shape of its input in the
 * end cell and what L^{-1} of its input must satisfy there; both are space
 * derivatives of u at the end, which the wave equation gives from the data by
 * inverse Lax-Wendroff, (d_xx)^j u = (d_tt / c^2)^j u, truncated at j <= P.
 *   Dirichlet plans (u(a, t) = u_L(t), u(b, t) = u_R(t)): the curvature of the
 *   input in the end cell and the value of L^{-1} at the end (even
 *   derivatives).  The end nodes of u_curr must hold u_L(t_n) and u_R(t_n);
 *   those of u_next receive u_L(t_{n+1}) and u_R(t_{n+1}).
 *   Neumann plans (u_x(a, t) = g_L(t), u_x(b, t) = g_R(t)): the slope of the
 *   input at the end (the end cell's quadratic passes through the end node
 *   and its neighbour with that slope) and the slope of L^{-1} at the end (odd
 *   derivatives); every node is updated.
 * bdata: HOST array of 2 (P + 2) doubles: d_t^{2j} of the data at a (u_L or
 * g_L) at t_n for j = 0..P, then u_L(t_{n+1}) (ignored for Neumann); the same
 * for b.  With zero data this is mol_step.  1D Dirichlet or Neumann plans,
 * else MOL_E_UNSUPPORTED.  Aliasing as mol_step.  Asynchronous on stream
 * (bdata is read before the call returns). */
mol_status mol_step_bdata(mol_plan *plan, const void *u_prev, const void *u_curr, void *u_next,
                          const double *bdata, void *stream);

/* nsteps >= 0 steps of the three-level scheme (eq. Full_2D; in 1D eq.
 * update_P) in place: on entry (u_prev_io, u_curr_io) = (u^{n-1}, u^n), on
 * return (u^{n+nsteps-1}, u^{n+nsteps}).  The two buffers must differ and
 * must not overlap.  On a non-NULL stream, unless MOL_NO_GRAPH is set, the
 * steps run as replays of two hipGraphs captured for this pair of buffers on
 * first use: a unit of 8 steps and the even remainder (nsteps mod 8, rounded
 * down to even; an odd last step is launched directly and the two buffers'
 * contents swapped with device copies).  On the NULL stream every launch is
 * direct.  Calls with another pair of buffers recapture.  2D box plans with
 * P >= 2 first launch one x sweep of u_curr (its D_x, kept in the workspace
 * for the first step).  Asynchronous on stream. */
mol_status mol_solve(mol_plan *plan, void *u_prev_io, void *u_curr_io, int64_t nsteps,
                     void *stream);

/* Captures and instantiates the hipGraphs that mol_solve(plan, u_prev_io,
 * u_curr_io, nsteps, stream) replays, without running a step (for callers
 * that keep graph instantiation out of a timed or latency-bound region).
 * No-op on the NULL stream or with MOL_NO_GRAPH. */
mol_status mol_solve_prepare(mol_plan *plan, void *u_prev_io, void *u_curr_io, int64_t nsteps,
                             void *stream);

/* nsteps steps in place like mol_solve with a separable source
 * S(x, t) = f(t) G(x), a point source switched on in time for instance (Sec. 4,
 * inclusion of source terms; the step of mol_step_source with S^m = f_m G):
 * the source part of a step is a_n G + b_n C[G] with
 *   P = 1: a_n = (c dt)^2 f_n,                                  b_n = 0
 *   P = 2: a_n = (c dt)^2 / 12 (f_{n+1} + 10 f_n + f_{n-1}),    b_n = -beta^2 (c dt)^2 / 12 f_n.
 * On entry (u_prev_io, u_curr_io) = (u^{n-1}, u^n), on return
 * (u^{n+nsteps-1}, u^{n+nsteps}).  G: device field (read only).  CG: device
 * field C[G], e.g. from mol_apply(plan, MOL_OP_C, G, CG) (read only; not read
 * for P = 1, may be NULL).  f: host array of nsteps + 2 values f(t_{n-1}),
 * f(t_n), ..., f(t_{n+nsteps}), read before the call returns.  In 2D with
 * P = 2 the steps are mol_solve's fused ones with G and C[G] read by their last
 * launch; launched directly (no graph).  Box plans with P = 1 or 2 in the
 * three-level form, else MOL_E_UNSUPPORTED.  Asynchronous on stream. */
mol_status mol_solve_source(mol_plan *plan, void *u_prev_io, void *u_curr_io, int64_t nsteps,
                            const void *G, const void *CG, const double *f, void *stream);

/* One step (eq. Full_2D; 1D eq. update_P) for each of count independent
 * plans, with the results of mol_step(plans[i], u_prev[i], u_curr[i],
 * u_next[i], stream) for every i, bit for bit.  The launches at the same
 * position of the plans' steps that use the same kernel instantiation run as
 * one launch over a table of their argument sets (plans created with
 * MOL_UNIFORM_CONFIG share instantiations across sizes); launches that cannot
 * share one (masked plans, exact two-pass sweeps) run by themselves at their
 * position.  Arrays of count HOST pointers to device fields; plans must be
 * distinct; u_next[i] must not be u_curr[i].  The argument tables are copied
 * through pinned staging into a stream-ordered allocation freed on the stream
 * after the launches.  Asynchronous on stream.  (Serving many requests
 * concurrently is the request server below.) */
mol_status mol_step_batch(mol_plan *const *plans, const void *const *u_prev,
                          const void *const *u_curr, void *const *u_next, int count,
                          void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step
 * like mol_step(plan, u_prev, u_curr, u_next, stream) for the plan desc
 * describes, with no plan and no device allocation.  The step's workspace
 * fields and carry table live in one device array of the library, of
 * mol_step_static_max_bytes() bytes (64 MiB; each GPU holds its own copy
 * until the process ends); a step that needs more returns MOL_E_INVALID and
 * says how much, a mask returns MOL_E_UNSUPPORTED.  Calls on one GPU share the
 * array: calls that overlap in time on one GPU (several streams or host
 * threads) race and must be serialised by the caller.  The schedule and launch
 * configurations are those of mol_plan_create's plan of desc, so the result
 * is bitwise that of mol_step.  Host work per call: building that schedule. */
size_t mol_step_static_max_bytes(void);
mol_status mol_step_static(const mol_desc *desc, const void *u_prev, const void *u_curr,
                           void *u_next, void *stream);

/* ---- Request server (serving many independent solves on one GPU) ----
 *
 * Continuous batching of independent requests of differing n, P, CFL and
 * dtype (any descriptor mol_plan_create accepts).  A request is admitted in
 * arrival order when its device footprint -- mol_workspace_bytes(desc) plus
 * two fields -- fits the server's byte budget next to the requests already
 * running; it then owns a plan and two resident fields, runs mol_start and
 * nsteps - 1 steps (mol_solve, graph-captured) on one stream of the server's
 * pool, and finishes with an event.  Requests on different streams run
 * concurrently.  Allocations are stream-ordered, from a memory pool the
 * server owns (one block per request's plan workspace, plus its two fields);
 * memory a finished request frees stays reserved in that pool, and is given
 * back to the device when the server is destroyed.  Admitting or retiring a
 * request never synchronises the device.  One host thread at a time per
 * server (calls are serialised by a mutex).
 *
 * Batched mode (mol_server_create_ex with MOL_SERVER_BATCHED): admitted
 * requests advance together in rounds of one time step each on one stream.
 * The k-th launch of every request's step whose kernel instantiation is the
 * same (same kernel, configuration, dtype and boundary type; sizes, orders and
 * coefficients may differ) runs as one batched launch over a table of the
 * requests' argument sets, so many small solves fill the GPU together.
 * Launches of masked requests run one by one inside the round.  Rounds are
 * issued by submit and poll, at most three ahead of the GPU.  The server's
 * plans take MOL_UNIFORM_CONFIG, so requests of different sizes share
 * kernels; each request's result is bitwise the same as the same descriptor
 * (with that flag) solved alone.
 */
typedef struct mol_server_ mol_server;

typedef struct mol_server_info {
    int64_t queued;         /* submitted, not admitted yet */
    int64_t running;        /* admitted, not finished */
    int64_t finished;       /* finished, result not taken yet */
    int64_t completed;      /* finished since creation */
    size_t bytes_in_use;    /* footprint of admitted requests and untaken results */
    size_t bytes_peak;
    size_t budget;
    double admit_seconds;   /* host time spent admitting requests (plan, copies, enqueue) */
    double admit_max_seconds;
    double round_seconds;   /* batched mode: host time spent issuing rounds */
    int64_t rounds;         /* batched mode: rounds issued */
    int64_t launches;       /* batched mode: kernel launches issued by rounds */
    int64_t sweeps;         /* batched mode: request sweeps those launches carried */
} mol_server_info;

enum { MOL_SERVER_BATCHED = 1 };

/* hbm_budget_bytes > 0: device bytes the server may hold; nstreams in 1..64
 * (default-priority, non-blocking streams on the current device). */
mol_status mol_server_create(size_t hbm_budget_bytes, int nstreams, mol_server **server);
/* As mol_server_create; flags = MOL_SERVER_BATCHED selects the batched mode
 * (rounds on the first stream of the pool), 0 the stream pool. */
mol_status mol_server_create_ex(size_t hbm_budget_bytes, int nstreams, int flags, mol_server **server);
/* Waits for running requests and frees everything, results not taken included. */
mol_status mol_server_destroy(mol_server *server);
/* Queues a request: the solution u^nsteps (nsteps >= 1) from u^0 = u0 with
 * zero initial velocity (Sec. 2, start of the three-level scheme).  u0 is a
 * host (u0_on_device = 0) or device pointer to one field of the descriptor's
 * shape and dtype (the server cannot check its size: a shorter buffer is read
 * beyond its end); it must stay valid and unchanged until the request is
 * reported finished.  A device u0 is read on a server stream with no ordering
 * against the caller's streams: its contents must be complete when submit is
 * called (synchronise the stream that wrote it first).  The descriptor (and its mask / cross arrays) is copied.
 * MOL_E_INVALID for a descriptor mol_plan_create would reject, MOL_E_NOMEM if
 * the footprint exceeds the budget.  *id receives the request id (> 0). */
mol_status mol_server_submit(mol_server *server, const mol_desc *desc, const void *u0,
                             int u0_on_device, int64_t nsteps, int64_t *id);
/* Retires finished requests, admits queued ones, and writes up to max ids of
 * requests that finished since the last poll to done_ids (*ndone of them).
 * Never blocks. */
mol_status mol_server_poll(mol_server *server, int64_t *done_ids, int max, int *ndone);
/* Copies the result of a finished request to dst (host or device pointer as
 * dst_on_device says, room for one field of the request's shape and dtype)
 * and releases the request; returns after the copy has completed.
 * MOL_E_DEVICE if the request failed (mol_server_last_error() tells why). */
mol_status mol_server_result(mol_server *server, int64_t id, void *dst, int dst_on_device);
mol_status mol_server_stats(mol_server *server, mol_server_info *info);
const char *mol_server_last_error(void);

/* Single operators, for testing and composition.  in and out must not overlap. */
typedef enum {
    MOL_OP_LINV_X = 0, MOL_OP_LINV_Y = 1, MOL_OP_LINV_Z = 2, /* L_gamma^{-1} (eq. LD_gam) */
    MOL_OP_D_X = 3, MOL_OP_D_Y = 4, MOL_OP_D_Z = 5,          /* D_gamma = 1 - L_gamma^{-1} */
    MOL_OP_C = 6,           /* C (1D: D; 2D: eq. C_def_ADI; 3D: eq. C_def_ADI_3) */
    MOL_OP_D = 7,           /* D (1D: D; 2D: eq. D_def_ADI; 3D: eq. D_def_ADI_3) */
    MOL_OP_RHS = 8          /* sum_{p,m} c_{p,m} C^m D^{p-m} (eq. Full_2D) */
} mol_op;
mol_status mol_apply(mol_plan *plan, int op, const void *in, void *out, void *stream);

/* Per-kernel timing of one step, for measurement tools.  Runs the kernels of
 * mol_step(plan, u_prev, u_curr, u_next) reps times on the stream with a pair
 * of hipEvents around every launch, synchronises, and writes for kernel i
 * (i < min(count, max)) its mean duration in ms (ms[i]), its algorithmic
 * bytes per launch (bytes[i]: every loaded and every written field streamed
 * once), its sweep direction (dir[i], 0 = x) and its swept combinations
 * (nsweep[i]).  Returns the kernel count of one step in *count.  Any array may
 * be NULL.  Same aliasing rules as mol_step. */
mol_status mol_profile_step(mol_plan *plan, const void *u_prev, const void *u_curr, void *u_next,
                            int reps, void *stream, int max, double *ms, double *bytes,
                            int *dir, int *nsweep, int *count);

/* Launch configurations, for the autotuner.  Kernel indices refer to the step
 * program mol_solve replays (as in mol_profile_step).  mol_plan_kernel_configs
 * writes up to max valid configuration ids of kernel `kernel` into ids, their
 * number into *count and the id in use into *current (pointers may be NULL).
 * mol_plan_set_kernel_config selects one (MOL_E_INVALID if not valid for that
 * kernel); it also applies to every other kernel of the plan with the same
 * direction, field count and sweep shape.  At creation a plan takes its
 * configurations from the tuning cache file named by the environment variable
 * MOLT_TUNE_CACHE, else tune_cache.txt beside the library, when it holds an
 * entry for the problem; otherwise built-in defaults. */
mol_status mol_plan_kernel_configs(const mol_plan *plan, int kernel, int *ids, int max, int *count,
                                   int *current);
mol_status mol_plan_set_kernel_config(mol_plan *plan, int kernel, int config);
/* The cache key of a plan's problem and of one of its kernels (for the tuner):
 * writes a NUL-terminated string of at most len bytes. */
mol_status mol_plan_tune_key(const mol_plan *plan, int kernel, char *buf, int len);

/* Message for the last failing call on this thread ("" if none). */
const char *mol_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOLT_H */
