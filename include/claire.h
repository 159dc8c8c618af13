/*
 * claire.h -- C ABI of the MI355X (gfx950) Gauss--Newton--Krylov
 * diffeomorphic registration engine.
 *
 * Problem (Section 2.2, eq. e:varopt-claire): given a template image m0 and a
 * reference image m1 on the periodic domain [0, 2*pi)^3, find a stationary
 * velocity v minimising
 *     J(v) = 1/2 ||m(1) - m1||^2 + alpha/2 <L v, v>,
 * where m solves the transport equation d_t m + grad m . v = 0, m(0) = m0,
 * and L = (-Laplacian)^p is the H^p seminorm operator (p = 1 or 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid:    n1 x n2 x n3 nodes x_i = i * 2*pi / n_a (Section 2.5.1), each
 *          extent in [8, 1024]. n3 (the contiguous axis) must be a power of
 *          two; n1 and n2 may be any even product of 2, 3 and 5 (e.g. the
 *          256 x 300 x 256 grid of the paper's NIREP runs). Every grid runs
 *          the LDS-staged gathers (ragged bricks and a wrapped stencil on
 *          extents other than powers of two); power-of-two grids run fused
 *          FFT passes, others mixed-radix (4, 2, 3, 5) column transforms. The
 *          warm-start network (claire_net.h) takes power-of-two grids only.
 * Layout:  scalar fields are float32, C-contiguous [n1][n2][n3] (x3 fastest);
 *          vector fields are structure-of-arrays [3][n1][n2][n3].
 * Memory:  every float/double array argument is a DEVICE pointer unless its
 *          comment says "host". The caller owns all argument memory; the
 *          library never frees it and keeps no pointer to it after a call
 *          returns (inputs are copied into the context where needed).
 * Streams: all device work is enqueued on the hipStream_t passed (as void*)
 *          at context creation or to the stateless call; NULL means the
 *          default stream. Calls that return host scalars synchronise it.
 * Errors:  every int-returning call returns CLAIRE_OK (0) on success, a
 *          negative CLAIRE_E* code on failure (outputs are then undefined),
 *          or a positive CLAIRE_W* code when it finished with a warning.
 *          claire_last_error() gives a message for the calling thread.
 *          Nothing throws across the ABI and nothing exits the process.
 * Threads: a context may be used by one thread at a time.
 */
#ifndef CLAIRE_H
#define CLAIRE_H

#ifdef __cplusplus
extern "C" {
#endif

enum claire_status {
    CLAIRE_OK = 0,
    CLAIRE_EINVAL = -1,      /* bad argument: NULL pointer, size, nt < 1, alpha <= 0 */
    CLAIRE_ENOMEM = -2,      /* device allocation failed */
    CLAIRE_EDEVICE = -3,     /* HIP runtime error */
    CLAIRE_ENONFINITE = -4,  /* a NaN/Inf appeared in the objective or gradient */
    CLAIRE_ESTATE = -5,      /* call out of order (e.g. matvec before set_velocity) */
    CLAIRE_WNOTCONV = 1,     /* Gauss--Newton stopped at max_gn iterations */
    CLAIRE_WLINESEARCH = 2,  /* Armijo line search found no acceptable step */
    CLAIRE_WPCGMAX = 3,      /* PCG hit max_pcg before its forcing tolerance */
    CLAIRE_WDETBOUND = 4,    /* det F(1) <= 0 somewhere (map not diffeomorphic) */
    CLAIRE_WNEGCURV = 5      /* PCG met nonpositive curvature <s, Hs> <= 0 and stopped
                                early (truncated CG: the current step, or the
                                preconditioned steepest-descent direction on the
                                first matvec) */
};

/* Options of the Gauss--Newton--Krylov solve (Section 2.5.5, Algorithms 1-2,
 * Section 2.6). claire_opts_default() fills the paper's defaults. */
typedef struct claire_opts {
    int reg_order;              /* 1: H1 seminorm (symbol |k|^2); 2: H2 seminorm (|k|^4) */
    int precision;              /* 0: float32 fields and FFTs; 1: mixed -- the Hessian
                                   matvec reads grad m^j from a float16 copy (float32
                                   arithmetic, fields and FFTs); gradient, objective,
                                   PCG dots and det F unchanged */
    double gtol;                /* stop when ||g||_inf <= gtol ||g_0||_inf (default 5e-2) */
    double gabs;                /* ... or when ||g||_inf <= gabs (default 1e-6) */
    int forcing;                /* PCG forcing: 0 superlinear eta = min(1/2, sqrt||g||_inf),
                                   1 quadratic eta = min(1/2, ||g||_inf) */
    int max_gn;                 /* Gauss--Newton iterations per continuation level (50) */
    int max_pcg;                /* PCG matvecs per Newton step (100) */
    int fixed_pcg_iters;        /* > 0: run exactly this many PCG matvecs per step */
    int max_linesearch;         /* Armijo trials, step halved each time (16) */
    double armijo_c1;           /* sufficient-decrease constant (1e-4) */
    const double *alpha_levels; /* host array: continuation weights, solved in order,
                                   each level warm-started from the previous one
                                   (Section 2.6). NULL: the single alpha argument. */
    int n_levels;               /* length of alpha_levels */
    int compute_det;            /* 1: report det F(1) statistics at the end */
    int tol_from_zero;          /* 1: g_0 of the gtol test is the gradient at v = 0 instead
                                   of the gradient at the initial guess (the plain model
                                   forms it without transport solves: the state is m0 and
                                   the adjoint m1 - m0 at all times; with beta > 0 one
                                   extra state + adjoint solve per level), so a warm-started solve
                                   stops at the same gradient norm as one from v = 0; an
                                   initial guess whose objective is not finite or exceeds
                                   J(v = 0) is then replaced by v = 0 (first level) */
    int derivative;             /* first derivatives (grad m, div v, grad v):
                                   CLAIRE_DERIV_SPECTRAL (default) or CLAIRE_DERIV_FD8 */
    int precond;                /* PCG preconditioner (Section 2.5.6):
                                   CLAIRE_PRECOND_REG (default) or CLAIRE_PRECOND_TWOLEVEL */
    double beta;                /* > 0: near-incompressible model (appendix) with this
                                   weight of the divergence penalty (the paper's runs use
                                   1e-4); 0 (default): the plain model. Needs reg_order 1;
                                   not combined with CLAIRE_PRECOND_TWOLEVEL */
} claire_opts;

/* Preconditioners of the reduced Hessian (Section 2.5.6): the inverse of the
 * regularisation operator, (alpha L)^{-1} with the k = 0 mode passed through;
 * or the two-level zero-velocity preconditioner
 *   P = R^{-1/2} [Q_P F_L K0_c^{-1} Q_R F_L + F_H] R^{-1/2},
 * R = alpha L (k = 0 mode passed through), F_L / F_H spectral cut-off
 * filters below / at or above the Nyquist of the grid of half the extents,
 * Q_R / Q_P spectral restriction to / prolongation from that grid, and
 * K0_c = R_c^{-1/2} (alpha L + grad m(1) grad m(1)^T) R_c^{-1/2} on it
 * (k = 0 handled as the identity on the mean), the zero-velocity Hessian at
 * the current state m(t = 1), inverted by CG to a tenth of the outer PCG
 * forcing eta (Section 2.6 settings), at most 200 iterations. Needs every
 * extent >= 16. */
enum { CLAIRE_PRECOND_REG = 0, CLAIRE_PRECOND_TWOLEVEL = 1 };

/* First-derivative discretisations (Section 2.5.3): Fourier differentiation,
 * or the 8th-order central finite differences of the paper's GPU code,
 * (3, -32, 168, -672, 0, 672, -168, 32, -3) / (840 h), periodic. Higher-order
 * operators (alpha L and its inverse) are spectral in both. */
enum { CLAIRE_DERIV_SPECTRAL = 0, CLAIRE_DERIV_FD8 = 1 };

/* Statistics of a solve (row labels of the paper's result tables). */
typedef struct claire_stats {
    int gn_iters;               /* accepted Gauss--Newton steps, all levels */
    int matvecs;                /* Hessian matvecs */
    int pde_solves;             /* state + adjoint + incremental solves */
    int linesearch_trials;      /* objective evaluations in the line search */
    int pcg_max_hits;           /* Newton steps where PCG hit max_pcg */
    double J0;                  /* objective at the initial velocity, first level */
    double J;                   /* objective at exit */
    double rel_mismatch;        /* ||m(1) - m1||_2 / ||m0 - m1||_2 at exit */
    double rel_grad;            /* ||g||_inf / ||g_0||_inf at exit, last level (g_0 as
                                   chosen by tol_from_zero) */
    double det_min, det_mean, det_max; /* det F(1), when compute_det = 1 */
    long long det_nonpositive;  /* voxels with det F(1) <= 0 */
    double seconds;             /* wall time of the solve (host clock) */
    int inner_iters;            /* coarse CG iterations of the two-level preconditioner */
    int initial_rejected;       /* 1: with tol_from_zero, the initial guess gave an
                                   objective that was not finite or above J(v = 0), and
                                   the solve started from v = 0 instead */
} claire_stats;

typedef struct claire_ctx claire_ctx;

/* Fill *opts with the defaults listed above (reg_order 1). */
void claire_opts_default(claire_opts *opts);

/* Message of the last failed call on this thread ("" if none). */
const char *claire_last_error(void);

/* ---------------------------------------------------------------- context */

/* Create a context for an n1 x n2 x n3 grid (nx is a host array), nt time
 * steps (h_t = 1/nt, Section 2.5.1), regularisation weight alpha > 0 and
 * order reg_order (1 or 2). Allocates the context's device workspace on the
 * current HIP device (about (30 + 5 nt) float32 fields). */
int claire_ctx_create(claire_ctx **out, const int nx[3], int nt, double alpha,
                      int reg_order, void *stream);
int claire_ctx_destroy(claire_ctx *ctx);

/* Change alpha (continuation). Invalidates the cached gradient. */
int claire_ctx_set_alpha(claire_ctx *ctx, double alpha);

/* Copy the template m0 and the reference m1 ([n] each) into the context. */
int claire_ctx_set_images(claire_ctx *ctx, const float *m0, const float *m1);

/* Per-velocity setup at v ([3][n]), Algorithm 1 lines 3-6: RK2 backtrace of
 * the characteristics of +v and -v (Section 2.5.2), state solve
 * (eq. e:transport) keeping m^j and grad m^j for j = 0..nt (spectral,
 * Section 2.5.3), objective J (eq. e:varopt-claire), adjoint
 * (eq. e:adjoint) and reduced gradient (eq. e:rgrad). */
int claire_ctx_set_velocity(claire_ctx *ctx, const float *v);

/* Results of the last set_velocity: g ([3][n], device, may be NULL) and
 * J (host double, may be NULL). */
int claire_ctx_gradient(claire_ctx *ctx, float *g, double *J);

/* Objective J(v) alone (backtrace, state, J): one Armijo trial. J is a host
 * double. Leaves the gradient cache invalid. */
int claire_ctx_objective(claire_ctx *ctx, const float *v, double *J);

/* Gauss--Newton Hessian matvec at the velocity of the last set_velocity,
 * eq. (e:matvec) with the incremental state (e:incstate) and incremental
 * adjoint (e:incadj), lambda-terms dropped (Section 2.5.5):
 * Hvt = alpha L vt + int_0^1 lambda~ grad m dt. vt and Hvt are [3][n] and
 * must not overlap. */
int claire_ctx_hessian_matvec(claire_ctx *ctx, const float *vt, float *Hvt);

/* Select the Hessian matvec's storage precision for later set_velocity /
 * hessian_matvec calls: 0 float32, 1 mixed (the matvec reads grad m^j from a
 * float16 copy made at set_velocity; float32 arithmetic, fields and FFTs;
 * the gradient path stays float32). Invalidates the cached setup (call
 * set_velocity again). */
int claire_ctx_set_precision(claire_ctx *ctx, int precision);

/* Near-incompressible model (appendix, "(Near-)Incompressible
 * Diffeomorphisms"): div v = w with the penalty beta/2 <w, (-Delta^{-1} + id) w>
 * on the second control w, w eliminated. For later set_velocity /
 * hessian_matvec / objective calls (beta = 0: the plain model):
 *   g   = alpha L v + K b,  b = int_0^1 lambda grad m dt,
 *   K   = I - grad M Delta^{-1} div,  M = (alpha (beta (-Delta^{-1} + id))^{-1} + id)^{-1},
 *   H v~ = alpha L v~ + K int_0^1 lambda~ grad m dt,
 *   J   = 1/2 ||m(1) - m1||^2 + alpha/2 <L v, v> + beta/2 <div v, (-Delta^{-1} + id) div v>
 * (g = K grad J; J is the line-search merit function). The operators of the
 * model are spectral (odd derivatives with the Nyquist mode zeroed) whatever
 * the derivative option. beta >= 0; beta > 0 needs reg_order 1 (the paper's
 * H1 seminorm). Allocates two [3][n] float32 fields on first use.
 * Invalidates the cached setup. */
int claire_ctx_set_beta(claire_ctx *ctx, double beta);

/* Select the first-derivative discretisation (CLAIRE_DERIV_SPECTRAL or
 * CLAIRE_DERIV_FD8, Section 2.5.3) of grad m^j and div v in later
 * set_velocity calls and of grad v in detdefgrad. Invalidates the cached
 * setup. */
int claire_ctx_set_derivative(claire_ctx *ctx, int derivative);

/* Regularisation preconditioner z = (alpha L)^{-1} r, k = 0 mode passed
 * through (Sections 2.5.5-2.5.6). r, z: [3][n]; may alias. */
int claire_ctx_precond(claire_ctx *ctx, const float *r, float *z);

/* Two-level zero-velocity preconditioner z = P r (CLAIRE_PRECOND_TWOLEVEL
 * above) at the state of the last set_velocity: the coarse operator uses its
 * grad m(t = 1). The inner CG on K0_c runs from zero until its residual's
 * 2-norm falls to inner_rtol times the right-hand side's, or for max_inner
 * iterations (1..1000); *inner_iters (host, may be NULL) receives the count.
 * r, z: [3][n], must not overlap. Allocates the coarse workspace (about
 * 4 n floats) on first use; synchronises the stream once per
 * inner iteration. Needs every extent >= 16. */
int claire_ctx_precond_twolevel(claire_ctx *ctx, const float *r, float *z, double inner_rtol,
                                int max_inner, int *inner_iters);

/* Gauss--Newton--Krylov solve (Algorithm 1 with Algorithm 2 inside) from the
 * initial guess in v_inout ([3][n]); the solution overwrites it. opts and
 * stats (host) may be NULL. Returns a CLAIRE_W* code on early exit. */
int claire_ctx_solve(claire_ctx *ctx, const claire_opts *opts, float *v_inout,
                     claire_stats *stats);

/* Trace of the last claire_ctx_solve on this context (Algorithm 1 with
 * Algorithm 2), for comparing a solve step by step. iters (host, may be
 * NULL) receives up to max_iters records of 8 doubles, one per visited
 * iterate in order: continuation level, Gauss--Newton index k, J, ||g||_inf,
 * PCG matvecs of the step taken from it, accepted step length (0 if the line
 * search failed or no step was taken), line-search trials, and the number of
 * residual values the step's PCG recorded. pcg_res (host, may be NULL)
 * receives up to max_res values: each step's PCG residual history
 * ||r_l||_inf from r_0 = -g through every residual update (matvecs + 1
 * values, or fewer when PCG stopped on nonpositive curvature), concatenated
 * in step order. counts (host int[2]) receives the numbers of records and residual
 * values available. Copies min(count, capacity) of each. */
int claire_ctx_solve_trace(claire_ctx *ctx, double *iters, int max_iters, double *pcg_res,
                           int max_res, int counts[2]);

/* Deformation gradient check (appendix, eq. e:def-grad): transport F with
 * d_t F + (v.grad) F = (grad v) F, F(0) = I, for the velocity of the last
 * set_velocity, and evaluate det F(1) in float64. det_out ([n] float64,
 * device) may be NULL; stats (host double[4]) receives min, mean, max and
 * the count of non-positive values. Returns CLAIRE_WDETBOUND if any
 * determinant is <= 0. */
int claire_ctx_detdefgrad(claire_ctx *ctx, double *det_out, double stats[4]);

/* ----------------------------------------------- building blocks (checks) */

/* Spectral operators (Section 2.5.3): op selects
 *   CLAIRE_OP_GRAD     in [n]    -> out [3][n]  grad (Nyquist of odd derivatives zero)
 *   CLAIRE_OP_DIV      in [3][n] -> out [n]     divergence
 *   CLAIRE_OP_REG      in [3][n] -> out [3][n]  alpha L
 *   CLAIRE_OP_REG_INV  in [3][n] -> out [3][n]  (alpha L)^{-1}, k = 0 passed through
 *   CLAIRE_OP_FD8_GRAD in [n]    -> out [3][n]  grad by FD8 central differences
 *   CLAIRE_OP_FD8_DIV  in [3][n] -> out [n]     divergence by FD8
 *   CLAIRE_OP_NI_PROJECT in [3][n] -> out [3][n] K = I - grad M Delta^{-1} div
 *   CLAIRE_OP_NI_PENALTY in [3][n] -> out [3][n] -grad beta (-Delta^{-1} + id) div
 * (the last two: near-incompressible model at the context's alpha and beta,
 * see claire_ctx_set_beta; CLAIRE_EINVAL when beta = 0).
 * in and out must not overlap. */
enum { CLAIRE_OP_GRAD = 0, CLAIRE_OP_DIV = 1, CLAIRE_OP_REG = 2, CLAIRE_OP_REG_INV = 3,
       CLAIRE_OP_FD8_GRAD = 4, CLAIRE_OP_FD8_DIV = 5, CLAIRE_OP_NI_PROJECT = 6,
       CLAIRE_OP_NI_PENALTY = 7 };
int claire_ctx_spectral(claire_ctx *ctx, int op, const float *in, float *out);

/* Tricubic Lagrange interpolation (Section 2.5.4, p = 3):
 * out[k][x] = f[k](x + disp(x)) for nfield fields f ([nfield][n]) and a
 * displacement disp ([3][n], in voxel units). out must not overlap f. */
int claire_ctx_interpolate(claire_ctx *ctx, const float *f, int nfield,
                           const float *disp, float *out);

/* Copy a field cached by the last set_velocity into out:
 *   CLAIRE_FIELD_DISP_PLUS   [3][n] departure displacement (voxels) of +v
 *   CLAIRE_FIELD_DISP_MINUS  [3][n] departure displacement of -v
 *   CLAIRE_FIELD_STATE       [n]    m^j, j = index in 0..nt
 *   CLAIRE_FIELD_GRAD_STATE  [3][n] grad m^j
 *   CLAIRE_FIELD_ADJOINT     [n]    lambda^j
 *   CLAIRE_FIELD_DIVV        [n]    div v */
enum { CLAIRE_FIELD_DISP_PLUS = 0, CLAIRE_FIELD_DISP_MINUS = 1, CLAIRE_FIELD_STATE = 2,
       CLAIRE_FIELD_GRAD_STATE = 3, CLAIRE_FIELD_ADJOINT = 4, CLAIRE_FIELD_DIVV = 5 };
int claire_ctx_get_field(claire_ctx *ctx, int which, int index, float *out);

/* Average duration of one launch of a single hot-path kernel, timed with HIP
 * events over `reps` back-to-back launches on the context's stream, with the
 * arguments the Hessian matvec uses (needs a prior set_velocity). kernel:
 *   CLAIRE_KERNEL_INC_STATE_STEP  one incremental-state SL step (gather of
 *                                 w^j at y+, source -grad m^{j+1}.v~)
 *   CLAIRE_KERNEL_INC_STATE_STEP_MIXED  the same step of the mixed-precision
 *                                 matvec, grad m^{j+1} read from the float16
 *                                 copy (needs set_precision(1) before the
 *                                 set_velocity; CLAIRE_EINVAL otherwise)
 *   CLAIRE_KERNEL_ADJOINT_STEP    one (incremental) adjoint SL step
 *   CLAIRE_KERNEL_ASSEMBLE        h_t sum_j c_j lambda~^j grad m^j + alpha L v~
 *   CLAIRE_KERNEL_COPY            a plain copy of 3n floats (bandwidth and
 *                                 counter calibration)
 *   CLAIRE_KERNEL_BACKTRACE       the RK2 backtrace of +v and -v (recomputes
 *                                 the cached departure displacements)
 * *avg_ms (host) receives milliseconds per launch. The launches overwrite the
 * context's scratch buffers (incremental fields, adjoint history), not v, g
 * or the state. */
enum { CLAIRE_KERNEL_INC_STATE_STEP = 0, CLAIRE_KERNEL_ADJOINT_STEP = 1,
       CLAIRE_KERNEL_ASSEMBLE = 2, CLAIRE_KERNEL_COPY = 3, CLAIRE_KERNEL_BACKTRACE = 4,
       CLAIRE_KERNEL_INC_STATE_STEP_MIXED = 5 };
int claire_ctx_time_kernel(claire_ctx *ctx, int kernel, int reps, double *avg_ms);

/* --------------------------------------------- stateless convenience calls
 * Each builds a context, runs, and destroys it (setup cost paid per call). */

/* m1_out = m(1): transport of m0 by the stationary v (eq. e:transport),
 * nt semi-Lagrangian steps. */
int claire_transport(const float *m0, const float *v, const int nx[3], int nt,
                     float *m1_out, void *stream);

/* Reduced gradient g_out ([3][n]) and objective *J_out (host) at v
 * (eq. e:rgrad). Either output may be NULL. */
int claire_gradient(const float *m0, const float *m1, const float *v,
                    const int nx[3], double alpha, int nt, int reg_order,
                    float *g_out, double *J_out, void *stream);

/* Hvt_out = H(v) vt, the Gauss--Newton Hessian matvec (eq. e:matvec). */
int claire_hessian_matvec(const float *m0, const float *m1, const float *v,
                          const float *vt, const int nx[3], double alpha, int nt,
                          int reg_order, float *Hvt_out, void *stream);

/* Full solve (Algorithm 1); alpha is used when opts->alpha_levels is NULL.
 * opts and stats are host pointers and may be NULL. */
int claire_solve(const float *m0, const float *m1, const int nx[3], double alpha,
                 int nt, const claire_opts *opts, float *v_inout,
                 claire_stats *stats, void *stream);

/* ------------------------------------------- allocation-free transport
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as claire_transport (identical kernels, bit-identical output), with
 * every intermediate buffer in a fixed device array that the library holds
 * per GPU until the process ends (7 float32 fields of the largest grid plus
 * a brick table: about 57 MiB). The call makes no device allocation.
 * Limit: n1 n2 n3 <= claire_transport_noalloc_max_voxels() (2^21, e.g.
 * 128^3); larger grids return CLAIRE_EINVAL with nothing launched. m1_out
 * must not alias m0. All calls on one GPU share its array and keep the last
 * call's contents: calls that overlap in time on one GPU (several streams or
 * threads) race, and the caller must serialise them. Synchronises stream. */
int claire_transport_noalloc(const float *m0, const float *v, const int nx[3], int nt,
                             float *m1_out, void *stream);
long long claire_transport_noalloc_max_voxels(void);

#ifdef __cplusplus
}
#endif
#endif /* CLAIRE_H */
