/*
 * qcpd -- derivative and adjoint of a quadratic cone program's solution map on one
 * MI355X (gfx950), in FP64.
 *
 * Problem (Sec. 2.1, eq. conic-pair):
 *     minimize 1/2 x'Px + q'x  subject to  Ax + s = b, s in K
 * with dual  Px + A'y = -q, y in K*.  The caller supplies the data theta = (P, A, q, b),
 * the cone K and a primal-dual solution (x, y, s) from any solver (Sec. 2.2: the derivative
 * needs the solution at theta, which a numerical solver provides).
 *
 * qcpd_jvp evaluates DS(theta)[dtheta] = (dx, dy, ds)          (Sec. 3.1)
 * qcpd_vjp evaluates DS(theta)'[(gx, gy, gs)] = (dP, dA, dq, db) (Sec. 3.2)
 * Both form z = (x, y - s, 1), and solve a least-squares problem with the derivative of the
 * normalised residual map, F = D_z N = D_u Q(Pi z) DPi(z) - DPi(z) + I (Sec. 2.4), by
 * matrix-free LSQR with a diagonal (Jacobi) right preconditioner. dP and dA live on the
 * stored patterns of P and A (Sec. 3.2, last paragraph).
 *
 * Conventions
 *   - All floating-point data is FP64; CSR index arrays are int32.
 *   - P is given in full symmetric CSR (both triangles, pattern and values symmetric).
 *     A perturbation dP must be symmetric on that pattern; the returned dP is symmetric.
 *     Inner products over dP, dA are sums over stored entries.
 *   - Cone rows are ordered: zero, nonnegative, second-order cones (t first), PSD cones
 *     (svec: lower triangle column-major, off-diagonals times sqrt 2), exponential cones,
 *     power cones, dual power cones ((x, y, z) each, per Appendix A). The batched form takes
 *     no power cones.
 *   - Pointers marked [device] are device (HBM) pointers on the current HIP device; [host]
 *     are host pointers. The caller owns every buffer it passes. qcpd_create copies or
 *     derives everything it needs, so its inputs may be freed once it returns.
 *   - Work is ordered on the stream given at create time (a hipStream_t passed as void*;
 *     NULL is the default stream). qcpd_jvp/qcpd_vjp return after the result is complete.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - No function throws; every one returns a status. Negative = error and no output
 *     written; positive = warning with outputs written.
 */
#ifndef QCPD_H
#define QCPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qcpd_status;

#define QCPD_OK                     0
#define QCPD_WARN_NOT_CONVERGED     1   /* the explicitly recomputed relative residual is
                                           above tol (LSQR hit max_iter, or its resumes ran
                                           out); outputs are written at the last iterate     */
#define QCPD_WARN_NONDIFF           2   /* a cone block lies within 1e-10 (relative) of a
                                           point where its projection is not differentiable;
                                           the listed tie-break rules were applied           */
#define QCPD_ERR_INVALID_ARG       -1   /* null pointer, negative size, bad option           */
#define QCPD_ERR_DIM               -2   /* inconsistent dimensions                           */
#define QCPD_ERR_CONE              -3   /* cone rows do not add up to m, or a bad cone size  */
#define QCPD_ERR_PATTERN           -4   /* P is not symmetric (pattern or values)            */
#define QCPD_ERR_NAN               -5   /* NaN or Inf in an input                            */
#define QCPD_ERR_HIP               -6   /* a HIP runtime call failed                         */
#define QCPD_ERR_OOM               -7   /* device allocation failed                          */

/* preconditioners for LSQR (right preconditioning; the residual is unchanged) */
#define QCPD_PRECOND_NONE    0
#define QCPD_PRECOND_JACOBI  1   /* 1 / column norms of the operator with each cone block's
                                    Jacobian replaced by its diagonal                        */
#define QCPD_PRECOND_CUSTOM  2   /* caller-supplied two-sided scaling (qcpd_set_precond), e.g.
                                    the output of a learned model                           */
#define QCPD_PRECOND_EQUIL   3   /* two-sided: rows and columns of F balanced in 2-norm by
                                    repeated square-root scaling sweeps (each cone block's
                                    Jacobian replaced by its diagonal); the systems are
                                    consistent, so a row scaling leaves the solution unchanged.
                                    The stop is decided on the unscaled residual.           */
#define QCPD_PRECOND_LEARNED 4   /* two-sided scaling predicted from per-index features of F
                                    by the model installed with qcpd_set_learned. When LSQR
                                    does not reach tol with it, the call is repeated with
                                    JACOBI, which also serves as the reference (info flags
                                    bit 2).                                                  */

/* Compressed sparse rows. [device] arrays: rowptr (nrows+1), colind (nnz), val (nnz). */
typedef struct {
    int32_t nrows, ncols, nnz;
    const int32_t *rowptr;
    const int32_t *colind;
    const double  *val;
} qcpd_csr;

/* Cone K as a Cartesian product, in row order (see Conventions). [host] arrays. */
typedef struct {
    int32_t n_zero;              /* zero cone rows ({0}; its dual is R)                     */
    int32_t n_nonneg;            /* nonnegative orthant rows                                */
    int32_t n_soc;               /* number of second-order cones                            */
    const int32_t *soc_dims;     /* n_soc dimensions, each in [1, 1024]                     */
    int32_t n_psd;               /* number of PSD cones                                     */
    const int32_t *psd_orders;   /* n_psd matrix orders k (1 <= k <= 64); k(k+1)/2 rows each */
    int32_t n_exp;               /* number of exponential cones, 3 rows each                */
    int32_t n_pow;               /* number of power cones K_pow,a, 3 rows each              */
    const double *pow_alpha;     /* n_pow exponents a, each in (0, 1)                       */
    int32_t n_dpow;              /* number of dual power cones K_pow,a*, 3 rows each         */
    const double *dpow_alpha;    /* n_dpow exponents a, each in (0, 1)                      */
} qcpd_cones;

typedef struct {
    double  tol;          /* stop when the LSQR residual estimate <= tol * ||rhs||  (1e-8)   */
    int32_t max_iter;     /* iteration cap; 0 = 100 * (n + m + 1)                             */
    int32_t precond;      /* QCPD_PRECOND_*                                   (JACOBI)         */
    int32_t graph_chunk;  /* LSQR iterations per captured HIP graph launch     (128)           */
    int32_t check_symmetry; /* verify that P is symmetric at create              (1)           */
    int32_t engine;       /* LSQR driver: QCPD_ENGINE_AUTO, _GRAPH, _PERSISTENT (AUTO)         */
    int32_t solver;       /* Krylov method: QCPD_SOLVER_LSQR or QCPD_SOLVER_LSMR (LSQR)      */
    /* Launch layout of the LSQR loop kernels, fixed at qcpd_create (qcpd_set_opts returns
     * QCPD_ERR_INVALID_ARG for a change). 0 in each = the library's choice. None of them
     * changes results beyond the order of floating-point sums. */
    int32_t staged;       /* QCPD_CHOICE_*: products that stage the input's x part (n doubles)
                             in LDS, one workgroup per CU; ON where it fits (n up to about
                             20 000), AUTO where it fits on large problems with n > 8 192    */
    int32_t deep;         /* QCPD_CHOICE_*: deep CSR sums (16 entries per lane in flight) in
                             the fused product with F' (AUTO: problems whose CSR rows
                             outnumber a launch's threads)                                   */
    int32_t nnz_per_lane_F;   /* stored entries per lane of a CSR row, product with F (2)    */
    int32_t nnz_per_lane_FT;  /* the same, fused product with F' (4; deep sums: about 25)    */
    int32_t lanes_x;      /* lanes per x row (P and A' rows) in the product with F and the
                             staged kernels, a power of two <= 64 (from nnz_per_lane_F)      */
    int32_t lanes_y;      /* the same for the y rows (A rows)                               */
    int32_t loop_grid;    /* most workgroups of a loop launch, <= 1024 (1024)                */
    int32_t persist_grid; /* workgroups of the PERSISTENT driver (one wave of the device)     */
    int32_t equil_sweeps; /* EQUIL scaling sweeps, rounded up to even (20)                    */
} qcpd_opts;

#define QCPD_CHOICE_AUTO 0
#define QCPD_CHOICE_OFF  1
#define QCPD_CHOICE_ON   2

/* Krylov methods for the least-squares problems (Sec. 3.1-3.2). Both build the same
 * Golub-Kahan bidiagonalisation from one product with the operator and one with its
 * transpose per iteration, and on these consistent systems both converge to a least-squares
 * solution, which gives the same outputs. LSQR (Paige & Saunders) minimises the residual
 * over the Krylov space; LSMR (Fong & Saunders), the method the paper uses, minimises the
 * norm of the transposed operator times the residual, and keeps one more direction vector.
 * The stopping rule is the same for both: the method's estimate of ||residual|| / ||rhs||
 * at or below tol, then the residual recomputed explicitly. LSMR runs on the GRAPH driver
 * (AUTO picks it; PERSISTENT is rejected with QCPD_ERR_INVALID_ARG) with one more launch per
 * iteration for its recurrences and iterate update. The batched form runs LSQR only. */
#define QCPD_SOLVER_LSQR        0
#define QCPD_SOLVER_LSMR        1

/* LSQR drivers of the single-problem path. GRAPH: two launches per iteration, captured in
 * HIP graphs of graph_chunk iterations, the host polling a device stop flag per graph; each
 * launch finalises the previous launch's reductions at entry, so the loop needs no fences.
 * PERSISTENT: the whole loop in one cooperative launch with two grid barriers per iteration
 * (each barrier writes back and invalidates L2, which costs more than a launch on MI355X).
 * AUTO picks GRAPH. Both give the same results up to the order of floating-point sums. */
#define QCPD_ENGINE_AUTO        0
#define QCPD_ENGINE_GRAPH       1
#define QCPD_ENGINE_PERSISTENT  2

typedef struct {
    int32_t  iters;          /* LSQR iterations                                              */
    double   est_residual;   /* the Krylov method's estimate ||residual|| / ||rhs|| at exit  */
    double   rel_residual;   /* explicit ||F dz + d|| / ||d|| (JVP) or ||F'w + dz|| / ||dz||
                                (VJP), recomputed from the returned iterate                  */
    uint32_t flags;          /* bit 0: not converged (rel_residual > tol or LSQR stopped at
                                the iteration cap); bit 1: non-differentiable warning;
                                bit 2: LEARNED fell back to JACOBI                            */
    float    ms_total;       /* wall time of the call on its stream (HIP events)             */
} qcpd_info;

typedef struct qcpd_handle qcpd_handle;

/* Default options. */
void qcpd_opts_default(qcpd_opts *opts);

/* Build a handle at a solution (Sec. 3.1, "First, we compute Pi z"): copies P, A, q, b, x,
 * y, s; builds A' (for the products with A'); computes Px, x'Px and c = -2Px - q; projects
 * z_y = y - s onto K* block by block and stores each block's Jacobian factors (Appendix A:
 * nonnegative mask, SOC scalars, exponential 3x3 matrices, PSD eigenvectors and the B
 * matrix); computes the Jacobi scales. P: n x n, A: m x n, q: n, b, y, s: m, x: n, all
 * [device]. K: [host]. opts may be NULL (defaults). stream: hipStream_t or NULL.
 * Returns QCPD_OK or QCPD_WARN_NONDIFF with *h set; on error *h is NULL. */
qcpd_status qcpd_create(qcpd_handle **h, const qcpd_csr *P, const qcpd_csr *A,
                        const double *q, const double *b, const qcpd_cones *K,
                        const double *x, const double *y, const double *s,
                        const qcpd_opts *opts, void *stream);

/* JVP (Sec. 3.1): (dx, dy, ds) = DS(theta)[(dP, dA, dq, db)].
 * Inputs [device]: dP_val (nnz P, symmetric on P's pattern), dA_val (nnz A), dq (n), db (m).
 * Outputs [device], caller-allocated: dx (n), dy (m), ds (m). info: [host], may be NULL. */
qcpd_status qcpd_jvp(qcpd_handle *h, const double *dP_val, const double *dA_val,
                     const double *dq, const double *db,
                     double *dx, double *dy, double *ds, qcpd_info *info);

/* VJP (Sec. 3.2): (dP, dA, dq, db) = DS(theta)'[(gx, gy, gs)].
 * Inputs [device]: gx (n), gy (m), gs (m). Outputs [device], caller-allocated:
 * dP_val (nnz P), dA_val (nnz A), dq (n), db (m). info: [host], may be NULL. */
qcpd_status qcpd_vjp(qcpd_handle *h, const double *gx, const double *gy, const double *gs,
                     double *dP_val, double *dA_val, double *dq, double *db,
                     qcpd_info *info);

/* Replace the handle's LSQR options (tolerance, iteration cap, chunk); precond is applied
 * from the next call. Returns QCPD_ERR_INVALID_ARG for bad values. */
qcpd_status qcpd_set_opts(qcpd_handle *h, const qcpd_opts *opts);

/* Supply the two-sided scaling used by QCPD_PRECOND_CUSTOM: LSQR then solves the JVP with
 * diag(d_row) F diag(d_col) and the VJP with diag(d_col) F' diag(d_row). d_col, d_row:
 * (n + m + 1) [device], entries > 0; the values are copied. */
qcpd_status qcpd_set_precond(qcpd_handle *h, const double *d_col, const double *d_row);

/* Copy out [device]: the Jacobi scales (d_jvp: columns of F, d_vjp: columns of F'), the
 * equilibration scales (eq_col, eq_row), each n + m + 1, and the diagonal of DPi_{K*}(z_y)
 * (jdiag, m). Any pointer may be NULL. */
qcpd_status qcpd_get_diagnostics(qcpd_handle *h, double *d_jvp, double *d_vjp, double *eq_col,
                                 double *eq_row, double *jdiag);

/* Measurement support: time the launches of one LSQR iteration of the JVP (the product
 * with F over CSR rows; the product with F': CSR rows of each cone block and its Jacobian
 * block, in one fused launch or in a rows launch followed by a cone launch) by launching each
 * `reps` times back to back on the handle's stream between HIP events, on the handle's
 * current vectors. ms_out [host] 4 entries, the average duration in milliseconds of: the
 * product with F, the product with F' (all its launches), the first launch of that product
 * alone, its second launch alone (0 when it has one launch). Leaves the LSQR state
 * undefined: call it between, not during, derivative evaluations. */
qcpd_status qcpd_profile_kernels(qcpd_handle *h, int32_t reps, float *ms_out);

/* One product with the operator of the least-squares problems, F = D_z N at z (Sec. 2.4):
 * out = F in (transpose = 0) or out = F' in (transpose = 1), unscaled. in, out [device],
 * n + m + 1 entries in the order (x | y | tau), distinct buffers. For users of the operator
 * itself and for checking it against a reference. */
qcpd_status qcpd_apply(qcpd_handle *h, int32_t transpose, const double *in, double *out);

/* Pi_{K*}(zy): the projection onto the dual cone of the handle's cone spec, block by block
 * (Appendix A: nonnegative, SOC, PSD by eigendecomposition, exponential and power cones by
 * their root-finds, dual cones by Moreau). zy, out [device], m entries each, distinct.
 * The handle's own factors are left as they are. Returns QCPD_ERR_CONE when a root-find or
 * an eigendecomposition fails. */
qcpd_status qcpd_proj_dual(qcpd_handle *h, const double *zy, double *out);

typedef struct {
    int32_t newton_iters;    /* Newton steps taken                                           */
    int32_t lsqr_iters;      /* LSQR iterations over all steps                               */
    double  residual;        /* ||G(x, y - s)|| / (1 + ||q|| + ||b||) at the returned point  */
    int32_t converged;       /* 1 when residual <= tol                                       */
} qcpd_resolve_info;

/* Forward solve by refinement from a nearby point (the solution a numerical solver supplies,
 * Sec. 2.2; the previous solution when theta moves in a learning loop, Sec. 3.4): Newton's
 * method on the optimality conditions (Sec. 2.1) in the variables (x, eta = y - s),
 *   G(x, eta) = (P x + A'y + q, -A x + b - y + eta),  y = Pi_{K*}(eta),  s = y - eta,
 * each step K_red step = -G solved as one JVP of this library at the current point along
 * (dP, dA, dq, db) = (0, 0, G_x, G_y), then x += dx, eta += dy - ds. Stops when
 * ||G|| <= tol (1 + ||q|| + ||b||) or after max_newton steps. P, A, q, b, K as in
 * qcpd_create; x (n), y, s (m) [device]: the starting point on entry, the refined solution
 * on return (y and s are always the projections of the final eta, so y is in K*, s in K
 * and y's = 0). opts: the LSQR options of the steps (NULL: defaults). info [host] may be
 * NULL. Returns QCPD_OK, QCPD_WARN_NOT_CONVERGED (the point after the last step is
 * returned), or an error of qcpd_create. Allocates a handle per step. */
qcpd_status qcpd_resolve(const qcpd_csr *P, const qcpd_csr *A, const double *q, const double *b,
                         const qcpd_cones *K, double *x, double *y, double *s,
                         const qcpd_opts *opts, double tol, int32_t max_newton,
                         qcpd_resolve_info *info, void *stream);

/* Launch shape of the LSQR loop, for tuning (an autotuner's choice): the product with F
 * over CSR rows runs on at most grid_F workgroups and the fused product with F' on at most
 * grid_FT (each loops over its work with a grid stride; 0 = the default cap, 512). Results
 * are unchanged up to the order of floating-point sums. Graphs captured earlier are
 * discarded. Synchronises the handle's stream. */
qcpd_status qcpd_set_launch(qcpd_handle *h, int32_t grid_F, int32_t grid_FT);

/* out [host] 4 entries: the current grid_F, grid_FT, and the largest useful values (the
 * work items of each launch). */
qcpd_status qcpd_get_launch(qcpd_handle *h, int32_t *out);

/* The launch layout qcpd_create chose (the options' QCPD_CHOICE_AUTO resolved). out [host]
 * 6 entries: 1 if the loop products stage the input's x part in LDS, 1 if the fused product
 * with F' uses deep CSR sums, 1 if its PSD cones run in a launch of their own, the lanes
 * per CSR row of the x rows and of the y rows in the product with F, and 1 if the staged
 * products read packed copies of P and A (held by the handle: rows padded to whole quads of
 * entries, 16-bit column indices, 10 bytes per entry instead of 12). */
qcpd_status qcpd_get_layout(qcpd_handle *h, int32_t *out);

/* ---------------------------------------------------------------------------------------
 * Learned preconditioner (an addition to the method: the iterative solves of Sec. 3.1-3.2
 * name no preconditioner). For each index i of z = (x, y, tau) a feature row of
 * QCPD_NFEAT floats is read off F; a 3-layer FP32 MLP (QCPD_NFEAT -> 64 -> 64 -> 2, tanh
 * hidden layers) maps it to log corrections (c_col, c_row) of the Jacobi column and row
 * scales: d_col = jacobi_col * exp(c_col), d_row = jacobi_row * exp(c_row).
 *
 * Feature row: 0 log column norm and 1 log row norm of F with each cone block's Jacobian
 * replaced by its diagonal; 2..8 one-hot kind (x, zero, nonneg, SOC, PSD, exp, tau);
 * 9 diagonal of DPi (1 for x and tau); 10 log(1 + |P_ii|) (x only); 11 log(1 + stored
 * entries in row i of [P A'] (x) or of A (y)).
 *
 * Parameter blob, QCPD_MLP_PARAMS floats: mu[F] sd[F] (feature standardisation, fixed at
 * init from data), W1[64][F] b1[64] W2[64][64] b2[64] W3[2][64] b3[2], W[out][in] row-major.
 * Training minimises the mean over rows of the squared error against target rows
 * (c_col, c_row); qcpd_learned_targets gives the corrections that reproduce the handle's
 * equilibration scales.
 * ------------------------------------------------------------------------------------- */
#define QCPD_NFEAT        12
#define QCPD_MLP_HIDDEN   64
#define QCPD_MLP_PARAMS   (2 * QCPD_NFEAT + QCPD_MLP_HIDDEN * QCPD_NFEAT + QCPD_MLP_HIDDEN + \
                           QCPD_MLP_HIDDEN * QCPD_MLP_HIDDEN + QCPD_MLP_HIDDEN +             \
                           2 * QCPD_MLP_HIDDEN + 2)

/* Feature rows of the handle's operator: feat [device] (n + m + 1) x QCPD_NFEAT, row-major. */
qcpd_status qcpd_features(qcpd_handle *h, float *feat);

/* Training targets of the handle: target [device] (n + m + 1) x 2, row-major, the log ratios
 * of the equilibration scales to the Jacobi scales (columns, rows). */
qcpd_status qcpd_learned_targets(qcpd_handle *h, float *target);

/* Install the scales predicted by a model (weights [device], QCPD_MLP_PARAMS floats) on the
 * handle, for QCPD_PRECOND_LEARNED. Features and inference run on the handle's stream; the
 * weights are not kept. Replaces earlier learned scales. */
qcpd_status qcpd_set_learned(qcpd_handle *h, const float *weights);

/* Initialise a model [device]: mu and sd from the first nrows feature rows (sd below 1e-3
 * becomes 1), Glorot-uniform weights from a SplitMix64 hash of (seed, index), zero biases. */
qcpd_status qcpd_mlp_init(const float *feat, int32_t nrows, uint64_t seed, float *weights,
                          void *stream);

/* Raw model outputs: out [device] nrows x 2 from feat [device] nrows x QCPD_NFEAT. */
qcpd_status qcpd_mlp_predict(const float *feat, int32_t nrows, const float *weights, float *out,
                             void *stream);

/* Floats of workspace qcpd_mlp_grad needs for nrows rows. */
int64_t qcpd_mlp_workspace_floats(int32_t nrows);

/* Gradient of the loss (1/nrows) sum_r ||MLP(feat_r) - target_r||^2 with respect to the
 * parameters: grad [device] QCPD_MLP_PARAMS + 1 floats, the last one the loss itself
 * (mu, sd entries are 0). workspace [device]: qcpd_mlp_workspace_floats(nrows) floats.
 * Asynchronous on the stream. Sums run in a fixed order (deterministic). */
qcpd_status qcpd_mlp_grad(const float *feat, const float *target, int32_t nrows,
                          const float *weights, float *workspace, float *grad, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): qcpd_mlp_grad with its workspace replaced by a
 * fixed array inside the library, one per GPU, held until the process ends (5.27 MB: the
 * partial gradients of the at most 256 workgroups one launch uses, so every nrows >= 1
 * fits; a launch that would need more is rejected with QCPD_ERR_INVALID_ARG). Same
 * arguments, kernels and summation order as qcpd_mlp_grad, so the results are identical.
 * Calls no hipMalloc / hipFree. The first call on a device resolves the array's address
 * (hipGetSymbolAddress); make that call outside graph capture. Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams, or host threads
 * without ordering) race and give wrong gradients. Asynchronous on the stream. */
qcpd_status qcpd_mlp_grad_noalloc(const float *feat, const float *target, int32_t nrows,
                                  const float *weights, float *grad, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on the trained
 * parameters; adam_m, adam_v [device] QCPD_MLP_PARAMS floats, zero before step 1. */
qcpd_status qcpd_mlp_adam(const float *grad, float *weights, float *adam_m, float *adam_v,
                          int32_t step, float lr, void *stream);

/* ---------------------------------------------------------------------------------------
 * Batched form: many QCPs of uneven sizes evaluated together. The LSQR iterations of all
 * problems advance in the same two launches per iteration (work items grouped by problem,
 * captured in HIP graphs); each problem keeps its own LSQR state, iteration count and
 * stopping test, so the results equal those of qcpd_jvp / qcpd_vjp on each problem up to
 * rounding. The vjp of the batch is the per-problem
 * adjoint of Sec. 3.2, the jvp the per-problem derivative of Sec. 3.1.
 * ------------------------------------------------------------------------------------- */
typedef struct qcpd_batch qcpd_batch;

/* Sizes of the problems of a batch; all arrays [host], nprob entries each. */
typedef struct {
    int32_t nprob;
    const int32_t *n;            /* variables of each problem (>= 1)               */
    const int32_t *m;            /* constraint rows of each problem (>= 0)         */
    const int32_t *nnz_P;        /* stored entries of each P                      */
    const int32_t *nnz_A;        /* stored entries of each A                      */
    const qcpd_cones *cones;     /* cone of each problem (same rules as above)     */
} qcpd_batch_layout;

/* Build a batch at the problems' solutions. All data arrays are [device] concatenations,
 * problem after problem: P_rowptr has sum(n_i + 1) entries (each problem's local row
 * pointers, starting at 0), P_colind / P_val sum(nnz_P) entries with local column indices;
 * A likewise with sum(m_i + 1) row pointers; q, x: sum(n_i); b, y, s: sum(m_i).
 * opts->precond may be NONE, JACOBI or EQUIL (each problem's two-sided equilibration is
 * computed here, 20 sweeps); opts->solver must be QCPD_SOLVER_LSQR (else
 * QCPD_ERR_INVALID_ARG); graph_chunk is the number of LSQR iterations (of all problems)
 * per captured HIP graph launch, at most 32 here (the host shrinks the launch lists to the
 * running problems between graph launches). Of the launch-layout fields of opts the batch
 * reads nnz_per_lane_F only: the stored entries per lane of a CSR row in its loop kernels
 * (0: 32; the autotuner's choice), fixed at create. */
qcpd_status qcpd_batch_create(qcpd_batch **hb, const qcpd_batch_layout *layout,
                              const int32_t *P_rowptr, const int32_t *P_colind, const double *P_val,
                              const int32_t *A_rowptr, const int32_t *A_colind, const double *A_val,
                              const double *q, const double *b, const double *x, const double *y,
                              const double *s, const qcpd_opts *opts, void *stream);

/* Per-problem JVPs in one launch. [device] concatenations as in qcpd_batch_create:
 * dP_val sum(nnz_P), dA_val sum(nnz_A), dq sum(n), db sum(m); outputs dx sum(n), dy and ds
 * sum(m). info: [host] array of nprob entries or NULL. Returns QCPD_WARN_NOT_CONVERGED when
 * any problem did not reach the tolerance. */
qcpd_status qcpd_batch_jvp(qcpd_batch *hb, const double *dP_val, const double *dA_val,
                           const double *dq, const double *db, double *dx, double *dy,
                           double *ds, qcpd_info *info);

/* Per-problem VJPs in one launch; layouts as above. */
qcpd_status qcpd_batch_vjp(qcpd_batch *hb, const double *gx, const double *gy, const double *gs,
                           double *dP_val, double *dA_val, double *dq, double *db,
                           qcpd_info *info);

/* Replace the batch's LSQR options (tolerance, iteration cap, NONE, JACOBI or EQUIL;
 * solver must be QCPD_SOLVER_LSQR). */
qcpd_status qcpd_batch_set_opts(qcpd_batch *hb, const qcpd_opts *opts);

/* Persistent workgroups of the batch's per-problem phases (right-hand side and first product
 * before the LSQR loop; owed update, residual and outputs after it), each taking whole
 * problems from a queue until it is empty: grid >= 1, capped at the number of problems; 0
 * restores the default (all workgroups that fit on the device at once). For tuning. */
qcpd_status qcpd_batch_set_launch(qcpd_batch *hb, int32_t grid);

/* out [host] 2 entries: the current grid and the default. */
qcpd_status qcpd_batch_get_launch(qcpd_batch *hb, int32_t *out);

/* Free a batch (NULL is allowed). */
void qcpd_batch_destroy(qcpd_batch *hb);

/* Free a handle (NULL is allowed). */
void qcpd_destroy(qcpd_handle *h);

/* Static string for a status code. */
const char *qcpd_status_str(qcpd_status s);

#ifdef __cplusplus
}
#endif

#endif /* QCPD_H */
