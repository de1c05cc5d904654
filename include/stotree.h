/*
 * stotree — dual proximal solvers for scenario-tree stochastic optimal control
 * on AMD Instinct MI355X (gfx950), FP64.
 *
 * Public C ABI.  Plain pointers and sizes only; no C++ or framework types.
 *
 * The problem (arXiv 2107.01745, Sec. II-A/II-B):
 *   minimise over u_i (non-leaf i) and x_i (i >= 1)
 *     sum_{i non-leaf} pi_i ([x_i;u_i]' [[Q_i,S_i'],[S_i,R_i]] [x_i;u_i] + q_i'x_i + r_i'u_i)
 *   + sum_{j leaf}     pi_j (x_j' P_j x_j + p_j' x_j)
 *   subject to x_0 = p,  x_j = A_j x_i + B_j u_i + c_j for every child j of i,
 *   xmin_i <= x_i <= xmax_i (every node), umin_i <= u_i <= umax_i (non-leaf).
 * Costs carry no factor 1/2.  Each non-leaf node owns the stage cost of its
 * (x_i, u_i) weighted by its own probability.
 *
 * Tree numbering (Sec. II-A): stage-major.  Root = 0; the nodes of stage t are
 * [stage_ptr[t], stage_ptr[t+1]); the children of node i are the contiguous
 * range [child_ptr[i], child_ptr[i+1]) and children appear in parent order;
 * all leaves sit at stage N and are numbered last, so the non-leaf nodes are
 * the prefix [0, V_nl) with V_nl = stage_ptr[N].
 *
 * Dual vector layout (Sec. II-C, the vector z = Hx and its dual y): for each
 * non-leaf node i, nx state rows then nu input rows at offset i*(nx+nu); for
 * each leaf j, nx state rows at offset V_nl*nu + j*nx.  Its length is
 * m = V_nl*(nx+nu) + (V - V_nl)*nx.
 *
 * Preconditioning (Sec. III-E): when enabled at tree_factor, every dual vector
 * handed to dual_grad and the solvers is the scaled dual ybar_i = y_i/sqrt(pi_i)
 * and residuals are reported in those units (plus unscaled, see solver_info).
 *
 * Matrices are row-major FP64.  Unless stated, every call is asynchronous on
 * the caller's HIP stream (void* hip_stream, NULL = default stream), device
 * pointers are borrowed for the duration of the call, and calls that share a
 * tree_factors handle must not overlap in time.
 *
 * Return codes: 0 OK; 1 NOT_CONVERGED (outputs hold the last iterate);
 * -1 ERR_ARG; -2 ERR_TREE (ordering/ranges/probabilities); -3 ERR_NOT_PD (a
 * Cholesky pivot of the factor step failed); -4 ERR_BOX (lo > hi); -5
 * ERR_NUMERIC (NaN/Inf); -6 ERR_DIVERGED; -7 ERR_DEVICE; -8 ERR_OOM.  After
 * a negative code stotree_last_error() describes the failure.
 */
#ifndef STOTREE_H
#define STOTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STOTREE_OK 0
#define STOTREE_NOT_CONVERGED 1
#define STOTREE_ERR_ARG (-1)
#define STOTREE_ERR_TREE (-2)
#define STOTREE_ERR_NOT_PD (-3)
#define STOTREE_ERR_BOX (-4)
#define STOTREE_ERR_NUMERIC (-5)
#define STOTREE_ERR_DIVERGED (-6)
#define STOTREE_ERR_DEVICE (-7)
#define STOTREE_ERR_OOM (-8)

/* Scenario tree (Sec. II-A).  All arrays are HOST memory. */
typedef struct {
    int32_t nx, nu, N, num_nodes;   /* state/input sizes, horizon, V         */
    const int32_t *stage_ptr;       /* [N+2]                                 */
    const int32_t *ancestor;        /* [V], -1 at the root                   */
    const int32_t *child_ptr;       /* [V_nl+1]                              */
    const double *prob;             /* [V]; pi_0 = 1, each stage sums to 1   */
} tree_desc;

/* Problem data (Sec. II-A dynamics, Sec. II-B costs, Sec. III-D boxes).
 * All arrays are HOST memory, row-major. */
typedef struct {
    const double *A;     /* [V][nx][nx]  dynamics into node j (row 0 unused) */
    const double *B;     /* [V][nx][nu]                                      */
    const double *c;     /* [V][nx]      offset of the dynamics (w_j)        */
    const double *Q;     /* [V_nl][nx][nx]                                   */
    const double *R;     /* [V_nl][nu][nu] positive definite                 */
    const double *S;     /* [V_nl][nu][nx] or NULL (zero)                    */
    const double *q;     /* [V_nl][nx] or NULL                               */
    const double *r;     /* [V_nl][nu] or NULL                               */
    const double *P;     /* [V-V_nl][nx][nx] terminal weights (leaf order)   */
    const double *p;     /* [V-V_nl][nx] or NULL                             */
    const double *xmin, *xmax;  /* [V][nx], +-INFINITY allowed              */
    const double *umin, *umax;  /* [V_nl][nu], +-INFINITY allowed           */
    /* Optional constraint map of Sec. II-B, the same at every node: rows
     * z_i = F x_i + G u_i at non-leaf nodes, z_j = FN x_j at leaves.  F NULL
     * (default): the rows are (x_i, u_i) and x_j themselves with the boxes
     * above.  Otherwise the dual has nc rows per non-leaf node and ncN per
     * leaf (m = V_nl nc + (V - V_nl) ncN, same node order), bounded by
     * zmin <= z <= zmax given in that layout, and the box arrays above are
     * not read (they may be NULL).  Not for tree_factor_shared. */
    int32_t nc, ncN;            /* rows per non-leaf node / leaf (nc >= 1)  */
    const double *F, *G, *FN;   /* [nc][nx], [nc][nu], [ncN][nx]             */
    const double *zmin, *zmax;  /* [m], +-INFINITY allowed                   */
    /* Optional soft rows (Sec. II-B: a distance-to-set function in place of
     * the indicator), in the dual layout; NULL: every row hard.  Row k of node
     * i adds pi_i wgt[k] psi(dist(z_k, [lo_k, hi_k])) to the cost, psi the
     * Huber function of threshold hub[k] (t^2/(2 hub) below hub, t - hub/2
     * above; hub = 0: the distance itself, an l1 penalty when lo = hi = 0);
     * wgt[k] = +INFINITY keeps row k a hard bound.  wgt > 0, hub >= 0. */
    const double *wgt, *hub;    /* [m] or NULL                               */
} problem_data;

typedef struct {
    double lambda;       /* step of the forward-backward map; 0 = 1/(1.1 L)
                            with L from dual_lipschitz (100 iterations)      */
    double eps;          /* stop when ||R_lambda||_inf <= eps (default 1e-6) */
    double eps_curv;     /* L-BFGS curvature guard eps' (default 1e-12)      */
    int32_t mem;         /* L-BFGS memory (default 5, at most 16)            */
    int32_t nu_max;      /* line-search trials tau = 2^-nu, nu = 0..nu_max
                            (default 10, at most 30)                        */
    int32_t max_iter;    /* default 1000                                     */
    int32_t check_every; /* host reads the stop flag every k iterations (1)  */
    /* lambda backtracking (Sec. III-B), MINFBE and NAMA; each halving empties
     * the L-BFGS memory and takes the update again from the same y:
     *   0  fixed lambda (default);
     *   1  halve when f-hat(T(w)) > f-hat(w) - lambda <grad f-hat(w), R(w)>
     *      + (1 - beta) lambda/2 ||R(w)||^2 at the point w the step was taken
     *      from, beta = bt_param in [0, 1);
     *   2  halve when lambda ||grad f-hat(T(y)) - grad f-hat(y)||
     *      > eps'' ||T(y) - y||, eps'' = bt_param in (0, 1/2).
     * With backtracking and lambda = 0 the start is 1/L from 5 power
     * iterations (an L from below, so a step at least 1/L). */
    int32_t backtrack;
    /* infeasibility test every div_window iterations (0: 50; < 0: off): the
     * change d of the dual over the window certifies that no point satisfies
     * the dynamics and the constraints (lambda ||H x-hat(d)|| <= 1e-3 ||d||:
     * d is annihilated by the dual Hessian, and the dual objective falls
     * along d at least 1e-4 ||d|| ||R||; for GPAD the first bound is
     * 1e-4 ||d||); when two consecutive windows pass, the instance stops
     * with ERR_DIVERGED.  The test is a numerical one: a
     * feasible problem whose dual optimum is orders of magnitude beyond the
     * dual's motion per window can be flagged (for example a constraint map
     * that forces an unstable closed loop). */
    int32_t div_window;
    double bt_param;
    /* DEVICE [instances][trace_iters][40] or NULL: row k of an instance
     * holds lambda, ||R(y^k)||_inf, the accepted nu (-1: tau = 0), nu_max, the
     * L-BFGS pairs of the direction, then phi(w_nu) - phi(y^k) for every
     * trial nu = 0..nu_max of update k (MINFBE and NAMA). */
    double *trace;
    int32_t trace_iters, reserved;
} solver_opts;

typedef struct {
    int32_t iters, sweeps_affine, sweeps_hom, ls_trials, lbfgs_push, lbfgs_skip, status;
    double res_scaled_inf;    /* ||R||_inf in the solver's (scaled) units    */
    double res_unscaled_inf;  /* ||z - Hx||_inf in the problem's units       */
    double lambda;            /* step used (the last one with backtracking)  */
    double seconds;           /* host wall time of the call                  */
    int32_t backtracks;       /* halvings of lambda                          */
    int32_t reserved;
} solver_info;

typedef struct tree_factors tree_factors;  /* opaque; owns device memory */

/*
 * Factor step (Sec. III-D, the Riccati-type recursion computed once before the
 * solves).  Validates the tree (stage-major order, contiguous child ranges,
 * every stage's probabilities sum to 1 within 1e-12, leaves only at stage N),
 * the boxes (lo <= hi) and finiteness, copies the data to the device, runs the
 * per-stage factor kernels (batched Cholesky of R-tilde and the feedback
 * gains) and packs every factor in the layout the sweeps stream.  precondition
 * = 1 selects the sqrt(pi) scaling of Sec. III-E.  The handle owns all device
 * memory it needs, including the solvers' workspace, which is sized at the
 * first solve and reused.  Synchronous with respect to hip_stream.
 * Errors: ERR_ARG (NULL pointers, nx < 1, nu < 1, N < 1, nx+nu > 256),
 * ERR_TREE, ERR_BOX, ERR_NUMERIC (non-finite data), ERR_NOT_PD, ERR_OOM,
 * ERR_DEVICE.  On error *out is NULL.
 */
int tree_factor(const tree_desc *tree, const problem_data *data, int precondition,
                void *hip_stream, tree_factors **out);

/* Releases the handle and its device memory (NULL is a no-op). */
void tree_factors_free(tree_factors *f);

/*
 * Batched factor step: count independent trees ("instances", each its own
 * tree_desc / problem_data, of any sizes and horizons) factored into one
 * handle.  Every other entry point then works on all instances at once with
 * the per-instance vectors concatenated in instance order: duals [sum m_b],
 * x [sum V_b nx_b], u [sum V_nl,b nu_b], x0 [sum nx_b] (offsets from
 * tree_instance_dims).  Each sweep is one set of launches covering every
 * instance (work lists of (instance, node) and (instance, chain) pairs).
 * count = 1 is exactly tree_factor.  Errors as tree_factor; the message names
 * the failing instance.
 */
int tree_factor_batch(int count, const tree_desc *trees, const problem_data *data, int precondition,
                      void *hip_stream, tree_factors **out);

/*
 * count instances that share one tree, its matrices, costs and boxes, and
 * differ in the initial state x0 (given per call, [count][nx]) and, if c is
 * not NULL, in the disturbances: HOST c [count][V][nx] (node 0 ignored)
 * replaces data->c for instance k (data->c still defines the factor step).
 * The factor step runs once and the handle keeps one copy of the matrices;
 * with c, the affine terms of each instance are derived from the value-
 * function Hessians of the factor step (chat_k = chat + P (c_k - c)).  Vectors
 * are concatenated in instance order as for tree_factor_batch (instance k at k
 * times the single-tree sizes).  When count is a multiple of 64 and
 * nx + nu <= 128, every sweep (dual_grad, the solvers, dual_lipschitz) runs as
 * panels of 64 instances on the FP64 matrix cores, streaming the matrices
 * once per panel (the extra parallelism of Sec. III-C across instances).
 * Errors as tree_factor, plus ERR_ARG for count < 1 and ERR_NUMERIC for a
 * non-finite c.
 */
int tree_factor_shared(const tree_desc *tree, const problem_data *data, int precondition, int count,
                       const double *c, void *hip_stream, tree_factors **out);

/* Sizes of a handle, written to HOST out[10]: instances, precondition flag,
 * total dual length, total primal length, sum V nx (x), sum V_nl nu (u),
 * sum nx (x0), total nodes, device bytes held, largest nx+nu.  ERR_ARG on
 * NULL. */
int tree_dims(const tree_factors *f, int64_t *out);

/* Sizes of instance b, written to HOST out[12]: nx, nu, N, V, V_nl, m, n,
 * s_star (first stage from which every node has one child), and the offsets
 * of the instance in the concatenated dual, x, u and x0 vectors.  ERR_ARG on
 * NULL or b out of range. */
int tree_instance_dims(const tree_factors *f, int b, int64_t *out);

/*
 * Dual gradient (Algorithm 3) and Hessian-vector products (Algorithm 4).
 * homogeneous = 0: x(y), the minimiser of the inner problem of Sec. III-D for
 * the dual y, with x_0 = x0; the dual gradient is -H x(y).  homogeneous = 1:
 * the linear part x-hat(y) (no affine terms, x_0 = 0); the Hessian-vector
 * product of the dual function is -H x-hat(y).  With preconditioning, y is the
 * scaled dual (the kernels apply sqrt(pi) per node) and x, u are unscaled.
 * DEVICE pointers: x0 [nrhs][nx] (ignored when homogeneous; may be NULL then),
 * y [nrhs][m], x [nrhs][V][nx] (x_0 included), u [nrhs][V_nl][nu] (for a
 * batched handle, the concatenated sizes of tree_dims).
 * nrhs >= 1; right-hand sides are swept 64 at a time on the FP64 matrix
 * cores while at least 64 remain (when every nx + nu <= 128), the rest two at
 * a time, each group sharing one streaming of the factors.  On a shared
 * handle (tree_factor_shared) whose copies form whole panels of 64, each
 * right-hand side sweeps its copies as panels when the copy count reaches
 * the schedule's panel minimum (sweep_schedule knobs[4]); otherwise, and on
 * other shared handles, the right-hand sides go two at a time.
 * Errors: ERR_ARG, ERR_OOM (workspace growth), ERR_DEVICE.
 */
int dual_grad(const tree_factors *f, const double *x0, const double *y, int homogeneous,
              int nrhs, double *x, double *u, void *hip_stream);

/*
 * dual_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * arguments, results and errors as dual_grad, but the per-call q-hat / k
 * workspace of the sweeps lives in a static device array of the library
 * (128 MiB per GPU, held from the first use of the library on that GPU until
 * the process ends) instead of the handle's workspace, and the call makes no
 * hipMalloc, hipFree or other allocating call.  The workspace needed is
 * w * (sum V nx + sum V_nl nu) doubles, w = 1 on a shared handle swept as
 * panels, 64 when nrhs >= 64 right-hand sides run as matrix-core panels,
 * else min(nrhs, 2); a call needing more than the 128 MiB returns ERR_ARG
 * before any work.  Every call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * undefined results.  Nothing in the array needs clearing between calls.
 */
int dual_grad_noalloc(const tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs,
                      double *x, double *u, void *hip_stream);

/*
 * Sweep schedule of a handle: how the stage-parallel sweeps of Sec. III-D
 * (Algorithms 3 and 4) are cut into GPU work.  HOST knobs[5]:
 *   knobs[0] smallest lane group walking one chain below s*: 8, 16, 32 or 64
 *            lanes (an instance's chains use the smallest power of two G at
 *            least this with 2G >= nx + nu, at most 64); default 8;
 *   knobs[1] chain order: 1 costliest wavefront items first (default), 0
 *            instance order;
 *   knobs[2] cap on the wavefronts sharing one node above s*: 1, 2, 4, 8 or
 *            16 (default 16);
 *   knobs[3] stages above s*: 0 one launch per stage, a workgroup per node
 *            (default); 1 the backward stages in one launch in which each
 *            node is taken up by the workgroup that finishes its last child;
 *            2 one launch per stage, the nodes of instances with nx + nu <= 64
 *            walked by lane groups as the chains are; 3 (4) each instance's
 *            first stages of at most 64 (256) nodes in one launch per
 *            direction, a workgroup per node that waits on device-wide
 *            counters for its children (backward) or its parent (forward),
 *            the other stages one launch each.  A wait in modes 3 and 4 that
 *            has not ended after about a second gives up: that sweep and
 *            every later one of the handle then write NaN to the nodes of
 *            those stages, until the schedule is set again;
 *   knobs[4] shared handles whose copies form whole panels of 64: the fewest
 *            unfinished copies for which a sweep runs as panels on the
 *            matrix cores (a panel whose copies have all finished is
 *            skipped); below it the solvers' sweeps take the lane-group
 *            route, which skips each finished copy.  0 .. 2^24 (any value
 *            above the copy count: never panels); default 16.  dual_grad
 *            counts every copy as unfinished.
 * knobs[1] changes no result bit; knobs[0], knobs[2], knobs[3] and knobs[4]
 * change the order of some per-node sums (equal to rounding).
 * sweep_schedule rebuilds the work lists (synchronous; ERR_ARG for values
 * outside these sets, ERR_OOM, ERR_DEVICE); sweep_schedule_get reads them.
 * A schedule change invalidates the handle's sweep graphs.
 */
int sweep_schedule(tree_factors *f, const int32_t *knobs);
int sweep_schedule_get(const tree_factors *f, int32_t *knobs);

/*
 * Autotuner: times homogeneous sweeps (Algorithm 4 streams the same data as
 * Algorithm 3) of nrhs in {1, 2} right-hand sides on zero duals, one untimed
 * and reps timed sweeps per candidate, over each knob in turn (coordinate
 * descent from the current schedule) and keeps the fastest.  On a shared
 * handle swept as panels it tunes knobs[0..3] on the lane-group route, then
 * times one panel sweep of all copies and sets knobs[4] where the two costs
 * meet, the lane-group cost taken as proportional to the unfinished copies
 * (copy count + 1 when the lane groups are faster even for all of them);
 * elsewhere knobs[4] is left as it is.  HOST knobs_out[5] and ms_out
 * (milliseconds per sweep of the kept schedule, all copies) may be NULL.
 * Allocates and frees its own scratch; synchronous.  Errors: ERR_ARG,
 * ERR_OOM, ERR_DEVICE.
 */
int sweep_autotune(tree_factors *f, int nrhs, int reps, int32_t *knobs_out, double *ms_out,
                   void *hip_stream);

/*
 * One dual_grad call recorded as a HIP graph (kernel nodes only) and replayed
 * with one launch.  Arguments as dual_grad with nrhs in {1, 2}; the device
 * pointers are bound at creation, so every replay reads x0, y and writes x, u
 * at those addresses.  sweep_graph_launch enqueues one replay on hip_stream;
 * it returns ERR_ARG if the handle's schedule changed since creation (record
 * a new graph then).  Free every graph of a handle before the handle.
 * Errors: ERR_ARG, ERR_OOM, ERR_DEVICE.
 */
typedef struct sweep_graph sweep_graph;
int sweep_graph_create(const tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs,
                       double *x, double *u, sweep_graph **out);
int sweep_graph_launch(sweep_graph *g, void *hip_stream);
void sweep_graph_free(sweep_graph *g);

/*
 * Lipschitz constant L of the dual gradient (largest eigenvalue of the dual
 * Hessian, in the scaled variables if the handle is preconditioned) by power
 * iteration on Algorithm 4, started from the all-ones vector; the step
 * lambda must lie in (0, 1/L) (Algorithm 1 input).  Writes HOST L_out[b]
 * for every instance b (one value for a single tree).  Synchronous.
 * Errors: ERR_ARG, ERR_DEVICE.
 */
int dual_lipschitz(const tree_factors *f, int iters, double *L_out, void *hip_stream);

/*
 * Dual MINFBE with L-BFGS directions (Algorithm 1).  Per iteration: one affine
 * sweep x(y), one homogeneous sweep for the FBE gradient, one homogeneous
 * sweep x-hat(d) for the line search, whose trial steps tau = 2^-nu are all
 * evaluated in one pass from tau-independent coefficients (Sec. III-B); the
 * largest tau with phi(y + tau d) <= phi(y) is taken (tau = 0 if none), then
 * y+ = T_lambda(y + tau d).  DEVICE: x0 [nx], y_inout [m] (initial dual on
 * entry, zeros for a cold start; last iterate on exit), x [V][nx],
 * u [V_nl][nu] (receive x(y) at the returned y).  HOST: opts (NULL =
 * defaults), info (may be NULL).  Synchronous.  On a batched handle every
 * instance iterates with its own step, line search, L-BFGS memory and stop
 * test in the same launches, and stops independently; lambda = 0 gives each
 * instance 1/(1.1 L_b); info summarises (iters = largest, status = worst) and
 * solve_info_batch gives the per-instance records.  Returns OK,
 * NOT_CONVERGED, ERR_NUMERIC (NaN/Inf in the iterates, or more than 50 halvings
 * of lambda), ERR_DIVERGED (the infeasibility test of solver_opts fired),
 * ERR_ARG, ERR_OOM, ERR_DEVICE.
 */
int minfbe_solve(const tree_factors *f, const double *x0, const solver_opts *opts,
                 double *y_inout, double *x, double *u, solver_info *info, void *hip_stream);

/*
 * NAMA on the dual (Algorithm 2) with the extra parallelism of Sec. III-C:
 * per iteration one affine sweep x(y) and ONE two-right-hand-side homogeneous
 * sweep giving x-hat(r) and x-hat(d) together; trial points
 * w = y - (1 - tau) lambda r + tau d (tau = 0 is the forward-backward step),
 * all tau evaluated in one pass; y+ = T_lambda(w).  Same arguments, outputs
 * and errors as minfbe_solve.
 */
int nama_solve(const tree_factors *f, const double *x0, const solver_opts *opts,
               double *y_inout, double *x, double *u, solver_info *info, void *hip_stream);

/*
 * Accelerated dual proximal gradient (GPAD): the warm start of Sec. III-F
 * and the comparison method of Sec. IV-A.  From y^0 = y^{-1} = y_inout and
 * theta_0 = theta_{-1} = 1, update k takes the forward-backward step at the
 * extrapolated point w^k = y^k + theta_k (1/theta_{k-1} - 1)(y^k - y^{k-1}):
 * y^{k+1} = T_lambda(w^k), theta_{k+1} = (sqrt(theta_k^4 + 4 theta_k^2) -
 * theta_k^2)/2; one affine sweep (Algorithm 3) per update.  The stop test is
 * ||R_lambda(w^k)||_inf <= eps; y_inout receives the last point evaluated,
 * w^k (so max_iter = 5 is the paper's five-iteration warm start, ending
 * with w^5).  lambda must lie in (0, 1/L]; lambda = 0 takes 1/(1.1 L).  The
 * L-BFGS, line-search and backtracking options are ignored.  Arguments,
 * outputs and errors as minfbe_solve.
 */
int gpad_solve(const tree_factors *f, const double *x0, const solver_opts *opts, double *y_inout, double *x,
               double *u, solver_info *info, void *hip_stream);

/*
 * Learned warm start (the warm-start slot of Sec. III-F, filled by a node-wise
 * MLP instead of accelerated-gradient iterations).  Features of node i of an
 * instance with initial state x0: [x0, c_i/c_scale, (mean of c on the path
 * root..i)/c_scale, one-hot(stage)], din = 3 nx + N + 1; network din -> dh ->
 * dh -> dout = nx + nu with ReLU, FP32 parameters in one flat array
 * [W1 (din x dh), b1, W2 (dh x dh), b2, W3 (dh x dout), b3], row-major, FP32
 * accumulation.  Rows are nodes in instance order (the sum of V over the
 * instances); all instances of a handle must share nx, nu and N (ERR_ARG).
 * All pointers are DEVICE pointers except where stated; calls are
 * asynchronous on hip_stream.  The solver's residual decides between the
 * prediction and the cold start (dual_select); accuracy never changes.
 */
int64_t warm_mlp_params(int din, int dh, int dout);            /* parameter count */
int64_t warm_mlp_work_len(int rows, int din, int dh, int dout); /* floats of work */
/* Y [rows][dout] = MLP(X [rows][din]); H (2 rows dh floats) keeps the
 * activations: the rows x dh block of layer 1, then the block of layer 2. */
int warm_mlp_forward(int rows, int din, int dh, int dout, const float *params, const float *X, float *H,
                     float *Y, void *hip_stream);
/* Gradient of the loss w.r.t. the parameters (grad [params]) given dY [rows][dout]
 * and the H of the forward pass; work [warm_mlp_work_len] floats.  The
 * reductions over rows run in a fixed order (deterministic). */
int warm_mlp_backward(int rows, int din, int dh, int dout, const float *params, const float *X,
                      const float *H, const float *dY, float *grad, float *work, void *hip_stream);
/* Masked squared error: dY = 2 mask (Y - T) inv_count; loss2 [2] receives
 * (sum mask (Y - T)^2, sum mask); part is DEVICE scratch of 512 doubles.
 * inv_count 0: 1 / max(1, sum mask) is formed on the device (no host read). */
int warm_mse_grad(int64_t n, const float *Y, const float *T, const float *mask, float inv_count, float *dY,
                  double *loss2, double *part, void *hip_stream);
/* Minibatch rows: dst [rows][cols] = src [idx[r]][cols] (src has src_rows
 * rows; idx [rows] int64).  An index outside [0, src_rows) sets the DEVICE
 * int *bad to 1 (it is never cleared here) and leaves that row of dst as it
 * was; the caller clears and reads bad when it synchronises anyway. */
int warm_gather(int64_t rows, int cols, const float *src, int64_t src_rows, const int64_t *idx, float *dst,
                int *bad, void *hip_stream);
/* One Adam step (Kingma and Ba) with bias correction at step >= 1. */
int warm_adam(int64_t n, float *params, const float *grad, float *m, float *v, float lr, float beta1,
              float beta2, float eps, int step, void *hip_stream);
/* Features X [sum V][din] of every node; x0 [sum nx] DEVICE. */
int warm_features(const tree_factors *f, const double *x0, float c_scale, float *X, void *hip_stream);
/* Dual vector y [m] from the rows Y [sum V][dout] times y_scale (root state
 * rows set to zero), and the inverse map with a mask of existing rows. */
int warm_scatter(const tree_factors *f, const float *Y, float y_scale, double *y, void *hip_stream);
int warm_targets(const tree_factors *f, const double *y, float y_scale, float *T, float *mask,
                 void *hip_stream);
/* Zero the dual rows of every instance b with keep[b] == 0 (HOST keep[count]). */
int dual_select(const tree_factors *f, double *y, const int32_t *keep, void *hip_stream);
/* Copy the dual rows of every instance b with keep[b] == 0 from y_other into
 * y (DEVICE y, y_other [m]; HOST keep[count]). */
int dual_merge(const tree_factors *f, double *y, const double *y_other, const int32_t *keep, void *hip_stream);

/* Per-instance records of the last minfbe_solve / nama_solve on this handle,
 * written to HOST infos[count].  ERR_ARG on NULL. */
int solve_info_batch(const tree_factors *f, solver_info *infos);

/*
 * Phase timing for measurement tools.  stotree_timing(1) makes every sweep
 * record HIP events around each of its phases on the stream it runs on
 * (0 backward chain kernel, 1 backward per-stage kernels, 2 forward per-stage
 * kernels, 3 forward chain kernel); stotree_timing(0) stops recording.
 * stotree_timing_read synchronises on the recorded events and writes, per
 * phase, the summed milliseconds (HOST ms[4]) and the number of launches
 * (HOST count[4]), then clears the record.  Process-wide state; not for use
 * while several threads sweep.  Errors: ERR_ARG, ERR_DEVICE.
 */
int stotree_timing(int enable);
int stotree_timing_read(double *ms, int64_t *count);

/* Message describing the last error on the calling thread ("" if none). */
const char *stotree_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STOTREE_H */
