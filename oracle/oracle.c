/*
 * Plain CPU oracle for the dual proximal solvers on scenario trees.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * Everything is FP64, row-major, plain sequential loops, written for a reader
 * to check against the paper (arXiv 2107.01745) by eye:
 *
 *   problem      Sec. II-A/II-B: tree dynamics x_j = A_j x_i + B_j u_i + c_j,
 *                quadratic costs with node probabilities, boxes on (x_i,u_i)
 *                at non-leaf nodes and on x_j at leaves.
 *   or_factor    Sec. III-D, the "Riccati-type recursion" that precomputes
 *                Phi, Theta, D, Lambda, K, sigma, c-hat.  The paper gives no
 *                formulas; they are the dynamic-programming solution of the
 *                inner problem of Sec. III-D (the problem x(y) minimises).
 *   or_sweep     Algorithm 3 (affine, x(y)) and Algorithm 4 (homogeneous,
 *                x-hat(r)), with the children's contributions accumulated.
 *                The nodes of a stage are independent: or_set_threads(n)
 *                runs them on n OpenMP threads with each node's sums in the
 *                same order (the CPU baseline's all-core variant).
 *   or_eval      Sec. II-D and III-A: z_lambda, R_lambda, T_lambda and the
 *                forward-backward envelope, in the diagonally preconditioned
 *                dual variables of Sec. III-E when asked.
 *   or_solve     Algorithm 1 (dual MINFBE) and Algorithm 2 (NAMA), with the
 *                FBE evaluated directly (one affine sweep per trial step),
 *                the two lambda-backtracking tests of Sec. III-B, and a
 *                primal-infeasibility certificate; GPAD (the accelerated dual
 *                proximal gradient method of Sec. III-F / IV-A) as method 2.
 *
 * Readings where the paper is silent or garbled are listed in the design
 * notes; the main ones appear next to the code they affect.
 *
 * Parity pins (the tests) tie each function to the mathematics: dense KKT
 * solves of the inner problem, central differences of the dual function,
 * the dense Hessian's symmetry and spectrum, the FBE's conjugate form, the
 * secant identity of L-BFGS, a dense interior-point solution of the whole
 * problem, textbook FISTA on the dense dual (GPAD's whole trajectory), its
 * O(1/k^2) bound, the descent lemma (backtracking), scalar minimisation of
 * each soft row's prox, and an LP that proves infeasibility.  The MINFBE and
 * NAMA trajectories have no printed trace in the paper: parity unpinned for
 * those trajectories (their end point is pinned).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- problem and factor containers (mirrored by the ctypes wrapper) ---- */
typedef struct {
    int nx, nu, N, V, Vnl;
    const int *stage_ptr, *anc, *child_ptr;
    const double *prob;
    const double *A, *B, *c;          /* [V][nx][nx], [V][nx][nu], [V][nx] */
    const double *Q, *R, *S, *q, *r;  /* [Vnl]...; S, q, r may be NULL      */
    const double *P, *p;              /* [Vl][nx][nx], [Vl][nx] (p NULL ok) */
    const double *xmin, *xmax;        /* [V][nx]                             */
    const double *umin, *umax;        /* [Vnl][nu]                           */
    /* Sec. II-B constraint map: z_i = F x_i + G u_i at non-leaf nodes and
     * z_j = FN x_j at leaves, the same matrices at every node.  F == NULL
     * selects the rows (x_i, u_i) and x_j themselves, bounded by the boxes
     * above; otherwise the rows are bounded by zmin/zmax. */
    int nc, ncN;
    const double *F, *G, *FN;         /* [nc][nx], [nc][nu], [ncN][nx]      */
    const double *zmin, *zmax;        /* [m] constraint-row bounds (F set)  */
    /* Sec. II-B soft rows (NULL: every row hard): row k of node i adds
     * pi_i wgt_k psi(dist(z_k, [lo_k, hi_k])) to the cost, psi the Huber
     * function of threshold hub_k (0: the distance itself, an l1-type
     * penalty); wgt_k = +inf keeps the row a hard bound. */
    const double *wgt, *hub;          /* [m]                                 */
} or_problem;

typedef struct {
    double *Pcal;   /* [V][nx][nx]        value-function Hessians            */
    double *K;      /* [Vnl][nu][nx]      feedback gains                     */
    double *Phi;    /* [Vnl][nu][nx+nu]   u-offset from the node's dual y_i  */
    double *D;      /* [Vnl][nx+nu][nx]   q-hat term D_i^T y_i               */
    double *sigma;  /* [Vnl][nu]                                              */
    double *chat;   /* [V][nx]                                                */
    double *Theta;  /* [V][nu][nx]        per edge (indexed by the child)    */
    double *Lambda; /* [V][nx][nx]        per edge (indexed by the child)    */
} or_factors;

typedef struct {
    double lambda, eps, eps_curv;
    int mem, nu_max, max_iter, precondition;
    int method;        /* 0 MINFBE (Alg. 1), 1 NAMA (Alg. 2), 2 GPAD (Sec. III-F) */
    int backtrack;     /* 0 fixed lambda; 1 the decrease test of Sec. III-B
                          (beta = bt_param); 2 the Linesearch-1 test
                          (eps'' = bt_param)                                   */
    int div_window;    /* divergence test every div_window updates (<= 0 off) */
    double bt_param;
    double *trace;     /* NULL or [trace_iters][OR_TRACE_COLS] per update      */
    int trace_iters;
} or_opts;

/* trace row of update k: lambda, ||R(y^k)||_inf, accepted nu (-1: tau = 0),
 * nu_max, L-BFGS pairs used by the direction, then phi(w_nu) - phi(y^k) for
 * every trial nu = 0..nu_max (all evaluated in trace mode). */
#define OR_TRACE_COLS 40
#define OR_TRACE_PHI 5
#define OR_BT_MAX 50       /* halvings of lambda before giving up */

typedef struct {
    int iters, sweeps_affine, sweeps_hom, ls_trials, lbfgs_push, lbfgs_skip, status;
    double res_scaled_inf, res_unscaled_inf, phi;
    int tau_hist[32];
    int backtracks;
    double lambda_final;
} or_info;

/* Deliberate-mistake switch used only by the tests that show the pins have
 * teeth: each nonzero value plants one plausible error.  0 = correct. */
int or_mutation = 0;

/* Threads for the node-parallel loops of the factor step and the sweeps
 * (the nodes of a stage are independent; each node's summation order is the
 * same for any thread count, so the results are too).  1: plain loops. */
int or_threads = 1;
void or_set_threads(int n) { or_threads = n > 1 ? n : 1; }

/* ---------------------------- small helpers ---------------------------- */
static int dual_off(const or_problem *pb, int i)
{
    /* (x, u) layout of the sweeps: non-leaf i holds (x-rows, u-rows); leaves
     * follow with their x-rows. */
    if (i < pb->Vnl) return i * (pb->nx + pb->nu);
    return pb->Vnl * (pb->nx + pb->nu) + (i - pb->Vnl) * pb->nx;
}

int or_dual_dim(const or_problem *pb)
{
    return pb->Vnl * (pb->nx + pb->nu) + (pb->V - pb->Vnl) * pb->nx;
}

static int node_rows(const or_problem *pb, int i)
{
    return i < pb->Vnl ? pb->nx + pb->nu : pb->nx;
}

/* Constraint (dual) layout of Sec. II-C: the rows z_i of node i, non-leaf
 * nodes first.  Without a constraint map it is the (x, u) layout. */
static int con_rows(const or_problem *pb, int i)
{
    if (!pb->F) return node_rows(pb, i);
    return i < pb->Vnl ? pb->nc : pb->ncN;
}

static int con_off(const or_problem *pb, int i)
{
    if (!pb->F) return dual_off(pb, i);
    if (i < pb->Vnl) return i * pb->nc;
    return pb->Vnl * pb->nc + (i - pb->Vnl) * pb->ncN;
}

int or_con_dim(const or_problem *pb)
{
    if (!pb->F) return or_dual_dim(pb);
    return pb->Vnl * pb->nc + (pb->V - pb->Vnl) * pb->ncN;
}

/* Cholesky factor L (lower) of the n x n SPD matrix M; returns 0 or -1. */
static int cholesky(int n, const double *M, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = M[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return -1;
        L[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = M[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    return 0;
}

/* Inverse of L L^T, column by column through two triangular solves. */
static void chol_inverse(int n, const double *L, double *Minv)
{
    double *col = malloc(sizeof(double) * n);
    for (int e = 0; e < n; ++e) {
        for (int i = 0; i < n; ++i) {           /* L w = e_e */
            double s = (i == e) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {      /* L^T v = w */
            double s = col[i];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int i = 0; i < n; ++i) Minv[i * n + e] = col[i];
    }
    free(col);
}

/* ------------------------------ factor step ----------------------------- */
/*
 * Dynamic programming on the inner problem (the problem whose minimiser is
 * x(y)).  With costs written without a 1/2 (Sec. II-B), the value function of
 * the subtree rooted at node i is  x' (Pcal_i / 2) x + (linear term) x.
 *
 *   leaves:      Pcal_j = 2 pi_j P_j,            chat_j = Pcal_j c_j + pi_j p_j
 *   non-leaf i:  Rt = 2 pi_i R_i + sum_j B_j' Pcal_j B_j          (Cholesky)
 *                St = 2 pi_i S_i + sum_j B_j' Pcal_j A_j
 *                K_i = -Rt^{-1} St
 *                Pcal_i = 2 pi_i Q_i + sum_j A_j' Pcal_j A_j + K_i' St
 *                Lambda_j = A_j + B_j K_i,   Theta_j = -Rt^{-1} B_j'
 *                Phi_i = [0, -Rt^{-1}],      D_i = [I; K_i]
 *                sigma_i = -Rt^{-1} pi_i r_i
 *                chat_i = Pcal_i c_i + pi_i q_i + K_i' pi_i r_i   (c_0 = 0)
 * Returns 0, or -3 when some Rt is not positive definite.
 */
/* The step for non-leaf node i (its children's Pcal are final).  Returns 0,
 * or -3 when Rt is not positive definite. */
static int factor_node(const or_problem *pb, or_factors *f, int i)
{
    const int nx = pb->nx, nu = pb->nu;
    const int nxu = nx + nu;
    double *Rt = malloc(sizeof(double) * nu * nu);
    double *Lc = malloc(sizeof(double) * nu * nu);
    double *Ri = malloc(sizeof(double) * nu * nu);
    double *St = malloc(sizeof(double) * nu * nx);
    double *PB = malloc(sizeof(double) * nx * nu);
    double *PA = malloc(sizeof(double) * nx * nx);
    int rc = 0;
    const double pi = pb->prob[i];
    /* Rt, St */
    for (int a = 0; a < nu; ++a)
        for (int b = 0; b < nu; ++b)
            Rt[a * nu + b] = 2.0 * pi * pb->R[(size_t)i * nu * nu + a * nu + b];
    for (int a = 0; a < nu; ++a)
        for (int b = 0; b < nx; ++b)
            St[a * nx + b] = pb->S ? 2.0 * pi * pb->S[(size_t)i * nu * nx + a * nx + b] : 0.0;
    double *Pi = f->Pcal + (size_t)i * nx * nx;
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < nx; ++b)
            Pi[a * nx + b] = 2.0 * pi * pb->Q[(size_t)i * nx * nx + a * nx + b];
    for (int j = pb->child_ptr[i]; j < pb->child_ptr[i + 1]; ++j) {
        const double *Aj = pb->A + (size_t)j * nx * nx;
        const double *Bj = pb->B + (size_t)j * nx * nu;
        const double *Pj = f->Pcal + (size_t)j * nx * nx;
        for (int a = 0; a < nx; ++a) {              /* PB = Pj Bj, PA = Pj Aj */
            for (int b = 0; b < nu; ++b) {
                double s = 0.0;
                for (int k = 0; k < nx; ++k) s += Pj[a * nx + k] * Bj[k * nu + b];
                PB[a * nu + b] = s;
            }
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int k = 0; k < nx; ++k) s += Pj[a * nx + k] * Aj[k * nx + b];
                PA[a * nx + b] = s;
            }
        }
        for (int a = 0; a < nu; ++a) {
            for (int b = 0; b < nu; ++b) {          /* Bj' Pj Bj */
                double s = 0.0;
                for (int k = 0; k < nx; ++k) s += Bj[k * nu + a] * PB[k * nu + b];
                Rt[a * nu + b] += s;
            }
            for (int b = 0; b < nx; ++b) {          /* Bj' Pj Aj */
                double s = 0.0;
                for (int k = 0; k < nx; ++k) s += Bj[k * nu + a] * PA[k * nx + b];
                St[a * nx + b] += s;
            }
        }
        for (int a = 0; a < nx; ++a)                /* Aj' Pj Aj */
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int k = 0; k < nx; ++k) s += Aj[k * nx + a] * PA[k * nx + b];
                Pi[a * nx + b] += s;
            }
    }
    if (cholesky(nu, Rt, Lc) != 0) { rc = -3; goto done; }
    chol_inverse(nu, Lc, Ri);
    double *Ki = f->K + (size_t)i * nu * nx;
    for (int a = 0; a < nu; ++a)
        for (int b = 0; b < nx; ++b) {
            double s = 0.0;
            for (int k = 0; k < nu; ++k) s += Ri[a * nu + k] * St[k * nx + b];
            Ki[a * nx + b] = -s;
        }
    if (or_mutation != 1) {
        for (int a = 0; a < nx; ++a)                /* + K' St */
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int k = 0; k < nu; ++k) s += Ki[k * nx + a] * St[k * nx + b];
                Pi[a * nx + b] += s;
            }
    }
    for (int j = pb->child_ptr[i]; j < pb->child_ptr[i + 1]; ++j) {
        const double *Aj = pb->A + (size_t)j * nx * nx;
        const double *Bj = pb->B + (size_t)j * nx * nu;
        double *Lj = f->Lambda + (size_t)j * nx * nx;
        double *Tj = f->Theta + (size_t)j * nu * nx;
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < nx; ++b) {
                double s = Aj[a * nx + b];
                for (int k = 0; k < nu; ++k) s += Bj[a * nu + k] * Ki[k * nx + b];
                Lj[a * nx + b] = s;
            }
        for (int a = 0; a < nu; ++a)
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int k = 0; k < nu; ++k) s += Ri[a * nu + k] * Bj[b * nu + k];
                Tj[a * nx + b] = -s;
            }
    }
    double *Ph = f->Phi + (size_t)i * nu * nxu;
    for (int a = 0; a < nu; ++a)
        for (int b = 0; b < nxu; ++b)
            Ph[a * nxu + b] = (b < nx) ? 0.0 : -Ri[a * nu + (b - nx)];
    double *Di = f->D + (size_t)i * nxu * nx;
    for (int a = 0; a < nxu; ++a)
        for (int b = 0; b < nx; ++b)
            Di[a * nx + b] = (a < nx) ? (a == b ? 1.0 : 0.0) : Ki[(a - nx) * nx + b];
    double *sg = f->sigma + (size_t)i * nu;
    for (int a = 0; a < nu; ++a) {
        double s = 0.0;
        if (pb->r)
            for (int k = 0; k < nu; ++k) s += Ri[a * nu + k] * pi * pb->r[(size_t)i * nu + k];
        sg[a] = -s;
    }
    double *ch = f->chat + (size_t)i * nx;
    for (int a = 0; a < nx; ++a) {
        double s = 0.0;
        if (i > 0)
            for (int k = 0; k < nx; ++k) s += Pi[a * nx + k] * pb->c[(size_t)i * nx + k];
        if (pb->q) s += pi * pb->q[(size_t)i * nx + a];
        if (pb->r)
            for (int k = 0; k < nu; ++k) s += Ki[k * nx + a] * pi * pb->r[(size_t)i * nu + k];
        ch[a] = s;
    }
done:
    free(Rt); free(Lc); free(Ri); free(St); free(PB); free(PA);
    return rc;
}

/*
 * Dynamic programming on the inner problem (the problem whose minimiser is
 * x(y)).  With costs written without a 1/2 (Sec. II-B), the value function of
 * the subtree rooted at node i is  x' (Pcal_i / 2) x + (linear term) x.
 *
 *   leaves:      Pcal_j = 2 pi_j P_j,            chat_j = Pcal_j c_j + pi_j p_j
 *   non-leaf i:  Rt = 2 pi_i R_i + sum_j B_j' Pcal_j B_j          (Cholesky)
 *                St = 2 pi_i S_i + sum_j B_j' Pcal_j A_j
 *                K_i = -Rt^{-1} St
 *                Pcal_i = 2 pi_i Q_i + sum_j A_j' Pcal_j A_j + K_i' St
 *                Lambda_j = A_j + B_j K_i,   Theta_j = -Rt^{-1} B_j'
 *                Phi_i = [0, -Rt^{-1}],      D_i = [I; K_i]
 *                sigma_i = -Rt^{-1} pi_i r_i
 *                chat_i = Pcal_i c_i + pi_i q_i + K_i' pi_i r_i   (c_0 = 0)
 * The nodes of a stage are independent (or_threads > 1 spreads them over
 * threads; every node's arithmetic is the same, so are the results).
 * Returns 0, or -3 when some Rt is not positive definite.
 */
int or_factor(const or_problem *pb, or_factors *f)
{
    const int nx = pb->nx, N = pb->N;
    int rc = 0;

    /* leaves */
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(static)
    for (int j = pb->Vnl; j < pb->V; ++j) {
        const int l = j - pb->Vnl;
        const double pj = pb->prob[j];
        double *Pc = f->Pcal + (size_t)j * nx * nx;
        for (int a = 0; a < nx * nx; ++a) Pc[a] = 2.0 * pj * pb->P[(size_t)l * nx * nx + a];
        double *ch = f->chat + (size_t)j * nx;
        for (int a = 0; a < nx; ++a) {
            double s = 0.0;
            for (int b = 0; b < nx; ++b) s += Pc[a * nx + b] * pb->c[(size_t)j * nx + b];
            if (pb->p) s += pj * pb->p[(size_t)l * nx + a];
            ch[a] = s;
        }
    }

    for (int t = N - 1; t >= 0 && rc == 0; --t) {
        int bad = 0;
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(dynamic, 8) reduction(| : bad)
        for (int i = pb->stage_ptr[t]; i < pb->stage_ptr[t + 1]; ++i)
            bad |= factor_node(pb, f, i) != 0;
        if (bad) rc = -3;
    }
    return rc;
}

/* ------------------------- Algorithms 3 and 4 --------------------------- */
/*
 * y is the dual vector in the paper's (unscaled) variables, laid out node by
 * node.  homogeneous = 0: Algorithm 3, x(y) with x_0 = p.  homogeneous = 1:
 * Algorithm 4, the linear part x-hat(y) (no sigma, c-hat, c, and x_0 = 0).
 * Outputs x [V][nx] (x_0 included) and u [Vnl][nu].
 */
void or_sweep(const or_problem *pb, const or_factors *f, const double *y,
              const double *p, int homogeneous, double *x, double *u)
{
    const int nx = pb->nx, nu = pb->nu, nxu = nx + nu, N = pb->N;
    const int aff = !homogeneous;
    double *qh = malloc(sizeof(double) * (size_t)pb->V * nx);

    /* leaves: q-hat_j = y_j (+ c-hat_j) */
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(static)
    for (int j = pb->Vnl; j < pb->V; ++j) {
        const double *yj = y + dual_off(pb, j);
        for (int a = 0; a < nx; ++a)
            qh[(size_t)j * nx + a] = yj[a] + (aff ? f->chat[(size_t)j * nx + a] : 0.0);
    }
    /* non-leaves: u_i = Phi_i y_i (+ sigma_i), q-hat_i = D_i' y_i (+ c-hat_i) */
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(static)
    for (int i = 0; i < pb->Vnl; ++i) {
        const double *yi = y + dual_off(pb, i);
        const double *Ph = f->Phi + (size_t)i * nu * nxu;
        const double *Di = f->D + (size_t)i * nxu * nx;
        for (int a = 0; a < nu; ++a) {
            double s = aff ? f->sigma[(size_t)i * nu + a] : 0.0;
            for (int b = 0; b < nxu; ++b) s += Ph[a * nxu + b] * yi[b];
            u[(size_t)i * nu + a] = s;
        }
        for (int a = 0; a < nx; ++a) {
            double s = aff ? f->chat[(size_t)i * nx + a] : 0.0;
            for (int b = 0; b < nxu; ++b) s += Di[b * nx + a] * yi[b];
            qh[(size_t)i * nx + a] = s;
        }
    }
    /* backward over stages: accumulate the children's contributions */
    for (int t = N - 1; t >= 0; --t) {
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(static)
        for (int i = pb->stage_ptr[t]; i < pb->stage_ptr[t + 1]; ++i) {
            double *ui = u + (size_t)i * nu;
            double *qi = qh + (size_t)i * nx;
            if (or_mutation == 2) {   /* overwrite instead of accumulate */
                for (int a = 0; a < nu; ++a) ui[a] = 0.0;
                for (int a = 0; a < nx; ++a) qi[a] = 0.0;
            }
            for (int j = pb->child_ptr[i]; j < pb->child_ptr[i + 1]; ++j) {
                const double *Tj = f->Theta + (size_t)j * nu * nx;
                const double *Lj = f->Lambda + (size_t)j * nx * nx;
                const double *qj = qh + (size_t)j * nx;
                for (int a = 0; a < nu; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < nx; ++b) s += Tj[a * nx + b] * qj[b];
                    ui[a] += s;
                }
                for (int a = 0; a < nx; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < nx; ++b)
                        s += (or_mutation == 3 ? Lj[a * nx + b] : Lj[b * nx + a]) * qj[b];
                    qi[a] += s;
                }
            }
        }
    }
    /* forward over stages */
    for (int a = 0; a < nx; ++a) x[a] = aff ? p[a] : 0.0;
    for (int t = 0; t < N; ++t) {
#pragma omp parallel for num_threads(or_threads) if (or_threads > 1) schedule(static)
        for (int i = pb->stage_ptr[t]; i < pb->stage_ptr[t + 1]; ++i) {
            const double *Ki = f->K + (size_t)i * nu * nx;
            const double *xi = x + (size_t)i * nx;
            double *ui = u + (size_t)i * nu;
            for (int a = 0; a < nu; ++a) {
                double s = ui[a];
                for (int b = 0; b < nx; ++b) s += Ki[a * nx + b] * xi[b];
                ui[a] = s;
            }
            for (int j = pb->child_ptr[i]; j < pb->child_ptr[i + 1]; ++j) {
                const double *Aj = pb->A + (size_t)j * nx * nx;
                const double *Bj = pb->B + (size_t)j * nx * nu;
                double *xj = x + (size_t)j * nx;
                for (int a = 0; a < nx; ++a) {
                    double s = (aff && or_mutation != 4) ? pb->c[(size_t)j * nx + a] : 0.0;
                    for (int b = 0; b < nx; ++b) s += Aj[a * nx + b] * xi[b];
                    for (int b = 0; b < nu; ++b) s += Bj[a * nu + b] * ui[b];
                    xj[a] = s;
                }
            }
        }
    }
    free(qh);
}

/* f(x): the probability-weighted quadratic cost of Sec. II-B (x_0 included). */
double or_cost(const or_problem *pb, const double *x, const double *u)
{
    const int nx = pb->nx, nu = pb->nu;
    double tot = 0.0;
    for (int i = 0; i < pb->Vnl; ++i) {
        const double *xi = x + (size_t)i * nx, *ui = u + (size_t)i * nu;
        const double *Q = pb->Q + (size_t)i * nx * nx, *R = pb->R + (size_t)i * nu * nu;
        double s = 0.0;
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < nx; ++b) s += xi[a] * Q[a * nx + b] * xi[b];
        for (int a = 0; a < nu; ++a)
            for (int b = 0; b < nu; ++b) s += ui[a] * R[a * nu + b] * ui[b];
        if (pb->S) {
            const double *S = pb->S + (size_t)i * nu * nx;
            for (int a = 0; a < nu; ++a)
                for (int b = 0; b < nx; ++b) s += 2.0 * ui[a] * S[a * nx + b] * xi[b];
        }
        if (pb->q) for (int a = 0; a < nx; ++a) s += pb->q[(size_t)i * nx + a] * xi[a];
        if (pb->r) for (int a = 0; a < nu; ++a) s += pb->r[(size_t)i * nu + a] * ui[a];
        tot += pb->prob[i] * s;
    }
    for (int j = pb->Vnl; j < pb->V; ++j) {
        const int l = j - pb->Vnl;
        const double *xj = x + (size_t)j * nx, *P = pb->P + (size_t)l * nx * nx;
        double s = 0.0;
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < nx; ++b) s += xj[a] * P[a * nx + b] * xj[b];
        if (pb->p) for (int a = 0; a < nx; ++a) s += pb->p[(size_t)l * nx + a] * xj[a];
        tot += pb->prob[j] * s;
    }
    return tot;
}

/* H x: the stacked (x_i, u_i) of non-leaf nodes, then x_j of leaves. */
void or_Hx(const or_problem *pb, const double *x, const double *u, double *hx)
{
    for (int i = 0; i < pb->V; ++i) {
        double *h = hx + dual_off(pb, i);
        for (int a = 0; a < pb->nx; ++a) h[a] = x[(size_t)i * pb->nx + a];
        if (i < pb->Vnl)
            for (int a = 0; a < pb->nu; ++a) h[pb->nx + a] = u[(size_t)i * pb->nu + a];
    }
}

/* The constraint map of Sec. II-B: z = H(x, u) in the constraint layout
 * (identity rows without F). */
void or_apply_H(const or_problem *pb, const double *x, const double *u, double *z)
{
    const int nx = pb->nx, nu = pb->nu;
    if (!pb->F) { or_Hx(pb, x, u, z); return; }
    for (int i = 0; i < pb->V; ++i) {
        double *zi = z + con_off(pb, i);
        const double *xi = x + (size_t)i * nx;
        if (i < pb->Vnl) {
            const double *ui = u + (size_t)i * nu;
            for (int a = 0; a < pb->nc; ++a) {
                double s = 0.0;
                for (int b = 0; b < nx; ++b) s += pb->F[a * nx + b] * xi[b];
                for (int b = 0; b < nu; ++b) s += pb->G[a * nu + b] * ui[b];
                zi[a] = s;
            }
        } else {
            for (int a = 0; a < pb->ncN; ++a) {
                double s = 0.0;
                for (int b = 0; b < nx; ++b) s += pb->FN[a * nx + b] * xi[b];
                zi[a] = s;
            }
        }
    }
}

/* Its adjoint: a constraint-layout dual y -> H' y in the (x, u) layout the
 * sweeps take (the term <y, Hx> of the inner problem is <H'y, (x, u)>). */
void or_apply_Ht(const or_problem *pb, const double *y, double *v)
{
    const int nx = pb->nx, nu = pb->nu;
    if (!pb->F) { memcpy(v, y, sizeof(double) * or_dual_dim(pb)); return; }
    for (int i = 0; i < pb->V; ++i) {
        const double *yi = y + con_off(pb, i);
        double *vi = v + dual_off(pb, i);
        if (i < pb->Vnl) {
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int a = 0; a < pb->nc; ++a) s += pb->F[a * nx + b] * yi[a];
                vi[b] = s;
            }
            for (int b = 0; b < nu; ++b) {
                double s = 0.0;
                for (int a = 0; a < pb->nc; ++a) s += pb->G[a * nu + b] * yi[a];
                vi[nx + b] = s;
            }
        } else {
            for (int b = 0; b < nx; ++b) {
                double s = 0.0;
                for (int a = 0; a < pb->ncN; ++a) s += pb->FN[a * nx + b] * yi[a];
                vi[b] = s;
            }
        }
    }
}

/* Per-row lower/upper bound in the constraint layout (unscaled). */
static void box_rows(const or_problem *pb, double *lo, double *hi)
{
    if (pb->F) {
        const int m = or_con_dim(pb);
        memcpy(lo, pb->zmin, sizeof(double) * m);
        memcpy(hi, pb->zmax, sizeof(double) * m);
        return;
    }
    for (int i = 0; i < pb->V; ++i) {
        const int o = dual_off(pb, i);
        for (int a = 0; a < pb->nx; ++a) {
            lo[o + a] = pb->xmin[(size_t)i * pb->nx + a];
            hi[o + a] = pb->xmax[(size_t)i * pb->nx + a];
        }
        if (i < pb->Vnl)
            for (int a = 0; a < pb->nu; ++a) {
                lo[o + pb->nx + a] = pb->umin[(size_t)i * pb->nu + a];
                hi[o + pb->nx + a] = pb->umax[(size_t)i * pb->nu + a];
            }
    }
}

/* Per-row scale of the preconditioning of Sec. III-E: sqrt(pi_i) for every row
 * of node i (1 when not preconditioning); pr receives pi_i per row. */
static void row_scale(const or_problem *pb, int precondition, double *sc, double *pr)
{
    for (int i = 0; i < pb->V; ++i) {
        double s = 1.0;
        if (precondition) s = (or_mutation == 8) ? pb->prob[i] : sqrt(pb->prob[i]);
        const int o = con_off(pb, i);
        for (int a = 0; a < con_rows(pb, i); ++a) {
            sc[o + a] = s;
            pr[o + a] = pb->prob[i];
        }
    }
}

/* ------------------------------ row penalties --------------------------- */
/* Huber function of threshold d (d = 0: the identity) at a distance t >= 0. */
static double huber(double t, double d)
{
    if (d > 0.0 && t <= d) return t * t / (2.0 * d);
    return t - 0.5 * d;
}

/*
 * One row of the prox of Sec. II-D, z = prox_{g/lambda}(v): minimise
 * g(z) + (lambda/2)(z - v)^2 for g(z) = w psi_d(dist(z, [lo, hi])), with
 * w = +inf meaning the indicator of [lo, hi] (projection).  Outside the
 * interval the distance t = v - hi (or lo - v) shrinks to the minimiser s of
 * w psi_d(s) + (lambda/2)(s - t)^2: s = t/(1 + w/(lambda d)) on the quadratic
 * part of psi (s <= d), else s = t - w/lambda, never below 0.  *gz = g(z).
 */
static double row_prox(double v, double lo, double hi, double w, double d, double lam, double *gz)
{
    *gz = 0.0;
    if (!(w < INFINITY)) return v < lo ? lo : (v > hi ? hi : v);
    double t, side;
    if (v > hi) { t = v - hi; side = 1.0; }
    else if (v < lo) { t = lo - v; side = -1.0; }
    else return v;
    const double wl = w / lam;
    double sh;
    if (d > 0.0 && t <= d + wl) sh = t / (1.0 + wl / ((or_mutation == 10) ? 1.0 : d));
    else sh = t - wl > 0.0 ? t - wl : 0.0;
    *gz = w * huber(sh, d);
    return side > 0.0 ? hi + sh : lo - sh;
}

/* ------------------------- evaluation at a dual point ------------------- */
typedef struct {
    const or_problem *pb;
    const or_factors *f;
    const double *p;       /* x0 */
    double lambda;
    int m, mxu, precondition;
    double *sc, *pr, *lo, *hi;  /* per row: scale, pi, unscaled bounds */
    double *ytmp, *yxu, *x, *u, *hx;
    int sweeps_affine, sweeps_hom;
} or_ctx;

static void ctx_init(or_ctx *c, const or_problem *pb, const or_factors *f,
                     const double *p, double lambda, int precondition)
{
    c->pb = pb; c->f = f; c->p = p; c->lambda = lambda;
    c->precondition = precondition;
    c->m = or_con_dim(pb);
    c->mxu = or_dual_dim(pb);
    c->sc = malloc(sizeof(double) * c->m);
    c->pr = malloc(sizeof(double) * c->m);
    c->lo = malloc(sizeof(double) * c->m);
    c->hi = malloc(sizeof(double) * c->m);
    c->ytmp = malloc(sizeof(double) * c->m);
    c->hx = malloc(sizeof(double) * c->m);
    c->yxu = malloc(sizeof(double) * c->mxu);
    c->x = malloc(sizeof(double) * (size_t)pb->V * pb->nx);
    c->u = malloc(sizeof(double) * (size_t)pb->Vnl * pb->nu);
    row_scale(pb, precondition, c->sc, c->pr);
    box_rows(pb, c->lo, c->hi);
    c->sweeps_affine = c->sweeps_hom = 0;
}

static void ctx_free(or_ctx *c)
{
    free(c->sc); free(c->pr); free(c->lo); free(c->hi); free(c->ytmp); free(c->hx);
    free(c->yxu); free(c->x); free(c->u);
}

/* Scaled penalty of row k: in the variables zb = s z of Sec. III-E the row
 * function pi w psi_d(dist(zb / s, [lo, hi])) equals w' psi_d'(dist(zb,
 * [s lo, s hi])) with w' = pi w / s and d' = s d. */
static void row_params(const or_ctx *c, int k, double *lo, double *hi, double *w, double *d)
{
    const double s = c->sc[k];
    *lo = s * c->lo[k];
    *hi = s * c->hi[k];
    *w = INFINITY;
    *d = 0.0;
    if (c->pb->wgt && c->pb->wgt[k] < INFINITY) {
        *w = c->pr[k] * c->pb->wgt[k] / s;
        *d = s * c->pb->hub[k];
    }
}

/*
 * At the (scaled) dual point yb: x = x(H'(sc*yb)) (Algorithm 3 on the
 * (x, u)-layout dual), Hbx = sc * H x, z = prox_{g/lambda}(yb/lambda + Hbx),
 * R = z - Hbx (Sec. II-D), and the FBE
 *   phi = -f(x) + <yb, R> - (lambda/2) ||R||^2 - g(z),
 * which equals f-hat + g*(T) - lambda <grad f-hat, R> + (lambda/2)||R||^2 of
 * Sec. III-A because g*(T) = <T, z> - g(z) (Fenchel-Young equality at the
 * prox point, T = lambda (v - z) being a subgradient of g at z).  Outputs Hbx,
 * R (each may be NULL), f-hat(yb) = -f(x) - <yb, Hbx> and g(z) (NULL ok);
 * returns phi.
 */
static double ctx_eval(or_ctx *c, const double *yb, double *Hbx, double *R, double *fhat, double *gsum)
{
    const int m = c->m;
    for (int k = 0; k < m; ++k) c->ytmp[k] = c->sc[k] * yb[k];
    or_apply_Ht(c->pb, c->ytmp, c->yxu);
    or_sweep(c->pb, c->f, c->yxu, c->p, 0, c->x, c->u);
    c->sweeps_affine++;
    or_apply_H(c->pb, c->x, c->u, c->hx);
    double inner = 0.0, nrm2 = 0.0, gs = 0.0, yh = 0.0;
    for (int k = 0; k < m; ++k) {
        const double h = c->sc[k] * c->hx[k];
        const double v = yb[k] / c->lambda + h;
        double lo, hi, w, d, gz;
        row_params(c, k, &lo, &hi, &w, &d);
        const double z = row_prox(v, lo, hi, w, d, c->lambda, &gz);
        const double r = z - h;
        if (Hbx) Hbx[k] = h;
        if (R) R[k] = r;
        inner += yb[k] * r;
        nrm2 += r * r;
        gs += gz;
        yh += yb[k] * h;
    }
    const double fx = or_cost(c->pb, c->x, c->u);
    if (fhat) *fhat = -fx - yh;
    if (gsum) *gsum = gs;
    if (or_mutation == 6) return -fx + inner + 0.5 * c->lambda * nrm2 - gs;
    return -fx + inner - 0.5 * c->lambda * nrm2 - gs;
}

/* Hb x-hat(H'(sc * v)): the linear part (Algorithm 4), scaled back; the
 * Hessian of the (scaled) dual function applied to v is minus this. */
static void ctx_hom(or_ctx *c, const double *v, double *out)
{
    for (int k = 0; k < c->m; ++k) c->ytmp[k] = c->sc[k] * v[k];
    or_apply_Ht(c->pb, c->ytmp, c->yxu);
    or_sweep(c->pb, c->f, c->yxu, c->p, 1, c->x, c->u);
    c->sweeps_hom++;
    or_apply_H(c->pb, c->x, c->u, c->hx);
    for (int k = 0; k < c->m; ++k) out[k] = c->sc[k] * c->hx[k];
}

/*
 * Exported evaluation: given a (scaled) dual point, return x, u (unscaled
 * primal, Algorithm 3), Hbx, z, R, T = y - lambda R, and grad_phi =
 * (I - lambda Hess f-hat) R = R + lambda Hb x-hat(sc R) (Sec. III-A).
 * extra[0] = f-hat(yb), extra[1] = g(z).  Any output pointer may be NULL.
 * Returns phi.
 */
double or_eval(const or_problem *pb, const or_factors *f, const double *p,
               double lambda, int precondition, const double *yb,
               double *x, double *u, double *Hbx, double *z, double *R,
               double *T, double *grad_phi, double *extra)
{
    or_ctx c;
    ctx_init(&c, pb, f, p, lambda, precondition);
    const int m = c.m;
    double *h = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    double fh, gs;
    const double phi = ctx_eval(&c, yb, h, r, &fh, &gs);
    if (extra) { extra[0] = fh; extra[1] = gs; }
    if (x) memcpy(x, c.x, sizeof(double) * (size_t)pb->V * pb->nx);
    if (u) memcpy(u, c.u, sizeof(double) * (size_t)pb->Vnl * pb->nu);
    for (int k = 0; k < m; ++k) {
        if (Hbx) Hbx[k] = h[k];
        if (z) z[k] = r[k] + h[k];
        if (R) R[k] = r[k];
        if (T) T[k] = (or_mutation == 5) ? yb[k] + lambda * r[k] : yb[k] - lambda * r[k];
    }
    if (grad_phi) {
        double *hv = malloc(sizeof(double) * m);
        ctx_hom(&c, r, hv);
        for (int k = 0; k < m; ++k) grad_phi[k] = r[k] + lambda * hv[k];
        free(hv);
    }
    free(h); free(r);
    ctx_free(&c);
    return phi;
}

/* v -> Hb x-hat(H'(sc v)), exported for the Hessian pins (the Hessian of the
 * scaled dual function is minus this map). */
void or_hess_neg(const or_problem *pb, const or_factors *f, int precondition,
                 const double *v, double *out)
{
    or_ctx c;
    ctx_init(&c, pb, f, NULL, 1.0, precondition);
    ctx_hom(&c, v, out);
    ctx_free(&c);
}

/* Largest eigenvalue L of the (scaled) dual Hessian, which is positive
 * semidefinite, by power iteration on v -> Hess(v) = -Hb x-hat(sc v), started
 * from v0 (length m). */
double or_power_iteration(const or_problem *pb, const or_factors *f,
                          int precondition, int iters, const double *v0)
{
    or_ctx c;
    ctx_init(&c, pb, f, NULL, 1.0, precondition);
    const int m = c.m;
    double *v = malloc(sizeof(double) * m), *w = malloc(sizeof(double) * m);
    double nrm = 0.0, L = 0.0;
    for (int k = 0; k < m; ++k) { v[k] = v0[k]; nrm += v[k] * v[k]; }
    nrm = sqrt(nrm);
    for (int k = 0; k < m; ++k) v[k] /= nrm;
    for (int it = 0; it < iters; ++it) {
        ctx_hom(&c, v, w);
        for (int k = 0; k < m; ++k) w[k] = -w[k];
        double ray = 0.0, n2 = 0.0;
        for (int k = 0; k < m; ++k) { ray += v[k] * w[k]; n2 += w[k] * w[k]; }
        L = ray;
        n2 = sqrt(n2);
        if (!(n2 > 0.0)) break;
        for (int k = 0; k < m; ++k) v[k] = w[k] / n2;
    }
    free(v); free(w);
    ctx_free(&c);
    return L;
}

/* ------------------------------- L-BFGS --------------------------------- */
/*
 * Two-loop recursion: d = -B g for the pairs (s_k, q_k), k = 0..cnt-1 listed
 * oldest first, with initial matrix gamma I, gamma = <s,q>/<q,q> of the
 * newest pair (I when the buffer is empty).
 */
void or_lbfgs_direction(int m, int cnt, const double *const *s, const double *const *q,
                        const double *g, double *d)
{
    double *alpha = malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
    double *rho = malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
    double *w = malloc(sizeof(double) * m);
    for (int k = 0; k < m; ++k) w[k] = g[k];
    for (int i = 0; i < cnt; ++i) {
        double sq = 0.0;
        for (int k = 0; k < m; ++k) sq += s[i][k] * q[i][k];
        rho[i] = 1.0 / sq;
    }
    const int fwd = (or_mutation == 7);
    for (int ii = 0; ii < cnt; ++ii) {
        const int i = fwd ? ii : cnt - 1 - ii;          /* newest first */
        double a = 0.0;
        for (int k = 0; k < m; ++k) a += s[i][k] * w[k];
        alpha[i] = rho[i] * a;
        for (int k = 0; k < m; ++k) w[k] -= alpha[i] * q[i][k];
    }
    double gamma = 1.0;
    if (cnt > 0) {
        double sq = 0.0, qq = 0.0;
        for (int k = 0; k < m; ++k) {
            sq += s[cnt - 1][k] * q[cnt - 1][k];
            qq += q[cnt - 1][k] * q[cnt - 1][k];
        }
        gamma = sq / qq;
    }
    for (int k = 0; k < m; ++k) w[k] *= gamma;
    for (int ii = 0; ii < cnt; ++ii) {
        const int i = fwd ? cnt - 1 - ii : ii;          /* oldest first */
        double b = 0.0;
        for (int k = 0; k < m; ++k) b += q[i][k] * w[k];
        b *= rho[i];
        for (int k = 0; k < m; ++k) w[k] += (alpha[i] - b) * s[i][k];
    }
    for (int k = 0; k < m; ++k) d[k] = -w[k];
    free(alpha); free(rho); free(w);
}

typedef struct {
    int mem, cnt, head;    /* ring buffer: head = slot of the next push */
    int m;
    double **s, **q;
    const double **so, **qo;  /* oldest-first views */
} or_lbfgs;

static void lb_init(or_lbfgs *b, int mem, int m)
{
    b->mem = mem; b->cnt = 0; b->head = 0; b->m = m;
    b->s = malloc(sizeof(double *) * mem);
    b->q = malloc(sizeof(double *) * mem);
    b->so = malloc(sizeof(double *) * mem);
    b->qo = malloc(sizeof(double *) * mem);
    for (int i = 0; i < mem; ++i) {
        b->s[i] = malloc(sizeof(double) * m);
        b->q[i] = malloc(sizeof(double) * m);
    }
}

static void lb_free(or_lbfgs *b)
{
    for (int i = 0; i < b->mem; ++i) { free(b->s[i]); free(b->q[i]); }
    free(b->s); free(b->q); free(b->so); free(b->qo);
}

static void lb_push(or_lbfgs *b, const double *s, const double *q)
{
    memcpy(b->s[b->head], s, sizeof(double) * b->m);
    memcpy(b->q[b->head], q, sizeof(double) * b->m);
    b->head = (b->head + 1) % b->mem;
    if (b->cnt < b->mem) b->cnt++;
}

static void lb_direction(or_lbfgs *b, const double *g, double *d)
{
    for (int i = 0; i < b->cnt; ++i) {
        const int slot = (b->head - b->cnt + i + b->mem) % b->mem;
        b->so[i] = b->s[slot];
        b->qo[i] = b->q[slot];
    }
    or_lbfgs_direction(b->m, b->cnt, (const double *const *)b->so,
                       (const double *const *)b->qo, g, d);
}

static void lb_clear(or_lbfgs *b) { b->cnt = 0; b->head = 0; }

/* --------------------------- Algorithms 1 and 2 -------------------------- */
static double dot(int m, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += a[k] * b[k];
    return s;
}

/* max |a_k|; NaN when any entry is NaN (fmax alone would skip it, and an
 * all-NaN residual would read as converged) */
static double inf_norm(int m, const double *a)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
        if (isnan(a[k]) && or_mutation != 12) return NAN;
        s = fmax(s, fabs(a[k]));
    }
    return s;
}

/*
 * Divergence test.  The problem is assumed feasible (Sec. II-C); when it is
 * not, the dual function F = f-hat + g* is unbounded below and the iterates
 * run off along a direction d with (i) H'd orthogonal to the directions of
 * the dynamics, so that f-hat is affine along d (its Hessian, minus the
 * Algorithm-4 map, annihilates d), and (ii) F decreasing linearly along d:
 *   sigma_Y(d) - <d, H x(y)> < 0,
 * sigma_Y the support function of the (scaled) boxes; such a d certifies
 * that no x satisfies the dynamics and the boxes (Farkas).  Every div_window
 * updates the increment d = y^k - y^{k - div_window} is tested:
 *   lambda ||Hb x-hat(sc d)||_inf <= eps_div ||d||_inf  and
 *   sigma(d) - <d, Hb x(y^k)> <= -eps_obj ||d||_inf ||R(y^k)||_inf,
 * with eps_div = 1e-3 and eps_obj = 1e-4; rows with an infinite bound (and soft rows, whose g*
 * has a bounded domain) must carry no part of d (|d_k| <= 1e-9 ||d||_inf).
 * Divergence is declared when two consecutive windows pass: along a true
 * divergence direction every later window passes too (for MINFBE and NAMA
 * the first ratio falls to rounding level, for GPAD it keeps falling), while
 * the path of a feasible problem out of its start point can pass once.  For
 * GPAD the first condition uses 1e-4 instead of eps_div: its momentum can
 * carry a feasible, slowly converging problem along a nearly null direction
 * for many windows (ratios of 2e-4 to 6e-4 were measured), while on
 * infeasible problems its ratio falls below 1e-4 within a few hundred
 * updates.  The second bound is
 * the looser one because the null-space ratio is what separates the two
 * cases: on infeasible problems whose iterates run along a null direction
 * (first ratio 1e-9 and below) the objective ratio settles between 5e-4
 * and 9e-4 in these norms, while the feasible paths that passed once had
 * first ratios near 5e-4 and objective ratios beyond 1e-3.
 * Returns 1 on divergence.  One Algorithm-4 sweep per test.
 */
#define OR_EPS_DIV 1e-3
#define OR_EPS_OBJ 1e-4
#define OR_EPS_NULL_GPAD 1e-4
#define OR_DIV_HITS 2
typedef struct { int last; double *yck; int hits; } or_divtest;

static int div_check(or_ctx *c, or_divtest *t, int window, int k, const double *y, const double *Hbx,
                     const double *R, double eps_null)
{
    const int m = c->m;
    if (window <= 0 || k % window != 0 || k == t->last) return 0;
    int diverged = 0;
    if (t->last >= 0) {
        double *d = malloc(sizeof(double) * m), *hv = malloc(sizeof(double) * m);
        double dn = 0.0, rn = 0.0;
        for (int kk = 0; kk < m; ++kk) {
            d[kk] = y[kk] - t->yck[kk];
            dn = fmax(dn, fabs(d[kk]));
            rn = fmax(rn, fabs(R[kk]));
        }
        if (dn > 0.0) {
            ctx_hom(c, d, hv);
            double hn = 0.0, lin = 0.0;
            int dom = 1;
            for (int kk = 0; kk < m; ++kk) {
                hn = fmax(hn, fabs(hv[kk]));
                if (d[kk] == 0.0) continue;
                double lo, hi, w, dd;
                row_params(c, kk, &lo, &hi, &w, &dd);
                const int tiny = fabs(d[kk]) <= 1e-9 * dn;
                if (w < INFINITY || (d[kk] > 0.0 && !(hi < INFINITY)) || (d[kk] < 0.0 && !(lo > -INFINITY))) {
                    if (!tiny) dom = 0;
                    lin -= d[kk] * Hbx[kk];
                    continue;
                }
                lin += (d[kk] > 0.0 ? hi * d[kk] : lo * d[kk]) - d[kk] * Hbx[kk];
            }
            const int pass = dom && c->lambda * hn <= eps_null * dn && lin <= -OR_EPS_OBJ * dn * rn;
            t->hits = pass ? t->hits + 1 : 0;
            diverged = t->hits >= OR_DIV_HITS;
        }
        free(d); free(hv);
    }
    memcpy(t->yck, y, sizeof(double) * m);
    t->last = k;
    return diverged;
}

/*
 * Accelerated dual proximal gradient (GPAD), the warm start of Sec. III-F and
 * the comparison method of Sec. IV-A: from y^0 = y^{-1} = y_inout and
 * theta_0 = theta_{-1} = 1, update k takes the forward-backward step at the
 * extrapolated point
 *   w^k = y^k + theta_k (1/theta_{k-1} - 1) (y^k - y^{k-1}),
 *   y^{k+1} = T_lambda(w^k),
 *   theta_{k+1} = (sqrt(theta_k^4 + 4 theta_k^2) - theta_k^2) / 2.
 * One Algorithm-3 sweep per update.  The termination test of the other
 * methods is applied to R_lambda(w^k); the last evaluated point w^k is
 * returned in y_inout (max_iter = k stops after k steps with w^k).
 */
static int gpad(const or_problem *pb, const or_factors *f, const double *p,
                const or_opts *o, double *y_inout, double *x, double *u, or_info *info)
{
    or_ctx c;
    const double lam = o->lambda;
    ctx_init(&c, pb, f, p, lam, o->precondition);
    const int m = c.m;
    double *y = malloc(sizeof(double) * m), *yp = malloc(sizeof(double) * m);
    double *w = y_inout, *R = malloc(sizeof(double) * m);
    memcpy(y, y_inout, sizeof(double) * m);
    memcpy(yp, y_inout, sizeof(double) * m);
    double th = 1.0, thp = 1.0;
    double *hb = malloc(sizeof(double) * m);
    or_divtest dt = {-1, malloc(sizeof(double) * m), 0};
    int status = 1, k = 0;
    double phi = 0.0;
    for (;;) {
        const double beta = (or_mutation == 9) ? th * (thp - 1.0) : th * (1.0 / thp - 1.0);
        for (int kk = 0; kk < m; ++kk) w[kk] = y[kk] + beta * (y[kk] - yp[kk]);
        phi = ctx_eval(&c, w, hb, R, NULL, NULL);
        const double rn = inf_norm(m, R);
        if (!isfinite(rn) || (!isfinite(phi) && or_mutation != 12)) { status = -5; break; }
        if (rn <= o->eps) { status = 0; break; }
        if (div_check(&c, &dt, o->div_window, k, w, hb, R, OR_EPS_NULL_GPAD)) { status = -6; break; }
        if (k >= o->max_iter) { status = 1; break; }
        for (int kk = 0; kk < m; ++kk) {
            yp[kk] = y[kk];
            y[kk] = w[kk] - lam * R[kk];
        }
        thp = th;
        th = 0.5 * (sqrt(th * th * th * th + 4.0 * th * th) - th * th);
        ++k;
    }
    memcpy(x, c.x, sizeof(double) * (size_t)pb->V * pb->nx);
    memcpy(u, c.u, sizeof(double) * (size_t)pb->Vnl * pb->nu);
    double unsc = 0.0;
    for (int kk = 0; kk < m; ++kk) unsc = fmax(unsc, fabs(R[kk] / c.sc[kk]));
    info->iters = k;
    info->sweeps_affine = c.sweeps_affine;
    info->status = status;
    info->res_scaled_inf = inf_norm(m, R);
    info->res_unscaled_inf = unsc;
    info->phi = phi;
    info->lambda_final = lam;
    free(y); free(yp); free(R); free(hb); free(dt.yck);
    ctx_free(&c);
    return status;
}

/*
 * Dual MINFBE (Algorithm 1, opts->method == 0), NAMA (Algorithm 2, method
 * 1) or GPAD (method 2) on the (scaled, if opts->precondition) dual.  y_inout
 * holds the initial dual on entry and the last iterate on exit; x, u receive
 * x(y).
 *
 * Readings: the line search takes the LARGEST step tau = 2^-nu, nu = 0..nu_max,
 * with phi(w) <= phi(y) (nu = 0 first), and falls back to tau = 0 after nu_max
 * failures; MINFBE's update is y+ = T(w); NAMA's trial point is
 * w = y - (1 - tau) lambda r + tau d, so tau = 0 gives the forward-backward
 * step T(y), and y+ = T(w); the stopping test is ||R||_inf <= eps in the
 * solver's variables.
 *
 * Backtracking on lambda (Sec. III-B), both tests with the L-BFGS buffer
 * emptied whenever lambda is halved, after which the update is taken again
 * from the same y^k with the new lambda (it does not count as an update):
 *   backtrack = 1: after y+ = T(w), halve lambda when
 *     f-hat(y+) > f-hat(w) - lambda <grad f-hat(w), R(w)>
 *                 + ((1 - beta) lambda / 2) ||R(w)||^2,   beta = bt_param
 *     (read at the point w the forward-backward step was taken from; w = y
 *     when tau = 0 in MINFBE);
 *   backtrack = 2: before the direction, halve lambda when
 *     lambda ||grad f-hat(T(y)) - grad f-hat(y)|| > eps'' ||T(y) - y||,
 *     eps'' = bt_param; both gradients are evaluated directly.
 * Returns 0 (converged), 1 (max_iter reached), -5 (non-finite values or more
 * than OR_BT_MAX halvings) or -6 (divergence test).
 */
int or_solve(const or_problem *pb, const or_factors *f, const double *p,
             const or_opts *o, double *y_inout, double *x, double *u, or_info *info)
{
    memset(info, 0, sizeof(*info));
    if (o->method == 2) return gpad(pb, f, p, o, y_inout, x, u, info);
    or_ctx c;
    double lam = o->lambda;
    ctx_init(&c, pb, f, p, lam, o->precondition);
    const int m = c.m;
    double *y = y_inout;
    double *R = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * m);
    double *d = malloc(sizeof(double) * m), *w = malloc(sizeof(double) * m);
    double *Rw = malloc(sizeof(double) * m), *yn = malloc(sizeof(double) * m);
    double *Rn = malloc(sizeof(double) * m), *gn = malloc(sizeof(double) * m);
    double *s = malloc(sizeof(double) * m), *qv = malloc(sizeof(double) * m);
    double *hv = malloc(sizeof(double) * m), *hw = malloc(sizeof(double) * m);
    double *yt = malloc(sizeof(double) * m), *Rt = malloc(sizeof(double) * m);
    or_lbfgs lb;
    lb_init(&lb, o->mem, m);
    int status = 1;
    double fh = 0.0;
    double *hb = malloc(sizeof(double) * m), *hbn = malloc(sizeof(double) * m);
    or_divtest dt = {-1, malloc(sizeof(double) * m), 0};

    /* phi, R (and grad phi for MINFBE) at y with the current lambda */
#define EVAL_AT_Y()                                                          \
    do {                                                                     \
        phi = ctx_eval(&c, y, hb, R, &fh, NULL);                             \
        if (o->method == 0) {                                                \
            ctx_hom(&c, R, hv);                                              \
            for (int kk = 0; kk < m; ++kk) g[kk] = R[kk] + lam * hv[kk];     \
        }                                                                    \
    } while (0)
    double phi;
    EVAL_AT_Y();
    int k = 0;
    for (;;) {
        const double rn = inf_norm(m, R);
        if (!isfinite(rn) || !isfinite(phi)) { status = -5; break; }
        if (rn <= o->eps) { status = 0; break; }
        if (div_check(&c, &dt, o->div_window, k, y, hb, R, OR_EPS_DIV)) { status = -6; break; }
        if (k >= o->max_iter) { status = 1; break; }

        int halve = 0;
        if (o->backtrack == 2) {
            /* T(y) and the dual gradient there, both directly */
            for (int kk = 0; kk < m; ++kk) yt[kk] = y[kk] - lam * R[kk];
            double *h0 = malloc(sizeof(double) * m);
            ctx_eval(&c, y, h0, NULL, NULL, NULL);
            ctx_eval(&c, yt, hw, Rt, NULL, NULL);
            double gd2 = 0.0, st2 = 0.0;
            for (int kk = 0; kk < m; ++kk) {
                const double gd = -(hw[kk] - h0[kk]);    /* grad f-hat = -Hb x */
                gd2 += gd * gd;
                st2 += (yt[kk] - y[kk]) * (yt[kk] - y[kk]);
            }
            free(h0);
            halve = lam * sqrt(gd2) > o->bt_param * sqrt(st2);
        }
        if (!halve) {
            const double *dir_src = (o->method == 0) ? g : R;
            const int used = lb.cnt;
            lb_direction(&lb, dir_src, d);

            int accepted = -1;
            double phiw = phi;
            double *row = (o->trace && k < o->trace_iters) ? o->trace + (size_t)k * OR_TRACE_COLS : NULL;
            if (row) {
                for (int cc = 0; cc < OR_TRACE_COLS; ++cc) row[cc] = NAN;
                row[0] = lam; row[1] = rn; row[3] = o->nu_max; row[4] = used;
            }
            for (int nu = 0; nu <= o->nu_max; ++nu) {
                const double tau = ldexp(1.0, -nu);
                for (int kk = 0; kk < m; ++kk)
                    w[kk] = (o->method == 0) ? y[kk] + tau * d[kk]
                                             : y[kk] - (1.0 - tau) * lam * R[kk] + tau * d[kk];
                phiw = ctx_eval(&c, w, NULL, Rw, NULL, NULL);
                if (accepted < 0) info->ls_trials++;
                if (row && OR_TRACE_PHI + nu < OR_TRACE_COLS) row[OR_TRACE_PHI + nu] = phiw - phi;
                if (accepted < 0 && phiw <= phi) {
                    accepted = nu;
                    if (!row) break;
                }
            }
            if (row) row[2] = accepted;
            /* w and its residual at the accepted trial */
            if (accepted < 0) {                         /* tau = 0 */
                for (int kk = 0; kk < m; ++kk)
                    w[kk] = (o->method == 0) ? y[kk] : y[kk] - lam * R[kk];
            } else {
                const double tau = ldexp(1.0, -accepted);
                for (int kk = 0; kk < m; ++kk)
                    w[kk] = (o->method == 0) ? y[kk] + tau * d[kk]
                                             : y[kk] - (1.0 - tau) * lam * R[kk] + tau * d[kk];
            }
            ctx_eval(&c, w, hw, Rw, NULL, NULL);
            for (int kk = 0; kk < m; ++kk)
                yn[kk] = (or_mutation == 5) ? w[kk] + lam * Rw[kk] : w[kk] - lam * Rw[kk];

            const double phin = ctx_eval(&c, yn, hbn, Rn, NULL, NULL);
            if (o->backtrack == 1) {
                /* f-hat is quadratic, so with delta = y+ - w = -lambda R(w)
                 * its increment is exactly
                 *   f-hat(y+) - f-hat(w) = <grad f-hat(w), delta>
                 *                          - (1/2) <delta, Hb x-hat(sc delta)>,
                 * the second term from one Algorithm-4 sweep.  The first term
                 * is the test's -lambda <grad f-hat(w), R(w)>, present on both
                 * sides, so the test compares the remaining terms (evaluating
                 * f-hat(y+) and f-hat(w) and subtracting would lose the test
                 * in rounding once ||R|| is small). */
                for (int kk = 0; kk < m; ++kk) s[kk] = yn[kk] - w[kk];
                ctx_hom(&c, s, qv);
                const double curv = -0.5 * dot(m, s, qv);
                const double bound = 0.5 * (1.0 - o->bt_param) * lam * dot(m, Rw, Rw);
                halve = curv > bound;
            }
            if (!halve) {
                if (accepted < 0) info->tau_hist[31]++;
                else info->tau_hist[accepted < 31 ? accepted : 30]++;
                phi = phin;
                if (o->method == 0) {
                    ctx_hom(&c, Rn, hv);
                    for (int kk = 0; kk < m; ++kk) gn[kk] = Rn[kk] + lam * hv[kk];
                }
                /* curvature-guarded push of (s, q) */
                const double *gold = (o->method == 0) ? g : R;
                const double *gnew = (o->method == 0) ? gn : Rn;
                for (int kk = 0; kk < m; ++kk) { s[kk] = yn[kk] - y[kk]; qv[kk] = gnew[kk] - gold[kk]; }
                const double sq = dot(m, s, qv);
                if (sq > o->eps_curv * dot(m, s, s) * dot(m, gold, gold)) {
                    lb_push(&lb, s, qv);
                    info->lbfgs_push++;
                } else {
                    info->lbfgs_skip++;
                }
                memcpy(y, yn, sizeof(double) * m);
                memcpy(R, Rn, sizeof(double) * m);
                memcpy(hb, hbn, sizeof(double) * m);
                if (o->method == 0) memcpy(g, gn, sizeof(double) * m);
                ++k;
                continue;
            }
        }
        /* halve lambda, empty the buffer, evaluate again at the same y */
        if (++info->backtracks > OR_BT_MAX) { status = -5; break; }
        lam *= 0.5;
        c.lambda = lam;
        if (or_mutation != 11) lb_clear(&lb);
        EVAL_AT_Y();
    }
#undef EVAL_AT_Y
    /* final primal x(y) and residuals */
    phi = ctx_eval(&c, y, NULL, R, NULL, NULL);
    memcpy(x, c.x, sizeof(double) * (size_t)pb->V * pb->nx);
    memcpy(u, c.u, sizeof(double) * (size_t)pb->Vnl * pb->nu);
    double unsc = 0.0;
    for (int kk = 0; kk < m; ++kk) unsc = fmax(unsc, fabs(R[kk] / c.sc[kk]));
    info->iters = k;
    info->sweeps_affine = c.sweeps_affine;
    info->sweeps_hom = c.sweeps_hom;
    info->status = status;
    info->res_scaled_inf = inf_norm(m, R);
    info->res_unscaled_inf = unsc;
    info->phi = phi;
    info->lambda_final = lam;
    lb_free(&lb);
    free(R); free(g); free(d); free(w); free(Rw); free(yn); free(Rn); free(gn);
    free(s); free(qv); free(hv); free(hw); free(yt); free(Rt); free(hb); free(hbn); free(dt.yck);
    ctx_free(&c);
    return status;
}
