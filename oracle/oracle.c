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
 *   or_eval      Sec. II-D and III-A: z_lambda, R_lambda, T_lambda and the
 *                forward-backward envelope, in the diagonally preconditioned
 *                dual variables of Sec. III-E when asked.
 *   or_solve     Algorithm 1 (dual MINFBE) and Algorithm 2 (NAMA), with the
 *                FBE evaluated directly (one affine sweep per trial step).
 *
 * Readings where the paper is silent or garbled are listed in the design
 * notes; the main ones appear next to the code they affect.
 *
 * Parity pins (the tests) tie each function to the mathematics: dense KKT
 * solves of the inner problem, central differences of the dual function,
 * the dense Hessian's symmetry and spectrum, the FBE's conjugate form, the
 * secant identity of L-BFGS, and a dense interior-point solution of the whole
 * problem.  The iteration trajectory itself has no printed trace in the paper:
 * parity unpinned for the trajectory (only its end point is pinned).
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
    int mem, nu_max, max_iter, precondition, method; /* method 0 MINFBE, 1 NAMA */
} or_opts;

typedef struct {
    int iters, sweeps_affine, sweeps_hom, ls_trials, lbfgs_push, lbfgs_skip, status;
    double res_scaled_inf, res_unscaled_inf, phi;
    int tau_hist[32];
} or_info;

/* Deliberate-mistake switch used only by the tests that show the pins have
 * teeth: each nonzero value plants one plausible error.  0 = correct. */
int or_mutation = 0;

/* ---------------------------- small helpers ---------------------------- */
static int dual_off(const or_problem *pb, int i)
{
    /* Dual vector layout: non-leaf i holds (x-rows, u-rows); leaves follow. */
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
int or_factor(const or_problem *pb, or_factors *f)
{
    const int nx = pb->nx, nu = pb->nu, N = pb->N;
    const int nxu = nx + nu;
    double *Rt = malloc(sizeof(double) * nu * nu);
    double *Lc = malloc(sizeof(double) * nu * nu);
    double *Ri = malloc(sizeof(double) * nu * nu);
    double *St = malloc(sizeof(double) * nu * nx);
    double *PB = malloc(sizeof(double) * nx * nu);
    double *PA = malloc(sizeof(double) * nx * nx);
    int rc = 0;

    /* leaves */
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
        for (int i = pb->stage_ptr[t]; i < pb->stage_ptr[t + 1]; ++i) {
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
            if (cholesky(nu, Rt, Lc) != 0) { rc = -3; break; }
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
        }
    }
    free(Rt); free(Lc); free(Ri); free(St); free(PB); free(PA);
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
    for (int j = pb->Vnl; j < pb->V; ++j) {
        const double *yj = y + dual_off(pb, j);
        for (int a = 0; a < nx; ++a)
            qh[(size_t)j * nx + a] = yj[a] + (aff ? f->chat[(size_t)j * nx + a] : 0.0);
    }
    /* non-leaves: u_i = Phi_i y_i (+ sigma_i), q-hat_i = D_i' y_i (+ c-hat_i) */
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

/* Per-row lower/upper box in the dual layout (unscaled). */
static void box_rows(const or_problem *pb, double *lo, double *hi)
{
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
 * of node i (1 when not preconditioning). */
static void row_scale(const or_problem *pb, int precondition, double *sc)
{
    for (int i = 0; i < pb->V; ++i) {
        double s = 1.0;
        if (precondition) s = (or_mutation == 8) ? pb->prob[i] : sqrt(pb->prob[i]);
        const int o = dual_off(pb, i);
        for (int a = 0; a < node_rows(pb, i); ++a) sc[o + a] = s;
    }
}

/* ------------------------- evaluation at a dual point ------------------- */
typedef struct {
    const or_problem *pb;
    const or_factors *f;
    const double *p;       /* x0 */
    double lambda;
    int m, precondition;
    double *sc, *lo, *hi;  /* per-row scale and (unscaled) box */
    double *ytmp, *x, *u, *hx;
    int sweeps_affine, sweeps_hom;
} or_ctx;

static void ctx_init(or_ctx *c, const or_problem *pb, const or_factors *f,
                     const double *p, double lambda, int precondition)
{
    c->pb = pb; c->f = f; c->p = p; c->lambda = lambda;
    c->precondition = precondition;
    c->m = or_dual_dim(pb);
    c->sc = malloc(sizeof(double) * c->m);
    c->lo = malloc(sizeof(double) * c->m);
    c->hi = malloc(sizeof(double) * c->m);
    c->ytmp = malloc(sizeof(double) * c->m);
    c->hx = malloc(sizeof(double) * c->m);
    c->x = malloc(sizeof(double) * (size_t)pb->V * pb->nx);
    c->u = malloc(sizeof(double) * (size_t)pb->Vnl * pb->nu);
    row_scale(pb, precondition, c->sc);
    box_rows(pb, c->lo, c->hi);
    c->sweeps_affine = c->sweeps_hom = 0;
}

static void ctx_free(or_ctx *c)
{
    free(c->sc); free(c->lo); free(c->hi); free(c->ytmp); free(c->hx);
    free(c->x); free(c->u);
}

/*
 * At the (scaled) dual point yb: x = x(sc*yb) (Algorithm 3), Hbx = sc*H x,
 * z = proj_{sc*Y}(yb/lambda + Hbx), R = z - Hbx (Sec. II-D), and the FBE
 *   phi = -f(x) + <yb, R> - (lambda/2) ||R||^2,
 * which equals f-hat + g*(T) - lambda <grad f-hat, R> + (lambda/2)||R||^2 of
 * Sec. III-A because g*(T) = <T, z> for a box (Fenchel-Young equality at the
 * projection).  Outputs Hbx, R (each may be NULL) and returns phi.
 */
static double ctx_eval(or_ctx *c, const double *yb, double *Hbx, double *R)
{
    const int m = c->m;
    for (int k = 0; k < m; ++k) c->ytmp[k] = c->sc[k] * yb[k];
    or_sweep(c->pb, c->f, c->ytmp, c->p, 0, c->x, c->u);
    c->sweeps_affine++;
    or_Hx(c->pb, c->x, c->u, c->hx);
    double inner = 0.0, nrm2 = 0.0;
    for (int k = 0; k < m; ++k) {
        const double h = c->sc[k] * c->hx[k];
        const double v = yb[k] / c->lambda + h;
        const double lo = c->sc[k] * c->lo[k], hi = c->sc[k] * c->hi[k];
        const double z = v < lo ? lo : (v > hi ? hi : v);
        const double r = z - h;
        if (Hbx) Hbx[k] = h;
        if (R) R[k] = r;
        inner += yb[k] * r;
        nrm2 += r * r;
    }
    const double fx = or_cost(c->pb, c->x, c->u);
    if (or_mutation == 6) return -fx + inner + 0.5 * c->lambda * nrm2;
    return -fx + inner - 0.5 * c->lambda * nrm2;
}

/* Hb x-hat(sc * v): the linear part (Algorithm 4), scaled back; the Hessian
 * of the (scaled) dual function applied to v is minus this. */
static void ctx_hom(or_ctx *c, const double *v, double *out)
{
    for (int k = 0; k < c->m; ++k) c->ytmp[k] = c->sc[k] * v[k];
    or_sweep(c->pb, c->f, c->ytmp, c->p, 1, c->x, c->u);
    c->sweeps_hom++;
    or_Hx(c->pb, c->x, c->u, c->hx);
    for (int k = 0; k < c->m; ++k) out[k] = c->sc[k] * c->hx[k];
}

/*
 * Exported evaluation: given a (scaled) dual point, return x, u (unscaled
 * primal, Algorithm 3), Hbx, z, R, T = y - lambda R, and grad_phi =
 * (I - lambda Hess f-hat) R = R + lambda Hb x-hat(sc R) (Sec. III-A).
 * Any output pointer may be NULL.  Returns phi.
 */
double or_eval(const or_problem *pb, const or_factors *f, const double *p,
               double lambda, int precondition, const double *yb,
               double *x, double *u, double *Hbx, double *z, double *R,
               double *T, double *grad_phi)
{
    or_ctx c;
    ctx_init(&c, pb, f, p, lambda, precondition);
    const int m = c.m;
    double *h = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    const double phi = ctx_eval(&c, yb, h, r);
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

/* v -> Hb x-hat(sc v), exported for the Hessian pins (the Hessian of the
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

/* --------------------------- Algorithms 1 and 2 -------------------------- */
static double dot(int m, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += a[k] * b[k];
    return s;
}

static double inf_norm(int m, const double *a)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) s = fmax(s, fabs(a[k]));
    return s;
}

/*
 * Dual MINFBE (Algorithm 1, opts->method == 0) or NAMA (Algorithm 2,
 * method == 1) on the (scaled, if opts->precondition) dual.  y_inout holds the
 * initial dual on entry and the last iterate on exit; x, u receive x(y).
 *
 * Readings: the line search takes the LARGEST step tau = 2^-nu, nu = 0..nu_max,
 * with phi(w) <= phi(y) (nu = 0 first), and falls back to tau = 0 after nu_max
 * failures; MINFBE's update is y+ = T(w); NAMA's trial point is
 * w = y - (1 - tau) lambda r + tau d, so tau = 0 gives the forward-backward
 * step T(y), and y+ = T(w); the stopping test is ||R||_inf <= eps in the
 * solver's variables.  Returns 0 (converged), 1 (max_iter reached) or -5
 * (non-finite values).
 */
int or_solve(const or_problem *pb, const or_factors *f, const double *p,
             const or_opts *o, double *y_inout, double *x, double *u, or_info *info)
{
    or_ctx c;
    const double lam = o->lambda;
    ctx_init(&c, pb, f, p, lam, o->precondition);
    const int m = c.m;
    double *y = y_inout;
    double *R = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * m);
    double *d = malloc(sizeof(double) * m), *w = malloc(sizeof(double) * m);
    double *Rw = malloc(sizeof(double) * m), *yn = malloc(sizeof(double) * m);
    double *Rn = malloc(sizeof(double) * m), *gn = malloc(sizeof(double) * m);
    double *s = malloc(sizeof(double) * m), *qv = malloc(sizeof(double) * m);
    double *hv = malloc(sizeof(double) * m);
    or_lbfgs lb;
    lb_init(&lb, o->mem, m);
    memset(info, 0, sizeof(*info));
    int status = 1;

    double phi = ctx_eval(&c, y, NULL, R);
    if (o->method == 0) {                           /* grad phi = R + lam Hb xhat(sc R) */
        ctx_hom(&c, R, hv);
        for (int k = 0; k < m; ++k) g[k] = R[k] + lam * hv[k];
    }
    int k = 0;
    for (;;) {
        const double rn = inf_norm(m, R);
        if (!isfinite(rn) || !isfinite(phi)) { status = -5; break; }
        if (rn <= o->eps) { status = 0; break; }
        if (k >= o->max_iter) { status = 1; break; }

        const double *dir_src = (o->method == 0) ? g : R;
        lb_direction(&lb, dir_src, d);

        int accepted = -1;
        double phiw = phi;
        for (int nu = 0; nu <= o->nu_max; ++nu) {
            const double tau = ldexp(1.0, -nu);
            for (int kk = 0; kk < m; ++kk)
                w[kk] = (o->method == 0) ? y[kk] + tau * d[kk]
                                         : y[kk] - (1.0 - tau) * lam * R[kk] + tau * d[kk];
            phiw = ctx_eval(&c, w, NULL, Rw);
            info->ls_trials++;
            if (phiw <= phi) { accepted = nu; break; }
        }
        if (accepted < 0) {                         /* tau = 0 */
            for (int kk = 0; kk < m; ++kk)
                w[kk] = (o->method == 0) ? y[kk] : y[kk] - lam * R[kk];
            if (o->method == 0) memcpy(Rw, R, sizeof(double) * m);
            else ctx_eval(&c, w, NULL, Rw);
            info->tau_hist[31]++;
        } else {
            info->tau_hist[accepted < 31 ? accepted : 30]++;
        }
        for (int kk = 0; kk < m; ++kk)
            yn[kk] = (or_mutation == 5) ? w[kk] + lam * Rw[kk] : w[kk] - lam * Rw[kk];

        phi = ctx_eval(&c, yn, NULL, Rn);
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
        if (o->method == 0) memcpy(g, gn, sizeof(double) * m);
        ++k;
    }
    /* final primal x(y) and residuals */
    phi = ctx_eval(&c, y, NULL, R);
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
    lb_free(&lb);
    free(R); free(g); free(d); free(w); free(Rw); free(yn); free(Rn); free(gn);
    free(s); free(qv); free(hv);
    ctx_free(&c);
    return status;
}
