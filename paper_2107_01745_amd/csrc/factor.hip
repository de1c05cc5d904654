// Factor step (arXiv 2107.01745, Sec. III-D: the Riccati-type recursion that
// precomputes the per-node factors once, before any solve).
//
// The paper names the factors (Phi, Theta, D, Lambda, K, sigma, c-hat) but
// gives no formulas; they follow from dynamic programming on the inner problem
// whose minimiser is x(y).  With costs written without 1/2 (Sec. II-B) the
// value function of the subtree of node i is x' (P_i/2) x + (linear terms):
//   leaves j:      P_j = 2 pi_j Pterm_j,   chat_j = P_j c_j + pi_j p_j
//   non-leaf i:    R~_i = 2 pi_i R_i + sum_j B_j' P_j B_j      (Cholesky)
//                  S~_i = 2 pi_i S_i + sum_j B_j' P_j A_j
//                  K_i  = -R~_i^{-1} S~_i
//                  P_i  = 2 pi_i Q_i + sum_j A_j' P_j A_j + K_i' S~_i
//                  chat_i = P_i c_i + pi_i q_i  (c_0 = 0),  sig_i = pi_i r_i
// (the K_i' pi_i r_i part of the paper's c-hat is applied in the sweep, where
// pi_i r_i enters g_i).  Stages run N-1..0, one kernel per stage, one
// workgroup per node; the products are small dense FP64 blocks computed with
// the workgroup's threads over output entries.
//
// The sweeps then stream, per edge j, M_j = [A_j B_j] row-major (backward,
// Mb) and its transpose (forward, Mf), and per non-leaf node K_i (Kb), K_i'
// (Kf) and -R~_i^{-1} (Rn); rows are padded to an even length so each row is
// one aligned 16-byte-per-lane load.
#include <cmath>
#include <cstring>

#include "internal.h"

namespace stotree {

namespace {

struct FactorArgs {
    int nx, nu, V, Vnl, ldM, ldx, ldu;
    const int *stage_ptr, *child_ptr;
    const double *prob, *A, *B, *c, *Q, *R, *S, *q, *r, *P, *p;
    double *Pcal, *scratch;
    long long slot;  // scratch doubles per workgroup
    double *Mb, *Mf, *Kb, *Kf, *Rn, *chat, *sig;
    int *err;
};

__global__ void pack_dynamics_kernel(FactorArgs a)
{
    const int nx = a.nx, nu = a.nu, W = nx + nu;
    const long long per_b = (long long)nx * a.ldM, per_f = (long long)W * a.ldx;
    const long long total = (long long)(a.V - 1) * (per_b + per_f);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = 1 + e / (per_b + per_f);
        const long long w = e % (per_b + per_f);
        if (w < per_b) {  // Mb[j][r][col]
            const int r = (int)(w / a.ldM), col = (int)(w % a.ldM);
            double v = 0.0;
            if (col < nx) v = a.A[(j * nx + r) * nx + col];
            else if (col < W) v = a.B[(j * nx + r) * nu + (col - nx)];
            a.Mb[j * per_b + w] = v;
        } else {           // Mf[j][col][r] = M_j[r][col]
            const long long wf = w - per_b;
            const int col = (int)(wf / a.ldx), r = (int)(wf % a.ldx);
            double v = 0.0;
            if (r < nx) v = (col < nx) ? a.A[(j * nx + r) * nx + col] : a.B[(j * nx + r) * nu + (col - nx)];
            a.Mf[j * per_f + wf] = v;
        }
    }
}

__global__ void factor_leaves_kernel(FactorArgs a)
{
    const int nx = a.nx;
    const int j = a.Vnl + blockIdx.x;
    if (j >= a.V) return;
    const long long l = j - a.Vnl;
    const double pj = a.prob[j];
    double *Pj = a.Pcal + (long long)j * nx * nx;
    for (int e = threadIdx.x; e < nx * nx; e += blockDim.x) Pj[e] = 2.0 * pj * a.P[l * nx * nx + e];
    __syncthreads();
    for (int r = threadIdx.x; r < nx; r += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nx; ++k) s = fma(Pj[r * nx + k], a.c[(long long)j * nx + k], s);
        if (a.p) s += pj * a.p[l * nx + r];
        a.chat[(long long)j * nx + r] = s;
    }
}

__global__ void __launch_bounds__(256) factor_stage_kernel(FactorArgs a, int t)
{
    const int nx = a.nx, nu = a.nu, W = nx + nu;
    const int i = a.stage_ptr[t] + blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    double *Wsc = a.scratch + (long long)blockIdx.x * a.slot;  // [nx][W]
    double *Rt = Wsc + (long long)nx * W;                      // [nu][nu] -> Cholesky L
    double *St = Rt + nu * nu;                                  // [nu][nx]
    double *Ri = St + nu * nx;                                  // [nu][nu]
    __shared__ int fail;
    const double pi = a.prob[i];
    double *Pi = a.Pcal + (long long)i * nx * nx;
    if (tid == 0) fail = 0;
    for (int e = tid; e < nu * nu; e += nt) Rt[e] = 2.0 * pi * a.R[(long long)i * nu * nu + e];
    for (int e = tid; e < nu * nx; e += nt) St[e] = a.S ? 2.0 * pi * a.S[(long long)i * nu * nx + e] : 0.0;
    for (int e = tid; e < nx * nx; e += nt) Pi[e] = 2.0 * pi * a.Q[(long long)i * nx * nx + e];
    __syncthreads();
    for (int j = a.child_ptr[i]; j < a.child_ptr[i + 1]; ++j) {
        const double *M = a.Mb + (long long)j * nx * a.ldM;
        const double *Pj = a.Pcal + (long long)j * nx * nx;
        for (int e = tid; e < nx * W; e += nt) {          // W = P_j [A_j B_j]
            const int r = e / W, col = e % W;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(Pj[r * nx + k], M[(long long)k * a.ldM + col], s);
            Wsc[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < nx * nx; e += nt) {          // P_i += A_j' P_j A_j
            const int r = e / nx, col = e % nx;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * a.ldM + r], Wsc[k * W + col], s);
            Pi[e] += s;
        }
        for (int e = tid; e < nu * nu; e += nt) {          // R~ += B_j' P_j B_j
            const int r = e / nu, col = e % nu;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * a.ldM + nx + r], Wsc[k * W + nx + col], s);
            Rt[e] += s;
        }
        for (int e = tid; e < nu * nx; e += nt) {          // S~ += B_j' P_j A_j
            const int r = e / nx, col = e % nx;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * a.ldM + nx + r], Wsc[k * W + col], s);
            St[e] += s;
        }
        __syncthreads();
    }
    // Cholesky R~ = L L' in place (lower triangle), column by column.
    for (int jc = 0; jc < nu; ++jc) {
        if (tid == 0) {
            double d = Rt[jc * nu + jc];
            for (int k = 0; k < jc; ++k) d -= Rt[jc * nu + k] * Rt[jc * nu + k];
            if (!(d > 0.0)) fail = 1;
            else Rt[jc * nu + jc] = sqrt(d);
        }
        __syncthreads();
        if (fail) break;
        for (int row = jc + 1 + tid; row < nu; row += nt) {
            double s = Rt[row * nu + jc];
            for (int k = 0; k < jc; ++k) s -= Rt[row * nu + k] * Rt[jc * nu + k];
            Rt[row * nu + jc] = s / Rt[jc * nu + jc];
        }
        __syncthreads();
    }
    if (fail) {
        if (tid == 0) atomicExch(a.err, STOTREE_ERR_NOT_PD);
        return;
    }
    // R~^{-1}, one column per thread: L w = e, L' v = w.
    for (int col = tid; col < nu; col += nt) {
        for (int row = 0; row < nu; ++row) {
            double s = (row == col) ? 1.0 : 0.0;
            for (int k = 0; k < row; ++k) s -= Rt[row * nu + k] * Ri[k * nu + col];
            Ri[row * nu + col] = s / Rt[row * nu + row];
        }
        for (int row = nu - 1; row >= 0; --row) {
            double s = Ri[row * nu + col];
            for (int k = row + 1; k < nu; ++k) s -= Rt[k * nu + row] * Ri[k * nu + col];
            Ri[row * nu + col] = s / Rt[row * nu + row];
        }
    }
    __syncthreads();
    double *Kb = a.Kb + (long long)i * nu * a.ldx;
    double *Kf = a.Kf + (long long)i * nx * a.ldu;
    double *Rn = a.Rn + (long long)i * nu * a.ldu;
    for (int e = tid; e < nu * nx; e += nt) {              // K = -R~^{-1} S~
        const int r = e / nx, col = e % nx;
        double s = 0.0;
        for (int k = 0; k < nu; ++k) s = fma(Ri[r * nu + k], St[k * nx + col], s);
        Kb[r * a.ldx + col] = -s;
        Kf[col * a.ldu + r] = -s;
    }
    for (int e = tid; e < nu * nu; e += nt) Rn[(e / nu) * a.ldu + (e % nu)] = -Ri[e];
    __syncthreads();
    for (int e = tid; e < nx * nx; e += nt) {              // P_i += K' S~
        const int r = e / nx, col = e % nx;
        double s = 0.0;
        for (int k = 0; k < nu; ++k) s = fma(Kb[k * a.ldx + r], St[k * nx + col], s);
        Pi[e] += s;
    }
    __syncthreads();
    for (int rr = tid; rr < nx; rr += nt) {
        double s = 0.0;
        if (i > 0)
            for (int k = 0; k < nx; ++k) s = fma(Pi[rr * nx + k], a.c[(long long)i * nx + k], s);
        if (a.q) s += pi * a.q[(long long)i * nx + rr];
        a.chat[(long long)i * nx + rr] = s;
    }
    for (int rr = tid; rr < nu; rr += nt) a.sig[(long long)i * nu + rr] = a.r ? pi * a.r[(long long)i * nu + rr] : 0.0;
}

__global__ void sqrt_prob_kernel(const double *prob, double *sc, int V)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < V) sc[i] = sqrt(prob[i]);
}

bool all_finite(const double *a, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(a[k])) return false;
    return true;
}

// Device buffer freed at scope exit.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

template <typename T>
int upload(DevBuf &b, const T *h, size_t n)
{
    if (!h) return STOTREE_OK;
    STOTREE_HIP(hipMalloc(&b.p, sizeof(T) * (n ? n : 1)));
    STOTREE_HIP(hipMemcpy(b.p, h, sizeof(T) * n, hipMemcpyHostToDevice));
    return STOTREE_OK;
}

}  // namespace

void free_tree(tree_factors *f)
{
    if (!f) return;
    for (void *p : {(void *)f->d_stage_ptr, (void *)f->d_child_ptr, (void *)f->Mb, (void *)f->Mf,
                    (void *)f->Kb, (void *)f->Kf, (void *)f->Rn, (void *)f->chat, (void *)f->sig,
                    (void *)f->cvec, (void *)f->sc, (void *)f->lo, (void *)f->hi, (void *)f->qhat,
                    (void *)f->kbuf, (void *)f->sws.buf})
        if (p) (void)hipFree(p);
    delete f;
}

int factor_tree(const tree_desc *t, const problem_data *d, int precondition, hipStream_t st,
                tree_factors **out)
{
    if (!out) { set_error("tree_factor: out is NULL"); return STOTREE_ERR_ARG; }
    *out = nullptr;
    if (!t || !d) { set_error("tree_factor: NULL tree or data"); return STOTREE_ERR_ARG; }
    const int nx = t->nx, nu = t->nu, N = t->N, V = t->num_nodes;
    if (nx < 1 || nu < 1 || N < 1 || V < 2 || nx + nu > kMaxWidth) {
        set_error("tree_factor: need nx>=1, nu>=1, N>=1, V>=2 and nx+nu<=256");
        return STOTREE_ERR_ARG;
    }
    if (!t->stage_ptr || !t->ancestor || !t->child_ptr || !t->prob || !d->A || !d->B || !d->c ||
        !d->Q || !d->R || !d->P || !d->xmin || !d->xmax || !d->umin || !d->umax) {
        set_error("tree_factor: a required array is NULL");
        return STOTREE_ERR_ARG;
    }
    // ---- tree validation (Sec. II-A) ----
    const int *sp = t->stage_ptr;
    if (sp[0] != 0 || sp[1] != 1 || sp[N + 1] != V) {
        set_error("tree_factor: stage_ptr must start 0,1 and end at num_nodes");
        return STOTREE_ERR_TREE;
    }
    for (int s = 0; s <= N; ++s)
        if (sp[s + 1] <= sp[s]) { set_error("tree_factor: empty stage"); return STOTREE_ERR_TREE; }
    const int Vnl = sp[N];
    if (t->ancestor[0] != -1) { set_error("tree_factor: ancestor[0] must be -1"); return STOTREE_ERR_TREE; }
    for (int s = 1; s <= N; ++s)
        for (int i = sp[s]; i < sp[s + 1]; ++i) {
            const int a = t->ancestor[i];
            if (a < sp[s - 1] || a >= sp[s]) {
                set_error("tree_factor: ancestor of a node is not in the previous stage");
                return STOTREE_ERR_TREE;
            }
        }
    const int *cp = t->child_ptr;
    if (cp[0] != 1 || cp[Vnl] != V) { set_error("tree_factor: child_ptr must span [1, V)"); return STOTREE_ERR_TREE; }
    for (int i = 0; i < Vnl; ++i) {
        if (cp[i + 1] <= cp[i]) { set_error("tree_factor: a non-leaf node has no child"); return STOTREE_ERR_TREE; }
        for (int j = cp[i]; j < cp[i + 1]; ++j)
            if (t->ancestor[j] != i) {
                set_error("tree_factor: child_ptr and ancestor disagree");
                return STOTREE_ERR_TREE;
            }
    }
    if (std::fabs(t->prob[0] - 1.0) > 1e-12) { set_error("tree_factor: prob[0] must be 1"); return STOTREE_ERR_TREE; }
    for (int s = 0; s <= N; ++s) {
        double tot = 0.0;
        for (int i = sp[s]; i < sp[s + 1]; ++i) {
            if (!(t->prob[i] > 0.0) || !std::isfinite(t->prob[i])) {
                set_error("tree_factor: node probabilities must be positive");
                return STOTREE_ERR_TREE;
            }
            tot += t->prob[i];
        }
        if (std::fabs(tot - 1.0) > 1e-12) {
            set_error("tree_factor: probabilities of stage " + std::to_string(s) + " do not sum to 1");
            return STOTREE_ERR_TREE;
        }
    }
    const size_t Vl = (size_t)V - Vnl;
    // ---- data validation ----
    struct Chk { const double *p; size_t n; const char *name; };
    const Chk chks[] = {{d->A, (size_t)V * nx * nx, "A"}, {d->B, (size_t)V * nx * nu, "B"},
                        {d->c, (size_t)V * nx, "c"}, {d->Q, (size_t)Vnl * nx * nx, "Q"},
                        {d->R, (size_t)Vnl * nu * nu, "R"}, {d->S, (size_t)Vnl * nu * nx, "S"},
                        {d->q, (size_t)Vnl * nx, "q"}, {d->r, (size_t)Vnl * nu, "r"},
                        {d->P, Vl * nx * nx, "P"}, {d->p, Vl * nx, "p"}};
    for (const Chk &c : chks)
        if (c.p && !all_finite(c.p, c.n)) {
            set_error(std::string("tree_factor: non-finite entry in ") + c.name);
            return STOTREE_ERR_NUMERIC;
        }
    for (size_t k = 0; k < (size_t)V * nx; ++k)
        if (std::isnan(d->xmin[k]) || std::isnan(d->xmax[k]) || d->xmin[k] > d->xmax[k]) {
            set_error("tree_factor: state box with lo > hi (or NaN)");
            return STOTREE_ERR_BOX;
        }
    for (size_t k = 0; k < (size_t)Vnl * nu; ++k)
        if (std::isnan(d->umin[k]) || std::isnan(d->umax[k]) || d->umin[k] > d->umax[k]) {
            set_error("tree_factor: input box with lo > hi (or NaN)");
            return STOTREE_ERR_BOX;
        }

    tree_factors *f = new tree_factors();
    f->nx = nx; f->nu = nu; f->N = N; f->V = V; f->Vnl = Vnl;
    f->m = (long long)Vnl * (nx + nu) + (long long)Vl * nx;
    f->n = (long long)Vnl * nu + (long long)(V - 1) * nx;
    f->precondition = precondition ? 1 : 0;
    f->ldM = pad2(nx + nu); f->ldx = pad2(nx); f->ldu = pad2(nu);
    f->stage_ptr.assign(sp, sp + N + 2);
    // s*: first stage from which every stage has as many nodes as the leaves
    int sstar = N;
    while (sstar > 0 && sp[sstar] - sp[sstar - 1] == sp[N + 1] - sp[N]) --sstar;
    f->sstar = sstar;
    f->nchains = sp[N + 1] - sp[N];
    struct Guard {
        tree_factors *&f;
        bool ok = false;
        ~Guard() { if (!ok) free_tree(f); }
    } guard{f};

    auto dalloc = [&](auto **p, size_t n) -> int {
        STOTREE_HIP(hipMalloc((void **)p, sizeof(**p) * (n ? n : 1)));
        f->bytes += sizeof(**p) * n;
        return STOTREE_OK;
    };
    int rc;
    if ((rc = dalloc(&f->d_stage_ptr, N + 2)) || (rc = dalloc(&f->d_child_ptr, Vnl + 1)) ||
        (rc = dalloc(&f->Mb, (size_t)V * nx * f->ldM)) ||
        (rc = dalloc(&f->Mf, (size_t)V * (nx + nu) * f->ldx)) ||
        (rc = dalloc(&f->Kb, (size_t)Vnl * nu * f->ldx)) ||
        (rc = dalloc(&f->Kf, (size_t)Vnl * nx * f->ldu)) ||
        (rc = dalloc(&f->Rn, (size_t)Vnl * nu * f->ldu)) || (rc = dalloc(&f->chat, (size_t)V * nx)) ||
        (rc = dalloc(&f->sig, (size_t)Vnl * nu)) || (rc = dalloc(&f->cvec, (size_t)V * nx)) ||
        (rc = dalloc(&f->sc, (size_t)V)) || (rc = dalloc(&f->lo, (size_t)f->m)) ||
        (rc = dalloc(&f->hi, (size_t)f->m)))
        return rc;
    STOTREE_HIP(hipMemcpyAsync(f->d_stage_ptr, sp, sizeof(int) * (N + 2), hipMemcpyHostToDevice, st));
    STOTREE_HIP(hipMemcpyAsync(f->d_child_ptr, cp, sizeof(int) * (Vnl + 1), hipMemcpyHostToDevice, st));
    STOTREE_HIP(hipMemcpyAsync(f->cvec, d->c, sizeof(double) * V * nx, hipMemcpyHostToDevice, st));
    // box rows in the dual layout (a data rearrangement, no arithmetic)
    {
        std::vector<double> lo((size_t)f->m), hi((size_t)f->m);
        for (int i = 0; i < V; ++i) {
            const size_t o = i < Vnl ? (size_t)i * (nx + nu) : (size_t)Vnl * nu + (size_t)i * nx;
            std::memcpy(&lo[o], d->xmin + (size_t)i * nx, sizeof(double) * nx);
            std::memcpy(&hi[o], d->xmax + (size_t)i * nx, sizeof(double) * nx);
            if (i < Vnl) {
                std::memcpy(&lo[o + nx], d->umin + (size_t)i * nu, sizeof(double) * nu);
                std::memcpy(&hi[o + nx], d->umax + (size_t)i * nu, sizeof(double) * nu);
            }
        }
        STOTREE_HIP(hipMemcpy(f->lo, lo.data(), sizeof(double) * f->m, hipMemcpyHostToDevice));
        STOTREE_HIP(hipMemcpy(f->hi, hi.data(), sizeof(double) * f->m, hipMemcpyHostToDevice));
    }
    DevBuf bA, bB, bc, bQ, bR, bS, bq, br, bP, bp, bprob, bPcal, bscr, berr;
    if ((rc = upload(bA, d->A, (size_t)V * nx * nx)) || (rc = upload(bB, d->B, (size_t)V * nx * nu)) ||
        (rc = upload(bc, d->c, (size_t)V * nx)) || (rc = upload(bQ, d->Q, (size_t)Vnl * nx * nx)) ||
        (rc = upload(bR, d->R, (size_t)Vnl * nu * nu)) || (rc = upload(bS, d->S, (size_t)Vnl * nu * nx)) ||
        (rc = upload(bq, d->q, (size_t)Vnl * nx)) || (rc = upload(br, d->r, (size_t)Vnl * nu)) ||
        (rc = upload(bP, d->P, Vl * nx * nx)) || (rc = upload(bp, d->p, Vl * nx)) ||
        (rc = upload(bprob, t->prob, (size_t)V)))
        return rc;
    int maxw = 0;
    for (int s = 0; s < N; ++s) maxw = std::max(maxw, sp[s + 1] - sp[s]);
    const long long slot = (long long)nx * (nx + nu) + 2LL * nu * nu + (long long)nu * nx;
    STOTREE_HIP(hipMalloc(&bPcal.p, sizeof(double) * (size_t)V * nx * nx));
    STOTREE_HIP(hipMalloc(&bscr.p, sizeof(double) * (size_t)maxw * slot));
    STOTREE_HIP(hipMalloc(&berr.p, sizeof(int)));
    STOTREE_HIP(hipMemsetAsync(berr.p, 0, sizeof(int), st));
    STOTREE_HIP(hipMemsetAsync(f->Mb, 0, sizeof(double) * f->ldM * nx, st));            // edge 0 unused
    STOTREE_HIP(hipMemsetAsync(f->Mf, 0, sizeof(double) * f->ldx * (nx + nu), st));
    STOTREE_HIP(hipMemsetAsync(f->Kb, 0, sizeof(double) * (size_t)Vnl * nu * f->ldx, st));
    STOTREE_HIP(hipMemsetAsync(f->Kf, 0, sizeof(double) * (size_t)Vnl * nx * f->ldu, st));
    STOTREE_HIP(hipMemsetAsync(f->Rn, 0, sizeof(double) * (size_t)Vnl * nu * f->ldu, st));

    FactorArgs a{};
    a.nx = nx; a.nu = nu; a.V = V; a.Vnl = Vnl; a.ldM = f->ldM; a.ldx = f->ldx; a.ldu = f->ldu;
    a.stage_ptr = f->d_stage_ptr; a.child_ptr = f->d_child_ptr;
    a.prob = (const double *)bprob.p; a.A = (const double *)bA.p; a.B = (const double *)bB.p;
    a.c = (const double *)bc.p; a.Q = (const double *)bQ.p; a.R = (const double *)bR.p;
    a.S = (const double *)bS.p; a.q = (const double *)bq.p; a.r = (const double *)br.p;
    a.P = (const double *)bP.p; a.p = (const double *)bp.p;
    a.Pcal = (double *)bPcal.p; a.scratch = (double *)bscr.p; a.slot = slot;
    a.Mb = f->Mb; a.Mf = f->Mf; a.Kb = f->Kb; a.Kf = f->Kf; a.Rn = f->Rn;
    a.chat = f->chat; a.sig = f->sig; a.err = (int *)berr.p;

    hipLaunchKernelGGL(pack_dynamics_kernel, dim3(4096), dim3(256), 0, st, a);
    hipLaunchKernelGGL(factor_leaves_kernel, dim3((unsigned)Vl), dim3(64), 0, st, a);
    for (int s = N - 1; s >= 0; --s)
        hipLaunchKernelGGL(factor_stage_kernel, dim3(sp[s + 1] - sp[s]), dim3(256), 0, st, a, s);
    hipLaunchKernelGGL(sqrt_prob_kernel, dim3((V + 255) / 256), dim3(256), 0, st,
                       (const double *)bprob.p, f->sc, V);
    STOTREE_HIP(hipGetLastError());
    int err = 0;
    STOTREE_HIP(hipMemcpyAsync(&err, berr.p, sizeof(int), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    if (err != 0) {
        set_error("tree_factor: R-tilde is not positive definite at some node");
        return err;
    }
    guard.ok = true;
    *out = f;
    return STOTREE_OK;
}

}  // namespace stotree
