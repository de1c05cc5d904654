// Device-resident dual MINFBE (Algorithm 1) and NAMA (Algorithm 2) of
// arXiv 2107.01745, Sec. III-B/III-C, in the preconditioned dual variables of
// Sec. III-E when the handle asks for it.
//
// Every iteration is a fixed sequence of kernels on the caller's stream; all
// scalars (residual norms, curvature test, L-BFGS coefficients, the accepted
// step) are reduced and decided on the device by single-block "finalize"
// kernels, so the host only reads a stop flag every check_every iterations.
// Once the flag is set every remaining kernel returns immediately.
//
// Vector passes (grid-stride over the m dual rows, row r of node i scaled by
// s_i = sqrt(pi_i)):
//   resid   z = proj_[s lo, s hi](y/lambda + s Hx), R = z - s Hx (Sec. II-D);
//           for NAMA also the L-BFGS pair s = y - y_prev, q = R - R_prev and
//           every inner product the compact L-BFGS form needs (one pass).
//   grad    (MINFBE) grad phi = R + lambda s H xhat(s R) (Sec. III-A), the
//           pair with the previous gradient, and the same inner products.
//   combine d = -B g in the compact representation of the L-BFGS inverse
//           Hessian (Byrd, Nocedal and Schnabel 1994), which equals the
//           two-loop recursion but needs one pass over the stored pairs.
//   ls      all trial steps tau = 2^-nu, nu = 0..nu_max, in one pass: since
//           x(.) is affine, H x(w) = s Hx + s H xhat(w - y) is formed from the
//           homogeneous sweeps already done, and the change of the FBE
//           phi(w) - phi(y) is accumulated row by row (Sec. III-B, the
//           tau-independent quantities of the line-search reformulation).
//   update  y+ = T_lambda(w) = w - lambda R(w).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace stotree {

namespace {

constexpr int kMemMax = 16;   // L-BFGS memory supported on the device
constexpr int kNuCap = 30;    // largest nu_max
constexpr int kVB = 256;      // threads per block of the vector kernels

// reduction slots
constexpr int R_MAX = 0, R_MAXU = 1, R_SS = 2, R_BAD = 3, PB = 4;
constexpr int kNMax = 2;  // slots [0, kNMax) are max-reduced, the rest summed
constexpr int nv_pair(int memcap) { return PB + 6 + 5 * memcap; }
constexpr int kNVMax = nv_pair(kMemMax) > kNuCap + 2 ? nv_pair(kMemMax) : kNuCap + 2;

struct Ctl {
    int done, status, iter, have_pair;
    int cnt, free_slot, pushes, skips;
    int ls_trials, sweeps_aff, sweeps_hom, accepted_nu;
    int max_iter, mem, nu_max, method;
    int order[kMemMax];
    double lam, eps, eps_curv, tau, cr;
    double res, resu, rr, gg_prev, gamma;
    double L, inv_norm;
    double SY[kMemMax + 1][kMemMax + 1];  // s_a . q_b by slot
    double QQ[kMemMax + 1][kMemMax + 1];  // q_a . q_b by slot
    double coefS[kMemMax], coefQ[kMemMax];
    double ls_val[kNuCap + 1];
};

struct VecArgs {
    long long m;
    unsigned nlr;  // rows owned by non-leaf nodes
    int nxu, nx, Vnl;
    const double *sc, *lo, *hi;
    Ctl *ctl;
    double *part;
    int nblocks, method;
    const double *y, *yp, *hx, *rp, *gp, *hr, *hd, *d;
    double *r, *g, *S, *Q, *yn;
};

__device__ __forceinline__ double row_scale(const VecArgs &a, long long k)
{
    if (!a.sc) return 1.0;
    const unsigned kk = (unsigned)k;
    const unsigned node = kk < a.nlr ? kk / (unsigned)a.nxu : (unsigned)a.Vnl + (kk - a.nlr) / (unsigned)a.nx;
    return a.sc[node];
}

__device__ __forceinline__ double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double wave_red(double x, bool is_max)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(x, off, 64);
        x = is_max ? fmax(x, o) : x + o;
    }
    return x;
}

// Block-reduce acc[0..nv) and store slot v of this block at part[v*nblocks+b].
template <int NV>
__device__ void block_store(double (&acc)[NV], int nv, double *part, int nblocks)
{
    __shared__ double red[kVB / 64][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            const double x = wave_red(acc[v], v < kNMax);
            if (lane == 0) red[w][v] = x;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        double x = red[0][v];
        for (int k = 1; k < kVB / 64; ++k) x = (v < kNMax) ? fmax(x, red[k][v]) : x + red[k][v];
        part[(long long)v * nblocks + blockIdx.x] = x;
    }
}

// Finalize-side reduction of nv slots over all blocks (fixed order) into out.
__device__ void reduce_partials(const double *part, int nblocks, int nv, double *out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int v = w; v < nv; v += nw) {
        const bool mx = v < kNMax;
        double x = mx ? 0.0 : 0.0;
        for (int b = lane; b < nblocks; b += 64) {
            const double p = part[(long long)v * nblocks + b];
            x = mx ? fmax(x, p) : x + p;
        }
        x = wave_red(x, mx);
        if (lane == 0) out[v] = x;
    }
    __syncthreads();
}

template <int MEMCAP>
__device__ __forceinline__ void pair_dots(const VecArgs &a, long long k, double s, double q, double g,
                                          bool have_pair, int cnt, int fslot, const int *order,
                                          double (&acc)[nv_pair(MEMCAP)])
{
    if (have_pair) {
        a.S[(long long)fslot * a.m + k] = s;
        a.Q[(long long)fslot * a.m + k] = q;
        acc[PB + 0] += s * q;
        acc[PB + 1] += s * s;
        acc[PB + 2] += q * q;
        acc[PB + 3] += s * g;
        acc[PB + 4] += q * g;
    }
    acc[PB + 5] += g * g;
#pragma unroll
    for (int j = 0; j < MEMCAP; ++j) {
        if (j < cnt) {
            const double sj = a.S[(long long)order[j] * a.m + k];
            const double qj = a.Q[(long long)order[j] * a.m + k];
            if (have_pair) {
                acc[PB + 6 + 5 * j + 0] += s * qj;
                acc[PB + 6 + 5 * j + 1] += sj * q;
                acc[PB + 6 + 5 * j + 2] += q * qj;
            }
            acc[PB + 6 + 5 * j + 3] += sj * g;
            acc[PB + 6 + 5 * j + 4] += qj * g;
        }
    }
}

// Residual pass.  PAIR (NAMA): g = R and the L-BFGS pair/dots.
template <bool PAIR, int MEMCAP>
__global__ void __launch_bounds__(kVB) resid_kernel(VecArgs a)
{
    const Ctl *c = a.ctl;
    if (c->done) return;
    constexpr int NV = PAIR ? nv_pair(MEMCAP) : PB;
    double acc[nv_pair(MEMCAP)];
#pragma unroll
    for (int v = 0; v < nv_pair(MEMCAP); ++v) acc[v] = 0.0;
    const double lam = c->lam;
    const bool have_pair = PAIR && c->have_pair;
    const int cnt = c->cnt, fslot = c->free_slot;
    int order[MEMCAP > 0 ? MEMCAP : 1];
#pragma unroll
    for (int j = 0; j < MEMCAP; ++j) order[j] = c->order[j];
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        const double s = row_scale(a, k);
        const double h = s * a.hx[k];
        const double yk = a.y[k];
        const double z = clampd(yk / lam + h, s * a.lo[k], s * a.hi[k]);
        const double R = z - h;
        a.r[k] = R;
        const double aR = fabs(R);
        acc[R_MAX] = fmax(acc[R_MAX], aR);
        acc[R_MAXU] = fmax(acc[R_MAXU], aR / s);
        acc[R_SS] += R * R;
        acc[R_BAD] += isfinite(R) ? 0.0 : 1.0;
        if constexpr (PAIR) {
            const double sv = have_pair ? yk - a.yp[k] : 0.0;
            const double qv = have_pair ? R - a.rp[k] : 0.0;
            pair_dots<MEMCAP>(a, k, sv, qv, R, have_pair, cnt, fslot, order, acc);
        }
    }
    block_store<nv_pair(MEMCAP)>(acc, NV, a.part, a.nblocks);
}

// MINFBE gradient of the FBE and the L-BFGS pair/dots.
template <int MEMCAP>
__global__ void __launch_bounds__(kVB) grad_kernel(VecArgs a)
{
    const Ctl *c = a.ctl;
    if (c->done) return;
    double acc[nv_pair(MEMCAP)];
#pragma unroll
    for (int v = 0; v < nv_pair(MEMCAP); ++v) acc[v] = 0.0;
    const double lam = c->lam;
    const bool have_pair = c->have_pair;
    const int cnt = c->cnt, fslot = c->free_slot;
    int order[MEMCAP > 0 ? MEMCAP : 1];
#pragma unroll
    for (int j = 0; j < MEMCAP; ++j) order[j] = c->order[j];
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        const double s = row_scale(a, k);
        const double g = a.r[k] + lam * s * a.hr[k];
        a.g[k] = g;
        const double sv = have_pair ? a.y[k] - a.yp[k] : 0.0;
        const double qv = have_pair ? g - a.gp[k] : 0.0;
        pair_dots<MEMCAP>(a, k, sv, qv, g, have_pair, cnt, fslot, order, acc);
    }
    block_store<nv_pair(MEMCAP)>(acc, nv_pair(MEMCAP), a.part, a.nblocks);
}

template <int MEMCAP>
__global__ void __launch_bounds__(kVB) combine_kernel(VecArgs a)
{
    const Ctl *c = a.ctl;
    if (c->done) return;
    const int cnt = c->cnt;
    const double gam = c->gamma;
    int order[MEMCAP > 0 ? MEMCAP : 1];
    double cs[MEMCAP > 0 ? MEMCAP : 1], cq[MEMCAP > 0 ? MEMCAP : 1];
#pragma unroll
    for (int j = 0; j < MEMCAP; ++j) { order[j] = c->order[j]; cs[j] = c->coefS[j]; cq[j] = c->coefQ[j]; }
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        double v = gam * a.g[k];
#pragma unroll
        for (int j = 0; j < MEMCAP; ++j)
            if (j < cnt)
                v += cs[j] * a.S[(long long)order[j] * a.m + k] + cq[j] * a.Q[(long long)order[j] * a.m + k];
        a.r[k] = -v;  // a.r points at the direction buffer here
    }
}

// All trial steps in one pass; slot nu holds sum over rows of the change of
// the FBE at w(tau_nu) relative to y.
__global__ void __launch_bounds__(kVB) ls_kernel(VecArgs a)
{
    const Ctl *c = a.ctl;
    if (c->done) return;
    const double lam = c->lam;
    const int numax = c->nu_max;
    const bool nama = a.method == 1;
    double acc[kNuCap + 2];
#pragma unroll
    for (int v = 0; v < kNuCap + 2; ++v) acc[v] = 0.0;
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        const double s = row_scale(a, k);
        const double lo = s * a.lo[k], hi = s * a.hi[k];
        const double yk = a.y[k], rk = a.rp[k], dk = a.d[k];
        const double ah = s * a.hx[k];
        const double br = nama ? s * a.hr[k] : 0.0;
        const double bd = s * a.hd[k];
        const double ey = yk * (rk + ah) - 0.5 * lam * rk * rk;
        double tau = 1.0;
#pragma unroll
        for (int nu = 0; nu <= kNuCap; ++nu) {
            if (nu <= numax) {
                const double cr = nama ? -(1.0 - tau) * lam : 0.0;
                const double dl = cr * rk + tau * dk;     // w - y
                const double hd = cr * br + tau * bd;     // s H xhat(w - y)
                const double w = yk + dl, hw = ah + hd;
                const double zw = clampd(w / lam + hw, lo, hi);
                const double Rw = zw - hw;
                acc[nu] += -ah * dl - 0.5 * dl * hd + w * zw - 0.5 * lam * Rw * Rw - ey;
            }
            tau *= 0.5;
        }
    }
    // slot layout for block_store: no max slots are used here, keep sums
    double packed[kNuCap + 2 + kNMax];
#pragma unroll
    for (int v = 0; v < kNMax; ++v) packed[v] = 0.0;
#pragma unroll
    for (int v = 0; v < kNuCap + 2; ++v) packed[kNMax + v] = acc[v];
    block_store<kNuCap + 2 + kNMax>(packed, kNMax + numax + 1, a.part, a.nblocks);
}

__global__ void __launch_bounds__(kVB) update_kernel(VecArgs a)
{
    const Ctl *c = a.ctl;
    if (c->done) return;
    const double lam = c->lam, tau = c->tau, cr = c->cr;
    const bool nama = a.method == 1;
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        const double s = row_scale(a, k);
        const double dl = cr * a.rp[k] + tau * a.d[k];
        const double hd = (nama ? cr * s * a.hr[k] : 0.0) + tau * s * a.hd[k];
        const double w = a.y[k] + dl, hw = s * a.hx[k] + hd;
        const double zw = clampd(w / lam + hw, s * a.lo[k], s * a.hi[k]);
        a.yn[k] = w - lam * (zw - hw);
    }
}

// ---------------------------- finalize kernels ---------------------------
__device__ void finish_residual(Ctl *c, const double *red)
{
    c->sweeps_aff++;
    c->res = red[R_MAX];
    c->resu = red[R_MAXU];
    c->rr = red[R_SS];
    if (red[R_BAD] > 0.0 || !isfinite(red[R_SS])) { c->done = 1; c->status = STOTREE_ERR_NUMERIC; }
    else if (red[R_MAX] <= c->eps) { c->done = 1; c->status = STOTREE_OK; }
    else if (c->iter >= c->max_iter) { c->done = 1; c->status = STOTREE_NOT_CONVERGED; }
}

// Cautious push of the candidate pair (Li and Fukushima: push when
// <s,q> > eps' ||s||^2 ||g_prev||^2) and the compact-form coefficients of
// d = -B g = -(gamma g + S p1 + gamma Q p2).
__device__ void lbfgs_update(Ctl *c, const double *red)
{
    int cnt = c->cnt, fs = c->free_slot;
    const int mem = c->mem;
    double sg[kMemMax + 1], qg[kMemMax + 1];
    for (int j = 0; j < cnt; ++j) {
        sg[c->order[j]] = red[PB + 6 + 5 * j + 3];
        qg[c->order[j]] = red[PB + 6 + 5 * j + 4];
    }
    if (c->have_pair) {
        const double sq = red[PB + 0], ss = red[PB + 1], qq = red[PB + 2];
        if (sq > c->eps_curv * ss * c->gg_prev && isfinite(sq) && qq > 0.0) {
            c->SY[fs][fs] = sq;
            c->QQ[fs][fs] = qq;
            for (int j = 0; j < cnt; ++j) {
                const int oj = c->order[j];
                c->SY[fs][oj] = red[PB + 6 + 5 * j + 0];
                c->SY[oj][fs] = red[PB + 6 + 5 * j + 1];
                c->QQ[fs][oj] = c->QQ[oj][fs] = red[PB + 6 + 5 * j + 2];
            }
            sg[fs] = red[PB + 3];
            qg[fs] = red[PB + 4];
            int evicted = -1;
            if (cnt == mem) {
                evicted = c->order[0];
                for (int j = 1; j < cnt; ++j) c->order[j - 1] = c->order[j];
                --cnt;
            }
            c->order[cnt++] = fs;
            if (evicted >= 0) {
                fs = evicted;
            } else {
                for (int sl = 0; sl <= mem; ++sl) {
                    bool used = false;
                    for (int j = 0; j < cnt; ++j) used |= (c->order[j] == sl);
                    if (!used) { fs = sl; break; }
                }
            }
            c->pushes++;
        } else {
            c->skips++;
        }
    }
    c->cnt = cnt;
    c->free_slot = fs;
    c->have_pair = 1;
    c->gg_prev = red[PB + 5];
    if (cnt == 0) {
        c->gamma = 1.0;
        return;
    }
    const int n = c->order[cnt - 1];
    const double gam = c->SY[n][n] / c->QQ[n][n];
    double u1[kMemMax], u2[kMemMax], p1[kMemMax], p2[kMemMax], t[kMemMax];
    for (int i = 0; i < cnt; ++i) {
        u1[i] = sg[c->order[i]];
        u2[i] = gam * qg[c->order[i]];
    }
    auto Rm = [&](int i, int j) { return c->SY[c->order[i]][c->order[j]]; };
    for (int i = cnt - 1; i >= 0; --i) {          // p2 = -R^{-1} u1
        double v = -u1[i];
        for (int j = i + 1; j < cnt; ++j) v -= Rm(i, j) * p2[j];
        p2[i] = v / Rm(i, i);
    }
    for (int i = 0; i < cnt; ++i) {               // t = (D + gamma Q'Q)(-p2) - u2
        double v = -Rm(i, i) * p2[i];
        for (int j = 0; j < cnt; ++j) v -= gam * c->QQ[c->order[i]][c->order[j]] * p2[j];
        t[i] = v - u2[i];
    }
    for (int i = 0; i < cnt; ++i) {               // p1 = R^{-T} t
        double v = t[i];
        for (int j = 0; j < i; ++j) v -= Rm(j, i) * p1[j];
        p1[i] = v / Rm(i, i);
    }
    for (int i = 0; i < cnt; ++i) {
        c->coefS[i] = p1[i];
        c->coefQ[i] = gam * p2[i];
    }
    c->gamma = gam;
}

__global__ void __launch_bounds__(kVB) fin_resid_kernel(Ctl *c, const double *part, int nblocks, int with_pair)
{
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, with_pair ? nv_pair(c->mem) : PB, red);
    if (threadIdx.x != 0) return;
    finish_residual(c, red);
    if (!c->done && with_pair) lbfgs_update(c, red);
}

__global__ void __launch_bounds__(kVB) fin_grad_kernel(Ctl *c, const double *part, int nblocks)
{
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, nv_pair(c->mem), red);
    if (threadIdx.x != 0) return;
    c->sweeps_hom++;
    lbfgs_update(c, red);
}

__global__ void __launch_bounds__(kVB) fin_ls_kernel(Ctl *c, const double *part, int nblocks)
{
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, kNMax + c->nu_max + 1, red);
    if (threadIdx.x != 0) return;
    int acc = -1;
    for (int nu = 0; nu <= c->nu_max; ++nu) {
        const double dphi = red[kNMax + nu];
        c->ls_val[nu] = dphi;
        if (isfinite(dphi) && dphi <= 0.0) { acc = nu; break; }
    }
    c->accepted_nu = acc;
    c->tau = acc >= 0 ? ldexp(1.0, -acc) : 0.0;
    c->cr = c->method == 1 ? -(1.0 - c->tau) * c->lam : 0.0;
    c->ls_trials += acc >= 0 ? acc + 1 : c->nu_max + 1;
    c->sweeps_hom += c->method == 1 ? 2 : 1;
    c->iter++;
}

// ----------------------------- power iteration ---------------------------
__global__ void __launch_bounds__(kVB) power_step_kernel(VecArgs a)
{
    // w = -s H xhat(s v) (the dual Hessian applied to v), slots: <v,w>, ||w||^2
    double acc[kNMax + 2] = {0.0, 0.0, 0.0, 0.0};
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB) {
        const double s = row_scale(a, k);
        const double w = -s * a.hx[k];
        acc[kNMax + 0] += a.y[k] * w;
        acc[kNMax + 1] += w * w;
        a.r[k] = w;
    }
    block_store<kNMax + 2>(acc, kNMax + 2, a.part, a.nblocks);
}

__global__ void __launch_bounds__(kVB) power_fin_kernel(Ctl *c, const double *part, int nblocks)
{
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, kNMax + 2, red);
    if (threadIdx.x != 0) return;
    c->L = red[kNMax + 0];
    const double nw = sqrt(red[kNMax + 1]);
    c->inv_norm = nw > 0.0 ? 1.0 / nw : 0.0;
}

__global__ void __launch_bounds__(kVB) power_scale_kernel(VecArgs a)
{
    const double inv = a.ctl->inv_norm;
    for (long long k = blockIdx.x * (long long)kVB + threadIdx.x; k < a.m; k += (long long)a.nblocks * kVB)
        a.yn[k] = a.r[k] * inv;
}

__global__ void fill_kernel(double *v, long long n, double val)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        v[k] = val;
}

// ------------------------------- host side -------------------------------
int ensure_solver_ws(tree_factors *f, int mem)
{
    SolverWS &w = f->sws;
    const long long m = f->m;
    const int nblocks = (int)std::min<long long>(1024, (m + kVB - 1) / kVB);
    if (w.buf && w.mem >= mem) return STOTREE_OK;
    if (w.buf) { (void)hipFree(w.buf); w.buf = nullptr; w.bytes = 0; }
    const long long nvec = 9 + 2LL * (mem + 1);
    const size_t bytes = sizeof(double) * ((size_t)nvec * m + (size_t)kNVMax * nblocks) + sizeof(Ctl) + 256;
    STOTREE_HIP(hipMalloc(&w.buf, bytes));
    w.bytes = bytes;
    w.mem = mem;
    w.nblocks = nblocks;
    double *p = w.buf;
    w.y[1] = p; p += m;
    w.r[0] = p; p += m;
    w.r[1] = p; p += m;
    w.g[0] = p; p += m;
    w.g[1] = p; p += m;
    w.hx = p; p += m;
    w.hr2 = p; p += 2 * m;  // hr, hd
    w.d = p; p += m;
    w.S = p; p += (long long)(mem + 1) * m;
    w.Qv = p; p += (long long)(mem + 1) * m;
    w.partials = p; p += (size_t)kNVMax * nblocks;
    w.ctl = p;
    return STOTREE_OK;
}

VecArgs vec_args(const tree_factors *f)
{
    VecArgs a{};
    a.m = f->m;
    a.nlr = (unsigned)((long long)f->Vnl * (f->nx + f->nu));
    a.nxu = f->nx + f->nu;
    a.nx = f->nx;
    a.Vnl = f->Vnl;
    a.sc = f->precondition ? f->sc : nullptr;
    a.lo = f->lo;
    a.hi = f->hi;
    a.ctl = reinterpret_cast<Ctl *>(f->sws.ctl);
    a.part = f->sws.partials;
    a.nblocks = f->sws.nblocks;
    return a;
}

// Sweep arguments writing H x (dual layout) for nrhs right-hand sides whose
// inputs/outputs are at (y, y + y_rs) and (out, out + o_rs).
SweepArgs dual_layout_sweep(const tree_factors *f, int affine, const double *x0, const double *y,
                            long long y_rs, double *out, long long o_rs, const int *done)
{
    SweepArgs a = sweep_args(f, affine);
    a.x0 = x0; a.x0_rs = 0;
    a.y = y; a.y_rs = y_rs;
    a.xo = out; a.xo_s = f->nx + f->nu;
    a.xl = out + (long long)f->Vnl * (f->nx + f->nu); a.xl_s = f->nx;
    a.uo = out + f->nx; a.uo_s = f->nx + f->nu;
    a.xo_rs = o_rs; a.uo_rs = o_rs;
    a.done = done;
    return a;
}

template <int MEMCAP>
hipError_t enqueue_iteration(const tree_factors *f, const double *x0, double *ybuf[2], int k, int method,
                             hipStream_t st)
{
    const SolverWS &w = f->sws;
    VecArgs a = vec_args(f);
    a.method = method;
    Ctl *ctl = a.ctl;
    const int *done = &ctl->done;
    const dim3 grid(a.nblocks), blk(kVB);
    double *y = ybuf[k & 1], *yn = ybuf[(k + 1) & 1];
    double *r = w.r[k & 1], *rp = w.r[(k + 1) & 1];
    double *g = w.g[k & 1], *gp = w.g[(k + 1) & 1];
    double *hr = w.hr2, *hd = w.hr2 + f->m;
    hipError_t e;
    // x(y) -> H x
    if ((e = launch_sweep_tree(f, dual_layout_sweep(f, 1, x0, y, 0, w.hx, 0, done), 1, st))) return e;
    a.y = y; a.yp = yn; a.hx = w.hx; a.rp = rp; a.r = r;
    a.S = w.S; a.Q = w.Qv;
    if (method == 1) {
        hipLaunchKernelGGL((resid_kernel<true, MEMCAP>), grid, blk, 0, st, a);
        hipLaunchKernelGGL(fin_resid_kernel, dim3(1), blk, 0, st, ctl, a.part, a.nblocks, 1);
        VecArgs cb = a;
        cb.g = r;           // g = R
        cb.r = w.d;         // output direction
        cb.S = w.S; cb.Q = w.Qv;
        hipLaunchKernelGGL((combine_kernel<MEMCAP>), grid, blk, 0, st, cb);
        // x-hat(r) and x-hat(d) in one two-right-hand-side sweep (p-NAMA)
        if ((e = launch_sweep_tree(f, dual_layout_sweep(f, 0, nullptr, r, w.d - r, hr, hd - hr, done), 2, st)))
            return e;
        VecArgs la = vec_args(f);
        la.method = 1;
        la.y = y; la.rp = r; la.d = w.d; la.hx = w.hx; la.hr = hr; la.hd = hd; la.yn = yn;
        hipLaunchKernelGGL(ls_kernel, grid, blk, 0, st, la);
        hipLaunchKernelGGL(fin_ls_kernel, dim3(1), blk, 0, st, ctl, a.part, a.nblocks);
        hipLaunchKernelGGL(update_kernel, grid, blk, 0, st, la);
    } else {
        hipLaunchKernelGGL((resid_kernel<false, 0>), grid, blk, 0, st, a);
        hipLaunchKernelGGL(fin_resid_kernel, dim3(1), blk, 0, st, ctl, a.part, a.nblocks, 0);
        // grad phi = R + lambda s H xhat(s R)
        if ((e = launch_sweep_tree(f, dual_layout_sweep(f, 0, nullptr, r, 0, hr, 0, done), 1, st))) return e;
        VecArgs ga = a;
        ga.hr = hr; ga.g = g; ga.gp = gp; ga.S = w.S; ga.Q = w.Qv;
        hipLaunchKernelGGL((grad_kernel<MEMCAP>), grid, blk, 0, st, ga);
        hipLaunchKernelGGL(fin_grad_kernel, dim3(1), blk, 0, st, ctl, a.part, a.nblocks);
        VecArgs cb = a;
        cb.g = g; cb.r = w.d; cb.S = w.S; cb.Q = w.Qv;
        hipLaunchKernelGGL((combine_kernel<MEMCAP>), grid, blk, 0, st, cb);
        if ((e = launch_sweep_tree(f, dual_layout_sweep(f, 0, nullptr, w.d, 0, hd, 0, done), 1, st))) return e;
        VecArgs la = vec_args(f);
        la.method = 0;
        la.y = y; la.rp = r; la.d = w.d; la.hx = w.hx; la.hr = hr; la.hd = hd; la.yn = yn;
        hipLaunchKernelGGL(ls_kernel, grid, blk, 0, st, la);
        hipLaunchKernelGGL(fin_ls_kernel, dim3(1), blk, 0, st, ctl, a.part, a.nblocks);
        hipLaunchKernelGGL(update_kernel, grid, blk, 0, st, la);
    }
    return hipGetLastError();
}

using IterFn = hipError_t (*)(const tree_factors *, const double *, double *[2], int, int, hipStream_t);

IterFn pick_iter(int mem)
{
    if (mem <= 4) return enqueue_iteration<4>;
    if (mem <= 8) return enqueue_iteration<8>;
    return enqueue_iteration<16>;
}

}  // namespace

int lipschitz(const tree_factors *fc, int iters, double *L, hipStream_t st)
{
    tree_factors *f = const_cast<tree_factors *>(fc);
    int rc = ensure_solver_ws(f, f->sws.buf ? f->sws.mem : 1);
    if (rc) return rc;
    if ((rc = ensure_sweep_ws(f, 2))) return rc;
    const SolverWS &w = f->sws;
    VecArgs a = vec_args(f);
    const dim3 grid(a.nblocks), blk(kVB);
    double *v = w.g[0], *wv = w.g[1], *hv = w.hx;
    hipLaunchKernelGGL(fill_kernel, dim3(1024), blk, 0, st, v, f->m, 1.0 / std::sqrt((double)f->m));
    for (int it = 0; it < iters; ++it) {
        hipError_t e = launch_sweep_tree(f, dual_layout_sweep(f, 0, nullptr, v, 0, hv, 0, nullptr), 1, st);
        if (e != hipSuccess) { set_error(std::string("dual_lipschitz: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
        VecArgs pa = a;
        pa.y = v; pa.hx = hv; pa.r = wv; pa.yn = v;
        hipLaunchKernelGGL(power_step_kernel, grid, blk, 0, st, pa);
        hipLaunchKernelGGL(power_fin_kernel, dim3(1), blk, 0, st, a.ctl, a.part, a.nblocks);
        hipLaunchKernelGGL(power_scale_kernel, grid, blk, 0, st, pa);
    }
    STOTREE_HIP(hipGetLastError());
    double Lh = 0.0;
    STOTREE_HIP(hipMemcpyAsync(&Lh, &a.ctl->L, sizeof(double), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    *L = Lh;
    return STOTREE_OK;
}

int solve(const tree_factors *fc, const double *x0, const solver_opts *opts_in, double *y_io, double *x,
          double *u, solver_info *info, hipStream_t st, int method)
{
    tree_factors *f = const_cast<tree_factors *>(fc);
    solver_opts o{0.0, 1e-6, 1e-12, 5, 10, 1000, 1};
    if (opts_in) o = *opts_in;
    if (o.mem < 1 || o.mem > kMemMax || o.nu_max < 0 || o.nu_max > kNuCap || o.max_iter < 0 ||
        o.check_every < 1 || !(o.eps >= 0.0) || !(o.lambda >= 0.0) || !(o.eps_curv >= 0.0)) {
        set_error("solve: options out of range (mem 1..16, nu_max 0..30, check_every >= 1)");
        return STOTREE_ERR_ARG;
    }
    int rc = ensure_solver_ws(f, o.mem);
    if (rc) return rc;
    if ((rc = ensure_sweep_ws(f, 2))) return rc;
    double lam = o.lambda;
    if (lam == 0.0) {
        double L = 0.0;
        if ((rc = lipschitz(f, 100, &L, st))) return rc;
        if (!(L > 0.0) || !std::isfinite(L)) { set_error("solve: could not estimate L"); return STOTREE_ERR_NUMERIC; }
        lam = 1.0 / (1.1 * L);
    }
    Ctl h{};
    h.done = 0; h.status = STOTREE_NOT_CONVERGED; h.iter = 0; h.have_pair = 0;
    h.cnt = 0; h.free_slot = 0;
    h.max_iter = o.max_iter; h.mem = o.mem; h.nu_max = o.nu_max; h.method = method;
    h.lam = lam; h.eps = o.eps; h.eps_curv = o.eps_curv; h.gamma = 1.0;
    const SolverWS &w = f->sws;
    Ctl *dctl = reinterpret_cast<Ctl *>(w.ctl);
    STOTREE_HIP(hipMemcpyAsync(dctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, st));
    double *ybuf[2] = {y_io, w.y[1]};
    IterFn iter = pick_iter(o.mem);
    int k = 0, done = 0;
    while (!done && k <= o.max_iter) {
        for (int c = 0; c < o.check_every && k <= o.max_iter; ++c, ++k) {
            hipError_t e = iter(f, x0, ybuf, k, method, st);
            if (e != hipSuccess) { set_error(std::string("solve: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
        }
        STOTREE_HIP(hipMemcpyAsync(&done, &dctl->done, sizeof(int), hipMemcpyDeviceToHost, st));
        STOTREE_HIP(hipStreamSynchronize(st));
    }
    STOTREE_HIP(hipMemcpyAsync(&h, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    double *yf = ybuf[h.iter & 1];
    if (yf != y_io) STOTREE_HIP(hipMemcpyAsync(y_io, yf, sizeof(double) * f->m, hipMemcpyDeviceToDevice, st));
    // x(y) at the returned dual, in the caller's layout
    SweepArgs a = sweep_args(f, 1);
    a.x0 = x0; a.y = y_io;
    a.xo = x; a.xo_s = f->nx; a.xl = x + (long long)f->Vnl * f->nx; a.xl_s = f->nx;
    a.uo = u; a.uo_s = f->nu;
    hipError_t e = launch_sweep_tree(f, a, 1, st);
    if (e != hipSuccess) { set_error(std::string("solve: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
    STOTREE_HIP(hipStreamSynchronize(st));
    info->iters = h.iter;
    info->sweeps_affine = h.sweeps_aff + 1;
    info->sweeps_hom = h.sweeps_hom;
    info->ls_trials = h.ls_trials;
    info->lbfgs_push = h.pushes;
    info->lbfgs_skip = h.skips;
    info->status = h.status;
    info->res_scaled_inf = h.res;
    info->res_unscaled_inf = h.resu;
    info->lambda = lam;
    if (h.status == STOTREE_ERR_NUMERIC) set_error("solve: non-finite values in the iterates");
    return h.status;
}

}  // namespace stotree
