// Device-resident dual MINFBE (Algorithm 1) and NAMA (Algorithm 2) of
// arXiv 2107.01745, Sec. III-B/III-C, in the preconditioned dual variables of
// Sec. III-E when the handle asks for it.  A batched handle runs every
// instance in the same launches: each block of a vector pass belongs to one
// instance, each instance has its own control block (step, L-BFGS memory,
// stop flag), and finished instances are skipped by every kernel.
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
constexpr int kNuDefault = 10; // default nu_max
constexpr int kVB = 256;      // threads per block of the vector kernels

// reduction slots
constexpr int R_MAX = 0, R_MAXU = 1, R_SS = 2, R_BAD = 3, PB = 4;
constexpr int kNMax = 2;  // slots [0, kNMax) are max-reduced, the rest summed
constexpr int nv_pair(int memcap) { return PB + 6 + 5 * memcap; }
constexpr int kNVMax = nv_pair(kMemMax) > kNuCap + 2 ? nv_pair(kMemMax) : kNuCap + 2;

struct Ctl {
    int done, status, iter, have_pair;
    int first_blk, nblk, pad0, pad1;
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
    const InstDesc *inst;
    const int *blk;  // per block: instance, block within the instance, blocks of the instance
    const double *sc, *lo, *hi;
    Ctl *ctl;
    int *ndone;
    long long m_tot;
    double *part;
    int nblocks, method;
    const double *y, *yp, *hx, *rp, *gp, *hr, *hd, *d;
    double *r, *g, *S, *Q, *yn;
};

// The rows a block visits: rows lb*kVB + tid + n*nblk*kVB of its instance.
struct BlockRows {
    int b, lb, nb;
    InstDesc I;
    unsigned nlr;  // rows owned by non-leaf nodes
};

__device__ __forceinline__ BlockRows block_rows(const VecArgs &a)
{
    BlockRows br;
    br.b = a.blk[3 * blockIdx.x];
    br.lb = a.blk[3 * blockIdx.x + 1];
    br.nb = a.blk[3 * blockIdx.x + 2];
    br.I = a.inst[br.b];
    br.nlr = (unsigned)((long long)br.I.Vnl * (br.I.nx + br.I.nu));
    return br;
}

// sqrt(pi) of the node owning local row k (1 without preconditioning).
__device__ __forceinline__ double row_scale(const VecArgs &a, const BlockRows &br, long long k)
{
    if (!a.sc) return 1.0;
    const unsigned kk = (unsigned)k;
    const unsigned node = kk < br.nlr ? kk / (unsigned)(br.I.nx + br.I.nu)
                                      : (unsigned)br.I.Vnl + (kk - br.nlr) / (unsigned)br.I.nx;
    return a.sc[br.I.sc + node];
}

#define FOR_BLOCK_ROWS(br, kl, k)                                                             \
    for (long long kl = (long long)(br).lb * kVB + threadIdx.x, k = (br).I.y + kl; kl < (br).I.m; \
         kl += (long long)(br).nb * kVB, k = (br).I.y + kl)

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

// Finalize-side reduction of nv slots over blocks [first, first+count) (fixed
// order) into out.
__device__ void reduce_partials(const double *part, int nblocks, int first, int count, int nv, double *out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int v = w; v < nv; v += nw) {
        const bool mx = v < kNMax;
        double x = 0.0;
        for (int b = first + lane; b < first + count; b += 64) {
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
        a.S[(long long)fslot * a.m_tot + k] = s;
        a.Q[(long long)fslot * a.m_tot + k] = q;
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
            const double sj = a.S[(long long)order[j] * a.m_tot + k];
            const double qj = a.Q[(long long)order[j] * a.m_tot + k];
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
    const BlockRows br = block_rows(a);
    const Ctl *c = a.ctl + br.b;
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
    FOR_BLOCK_ROWS(br, kl, k) {
        const double s = row_scale(a, br, kl);
        const double h = s * a.hx[k];
        const double yk = a.y[k];
        const double z = clampd(yk / lam + h, s * a.lo[br.I.box + kl], s * a.hi[br.I.box + kl]);
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
    const BlockRows br = block_rows(a);
    const Ctl *c = a.ctl + br.b;
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
    FOR_BLOCK_ROWS(br, kl, k) {
        const double s = row_scale(a, br, kl);
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
    const BlockRows br = block_rows(a);
    const Ctl *c = a.ctl + br.b;
    if (c->done) return;
    const int cnt = c->cnt;
    const double gam = c->gamma;
    int order[MEMCAP > 0 ? MEMCAP : 1];
    double cs[MEMCAP > 0 ? MEMCAP : 1], cq[MEMCAP > 0 ? MEMCAP : 1];
#pragma unroll
    for (int j = 0; j < MEMCAP; ++j) { order[j] = c->order[j]; cs[j] = c->coefS[j]; cq[j] = c->coefQ[j]; }
    FOR_BLOCK_ROWS(br, kl, k) {
        double v = gam * a.g[k];
#pragma unroll
        for (int j = 0; j < MEMCAP; ++j)
            if (j < cnt)
                v += cs[j] * a.S[(long long)order[j] * a.m_tot + k] + cq[j] * a.Q[(long long)order[j] * a.m_tot + k];
        a.r[k] = -v;  // a.r points at the direction buffer here
    }
}

// All trial steps in one pass; slot nu holds sum over rows of the change of
// the FBE at w(tau_nu) relative to y.  NUC: the largest nu_max the variant
// serves (its accumulators, and so its register demand, scale with it).
template <int NUC>
__global__ void __launch_bounds__(kVB) ls_kernel(VecArgs a)
{
    const BlockRows br = block_rows(a);
    const Ctl *c = a.ctl + br.b;
    if (c->done) return;
    const double lam = c->lam;
    const int numax = c->nu_max;
    const bool nama = a.method == 1;
    double acc[NUC + 1];
#pragma unroll
    for (int v = 0; v < NUC + 1; ++v) acc[v] = 0.0;
    FOR_BLOCK_ROWS(br, kl, k) {
        const double s = row_scale(a, br, kl);
        const double lo = s * a.lo[br.I.box + kl], hi = s * a.hi[br.I.box + kl];
        const double yk = a.y[k], rk = a.rp[k], dk = a.d[k];
        const double ah = s * a.hx[k];
        const double brk = nama ? s * a.hr[k] : 0.0;
        const double bd = s * a.hd[k];
        const double ey = yk * (rk + ah) - 0.5 * lam * rk * rk;
        double tau = 1.0;
#pragma unroll
        for (int nu = 0; nu <= NUC; ++nu) {
            if (nu <= numax) {
                const double cr = nama ? -(1.0 - tau) * lam : 0.0;
                const double dl = cr * rk + tau * dk;     // w - y
                const double hd = cr * brk + tau * bd;    // s H xhat(w - y)
                const double w = yk + dl, hw = ah + hd;
                const double zw = clampd(w / lam + hw, lo, hi);
                const double Rw = zw - hw;
                acc[nu] += -ah * dl - 0.5 * dl * hd + w * zw - 0.5 * lam * Rw * Rw - ey;
            }
            tau *= 0.5;
        }
    }
    // slots [0, kNMax) are the max-reduced ones; the sums follow them
    double packed[kNMax + NUC + 1];
#pragma unroll
    for (int v = 0; v < kNMax; ++v) packed[v] = 0.0;
#pragma unroll
    for (int v = 0; v < NUC + 1; ++v) packed[kNMax + v] = acc[v];
    block_store<kNMax + NUC + 1>(packed, kNMax + NUC + 1, a.part, a.nblocks);
}

__global__ void __launch_bounds__(kVB) update_kernel(VecArgs a)
{
    const BlockRows br = block_rows(a);
    const Ctl *c = a.ctl + br.b;
    if (c->done) return;
    const double lam = c->lam, tau = c->tau, cr = c->cr;
    const bool nama = a.method == 1;
    FOR_BLOCK_ROWS(br, kl, k) {
        const double s = row_scale(a, br, kl);
        const double dl = cr * a.rp[k] + tau * a.d[k];
        const double hd = (nama ? cr * s * a.hr[k] : 0.0) + tau * s * a.hd[k];
        const double w = a.y[k] + dl, hw = s * a.hx[k] + hd;
        const double zw = clampd(w / lam + hw, s * a.lo[br.I.box + kl], s * a.hi[br.I.box + kl]);
        a.yn[k] = w - lam * (zw - hw);
    }
}

// ---------------------------- finalize kernels ---------------------------
// One block per instance; lane 0 of the block takes the scalar decisions.
__device__ void finish_residual(Ctl *c, const double *red, int *ndone)
{
    c->sweeps_aff++;
    c->res = red[R_MAX];
    c->resu = red[R_MAXU];
    c->rr = red[R_SS];
    if (red[R_BAD] > 0.0 || !isfinite(red[R_SS])) { c->done = 1; c->status = STOTREE_ERR_NUMERIC; }
    else if (red[R_MAX] <= c->eps) { c->done = 1; c->status = STOTREE_OK; }
    else if (c->iter >= c->max_iter) { c->done = 1; c->status = STOTREE_NOT_CONVERGED; }
    if (c->done) atomicAdd(ndone, 1);
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

__global__ void __launch_bounds__(kVB) fin_resid_kernel(Ctl *ctl, const double *part, int nblocks,
                                                        int with_pair, int *ndone)
{
    Ctl *c = ctl + blockIdx.x;
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, c->first_blk, c->nblk, with_pair ? nv_pair(c->mem) : PB, red);
    if (threadIdx.x != 0) return;
    finish_residual(c, red, ndone);
    if (!c->done && with_pair) lbfgs_update(c, red);
}

__global__ void __launch_bounds__(kVB) fin_grad_kernel(Ctl *ctl, const double *part, int nblocks)
{
    Ctl *c = ctl + blockIdx.x;
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, c->first_blk, c->nblk, nv_pair(c->mem), red);
    if (threadIdx.x != 0) return;
    c->sweeps_hom++;
    lbfgs_update(c, red);
}

__global__ void __launch_bounds__(kVB) fin_ls_kernel(Ctl *ctl, const double *part, int nblocks)
{
    Ctl *c = ctl + blockIdx.x;
    if (c->done) return;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, c->first_blk, c->nblk, kNMax + c->nu_max + 1, red);
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

// Final dual of every instance into the caller's buffer (buffer 0): the
// instances whose last iterate sits in buffer 1 are copied.
__global__ void __launch_bounds__(kVB) gather_final_kernel(VecArgs a)
{
    const BlockRows br = block_rows(a);
    if (!(a.ctl[br.b].iter & 1)) return;
    FOR_BLOCK_ROWS(br, kl, k) a.yn[k] = a.y[k];
}

// ----------------------------- power iteration ---------------------------
__global__ void __launch_bounds__(kVB) power_init_kernel(VecArgs a)
{
    const BlockRows br = block_rows(a);
    const double v = 1.0 / sqrt((double)br.I.m);
    FOR_BLOCK_ROWS(br, kl, k) a.yn[k] = v;
}

__global__ void __launch_bounds__(kVB) power_step_kernel(VecArgs a)
{
    // w = -s H xhat(s v) (the dual Hessian applied to v), slots: <v,w>, ||w||^2
    const BlockRows br = block_rows(a);
    double acc[kNMax + 2] = {0.0, 0.0, 0.0, 0.0};
    FOR_BLOCK_ROWS(br, kl, k) {
        const double s = row_scale(a, br, kl);
        const double w = -s * a.hx[k];
        acc[kNMax + 0] += a.y[k] * w;
        acc[kNMax + 1] += w * w;
        a.r[k] = w;
    }
    block_store<kNMax + 2>(acc, kNMax + 2, a.part, a.nblocks);
}

__global__ void __launch_bounds__(kVB) power_fin_kernel(Ctl *ctl, const double *part, int nblocks)
{
    Ctl *c = ctl + blockIdx.x;
    __shared__ double red[kNVMax];
    reduce_partials(part, nblocks, c->first_blk, c->nblk, kNMax + 2, red);
    if (threadIdx.x != 0) return;
    c->L = red[kNMax + 0];
    const double nw = sqrt(red[kNMax + 1]);
    c->inv_norm = nw > 0.0 ? 1.0 / nw : 0.0;
}

__global__ void __launch_bounds__(kVB) power_scale_kernel(VecArgs a)
{
    const BlockRows br = block_rows(a);
    const double inv = a.ctl[br.b].inv_norm;
    FOR_BLOCK_ROWS(br, kl, k) a.yn[k] = a.r[k] * inv;
}

// ------------------------------- host side -------------------------------
// need_g: the two FBE-gradient vectors (MINFBE only).
int ensure_solver_ws(tree_factors *f, int mem, bool need_g)
{
    SolverWS &w = f->sws;
    if (w.buf && w.mem >= mem && (w.has_g || !need_g)) return STOTREE_OK;
    if (w.buf) { (void)hipFree(w.buf); w.buf = nullptr; w.bytes = 0; }
    // blocks per instance: one per 1024 rows, at most 1024
    std::vector<int> blk;
    w.blk_first.assign(f->ninst, 0);
    for (int b = 0; b < f->ninst; ++b) {
        const long long m = f->inst[b].m;
        const int nb = (int)std::max<long long>(1, std::min<long long>(1024, (m + 4 * kVB - 1) / (4 * kVB)));
        w.blk_first[b] = (int)(blk.size() / 3);
        for (int l = 0; l < nb; ++l) { blk.push_back(b); blk.push_back(l); blk.push_back(nb); }
    }
    const int nblocks = (int)(blk.size() / 3);
    const long long m = f->m_tot;
    const long long nvec = (need_g ? 9 : 7) + 2LL * (mem + 1);
    const size_t vec_bytes = sizeof(double) * ((size_t)nvec * m + (size_t)kNVMax * nblocks);
    const size_t ctl_bytes = sizeof(Ctl) * (size_t)f->ninst;
    const size_t bytes = vec_bytes + ctl_bytes + sizeof(int) * (blk.size() + 1) + 512;
    STOTREE_HIP(hipMalloc(&w.buf, bytes));
    w.bytes = bytes;
    w.mem = mem;
    w.nblocks = nblocks;
    double *p = w.buf;
    w.y[1] = p; p += m;
    w.r[0] = p; p += m;
    w.r[1] = p; p += m;
    w.has_g = need_g;
    w.g[0] = w.g[1] = nullptr;
    if (need_g) {
        w.g[0] = p; p += m;
        w.g[1] = p; p += m;
    }
    w.hx = p; p += m;
    w.hr2 = p; p += 2 * m;  // hr, hd
    w.d = p; p += m;
    w.S = p; p += (long long)(mem + 1) * m;
    w.Qv = p; p += (long long)(mem + 1) * m;
    w.partials = p; p += (size_t)kNVMax * nblocks;
    w.ctl = p;
    char *q = reinterpret_cast<char *>(p) + ctl_bytes;
    w.blk = reinterpret_cast<int *>(q);
    w.ndone = w.blk + blk.size();
    STOTREE_HIP(hipMemcpy(w.blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice));
    return STOTREE_OK;
}

VecArgs vec_args(const tree_factors *f)
{
    VecArgs a{};
    a.inst = f->d_inst;
    a.blk = f->sws.blk;
    a.sc = f->precondition ? f->sc : nullptr;
    a.lo = f->lo;
    a.hi = f->hi;
    a.ctl = reinterpret_cast<Ctl *>(f->sws.ctl);
    a.ndone = f->sws.ndone;
    a.m_tot = f->m_tot;
    a.part = f->sws.partials;
    a.nblocks = f->sws.nblocks;
    return a;
}

// Sweep arguments writing H x (dual layout) for right-hand sides whose
// inputs/outputs are at (y, y + y_rs) and (out, out + o_rs).
SweepArgs dual_layout_sweep(const tree_factors *f, int affine, const double *x0, const double *y,
                            long long y_rs, double *out, long long o_rs, const Ctl *ctl)
{
    SweepArgs a = sweep_args(f, affine);
    a.x0 = x0; a.x0_rs = 0;
    a.y = y; a.y_rs = y_rs;
    a.xo = out; a.xo_rs = o_rs;
    a.dual_out = 1;
    a.done = ctl ? &ctl->done : nullptr;
    a.done_stride = (int)(sizeof(Ctl) / sizeof(int));
    return a;
}

template <int MEMCAP, int NUC>
hipError_t enqueue_iteration(const tree_factors *f, const double *x0, double *ybuf[2], int k, int method,
                             int active, hipStream_t st)
{
    const SolverWS &w = f->sws;
    VecArgs a = vec_args(f);
    a.method = method;
    Ctl *ctl = a.ctl;
    const dim3 grid(a.nblocks), blk(kVB), fgrid(f->ninst);
    double *y = ybuf[k & 1], *yn = ybuf[(k + 1) & 1];
    double *r = w.r[k & 1], *rp = w.r[(k + 1) & 1];
    double *g = w.g[k & 1], *gp = w.g[(k + 1) & 1];
    double *hr = w.hr2, *hd = w.hr2 + f->m_tot;
    hipError_t e;
    // x(y) -> H x
    if ((e = launch_sweep_any(f, dual_layout_sweep(f, 1, x0, y, 0, w.hx, 0, ctl), 1, st, active))) return e;
    a.y = y; a.yp = yn; a.hx = w.hx; a.rp = rp; a.r = r;
    a.S = w.S; a.Q = w.Qv;
    if (method == 1) {
        hipLaunchKernelGGL((resid_kernel<true, MEMCAP>), grid, blk, 0, st, a);
        hipLaunchKernelGGL(fin_resid_kernel, fgrid, blk, 0, st, ctl, a.part, a.nblocks, 1, a.ndone);
        VecArgs cb = a;
        cb.g = r;           // g = R
        cb.r = w.d;         // output direction
        hipLaunchKernelGGL((combine_kernel<MEMCAP>), grid, blk, 0, st, cb);
        // x-hat(r) and x-hat(d) in one two-right-hand-side sweep (p-NAMA)
        if ((e = launch_sweep_any(f, dual_layout_sweep(f, 0, nullptr, r, w.d - r, hr, hd - hr, ctl), 2, st,
                                  active)))
            return e;
    } else {
        hipLaunchKernelGGL((resid_kernel<false, 0>), grid, blk, 0, st, a);
        hipLaunchKernelGGL(fin_resid_kernel, fgrid, blk, 0, st, ctl, a.part, a.nblocks, 0, a.ndone);
        // grad phi = R + lambda s H xhat(s R)
        if ((e = launch_sweep_any(f, dual_layout_sweep(f, 0, nullptr, r, 0, hr, 0, ctl), 1, st, active)))
            return e;
        VecArgs ga = a;
        ga.hr = hr; ga.g = g; ga.gp = gp;
        hipLaunchKernelGGL((grad_kernel<MEMCAP>), grid, blk, 0, st, ga);
        hipLaunchKernelGGL(fin_grad_kernel, fgrid, blk, 0, st, ctl, a.part, a.nblocks);
        VecArgs cb = a;
        cb.g = g; cb.r = w.d;
        hipLaunchKernelGGL((combine_kernel<MEMCAP>), grid, blk, 0, st, cb);
        if ((e = launch_sweep_any(f, dual_layout_sweep(f, 0, nullptr, w.d, 0, hd, 0, ctl), 1, st, active)))
            return e;
    }
    VecArgs la = vec_args(f);
    la.method = method;
    la.y = y; la.rp = r; la.d = w.d; la.hx = w.hx; la.hr = hr; la.hd = hd; la.yn = yn;
    hipLaunchKernelGGL(ls_kernel<NUC>, grid, blk, 0, st, la);
    hipLaunchKernelGGL(fin_ls_kernel, fgrid, blk, 0, st, ctl, a.part, a.nblocks);
    hipLaunchKernelGGL(update_kernel, grid, blk, 0, st, la);
    return hipGetLastError();
}

using IterFn = hipError_t (*)(const tree_factors *, const double *, double *[2], int, int, int, hipStream_t);

// Variant for the L-BFGS memory (accumulators per pair slot) and the number
// of line-search trials; the default options (mem 5, nu_max 10) have their own.
template <int NUC>
IterFn pick_iter_mem(int mem)
{
    if (mem <= 4) return enqueue_iteration<4, NUC>;
    if (mem == 5) return enqueue_iteration<5, NUC>;
    if (mem <= 8) return enqueue_iteration<8, NUC>;
    return enqueue_iteration<16, NUC>;
}

IterFn pick_iter(int mem, int nu_max)
{
    return nu_max <= kNuDefault ? pick_iter_mem<kNuDefault>(mem) : pick_iter_mem<kNuCap>(mem);
}

// Power iteration on every instance (per-instance normalisation); leaves
// L_b in the control blocks.
int power_iterations(tree_factors *f, int iters, hipStream_t st)
{
    const SolverWS &w = f->sws;
    VecArgs a = vec_args(f);
    const dim3 grid(a.nblocks), blk(kVB), fgrid(f->ninst);
    double *v = w.r[0], *wv = w.r[1], *hv = w.hx;
    VecArgs pa = a;
    pa.yn = v;
    hipLaunchKernelGGL(power_init_kernel, grid, blk, 0, st, pa);
    for (int it = 0; it < iters; ++it) {
        hipError_t e = launch_sweep_any(f, dual_layout_sweep(f, 0, nullptr, v, 0, hv, 0, nullptr), 1, st);
        if (e != hipSuccess) { set_error(std::string("dual_lipschitz: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
        pa.y = v; pa.hx = hv; pa.r = wv; pa.yn = v;
        hipLaunchKernelGGL(power_step_kernel, grid, blk, 0, st, pa);
        hipLaunchKernelGGL(power_fin_kernel, fgrid, blk, 0, st, a.ctl, a.part, a.nblocks);
        hipLaunchKernelGGL(power_scale_kernel, grid, blk, 0, st, pa);
    }
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

// Host copy of the control blocks with the block ranges filled in.
std::vector<Ctl> fresh_ctl(const tree_factors *f)
{
    std::vector<Ctl> h(f->ninst);
    for (int b = 0; b < f->ninst; ++b) {
        Ctl &c = h[b];
        std::memset(&c, 0, sizeof(Ctl));
        c.first_blk = f->sws.blk_first[b];
        const int next = b + 1 < f->ninst ? f->sws.blk_first[b + 1] : f->sws.nblocks;
        c.nblk = next - c.first_blk;
        c.gamma = 1.0;
        c.status = STOTREE_NOT_CONVERGED;
    }
    return h;
}

}  // namespace

int lipschitz(const tree_factors *fc, int iters, double *L, hipStream_t st)
{
    tree_factors *f = const_cast<tree_factors *>(fc);
    int rc = ensure_solver_ws(f, f->sws.buf ? f->sws.mem : 1, false);
    if (rc) return rc;
    if ((rc = ensure_sweep_ws(f, 2))) return rc;
    std::vector<Ctl> h = fresh_ctl(f);
    Ctl *dctl = reinterpret_cast<Ctl *>(f->sws.ctl);
    STOTREE_HIP(hipMemcpyAsync(dctl, h.data(), sizeof(Ctl) * h.size(), hipMemcpyHostToDevice, st));
    if ((rc = power_iterations(f, iters, st))) return rc;
    STOTREE_HIP(hipMemcpyAsync(h.data(), dctl, sizeof(Ctl) * h.size(), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < f->ninst; ++b) L[b] = h[b].L;
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
    int rc = ensure_solver_ws(f, o.mem, method == 0);
    if (rc) return rc;
    if ((rc = ensure_sweep_ws(f, 2))) return rc;
    const SolverWS &w = f->sws;
    Ctl *dctl = reinterpret_cast<Ctl *>(w.ctl);
    std::vector<Ctl> h = fresh_ctl(f);
    std::vector<double> lam(f->ninst, o.lambda);
    if (o.lambda == 0.0) {
        std::vector<double> L(f->ninst);
        if ((rc = lipschitz(f, 100, L.data(), st))) return rc;
        for (int b = 0; b < f->ninst; ++b) {
            if (!(L[b] > 0.0) || !std::isfinite(L[b])) {
                set_error("solve: could not estimate L of instance " + std::to_string(b));
                return STOTREE_ERR_NUMERIC;
            }
            lam[b] = 1.0 / (1.1 * L[b]);
        }
    }
    for (int b = 0; b < f->ninst; ++b) {
        Ctl &c = h[b];
        c.max_iter = o.max_iter; c.mem = o.mem; c.nu_max = o.nu_max; c.method = method;
        c.lam = lam[b]; c.eps = o.eps; c.eps_curv = o.eps_curv;
    }
    STOTREE_HIP(hipMemcpyAsync(dctl, h.data(), sizeof(Ctl) * h.size(), hipMemcpyHostToDevice, st));
    STOTREE_HIP(hipMemsetAsync(w.ndone, 0, sizeof(int), st));
    double *ybuf[2] = {y_io, w.y[1]};
    IterFn iter = pick_iter(o.mem, o.nu_max);
    int k = 0, ndone = 0;
    while (ndone < f->ninst && k <= o.max_iter) {
        // instances finished by the last check are skipped by the sweeps (the
        // count may lag behind by check_every iterations; it only grows)
        for (int c = 0; c < o.check_every && k <= o.max_iter; ++c, ++k) {
            hipError_t e = iter(f, x0, ybuf, k, method, f->ninst - ndone, st);
            if (e != hipSuccess) { set_error(std::string("solve: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
        }
        STOTREE_HIP(hipMemcpyAsync(&ndone, w.ndone, sizeof(int), hipMemcpyDeviceToHost, st));
        STOTREE_HIP(hipStreamSynchronize(st));
    }
    // last iterate of every instance into y_io, then x(y) in the caller's layout
    VecArgs ga = vec_args(f);
    ga.y = w.y[1]; ga.yn = y_io;
    hipLaunchKernelGGL(gather_final_kernel, dim3(ga.nblocks), dim3(kVB), 0, st, ga);
    SweepArgs a = sweep_args(f, 1);
    a.x0 = x0; a.y = y_io;
    a.xo = x; a.uo = u; a.dual_out = 0;
    hipError_t e = launch_sweep_any(f, a, 1, st);
    if (e != hipSuccess) { set_error(std::string("solve: ") + hipGetErrorString(e)); return STOTREE_ERR_DEVICE; }
    STOTREE_HIP(hipMemcpyAsync(h.data(), dctl, sizeof(Ctl) * h.size(), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    solver_info agg{};
    agg.status = STOTREE_OK;
    for (int b = 0; b < f->ninst; ++b) {
        const Ctl &c = h[b];
        solver_info &in = f->last_info[b];
        in = solver_info{};
        in.iters = c.iter;
        in.sweeps_affine = c.sweeps_aff + 1;
        in.sweeps_hom = c.sweeps_hom;
        in.ls_trials = c.ls_trials;
        in.lbfgs_push = c.pushes;
        in.lbfgs_skip = c.skips;
        in.status = c.status;
        in.res_scaled_inf = c.res;
        in.res_unscaled_inf = c.resu;
        in.lambda = c.lam;
        agg.iters = std::max(agg.iters, in.iters);
        agg.sweeps_affine = std::max(agg.sweeps_affine, in.sweeps_affine);
        agg.sweeps_hom = std::max(agg.sweeps_hom, in.sweeps_hom);
        agg.ls_trials += in.ls_trials;
        agg.lbfgs_push += in.lbfgs_push;
        agg.lbfgs_skip += in.lbfgs_skip;
        agg.res_scaled_inf = std::max(agg.res_scaled_inf, in.res_scaled_inf);
        agg.res_unscaled_inf = std::max(agg.res_unscaled_inf, in.res_unscaled_inf);
        if (in.status < 0) agg.status = std::min(agg.status, in.status);
        else if (agg.status >= 0 && in.status == STOTREE_NOT_CONVERGED) agg.status = STOTREE_NOT_CONVERGED;
    }
    agg.lambda = h[0].lam;
    *info = agg;
    if (agg.status == STOTREE_ERR_NUMERIC) set_error("solve: non-finite values in the iterates");
    return agg.status;
}

}  // namespace stotree
