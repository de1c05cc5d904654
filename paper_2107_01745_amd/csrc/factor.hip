// Factor step (arXiv 2107.01745, Sec. III-D: the Riccati-type recursion that
// precomputes the per-node factors once, before any solve), for a forest of
// independent trees.
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
// pi_i r_i enters g_i).  Stages run from the deepest down to 0; one kernel per
// stage covers that stage of every instance, one workgroup per node; the
// products are small dense FP64 blocks computed over output entries.
//
// The sweeps then stream, per edge j, M_j = [A_j B_j] row-major (backward,
// Mb) and its transpose (forward, Mf), and per non-leaf node K_i (Kb), K_i'
// (Kf) and -R~_i^{-1} (Rn); rows are padded to an even length so each row is
// one aligned 16-byte-per-lane load.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace stotree {

namespace {

// Offsets of one instance in the raw (input-layout) pools.
struct RawDesc {
    long long A, B, c, Q, R, S, q, r, P, p, prob, Pcal;
};

struct FactorArgs {
    const InstDesc *inst;
    const RawDesc *raw;
    const Item *items;
    const int *sp, *cp;
    const double *prob, *A, *B, *c, *Q, *R, *S, *q, *r, *P, *p;
    int hasS, hasq, hasr, hasp;
    double *Pcal, *scratch;
    long long slot;  // scratch doubles per workgroup
    double *Mb, *Mf, *Kb, *Kf, *Rn, *chat, *sig, *cvec, *sc;
    int *err;
};

// Mb, Mf and c of every edge of instance b.
__global__ void pack_dynamics_kernel(FactorArgs a, int b)
{
    const InstDesc I = a.inst[b];
    const RawDesc Rw = a.raw[b];
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const long long per_b = (long long)nx * I.ldM, per_f = (long long)W * I.ldx;
    const long long total = (long long)I.V * (per_b + per_f);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = e / (per_b + per_f);
        const long long w = e % (per_b + per_f);
        const double *Aj = a.A + Rw.A + j * nx * nx;
        const double *Bj = a.B + Rw.B + j * nx * nu;
        if (w < per_b) {  // Mb[j][r][col]
            const int r = (int)(w / I.ldM), col = (int)(w % I.ldM);
            double v = 0.0;
            if (j > 0) {
                if (col < nx) v = Aj[r * nx + col];
                else if (col < W) v = Bj[r * nu + (col - nx)];
            }
            a.Mb[I.Mb + j * per_b + w] = v;
        } else {           // Mf[j][col][r] = M_j[r][col]
            const long long wf = w - per_b;
            const int col = (int)(wf / I.ldx), r = (int)(wf % I.ldx);
            double v = 0.0;
            if (j > 0 && r < nx) v = (col < nx) ? Aj[r * nx + col] : Bj[r * nu + (col - nx)];
            a.Mf[I.Mf + j * per_f + wf] = v;
        }
    }
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)I.V * nx;
         e += (long long)gridDim.x * blockDim.x) {
        a.cvec[I.c + e] = (e < nx) ? 0.0 : a.c[Rw.c + e];
    }
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < I.V;
         e += (long long)gridDim.x * blockDim.x)
        a.sc[I.sc + e] = sqrt(a.prob[Rw.prob + e]);
}

__global__ void factor_leaves_kernel(FactorArgs a, int b)
{
    const InstDesc I = a.inst[b];
    const RawDesc Rw = a.raw[b];
    const int nx = I.nx;
    const int j = I.Vnl + blockIdx.x;
    if (j >= I.V) return;
    const long long l = j - I.Vnl;
    const double pj = a.prob[Rw.prob + j];
    double *Pj = a.Pcal + Rw.Pcal + (long long)j * nx * nx;
    for (int e = threadIdx.x; e < nx * nx; e += blockDim.x) Pj[e] = 2.0 * pj * a.P[Rw.P + l * nx * nx + e];
    __syncthreads();
    for (int r = threadIdx.x; r < nx; r += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nx; ++k) s = fma(Pj[r * nx + k], a.c[Rw.c + (long long)j * nx + k], s);
        if (a.hasp) s += pj * a.p[Rw.p + l * nx + r];
        a.chat[I.chat + (long long)j * nx + r] = s;
    }
}

// The children's products of a node, H = sum_j [A_j B_j]' P_j [A_j B_j]
// (the blocks [Q-like ; S~] and R~ of it), tiled through LDS: the first
// product T = P_j [A_j B_j] and then H += [A_j B_j]' T, both over chunks of
// KC (16, or 8 where 16 does not fit) rows of the K dimension staged in LDS
// (zero-padded to whole 4x4 blocks),
// each thread accumulating kFB blocks of 4x4 outputs in registers; H stays in
// registers across the children.  Used when the node's sizes fit kFactorLds
// doubles of LDS and kFB blocks per thread; otherwise the entry-by-entry loop
// below.
constexpr int kFB = 2;
constexpr int kFactorThreads = 256;
constexpr int kFactorLds = 8192;

struct FactorTiles {
    int kc, nx4, nu4, ldB, nxK, cbT, nbT, cx, cu, nbH1, nbH;
    __host__ __device__ FactorTiles(int nx, int nu, int kc_) : kc(kc_)
    {
        nx4 = (nx + 3) & ~3;
        nu4 = (nu + 3) & ~3;
        ldB = nx4 + nu4;
        nxK = (nx + kc - 1) / kc * kc;
        cbT = (nx + nu + 3) >> 2;
        nbT = (nx4 >> 2) * cbT;
        cx = nx4 >> 2;
        cu = nu4 >> 2;
        nbH1 = cbT * cx;
        nbH = nbH1 + cu * cu;
    }
    // the node's tail after the products: R~ (then L), L^{-1}, R~^{-1}, S~ and K
    __host__ __device__ int tail_doubles(int nx, int nu) const { return 3 * nu * nu + 2 * nu * nx; }
    __host__ __device__ int lds_doubles(int nx, int nu) const
    {
        const int prod = nx4 * kc + kc * ldB + nxK * ldB, tail = tail_doubles(nx, nu);
        return prod > tail ? prod : tail;
    }
    __host__ __device__ bool fits(int nx, int nu) const
    {
        return lds_doubles(nx, nu) <= kFactorLds && nbT <= kFB * kFactorThreads && nbH <= kFB * kFactorThreads;
    }
};

// sum_{k0 <= k < k1} x[k sx] y[k sy] in four independent partial sums (the
// loads of four terms in flight together)
__device__ __forceinline__ double dot4(const double *x, int sx, const double *y, int sy, int k0, int k1)
{
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int k = k0;
    for (; k + 3 < k1; k += 4) {
        v0 = fma(x[k * sx], y[k * sy], v0);
        v1 = fma(x[(k + 1) * sx], y[(k + 1) * sy], v1);
        v2 = fma(x[(k + 2) * sx], y[(k + 2) * sy], v2);
        v3 = fma(x[(k + 3) * sx], y[(k + 3) * sy], v3);
    }
    for (; k < k1; ++k) v0 = fma(x[k * sx], y[k * sy], v0);
    return (v0 + v1) + (v2 + v3);
}

template <bool kTiled, int KC = 8>
__global__ void __launch_bounds__(kFactorThreads) factor_stage_kernel(FactorArgs a)
{
    const Item it = a.items[blockIdx.x];
    const InstDesc I = a.inst[it.inst];
    const RawDesc Rw = a.raw[it.inst];
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const int i = it.idx;
    const int *cp = a.cp + I.cp;
    const int tid = threadIdx.x, nt = blockDim.x;
    double *Wsc = a.scratch + (long long)blockIdx.x * a.slot;  // [nx][W]
    double *Rt = Wsc + (long long)nx * W;                      // [nu][nu] -> Cholesky L
    double *St = Rt + nu * nu;                                  // [nu][nx]
    double *Ri = St + nu * nx;                                  // [nu][nu]
    __shared__ int fail;
    const double pi = a.prob[Rw.prob + i];
    double *Pi = a.Pcal + Rw.Pcal + (long long)i * nx * nx;
    if (tid == 0) fail = 0;
    if (kTiled) {
        extern __shared__ double fl[];
        const FactorTiles ft(nx, nu, KC);
        const int ldB = ft.ldB;
        double *sA = fl, *sB = sA + ft.nx4 * KC, *sT = sB + KC * ldB;
        // H blocks of this thread: rows [0, W) x columns [0, nx) (P and S~),
        // then rows and columns [nx, W) (R~); origin -1: no block
        double h[kFB][4][4];
        int hr[kFB], hc[kFB];
#pragma unroll
        for (int s = 0; s < kFB; ++s) {
            const int q = tid + kFactorThreads * s;
            if (q < ft.nbH1) {
                hr[s] = 4 * (q / ft.cx);
                hc[s] = 4 * (q % ft.cx);
            } else if (q < ft.nbH) {
                const int q2 = q - ft.nbH1;
                hr[s] = nx + 4 * (q2 / ft.cu);
                hc[s] = nx + 4 * (q2 % ft.cu);
            } else {
                hr[s] = hc[s] = -1;
            }
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = hr[s] + d, c = hc[s] + e;
                    double v = 0.0;
                    if (hr[s] >= 0 && r < W && c < W) {
                        if (r < nx && c < nx)
                            v = 2.0 * pi * a.Q[Rw.Q + (long long)i * nx * nx + r * nx + c];
                        else if (r >= nx && c < nx)
                            v = a.hasS ? 2.0 * pi * a.S[Rw.S + (long long)i * nu * nx + (r - nx) * nx + c] : 0.0;
                        else if (r >= nx && c >= nx)
                            v = 2.0 * pi * a.R[Rw.R + (long long)i * nu * nu + (r - nx) * nu + (c - nx)];
                    }
                    h[s][d][e] = v;
                }
        }
        for (int e = tid; e < ft.nxK * ldB; e += nt) sT[e] = 0.0;   // rows and columns past T stay zero
        __syncthreads();
        for (int j = cp[i]; j < cp[i + 1]; ++j) {
            const double *M = a.Mb + I.Mb + (long long)j * nx * I.ldM;
            const double *Pj = a.Pcal + Rw.Pcal + (long long)j * nx * nx;
            auto stage_M = [&](int k0) {          // sB[kk][c] = M[k0 + kk][c] (zero past the matrix)
                for (int e = tid; e < KC * ldB; e += nt) {
                    const int kk = e / ldB, c = e - kk * ldB, k = k0 + kk;
                    sB[e] = k < nx && c < W ? M[(long long)k * I.ldM + c] : 0.0;
                }
            };
            // T = P_j [A_j B_j] (rows [0, nx4), columns [0, 4 cbT))
            double t[kFB][4][4];
#pragma unroll
            for (int s = 0; s < kFB; ++s)
#pragma unroll
                for (int d = 0; d < 4; ++d)
#pragma unroll
                    for (int e = 0; e < 4; ++e) t[s][d][e] = 0.0;
            for (int k0 = 0; k0 < nx; k0 += KC) {
                for (int e = tid; e < ft.nx4 * KC; e += nt) {
                    const int r = e / KC, k = k0 + e - r * KC;
                    sA[e] = r < nx && k < nx ? Pj[r * nx + k] : 0.0;
                }
                stage_M(k0);
                __syncthreads();
#pragma unroll
                for (int s = 0; s < kFB; ++s) {
                    const int q = tid + kFactorThreads * s;
                    if (q >= ft.nbT) continue;
                    const int r0 = 4 * (q / ft.cbT), c0 = 4 * (q % ft.cbT);
#pragma unroll 8
                    for (int kk = 0; kk < KC; ++kk) {
                        double av[4], bv[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) av[d] = sA[(r0 + d) * KC + kk];
#pragma unroll
                        for (int e = 0; e < 4; ++e) bv[e] = sB[kk * ldB + c0 + e];
#pragma unroll
                        for (int d = 0; d < 4; ++d)
#pragma unroll
                            for (int e = 0; e < 4; ++e) t[s][d][e] = fma(av[d], bv[e], t[s][d][e]);
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int s = 0; s < kFB; ++s) {
                const int q = tid + kFactorThreads * s;
                if (q >= ft.nbT) continue;
                const int r0 = 4 * (q / ft.cbT), c0 = 4 * (q % ft.cbT);
#pragma unroll
                for (int d = 0; d < 4; ++d)
#pragma unroll
                    for (int e = 0; e < 4; ++e) sT[(r0 + d) * ldB + c0 + e] = t[s][d][e];
            }
            // H += [A_j B_j]' T
            for (int k0 = 0; k0 < nx; k0 += KC) {
                stage_M(k0);
                __syncthreads();
#pragma unroll
                for (int s = 0; s < kFB; ++s) {
                    if (hr[s] < 0) continue;
#pragma unroll 8
                    for (int kk = 0; kk < KC; ++kk) {
                        double av[4], bv[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) av[d] = sB[kk * ldB + hr[s] + d];
#pragma unroll
                        for (int e = 0; e < 4; ++e) bv[e] = sT[(k0 + kk) * ldB + hc[s] + e];
#pragma unroll
                        for (int d = 0; d < 4; ++d)
#pragma unroll
                            for (int e = 0; e < 4; ++e) h[s][d][e] = fma(av[d], bv[e], h[s][d][e]);
                    }
                }
                __syncthreads();
            }
        }
        // P_i to its slot; R~ and S~ into LDS for the tail (the products' LDS is free now)
        double *sR = fl, *sLi = sR + nu * nu, *sRi = sLi + nu * nu, *sS = sRi + nu * nu, *sK = sS + nu * nx;
#pragma unroll
        for (int s = 0; s < kFB; ++s) {
            if (hr[s] < 0) continue;
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = hr[s] + d, c = hc[s] + e;
                    if (r >= W || c >= W) continue;
                    if (hc[s] < nx) {           // a block of columns [0, nx): P_i and S~ (padding columns dropped)
                        if (c >= nx) continue;
                        if (r < nx)
                            Pi[r * nx + c] = h[s][d][e];
                        else
                            sS[(r - nx) * nx + c] = h[s][d][e];
                    } else {                    // a block of R~
                        sR[(r - nx) * nu + (c - nx)] = h[s][d][e];
                    }
                }
        }
        __syncthreads();
        // Cholesky R~ = L L' (lower triangle of sR), right-looking: pivot,
        // column below it, then the trailing lower triangle in parallel
        for (int jc = 0; jc < nu; ++jc) {
            if (tid == 0) {
                const double d = sR[jc * nu + jc];
                if (!(d > 0.0)) fail = 1;
                else sR[jc * nu + jc] = sqrt(d);
            }
            __syncthreads();
            if (fail) break;
            const double piv = sR[jc * nu + jc];
            for (int r = jc + 1 + tid; r < nu; r += nt) sR[r * nu + jc] /= piv;
            __syncthreads();
            const int m = nu - jc - 1;
            for (int e = tid; e < m * m; e += nt) {
                const int r = jc + 1 + e / m, c = jc + 1 + e % m;
                if (c <= r) sR[r * nu + c] -= sR[r * nu + jc] * sR[c * nu + jc];
            }
            __syncthreads();
        }
        if (fail) {
            if (tid == 0) atomicExch(a.err, STOTREE_ERR_NOT_PD);
            return;
        }
        // L^{-1} (lower), row by row: all columns of a row in parallel
        for (int e = tid; e < nu * nu; e += nt) sLi[e] = 0.0;
        __syncthreads();
        for (int r = 0; r < nu; ++r) {
            for (int c = tid; c <= r; c += nt) {
                const double v = (r == c ? 1.0 : 0.0) - dot4(sR + r * nu, 1, sLi + c, nu, c, r);
                sLi[r * nu + c] = v / sR[r * nu + r];
            }
            __syncthreads();
        }
        // R~^{-1} = L^{-T} L^{-1}
        for (int e = tid; e < nu * nu; e += nt) {
            const int r = e / nu, c = e - r * nu, k0 = r > c ? r : c;
            sRi[e] = dot4(sLi + r, nu, sLi + c, nu, k0, nu);
        }
        __syncthreads();
        // K = -R~^{-1} S~ (sK and both stored layouts), -R~^{-1} (Rn)
        double *Kb = a.Kb + I.Kb + (long long)i * nu * I.ldx;
        double *Kf = a.Kf + I.Kf + (long long)i * nx * I.ldu;
        double *Rn = a.Rn + I.Rn + (long long)i * nu * I.ldu;
        for (int e = tid; e < nu * nx; e += nt) {
            const int r = e / nx, c = e - r * nx;
            const double v = dot4(sRi + r * nu, 1, sS + c, nx, 0, nu);
            sK[e] = -v;
            Kb[r * I.ldx + c] = -v;
            Kf[c * I.ldu + r] = -v;
        }
        for (int e = tid; e < nu * (I.ldx - nx); e += nt) Kb[(e / (I.ldx - nx)) * I.ldx + nx + e % (I.ldx - nx)] = 0.0;
        for (int e = tid; e < nx * (I.ldu - nu); e += nt) Kf[(e / (I.ldu - nu)) * I.ldu + nu + e % (I.ldu - nu)] = 0.0;
        for (int e = tid; e < nu * I.ldu; e += nt) {
            const int r = e / I.ldu, c = e - r * I.ldu;
            Rn[e] = c < nu ? -sRi[r * nu + c] : 0.0;
        }
        __syncthreads();
        // P_i += K' S~
        for (int e = tid; e < nx * nx; e += nt) {
            const int r = e / nx, c = e - r * nx;
            Pi[e] += dot4(sK + r, nx, sS + c, nx, 0, nu);
        }
        __syncthreads();
        for (int rr = tid; rr < nx; rr += nt) {
            double v = i > 0 ? dot4(Pi + rr * nx, 1, a.c + Rw.c + (long long)i * nx, 1, 0, nx) : 0.0;
            if (a.hasq) v += pi * a.q[Rw.q + (long long)i * nx + rr];
            a.chat[I.chat + (long long)i * nx + rr] = v;
        }
        for (int rr = tid; rr < nu; rr += nt)
            a.sig[I.sig + (long long)i * nu + rr] = a.hasr ? pi * a.r[Rw.r + (long long)i * nu + rr] : 0.0;
        return;
    } else {
    for (int e = tid; e < nu * nu; e += nt) Rt[e] = 2.0 * pi * a.R[Rw.R + (long long)i * nu * nu + e];
    for (int e = tid; e < nu * nx; e += nt) St[e] = a.hasS ? 2.0 * pi * a.S[Rw.S + (long long)i * nu * nx + e] : 0.0;
    for (int e = tid; e < nx * nx; e += nt) Pi[e] = 2.0 * pi * a.Q[Rw.Q + (long long)i * nx * nx + e];
    __syncthreads();
    for (int j = cp[i]; j < cp[i + 1]; ++j) {
        const double *M = a.Mb + I.Mb + (long long)j * nx * I.ldM;
        const double *Pj = a.Pcal + Rw.Pcal + (long long)j * nx * nx;
        for (int e = tid; e < nx * W; e += nt) {          // W = P_j [A_j B_j]
            const int r = e / W, col = e % W;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(Pj[r * nx + k], M[(long long)k * I.ldM + col], s);
            Wsc[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < nx * nx; e += nt) {          // P_i += A_j' P_j A_j
            const int r = e / nx, col = e % nx;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * I.ldM + r], Wsc[k * W + col], s);
            Pi[e] += s;
        }
        for (int e = tid; e < nu * nu; e += nt) {          // R~ += B_j' P_j B_j
            const int r = e / nu, col = e % nu;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * I.ldM + nx + r], Wsc[k * W + nx + col], s);
            Rt[e] += s;
        }
        for (int e = tid; e < nu * nx; e += nt) {          // S~ += B_j' P_j A_j
            const int r = e / nx, col = e % nx;
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s = fma(M[(long long)k * I.ldM + nx + r], Wsc[k * W + col], s);
            St[e] += s;
        }
        __syncthreads();
    }
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
    double *Kb = a.Kb + I.Kb + (long long)i * nu * I.ldx;
    double *Kf = a.Kf + I.Kf + (long long)i * nx * I.ldu;
    double *Rn = a.Rn + I.Rn + (long long)i * nu * I.ldu;
    for (int e = tid; e < nu * I.ldx; e += nt) {           // K = -R~^{-1} S~ (pad columns zero)
        const int r = e / I.ldx, col = e % I.ldx;
        double s = 0.0;
        if (col < nx)
            for (int k = 0; k < nu; ++k) s = fma(Ri[r * nu + k], St[k * nx + col], s);
        Kb[e] = -s;
    }
    for (int e = tid; e < nx * I.ldu; e += nt) {           // K' (pad columns zero)
        const int col = e / I.ldu, r = e % I.ldu;
        double s = 0.0;
        if (r < nu)
            for (int k = 0; k < nu; ++k) s = fma(Ri[r * nu + k], St[k * nx + col], s);
        Kf[e] = -s;
    }
    for (int e = tid; e < nu * I.ldu; e += nt) {
        const int r = e / I.ldu, col = e % I.ldu;
        Rn[e] = col < nu ? -Ri[r * nu + col] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < nx * nx; e += nt) {              // P_i += K' S~
        const int r = e / nx, col = e % nx;
        double s = 0.0;
        for (int k = 0; k < nu; ++k) s = fma(Kb[k * I.ldx + r], St[k * nx + col], s);
        Pi[e] += s;
    }
    __syncthreads();
    for (int rr = tid; rr < nx; rr += nt) {
        double s = 0.0;
        if (i > 0)
            for (int k = 0; k < nx; ++k) s = fma(Pi[rr * nx + k], a.c[Rw.c + (long long)i * nx + k], s);
        if (a.hasq) s += pi * a.q[Rw.q + (long long)i * nx + rr];
        a.chat[I.chat + (long long)i * nx + rr] = s;
    }
    for (int rr = tid; rr < nu; rr += nt)
        a.sig[I.sig + (long long)i * nu + rr] = a.hasr ? pi * a.r[Rw.r + (long long)i * nu + rr] : 0.0;
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

int validate(const tree_desc *t, const problem_data *d, const std::string &who)
{
    if (!t || !d) { set_error(who + ": NULL tree or data"); return STOTREE_ERR_ARG; }
    const int nx = t->nx, nu = t->nu, N = t->N, V = t->num_nodes;
    if (nx < 1 || nu < 1 || N < 1 || V < 2 || nx + nu > kMaxWidth) {
        set_error(who + ": need nx>=1, nu>=1, N>=1, V>=2 and nx+nu<=256");
        return STOTREE_ERR_ARG;
    }
    const bool cmap = d->F != nullptr;
    if (!t->stage_ptr || !t->ancestor || !t->child_ptr || !t->prob || !d->A || !d->B || !d->c ||
        !d->Q || !d->R || !d->P ||
        (!cmap && (!d->xmin || !d->xmax || !d->umin || !d->umax)) ||
        (cmap && (!d->G || !d->zmin || !d->zmax || (d->ncN > 0 && !d->FN)))) {
        set_error(who + ": a required array is NULL");
        return STOTREE_ERR_ARG;
    }
    if (cmap && (d->nc < 1 || d->ncN < 0 || d->nc > 4 * kMaxWidth || d->ncN > 4 * kMaxWidth)) {
        set_error(who + ": constraint map needs 1 <= nc and 0 <= ncN (at most 1024 rows per node)");
        return STOTREE_ERR_ARG;
    }
    const int *sp = t->stage_ptr;
    if (sp[0] != 0 || sp[1] != 1 || sp[N + 1] != V) {
        set_error(who + ": stage_ptr must start 0,1 and end at num_nodes");
        return STOTREE_ERR_TREE;
    }
    for (int s = 0; s <= N; ++s)
        if (sp[s + 1] <= sp[s]) { set_error(who + ": empty stage"); return STOTREE_ERR_TREE; }
    const int Vnl = sp[N];
    if (t->ancestor[0] != -1) { set_error(who + ": ancestor[0] must be -1"); return STOTREE_ERR_TREE; }
    for (int s = 1; s <= N; ++s)
        for (int i = sp[s]; i < sp[s + 1]; ++i) {
            const int a = t->ancestor[i];
            if (a < sp[s - 1] || a >= sp[s]) {
                set_error(who + ": ancestor of a node is not in the previous stage");
                return STOTREE_ERR_TREE;
            }
        }
    const int *cp = t->child_ptr;
    if (cp[0] != 1 || cp[Vnl] != V) { set_error(who + ": child_ptr must span [1, V)"); return STOTREE_ERR_TREE; }
    for (int i = 0; i < Vnl; ++i) {
        if (cp[i + 1] <= cp[i]) { set_error(who + ": a non-leaf node has no child"); return STOTREE_ERR_TREE; }
        for (int j = cp[i]; j < cp[i + 1]; ++j)
            if (t->ancestor[j] != i) {
                set_error(who + ": child_ptr and ancestor disagree");
                return STOTREE_ERR_TREE;
            }
    }
    if (std::fabs(t->prob[0] - 1.0) > 1e-12) { set_error(who + ": prob[0] must be 1"); return STOTREE_ERR_TREE; }
    for (int s = 0; s <= N; ++s) {
        double tot = 0.0;
        for (int i = sp[s]; i < sp[s + 1]; ++i) {
            if (!(t->prob[i] > 0.0) || !std::isfinite(t->prob[i])) {
                set_error(who + ": node probabilities must be positive");
                return STOTREE_ERR_TREE;
            }
            tot += t->prob[i];
        }
        if (std::fabs(tot - 1.0) > 1e-12) {
            set_error(who + ": probabilities of stage " + std::to_string(s) + " do not sum to 1");
            return STOTREE_ERR_TREE;
        }
    }
    const size_t Vl = (size_t)V - Vnl;
    struct Chk { const double *p; size_t n; const char *name; };
    const Chk chks[] = {{d->A, (size_t)V * nx * nx, "A"}, {d->B, (size_t)V * nx * nu, "B"},
                        {d->c, (size_t)V * nx, "c"}, {d->Q, (size_t)Vnl * nx * nx, "Q"},
                        {d->R, (size_t)Vnl * nu * nu, "R"}, {d->S, (size_t)Vnl * nu * nx, "S"},
                        {d->q, (size_t)Vnl * nx, "q"}, {d->r, (size_t)Vnl * nu, "r"},
                        {d->P, Vl * nx * nx, "P"}, {d->p, Vl * nx, "p"}};
    for (const Chk &c : chks)
        if (c.p && !all_finite(c.p, c.n)) {
            set_error(who + ": non-finite entry in " + c.name);
            return STOTREE_ERR_NUMERIC;
        }
    size_t m = (size_t)Vnl * (nx + nu) + Vl * nx;
    if (cmap) {
        m = (size_t)Vnl * d->nc + Vl * d->ncN;
        if (!all_finite(d->F, (size_t)d->nc * nx) || !all_finite(d->G, (size_t)d->nc * nu) ||
            (d->ncN > 0 && !all_finite(d->FN, (size_t)d->ncN * nx))) {
            set_error(who + ": non-finite entry in the constraint map");
            return STOTREE_ERR_NUMERIC;
        }
        for (size_t k = 0; k < m; ++k)
            if (std::isnan(d->zmin[k]) || std::isnan(d->zmax[k]) || d->zmin[k] > d->zmax[k]) {
                set_error(who + ": constraint row with lo > hi (or NaN)");
                return STOTREE_ERR_BOX;
            }
    } else {
        for (size_t k = 0; k < (size_t)V * nx; ++k)
            if (std::isnan(d->xmin[k]) || std::isnan(d->xmax[k]) || d->xmin[k] > d->xmax[k]) {
                set_error(who + ": state box with lo > hi (or NaN)");
                return STOTREE_ERR_BOX;
            }
        for (size_t k = 0; k < (size_t)Vnl * nu; ++k)
            if (std::isnan(d->umin[k]) || std::isnan(d->umax[k]) || d->umin[k] > d->umax[k]) {
                set_error(who + ": input box with lo > hi (or NaN)");
                return STOTREE_ERR_BOX;
            }
    }
    if (d->wgt)
        for (size_t k = 0; k < m; ++k) {
            const double hb = d->hub ? d->hub[k] : 0.0;
            if (!(d->wgt[k] > 0.0) || !(hb >= 0.0) || !std::isfinite(hb)) {
                set_error(who + ": soft rows need wgt > 0 (or +inf) and a finite hub >= 0");
                return STOTREE_ERR_ARG;
            }
        }
    return STOTREE_OK;
}

// Wavefronts per node for a stage of n nodes: at most 2048 in the stage, so
// that a wide stage fits the chip in one round at the per-node kernels'
// register use (4096 left a 1024-node stage running in two rounds; 2048 was
// 0.5% faster per large-tree sweep), within the LDS budget of the reduction
// buffers.  Rows
// wider than two entries per lane take at most 8: at 16 wavefronts (1024
// threads) the two-chunk row code runs out of registers and its loads wait
// for one another (the stages of an nx=100, nu=40 tree ran 3-7x slower).
int trunk_waves(int n, int nrhs_max, int ldM, int cap)
{
    int nw = ldM > 2 * kWave && cap > 8 ? 8 : cap;
    while (nw > 1 && (long long)n * nw > 2048) nw /= 2;
    while (nw > 1 && (size_t)(nw + 2) * nrhs_max * ldM * sizeof(double) > 40 * 1024) nw /= 2;
    return nw;
}

void free_level(LevelPlan &lv)
{
    if (lv.items) (void)hipFree(lv.items);
    if (lv.wide_items) (void)hipFree(lv.wide_items);
    for (auto &g : lv.narrow)
        if (g.items) (void)hipFree(g.items);
    lv.items = lv.wide_items = nullptr;
    lv.narrow.clear();
}

}  // namespace

void free_tree(tree_factors *f)
{
    if (!f) return;
    for (void *p : {(void *)f->d_inst, (void *)f->d_sp, (void *)f->d_cp, (void *)f->d_anc, (void *)f->Mb, (void *)f->Mf,
                    (void *)f->Kb, (void *)f->Kf, (void *)f->Rn, (void *)f->chat, (void *)f->sig,
                    (void *)f->cvec, (void *)f->sc, (void *)f->lo, (void *)f->hi, (void *)f->qhat,
                    (void *)f->kbuf, (void *)f->sws.buf, (void *)f->pw, (void *)f->hub, (void *)f->Fm,
                    (void *)f->map_ws})
        if (p) (void)hipFree(p);
    if (f->d_inst_xu && f->d_inst_xu != f->d_inst) (void)hipFree(f->d_inst_xu);
    for (auto &cp : f->chains)
        if (cp.items) (void)hipFree(cp.items);
    for (auto &lv : f->levels) free_level(lv);
    for (auto &lv : f->panel_levels) free_level(lv);
    for (auto &lv : f->rest_levels) free_level(lv);
    free_level(f->fused_bwd);
    free_level(f->fused_fwd);
    for (void *p : {(void *)f->panel_chain_items, (void *)f->trunk_entry.items, (void *)f->trunk_cnt,
                    (void *)f->Pcal})
        if (p) (void)hipFree(p);
    delete f;
}

int chain_group(int ldM, int group_min)
{
    int G = 8;
    while (G < kWave && 2 * G < ldM) G *= 2;
    return G < group_min ? group_min : G;
}

// Work lists of a sweep: the chains, one plan per lane-group width (each item
// a wavefront's worth of consecutive chains of one instance; the costliest
// first when chain_order is set) and, per stage above s*, all (instance,
// node) pairs of that stage.
int build_schedule(tree_factors *f)
{
    for (auto &cp : f->chains)
        if (cp.items) (void)hipFree(cp.items);
    f->chains.clear();
    for (auto &lv : f->levels) free_level(lv);
    f->levels.clear();
    int max_sstar = 0, max_ldM = 0;
    std::map<int, std::vector<std::pair<double, Item>>> by_G;
    std::map<int, int> ldq_G;
    for (int b = 0; b < f->ninst; ++b) {
        const InstDesc &I = f->inst[b];
        max_sstar = std::max(max_sstar, I.sstar);
        max_ldM = std::max(max_ldM, I.ldM);
        if (I.sstar >= I.N) continue;
        const int G = chain_group(I.ldM, f->group_min);
        const int per = kWave / G;
        ldq_G[G] = std::max(ldq_G[G], I.ldM);
        for (int c = 0; c < I.nchains; c += per) {
            const int n = std::min(per, I.nchains - c);
            by_G[G].push_back({(double)(I.N - I.sstar) * I.nx * (I.nx + I.nu) * n, Item{b, c}});
        }
    }
    if (f->panel_chain_items) { (void)hipFree(f->panel_chain_items); f->panel_chain_items = nullptr; }
    for (auto &lv : f->panel_levels) free_level(lv);
    f->panel_levels.clear();
    const int panel_inst = f->shared > 1 ? 1 : f->ninst;   // a shared handle's panels cover instance 0's nodes
    {
        std::vector<Item> all;
        for (int b = 0; b < panel_inst; ++b) {
            const InstDesc &I = f->inst[b];
            if (I.sstar < I.N)
                for (int c = 0; c < I.nchains; ++c) all.push_back({b, c});
        }
        f->npanel_chain_items = (int)all.size();
        if (!all.empty()) {
            STOTREE_HIP(hipMalloc(&f->panel_chain_items, sizeof(Item) * all.size()));
            STOTREE_HIP(hipMemcpy(f->panel_chain_items, all.data(), sizeof(Item) * all.size(),
                                  hipMemcpyHostToDevice));
        }
    }
    for (auto &kv : by_G) {
        auto &v = kv.second;
        if (f->chain_order)
            std::stable_sort(v.begin(), v.end(), [](const auto &p, const auto &q) { return p.first > q.first; });
        std::vector<Item> items(v.size());
        for (size_t k = 0; k < v.size(); ++k) items[k] = v[k].second;
        ChainPlan cp{};
        cp.G = kv.first;
        cp.ldq = ldq_G[kv.first];
        cp.CH = cp.ldq > 2 * cp.G ? 2 : 1;
        cp.count = (int)items.size();
        STOTREE_HIP(hipMalloc(&cp.items, sizeof(Item) * items.size()));
        f->chains.push_back(cp);
        STOTREE_HIP(hipMemcpy(cp.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    }
    for (int t = 0; t < max_sstar; ++t) {
        std::vector<Item> items;
        for (int b = 0; b < f->ninst; ++b) {
            const InstDesc &I = f->inst[b];
            if (t >= I.sstar) continue;
            const int *sp = f->sp_pool.data() + I.sp;
            for (int i = sp[t]; i < sp[t + 1]; ++i) items.push_back({b, i});
        }
        LevelPlan lv{};
        lv.t = t;
        lv.count = (int)items.size();
        lv.nw = trunk_waves(lv.count, 2, max_ldM, f->trunk_cap);
        STOTREE_HIP(hipMalloc(&lv.items, sizeof(Item) * std::max<size_t>(1, items.size())));
        f->levels.push_back(lv);
        STOTREE_HIP(hipMemcpy(lv.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
        if (f->trunk_fused == 2) {
            // lane groups for the nodes of narrow instances, workgroups for the rest
            LevelPlan &L = f->levels.back();
            std::vector<Item> wide;
            std::map<int, std::vector<Item>> groups;
            std::map<int, int> gldq;
            int wide_ldM = 2;
            for (int b = 0; b < f->ninst; ++b) {
                const InstDesc &I = f->inst[b];
                if (t >= I.sstar) continue;
                const int *sp = f->sp_pool.data() + I.sp;
                const int G = chain_group(I.ldM, f->group_min);
                if (G == kWave) {
                    for (int i = sp[t]; i < sp[t + 1]; ++i) wide.push_back({b, i});
                    wide_ldM = std::max(wide_ldM, I.ldM);
                    continue;
                }
                gldq[G] = std::max(gldq[G], I.ldM);
                for (int i = sp[t]; i < sp[t + 1]; i += kWave / G) groups[G].push_back({b, i});
            }
            L.wide_count = (int)wide.size();
            L.wide_nw = trunk_waves(L.wide_count, 2, wide_ldM, f->trunk_cap);
            if (!wide.empty()) {
                STOTREE_HIP(hipMalloc(&L.wide_items, sizeof(Item) * wide.size()));
                STOTREE_HIP(hipMemcpy(L.wide_items, wide.data(), sizeof(Item) * wide.size(), hipMemcpyHostToDevice));
            }
            for (auto &kv : groups) {
                ChainPlan g{};
                g.G = kv.first;
                g.CH = 1;
                g.ldq = gldq[kv.first];
                g.count = (int)kv.second.size();
                STOTREE_HIP(hipMalloc(&g.items, sizeof(Item) * kv.second.size()));
                L.narrow.push_back(g);
                STOTREE_HIP(hipMemcpy(g.items, kv.second.data(), sizeof(Item) * kv.second.size(),
                                      hipMemcpyHostToDevice));
            }
        }
        if (panel_inst < f->ninst) {
            const InstDesc &I = f->inst[0];
            LevelPlan pl{};
            pl.t = t;
            pl.nw = lv.nw;
            pl.count = t < I.sstar ? f->sp_pool[I.sp + t + 1] - f->sp_pool[I.sp + t] : 0;
            STOTREE_HIP(hipMalloc(&pl.items, sizeof(Item) * std::max(1, pl.count)));
            f->panel_levels.push_back(pl);
            STOTREE_HIP(hipMemcpy(pl.items, items.data(), sizeof(Item) * pl.count, hipMemcpyHostToDevice));
        }
    }
    // trunk modes 3 and 4: each instance's first stages with at most
    // fuse_limit nodes run in one launch per direction (deepest stage first
    // backward, root first forward); the other stages above s* one launch each
    free_level(f->fused_bwd);
    free_level(f->fused_fwd);
    f->fused_bwd = LevelPlan{};
    f->fused_fwd = LevelPlan{};
    for (auto &lv : f->rest_levels) free_level(lv);
    f->rest_levels.clear();
    if (f->trunk_fused >= 3) {
        const int lim = fuse_limit(f->trunk_fused);
        std::vector<int> depth(f->ninst, 0);
        int dmax = 0;
        for (int b = 0; b < f->ninst; ++b) {
            const InstDesc &I = f->inst[b];
            const int *sp = f->sp_pool.data() + I.sp;
            int d = 0;
            while (d < I.sstar && sp[d + 1] - sp[d] <= lim) ++d;
            depth[b] = d;
            dmax = std::max(dmax, d);
        }
        std::vector<std::vector<Item>> by_stage(dmax);
        int widest = 1;
        for (int t = 0; t < dmax; ++t) {
            for (int b = 0; b < f->ninst; ++b) {
                if (t >= depth[b]) continue;
                const int *sp = f->sp_pool.data() + f->inst[b].sp;
                const int flag = t + 1 < depth[b] ? kFusedKids : 0;
                for (int i = sp[t]; i < sp[t + 1]; ++i) by_stage[t].push_back({b, i | flag});
            }
            widest = std::max(widest, (int)by_stage[t].size());
        }
        std::vector<Item> bwd, fwd;
        for (int t = dmax - 1; t >= 0; --t) bwd.insert(bwd.end(), by_stage[t].begin(), by_stage[t].end());
        for (int t = 0; t < dmax; ++t) fwd.insert(fwd.end(), by_stage[t].begin(), by_stage[t].end());
        for (int dir = 0; dir < 2; ++dir) {
            LevelPlan &lv = dir == 0 ? f->fused_bwd : f->fused_fwd;
            const std::vector<Item> &v = dir == 0 ? bwd : fwd;
            lv.t = -1;
            lv.count = (int)v.size();
            lv.nw = trunk_waves(widest, 2, max_ldM, f->trunk_cap);
            if (v.empty()) continue;
            STOTREE_HIP(hipMalloc(&lv.items, sizeof(Item) * v.size()));
            STOTREE_HIP(hipMemcpy(lv.items, v.data(), sizeof(Item) * v.size(), hipMemcpyHostToDevice));
        }
        for (int t = 0; t < max_sstar; ++t) {
            std::vector<Item> items;
            for (int b = 0; b < f->ninst; ++b) {
                const InstDesc &I = f->inst[b];
                if (t < depth[b] || t >= I.sstar) continue;
                const int *sp = f->sp_pool.data() + I.sp;
                for (int i = sp[t]; i < sp[t + 1]; ++i) items.push_back({b, i});
            }
            if (items.empty()) continue;
            LevelPlan lv{};
            lv.t = t;
            lv.count = (int)items.size();
            lv.nw = trunk_waves(lv.count, 2, max_ldM, f->trunk_cap);
            STOTREE_HIP(hipMalloc(&lv.items, sizeof(Item) * items.size()));
            f->rest_levels.push_back(lv);
            STOTREE_HIP(hipMemcpy(lv.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
        }
    }
    // one-launch backward trunk: its entry nodes and the per-node counters
    if (f->trunk_entry.items) { (void)hipFree(f->trunk_entry.items); f->trunk_entry.items = nullptr; }
    f->trunk_entry.count = 0;
    {
        std::vector<Item> entry;
        for (int b = 0; b < f->ninst; ++b) {
            const InstDesc &I = f->inst[b];
            if (I.sstar < 1) continue;
            const int *sp = f->sp_pool.data() + I.sp;
            for (int i = sp[I.sstar - 1]; i < sp[I.sstar]; ++i) entry.push_back({b, i});
        }
        f->trunk_entry.t = -1;
        f->trunk_entry.count = (int)entry.size();
        f->trunk_entry.nw = trunk_waves(f->trunk_entry.count, 2, max_ldM, f->trunk_cap);
        if (!entry.empty()) {
            STOTREE_HIP(hipMalloc(&f->trunk_entry.items, sizeof(Item) * entry.size()));
            STOTREE_HIP(hipMemcpy(f->trunk_entry.items, entry.data(), sizeof(Item) * entry.size(),
                                  hipMemcpyHostToDevice));
            if (!f->trunk_cnt) STOTREE_HIP(hipMalloc(&f->trunk_cnt, sizeof(int) * (size_t)(f->V_tot + 1)));
            // counters, flags and the fused launches' error word start at zero
            STOTREE_HIP(hipMemset(f->trunk_cnt, 0, sizeof(int) * (size_t)(f->V_tot + 1)));
        }
    }
    return STOTREE_OK;
}

namespace {

// Affine terms of copy k with disturbances c_k (node 0 ignored): chat_k,i =
// chat_0,i + P_i (c_k,i - c_0,i) for i >= 1 (the q / p parts are those of
// copy 0), chat_k,0 = chat_0,0; cvec_k = c_k with node 0 zero.
__global__ void copy_affine_kernel(const double *Pcal, const double *chat0, const double *c0, const double *ck_all,
                                   double *chat, double *cvec, int count, int V, int nx)
{
    const long long per = (long long)V * nx;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)count * per;
         e += (long long)gridDim.x * blockDim.x) {
        const long long k = e / per, rem = e - k * per;
        const int i = (int)(rem / nx), r = (int)(rem - (long long)i * nx);
        const double *ck = ck_all + k * per;
        double s = chat0[rem];
        if (i > 0) {
            const double *Pi = Pcal + (long long)i * nx * nx + (long long)r * nx;
            for (int c = 0; c < nx; ++c) s = fma(Pi[c], ck[(long long)i * nx + c] - c0[(long long)i * nx + c], s);
        }
        chat[e] = s;
        cvec[e] = i > 0 ? ck[rem] : 0.0;
    }
}

}  // namespace

// Turn a one-instance handle into count instances that share its tree,
// factors and boxes (each with its own x0 and vectors, concatenated in
// instance order; with c_host, also its own disturbances).
int replicate_instances(tree_factors *f, int count, const double *c_host, hipStream_t st)
{
    if (f->ninst != 1 || count < 1) { set_error("tree_factor_shared: bad instance count"); return STOTREE_ERR_ARG; }
    if (f->cmap) { set_error("tree_factor_shared: a constraint map is not supported on shared handles"); return STOTREE_ERR_ARG; }
    const InstDesc I0 = f->inst[0];
    const long long xl = (long long)I0.V * I0.nx, ul = (long long)I0.Vnl * I0.nu;
    if (c_host) {
        if (!f->Pcal) { set_error("tree_factor_shared: value-function Hessians were not kept"); return STOTREE_ERR_ARG; }
        for (long long e = 0; e < (long long)count * xl; ++e)
            if (!std::isfinite(c_host[e]) && e % xl >= I0.nx) {
                set_error("tree_factor_shared: non-finite disturbance");
                return STOTREE_ERR_NUMERIC;
            }
        double *dc = nullptr, *chat = nullptr, *cvec = nullptr;
        struct Tmp { double *&p; ~Tmp() { if (p) (void)hipFree(p); } } tdc{dc};
        STOTREE_HIP(hipMalloc(&dc, sizeof(double) * (size_t)(count * xl)));
        STOTREE_HIP(hipMemcpy(dc, c_host, sizeof(double) * (size_t)(count * xl), hipMemcpyHostToDevice));
        STOTREE_HIP(hipMalloc(&chat, sizeof(double) * (size_t)(count * xl)));
        if (hipMalloc(&cvec, sizeof(double) * (size_t)(count * xl)) != hipSuccess) {
            (void)hipFree(chat);
            set_error("tree_factor_shared: out of memory");
            return STOTREE_ERR_OOM;
        }
        const long long n = count * xl;
        const unsigned g = (unsigned)std::min<long long>(65535, (n + 255) / 256);
        hipLaunchKernelGGL(copy_affine_kernel, dim3(g), dim3(256), 0, st, f->Pcal, f->chat + I0.chat,
                           f->cvec + I0.c, dc, chat, cvec, count, I0.V, I0.nx);
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(chat);
            (void)hipFree(cvec);
            set_error(std::string("tree_factor_shared: ") + hipGetErrorString(e));
            return STOTREE_ERR_DEVICE;
        }
        (void)hipFree(f->chat);
        (void)hipFree(f->cvec);
        f->chat = chat;
        f->cvec = cvec;
        f->bytes += (size_t)(count - 1) * xl * 2 * sizeof(double);
    }
    if (f->Pcal) { (void)hipFree(f->Pcal); f->Pcal = nullptr; }
    if (count == 1 && !c_host) return STOTREE_OK;
    f->inst.assign(count, I0);
    for (int k = 0; k < count; ++k) {
        InstDesc &I = f->inst[k];
        I.y = k * I0.m; I.x = k * xl; I.u = k * ul; I.x0 = (long long)k * I0.nx; I.box = 0;
        I.node0 = (long long)k * I0.V;
        if (c_host) { I.chat = k * xl; I.c = k * xl; }
    }
    f->ninst = count;
    f->shared = count;
    f->m_tot = count * I0.m; f->n_tot *= count; f->x_tot = count * xl; f->u_tot = count * ul;
    f->nx_tot = (long long)count * I0.nx;
    f->V_tot = (long long)count * I0.V;
    if (f->trunk_cnt) { (void)hipFree(f->trunk_cnt); f->trunk_cnt = nullptr; }
    if (f->d_inst) (void)hipFree(f->d_inst);
    f->d_inst = nullptr;
    STOTREE_HIP(hipMalloc(&f->d_inst, sizeof(InstDesc) * count));
    STOTREE_HIP(hipMemcpy(f->d_inst, f->inst.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice));
    f->d_inst_xu = f->d_inst;
    f->mxu_tot = f->m_tot;
    f->last_info.assign(count, solver_info{});
    return build_schedule(f);
}

int factor_forest(int count, const tree_desc *trees, const problem_data *datas, int precondition,
                  hipStream_t st, tree_factors **out, bool keep_pcal)
{
    if (!out) { set_error("tree_factor: out is NULL"); return STOTREE_ERR_ARG; }
    *out = nullptr;
    if (count < 1 || !trees || !datas) { set_error("tree_factor: no instances"); return STOTREE_ERR_ARG; }
    for (int b = 0; b < count; ++b) {
        const int rc = validate(&trees[b], &datas[b], count == 1 ? "tree_factor" :
                                "tree_factor_batch[" + std::to_string(b) + "]");
        if (rc) return rc;
    }
    tree_factors *f = new tree_factors();
    struct Guard {
        tree_factors *&f;
        bool ok = false;
        ~Guard() { if (!ok) free_tree(f); }
    } guard{f};
    f->ninst = count;
    f->precondition = precondition ? 1 : 0;
    f->inst.resize(count);
    std::vector<RawDesc> raw(count);
    long long oMb = 0, oMf = 0, oKb = 0, oKf = 0, oRn = 0, ochat = 0, osig = 0, osc = 0, oy = 0, ox = 0,
              ou = 0, ox0 = 0, onode = 0, oF = 0, oxu = 0;
    bool anyW = false;
    RawDesc ro{};
    int osp = 0, ocp = 0;
    bool anyS = false, anyq = false, anyr = false, anyp = false;
    long long max_slot = 0;
    for (int b = 0; b < count; ++b) {
        const tree_desc &t = trees[b];
        const problem_data &d = datas[b];
        InstDesc &I = f->inst[b];
        I.nx = t.nx; I.nu = t.nu; I.N = t.N; I.V = t.num_nodes; I.Vnl = t.stage_ptr[t.N];
        I.ldM = pad2(I.nx + I.nu); I.ldx = pad2(I.nx); I.ldu = pad2(I.nu);
        const int *sp = t.stage_ptr;
        int sstar = I.N;
        while (sstar > 0 && sp[sstar] - sp[sstar - 1] == sp[I.N + 1] - sp[I.N]) --sstar;
        I.sstar = sstar;
        I.nchains = sp[I.N + 1] - sp[I.N];
        I.sp = osp; I.cp = ocp;
        I.Mb = oMb; I.Mf = oMf; I.Kb = oKb; I.Kf = oKf; I.Rn = oRn;
        I.chat = ochat; I.c = ochat; I.sig = osig; I.sc = osc;
        I.y = oy; I.x = ox; I.u = ou; I.x0 = ox0; I.box = oy; I.node0 = onode;
        I.cmap = d.F != nullptr;
        I.nc = I.cmap ? d.nc : I.nx + I.nu;
        I.ncN = I.cmap ? d.ncN : I.nx;
        I.Fo = oF;
        if (I.cmap) oF += (long long)d.nc * (I.nx + I.nu) + (long long)d.ncN * I.nx;
        I.m = (long long)I.Vnl * I.nc + (long long)(I.V - I.Vnl) * I.ncN;
        oxu += (long long)I.Vnl * (I.nx + I.nu) + (long long)(I.V - I.Vnl) * I.nx;
        f->cmap |= I.cmap;
        anyW |= d.wgt != nullptr;
        const long long V = I.V, Vnl = I.Vnl, Vl = I.V - I.Vnl, nx = I.nx, nu = I.nu;
        oMb += V * nx * I.ldM; oMf += V * (nx + nu) * I.ldx; oKb += Vnl * nu * I.ldx;
        oKf += Vnl * nx * I.ldu; oRn += Vnl * nu * I.ldu; ochat += V * nx; osig += Vnl * nu; osc += V;
        oy += I.m; ox += V * nx; ou += Vnl * nu; ox0 += nx; onode += V;
        osp += I.N + 2; ocp += I.Vnl + 1;
        RawDesc &R = raw[b];
        R = ro;
        ro.A += V * nx * nx; ro.B += V * nx * nu; ro.c += V * nx; ro.Q += Vnl * nx * nx;
        ro.R += Vnl * nu * nu; ro.S += Vnl * nu * nx; ro.q += Vnl * nx; ro.r += Vnl * nu;
        ro.P += Vl * nx * nx; ro.p += Vl * nx; ro.prob += V; ro.Pcal += V * nx * nx;
        anyS |= d.S != nullptr; anyq |= d.q != nullptr; anyr |= d.r != nullptr; anyp |= d.p != nullptr;
        max_slot = std::max(max_slot, nx * (nx + nu) + 2 * nu * nu + nu * nx);
        f->max_width = std::max(f->max_width, I.nx + I.nu);
        f->n_tot += Vnl * nu + (V - 1) * nx;
        f->V_tot += V;
    }
    f->m_tot = oy; f->x_tot = ox; f->u_tot = ou; f->nx_tot = ox0; f->mxu_tot = oxu;
    // host pools of the stage/child pointers
    f->sp_pool.resize(osp);
    std::vector<int> cp_pool(ocp);
    for (int b = 0; b < count; ++b) {
        const InstDesc &I = f->inst[b];
        std::memcpy(f->sp_pool.data() + I.sp, trees[b].stage_ptr, sizeof(int) * (I.N + 2));
        std::memcpy(cp_pool.data() + I.cp, trees[b].child_ptr, sizeof(int) * (I.Vnl + 1));
    }
    auto dalloc = [&](auto **p, size_t n) -> int {
        STOTREE_HIP(hipMalloc((void **)p, sizeof(**p) * (n ? n : 1)));
        f->bytes += sizeof(**p) * n;
        return STOTREE_OK;
    };
    int rc;
    if ((rc = dalloc(&f->d_inst, count)) || (rc = dalloc(&f->d_sp, osp)) || (rc = dalloc(&f->d_cp, ocp)) ||
        (rc = dalloc(&f->d_anc, osc)) ||
        (rc = dalloc(&f->Mb, oMb)) || (rc = dalloc(&f->Mf, oMf)) || (rc = dalloc(&f->Kb, oKb)) ||
        (rc = dalloc(&f->Kf, oKf)) || (rc = dalloc(&f->Rn, oRn)) || (rc = dalloc(&f->chat, ochat)) ||
        (rc = dalloc(&f->sig, osig)) || (rc = dalloc(&f->cvec, ochat)) || (rc = dalloc(&f->sc, osc)) ||
        (rc = dalloc(&f->lo, oy)) || (rc = dalloc(&f->hi, oy)))
        return rc;
    STOTREE_HIP(hipMemcpy(f->d_inst, f->inst.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice));
    f->d_inst_xu = f->d_inst;
    if (f->cmap) {
        // the sweeps read and write the (x, u) layout: their descriptors
        // place each instance in that layout
        std::vector<InstDesc> ixu = f->inst;
        long long o = 0;
        for (InstDesc &I : ixu) {
            I.y = o;
            I.m = (long long)I.Vnl * (I.nx + I.nu) + (long long)(I.V - I.Vnl) * I.nx;
            o += I.m;
        }
        STOTREE_HIP(hipMalloc(&f->d_inst_xu, sizeof(InstDesc) * count));
        f->bytes += sizeof(InstDesc) * count;
        STOTREE_HIP(hipMemcpy(f->d_inst_xu, ixu.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice));
        std::vector<double> Fm((size_t)std::max(1LL, oF));
        for (int b = 0; b < count; ++b) {
            const InstDesc &I = f->inst[b];
            if (!I.cmap) continue;
            const problem_data &d = datas[b];
            double *dst = Fm.data() + I.Fo;
            std::memcpy(dst, d.F, sizeof(double) * I.nc * I.nx);
            std::memcpy(dst + (size_t)I.nc * I.nx, d.G, sizeof(double) * I.nc * I.nu);
            if (I.ncN > 0)
                std::memcpy(dst + (size_t)I.nc * (I.nx + I.nu), d.FN, sizeof(double) * I.ncN * I.nx);
        }
        if ((rc = dalloc(&f->Fm, oF))) return rc;
        STOTREE_HIP(hipMemcpy(f->Fm, Fm.data(), sizeof(double) * oF, hipMemcpyHostToDevice));
    }
    if (anyW) {
        // soft rows: pi_i * wgt (+inf: hard) and the Huber thresholds
        std::vector<double> pw((size_t)oy), hb((size_t)oy, 0.0);
        for (int b = 0; b < count; ++b) {
            const InstDesc &I = f->inst[b];
            const problem_data &d = datas[b];
            for (int i = 0; i < I.V; ++i) {
                const int rows = i < I.Vnl ? I.nc : I.ncN;
                const long long o = i < I.Vnl ? (long long)i * I.nc
                                              : (long long)I.Vnl * I.nc + (long long)(i - I.Vnl) * I.ncN;
                for (int a = 0; a < rows; ++a) {
                    const size_t k = (size_t)(I.y + o + a), kl = (size_t)(o + a);
                    pw[k] = d.wgt ? trees[b].prob[i] * d.wgt[kl] : INFINITY;
                    hb[k] = (d.wgt && d.hub) ? d.hub[kl] : 0.0;
                }
            }
        }
        if ((rc = dalloc(&f->pw, oy)) || (rc = dalloc(&f->hub, oy))) return rc;
        STOTREE_HIP(hipMemcpy(f->pw, pw.data(), sizeof(double) * oy, hipMemcpyHostToDevice));
        STOTREE_HIP(hipMemcpy(f->hub, hb.data(), sizeof(double) * oy, hipMemcpyHostToDevice));
    }
    STOTREE_HIP(hipMemcpy(f->d_sp, f->sp_pool.data(), sizeof(int) * osp, hipMemcpyHostToDevice));
    STOTREE_HIP(hipMemcpy(f->d_cp, cp_pool.data(), sizeof(int) * ocp, hipMemcpyHostToDevice));
    for (int b = 0; b < count; ++b)
        STOTREE_HIP(hipMemcpy(f->d_anc + f->inst[b].sc, trees[b].ancestor, sizeof(int) * f->inst[b].V,
                              hipMemcpyHostToDevice));
    // box rows in the dual layout (a data rearrangement, no arithmetic)
    {
        std::vector<double> lo((size_t)oy), hi((size_t)oy);
        for (int b = 0; b < count; ++b) {
            const InstDesc &I = f->inst[b];
            const problem_data &d = datas[b];
            if (I.cmap) {
                std::memcpy(&lo[I.y], d.zmin, sizeof(double) * I.m);
                std::memcpy(&hi[I.y], d.zmax, sizeof(double) * I.m);
                continue;
            }
            for (int i = 0; i < I.V; ++i) {
                const size_t o = I.y + (i < I.Vnl ? (size_t)i * (I.nx + I.nu) : (size_t)I.Vnl * I.nu + (size_t)i * I.nx);
                std::memcpy(&lo[o], d.xmin + (size_t)i * I.nx, sizeof(double) * I.nx);
                std::memcpy(&hi[o], d.xmax + (size_t)i * I.nx, sizeof(double) * I.nx);
                if (i < I.Vnl) {
                    std::memcpy(&lo[o + I.nx], d.umin + (size_t)i * I.nu, sizeof(double) * I.nu);
                    std::memcpy(&hi[o + I.nx], d.umax + (size_t)i * I.nu, sizeof(double) * I.nu);
                }
            }
        }
        STOTREE_HIP(hipMemcpy(f->lo, lo.data(), sizeof(double) * oy, hipMemcpyHostToDevice));
        STOTREE_HIP(hipMemcpy(f->hi, hi.data(), sizeof(double) * oy, hipMemcpyHostToDevice));
    }
    // raw inputs: concatenated pools (a single instance is uploaded in place)
    DevBuf bA, bB, bc, bQ, bR, bS, bq, br, bP, bp, bprob, bPcal, bscr, berr, braw, bitems;
    auto upload = [&](DevBuf &buf, long long total, auto get, auto len) -> int {
        STOTREE_HIP(hipMalloc(&buf.p, sizeof(double) * (total ? total : 1)));
        long long o = 0;
        for (int b = 0; b < count; ++b) {
            const double *h = get(b);
            const long long n = len(b);
            if (h) STOTREE_HIP(hipMemcpy((double *)buf.p + o, h, sizeof(double) * n, hipMemcpyHostToDevice));
            else STOTREE_HIP(hipMemset((double *)buf.p + o, 0, sizeof(double) * n));
            o += n;
        }
        return STOTREE_OK;
    };
#define NODES(expr) [&](int b) -> long long { const InstDesc &I = f->inst[b]; (void)I; return (expr); }
    if ((rc = upload(bA, ro.A, [&](int b) { return datas[b].A; }, NODES((long long)I.V * I.nx * I.nx))) ||
        (rc = upload(bB, ro.B, [&](int b) { return datas[b].B; }, NODES((long long)I.V * I.nx * I.nu))) ||
        (rc = upload(bc, ro.c, [&](int b) { return datas[b].c; }, NODES((long long)I.V * I.nx))) ||
        (rc = upload(bQ, ro.Q, [&](int b) { return datas[b].Q; }, NODES((long long)I.Vnl * I.nx * I.nx))) ||
        (rc = upload(bR, ro.R, [&](int b) { return datas[b].R; }, NODES((long long)I.Vnl * I.nu * I.nu))) ||
        (anyS && (rc = upload(bS, ro.S, [&](int b) { return datas[b].S; }, NODES((long long)I.Vnl * I.nu * I.nx)))) ||
        (anyq && (rc = upload(bq, ro.q, [&](int b) { return datas[b].q; }, NODES((long long)I.Vnl * I.nx)))) ||
        (anyr && (rc = upload(br, ro.r, [&](int b) { return datas[b].r; }, NODES((long long)I.Vnl * I.nu)))) ||
        (rc = upload(bP, ro.P, [&](int b) { return datas[b].P; }, NODES((long long)(I.V - I.Vnl) * I.nx * I.nx))) ||
        (anyp && (rc = upload(bp, ro.p, [&](int b) { return datas[b].p; }, NODES((long long)(I.V - I.Vnl) * I.nx))) ) ||
        (rc = upload(bprob, ro.prob, [&](int b) { return trees[b].prob; }, NODES((long long)I.V))))
        return rc;
#undef NODES
    // scratch for the widest stage
    int maxw = 1;
    int max_depth = 0;
    for (int b = 0; b < count; ++b) max_depth = std::max(max_depth, f->inst[b].N);
    std::vector<std::vector<Item>> level_items(max_depth);
    for (int b = 0; b < count; ++b) {
        const InstDesc &I = f->inst[b];
        const int *sp = f->sp_pool.data() + I.sp;
        for (int t = 0; t < I.N; ++t)
            for (int i = sp[t]; i < sp[t + 1]; ++i) level_items[t].push_back({b, i});
    }
    for (auto &li : level_items) maxw = std::max<int>(maxw, (int)li.size());
    STOTREE_HIP(hipMalloc(&bPcal.p, sizeof(double) * (size_t)std::max(1LL, ro.Pcal)));
    STOTREE_HIP(hipMalloc(&bscr.p, sizeof(double) * (size_t)maxw * max_slot));
    STOTREE_HIP(hipMalloc(&berr.p, sizeof(int)));
    STOTREE_HIP(hipMalloc(&braw.p, sizeof(RawDesc) * count));
    std::vector<Item> all_items;
    std::vector<size_t> level_off(max_depth + 1, 0);
    for (int t = 0; t < max_depth; ++t) {
        level_off[t] = all_items.size();
        all_items.insert(all_items.end(), level_items[t].begin(), level_items[t].end());
    }
    level_off[max_depth] = all_items.size();
    STOTREE_HIP(hipMalloc(&bitems.p, sizeof(Item) * std::max<size_t>(1, all_items.size())));
    STOTREE_HIP(hipMemcpy(bitems.p, all_items.data(), sizeof(Item) * all_items.size(), hipMemcpyHostToDevice));
    STOTREE_HIP(hipMemcpy(braw.p, raw.data(), sizeof(RawDesc) * count, hipMemcpyHostToDevice));
    STOTREE_HIP(hipMemset(berr.p, 0, sizeof(int)));

    FactorArgs a{};
    a.inst = f->d_inst; a.raw = (const RawDesc *)braw.p; a.sp = f->d_sp; a.cp = f->d_cp;
    a.prob = (const double *)bprob.p; a.A = (const double *)bA.p; a.B = (const double *)bB.p;
    a.c = (const double *)bc.p; a.Q = (const double *)bQ.p; a.R = (const double *)bR.p;
    a.S = (const double *)bS.p; a.q = (const double *)bq.p; a.r = (const double *)br.p;
    a.P = (const double *)bP.p; a.p = (const double *)bp.p;
    a.hasS = anyS; a.hasq = anyq; a.hasr = anyr; a.hasp = anyp;
    a.Pcal = (double *)bPcal.p; a.scratch = (double *)bscr.p; a.slot = max_slot;
    a.Mb = f->Mb; a.Mf = f->Mf; a.Kb = f->Kb; a.Kf = f->Kf; a.Rn = f->Rn;
    a.chat = f->chat; a.sig = f->sig; a.cvec = f->cvec; a.sc = f->sc; a.err = (int *)berr.p;
    for (int b = 0; b < count; ++b) {
        const InstDesc &I = f->inst[b];
        const long long work = (long long)I.V * (I.nx * I.ldM + (I.nx + I.nu) * I.ldx);
        const unsigned g = (unsigned)std::min<long long>(4096, (work + 255) / 256);
        hipLaunchKernelGGL(pack_dynamics_kernel, dim3(g), dim3(256), 0, st, a, b);
        hipLaunchKernelGGL(factor_leaves_kernel, dim3((unsigned)(I.V - I.Vnl)), dim3(64), 0, st, a, b);
    }
    // the tiled children's products when every instance's sizes fit
    bool tiled = true, wide_k = true;
    int lds8 = 0, lds16 = 0;
    for (int b = 0; b < count; ++b) {
        const int nx = f->inst[b].nx, nu = f->inst[b].nu;
        const FactorTiles f8(nx, nu, 8), f16(nx, nu, 16);
        tiled = tiled && f8.fits(nx, nu);
        wide_k = wide_k && f16.fits(nx, nu);
        lds8 = std::max(lds8, f8.lds_doubles(nx, nu));
        lds16 = std::max(lds16, f16.lds_doubles(nx, nu));
    }
    for (int t = max_depth - 1; t >= 0; --t) {
        const size_t n = level_off[t + 1] - level_off[t];
        if (n == 0) continue;
        a.items = (const Item *)bitems.p + level_off[t];
        if (tiled && wide_k)
            hipLaunchKernelGGL((factor_stage_kernel<true, 16>), dim3((unsigned)n), dim3(kFactorThreads),
                               sizeof(double) * (size_t)lds16, st, a);
        else if (tiled)
            hipLaunchKernelGGL((factor_stage_kernel<true, 8>), dim3((unsigned)n), dim3(kFactorThreads),
                               sizeof(double) * (size_t)lds8, st, a);
        else
            hipLaunchKernelGGL(factor_stage_kernel<false>, dim3((unsigned)n), dim3(kFactorThreads), 0, st, a);
    }
    STOTREE_HIP(hipGetLastError());
    int err = 0;
    STOTREE_HIP(hipMemcpyAsync(&err, berr.p, sizeof(int), hipMemcpyDeviceToHost, st));
    STOTREE_HIP(hipStreamSynchronize(st));
    if (err != 0) {
        set_error("tree_factor: R-tilde is not positive definite at some node");
        return err;
    }
    if ((rc = build_schedule(f))) return rc;
    if (keep_pcal) {
        f->Pcal = (double *)bPcal.p;
        bPcal.p = nullptr;
    }
    f->last_info.assign(count, solver_info{});
    guard.ok = true;
    *out = f;
    return STOTREE_OK;
}

}  // namespace stotree
