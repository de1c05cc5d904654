// Stage-parallel sweeps over the scenario tree: Algorithm 3 (dual gradient
// x(y)) and Algorithm 4 (Hessian-vector products x-hat(r)) of arXiv 2107.01745,
// Sec. III-D, written for CDNA4 wavefronts.
//
// Algebra.  With R~_i the input Hessian of node i's subproblem and K_i its
// feedback gain, the paper's per-edge factors are Theta_j = -R~_i^{-1} B_j' and
// Lambda_j = A_j + B_j K_i, and its per-node terms are Phi_i y_i =
// -R~_i^{-1} y_i^u, D_i' y_i = y_i^x + K_i' y_i^u.  Collecting the terms per
// node, the backward step of node i reads
//     g_i    = s_i y_i^u + pi_i r_i + sum_j B_j' qhat_j          (nu)
//     k_i    = -R~_i^{-1} g_i                                    (u offset)
//     qhat_i = chat_i + s_i y_i^x + sum_j A_j' qhat_j + K_i' g_i (nx)
// which is the paper's recursion regrouped so that the per-edge matrices
// streamed are the dynamics [A_j B_j] themselves (read once backward, once
// forward) and no Lambda/Theta copies are stored.  The forward step is
// u_i = K_i x_i + k_i and x_j = A_j x_i + B_j u_i + c_j.  s_i = sqrt(pi_i)
// under the preconditioning of Sec. III-E (1 otherwise).  Algorithm 4 drops
// pi r, chat, c and uses x_0 = 0.
//
// Forest.  A handle may hold many independent trees of different sizes; every
// launch walks a flat work list of (instance, node) or (instance, chain)
// pairs and reads the instance's sizes and pool offsets from its descriptor.
//
// Mapping.  One wavefront per node (per chain, below).  Each lane owns two
// adjacent output entries; matrices are stored in the orientation of the pass
// that reads them, so every row of a matrix is one contiguous, 16-byte-aligned
// load across the wavefront, multiplied by a broadcast entry of the input
// vector held in LDS.  The nodes from stage s* on have one child each (the
// scenario fan-out has ended); the tree below s* is a set of independent
// chains, each walked by one wavefront through all its stages with qhat / x
// carried in LDS, so those stages need no grid-wide synchronisation.  Stages
// above s* are launched stage by stage.
#include <algorithm>

#include "internal.h"

namespace stotree {

namespace {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dual-layout offset of node i inside its instance.
__device__ __forceinline__ long long dual_off(const InstDesc &I, int i)
{
    return i < I.Vnl ? (long long)i * (I.nx + I.nu) : (long long)I.Vnl * I.nu + (long long)i * I.nx;
}
__device__ __forceinline__ const double *y_ptr(const SweepArgs &a, const InstDesc &I, int k, int i)
{
    return a.y + k * a.y_rs + I.y + dual_off(I, i);
}
__device__ __forceinline__ double *x_ptr(const SweepArgs &a, const InstDesc &I, int k, int i)
{
    return a.dual_out ? a.xo + k * a.xo_rs + I.y + dual_off(I, i)
                      : a.xo + k * a.xo_rs + I.x + (long long)i * I.nx;
}
__device__ __forceinline__ double *u_ptr(const SweepArgs &a, const InstDesc &I, int k, int i)
{
    return a.dual_out ? a.xo + k * a.xo_rs + I.y + (long long)i * (I.nx + I.nu) + I.nx
                      : a.uo + k * a.uo_rs + I.u + (long long)i * I.nu;
}
__device__ __forceinline__ double *qhat_ptr(const SweepArgs &a, const InstDesc &I, int k, int i)
{
    return a.qhat + k * a.qhat_rs + I.x + (long long)i * I.nx;
}
__device__ __forceinline__ double *kbuf_ptr(const SweepArgs &a, const InstDesc &I, int k, int i)
{
    return a.kbuf + k * a.kbuf_rs + I.u + (long long)i * I.nu;
}
__device__ __forceinline__ bool skipped(const SweepArgs &a, int b)
{
    return a.done && a.done[(long long)b * a.done_stride];
}

// acc[k][ch][e] += sum_{r0<=r<r1} M[r][c] * v_k[r] for the lane's columns
// c = 2*lane + 128*ch + e < W, with M row-major of leading dimension ld and v_k
// in LDS at v + k*ldv.  The loads carry no lane condition (lanes past W re-read
// column 0 and their sums are never stored) and rows go in batches of
// kRowBatch, double-buffered: the next batch is issued before the current one
// is multiplied, so up to 2*kRowBatch row loads are in flight per wavefront.
constexpr int kRowBatch = 8;

template <int CH>
__device__ __forceinline__ void load_rows(double2 (&m)[kRowBatch][CH], const double *__restrict__ M,
                                          int ld, int r, const int (&col)[CH])
{
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
            m[u][ch] = *reinterpret_cast<const double2 *>(M + (long long)(r + u) * ld + col[ch]);
}

template <int NRHS, int CH>
__device__ __forceinline__ void fma_rows(const double2 (&m)[kRowBatch][CH], const double *v, int ldv,
                                         int r, double (&acc)[NRHS][CH][2])
{
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double vk = v[k * ldv + r + u];
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                acc[k][ch][0] = fma(m[u][ch].x, vk, acc[k][ch][0]);
                acc[k][ch][1] = fma(m[u][ch].y, vk, acc[k][ch][1]);
            }
        }
}

template <int NRHS, int CH>
__device__ __forceinline__ void gemv_rows(const double *__restrict__ M, int ld, int r0, int r1, int W,
                                          const double *v, int ldv, double (&acc)[NRHS][CH][2],
                                          int lane)
{
    int col[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
        col[ch] = c0 < W ? c0 : 0;
    }
    int r = r0;
    int nb = (r1 - r0) / kRowBatch;
    double2 m0[kRowBatch][CH], m1[kRowBatch][CH];
    if (nb > 0) load_rows<CH>(m0, M, ld, r, col);
    while (nb >= 2) {
        load_rows<CH>(m1, M, ld, r + kRowBatch, col);
        fma_rows<NRHS, CH>(m0, v, ldv, r, acc);
        if (nb >= 3) load_rows<CH>(m0, M, ld, r + 2 * kRowBatch, col);
        fma_rows<NRHS, CH>(m1, v, ldv, r + kRowBatch, acc);
        r += 2 * kRowBatch;
        nb -= 2;
    }
    if (nb == 1) {
        fma_rows<NRHS, CH>(m0, v, ldv, r, acc);
        r += kRowBatch;
    }
    for (; r < r1; ++r) {
        double2 m[CH];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
            m[ch] = *reinterpret_cast<const double2 *>(M + (long long)r * ld + col[ch]);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double vk = v[k * ldv + r];
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                acc[k][ch][0] = fma(m[ch].x, vk, acc[k][ch][0]);
                acc[k][ch][1] = fma(m[ch].y, vk, acc[k][ch][1]);
            }
        }
    }
}

// dst[k*ld + off + c] = acc[k][.][.] for the lane's columns c < dim.
template <int NRHS, int CH>
__device__ __forceinline__ void store_acc(double *dst, int ld, int off, int dim,
                                          const double (&acc)[NRHS][CH][2], int lane)
{
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (c0 < dim) dst[k * ld + off + c0] = acc[k][ch][0];
            if (c0 + 1 < dim) dst[k * ld + off + c0 + 1] = acc[k][ch][1];
        }
    }
}

template <int NRHS, int CH>
__device__ __forceinline__ void zero(double (&acc)[NRHS][CH][2])
{
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) acc[k][ch][0] = acc[k][ch][1] = 0.0;
}

// Per-wave LDS of the chain kernels: qx [NRHS][ldq] (qhat or [x;u]), as
// [NRHS][ldq], gs [NRHS][ldq], with ldq the largest padded width.
struct WaveLds {
    double *qx, *as, *gs;
    int ldq;
};

__device__ __forceinline__ WaveLds wave_lds(int ldq, int nrhs, int wave)
{
    extern __shared__ double lds[];
    WaveLds w;
    w.qx = lds + wave * 3 * nrhs * ldq;
    w.as = w.qx + nrhs * ldq;
    w.gs = w.as + nrhs * ldq;
    w.ldq = ldq;
    return w;
}

// Backward step of non-leaf node i of instance I by one wavefront.  If
// child_in_lds, qhat of the (single) child is already in L.qx; otherwise each
// child's qhat is staged from the leaf data or from the global qhat buffer.
// The result qhat_i is left in L.qx and, if store_q, written to the global
// buffer; k_i always goes to kbuf.
template <int NRHS, int CH>
__device__ void bwd_node(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L,
                         bool child_in_lds, bool store_q, int lane)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const int *cp = a.cp + I.cp;
    double acc[NRHS][CH][2];
    zero(acc);
    const int j0 = cp[i], j1 = cp[i + 1];
    for (int j = j0; j < j1; ++j) {
        if (!child_in_lds) {
            if (j >= I.Vnl) {
                const double sj = a.sc ? a.sc[I.sc + j] : 1.0;
                for (int r = lane; r < nx; r += kWave)
#pragma unroll
                    for (int k = 0; k < NRHS; ++k)
                        L.qx[k * L.ldq + r] = sj * y_ptr(a, I, k, j)[r] +
                                              (a.affine ? a.chat[I.chat + (long long)j * nx + r] : 0.0);
            } else {
                for (int r = lane; r < nx; r += kWave)
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) L.qx[k * L.ldq + r] = qhat_ptr(a, I, k, j)[r];
            }
            wave_sync();
        }
        gemv_rows<NRHS, CH>(a.Mb + I.Mb + (long long)j * nx * I.ldM, I.ldM, 0, nx, W, L.qx, L.ldq, acc, lane);
        wave_sync();
    }
    store_acc<NRHS, CH>(L.as, L.ldq, 0, W, acc, lane);  // [sum A'q ; sum B'q]
    wave_sync();
    const double si = a.sc ? a.sc[I.sc + i] : 1.0;
    for (int c = lane; c < nu; c += kWave)
#pragma unroll
        for (int k = 0; k < NRHS; ++k)
            L.gs[k * L.ldq + c] = L.as[k * L.ldq + nx + c] + si * y_ptr(a, I, k, i)[nx + c] +
                                  (a.affine ? a.sig[I.sig + (long long)i * nu + c] : 0.0);
    wave_sync();
    double kacc[NRHS][CH][2], qacc[NRHS][CH][2];
    zero(kacc);
    zero(qacc);
    gemv_rows<NRHS, CH>(a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, 0, nu, nu, L.gs, L.ldq, kacc, lane);
    gemv_rows<NRHS, CH>(a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, 0, nu, nx, L.gs, L.ldq, qacc, lane);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            double *kb = kbuf_ptr(a, I, k, i);
            if (c0 < nu) kb[c0] = kacc[k][ch][0];
            if (c0 + 1 < nu) kb[c0 + 1] = kacc[k][ch][1];
        }
    }
    // qhat_i = [sum A'q]_c + s_i y_i^x + chat_i + (K_i' g_i)
    double qv[NRHS][CH][2];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                double v = 0.0;
                if (c < nx)
                    v = L.as[k * L.ldq + c] + si * y_ptr(a, I, k, i)[c] +
                        (a.affine ? a.chat[I.chat + (long long)i * nx + c] : 0.0) + qacc[k][ch][e];
                qv[k][ch][e] = v;
            }
        }
    }
    wave_sync();  // every lane has finished reading L.qx / L.as
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
            if (c < nx) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) {
                    L.qx[k * L.ldq + c] = qv[k][ch][e];
                    if (store_q) qhat_ptr(a, I, k, i)[c] = qv[k][ch][e];
                }
            }
        }
    }
    wave_sync();
}

// Forward step of non-leaf node i with x_i in L.qx[0..nx).  Writes u_i and the
// children's x_j to the outputs; for a single-child chain the child's x is
// left in L.qx.
template <int NRHS, int CH>
__device__ void fwd_node(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L, bool keep_child,
                         int lane)
{
    const int nx = I.nx, nu = I.nu;
    const int *cp = a.cp + I.cp;
    double uacc[NRHS][CH][2];
    zero(uacc);
    gemv_rows<NRHS, CH>(a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, 0, nx, nu, L.qx, L.ldq, uacc, lane);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 128 * ch;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
            if (c < nu) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) {
                    const double uval = uacc[k][ch][e] + kbuf_ptr(a, I, k, i)[c];
                    u_ptr(a, I, k, i)[c] = uval;
                    L.qx[k * L.ldq + nx + c] = uval;
                }
            }
        }
    }
    wave_sync();
    const int j0 = cp[i], j1 = cp[i + 1];
    double keep[NRHS][CH][2];
    zero(keep);
    for (int j = j0; j < j1; ++j) {
        double xacc[NRHS][CH][2];
        zero(xacc);
        gemv_rows<NRHS, CH>(a.Mf + I.Mf + (long long)j * (nx + nu) * I.ldx, I.ldx, 0, nx + nu, nx, L.qx, L.ldq,
                            xacc, lane);
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = 2 * lane + 128 * ch;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = c0 + e;
                if (c < nx) {
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) {
                        const double xv = xacc[k][ch][e] + (a.affine ? a.cvec[I.c + (long long)j * nx + c] : 0.0);
                        x_ptr(a, I, k, j)[c] = xv;
                        keep[k][ch][e] = xv;
                    }
                }
            }
        }
    }
    if (keep_child) {
        wave_sync();
        store_acc<NRHS, CH>(L.qx, L.ldq, 0, nx, keep, lane);
        wave_sync();
    }
}

// x_i of the first node a forward pass visits: x0 at the root (written to
// the output too), else the value the previous stage stored.
template <int NRHS>
__device__ void load_x(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L, int lane)
{
    for (int c = lane; c < I.nx; c += kWave)
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            double v;
            if (i == 0) {
                v = a.affine ? a.x0[k * a.x0_rs + I.x0 + c] : 0.0;
                x_ptr(a, I, k, 0)[c] = v;
            } else {
                v = x_ptr(a, I, k, i)[c];
            }
            L.qx[k * L.ldq + c] = v;
        }
    wave_sync();
}

// ---- stages above s*: one workgroup of NW wavefronts per node ----
//
// Backward: the rows of all children's [A_j B_j] are split into NW contiguous
// ranges, one per wavefront; the partial sums meet in LDS in a fixed order
// (deterministic), then the node's -R~^{-1} and K_i rows are split the same
// way.  Forward: the rows of K_i' are split for u_i; the children are dealt
// round-robin to the wavefronts, or, with fewer children than wavefronts,
// each child's rows are split into NW/b blocks reduced through LDS.
__host__ __device__ inline int child_batch(int nrhs, int ldx)
{
    const int cb = 2048 / (nrhs * ldx);
    return cb < 1 ? 1 : (cb > 8 ? 8 : cb);
}

template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) bwd_trunk_kernel(SweepArgs a)
{
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i = it.idx;
    const int nx = I.nx, nu = I.nu, W = nx + nu, ldq = I.ldx, ldM = I.ldM;
    const int *cp = a.cp + I.cp;
    const int CB = child_batch(NRHS, ldq);
    extern __shared__ double lds[];
    double *qs = lds;                          // [CB][NRHS][ldq]
    double *red = qs + CB * NRHS * ldq;        // [NW][NRHS][ldM]
    double *as = red + NW * NRHS * ldM;        // [NRHS][ldM]
    double *gs = as + NRHS * ldM;              // [NRHS][ldu]
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    double acc[NRHS][CH][2];
    zero(acc);
    for (int cb = 0; cb < nch; cb += CB) {
        const int nb = nch - cb < CB ? nch - cb : CB;
        for (int e = threadIdx.x; e < nb * nx; e += blockDim.x) {
            const int c = e / nx, r = e - c * nx, j = j0 + cb + c;
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                double q;
                if (j >= I.Vnl) {
                    const double sj = a.sc ? a.sc[I.sc + j] : 1.0;
                    q = sj * y_ptr(a, I, k, j)[r] + (a.affine ? a.chat[I.chat + (long long)j * nx + r] : 0.0);
                } else {
                    q = qhat_ptr(a, I, k, j)[r];
                }
                qs[(c * NRHS + k) * ldq + r] = q;
            }
        }
        __syncthreads();
        const int R = nb * nx;
        const int r0 = (int)((long long)R * w / NW), r1 = (int)((long long)R * (w + 1) / NW);
        for (int c = r0 / nx; c < nb && c * nx < r1; ++c) {
            const int lo = (r0 > c * nx ? r0 : c * nx) - c * nx;
            const int hi = (r1 < (c + 1) * nx ? r1 : (c + 1) * nx) - c * nx;
            if (lo < hi)
                gemv_rows<NRHS, CH>(a.Mb + I.Mb + (long long)(j0 + cb + c) * nx * ldM, ldM, lo, hi, W,
                                    qs + c * NRHS * ldq, ldq, acc, lane);
        }
        __syncthreads();
    }
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, W, acc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
        const int k = e / W, c = e - k * W;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        as[k * ldM + c] = s;
    }
    __syncthreads();
    const double si = a.sc ? a.sc[I.sc + i] : 1.0;
    for (int e = threadIdx.x; e < NRHS * nu; e += blockDim.x) {
        const int k = e / nu, c = e - k * nu;
        gs[k * I.ldu + c] = as[k * ldM + nx + c] + si * y_ptr(a, I, k, i)[nx + c] +
                            (a.affine ? a.sig[I.sig + (long long)i * nu + c] : 0.0);
    }
    __syncthreads();
    double kacc[NRHS][CH][2], qacc[NRHS][CH][2];
    zero(kacc);
    zero(qacc);
    {
        const int R = 2 * nu;
        const int r0 = R * w / NW, r1 = R * (w + 1) / NW;
        if (r0 < nu)
            gemv_rows<NRHS, CH>(a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, r0, r1 < nu ? r1 : nu, nu, gs,
                                I.ldu, kacc, lane);
        if (r1 > nu)
            gemv_rows<NRHS, CH>(a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, (r0 > nu ? r0 : nu) - nu,
                                r1 - nu, nx, gs, I.ldu, qacc, lane);
    }
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nu, kacc, lane);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, nu, nx, qacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
        const int k = e / W, c = e - k * W;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        if (c < nu) {
            kbuf_ptr(a, I, k, i)[c] = s;
        } else {
            const int cx = c - nu;
            qhat_ptr(a, I, k, i)[cx] = as[k * ldM + cx] + si * y_ptr(a, I, k, i)[cx] +
                                       (a.affine ? a.chat[I.chat + (long long)i * nx + cx] : 0.0) + s;
        }
    }
}

template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) fwd_trunk_kernel(SweepArgs a)
{
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i = it.idx;
    const int nx = I.nx, nu = I.nu, W = nx + nu, ldM = I.ldM;
    const int *cp = a.cp + I.cp;
    extern __shared__ double lds[];
    double *xs = lds;                 // [NRHS][ldM]: x_i then u_i
    double *red = xs + NRHS * ldM;    // [NW][NRHS][ldM]
    for (int e = threadIdx.x; e < NRHS * nx; e += blockDim.x) {
        const int k = e / nx, c = e - k * nx;
        double v;
        if (i == 0) {
            v = a.affine ? a.x0[k * a.x0_rs + I.x0 + c] : 0.0;
            x_ptr(a, I, k, 0)[c] = v;
        } else {
            v = x_ptr(a, I, k, i)[c];
        }
        xs[k * ldM + c] = v;
    }
    __syncthreads();
    double uacc[NRHS][CH][2];
    zero(uacc);
    {
        const int r0 = nx * w / NW, r1 = nx * (w + 1) / NW;
        if (r0 < r1)
            gemv_rows<NRHS, CH>(a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, r0, r1, nu, xs, ldM, uacc, lane);
    }
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nu, uacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * nu; e += blockDim.x) {
        const int k = e / nu, c = e - k * nu;
        double s = kbuf_ptr(a, I, k, i)[c];
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        u_ptr(a, I, k, i)[c] = s;
        xs[k * ldM + nx + c] = s;
    }
    __syncthreads();
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    const int RB = nch >= NW ? 1 : NW / nch;
    if (RB == 1) {
        for (int c = w; c < nch; c += NW) {
            const int j = j0 + c;
            double xacc[NRHS][CH][2];
            zero(xacc);
            gemv_rows<NRHS, CH>(a.Mf + I.Mf + (long long)j * W * I.ldx, I.ldx, 0, W, nx, xs, ldM, xacc, lane);
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                const int c0 = 2 * lane + 128 * ch;
#pragma unroll
                for (int e2 = 0; e2 < 2; ++e2) {
                    const int col = c0 + e2;
                    if (col < nx)
#pragma unroll
                        for (int k = 0; k < NRHS; ++k)
                            x_ptr(a, I, k, j)[col] =
                                xacc[k][ch][e2] + (a.affine ? a.cvec[I.c + (long long)j * nx + col] : 0.0);
                }
            }
        }
    } else {
        double xacc[NRHS][CH][2];
        zero(xacc);
        if (w < nch * RB) {
            const int c = w / RB, blk = w - c * RB;
            const int rr0 = W * blk / RB, rr1 = W * (blk + 1) / RB;
            gemv_rows<NRHS, CH>(a.Mf + I.Mf + (long long)(j0 + c) * W * I.ldx, I.ldx, rr0, rr1, nx, xs, ldM,
                                xacc, lane);
        }
        store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nx, xacc, lane);
        __syncthreads();
        for (int e = threadIdx.x; e < nch * NRHS * nx; e += blockDim.x) {
            const int c = e / (NRHS * nx), rem = e - c * NRHS * nx, k = rem / nx, col = rem - k * nx;
            const int j = j0 + c;
            double s = a.affine ? a.cvec[I.c + (long long)j * nx + col] : 0.0;
            for (int blk = 0; blk < RB; ++blk) s += red[((c * RB + blk) * NRHS + k) * ldM + col];
            x_ptr(a, I, k, j)[col] = s;
        }
    }
}

// ---- stages s*..N-1: chain c of an instance covers the nodes
// stage_ptr[t] + c for t = s*..N-1 (one child each) and its leaf ----
template <int NRHS, int CH>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) bwd_chain_kernel(SweepArgs a, int ldq)
{
    const int lane = threadIdx.x & (kWave - 1), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = blockIdx.x * kWavesPerBlock + wave;
    if (item >= a.nitems) return;
    const Item it = a.items[item];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int *sp = a.sp + I.sp;
    const WaveLds L = wave_lds(ldq, NRHS, wave);
    for (int t = I.N - 1; t >= I.sstar; --t)
        bwd_node<NRHS, CH>(a, I, sp[t] + it.idx, L, t != I.N - 1, t == I.sstar && t > 0, lane);
}

template <int NRHS, int CH>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) fwd_chain_kernel(SweepArgs a, int ldq)
{
    const int lane = threadIdx.x & (kWave - 1), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = blockIdx.x * kWavesPerBlock + wave;
    if (item >= a.nitems) return;
    const Item it = a.items[item];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int *sp = a.sp + I.sp;
    const WaveLds L = wave_lds(ldq, NRHS, wave);
    load_x<NRHS>(a, I, sp[I.sstar] + it.idx, L, lane);
    for (int t = I.sstar; t < I.N; ++t) fwd_node<NRHS, CH>(a, I, sp[t] + it.idx, L, t + 1 < I.N, lane);
}

}  // namespace

SweepArgs sweep_args(const tree_factors *f, int affine)
{
    SweepArgs a{};
    a.inst = f->d_inst;
    a.sp = f->d_sp; a.cp = f->d_cp;
    a.Mb = f->Mb; a.Mf = f->Mf; a.Kb = f->Kb; a.Kf = f->Kf; a.Rn = f->Rn;
    a.chat = f->chat; a.sig = f->sig; a.cvec = f->cvec; a.sc = f->precondition ? f->sc : nullptr;
    a.qhat = f->qhat; a.kbuf = f->kbuf;
    a.qhat_rs = f->x_tot;
    a.kbuf_rs = f->u_tot;
    a.affine = affine;
    return a;
}

int ensure_sweep_ws(tree_factors *f, int nrhs)
{
    if (f->ws_nrhs >= nrhs) return STOTREE_OK;
    if (f->qhat) { (void)hipFree(f->qhat); f->bytes -= (size_t)f->ws_nrhs * f->x_tot * 8; }
    if (f->kbuf) { (void)hipFree(f->kbuf); f->bytes -= (size_t)f->ws_nrhs * f->u_tot * 8; }
    f->qhat = f->kbuf = nullptr;
    f->ws_nrhs = 0;
    STOTREE_HIP(hipMalloc(&f->qhat, sizeof(double) * (size_t)nrhs * f->x_tot));
    STOTREE_HIP(hipMalloc(&f->kbuf, sizeof(double) * (size_t)nrhs * f->u_tot));
    f->ws_nrhs = nrhs;
    f->bytes += (size_t)nrhs * ((size_t)f->x_tot + (size_t)f->u_tot) * 8;
    return STOTREE_OK;
}
// ---- optional phase timing (HIP events around each phase) ----
namespace {
struct TimingState {
    bool on = false;
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
};
TimingState g_timing;

struct PhaseTimer {
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(int ph, hipStream_t s) : phase(ph), st(s)
    {
        if (!g_timing.on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, st);
    }
    ~PhaseTimer()
    {
        if (!a) return;
        (void)hipEventRecord(b, st);
        g_timing.recs.push_back({phase, a, b});
    }
};
}  // namespace

int timing_enable(int on)
{
    g_timing.on = on != 0;
    return STOTREE_OK;
}

int timing_read(double *ms, long long *count)
{
    for (int p = 0; p < 4; ++p) { ms[p] = 0.0; count[p] = 0; }
    int rc = STOTREE_OK;
    for (auto &r : g_timing.recs) {
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            rc = STOTREE_ERR_DEVICE;
        ms[r.phase] += t;
        count[r.phase] += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_timing.recs.clear();
    if (rc) set_error("stotree_timing_read: event query failed");
    return rc;
}

template <int NRHS, int CH, int NW>
static void launch_trunk_nw(bool backward, SweepArgs a, const LevelPlan &lv, int max_ldM, int max_qs,
                            int max_ldu, hipStream_t st)
{
    a.items = lv.items;
    a.nitems = lv.count;
    a.t = lv.t;
    if (backward) {
        // max_qs: largest child_batch(NRHS, ldx) * ldx over the instances
        const size_t lds = sizeof(double) * ((size_t)max_qs * NRHS + (size_t)(NW + 1) * NRHS * max_ldM +
                                             (size_t)NRHS * max_ldu);
        hipLaunchKernelGGL((bwd_trunk_kernel<NRHS, CH, NW>), dim3(lv.count), dim3(kWave * NW), lds, st, a);
    } else {
        const size_t lds = sizeof(double) * (size_t)(NW + 1) * NRHS * max_ldM;
        hipLaunchKernelGGL((fwd_trunk_kernel<NRHS, CH, NW>), dim3(lv.count), dim3(kWave * NW), lds, st, a);
    }
}

template <int NRHS, int CH>
static void launch_trunk(bool backward, const SweepArgs &a, const LevelPlan &lv, int max_ldM, int max_qs,
                         int max_ldu, hipStream_t st)
{
    switch (lv.nw) {
    case 16: launch_trunk_nw<NRHS, CH, 16>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 8: launch_trunk_nw<NRHS, CH, 8>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 4: launch_trunk_nw<NRHS, CH, 4>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 2: launch_trunk_nw<NRHS, CH, 2>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    default: launch_trunk_nw<NRHS, CH, 1>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    }
}

template <int NRHS, int CH>
static hipError_t sweep_impl(const tree_factors *f, SweepArgs a, hipStream_t st)
{
    int ldM = 2, qs = 2, ldu = 2;
    for (const InstDesc &I : f->inst) {
        ldM = std::max(ldM, I.ldM);
        qs = std::max(qs, child_batch(NRHS, I.ldx) * I.ldx);
        ldu = std::max(ldu, I.ldu);
    }
    const dim3 blk(kWave * kWavesPerBlock);
    const size_t chain_lds = sizeof(double) * kWavesPerBlock * 3 * NRHS * ldM;
    const dim3 cgrid((f->nchain_items + kWavesPerBlock - 1) / kWavesPerBlock);
    SweepArgs ca = a;
    ca.items = f->chain_items;
    ca.nitems = f->nchain_items;
    if (f->nchain_items > 0) {
        PhaseTimer tm(0, st);
        hipLaunchKernelGGL((bwd_chain_kernel<NRHS, CH>), cgrid, blk, chain_lds, st, ca, ldM);
    }
    if (!f->levels.empty()) {
        PhaseTimer tm(1, st);
        for (int k = (int)f->levels.size() - 1; k >= 0; --k)
            launch_trunk<NRHS, CH>(true, a, f->levels[k], ldM, qs, ldu, st);
    }
    if (!f->levels.empty()) {
        PhaseTimer tm(2, st);
        for (size_t k = 0; k < f->levels.size(); ++k)
            launch_trunk<NRHS, CH>(false, a, f->levels[k], ldM, qs, ldu, st);
    }
    if (f->nchain_items > 0) {
        PhaseTimer tm(3, st);
        hipLaunchKernelGGL((fwd_chain_kernel<NRHS, CH>), cgrid, blk, chain_lds, st, ca, ldM);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_tree(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st)
{
    const bool wide = f->max_width > 128;
    if (nrhs == 1) return wide ? sweep_impl<1, 2>(f, a, st) : sweep_impl<1, 1>(f, a, st);
    if (nrhs == 2) return wide ? sweep_impl<2, 2>(f, a, st) : sweep_impl<2, 1>(f, a, st);
    return hipErrorInvalidValue;
}

}  // namespace stotree
