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
// Mapping.  One wavefront per node above s*; below it a group of G lanes
// (G = 64, 32, 16 or 8, by default the smallest with 2G >= nx+nu) per chain.
// Each lane owns two adjacent output entries; matrices are stored in the
// orientation of the pass that reads them, so every row of a matrix is one
// contiguous, 16-byte-aligned load across the lane group, multiplied by a
// broadcast entry of the input vector held in LDS.  The nodes from stage s*
// on have one child each (the scenario fan-out has ended); the tree below s*
// is a set of independent chains, each walked by one lane group through all
// its stages with qhat / x carried in LDS, so those stages need no grid-wide
// synchronisation.  Stages above s* are launched stage by stage.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "sweep_common.h"

namespace stotree {

namespace {

using namespace dev;


// acc[k][ch][e] += sum_{r0<=r<r1} M[r][c] * v_k[r] for the lane's columns
// c = 2*lane + 2*G*ch + e < W (lane within a group of G lanes that shares
// the matrix), with M row-major of leading dimension ld and v_k in LDS at
// v + k*ldv.  The loads carry no lane condition (lanes past W re-read column
// 0 and their sums are never stored) and rows go in batches of kRowBatch,
// double-buffered: the next batch is issued before the current one is
// multiplied, so up to 2*kRowBatch row loads are in flight per lane group.  A
// last, partial batch re-reads its final row in the unused slots (and skips
// them in the sums), so no row is ever loaded on its own.
constexpr int kRowBatch = 8;
// the backward chain steps of 64-lane groups measured fastest with batches of 6 rows
constexpr int kChainRowBatch = 6;

template <int CH, int RB = kRowBatch>
__device__ __forceinline__ void load_rows(double2 (&m)[RB][CH], const double *__restrict__ M,
                                          int ld, int r, int cnt, const int (&col)[CH])
{
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        const int rr = r + (u < cnt ? u : cnt - 1);
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
            m[u][ch] = *reinterpret_cast<const double2 *>(M + (long long)rr * ld + col[ch]);
    }
}

template <int NRHS, int CH, int RB = kRowBatch>
__device__ __forceinline__ void fma_rows(const double2 (&m)[RB][CH], const double *v, int ldv,
                                         int r, int cnt, double (&acc)[NRHS][CH][2])
{
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        if (u >= cnt) break;
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
}

template <int NRHS, int CH, int G = kWave, int RB = kRowBatch>
__device__ __forceinline__ void gemv_rows(const double *__restrict__ M, int ld, int r0, int r1, int W,
                                          const double *v, int ldv, double (&acc)[NRHS][CH][2],
                                          int lane)
{
    const int n = r1 - r0;
    if (n <= 0) return;
    int col[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * G * ch;
        col[ch] = c0 < W ? c0 : 0;
    }
    const int nbt = (n + RB - 1) / RB;   // batches, the last one possibly partial
    auto cnt = [&](int b) { return n - b * RB < RB ? n - b * RB : RB; };
    double2 m0[RB][CH], m1[RB][CH];
    load_rows<CH, RB>(m0, M, ld, r0, cnt(0), col);
    int b = 0;
    for (; b + 2 <= nbt; b += 2) {
        load_rows<CH, RB>(m1, M, ld, r0 + (b + 1) * RB, cnt(b + 1), col);
        fma_rows<NRHS, CH, RB>(m0, v, ldv, r0 + b * RB, RB, acc);
        if (b + 2 < nbt) load_rows<CH, RB>(m0, M, ld, r0 + (b + 2) * RB, cnt(b + 2), col);
        fma_rows<NRHS, CH, RB>(m1, v, ldv, r0 + (b + 1) * RB, cnt(b + 1), acc);
    }
    if (b < nbt) fma_rows<NRHS, CH, RB>(m0, v, ldv, r0 + b * RB, cnt(b), acc);
}

// The product of gemv_rows split in two so that its loads can be issued
// before the vector exists: stream_open<D> loads the range's first D (1 or
// 2) batches of rows (the rows only depend on the node), stream_run
// multiplies them once v is in LDS and streams the rest double-buffered.
// Used where a node's latency, not its bandwidth, bounds the step: the
// stages above s*.  An open stream holds D*kRowBatch*CH double2 registers.
template <int CH>
struct RowStream {
    const double *M;
    int ld, r0, n;
    int col[CH];
    double2 m0[kRowBatch][CH], m1[kRowBatch][CH];
};

template <int CH>
__device__ __forceinline__ int stream_cnt(const RowStream<CH> &s, int b)
{
    return s.n - b * kRowBatch < kRowBatch ? s.n - b * kRowBatch : kRowBatch;
}

template <int D, int CH>
__device__ __forceinline__ void stream_open(RowStream<CH> &s, const double *__restrict__ M, int ld, int r0, int r1,
                                            int W, int lane)
{
    s.M = M;
    s.ld = ld;
    s.r0 = r0;
    s.n = r1 > r0 ? r1 - r0 : 0;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * kWave * ch;
        s.col[ch] = c0 < W ? c0 : 0;
    }
    if (s.n > 0) load_rows<CH>(s.m0, M, ld, r0, stream_cnt(s, 0), s.col);
    if (D == 2 && s.n > kRowBatch) load_rows<CH>(s.m1, M, ld, r0 + kRowBatch, stream_cnt(s, 1), s.col);
}

template <int D, int NRHS, int CH>
__device__ __forceinline__ void stream_run(RowStream<CH> &s, const double *v, int ldv, double (&acc)[NRHS][CH][2])
{
    const int nbt = (s.n + kRowBatch - 1) / kRowBatch;
    if (D == 1 && nbt > 1) load_rows<CH>(s.m1, s.M, s.ld, s.r0 + kRowBatch, stream_cnt(s, 1), s.col);
    for (int b = 0; b < nbt; b += 2) {
        fma_rows<NRHS, CH>(s.m0, v, ldv, s.r0 + b * kRowBatch, stream_cnt(s, b), acc);
        if (b + 2 < nbt) load_rows<CH>(s.m0, s.M, s.ld, s.r0 + (b + 2) * kRowBatch, stream_cnt(s, b + 2), s.col);
        if (b + 1 < nbt) {
            fma_rows<NRHS, CH>(s.m1, v, ldv, s.r0 + (b + 1) * kRowBatch, stream_cnt(s, b + 1), acc);
            if (b + 3 < nbt)
                load_rows<CH>(s.m1, s.M, s.ld, s.r0 + (b + 3) * kRowBatch, stream_cnt(s, b + 3), s.col);
        }
    }
}

// The same product for W <= G columns on a lane group of G lanes: each load
// instruction brings in two rows per group, the even rows of the range in the
// lower half of the group and the odd rows in the upper half (lane l of a
// half owns columns 2l, 2l+1); the halves' partial sums are added at the end,
// so the lower half holds the sums and the upper half (whose own columns are
// >= G) a copy.
template <int RB = kRowBatch>
__device__ __forceinline__ void load_pairs(double2 (&m)[RB], const double *__restrict__ M, int ld,
                                           int rfirst, int rlast, int col)
{
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        const int r = rfirst + 2 * u;
        m[u] = *reinterpret_cast<const double2 *>(M + (long long)(r < rlast ? r : rlast) * ld + col);
    }
}

template <int NRHS, int RB = kRowBatch>
__device__ __forceinline__ void fma_pairs(const double2 (&m)[RB], const double *v, int ldv, int rfirst,
                                          int r1, double (&acc)[NRHS][1][2])
{
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        const int r = rfirst + 2 * u;
        const bool in = r < r1;
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double vk = in ? v[k * ldv + r] : 0.0;
            acc[k][0][0] = fma(m[u].x, vk, acc[k][0][0]);
            acc[k][0][1] = fma(m[u].y, vk, acc[k][0][1]);
        }
    }
}

template <int NRHS, int G = kWave, int RB = kRowBatch>
__device__ __forceinline__ void gemv_pairs(const double *__restrict__ M, int ld, int r0, int r1, int W,
                                           const double *v, int ldv, double (&acc)[NRHS][1][2], int lane)
{
    const int h = lane >= G / 2 ? 1 : 0, l = lane & (G / 2 - 1);
    const int col = 2 * l < W ? 2 * l : 0;
    const int np = (r1 - r0 + 1) / 2;
    const int nbt = (np + RB - 1) / RB;
    const int rlast = r1 - 1;
    double part[NRHS][1][2];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) part[k][0][0] = part[k][0][1] = 0.0;
    double2 m0[RB], m1[RB];
    load_pairs<RB>(m0, M, ld, r0 + h, rlast, col);
    int b = 0;
    for (; b + 2 <= nbt; b += 2) {
        load_pairs<RB>(m1, M, ld, r0 + 2 * (b + 1) * RB + h, rlast, col);
        fma_pairs<NRHS, RB>(m0, v, ldv, r0 + 2 * b * RB + h, r1, part);
        if (b + 2 < nbt) load_pairs<RB>(m0, M, ld, r0 + 2 * (b + 2) * RB + h, rlast, col);
        fma_pairs<NRHS, RB>(m1, v, ldv, r0 + 2 * (b + 1) * RB + h, r1, part);
    }
    if (b < nbt) fma_pairs<NRHS, RB>(m0, v, ldv, r0 + 2 * b * RB + h, r1, part);
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double o = __shfl_xor(part[k][0][e], G / 2, kWave);
            acc[k][0][e] += h ? o + part[k][0][e] : part[k][0][e] + o;
        }
}

// dst[k*ld + off + c] = acc[k][.][.] for the lane's columns c < dim.
template <int NRHS, int CH, int G = kWave>
__device__ __forceinline__ void store_acc(double *dst, int ld, int off, int dim,
                                          const double (&acc)[NRHS][CH][2], int lane)
{
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * G * ch;
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

// LDS of one lane group in the chain kernels: qx [NRHS][ldq] (qhat or
// [x;u]), as [NRHS][ldq], gs [NRHS][ldq], with ldq the largest padded width.
struct WaveLds {
    double *qx, *as, *gs;
    int ldq;
};

__device__ __forceinline__ WaveLds wave_lds(int ldq, int nrhs, int slot)
{
    extern __shared__ double lds[];
    WaveLds w;
    w.qx = lds + slot * 3 * nrhs * ldq;
    w.as = w.qx + nrhs * ldq;
    w.gs = w.as + nrhs * ldq;
    w.ldq = ldq;
    return w;
}

// The raw values behind the lane's entries of node i's own terms
// s_i y_i + [chat_i ; sigma_i] (columns 2*lane + 2*G*ch + e, clamped to the
// row), requested at the start of the node's backward step and combined only
// where they are added to its children's product, once that is done: no
// load of them waits before the product.  (A select or a branch on a loaded
// value, or seeding the accumulator with it, made the compiler wait for the
// loads right away.)  chat and sigma are allocated for every handle, so the
// loads carry no condition; without disturbances their values are not used.
template <int NRHS, int CH>
struct NodeTerms {
    double si;
    double y[NRHS][CH][2];
    double h[CH][2];
};

template <int NRHS, int CH, int G>
__device__ __forceinline__ void node_terms(const SweepArgs &a, const InstDesc &I, int i, int lane,
                                           NodeTerms<NRHS, CH> &t)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    t.si = a.sc ? a.sc[I.sc + i] : 1.0;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = 2 * lane + 2 * G * ch + e, cw = c < W ? c : W - 1;
            const double *h = cw < nx ? a.chat + I.chat + (long long)i * nx + cw
                                      : a.sig + I.sig + (long long)i * nu + (cw - nx);
            t.h[ch][e] = *h;
#pragma unroll
            for (int k = 0; k < NRHS; ++k) t.y[k][ch][e] = y_ptr(a, I, k, i)[cw];
        }
}

// acc += s_i y_i + [chat_i ; sigma_i] (the last term only with disturbances)
template <int NRHS, int CH>
__device__ __forceinline__ void add_node_terms(const SweepArgs &a, double (&acc)[NRHS][CH][2],
                                               const NodeTerms<NRHS, CH> &t)
{
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e)
                acc[k][ch][e] += t.si * t.y[k][ch][e] + (a.affine ? t.h[ch][e] : 0.0);
}

template <int NRHS, int CH>
__device__ __forceinline__ void add_to(double (&acc)[NRHS][CH][2], const double (&v)[NRHS][CH][2])
{
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            acc[k][ch][0] += v[k][ch][0];
            acc[k][ch][1] += v[k][ch][1];
        }
}

// Backward step of non-leaf node i of instance I by one wavefront.  If
// child_in_lds, qhat of the (single) child is already in L.qx; otherwise each
// child's qhat is staged from the leaf data or from the global qhat buffer.
// For a chain node (kChain) jc is the index of its only child; otherwise the
// children are read from the child pointers.  The result qhat_i is left in
// L.qx and, if store_q, written to the global buffer; k_i always goes to kbuf.
template <int NRHS, int CH, int G, bool kChain = false, int RB = kRowBatch>
__device__ void bwd_node(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L,
                         bool child_in_lds, bool store_q, int lane, int jc = -1)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const int *cp = a.cp + I.cp;
    // Narrow lane groups request the node's own terms up front (their
    // chains gain from it); 64-lane groups load them after the product, as
    // a coalesced pass per vector, which measured faster for them.
    constexpr bool kEarly = G < kWave;
    NodeTerms<NRHS, CH> nt;
    if constexpr (kEarly) node_terms<NRHS, CH, G>(a, I, i, lane, nt);
    double acc[NRHS][CH][2];
    zero(acc);
    const int j0 = kChain ? jc : cp[i], j1 = kChain ? jc + 1 : cp[i + 1];
    for (int j = j0; j < j1; ++j) {
        if (!child_in_lds) {
            if (j >= I.Vnl) {
                const double sj = a.sc ? a.sc[I.sc + j] : 1.0;
                for (int r = lane; r < nx; r += G)
#pragma unroll
                    for (int k = 0; k < NRHS; ++k)
                        L.qx[k * L.ldq + r] = sj * y_ptr(a, I, k, j)[r] +
                                              (a.affine ? a.chat[I.chat + (long long)j * nx + r] : 0.0);
            } else {
                for (int r = lane; r < nx; r += G)
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) L.qx[k * L.ldq + r] = qhat_ptr(a, I, k, j)[r];
            }
            wave_sync();
        }
        gemv_rows<NRHS, CH, G, RB>(a.Mb + I.Mb + (long long)j * nx * I.ldM, I.ldM, 0, nx, W, L.qx, L.ldq, acc, lane);
        wave_sync();
    }
    // early: L.as = [sum A'q + s_i y_i^x + chat_i ; g_i], g_i = sum B'q + s_i y_i^u + sigma_i;
    // otherwise L.as = [sum A'q ; sum B'q] and g_i is formed in L.gs
    if constexpr (kEarly) add_node_terms(a, acc, nt);
    store_acc<NRHS, CH, G>(L.as, L.ldq, 0, W, acc, lane);
    wave_sync();
    const double *gs = L.as + nx;
    const double si = kEarly ? 0.0 : (a.sc ? a.sc[I.sc + i] : 1.0);
    if constexpr (!kEarly) {
        for (int c = lane; c < nu; c += G)
#pragma unroll
            for (int k = 0; k < NRHS; ++k)
                L.gs[k * L.ldq + c] = L.as[k * L.ldq + nx + c] + si * y_ptr(a, I, k, i)[nx + c] +
                                      (a.affine ? a.sig[I.sig + (long long)i * nu + c] : 0.0);
        wave_sync();
        gs = L.gs;
    }
    double kacc[NRHS][CH][2], qacc[NRHS][CH][2];
    zero(kacc);
    zero(qacc);
    if constexpr (CH == 1) {
        if (nx <= G && nu >= 2) {
            gemv_pairs<NRHS, G, RB>(a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, 0, nu, nu, gs, L.ldq, kacc, lane);
            gemv_pairs<NRHS, G, RB>(a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, 0, nu, nx, gs, L.ldq, qacc, lane);
        } else {
            gemv_rows<NRHS, CH, G, RB>(a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, 0, nu, nu, gs, L.ldq, kacc, lane);
            gemv_rows<NRHS, CH, G, RB>(a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, 0, nu, nx, gs, L.ldq, qacc, lane);
        }
    } else {
        gemv_rows<NRHS, CH, G, RB>(a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, 0, nu, nu, gs, L.ldq, kacc, lane);
        gemv_rows<NRHS, CH, G, RB>(a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, 0, nu, nx, gs, L.ldq, qacc, lane);
    }
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * G * ch;
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
        const int c0 = 2 * lane + 2 * G * ch;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                double v = 0.0;
                if constexpr (kEarly) {
                    if (c < nx) v = L.as[k * L.ldq + c] + qacc[k][ch][e];
                } else {
                    if (c < nx)
                        v = L.as[k * L.ldq + c] + si * y_ptr(a, I, k, i)[c] +
                            (a.affine ? a.chat[I.chat + (long long)i * nx + c] : 0.0) + qacc[k][ch][e];
                }
                qv[k][ch][e] = v;
            }
        }
    }
    wave_sync();  // every lane has finished reading L.qx / L.as
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * G * ch;
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
// left in L.qx.  For a chain node (kChain) jc is the index of its only
// child; otherwise the children are read from the child pointers.  k_i and
// each c_j are requested before the product they are added to.
template <int NRHS, int CH, int G, bool kChain = false>
__device__ void fwd_node(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L, bool keep_child,
                         int lane, int jc = -1)
{
    const int nx = I.nx, nu = I.nu;
    const int *cp = a.cp + I.cp;
    double kv[NRHS][CH][2], uacc[NRHS][CH][2];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = 2 * lane + 2 * G * ch + e;
#pragma unroll
            for (int k = 0; k < NRHS; ++k) kv[k][ch][e] = kbuf_ptr(a, I, k, i)[c < nu ? c : nu - 1];
        }
    zero(uacc);
    const int j0 = kChain ? jc : cp[i], j1 = kChain ? jc + 1 : cp[i + 1];
    if constexpr (CH == 1) {
        if (nu <= G && nx >= 2)
            gemv_pairs<NRHS, G>(a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, 0, nx, nu, L.qx, L.ldq, uacc, lane);
        else
            gemv_rows<NRHS, CH, G>(a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, 0, nx, nu, L.qx, L.ldq, uacc, lane);
    } else {
        gemv_rows<NRHS, CH, G>(a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, 0, nx, nu, L.qx, L.ldq, uacc, lane);
    }
    // both of a lane's entries are formed before either is stored (the empty
    // asm keeps the compiler from sinking each sum into its store's branch,
    // where the second reused the first store's registers and waited on it)
    add_to(uacc, kv);
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) asm volatile("" : "+v"(uacc[k][ch][0]), "+v"(uacc[k][ch][1]));
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c0 = 2 * lane + 2 * G * ch;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
            if (c < nu) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) {
                    u_ptr(a, I, k, i)[c] = uacc[k][ch][e];
                    L.qx[k * L.ldq + nx + c] = uacc[k][ch][e];
                }
            }
        }
    }
    wave_sync();
    double keep[NRHS][CH][2];
    zero(keep);
    for (int j = j0; j < j1; ++j) {
        double xacc[NRHS][CH][2], cv[CH][2];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = 2 * lane + 2 * G * ch + e;
                cv[ch][e] = a.cvec[I.c + (long long)j * nx + (c < nx ? c : nx - 1)];   // allocated always
            }
        zero(xacc);
        if constexpr (CH == 1) {
            if (nx <= G)
                gemv_pairs<NRHS, G>(a.Mf + I.Mf + (long long)j * (nx + nu) * I.ldx, I.ldx, 0, nx + nu, nx, L.qx,
                                    L.ldq, xacc, lane);
            else
                gemv_rows<NRHS, CH, G>(a.Mf + I.Mf + (long long)j * (nx + nu) * I.ldx, I.ldx, 0, nx + nu, nx, L.qx,
                                       L.ldq, xacc, lane);
        } else {
            gemv_rows<NRHS, CH, G>(a.Mf + I.Mf + (long long)j * (nx + nu) * I.ldx, I.ldx, 0, nx + nu, nx, L.qx, L.ldq,
                                   xacc, lane);
        }
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            const int c0 = 2 * lane + 2 * G * ch;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = c0 + e;
                if (c < nx) {
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) {
                        const double xv = xacc[k][ch][e] + (a.affine ? cv[ch][e] : 0.0);
                        x_ptr(a, I, k, j)[c] = xv;
                        keep[k][ch][e] = xv;
                    }
                }
            }
        }
    }
    if (keep_child) {
        wave_sync();
        store_acc<NRHS, CH, G>(L.qx, L.ldq, 0, nx, keep, lane);
        wave_sync();
    }
}

// x_i of the first node a forward pass visits: x0 at the root (written to
// the output too), else the value the previous stage stored.
template <int NRHS, int G>
__device__ void load_x(const SweepArgs &a, const InstDesc &I, int i, const WaveLds &L, int lane)
{
    for (int c = lane; c < I.nx; c += G)
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
__device__ void bwd_trunk_node(const SweepArgs &a, const InstDesc &I, int i, int w, int lane)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu, ldq = I.ldx, ldM = I.ldM;
    const int *cp = a.cp + I.cp;
    // batches of [A_j B_j] rows requested up front (two where the registers allow)
    constexpr int kDepth = CH == 1 && NW <= 8 ? 2 : 1;
    const int CB = child_batch(NRHS, ldq), ldv = CB * ldq;
    extern __shared__ double lds[];
    double *qs = lds;                          // [NRHS][ldv]: a batch's children's qhat, child after child
    double *red = qs + NRHS * ldv;             // [NW][NRHS][ldM]
    double *as = red + NW * NRHS * ldM;        // [NRHS][ldM]: [sum A'q ; g_i] plus the node's own terms
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    // Everything that depends on node i alone is requested before the
    // children's qhat: the wavefront's rows of -R~^{-1} and K_i (split over
    // the 2nu rows as below) and the node's own terms s_i y_i + [chat_i ;
    // sigma_i], which wavefront 0 adds to its partial sum.
    // (With two column chunks or 16 wavefronts the registers of all three
    // streams would not fit: those rows are then requested after the
    // children's product.)
    RowStream<CH> rk, rq;
    auto open_rk = [&]() {
        const int R = 2 * nu, r0 = R * w / NW, r1 = R * (w + 1) / NW;
        stream_open<1, CH>(rk, a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, r0, r1 < nu ? r1 : nu, nu, lane);
        stream_open<1, CH>(rq, a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, (r0 > nu ? r0 : nu) - nu, r1 - nu,
                           nx, lane);
    };
    if (CH == 1 && NW <= 8) open_rk();
    NodeTerms<NRHS, CH> nt;
    node_terms<NRHS, CH, kWave>(a, I, i, lane, nt);
    double acc[NRHS][CH][2];
    zero(acc);
    for (int cb = 0; cb < nch; cb += CB) {
        const int nb = nch - cb < CB ? nch - cb : CB;
        // the batch's rows of [A_j B_j] are contiguous (children are
        // consecutive nodes): one range of R rows split over the wavefronts
        const int R = nb * nx, r0 = (int)((long long)R * w / NW), r1 = (int)((long long)R * (w + 1) / NW);
        RowStream<CH> mb;
        stream_open<kDepth, CH>(mb, a.Mb + I.Mb + (long long)(j0 + cb) * nx * ldM, ldM, r0, r1, W, lane);
        for (int e = threadIdx.x; e < R; e += blockDim.x) {
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
                qs[k * ldv + e] = q;
            }
        }
        __syncthreads();
        stream_run<kDepth, NRHS, CH>(mb, qs, ldv, acc);
        if (cb + CB < nch) __syncthreads();   // qs is refilled
    }
    if (!(CH == 1 && NW <= 8)) open_rk();
    if (w == 0) add_node_terms(a, acc, nt);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, W, acc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
        const int k = e / W, c = e - k * W;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        as[k * ldM + c] = s;
    }
    __syncthreads();
    // g_i = as[nx:]: k_i = -R~^{-1} g_i and K_i' g_i
    double kacc[NRHS][CH][2], qacc[NRHS][CH][2];
    zero(kacc);
    zero(qacc);
    stream_run<1, NRHS, CH>(rk, as + nx, ldM, kacc);
    stream_run<1, NRHS, CH>(rq, as + nx, ldM, qacc);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nu, kacc, lane);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, nu, nx, qacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
        const int k = e / W, c = e - k * W;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        if (c < nu)
            kbuf_ptr(a, I, k, i)[c] = s;
        else
            qhat_ptr(a, I, k, i)[c - nu] = as[k * ldM + c - nu] + s;
    }
}

template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) bwd_trunk_kernel(SweepArgs a)
{
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    bwd_trunk_node<NRHS, CH, NW>(a, I, it.idx, w, lane);
}

// All stages above s* in one launch: a workgroup starts at a node of stage
// s*-1 and, after finishing a node, counts it in at its parent; the workgroup
// that brings the parent's count to its number of children goes on with the
// parent (every child's qhat is then in memory), the others stop.  No
// workgroup waits on another, the root is finished by exactly one, and each
// parent's counter is reset by the workgroup that takes the parent, so the
// counters are zero again when the launch ends.
template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) bwd_trunk_tree_kernel(SweepArgs a, int *counters)
{
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    __shared__ int go;
    int i = it.idx;
    for (;;) {
        bwd_trunk_node<NRHS, CH, NW>(a, I, i, w, lane);
        if (i == 0) break;
        const int p = a.anc[I.sc + i];
        // Every wavefront releases its own stores of node i's qhat and k
        // device-wide (the fence waits for them and writes them back past
        // this XCD's L2) before the barrier; a fence on one wavefront would
        // cover only that wavefront's stores.
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nch = a.cp[I.cp + p + 1] - a.cp[I.cp + p];
            const int last = atomicAdd(&counters[I.node0 + p], 1) == nch - 1;
            if (last) {
                counters[I.node0 + p] = 0;
                __threadfence();   // acquire the siblings' qhat
            }
            go = last;
        }
        __syncthreads();
        if (!go) break;
        i = p;
    }
}

// The lane's entries of c_j (allocated for every handle; used only with
// disturbances), added to the partial sum of the wavefront that owns x_j's
// first rows.
template <int CH>
__device__ __forceinline__ void load_cvec(const SweepArgs &a, const InstDesc &I, int j, int lane, double (&cv)[CH][2])
{
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = 2 * lane + 2 * kWave * ch + e;
            cv[ch][e] = a.cvec[I.c + (long long)j * I.nx + (c < I.nx ? c : I.nx - 1)];
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
    // batches of [A_j B_j]' rows requested up front (two where the registers allow)
    constexpr int kDepth = CH == 1 && NW <= 8 ? 2 : 1;
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    const int RB = nch >= NW ? 1 : NW / nch;
    // Requested before x_i: the wavefront's rows of K_i' and k_i (which
    // wavefront 0 adds to its partial sum), and its first rows of a child's
    // [A_j B_j]' with c_j; children go round-robin to the wavefronts, or,
    // with fewer children than wavefronts, each child's rows are split into
    // RB blocks.
    RowStream<CH> kf, mf;
    double kv[NRHS][CH][2], uacc[NRHS][CH][2];
    zero(uacc);
    {
        const int r0 = nx * w / NW, r1 = nx * (w + 1) / NW;
        stream_open<1, CH>(kf, a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, r0, r1, nu, lane);
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = 2 * lane + 2 * kWave * ch + e;
#pragma unroll
                for (int k = 0; k < NRHS; ++k) kv[k][ch][e] = kbuf_ptr(a, I, k, i)[c < nu ? c : nu - 1];
            }
    }
    int c = RB == 1 ? w : w / RB;
    const int blk = RB == 1 ? 0 : w - c * RB;
    double cv[CH][2];
    if (c < nch) {
        const int rr0 = W * blk / RB, rr1 = W * (blk + 1) / RB;
        stream_open<kDepth, CH>(mf, a.Mf + I.Mf + (long long)(j0 + c) * W * I.ldx, I.ldx, rr0, rr1, nx, lane);
        load_cvec<CH>(a, I, j0 + c, lane, cv);
    }
    for (int e = threadIdx.x; e < NRHS * nx; e += blockDim.x) {
        const int k = e / nx, cc = e - k * nx;
        double v;
        if (i == 0) {
            v = a.affine ? a.x0[k * a.x0_rs + I.x0 + cc] : 0.0;
            x_ptr(a, I, k, 0)[cc] = v;
        } else {
            v = x_ptr(a, I, k, i)[cc];
        }
        xs[k * ldM + cc] = v;
    }
    __syncthreads();
    stream_run<1, NRHS, CH>(kf, xs, ldM, uacc);
    if (w == 0) add_to(uacc, kv);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nu, uacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * nu; e += blockDim.x) {
        const int k = e / nu, cc = e - k * nu;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + cc];
        u_ptr(a, I, k, i)[cc] = s;
        xs[k * ldM + nx + cc] = s;
    }
    __syncthreads();
    if (RB == 1) {
        for (; c < nch; c += NW) {
            double xacc[NRHS][CH][2];
            zero(xacc);
            stream_run<kDepth, NRHS, CH>(mf, xs, ldM, xacc);
#pragma unroll
            for (int k = 0; k < NRHS; ++k)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch) {
                    xacc[k][ch][0] += a.affine ? cv[ch][0] : 0.0;
                    xacc[k][ch][1] += a.affine ? cv[ch][1] : 0.0;
                }
            const int j = j0 + c;
            if (c + NW < nch) {   // the next child's rows are in flight while x_j is stored
                stream_open<kDepth, CH>(mf, a.Mf + I.Mf + (long long)(j + NW) * W * I.ldx, I.ldx, 0, W, nx, lane);
                load_cvec<CH>(a, I, j + NW, lane, cv);
            }
#pragma unroll
            for (int ch = 0; ch < CH; ++ch)
#pragma unroll
                for (int e2 = 0; e2 < 2; ++e2) {
                    const int col = 2 * lane + 2 * kWave * ch + e2;
                    if (col < nx)
#pragma unroll
                        for (int k = 0; k < NRHS; ++k) x_ptr(a, I, k, j)[col] = xacc[k][ch][e2];
                }
        }
    } else {
        double xacc[NRHS][CH][2];
        zero(xacc);
        if (c < nch) {
            stream_run<kDepth, NRHS, CH>(mf, xs, ldM, xacc);
            if (blk == 0)
#pragma unroll
                for (int k = 0; k < NRHS; ++k)
#pragma unroll
                    for (int ch = 0; ch < CH; ++ch) {
                        xacc[k][ch][0] += a.affine ? cv[ch][0] : 0.0;
                        xacc[k][ch][1] += a.affine ? cv[ch][1] : 0.0;
                    }
        }
        store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nx, xacc, lane);
        __syncthreads();
        for (int e = threadIdx.x; e < nch * NRHS * nx; e += blockDim.x) {
            const int cc = e / (NRHS * nx), rem = e - cc * NRHS * nx, k = rem / nx, col = rem - k * nx;
            double s = 0.0;
            for (int b = 0; b < RB; ++b) s += red[((cc * RB + b) * NRHS + k) * ldM + col];
            x_ptr(a, I, k, j0 + cc)[col] = s;
        }
    }
}

// ---- the first stages above s* in one launch per direction ----
//
// The nodes of an instance's first stages (each with at most a set number of
// nodes) form one work list per direction: deepest stage first backward, root
// first forward, so a workgroup is dispatched only after every workgroup it
// waits for (workgroups of a launch are dispatched in order; a waiting one
// never holds back one it waits for).  A workgroup requests every row its
// node needs first, then waits for its inputs: backward until each child has
// counted itself in at the node's counter, forward until the parent has
// raised the node's flag; it then clears that counter or flag, so all are
// zero again when the launch ends.  The per-edge products are formed on the
// child's side of each hand-off (backward, the child sends [A_j B_j]' qhat_j;
// forward, the child forms its own x_j from its parent's x and u), so after a
// wait a node reads one short vector per child and multiplies rows it already
// holds.  Hand-offs are device-wide (the producing XCD's L2 is written back):
// every thread completes its own stores before the barrier that precedes the
// count, and thread 0 then releases them all device-wide with the count; on
// the waiting side thread 0 acquires device-wide (the CU's caches are
// invalidated) before the barrier that lets the workgroup read.  One
// device-scope fence per node and side: a fence on every thread cost more
// than the launches it replaced.  A wait gives up after kSpinLimit polls
// (about a second; a correct launch waits microseconds) and records the
// failure in the error word; from then on the fused launches of the handle
// write NaN to their outputs and wait no more, until the schedule is rebuilt
// (which clears the word and the counters).
constexpr int kSpinLimit = 1 << 20;

struct FusedWait {
    int *c;        // counter or flag to wait for (null: inputs come from earlier launches)
    int target;    // value it must reach
    int *err;      // the handle's error word
    int bad;       // the error word as read when the workgroup started
    int *poison;   // LDS: this workgroup writes NaN (thread 0's decision; the node's
                   // later barriers publish it)
    __device__ void operator()() const
    {
        if (!c) {
            if (threadIdx.x == 0) *poison = bad;
            return;
        }
        if (threadIdx.x == 0) {
            int b = bad;
            if (!b) {
                int spins = 0;
                while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins >= kSpinLimit) {
                        b = 1;
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
                __hip_atomic_store(c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            *poison = b;
        }
        __syncthreads();
    }
};

// Every thread waits until its stores of this node have reached the L2 (the
// workgroup-scope fence alone does not wait for them on this chip), then,
// after the barrier, thread 0 releases them all device-wide with the count or
// flag stores that publish them.
__device__ __forceinline__ void release_node()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): every vector memory access of this wave done
    __syncthreads();
}

// Backward step of a node of the fused list.  A node whose children are in
// the list too (kids) does not form their products: each child j has sent
// p_j = [A_j B_j]' qhat_j, written where the forward pass later writes x_j and
// u_j (nothing reads those outputs before), so after its wait the node only
// adds the p_j to its own terms.  A node whose parent is in the list (i != 0)
// then sends its own p_i.  Nodes of the deepest listed stage form their
// children's products as the per-stage kernel does.  Every row this needs
// is requested before the wait.
template <int NRHS, int CH, int NW>
__device__ void bwd_fused_node(const SweepArgs &a, const InstDesc &I, int i, int w, int lane, bool kids,
                               const FusedWait &wait)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu, ldq = I.ldx, ldM = I.ldM;
    const int *cp = a.cp + I.cp;
    constexpr int kDepth = CH == 1 && NW <= 8 ? 2 : 1;
    const int CB = child_batch(NRHS, ldq), ldv = CB * ldq;
    extern __shared__ double lds[];
    double *qs = lds;                          // [NRHS][ldv]: children's qhat, later this node's qhat
    double *red = qs + NRHS * ldv;             // [NW][NRHS][ldM]
    double *as = red + NW * NRHS * ldM;        // [NRHS][ldM]: [sum A'q ; g_i] plus the node's own terms
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    const bool up = i != 0;
    const int pr0 = nx * w / NW, pr1 = nx * (w + 1) / NW;
    RowStream<CH> rk, rq, pm;
    {
        const int R = 2 * nu, r0 = R * w / NW, r1 = R * (w + 1) / NW;
        stream_open<1, CH>(rk, a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, r0, r1 < nu ? r1 : nu, nu, lane);
        stream_open<1, CH>(rq, a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, (r0 > nu ? r0 : nu) - nu, r1 - nu,
                           nx, lane);
    }
    if (kids) {
        if (up) stream_open<1, CH>(pm, a.Mb + I.Mb + (long long)i * nx * ldM, ldM, pr0, pr1, W, lane);
        const double si = a.sc ? a.sc[I.sc + i] : 1.0;
        // the node's own terms s_i y_i + [chat_i ; sigma_i], requested before the wait
        const int e0 = threadIdx.x < NRHS * W ? threadIdx.x : 0, k0 = e0 / W, c0 = e0 - k0 * W;
        const double y0 = y_ptr(a, I, k0, i)[c0];
        const double h0 = c0 < nx ? a.chat[I.chat + (long long)i * nx + c0] : a.sig[I.sig + (long long)i * nu + c0 - nx];
        wait();
        for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
            const int k = e / W, c = e - k * W;
            double s;
            if (e == e0) {
                s = si * y0 + (a.affine ? h0 : 0.0);
            } else {
                const double h = c < nx ? a.chat[I.chat + (long long)i * nx + c] : a.sig[I.sig + (long long)i * nu + c - nx];
                s = si * y_ptr(a, I, k, i)[c] + (a.affine ? h : 0.0);
            }
            // the children's p_j, eight loads in flight at a time (a chunk's
            // unused slots re-read its first child and are not added)
            for (int j = j0; j < j0 + nch; j += 8) {
                double v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int jj = j + t < j0 + nch ? j + t : j;
                    v[t] = c < nx ? x_ptr(a, I, k, jj)[c] : u_ptr(a, I, k, jj)[c - nx];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (j + t < j0 + nch) s += v[t];
            }
            as[k * ldM + c] = s;
        }
    } else {
        NodeTerms<NRHS, CH> nt;
        node_terms<NRHS, CH, kWave>(a, I, i, lane, nt);
        double acc[NRHS][CH][2];
        zero(acc);
        for (int cb = 0; cb < nch; cb += CB) {
            const int nb = nch - cb < CB ? nch - cb : CB;
            const int R = nb * nx, r0 = (int)((long long)R * w / NW), r1 = (int)((long long)R * (w + 1) / NW);
            RowStream<CH> mb;
            stream_open<kDepth, CH>(mb, a.Mb + I.Mb + (long long)(j0 + cb) * nx * ldM, ldM, r0, r1, W, lane);
            if (cb == 0) wait();
            for (int e = threadIdx.x; e < R; e += blockDim.x) {
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
                    qs[k * ldv + e] = q;
                }
            }
            __syncthreads();
            stream_run<kDepth, NRHS, CH>(mb, qs, ldv, acc);
            __syncthreads();   // qs is refilled (or, last, holds this node's qhat)
        }
        if (up) stream_open<1, CH>(pm, a.Mb + I.Mb + (long long)i * nx * ldM, ldM, pr0, pr1, W, lane);
        if (w == 0) add_node_terms(a, acc, nt);
        store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, W, acc, lane);
        __syncthreads();
        for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
            const int k = e / W, c = e - k * W;
            double s = 0.0;
            for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
            as[k * ldM + c] = s;
        }
    }
    __syncthreads();
    // g_i = as[nx:]: k_i = -R~_i^{-1} g_i and qhat_i = as[:nx] + K_i' g_i
    double kacc[NRHS][CH][2], qacc[NRHS][CH][2];
    zero(kacc);
    zero(qacc);
    stream_run<1, NRHS, CH>(rk, as + nx, ldM, kacc);
    stream_run<1, NRHS, CH>(rq, as + nx, ldM, qacc);
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
            const double q = as[k * ldM + c - nu] + s;
            qhat_ptr(a, I, k, i)[c - nu] = q;
            qs[k * ldq + c - nu] = q;
        }
    }
    if (!up) return;
    // p_i = [A_i B_i]' qhat_i for the parent
    __syncthreads();
    double pacc[NRHS][CH][2];
    zero(pacc);
    stream_run<1, NRHS, CH>(pm, qs, ldq, pacc);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, W, pacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
        const int k = e / W, c = e - k * W;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + c];
        if (c < nx)
            x_ptr(a, I, k, i)[c] = s;
        else
            u_ptr(a, I, k, i)[c - nx] = s;
    }
}

// Forward step of a node of the fused list: x_i = A_i x_p + B_i u_p + c_i
// from its parent's x_p and u_p (x_0 at the root), then u_i = K_i x_i + k_i;
// a node whose children are not in the list also forms their x_j, as the
// per-stage kernel does.  Every row this needs is requested before the wait.
template <int NRHS, int CH, int NW>
__device__ void fwd_fused_node(const SweepArgs &a, const InstDesc &I, int i, int w, int lane, bool kids,
                               const FusedWait &wait)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu, ldM = I.ldM;
    const int *cp = a.cp + I.cp;
    extern __shared__ double lds[];
    double *xs = lds;                     // [NRHS][ldM]: x_i then u_i
    double *red = xs + NRHS * ldM;        // [NW][NRHS][ldM]
    double *xp = red + NW * NRHS * ldM;   // [NRHS][ldM]: the parent's x and u
    const bool root = i == 0;
    RowStream<CH> me, kf, mf;
    double cme[CH][2], kv[NRHS][CH][2], cv[CH][2];
    if (!root) {
        const int r0 = W * w / NW, r1 = W * (w + 1) / NW;
        stream_open<1, CH>(me, a.Mf + I.Mf + (long long)i * W * I.ldx, I.ldx, r0, r1, nx, lane);
        load_cvec<CH>(a, I, i, lane, cme);
    }
    {
        const int r0 = nx * w / NW, r1 = nx * (w + 1) / NW;
        stream_open<1, CH>(kf, a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, r0, r1, nu, lane);
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = 2 * lane + 2 * kWave * ch + e;
#pragma unroll
                for (int k = 0; k < NRHS; ++k) kv[k][ch][e] = kbuf_ptr(a, I, k, i)[c < nu ? c : nu - 1];
            }
    }
    const int j0 = cp[i], nch = cp[i + 1] - j0;
    const int RB = nch >= NW ? 1 : NW / nch;
    int c = RB == 1 ? w : w / RB;
    const int blk = RB == 1 ? 0 : w - c * RB;
    if (!kids && c < nch) {
        const int rr0 = W * blk / RB, rr1 = W * (blk + 1) / RB;
        stream_open<1, CH>(mf, a.Mf + I.Mf + (long long)(j0 + c) * W * I.ldx, I.ldx, rr0, rr1, nx, lane);
        load_cvec<CH>(a, I, j0 + c, lane, cv);
    }
    wait();
    if (root) {
        for (int e = threadIdx.x; e < NRHS * nx; e += blockDim.x) {
            const int k = e / nx, cc = e - k * nx;
            const double v = a.affine ? a.x0[k * a.x0_rs + I.x0 + cc] : 0.0;
            x_ptr(a, I, k, 0)[cc] = v;
            xs[k * ldM + cc] = v;
        }
    } else {
        const int p = a.anc[I.sc + i];
        for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
            const int k = e / W, cc = e - k * W;
            xp[k * ldM + cc] = cc < nx ? x_ptr(a, I, k, p)[cc] : u_ptr(a, I, k, p)[cc - nx];
        }
        __syncthreads();
        double xacc[NRHS][CH][2];
        zero(xacc);
        stream_run<1, NRHS, CH>(me, xp, ldM, xacc);
        if (w == 0)
#pragma unroll
            for (int k = 0; k < NRHS; ++k)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch) {
                    xacc[k][ch][0] += a.affine ? cme[ch][0] : 0.0;
                    xacc[k][ch][1] += a.affine ? cme[ch][1] : 0.0;
                }
        store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nx, xacc, lane);
        __syncthreads();
        for (int e = threadIdx.x; e < NRHS * nx; e += blockDim.x) {
            const int k = e / nx, cc = e - k * nx;
            double s = 0.0;
            for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + cc];
            x_ptr(a, I, k, i)[cc] = s;
            xs[k * ldM + cc] = s;
        }
    }
    __syncthreads();
    double uacc[NRHS][CH][2];
    zero(uacc);
    stream_run<1, NRHS, CH>(kf, xs, ldM, uacc);
    if (w == 0) add_to(uacc, kv);
    store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nu, uacc, lane);
    __syncthreads();
    for (int e = threadIdx.x; e < NRHS * nu; e += blockDim.x) {
        const int k = e / nu, cc = e - k * nu;
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[(ww * NRHS + k) * ldM + cc];
        u_ptr(a, I, k, i)[cc] = s;
        xs[k * ldM + nx + cc] = s;
    }
    if (kids) return;
    __syncthreads();
    // the children's x_j = [A_j B_j]' [x_i ; u_i] + c_j (as the per-stage kernel)
    if (RB == 1) {
        for (; c < nch; c += NW) {
            double xacc[NRHS][CH][2];
            zero(xacc);
            stream_run<1, NRHS, CH>(mf, xs, ldM, xacc);
#pragma unroll
            for (int k = 0; k < NRHS; ++k)
#pragma unroll
                for (int ch = 0; ch < CH; ++ch) {
                    xacc[k][ch][0] += a.affine ? cv[ch][0] : 0.0;
                    xacc[k][ch][1] += a.affine ? cv[ch][1] : 0.0;
                }
            const int j = j0 + c;
            if (c + NW < nch) {
                stream_open<1, CH>(mf, a.Mf + I.Mf + (long long)(j + NW) * W * I.ldx, I.ldx, 0, W, nx, lane);
                load_cvec<CH>(a, I, j + NW, lane, cv);
            }
#pragma unroll
            for (int ch = 0; ch < CH; ++ch)
#pragma unroll
                for (int e2 = 0; e2 < 2; ++e2) {
                    const int col = 2 * lane + 2 * kWave * ch + e2;
                    if (col < nx)
#pragma unroll
                        for (int k = 0; k < NRHS; ++k) x_ptr(a, I, k, j)[col] = xacc[k][ch][e2];
                }
        }
    } else {
        double xacc[NRHS][CH][2];
        zero(xacc);
        if (c < nch) {
            stream_run<1, NRHS, CH>(mf, xs, ldM, xacc);
            if (blk == 0)
#pragma unroll
                for (int k = 0; k < NRHS; ++k)
#pragma unroll
                    for (int ch = 0; ch < CH; ++ch) {
                        xacc[k][ch][0] += a.affine ? cv[ch][0] : 0.0;
                        xacc[k][ch][1] += a.affine ? cv[ch][1] : 0.0;
                    }
        }
        store_acc<NRHS, CH>(red + w * NRHS * ldM, ldM, 0, nx, xacc, lane);
        __syncthreads();
        for (int e = threadIdx.x; e < nch * NRHS * nx; e += blockDim.x) {
            const int cc = e / (NRHS * nx), rem = e - cc * NRHS * nx, k = rem / nx, col = rem - k * nx;
            double s = 0.0;
            for (int b = 0; b < RB; ++b) s += red[((cc * RB + b) * NRHS + k) * ldM + col];
            x_ptr(a, I, k, j0 + cc)[col] = s;
        }
    }
}

template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) bwd_trunk_fused_kernel(SweepArgs a, int *cnt, int *err)
{
    const int bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i = it.idx & ~kFusedKids;
    const bool kids = (it.idx & kFusedKids) != 0;
    __shared__ int poison;
    FusedWait fw{nullptr, 0, err, bad, &poison};
    if (kids) {
        fw.c = cnt + I.node0 + i;
        fw.target = a.cp[I.cp + i + 1] - a.cp[I.cp + i];
    }
    bwd_fused_node<NRHS, CH, NW>(a, I, i, w, lane, kids, fw);
    if (poison) {
        __syncthreads();
        const double nan = __builtin_nan("");
        const int W = I.nx + I.nu;
        for (int e = threadIdx.x; e < NRHS * W; e += blockDim.x) {
            const int k = e / W, c = e - k * W;
            if (c < I.nu)
                kbuf_ptr(a, I, k, i)[c] = nan;
            else
                qhat_ptr(a, I, k, i)[c - I.nu] = nan;
            if (i != 0) {
                if (c < I.nx)
                    x_ptr(a, I, k, i)[c] = nan;
                else
                    u_ptr(a, I, k, i)[c - I.nx] = nan;
            }
        }
    }
    if (i == 0) return;
    release_node();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(cnt + I.node0 + a.anc[I.sc + i], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NRHS, int CH, int NW>
__global__ void __launch_bounds__(kWave *NW) fwd_trunk_fused_kernel(SweepArgs a, int *cnt, int *err)
{
    const int bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Item it = a.items[blockIdx.x];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (kWave - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i = it.idx & ~kFusedKids;
    const bool kids = (it.idx & kFusedKids) != 0;
    __shared__ int poison;
    FusedWait fw{i == 0 ? nullptr : cnt + I.node0 + i, 1, err, bad, &poison};
    fwd_fused_node<NRHS, CH, NW>(a, I, i, w, lane, kids, fw);
    const int j0 = a.cp[I.cp + i], nch = a.cp[I.cp + i + 1] - j0;
    if (poison) {
        __syncthreads();
        const double nan = __builtin_nan("");
        const int per = I.nx + I.nu + (kids ? 0 : nch * I.nx);
        for (int e = threadIdx.x; e < NRHS * per; e += blockDim.x) {
            const int k = e / per, r = e - k * per;
            if (r < I.nx)
                x_ptr(a, I, k, i)[r] = nan;
            else if (r < I.nx + I.nu)
                u_ptr(a, I, k, i)[r - I.nx] = nan;
            else
                x_ptr(a, I, k, j0 + (r - I.nx - I.nu) / I.nx)[(r - I.nx - I.nu) % I.nx] = nan;
        }
    }
    if (!kids) return;
    release_node();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (int j = j0; j < j0 + nch; ++j)
            __hip_atomic_store(cnt + I.node0 + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---- stages s*..N-1: chain c of an instance covers the nodes
// stage_ptr[t] + c for t = s*..N-1 (one child each) and its leaf ----
//
// A group of G lanes walks one chain; a wavefront holds kWave/G groups, all
// on consecutive chains of one instance (item = instance, first chain), so
// the instance's sizes, loop bounds and branches stay wavefront-uniform and a
// single row load brings in one row of kWave/G different chains' matrices.
template <int NRHS, int CH, int G>
__device__ __forceinline__ void bwd_chain_body(const SweepArgs &a, const Item *items, int nitems, int blk, int ldq)
{
    constexpr int kGroups = kWave / G;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = blk * kWavesPerBlock + wave;
    if (item >= nitems) return;
    const Item it = items[item];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (G - 1), grp = (threadIdx.x & (kWave - 1)) / G;
    const int chain = it.idx + grp;
    if (chain >= I.nchains) return;
    const int *sp = a.sp + I.sp;
    const WaveLds L = wave_lds(ldq, NRHS, wave * kGroups + grp);
    // every stage from s* on holds the nchains chain nodes in chain order:
    // the chain's node of stage t is sp[s*] + chain + (t - s*) nchains, and
    // its child is nchains further on (64-lane groups read it from the child
    // pointers instead, which measured faster for them)
    const int head = sp[I.sstar] + chain;
    for (int t = I.N - 1; t >= I.sstar; --t) {
        const int i = head + (t - I.sstar) * I.nchains;
        bwd_node<NRHS, CH, G, (G < kWave), G == kWave ? kChainRowBatch : kRowBatch>(
            a, I, i, L, t != I.N - 1, t == I.sstar && t > 0, lane, i + I.nchains);
    }
}

template <int NRHS, int CH, int G>
__device__ __forceinline__ void fwd_chain_body(const SweepArgs &a, const Item *items, int nitems, int blk, int ldq)
{
    constexpr int kGroups = kWave / G;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = blk * kWavesPerBlock + wave;
    if (item >= nitems) return;
    const Item it = items[item];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (G - 1), grp = (threadIdx.x & (kWave - 1)) / G;
    const int chain = it.idx + grp;
    if (chain >= I.nchains) return;
    const int *sp = a.sp + I.sp;
    const WaveLds L = wave_lds(ldq, NRHS, wave * kGroups + grp);
    load_x<NRHS, G>(a, I, sp[I.sstar] + chain, L, lane);
    // the chain's node of stage t and its child, as in the backward pass
    const int head = sp[I.sstar] + chain;
    for (int t = I.sstar; t < I.N; ++t) {
        const int i = head + (t - I.sstar) * I.nchains;
        fwd_node<NRHS, CH, G, true>(a, I, i, L, t + 1 < I.N, lane, i + I.nchains);
    }
}

// Chains of one lane-group width (G = 64).
template <int NRHS, int CH, int G>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) bwd_chain_kernel(SweepArgs a, int ldq)
{
    bwd_chain_body<NRHS, CH, G>(a, a.items, a.nitems, blockIdx.x, ldq);
}

template <int NRHS, int CH, int G>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) fwd_chain_kernel(SweepArgs a, int ldq)
{
    fwd_chain_body<NRHS, CH, G>(a, a.items, a.nitems, blockIdx.x, ldq);
}

// Chains of the narrow widths (G = 8, 16, 32) in one launch: the grid is cut
// into consecutive block ranges, one per width, so that instances of every
// size share the machine without a launch (and its tail) per width.
struct NarrowChains {
    int n;
    int G[3], ldq[3], count[3];
    int first_block[4];
    const Item *items[3];
};

// Nodes of one stage above s* (stage a.t) of narrow instances, a lane group
// per node (item = instance, first node of kWave/G consecutive nodes).
template <int NRHS, int G, bool BWD>
__device__ __forceinline__ void level_body(const SweepArgs &a, const Item *items, int nitems, int blk, int ldq)
{
    constexpr int kGroups = kWave / G;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = blk * kWavesPerBlock + wave;
    if (item >= nitems) return;
    const Item it = items[item];
    if (skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int lane = threadIdx.x & (G - 1), grp = (threadIdx.x & (kWave - 1)) / G;
    const int node = it.idx + grp;
    if (node >= a.sp[I.sp + a.t + 1]) return;
    const WaveLds L = wave_lds(ldq, NRHS, wave * kGroups + grp);
    if (BWD) {
        bwd_node<NRHS, 1, G>(a, I, node, L, false, true, lane);
    } else {
        load_x<NRHS, G>(a, I, node, L, lane);
        fwd_node<NRHS, 1, G>(a, I, node, L, false, lane);
    }
}

template <int NRHS, bool BWD>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) narrow_level_kernel(SweepArgs a, NarrowChains nc)
{
    int c = 0;
    while (c + 1 < nc.n && (int)blockIdx.x >= nc.first_block[c + 1]) ++c;
    const int blk = blockIdx.x - nc.first_block[c];
    switch (nc.G[c]) {
    case 8: level_body<NRHS, 8, BWD>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]); break;
    case 16: level_body<NRHS, 16, BWD>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]); break;
    default: level_body<NRHS, 32, BWD>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]); break;
    }
}

template <int NRHS, bool BWD>
__global__ void __launch_bounds__(kWave *kWavesPerBlock, 2) narrow_chain_kernel(SweepArgs a, NarrowChains nc)
{
    int c = 0;
    while (c + 1 < nc.n && (int)blockIdx.x >= nc.first_block[c + 1]) ++c;
    const int blk = blockIdx.x - nc.first_block[c];
    switch (nc.G[c]) {
    case 8:
        if (BWD) bwd_chain_body<NRHS, 1, 8>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        else fwd_chain_body<NRHS, 1, 8>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        break;
    case 16:
        if (BWD) bwd_chain_body<NRHS, 1, 16>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        else fwd_chain_body<NRHS, 1, 16>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        break;
    default:
        if (BWD) bwd_chain_body<NRHS, 1, 32>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        else fwd_chain_body<NRHS, 1, 32>(a, nc.items[c], nc.count[c], blk, nc.ldq[c]);
        break;
    }
}

}  // namespace

SweepArgs sweep_args(const tree_factors *f, int affine)
{
    SweepArgs a{};
    a.inst = f->d_inst_xu;   // the sweeps work in the (x, u) layout
    a.sp = f->d_sp; a.cp = f->d_cp; a.anc = f->d_anc;
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

bool timing_on() { return g_timing.on; }

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
        const size_t lds = sizeof(double) * ((size_t)max_qs * NRHS + (size_t)(NW + 1) * NRHS * max_ldM);
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
    // rows wider than 128 entries (CH = 2) never get more than 8 wavefronts
    case 16: launch_trunk_nw<NRHS, CH, CH == 1 ? 16 : 8>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 8: launch_trunk_nw<NRHS, CH, 8>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 4: launch_trunk_nw<NRHS, CH, 4>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    case 2: launch_trunk_nw<NRHS, CH, 2>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    default: launch_trunk_nw<NRHS, CH, 1>(backward, a, lv, max_ldM, max_qs, max_ldu, st); break;
    }
}

template <int NRHS, int CH, int NW>
static void launch_trunk_tree_nw(SweepArgs a, const tree_factors *f, int max_ldM, int max_qs, int max_ldu,
                                 hipStream_t st)
{
    a.items = f->trunk_entry.items;
    a.nitems = f->trunk_entry.count;
    const size_t lds = sizeof(double) * ((size_t)max_qs * NRHS + (size_t)(NW + 1) * NRHS * max_ldM);
    hipLaunchKernelGGL((bwd_trunk_tree_kernel<NRHS, CH, NW>), dim3(a.nitems), dim3(kWave * NW), lds, st, a,
                       f->trunk_cnt);
}

template <int NRHS, int CH>
static void launch_trunk_tree(const SweepArgs &a, const tree_factors *f, int max_ldM, int max_qs, int max_ldu,
                              hipStream_t st)
{
    switch (f->trunk_entry.nw) {
    case 16: launch_trunk_tree_nw<NRHS, CH, CH == 1 ? 16 : 8>(a, f, max_ldM, max_qs, max_ldu, st); break;
    case 8: launch_trunk_tree_nw<NRHS, CH, 8>(a, f, max_ldM, max_qs, max_ldu, st); break;
    case 4: launch_trunk_tree_nw<NRHS, CH, 4>(a, f, max_ldM, max_qs, max_ldu, st); break;
    case 2: launch_trunk_tree_nw<NRHS, CH, 2>(a, f, max_ldM, max_qs, max_ldu, st); break;
    default: launch_trunk_tree_nw<NRHS, CH, 1>(a, f, max_ldM, max_qs, max_ldu, st); break;
    }
}

template <int NRHS, int CH, int NW>
static void launch_trunk_fused_nw(bool backward, SweepArgs a, const tree_factors *f, int max_ldM, int max_qs,
                                  hipStream_t st)
{
    const LevelPlan &lv = backward ? f->fused_bwd : f->fused_fwd;
    a.items = lv.items;
    a.nitems = lv.count;
    a.t = -1;
    int *err = f->trunk_cnt + f->V_tot;
    if (backward) {
        const size_t lds = sizeof(double) * ((size_t)max_qs * NRHS + (size_t)(NW + 1) * NRHS * max_ldM);
        hipLaunchKernelGGL((bwd_trunk_fused_kernel<NRHS, CH, NW>), dim3(lv.count), dim3(kWave * NW), lds, st, a,
                           f->trunk_cnt, err);
    } else {
        const size_t lds = sizeof(double) * (size_t)(NW + 2) * NRHS * max_ldM;
        hipLaunchKernelGGL((fwd_trunk_fused_kernel<NRHS, CH, NW>), dim3(lv.count), dim3(kWave * NW), lds, st, a,
                           f->trunk_cnt, err);
    }
}

template <int NRHS, int CH>
static void launch_trunk_fused(bool backward, const SweepArgs &a, const tree_factors *f, int max_ldM, int max_qs,
                               hipStream_t st)
{
    // every row of a node is held in registers across its wait: at most 8
    // wavefronts per node (4 for rows wider than 128 entries) keep them unspilled
    switch ((backward ? f->fused_bwd : f->fused_fwd).nw) {
    case 16:
    case 8: launch_trunk_fused_nw<NRHS, CH, CH == 1 ? 8 : 4>(backward, a, f, max_ldM, max_qs, st); break;
    case 4: launch_trunk_fused_nw<NRHS, CH, 4>(backward, a, f, max_ldM, max_qs, st); break;
    case 2: launch_trunk_fused_nw<NRHS, CH, 2>(backward, a, f, max_ldM, max_qs, st); break;
    default: launch_trunk_fused_nw<NRHS, CH, 1>(backward, a, f, max_ldM, max_qs, st); break;
    }
}

// One stage above s*: per-node workgroups for every node, or (trunk mode 2)
// lane groups for the narrow instances' nodes plus workgroups for the rest.
template <int NRHS, int CH>
static void launch_level(bool backward, const SweepArgs &a, const tree_factors *f, const LevelPlan &lv, int ldM,
                         int qs, int ldu, hipStream_t st)
{
    if (f->trunk_fused != 2) {
        launch_trunk<NRHS, CH>(backward, a, lv, ldM, qs, ldu, st);
        return;
    }
    if (lv.wide_count > 0) {
        LevelPlan w{};
        w.t = lv.t;
        w.count = lv.wide_count;
        w.nw = lv.wide_nw;
        w.items = lv.wide_items;
        launch_trunk<NRHS, CH>(backward, a, w, ldM, qs, ldu, st);
    }
    if (lv.narrow.empty()) return;
    NarrowChains nc{};
    size_t lds = 0;
    for (const ChainPlan &g : lv.narrow) {
        const int blocks = (g.count + kWavesPerBlock - 1) / kWavesPerBlock;
        nc.G[nc.n] = g.G;
        nc.ldq[nc.n] = g.ldq;
        nc.count[nc.n] = g.count;
        nc.items[nc.n] = g.items;
        nc.first_block[nc.n + 1] = nc.first_block[nc.n] + blocks;
        ++nc.n;
        lds = std::max(lds, sizeof(double) * (size_t)kWavesPerBlock * (kWave / g.G) * 3 * NRHS * g.ldq);
    }
    SweepArgs la = a;
    la.t = lv.t;
    const dim3 blk(kWave * kWavesPerBlock), grid(nc.first_block[nc.n]);
    if (backward)
        hipLaunchKernelGGL((narrow_level_kernel<NRHS, true>), grid, blk, lds, st, la, nc);
    else
        hipLaunchKernelGGL((narrow_level_kernel<NRHS, false>), grid, blk, lds, st, la, nc);
}

// Chain launches: one for all narrow widths together, one per wide plan.
template <int NRHS>
static void launch_chains(bool backward, const SweepArgs &a, const tree_factors *f, hipStream_t st)
{
    const dim3 blk(kWave * kWavesPerBlock);
    NarrowChains nc{};
    size_t narrow_lds = 0;
    for (const ChainPlan &cp : f->chains) {
        const int blocks = (cp.count + kWavesPerBlock - 1) / kWavesPerBlock;
        const size_t lds = sizeof(double) * (size_t)kWavesPerBlock * (kWave / cp.G) * 3 * NRHS * cp.ldq;
        if (cp.G < kWave) {
            nc.G[nc.n] = cp.G;
            nc.ldq[nc.n] = cp.ldq;
            nc.count[nc.n] = cp.count;
            nc.items[nc.n] = cp.items;
            nc.first_block[nc.n + 1] = nc.first_block[nc.n] + blocks;
            ++nc.n;
            narrow_lds = std::max(narrow_lds, lds);
            continue;
        }
        SweepArgs ca = a;
        ca.items = cp.items;
        ca.nitems = cp.count;
        if (cp.CH == 1) {
            if (backward)
                hipLaunchKernelGGL((bwd_chain_kernel<NRHS, 1, kWave>), dim3(blocks), blk, lds, st, ca, cp.ldq);
            else
                hipLaunchKernelGGL((fwd_chain_kernel<NRHS, 1, kWave>), dim3(blocks), blk, lds, st, ca, cp.ldq);
        } else {
            if (backward)
                hipLaunchKernelGGL((bwd_chain_kernel<NRHS, 2, kWave>), dim3(blocks), blk, lds, st, ca, cp.ldq);
            else
                hipLaunchKernelGGL((fwd_chain_kernel<NRHS, 2, kWave>), dim3(blocks), blk, lds, st, ca, cp.ldq);
        }
    }
    if (nc.n > 0) {
        const dim3 grid(nc.first_block[nc.n]);
        if (backward)
            hipLaunchKernelGGL((narrow_chain_kernel<NRHS, true>), grid, blk, narrow_lds, st, a, nc);
        else
            hipLaunchKernelGGL((narrow_chain_kernel<NRHS, false>), grid, blk, narrow_lds, st, a, nc);
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
    if (!f->chains.empty()) {
        PhaseTimer tm(0, st);
        launch_chains<NRHS>(true, a, f, st);
    }
    if (!f->levels.empty()) {
        PhaseTimer tm(1, st);
        if (f->trunk_fused == 1 && f->trunk_entry.count > 0) {
            launch_trunk_tree<NRHS, CH>(a, f, ldM, qs, ldu, st);
        } else if (f->trunk_fused >= 3) {
            // the deeper stages one launch each, then the first stages in one
            for (int k = (int)f->rest_levels.size() - 1; k >= 0; --k)
                launch_trunk<NRHS, CH>(true, a, f->rest_levels[k], ldM, qs, ldu, st);
            if (f->fused_bwd.count > 0) launch_trunk_fused<NRHS, CH>(true, a, f, ldM, qs, st);
        } else {
            for (int k = (int)f->levels.size() - 1; k >= 0; --k)
                launch_level<NRHS, CH>(true, a, f, f->levels[k], ldM, qs, ldu, st);
        }
    }
    if (!f->levels.empty()) {
        PhaseTimer tm(2, st);
        if (f->trunk_fused >= 3) {
            if (f->fused_fwd.count > 0) launch_trunk_fused<NRHS, CH>(false, a, f, ldM, qs, st);
            for (size_t k = 0; k < f->rest_levels.size(); ++k)
                launch_trunk<NRHS, CH>(false, a, f->rest_levels[k], ldM, qs, ldu, st);
        } else {
            for (size_t k = 0; k < f->levels.size(); ++k)
                launch_level<NRHS, CH>(false, a, f, f->levels[k], ldM, qs, ldu, st);
        }
    }
    if (!f->chains.empty()) {
        PhaseTimer tm(3, st);
        launch_chains<NRHS>(false, a, f, st);
    }
    return hipGetLastError();
}

// Right-hand sides of q-hat / k workspace a dual_grad call needs: one on a
// shared handle's panel route, a panel's worth for 64-wide matrix-core
// panels, else a pair (or one).
int dual_grad_ws_rhs(const tree_factors *f, int nrhs)
{
    if (panel_route(f, f->ninst)) return 1;
    if (nrhs >= kRhsPanel && panel_tpw(f) > 0 && f->shared <= 1) return kRhsPanel;
    return nrhs >= 2 ? 2 : 1;
}

// ws: null, the handle's own workspace (grown on demand); otherwise caller
// memory of dual_grad_ws_rhs(f, nrhs) * (x_tot + u_tot) doubles, q-hat first.
// y is in the (x, u) layout the sweeps read, mxu_tot per right-hand side.
int enqueue_dual_grad(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                      double *u, hipStream_t st, double *ws)
{
    const int ws_rhs = dual_grad_ws_rhs(f, nrhs);
    if (!ws) {
        int rc = ensure_sweep_ws(f, ws_rhs);
        if (rc) return rc;
    }
    SweepArgs a = sweep_args(f, homogeneous ? 0 : 1);
    if (ws) {
        a.qhat = ws;
        a.kbuf = ws + (long long)ws_rhs * f->x_tot;
    }
    a.dual_out = 0;
    // shared handle: each right-hand side covers all instances in panels
    if (panel_route(f, f->ninst)) {
        for (int k = 0; k < nrhs; ++k) {
            a.x0 = x0 ? x0 + (long long)k * f->nx_tot : nullptr;
            a.y = y + (long long)k * f->mxu_tot;
            a.xo = x + (long long)k * f->x_tot;
            a.uo = u + (long long)k * f->u_tot;
            const hipError_t e = launch_sweep_any(f, a, 1, st, f->ninst);
            if (e != hipSuccess) {
                set_error(std::string("dual_grad: ") + hipGetErrorString(e));
                return STOTREE_ERR_DEVICE;
            }
        }
        return STOTREE_OK;
    }
    // panels of kRhsPanel right-hand sides on the matrix cores, the rest in
    // pairs (a shared handle's panel work lists hold instance 0's nodes only)
    const bool panel = ws_rhs == kRhsPanel;
    const int npanel = panel ? nrhs / kRhsPanel * kRhsPanel : 0;
    a.y_rs = f->mxu_tot;
    a.x0_rs = f->nx_tot;
    a.xo_rs = f->x_tot;
    a.uo_rs = f->u_tot;
    for (int k0 = 0; k0 < nrhs;) {
        const int nk = k0 < npanel ? kRhsPanel : (nrhs - k0 >= 2 ? 2 : 1);
        a.x0 = x0 ? x0 + (long long)k0 * f->nx_tot : nullptr;
        a.y = y + (long long)k0 * f->mxu_tot;
        a.xo = x + (long long)k0 * f->x_tot;
        a.uo = u + (long long)k0 * f->u_tot;
        hipError_t e = nk == kRhsPanel ? launch_panel_sweep(f, a, st) : launch_sweep_tree(f, a, nk, st);
        if (e != hipSuccess) {
            set_error(std::string("dual_grad: ") + hipGetErrorString(e));
            return STOTREE_ERR_DEVICE;
        }
        k0 += nk;
    }
    return STOTREE_OK;
}

hipError_t launch_sweep_tree(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st)
{
    const bool wide = f->max_width > 128;
    if (nrhs == 1) return wide ? sweep_impl<1, 2>(f, a, st) : sweep_impl<1, 1>(f, a, st);
    if (nrhs == 2) return wide ? sweep_impl<2, 2>(f, a, st) : sweep_impl<2, 1>(f, a, st);
    return hipErrorInvalidValue;
}

// ---- dual_grad without allocation: static device scratch ----
// The q-hat / k workspace of dual_grad_noalloc lives in this file-scope
// device array (one copy per GPU, alive until the process ends).  In host
// code its name is only a stand-in for the symbol: kernels get the device
// address that hipGetSymbolAddress returns for the current device.
constexpr long long kScratchDoubles = 16LL << 20;   // 128 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;   // device ordinal -> address of its scratch

// Address of this device's scratch, looked up once per device.
int scratch_address(double **out)
{
    int dev = -1;
    STOTREE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        STOTREE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        it = g_scratch_ptr.emplace(dev, static_cast<double *>(p)).first;
    }
    *out = it->second;
    return STOTREE_OK;
}
}  // namespace

int dual_grad_noalloc_impl(const tree_factors *fc, const double *x0, const double *y, int homogeneous, int nrhs,
                           double *x, double *u, hipStream_t st)
{
    tree_factors *f = const_cast<tree_factors *>(fc);
    if (f->cmap) {
        set_error("dual_grad_noalloc: handles with a constraint map are not supported");
        return STOTREE_ERR_ARG;
    }
    const long long need = (long long)dual_grad_ws_rhs(f, nrhs) * (f->x_tot + f->u_tot);
    if (need > kScratchDoubles) {
        set_error("dual_grad_noalloc: the sweep workspace needs " + std::to_string(need * 8) +
                  " bytes, more than the " + std::to_string(kScratchDoubles * 8) + "-byte static scratch");
        return STOTREE_ERR_ARG;
    }
    double *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    return enqueue_dual_grad(f, x0, y, homogeneous, nrhs, x, u, st, ws);
}

}  // namespace stotree
