// Sweeps of 64 right-hand sides that share one tree's factors (Algorithms 3
// and 4 of arXiv 2107.01745, Sec. III-D, with the extra parallelism of
// Sec. III-C taken to many dual vectors): every per-node product becomes a
// small dense matrix product, factor (rows x cols) times a panel of 64
// right-hand sides, which runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).
//
// The algebra is the regrouped recursion of the single-vector sweep
// (sweep.hip): backward g_i = s_i y_i^u + pi_i r_i + sum_j B_j' qhat_j,
// k_i = -R~_i^{-1} g_i, qhat_i = chat_i + s_i y_i^x + sum_j A_j' qhat_j +
// K_i' g_i; forward u_i = K_i x_i + k_i, x_j = A_j x_i + B_j u_i + c_j.
//
// Mapping.  One workgroup of four wavefronts per node (per chain below s*).
// The input panel of a product (qhat, g or [x; u] of all 64 right-hand
// sides, one LDS row per vector entry) sits in LDS; the factor operand is read
// straight from HBM in the layout the single-vector sweep streams.  The output
// of a product is cut into 16-row tiles of the x part and of the u part, each
// tile in two halves of 32 right-hand sides; the (tile, half) tasks are dealt
// round-robin to the wavefronts, and every task keeps its two 16x16 result
// blocks in registers.  The result accumulators start at the node's own
// vector terms (s_i y_i + chat_i / sig_i backward, k_i and c_j forward); the
// finished blocks go to the LDS panel, where they are the input of the next
// product (g for [K; -R~^{-1}] g, [x; u] for the children), and each lane
// completes its own entries of qhat_i there.  No load sits under a branch:
// the factor rows of a batch are all in flight together, and the next batch
// is loaded before the current one is multiplied.  Sums over the K dimension
// run in a fixed order (deterministic results).
//
// Operand layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16x4, B 4x16):
// lane l holds A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4e][l%16], e < 4
// (checked on the device against a plain product of known operands).
#include <vector>

#include "sweep_common.h"

namespace stotree {

namespace {

using namespace dev;

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kPanel = kRhsPanel;      // right-hand sides per launch (64)
constexpr int kLdv = kPanel + 2;       // LDS row stride of a panel (doubles)
constexpr int kWg = 4;                 // wavefronts per workgroup
constexpr int kTpwMax = 4;             // most tasks one wavefront can hold
constexpr int kKu = 4;                 // K steps (of 4 rows) per batch of operand loads
// Wavefronts per SIMD each kernel is compiled for (register budget without
// spills): backward kernels three up to three tasks per wavefront (panels of
// <= 96 rows fit three to the LDS), forward kernels three up to two tasks.
template <int TPW>
constexpr int kMinWavesBwd = TPW <= 3 ? 3 : 2;
template <int TPW>
constexpr int kMinWavesFwd = TPW <= 2 ? 3 : 2;

// Source of one output part of a product: out[c] = sum_r M[r][col0 + c] v[r]
// for c < ncols, M row-major with leading dimension ld.
struct Part {
    const double *M;
    int ld, col0, ncols;
};

// Tasks of a product: tiles of part 0 then part 1 (ceil(ncols/16) each),
// two halves each; wavefront w owns tasks w, w + kWg, ...
struct Tasks {
    int t0, t1;                        // tiles of part 0 / part 1
    __device__ int count() const { return 2 * (t0 + t1); }
};

__host__ __device__ inline int tiles(int n) { return (n + 15) >> 4; }

// The factor side of one product for wavefront w: column pointers of its
// tasks w + kWg*s (owned while below the task count; advanced batch by batch)
// and the first batch of 16 rows, which stream_open loads so that it can be
// issued ahead of the point where stream_run multiplies.
template <int TPW>
struct FactorStream {
    const double *ap[TPW];
    long long ld[TPW];
    bool own[TPW];
    double a0[kKu][TPW];
};

template <int TPW>
__device__ __forceinline__ void stream_load(FactorStream<TPW> &f, double (&a)[kKu][TPW])
{
#pragma unroll
    for (int u = 0; u < kKu; ++u)
#pragma unroll
        for (int s = 0; s < TPW; ++s) a[u][s] = f.ap[s][4 * u * f.ld[s]];
#pragma unroll
    for (int s = 0; s < TPW; ++s) f.ap[s] += 4 * kKu * f.ld[s];
}

// Every load is unconditional (a task past the count re-reads the first
// columns, a cache hit; columns past a part re-read its first column, whose
// rows of D are never stored), so the loads of a batch are all in flight
// together; only the matrix operations of unowned tasks are skipped, on a
// wavefront-uniform test.
template <int TPW>
__device__ __forceinline__ void stream_open(FactorStream<TPW> &f, const Part (&p)[2], const Tasks &tk, int R,
                                            int wave, int lane)
{
    const int n = tk.count();
    const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int task = wave + kWg * s;
        f.own[s] = task < n;
        const int tile = (f.own[s] ? task : 0) >> 1;
        const int part = tile < tk.t0 ? 0 : 1;
        const int c = (part ? tile - tk.t0 : tile) * 16 + lc;
        f.ap[s] = p[part].M + p[part].col0 + (c < p[part].ncols ? c : 0) + (long long)lr * p[part].ld;
        f.ld[s] = p[part].ld;
    }
    if (R >= 4 * kKu) stream_load(f, f.a0);
}

// acc[s][h] (+)= the product of task s with the LDS input panel V (R rows of
// kLdv).  Every task of a wavefront has half (w & 1), so they share the B
// operand.  Whole batches of 16 rows run with the factor loads of the next
// batch issued before the matrix operations of the current one (two register
// buffers); the last R mod 16 rows are a tail whose rows past R read a valid
// row and are zeroed (the panel needs no padding rows).
template <int TPW>
__device__ __forceinline__ void stream_run(FactorStream<TPW> &f, int R, const double *V, v4d (&acc)[TPW][2],
                                           int wave, int lane)
{
    const int lr = lane >> 4, lc = lane & 15;
    const double *vb = V + lr * kLdv + (wave & 1) * 32 + lc;   // this lane's B entry of row lr
    auto mma = [&](const double (&a)[kKu][TPW], const double (&b)[kKu][2]) {
#pragma unroll
        for (int u = 0; u < kKu; ++u)
#pragma unroll
            for (int s = 0; s < TPW; ++s)
                if (f.own[s]) {
                    acc[s][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], b[u][0], acc[s][0], 0, 0, 0);
                    acc[s][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], b[u][1], acc[s][1], 0, 0, 0);
                }
    };
    auto bload = [&](double (&b)[kKu][2], int k0) {
#pragma unroll
        for (int u = 0; u < kKu; ++u) {
            b[u][0] = vb[(k0 + 4 * u) * kLdv];
            b[u][1] = vb[(k0 + 4 * u) * kLdv + 16];
        }
    };
    const int nfull = R / (4 * kKu);
    double a1[kKu][TPW], b[kKu][2];
    int q = 0;
    for (; q + 2 <= nfull; q += 2) {
        stream_load(f, a1);
        bload(b, q * 4 * kKu);
        mma(f.a0, b);
        if (q + 2 < nfull) stream_load(f, f.a0);
        bload(b, (q + 1) * 4 * kKu);
        mma(a1, b);
    }
    if (q < nfull) {
        bload(b, q * 4 * kKu);
        mma(f.a0, b);
    }
    const int k0 = nfull * 4 * kKu;
    if (k0 < R) {
        // ap[s] points at row k0 + lr of its column; rows past R read row R - 1
        const int last = R - 1 - k0;
#pragma unroll
        for (int u = 0; u < kKu; ++u) {
            const bool in = 4 * u + lr <= last;
            const int d = (in ? 4 * u + lr : last) - lr;
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const double v = f.ap[s][d * f.ld[s]];
                f.a0[u][s] = in ? v : 0.0;
            }
            const double v0 = vb[(k0 + d) * kLdv], v1 = vb[(k0 + d) * kLdv + 16];
            b[u][0] = in ? v0 : 0.0;
            b[u][1] = in ? v1 : 0.0;
        }
        mma(f.a0, b);    // the steps past R add zero products
    }
}


template <int TPW>
__device__ __forceinline__ void product(const Part (&p)[2], const Tasks &tk, int R, const double *V,
                                        v4d (&acc)[TPW][2], int wave, int lane)
{
    FactorStream<TPW> f;
    stream_open(f, p, tk, R, wave, lane);
    stream_run(f, R, V, acc, wave, lane);
}

template <int TPW>
__device__ __forceinline__ void zero(v4d (&acc)[TPW][2])
{
#pragma unroll
    for (int s = 0; s < TPW; ++s) acc[s][0] = acc[s][1] = v4d{0.0, 0.0, 0.0, 0.0};
}

// Position of element (s, h, e) of this lane's results: part, row within the
// part, right-hand side.  valid is false for rows past the part's size and
// for tasks this wavefront does not own.
struct Slot {
    int part, row, rhs;
    bool valid;
};

__device__ __forceinline__ Slot slot(const Tasks &tk, const int (&ncols)[2], int s, int h, int e, int wave,
                                     int lane)
{
    Slot o;
    const int task = wave + kWg * s;
    const int tile = task >> 1;
    o.part = tile < tk.t0 ? 0 : 1;
    o.row = (o.part ? tile - tk.t0 : tile) * 16 + (lane >> 4) + 4 * e;
    o.rhs = (task & 1) * 32 + h * 16 + (lane & 15);
    o.valid = task < tk.count() && o.row < ncols[o.part];
    return o;
}

// Stage rows [0, n) of one node vector of every right-hand side into the
// panel rows [r0, r0 + n): V[r0 + r][k] = src(k, r).  A wavefront reads one
// right-hand side per instruction (consecutive rows on consecutive lanes),
// all its loads issued before the first LDS write.
template <typename Src>
__device__ __forceinline__ void stage(double *V, int r0, int n, Src src)
{
    constexpr int Q = 8;               // right-hand sides per round (loads in flight per lane)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    for (int rb = 0; rb < n; rb += kWave) {
        const int r = rb + lane;
        const bool in = r < n;
        const int rc = in ? r : n - 1;     // lanes past n read a valid entry and store nothing
        for (int k0 = wave; k0 < kPanel; k0 += Q * kWg) {
            double v[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] = src(k0 + kWg * q, rc);
            if (in) {
#pragma unroll
                for (int q = 0; q < Q; ++q) V[(r0 + r) * kLdv + k0 + kWg * q] = v[q];
            }
        }
    }
}

// Backward step of non-leaf node i (Algorithm 3 / 4 body) for the panel.  On
// entry, if child_in_lds, rows [0, nx) of V hold qhat of the single child; on
// exit they hold qhat_i.  k_i goes to kbuf; qhat_i to the global buffer if
// store_q.  The accumulators of the children's products start at
// s_i y_i + (chat_i; pi r = sig) of their slots, loaded together with the
// first factor batch, so they end as sum A'qhat + s_i y^x + chat_i (rows
// [0, nx), completed to qhat_i after the second product) and g_i (rows
// [nx, nx + nu), the input of the second product).
template <int TPW>
__device__ void bwd_node64(const SweepArgs &a, const InstDesc &I, int i, double *V, bool child_in_lds,
                           bool store_q, int wave, int lane)
{
    const int nx = I.nx, nu = I.nu;
    const int *cp = a.cp + I.cp;
    const Tasks tk{tiles(nx), tiles(nu)};
    const int ncols[2] = {nx, nu};
    const double si = a.sc ? a.sc[I.sc + i] : 1.0;
    v4d S[TPW][2];
    {
        // rows past a part read its last row; slots of unowned tasks are never stored
        const double *ch = a.chat + I.chat + (long long)i * nx;
        const double *sg = a.sig + I.sig + (long long)i * nu;
        const bool aff = a.affine;
#pragma unroll
        for (int s = 0; s < TPW; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                    const int row = o.row < ncols[o.part] ? o.row : ncols[o.part] - 1;
                    S[s][h][e] = si * y_ptr(a, I, o.rhs, i)[o.part ? nx + row : row];
                }
        if (aff) {
#pragma unroll
            for (int s = 0; s < TPW; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                        const int row = o.row < ncols[o.part] ? o.row : ncols[o.part] - 1;
                        S[s][h][e] += o.part ? sg[row] : ch[o.rhs * a.chat_rs + row];
                    }
        }
    }
    for (int j = cp[i]; j < cp[i + 1]; ++j) {
        if (!child_in_lds) {
            if (j >= I.Vnl) {
                const double sj = a.sc ? a.sc[I.sc + j] : 1.0;
                const double *cj = a.chat + I.chat + (long long)j * nx;
                if (a.affine)
                    stage(V, 0, nx,
                          [&](int k, int r) { return sj * y_ptr(a, I, k, j)[r] + cj[k * a.chat_rs + r]; });
                else
                    stage(V, 0, nx, [&](int k, int r) { return sj * y_ptr(a, I, k, j)[r]; });
            } else {
                stage(V, 0, nx, [&](int k, int r) { return qhat_ptr(a, I, k, j)[r]; });
            }
            __syncthreads();
        }
        const double *Mb = a.Mb + I.Mb + (long long)j * nx * I.ldM;
        const Part p[2] = {{Mb, I.ldM, 0, nx}, {Mb, I.ldM, nx, nu}};
        product(p, tk, nx, V, S, wave, lane);
        if (j + 1 < cp[i + 1]) __syncthreads();   // every wavefront is done with the child panel
    }
    // first batch of [K' ; -R~^{-1}] in flight across the barriers
    FactorStream<TPW> f2;
    {
        const Part p[2] = {{a.Kb + I.Kb + (long long)i * nu * I.ldx, I.ldx, 0, nx},
                           {a.Rn + I.Rn + (long long)i * nu * I.ldu, I.ldu, 0, nu}};
        stream_open(f2, p, tk, nu, wave, lane);
    }
    __syncthreads();       // every wavefront is done with the child panel
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                if (o.valid) V[(o.part ? nx + o.row : o.row) * kLdv + o.rhs] = S[s][h][e];
            }
    __syncthreads();
    // [K' g ; -R~^{-1} g]
    v4d T[TPW][2];
    zero(T);
    stream_run(f2, nu, V + nx * kLdv, T, wave, lane);
    // each lane completes its own entries of rows [0, nx); the g rows are not written
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                if (!o.valid) continue;
                if (o.part == 1) {
                    kbuf_ptr(a, I, o.rhs, i)[o.row] = T[s][h][e];
                } else {
                    const double q = V[o.row * kLdv + o.rhs] + T[s][h][e];
                    V[o.row * kLdv + o.rhs] = q;
                    if (store_q) qhat_ptr(a, I, o.rhs, i)[o.row] = q;
                }
            }
    __syncthreads();
}

// Forward step of non-leaf node i with x_i in panel rows [0, nx).  Writes u_i
// and the children's x_j; for a single-child chain (keep_child) the child's x
// replaces x_i in the panel.  The accumulators start at k_i (for u_i = K_i x_i
// + k_i) and at c_j (for x_j = A_j x_i + B_j u_i + c_j), loaded with the first
// factor batch.
template <int TPW>
__device__ void fwd_node64(const SweepArgs &a, const InstDesc &I, int i, double *V, bool keep_child, int wave,
                           int lane)
{
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const int *cp = a.cp + I.cp;
    const int ncols[2] = {nx, nu};
    const Tasks tkx{tiles(nx), 0};
    const int j0 = cp[i], j1 = cp[i + 1];
    FactorStream<TPW> fx;     // the first child's [A B], opened before the u_i barrier
    {
        const Tasks tk{0, tiles(nu)};
        v4d U[TPW][2];
        // rows past nu read row nu - 1; slots of unowned tasks are never stored
#pragma unroll
        for (int s = 0; s < TPW; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                    U[s][h][e] = kbuf_ptr(a, I, o.rhs, i)[o.row < nu ? o.row : nu - 1];
                }
        const Part p[2] = {{nullptr, 0, 0, 0}, {a.Kf + I.Kf + (long long)i * nx * I.ldu, I.ldu, 0, nu}};
        product(p, tk, nx, V, U, wave, lane);
        // rows [nx, W) are not read by K x_i: u_i goes there directly
#pragma unroll
        for (int s = 0; s < TPW; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const Slot o = slot(tk, ncols, s, h, e, wave, lane);
                    if (!o.valid) continue;
                    u_ptr(a, I, o.rhs, i)[o.row] = U[s][h][e];
                    V[(nx + o.row) * kLdv + o.rhs] = U[s][h][e];
                }
        const Part px[2] = {{a.Mf + I.Mf + (long long)j0 * W * I.ldx, I.ldx, 0, nx}, {nullptr, 0, 0, 0}};
        stream_open(fx, px, tkx, W, wave, lane);
        __syncthreads();
    }
    v4d X[TPW][2];
    for (int j = j0; j < j1; ++j) {
        if (a.affine) {
            const double *cj = a.cvec + I.c + (long long)j * nx;
#pragma unroll
            for (int s = 0; s < TPW; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const Slot o = slot(tkx, ncols, s, h, e, wave, lane);
                        X[s][h][e] = cj[o.rhs * a.c_rs + (o.row < nx ? o.row : nx - 1)];
                    }
        } else {
            zero(X);
        }
        if (j > j0) {
            const Part p[2] = {{a.Mf + I.Mf + (long long)j * W * I.ldx, I.ldx, 0, nx}, {nullptr, 0, 0, 0}};
            stream_open(fx, p, tkx, W, wave, lane);
        }
        stream_run(fx, W, V, X, wave, lane);
#pragma unroll
        for (int s = 0; s < TPW; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const Slot o = slot(tkx, ncols, s, h, e, wave, lane);
                    if (o.valid) x_ptr(a, I, o.rhs, j)[o.row] = X[s][h][e];
                }
    }
    if (keep_child) {
        __syncthreads();   // every wavefront is done reading [x_i; u_i]
#pragma unroll
        for (int s = 0; s < TPW; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const Slot o = slot(tkx, ncols, s, h, e, wave, lane);
                    if (o.valid) V[o.row * kLdv + o.rhs] = X[s][h][e];
                }
        __syncthreads();
    }
}

// x_i into panel rows [0, nx): x0 at the root (also written to the output),
// else the values the previous stage stored.
__device__ void load_x64(const SweepArgs &a, const InstDesc &I, int i, double *V)
{
    const int nx = I.nx;
    if (i != 0) {
        stage(V, 0, nx, [&](int k, int r) { return x_ptr(a, I, k, i)[r]; });
    } else if (a.affine) {
        stage(V, 0, nx, [&](int k, int r) { return a.x0[k * a.x0_rs + I.x0 + r]; });
        __syncthreads();
        // the root's x is x0: written out too (lanes past nx store nothing)
        for (int k = threadIdx.x / kWave; k < kPanel; k += kWg)
            for (int r = threadIdx.x & (kWave - 1); r < nx; r += kWave) x_ptr(a, I, k, 0)[r] = V[r * kLdv + k];
    } else {
        stage(V, 0, nx, [&](int k, int r) { return 0.0; });
        for (int k = threadIdx.x / kWave; k < kPanel; k += kWg)
            for (int r = threadIdx.x & (kWave - 1); r < nx; r += kWave) x_ptr(a, I, k, 0)[r] = 0.0;
    }
    __syncthreads();
}

// A workgroup leaves at once when its instance has finished or, on a shared
// panel, when every copy of the panel has (one flag per lane; the same
// answer in every wavefront).
__device__ __forceinline__ bool panel_skipped(const SweepArgs &a, int inst)
{
    if (!a.panel_done) return skipped(a, inst);
    const int lane = threadIdx.x & (kWave - 1);
    return __all(a.done[(long long)lane * a.done_stride] != 0);
}

template <int TPW>
__global__ void __launch_bounds__(kWave *kWg, kMinWavesBwd<TPW>) bwd_trunk64_kernel(SweepArgs a)
{
    extern __shared__ double lds[];
    const Item it = a.items[blockIdx.x];
    if (panel_skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    bwd_node64<TPW>(a, I, it.idx, lds, false, true, wave, lane);
}

template <int TPW>
__global__ void __launch_bounds__(kWave *kWg, kMinWavesFwd<TPW>) fwd_trunk64_kernel(SweepArgs a)
{
    extern __shared__ double lds[];
    const Item it = a.items[blockIdx.x];
    if (panel_skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    load_x64(a, I, it.idx, lds);
    fwd_node64<TPW>(a, I, it.idx, lds, false, wave, lane);
}

// The lane and wavefront ids as values the compiler cannot see through: the
// chain loops pass these so that the per-lane addresses of a node step are
// formed inside the step instead of being hoisted out of the loop and held
// in registers across it.
__device__ __forceinline__ void opaque_ids(int &wave, int &lane)
{
    asm volatile("" : "+s"(wave));
    asm volatile("" : "+v"(lane));
}

// Chains below s*: one workgroup per chain (items: instance, chain).
template <int TPW>
__global__ void __launch_bounds__(kWave *kWg, kMinWavesBwd<TPW>) bwd_chain64_kernel(SweepArgs a)
{
    extern __shared__ double lds[];
    const Item it = a.items[blockIdx.x];
    if (panel_skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    const int *sp = a.sp + I.sp;
    for (int t = I.N - 1; t >= I.sstar; --t) {
        int w = wave, l = lane;
        opaque_ids(w, l);
        bwd_node64<TPW>(a, I, sp[t] + it.idx, lds, t != I.N - 1, t == I.sstar && t > 0, w, l);
    }
}

template <int TPW>
__global__ void __launch_bounds__(kWave *kWg, kMinWavesFwd<TPW>) fwd_chain64_kernel(SweepArgs a)
{
    extern __shared__ double lds[];
    const Item it = a.items[blockIdx.x];
    if (panel_skipped(a, it.inst)) return;
    const InstDesc I = a.inst[it.inst];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    const int *sp = a.sp + I.sp;
    load_x64(a, I, sp[I.sstar] + it.idx, lds);
    for (int t = I.sstar; t < I.N; ++t) {
        int w = wave, l = lane;
        opaque_ids(w, l);
        fwd_node64<TPW>(a, I, sp[t] + it.idx, lds, t + 1 < I.N, w, l);
    }
}

}  // namespace

// Tasks per wavefront the largest instance needs (0: too wide for the panel sweep).
int panel_tpw(const tree_factors *f)
{
    int t = 1;
    for (const InstDesc &I : f->inst) {
        const int need = (2 * (tiles(I.nx) + tiles(I.nu)) + kWg - 1) / kWg;
        t = need > t ? need : t;
    }
    return t <= kTpwMax ? t : 0;
}

// Tasks per wavefront of the forward products alone (K x: 2 tiles(nu) tasks,
// [A B][x; u]: 2 tiles(nx)); at most panel_tpw.
static int panel_tpw_fwd(const tree_factors *f)
{
    int t = 1;
    for (const InstDesc &I : f->inst) {
        const int tl = tiles(I.nx) > tiles(I.nu) ? tiles(I.nx) : tiles(I.nu);
        const int need = (2 * tl + kWg - 1) / kWg;
        t = need > t ? need : t;
    }
    return t;
}

// TB tasks per wavefront in the backward kernels, TF in the forward ones.
template <int TB, int TF>
static void launch_panel(const tree_factors *f, const SweepArgs &a, size_t lds, hipStream_t st)
{
    const dim3 blk(kWave * kWg);
    SweepArgs ca = a;
    ca.items = f->panel_chain_items;
    ca.nitems = f->npanel_chain_items;
    const std::vector<LevelPlan> &levels = f->shared > 1 ? f->panel_levels : f->levels;
    if (ca.nitems > 0) hipLaunchKernelGGL(bwd_chain64_kernel<TB>, dim3(ca.nitems), blk, lds, st, ca);
    for (int k = (int)levels.size() - 1; k >= 0; --k) {
        SweepArgs la = a;
        la.items = levels[k].items;
        la.nitems = levels[k].count;
        if (la.nitems > 0) hipLaunchKernelGGL(bwd_trunk64_kernel<TB>, dim3(la.nitems), blk, lds, st, la);
    }
    for (size_t k = 0; k < levels.size(); ++k) {
        SweepArgs la = a;
        la.items = levels[k].items;
        la.nitems = levels[k].count;
        if (la.nitems > 0) hipLaunchKernelGGL(fwd_trunk64_kernel<TF>, dim3(la.nitems), blk, lds, st, la);
    }
    if (ca.nitems > 0) hipLaunchKernelGGL(fwd_chain64_kernel<TF>, dim3(ca.nitems), blk, lds, st, ca);
}

hipError_t launch_panel_sweep(const tree_factors *f, const SweepArgs &a, hipStream_t st)
{
    int W = 2;
    for (const InstDesc &I : f->inst) W = W > I.nx + I.nu ? W : I.nx + I.nu;
    const size_t lds = sizeof(double) * (size_t)W * kLdv;
    const int tb = panel_tpw(f), tf = panel_tpw_fwd(f);
    switch (tb * 8 + tf) {
    case 1 * 8 + 1: launch_panel<1, 1>(f, a, lds, st); break;
    case 2 * 8 + 1: launch_panel<2, 1>(f, a, lds, st); break;
    case 2 * 8 + 2: launch_panel<2, 2>(f, a, lds, st); break;
    case 3 * 8 + 2: launch_panel<3, 2>(f, a, lds, st); break;
    case 3 * 8 + 3: launch_panel<3, 3>(f, a, lds, st); break;
    case 4 * 8 + 2: launch_panel<4, 2>(f, a, lds, st); break;
    case 4 * 8 + 3: launch_panel<4, 3>(f, a, lds, st); break;
    case 4 * 8 + 4: launch_panel<4, 4>(f, a, lds, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool shared_panels(const tree_factors *f)
{
    return f->shared >= kRhsPanel && f->shared % kRhsPanel == 0 && f->ninst == f->shared && panel_tpw(f) > 0;
}

bool panel_route(const tree_factors *f, int active)
{
    return shared_panels(f) && (active < 0 ? f->ninst : active) >= f->panel_min;
}

// On a shared handle the instances are the panel's right-hand sides: group g
// of kRhsPanel instances is one panel starting at instance g*kRhsPanel, with
// the instance strides as right-hand-side strides; the nrhs right-hand sides
// of the call (directions, strides of a) are swept one after the other.
hipError_t launch_sweep_any(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st, int active)
{
    if (!panel_route(f, active)) return launch_sweep_tree(f, a, nrhs, st);
    const InstDesc &I0 = f->inst[0], &I1 = f->inst[1];
    for (int d = 0; d < nrhs; ++d)
        for (int g = 0; g < f->ninst / kRhsPanel; ++g) {
            SweepArgs p = a;
            p.inst = f->d_inst_xu + (long long)g * kRhsPanel;
            // a panel is swept whole while any of its copies is unfinished
            p.done = a.done ? a.done + (long long)g * kRhsPanel * a.done_stride : nullptr;
            p.panel_done = a.done ? 1 : 0;
            p.y = a.y + d * a.y_rs;
            p.xo = a.xo + d * a.xo_rs;
            p.uo = a.uo ? a.uo + d * a.uo_rs : nullptr;
            p.x0 = a.x0 ? a.x0 + d * a.x0_rs : nullptr;
            p.y_rs = I1.y - I0.y;
            p.x0_rs = I1.x0 - I0.x0;
            p.xo_rs = a.dual_out ? I1.y - I0.y : I1.x - I0.x;
            p.uo_rs = I1.u - I0.u;
            p.qhat_rs = I1.x - I0.x;
            p.kbuf_rs = I1.u - I0.u;
            p.chat_rs = I1.chat - I0.chat;   // 0 unless the copies have their own disturbances
            p.c_rs = I1.c - I0.c;
            const hipError_t e = launch_panel_sweep(f, p, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace stotree
