// Learned warm start: a node-wise MLP that predicts the (preconditioned)
// optimal dual of every node from the initial state, the disturbance path
// and the stage, trained on the GPU by the kernels below.  The paper
// warm-starts its solvers from a few iterations of an accelerated gradient
// method (Sec. III-F); the MLP takes that slot, and the solver's own
// residual decides whether its prediction or the cold start is used.
//
// Features of node i (stage t_i) of an instance with initial state x0:
//   [ x0, c_i / c_scale, (mean of c over the path root->i) / c_scale,
//     one-hot(t_i) ]                       (3 nx + N + 1 values; c_0 = 0)
// Network: din -> dh -> dh -> dout (= nx + nu), ReLU, FP32 weights and
// FP32 accumulation.  Parameters are one flat array
//   [W1 (din x dh), b1, W2 (dh x dh), b2, W3 (dh x dout), b3], row-major.
// Outputs map to the node's dual rows (leaves use the first nx; the root's
// state rows are zero because they carry infinite bounds).
#include <cmath>

#include "internal.h"

namespace stotree {

namespace {

constexpr int kTile = 64;    // output tile (rows and columns)
constexpr int kKt = 16;      // reduction tile
constexpr int kGB = 256;     // threads per GEMM block (16 x 16, 4 x 4 outputs each)

// C[m][n] (+)= sum_k opA(m,k) opB(k,n) over k in [k0, k1), with
// opA(m,k) = TA ? A[k*lda+m] : A[m*lda+k], opB(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].
// Epilogue: + bias[n]; ReLU; or multiplication by the gate (G[m][n] > 0).
// blockIdx.z selects a slice of the reduction (partial sums for the weight
// gradients): A and B advance by z*kslice rows of the reduction, C by z*M*N.
template <bool TA, bool TB>
__global__ void __launch_bounds__(kGB) gemm_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                 const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                 int ldc, const float *__restrict__ bias, int relu,
                                                 const float *__restrict__ gate, int ldg, int kslice)
{
    __shared__ float As[kKt][kTile + 4];
    __shared__ float Bs[kKt][kTile + 4];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    int kbeg = 0, kend = K;
    if (kslice > 0) {
        kbeg = blockIdx.z * kslice;
        kend = min(K, kbeg + kslice);
        C += (long long)blockIdx.z * M * ldc;
    }
    float acc[4][4] = {};
    for (int k0 = kbeg; k0 < kend; k0 += kKt) {
        // loads ordered so that consecutive threads read consecutive addresses
        for (int e = threadIdx.x; e < kKt * kTile; e += kGB) {
            const int kk = TA ? e / kTile : e % kKt, mm = TA ? e % kTile : e / kKt;
            const int m = m0 + mm, k = k0 + kk;
            As[kk][mm] = (m < M && k < kend) ? (TA ? A[(long long)k * lda + m] : A[(long long)m * lda + k]) : 0.0f;
        }
        for (int e = threadIdx.x; e < kKt * kTile; e += kGB) {
            const int kk = TB ? e % kKt : e / kTile, nn = TB ? e / kKt : e % kTile;
            const int n = n0 + nn, k = k0 + kk;
            Bs[kk][nn] = (n < N && k < kend) ? (TB ? B[(long long)n * ldb + k] : B[(long long)k * ldb + n]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKt; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty + 16 * i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx + 16 * j;
            if (n >= N) continue;
            float v = acc[i][j];
            if (bias) v += bias[n];
            if (relu) v = fmaxf(v, 0.0f);
            if (gate && !(gate[(long long)m * ldg + n] > 0.0f)) v = 0.0f;
            C[(long long)m * ldc + n] = v;
        }
    }
}

// out[j] = sum_s part[s*n + j] (fixed order); also used for bias gradients
// with part = dH (rows x n).
__global__ void sum_rows_kernel(const float *part, int S, int n, float *out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += part[(long long)k * n + j];
    out[j] = (float)s;
}

// Loss 1/count sum mask (Y - T)^2 and its gradient dY = 2 mask (Y - T)/count.
// Per-block partial sums of the loss and of the mask go to part[2*block].
// Device-side count of the mask: per-block sums (fixed order) into part,
// then one thread forms 1 / max(1, sum).
__global__ void mask_count_kernel(long long n, const float *mask, double *part)
{
    __shared__ double red[256];
    double c = 0.0;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        c += mask[k];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void mask_inverse_kernel(const double *part, int nb, float *inv_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double c = 0.0;
    for (int b = 0; b < nb; ++b) c += part[b];
    inv_out[0] = (float)(1.0 / (c > 1.0 ? c : 1.0));
}

// inv_dev: the inverse count from mask_count_kernel, or null (inv_count given)
__global__ void mse_grad_kernel(long long n, const float *Y, const float *T, const float *mask, float inv_count,
                                const float *inv_dev, float *dY, double *part)
{
    __shared__ double red[2][256];
    double l = 0.0, c = 0.0;
    const float inv = inv_dev ? inv_dev[0] : inv_count;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const float d = Y[k] - T[k];
        const float w = mask[k];
        dY[k] = 2.0f * w * d * inv;
        l += (double)w * d * d;
        c += w;
    }
    red[0][threadIdx.x] = l;
    red[1][threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ void sum_pairs_kernel(const double *part, int nb, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = 0.0, c = 0.0;
    for (int b = 0; b < nb; ++b) { l += part[2 * b]; c += part[2 * b + 1]; }
    out[0] = l;
    out[1] = c;
}

// Adam (Kingma and Ba 2015) with bias correction.
__global__ void adam_kernel(long long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.0f - b1) * gk;
        const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    }
}

struct WarmArgs {
    const InstDesc *inst;
    const int *sp, *anc;
    const double *cvec, *x0;
    int din, dout, Nmax;
    float c_scale;
};

// One thread per (node, feature).
__global__ void features_kernel(WarmArgs a, int b, float *X, long long row0)
{
    const InstDesc I = a.inst[b];
    const int *sp = a.sp + I.sp;
    const int *anc = a.anc + I.sc;  // node-indexed pools share the sc offset
    const long long total = (long long)I.V * a.din;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / a.din), f = (int)(e % a.din);
        int t = 0;
        while (t < I.N && sp[t + 1] <= i) ++t;
        float v = 0.0f;
        if (f < I.nx) {
            v = (float)a.x0[I.x0 + f];
        } else if (f < 2 * I.nx) {
            v = (float)(a.cvec[I.c + (long long)i * I.nx + (f - I.nx)] / a.c_scale);
        } else if (f < 3 * I.nx) {
            const int col = f - 2 * I.nx;
            double s = 0.0;
            for (int j = i; j > 0; j = anc[j]) s += a.cvec[I.c + (long long)j * I.nx + col];
            v = t > 0 ? (float)(s / t / a.c_scale) : 0.0f;
        } else {
            v = (f - 3 * I.nx == t) ? 1.0f : 0.0f;
        }
        X[(row0 + i) * a.din + f] = v;
    }
}

// Y rows (scaled by y_scale) -> dual vector (root state rows 0), and the
// inverse map dual -> target rows with a mask of the rows that exist.
__global__ void scatter_kernel(WarmArgs a, int b, const float *Y, long long row0, double *y, float y_scale)
{
    const InstDesc I = a.inst[b];
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < I.m;
         k += (long long)gridDim.x * blockDim.x) {
        const long long nl = (long long)I.Vnl * (I.nx + I.nu);
        int i, col;
        if (k < nl) { i = (int)(k / (I.nx + I.nu)); col = (int)(k % (I.nx + I.nu)); }
        else { i = I.Vnl + (int)((k - nl) / I.nx); col = (int)((k - nl) % I.nx); }
        const double v = (i == 0 && col < I.nx) ? 0.0 : (double)Y[(row0 + i) * a.dout + col] * y_scale;
        y[I.y + k] = v;
    }
}

__global__ void targets_kernel(WarmArgs a, int b, const double *y, long long row0, float *T, float *mask,
                               float inv_scale)
{
    const InstDesc I = a.inst[b];
    const long long total = (long long)I.V * a.dout;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / a.dout), col = (int)(e % a.dout);
        const int w = i < I.Vnl ? I.nx + I.nu : I.nx;
        float t = 0.0f, mk = 0.0f;
        if (col < w && !(i == 0 && col < I.nx)) {
            const long long o = i < I.Vnl ? (long long)i * (I.nx + I.nu) : (long long)I.Vnl * I.nu + (long long)i * I.nx;
            t = (float)(y[I.y + o + col] * inv_scale);
            mk = 1.0f;
        }
        T[(row0 + i) * a.dout + col] = t;
        mask[(row0 + i) * a.dout + col] = mk;
    }
}

int launch_gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C,
                int ldc, const float *bias, int relu, const float *gate, int ldg, int kslice, int nslices,
                hipStream_t st)
{
    const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile, nslices);
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(kGB), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                           bias, relu, gate, ldg, kslice);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(kGB), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                           bias, relu, gate, ldg, kslice);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(kGB), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                           bias, relu, gate, ldg, kslice);
    else
        return STOTREE_ERR_ARG;
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

struct Layout {
    long long W1, b1, W2, b2, W3, b3, n;
};

Layout layout(int din, int dh, int dout)
{
    Layout L;
    L.W1 = 0;
    L.b1 = L.W1 + (long long)din * dh;
    L.W2 = L.b1 + dh;
    L.b2 = L.W2 + (long long)dh * dh;
    L.W3 = L.b2 + dh;
    L.b3 = L.W3 + (long long)dh * dout;
    L.n = L.b3 + dout;
    return L;
}

// rows per slice of the weight-gradient reductions: a 65,536-row minibatch
// gives 128 slices, so a 128 x 128 weight gradient runs 512 workgroups
// (4,096-row slices left most of the chip idle: 64 workgroups, 0.75 ms each)
constexpr int kSliceRows = 512;

WarmArgs warm_args(const tree_factors *f, const double *x0, float c_scale)
{
    WarmArgs a{};
    a.inst = f->d_inst;
    a.sp = f->d_sp;
    a.anc = f->d_anc;
    a.cvec = f->cvec;
    a.x0 = x0;
    const InstDesc &I = f->inst[0];
    a.din = 3 * I.nx + I.N + 1;
    a.dout = I.nx + I.nu;
    a.Nmax = I.N;
    a.c_scale = c_scale;
    return a;
}

int uniform_instances(const tree_factors *f, const char *who)
{
    for (const InstDesc &I : f->inst)
        if (I.nx != f->inst[0].nx || I.nu != f->inst[0].nu || I.N != f->inst[0].N) {
            set_error(std::string(who) + ": every instance needs the same nx, nu and N");
            return STOTREE_ERR_ARG;
        }
    return STOTREE_OK;
}

}  // namespace

long long mlp_param_count(int din, int dh, int dout) { return layout(din, dh, dout).n; }

int mlp_forward_impl(int rows, int din, int dh, int dout, const float *P, const float *X, float *H, float *Y,
                     hipStream_t st)
{
    const Layout L = layout(din, dh, dout);
    float *H1 = H, *H2 = H + (long long)rows * dh;
    int rc;
    if ((rc = launch_gemm(false, false, rows, dh, din, X, din, P + L.W1, dh, H1, dh, P + L.b1, 1, nullptr, 0, 0, 1, st)))
        return rc;
    if ((rc = launch_gemm(false, false, rows, dh, dh, H1, dh, P + L.W2, dh, H2, dh, P + L.b2, 1, nullptr, 0, 0, 1, st)))
        return rc;
    return launch_gemm(false, false, rows, dout, dh, H2, dh, P + L.W3, dout, Y, dout, P + L.b3, 0, nullptr, 0, 0, 1, st);
}

long long mlp_work_len(int rows, int din, int dh, int dout)
{
    const long long slices = (rows + kSliceRows - 1) / kSliceRows;
    const long long wmax = std::max<long long>((long long)din * dh, std::max<long long>((long long)dh * dh, (long long)dh * dout));
    return 2LL * rows * dh + slices * wmax + rows + slices * std::max(dh, dout);
}

namespace {
// dst[r][:] = src[idx[r]][:] for r < rows (cols floats per row)
__global__ void gather_rows_kernel(long long rows, int cols, const float *src, long long src_rows,
                                   const long long *idx, float *dst, int *bad)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < rows * cols;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / cols;
        const int c = (int)(e - r * cols);
        const long long s = idx[r];
        if (s < 0 || s >= src_rows) {   // an index outside the source: flagged, entry left as is
            *bad = 1;
            continue;
        }
        dst[e] = src[s * cols + c];
    }
}

__global__ void fill_f32_kernel(float *v, long long n, float val)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        v[k] = val;
}

// out[n] = sum over rows of D (rows x n), as ones' D in fixed-order slices.
int colsum(int rows, int n, const float *D, const float *ones, float *part, float *out, hipStream_t st)
{
    const int slices = (rows + kSliceRows - 1) / kSliceRows;
    int rc = launch_gemm(true, false, 1, n, rows, ones, 1, D, n, part, n, nullptr, 0, nullptr, 0, kSliceRows, slices, st);
    if (rc) return rc;
    hipLaunchKernelGGL(sum_rows_kernel, dim3((n + 255) / 256), dim3(256), 0, st, part, slices, n, out);
    return STOTREE_OK;
}
}  // namespace

int mlp_backward_impl(int rows, int din, int dh, int dout, const float *P, const float *X, const float *H,
                      const float *dY, float *G, float *work, hipStream_t st)
{
    const Layout L = layout(din, dh, dout);
    const float *H1 = H, *H2 = H + (long long)rows * dh;
    float *dH2 = work, *dH1 = work + (long long)rows * dh, *part = work + 2LL * rows * dh;
    const int slices = (rows + kSliceRows - 1) / kSliceRows;
    const long long wmax = std::max<long long>((long long)din * dh, std::max<long long>((long long)dh * dh, (long long)dh * dout));
    float *ones = part + (long long)slices * wmax, *partb = ones + rows;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(256), dim3(256), 0, st, ones, (long long)rows, 1.0f);
    int rc;
    // layer 3
    if ((rc = launch_gemm(true, false, dh, dout, rows, H2, dh, dY, dout, part, dout, nullptr, 0, nullptr, 0,
                          kSliceRows, slices, st)))
        return rc;
    hipLaunchKernelGGL(sum_rows_kernel, dim3((dh * dout + 255) / 256), dim3(256), 0, st, part, slices, dh * dout, G + L.W3);
    if ((rc = colsum(rows, dout, dY, ones, partb, G + L.b3, st))) return rc;
    if ((rc = launch_gemm(false, true, rows, dh, dout, dY, dout, P + L.W3, dout, dH2, dh, nullptr, 0, H2, dh, 0, 1, st)))
        return rc;
    // layer 2
    if ((rc = launch_gemm(true, false, dh, dh, rows, H1, dh, dH2, dh, part, dh, nullptr, 0, nullptr, 0, kSliceRows,
                          slices, st)))
        return rc;
    hipLaunchKernelGGL(sum_rows_kernel, dim3((dh * dh + 255) / 256), dim3(256), 0, st, part, slices, dh * dh, G + L.W2);
    if ((rc = colsum(rows, dh, dH2, ones, partb, G + L.b2, st))) return rc;
    if ((rc = launch_gemm(false, true, rows, dh, dh, dH2, dh, P + L.W2, dh, dH1, dh, nullptr, 0, H1, dh, 0, 1, st)))
        return rc;
    // layer 1
    if ((rc = launch_gemm(true, false, din, dh, rows, X, din, dH1, dh, part, dh, nullptr, 0, nullptr, 0, kSliceRows,
                          slices, st)))
        return rc;
    hipLaunchKernelGGL(sum_rows_kernel, dim3((din * dh + 255) / 256), dim3(256), 0, st, part, slices, din * dh, G + L.W1);
    if ((rc = colsum(rows, dh, dH1, ones, partb, G + L.b1, st))) return rc;
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int mse_grad_impl(long long n, const float *Y, const float *T, const float *mask, float inv_count, float *dY,
                  double *loss2, double *part, hipStream_t st)
{
    // 255 blocks: their (loss, count) pairs fill the first 510 of the 512
    // scratch doubles; with inv_count 0 the inverse count, 1 / max(1, sum
    // mask), formed on the device, goes in the 511th
    const int nb = 255;
    float *inv_dev = nullptr;
    if (inv_count == 0.0f) {
        // the per-block counts use the scratch before the loss pairs overwrite it
        inv_dev = reinterpret_cast<float *>(part + 2 * nb);
        hipLaunchKernelGGL(mask_count_kernel, dim3(nb), dim3(256), 0, st, n, mask, part);
        hipLaunchKernelGGL(mask_inverse_kernel, dim3(1), dim3(64), 0, st, part, nb, inv_dev);
    }
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, st, n, Y, T, mask, inv_count, inv_dev, dY, part);
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(64), 0, st, part, nb, loss2);
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int gather_rows_impl(long long rows, int cols, const float *src, long long src_rows, const long long *idx,
                     float *dst, int *bad, hipStream_t st)
{
    const unsigned g = (unsigned)std::min<long long>(2048, (rows * cols + 255) / 256);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(256), 0, st, rows, cols, src, src_rows, idx, dst, bad);
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int adam_impl(long long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
              int step, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(512), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int warm_features_impl(const tree_factors *f, const double *x0, float c_scale, float *X, hipStream_t st)
{
    int rc = uniform_instances(f, "warm_features");
    if (rc) return rc;
    const WarmArgs a = warm_args(f, x0, c_scale);
    long long row = 0;
    for (int b = 0; b < f->ninst; ++b) {
        const InstDesc &I = f->inst[b];
        const unsigned g = (unsigned)std::min<long long>(1024, ((long long)I.V * a.din + 255) / 256);
        hipLaunchKernelGGL(features_kernel, dim3(g), dim3(256), 0, st, a, b, X, row);
        row += I.V;
    }
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int warm_scatter_impl(const tree_factors *f, const float *Y, float y_scale, double *y, hipStream_t st)
{
    int rc = uniform_instances(f, "warm_scatter");
    if (rc) return rc;
    const WarmArgs a = warm_args(f, nullptr, 1.0f);
    long long row = 0;
    for (int b = 0; b < f->ninst; ++b) {
        const InstDesc &I = f->inst[b];
        const unsigned g = (unsigned)std::min<long long>(1024, (I.m + 255) / 256);
        hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, st, a, b, Y, row, y, y_scale);
        row += I.V;
    }
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

int warm_targets_impl(const tree_factors *f, const double *y, float y_scale, float *T, float *mask, hipStream_t st)
{
    int rc = uniform_instances(f, "warm_targets");
    if (rc) return rc;
    const WarmArgs a = warm_args(f, nullptr, 1.0f);
    long long row = 0;
    for (int b = 0; b < f->ninst; ++b) {
        const InstDesc &I = f->inst[b];
        const unsigned g = (unsigned)std::min<long long>(1024, ((long long)I.V * a.dout + 255) / 256);
        hipLaunchKernelGGL(targets_kernel, dim3(g), dim3(256), 0, st, a, b, y, row, T, mask, 1.0f / y_scale);
        row += I.V;
    }
    STOTREE_HIP(hipGetLastError());
    return STOTREE_OK;
}

}  // namespace stotree
