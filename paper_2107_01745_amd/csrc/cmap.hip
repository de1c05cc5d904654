// The constraint map of Sec. II-B around the sweeps: instances whose rows
// are z_i = F x_i + G u_i (non-leaf) and z_j = FN x_j (leaf) keep their
// duals in that row layout, while Algorithms 3 and 4 read a dual in the
// (x, u) layout and write H x there.  Two passes connect them:
//   to_xu    v_i = [F G]' y_i (non-leaf), v_j = FN' y_j (leaf): the term
//            <y, H x> of the inner problem is <v, (x, u)>;
//   from_xu  z_i = [F G] (x_i, u_i), z_j = FN x_j.
// Instances without a map copy the rows unchanged.  Preconditioning scales
// by sqrt(pi) per node, so it commutes with both passes and stays inside the
// sweeps and the solver's vector kernels.
//
// Each thread produces one output row: a dot product of length nc / ncN
// (to_xu) or nx + nu / nx (from_xu) with the instance's matrices, which are
// a few KB and stay in the caches; the passes are bound by streaming the
// two vectors.
#include <algorithm>

#include "internal.h"

namespace stotree {

namespace {

constexpr int kMapBlock = 256;

// Node owning local row r of a layout with rn rows per non-leaf node and rl
// per leaf; sets the row within the node.
__device__ __forceinline__ int row_node(long long r, int Vnl, int rn, int rl, int &within)
{
    const long long nlr = (long long)Vnl * rn;
    if (r < nlr) {
        const int i = (int)(r / rn);
        within = (int)(r - (long long)i * rn);
        return i;
    }
    const long long q = r - nlr;
    const int j = (int)(q / rl);
    within = (int)(q - (long long)j * rl);
    return Vnl + j;
}

// blockIdx.y: instance; blockIdx.z: right-hand side.
__global__ void __launch_bounds__(kMapBlock) to_xu_kernel(const InstDesc *inst, const InstDesc *inst_xu,
                                                          const double *Fm, const double *y, long long y_rs,
                                                          double *v, long long v_rs)
{
    const int b = blockIdx.y;
    const InstDesc I = inst[b];
    const long long oxu = inst_xu[b].y;
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const long long mxu = (long long)I.Vnl * W + (long long)(I.V - I.Vnl) * nx;
    const double *yk = y + blockIdx.z * y_rs + I.y;
    double *vk = v + blockIdx.z * v_rs + oxu;
    for (long long r = blockIdx.x * (long long)kMapBlock + threadIdx.x; r < mxu;
         r += (long long)gridDim.x * kMapBlock) {
        if (!I.cmap) {
            vk[r] = yk[r];
            continue;
        }
        int c;
        const int i = row_node(r, I.Vnl, W, nx, c);
        double s = 0.0;
        if (i < I.Vnl) {
            // column c of [F G]: F[a][c] for c < nx, G[a][c - nx] otherwise
            const double *M = c < nx ? Fm + I.Fo + c : Fm + I.Fo + (long long)I.nc * nx + (c - nx);
            const int ld = c < nx ? nx : nu;
            const double *yi = yk + (long long)i * I.nc;
            for (int a = 0; a < I.nc; ++a) s += M[(long long)a * ld] * yi[a];
        } else {
            const double *M = Fm + I.Fo + (long long)I.nc * W + c;
            const double *yj = yk + (long long)I.Vnl * I.nc + (long long)(i - I.Vnl) * I.ncN;
            for (int a = 0; a < I.ncN; ++a) s += M[(long long)a * nx] * yj[a];
        }
        vk[r] = s;
    }
}

__global__ void __launch_bounds__(kMapBlock) from_xu_kernel(const InstDesc *inst, const InstDesc *inst_xu,
                                                            const double *Fm, const double *xu, long long x_rs,
                                                            double *z, long long z_rs)
{
    const int b = blockIdx.y;
    const InstDesc I = inst[b];
    const long long oxu = inst_xu[b].y;
    const int nx = I.nx, nu = I.nu, W = nx + nu;
    const double *xk = xu + blockIdx.z * x_rs + oxu;
    double *zk = z + blockIdx.z * z_rs + I.y;
    for (long long r = blockIdx.x * (long long)kMapBlock + threadIdx.x; r < I.m;
         r += (long long)gridDim.x * kMapBlock) {
        if (!I.cmap) {
            zk[r] = xk[r];
            continue;
        }
        int a;
        const int i = row_node(r, I.Vnl, I.nc, I.ncN, a);
        double s = 0.0;
        if (i < I.Vnl) {
            const double *Fr = Fm + I.Fo + (long long)a * nx;
            const double *Gr = Fm + I.Fo + (long long)I.nc * nx + (long long)a * nu;
            const double *xi = xk + (long long)i * W;
            for (int c = 0; c < nx; ++c) s += Fr[c] * xi[c];
            for (int c = 0; c < nu; ++c) s += Gr[c] * xi[nx + c];
        } else {
            const double *Fr = Fm + I.Fo + (long long)I.nc * W + (long long)a * nx;
            const double *xj = xk + (long long)I.Vnl * W + (long long)(i - I.Vnl) * nx;
            for (int c = 0; c < nx; ++c) s += Fr[c] * xj[c];
        }
        zk[r] = s;
    }
}

dim3 map_grid(const tree_factors *f, int nrhs)
{
    long long most = 1;
    for (const InstDesc &I : f->inst)
        most = std::max(most, std::max<long long>(I.m, (long long)I.Vnl * (I.nx + I.nu) + (long long)(I.V - I.Vnl) * I.nx));
    const unsigned gx = (unsigned)std::min<long long>(2048, (most + kMapBlock - 1) / kMapBlock);
    return dim3(gx, (unsigned)f->ninst, (unsigned)nrhs);
}

}  // namespace

hipError_t map_to_xu(const tree_factors *f, const double *y, long long y_rs, double *out, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(to_xu_kernel, map_grid(f, nrhs), dim3(kMapBlock), 0, st, f->d_inst, f->d_inst_xu, f->Fm,
                       y, y_rs, out, f->mxu_tot);
    return hipGetLastError();
}

hipError_t map_from_xu(const tree_factors *f, const double *xu, double *out, long long o_rs, int nrhs,
                       hipStream_t st)
{
    hipLaunchKernelGGL(from_xu_kernel, map_grid(f, nrhs), dim3(kMapBlock), 0, st, f->d_inst, f->d_inst_xu,
                       f->Fm, xu, f->mxu_tot, out, o_rs);
    return hipGetLastError();
}

// dual_grad on a handle with a constraint map: the constraint-layout duals
// go through to_xu into the handle's (x, u)-layout buffer, then the sweeps.
int dual_grad_mapped(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                     double *u, hipStream_t st)
{
    const long long need = (long long)nrhs * f->mxu_tot;
    if (f->map_ws_len < need) {
        if (f->map_ws) {
            STOTREE_HIP(hipStreamSynchronize(st));
            (void)hipFree(f->map_ws);
            f->bytes -= (size_t)f->map_ws_len * sizeof(double);
        }
        f->map_ws = nullptr;
        f->map_ws_len = 0;
        STOTREE_HIP(hipMalloc(&f->map_ws, sizeof(double) * (size_t)need));
        f->map_ws_len = need;
        f->bytes += (size_t)need * sizeof(double);
    }
    STOTREE_HIP(map_to_xu(f, y, f->m_tot, f->map_ws, nrhs, st));
    return enqueue_dual_grad(f, x0, f->map_ws, homogeneous, nrhs, x, u, st);
}

}  // namespace stotree
