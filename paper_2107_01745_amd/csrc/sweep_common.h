// Device helpers shared by the sweep kernels (sweep.hip, sweep_mfma.hip):
// addressing of the per-node vectors of a (possibly batched) handle.
#pragma once

#include "internal.h"

namespace stotree {
namespace dev {

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

}  // namespace dev
}  // namespace stotree
