// Deterministic block reductions shared by the reduction kernels.
#pragma once

#include "gals_internal.h"
#include "velocity.h"

namespace gals {

// ---------------------------------------------------------------------------
// Deterministic reductions: a fixed grid of kRedBlocks blocks walks the nodes
// with a fixed stride; each block reduces its slots (wave64 shuffles, then the
// four waves in order) to one partial; a single block then folds the partials
// in a fixed order. Bit b of maxmask selects max (set) or sum (clear) for
// slot b. ACC adds the block's result to out instead of storing it (a block
// then owns its out slots across launches).
// ---------------------------------------------------------------------------
template <int NS, bool ACC = false>
__device__ __forceinline__ void block_reduce(double *acc, unsigned maxmask, double *out)
{
    __shared__ double sm[kBlock / 64][NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        double a = acc[s];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(a, off, 64);
            a = ((maxmask >> s) & 1) ? fmax(a, o) : a + o;
        }
        acc[s] = a;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NS; s++) sm[w][s] = acc[s];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NS; s++) {
            double a = sm[0][s];
            for (int k = 1; k < kBlock / 64; k++)
                a = ((maxmask >> s) & 1) ? fmax(a, sm[k][s]) : a + sm[k][s];
            out[s] = ACC ? out[s] + a : a;
        }
    }
}

// Fold the per-block partials (kRedSlots apart) in a fixed order.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_fold(const double *__restrict__ partials, int nparts,
                                                 unsigned maxmask, double *__restrict__ out)
{
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) acc[s] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const double v = partials[int64_t(b) * kRedSlots + s];
            acc[s] = ((maxmask >> s) & 1) ? fmax(acc[s], v) : acc[s] + v;
        }
    }
    block_reduce<NS>(acc, maxmask, out);
}

// Smoothed Heaviside of the shape error, volume and loss diagnostics:
// 0 for s < -eps, 1 for s > eps, (1 + s/eps + sin(pi s/eps)/pi)/2 between;
// and its derivative (1 + cos(pi s/eps)) / (2 eps) on [-eps, eps].
__device__ __forceinline__ double heaviside_eps(double s, double eps)
{
    if (s < -eps) return 0.0;
    if (s > eps) return 1.0;
    return 0.5 * (1.0 + s / eps + sin(kPi * s / eps) / kPi);
}

__device__ __forceinline__ double heaviside_eps_deriv(double s, double eps)
{
    if (s < -eps || s > eps) return 0.0;
    return 0.5 * (1.0 + cos(kPi * s / eps)) / eps;
}

}  // namespace gals
