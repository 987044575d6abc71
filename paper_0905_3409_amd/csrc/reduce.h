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

// Sums of 16 slots over the block in a fixed order, with no LDS traffic
// inside a wave: the wave halves its slots twice (lane pairs l, l ^ 32, then
// l, l ^ 16, swap the halves they do not keep and add: one permlane-swap
// instruction per 32-bit word), leaving each lane 4 slots shared by its
// 16-lane row; DPP moves within the row (lane i with i ^ 8, with 7 - i in
// its half-row, then across the quad) finish the row sums; the four waves'
// sums are then added in order. After a swap of (a, b) = (slot s, slot
// s + h) both registers of a lane hold the same slot, whichever half the
// lane keeps; the slot is found by swapping the slot numbers the same way.
// Every lane of a group adds the same two values (in either order), so all
// of them hold identical sums.
template <int O>
__device__ __forceinline__ void lane_swap(unsigned &a, unsigned &b)
{
    if constexpr (O == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int O>
__device__ __forceinline__ void lane_swap(double &a, double &b)
{
    const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
    unsigned alo = unsigned(ua), ahi = unsigned(ua >> 32), blo = unsigned(ub), bhi = unsigned(ub >> 32);
    lane_swap<O>(alo, blo);
    lane_swap<O>(ahi, bhi);
    a = __builtin_bit_cast(double, uint64_t(alo) | (uint64_t(ahi) << 32));
    b = __builtin_bit_cast(double, uint64_t(blo) | (uint64_t(bhi) << 32));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(u)), CTRL, 0xF, 0xF, false));
    const unsigned hi =
        unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(u >> 32)), CTRL, 0xF, 0xF, false));
    return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}

__device__ __forceinline__ double row_sum(double v)
{
    v += dpp_move<0x128>(v);  // row_ror:8: lane i and i ^ 8
    v += dpp_move<0x141>(v);  // row_half_mirror: i and 7 - i within 8 lanes
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    return v;
}

// Minimum over the wave, in every lane: the row tree of row_sum, then the
// pairs across the 16-lane rows and the 32-lane halves by permlane swaps of
// two copies (a lane then holds its own value and its partner's).
__device__ __forceinline__ int wave_min(int v)
{
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
    unsigned a = unsigned(v), b = unsigned(v);
    lane_swap<16>(a, b);
    v = min(int(a), int(b));
    a = unsigned(v);
    b = unsigned(v);
    lane_swap<32>(a, b);
    return min(int(a), int(b));
}

template <bool ACC = false>
__device__ __forceinline__ void block_sum16(double *acc, double *out)
{
    __shared__ double sm[kBlock / 64][16];
#pragma unroll
    for (int s = 0; s < 8; s++) {
        double a = acc[s], b = acc[s + 8];
        lane_swap<32>(a, b);
        acc[s] = a + b;
    }
#pragma unroll
    for (int s = 0; s < 4; s++) {
        double a = acc[s], b = acc[s + 4];
        lane_swap<16>(a, b);
        acc[s] = a + b;
    }
    unsigned s0 = 0, s1 = 8, r0 = 0, r1 = 4;
    lane_swap<32>(s0, s1);
    lane_swap<16>(r0, r1);
    const int base = int(s0 + r0);  // this lane's first slot
    double tot[4];
#pragma unroll
    for (int s = 0; s < 4; s++) tot[s] = row_sum(acc[s]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if ((lane & 15) == 0) {
#pragma unroll
        for (int s = 0; s < 4; s++) sm[w][base + s] = tot[s];
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        double v = sm[0][threadIdx.x];
        for (int k = 1; k < kBlock / 64; k++) v += sm[k][threadIdx.x];
        out[threadIdx.x] = ACC ? out[threadIdx.x] + v : v;
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
