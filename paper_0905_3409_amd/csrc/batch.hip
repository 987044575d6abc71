// Many independent 2D grids with sine stream-function fields advanced by one
// persistent launch per step. The work list is a flat array of tiles over all
// problems; XCD x owns a contiguous band of it (so halo rows stay in its L2)
// and the blocks on that XCD stride through the band. A tile is 4 waves; a
// wave covers WX x (64/WX) nodes with WX = 64, 32 or 16 chosen per problem,
// so narrow grids do not leave most lanes idle. Per-node arithmetic is the
// single-grid kernel's (stream_node), so batched and single runs agree bit
// for bit.
#include "stream2d.h"

namespace gals {

// FP64 tables of every problem: block (x, p) fills entries of problem p.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_tables(const BatchProb<double> *__restrict__ probs,
                                                         T *__restrict__ tab)
{
    const BatchProb<double> &P = probs[blockIdx.y];
    const int id = int(blockIdx.x) * kBlock + int(threadIdx.x);
    T *col = tab + P.tab;
    T *row = col + int64_t(P.g.n[0]) * kJet;
    stream_table_entry(P.g, P.S, id, col, row);
}

template <typename T, int MIX, bool TAYLOR, unsigned WX>
__device__ __forceinline__ void batch_tile(const BatchProb<T> &P, unsigned local, const Stage<T> &st,
                                           double dt, const T *__restrict__ tab,
                                           const T *__restrict__ in, T *__restrict__ out)
{
    constexpr unsigned WY = 64u / WX;  // rows per wave
    const unsigned tx = local % P.tiles_x, ty = local / P.tiles_x;
    const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const int i = int(tx * WX + lane % WX);
    int j = int(ty * 4u * WY + wave * WY + lane / WX);
    if constexpr (WY == 1) j = __builtin_amdgcn_readfirstlane(j);
    const Geom &g = P.g;
    if (j >= g.n[1] || i >= g.n[0]) return;
    const T *col = tab + P.tab;
    const T *row = col + int64_t(g.n[0]) * kJet;
    const T *phi = in + P.off;
    T *po = out + P.off;
    stream_node<T, MIX, TAYLOR>(g, P, st, dt, col + int64_t(i) * kJet, row + int64_t(j) * kJet,
                                plane_rsrc(phi, g.plane), plane_rsrc(phi + g.plane, g.plane),
                                plane_rsrc(phi + 2 * g.plane, g.plane), po, po + g.plane,
                                po + 2 * g.plane, i, j);
}

template <typename T, int MIX, bool TAYLOR>
__global__ __launch_bounds__(kBlock) void k_batch_step(const BatchProb<T> *__restrict__ probs,
                                                       const TileRef *__restrict__ tiles,
                                                       unsigned ntiles, Stage<T> st, double dt,
                                                       const T *__restrict__ tab,
                                                       const T *__restrict__ in,
                                                       T *__restrict__ out)
{
    const unsigned xcd = blockIdx.x % 8u, lb = blockIdx.x / 8u, nb = gridDim.x / 8u;
    const unsigned per = (ntiles + 7u) / 8u;
    const unsigned t0 = xcd * per;
    const unsigned t1 = t0 + per < ntiles ? t0 + per : ntiles;
    for (unsigned t = t0 + lb; t < t1; t += nb) {
        const TileRef tr = tiles[t];
        const BatchProb<T> &P = probs[tr.prob];
        if (P.wx == 64u)
            batch_tile<T, MIX, TAYLOR, 64u>(P, tr.local, st, dt, tab, in, out);
        else if (P.wx == 32u)
            batch_tile<T, MIX, TAYLOR, 32u>(P, tr.local, st, dt, tab, in, out);
        else
            batch_tile<T, MIX, TAYLOR, 16u>(P, tr.local, st, dt, tab, in, out);
    }
}

// Copy the valid nodes of every problem (phi, psi_x, psi_y) from in to out.
template <typename T, unsigned WX>
__device__ __forceinline__ void copy_tile(const BatchProb<T> &P, unsigned local,
                                          const T *__restrict__ in, T *__restrict__ out)
{
    constexpr unsigned WY = 64u / WX;
    const unsigned tx = local % P.tiles_x, ty = local / P.tiles_x;
    const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const int i = int(tx * WX + lane % WX);
    const int j = int(ty * 4u * WY + wave * WY + lane / WX);
    if (j >= P.g.n[1] || i >= P.g.n[0]) return;
    const int64_t o = P.off + int64_t(j) * P.g.pitch + i;
    out[o] = in[o];
    out[o + P.g.plane] = in[o + P.g.plane];
    out[o + 2 * P.g.plane] = in[o + 2 * P.g.plane];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_copy(const BatchProb<T> *__restrict__ probs,
                                                       const TileRef *__restrict__ tiles,
                                                       unsigned ntiles, const T *__restrict__ in,
                                                       T *__restrict__ out)
{
    for (unsigned t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const BatchProb<T> &P = probs[tr.prob];
        if (P.wx == 64u) copy_tile<T, 64u>(P, tr.local, in, out);
        else if (P.wx == 32u) copy_tile<T, 32u>(P, tr.local, in, out);
        else copy_tile<T, 16u>(P, tr.local, in, out);
    }
}

hipError_t launch_batch_tables(int prec, const void *probs_f64, int nprob, int max_entries,
                               void *tab, hipStream_t s)
{
    const dim3 grid(unsigned((max_entries + kBlock - 1) / kBlock), unsigned(nprob));
    if (prec == GALS_F32)
        hipLaunchKernelGGL(k_batch_tables<float>, grid, dim3(kBlock), 0, s,
                           (const BatchProb<double> *)probs_f64, (float *)tab);
    else
        hipLaunchKernelGGL(k_batch_tables<double>, grid, dim3(kBlock), 0, s,
                           (const BatchProb<double> *)probs_f64, (double *)tab);
    return hipGetLastError();
}

hipError_t launch_batch_step(int prec, int mixed, const void *probs, const TileRef *tiles,
                             unsigned ntiles, double dt, double c1, double c2, double c3,
                             const void *tab, const void *in, void *out, unsigned blocks,
                             hipStream_t s)
{
    if (prec == GALS_F32) {
        const Stage<float> st{float(c1), float(c2), float(c3)};
        if (mixed == GALS_MIXED_ZERO)
            hipLaunchKernelGGL((k_batch_step<float, GALS_MIXED_ZERO, true>), dim3(blocks),
                               dim3(kBlock), 0, s, (const BatchProb<float> *)probs, tiles, ntiles,
                               st, dt, (const float *)tab, (const float *)in, (float *)out);
        else
            hipLaunchKernelGGL((k_batch_step<float, GALS_MIXED_CENTRAL, true>), dim3(blocks),
                               dim3(kBlock), 0, s, (const BatchProb<float> *)probs, tiles, ntiles,
                               st, dt, (const float *)tab, (const float *)in, (float *)out);
    } else {
        const Stage<double> st{c1, c2, c3};
        if (mixed == GALS_MIXED_ZERO)
            hipLaunchKernelGGL((k_batch_step<double, GALS_MIXED_ZERO, false>), dim3(blocks),
                               dim3(kBlock), 0, s, (const BatchProb<double> *)probs, tiles,
                               ntiles, st, dt, (const double *)tab, (const double *)in,
                               (double *)out);
        else
            hipLaunchKernelGGL((k_batch_step<double, GALS_MIXED_CENTRAL, false>), dim3(blocks),
                               dim3(kBlock), 0, s, (const BatchProb<double> *)probs, tiles,
                               ntiles, st, dt, (const double *)tab, (const double *)in,
                               (double *)out);
    }
    return hipGetLastError();
}

// Blocks of the step kernel that fit on one CU at once (its register use
// decides); the persistent grid is sized to exactly that so every block is
// resident from the start and the static tile shares finish together.
hipError_t batch_step_blocks_per_cu(int prec, int mixed, int *blocks)
{
    *blocks = 0;
    if (prec == GALS_F32)
        return mixed == GALS_MIXED_ZERO
                   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                         blocks, k_batch_step<float, GALS_MIXED_ZERO, true>, kBlock, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                         blocks, k_batch_step<float, GALS_MIXED_CENTRAL, true>, kBlock, 0);
    return mixed == GALS_MIXED_ZERO
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks, k_batch_step<double, GALS_MIXED_ZERO, false>, kBlock, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks, k_batch_step<double, GALS_MIXED_CENTRAL, false>, kBlock, 0);
}

hipError_t launch_batch_copy(int prec, const void *probs, const TileRef *tiles, unsigned ntiles,
                             const void *in, void *out, unsigned blocks, hipStream_t s)
{
    if (prec == GALS_F32)
        hipLaunchKernelGGL(k_batch_copy<float>, dim3(blocks), dim3(kBlock), 0, s,
                           (const BatchProb<float> *)probs, tiles, ntiles, (const float *)in,
                           (float *)out);
    else
        hipLaunchKernelGGL(k_batch_copy<double>, dim3(blocks), dim3(kBlock), 0, s,
                           (const BatchProb<double> *)probs, tiles, ntiles, (const double *)in,
                           (double *)out);
    return hipGetLastError();
}

}  // namespace gals
