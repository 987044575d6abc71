// Many independent 2D grids with sine stream-function fields advanced by one
// launch per step. The work list is a flat array of tiles over all problems,
// one block per tile; XCD x takes a contiguous band of it (so the halo rows a
// tile gathers were just fetched into the same L2 by its neighbours). Tiles
// cost unevenly (small grids leave the Taylor range, ragged tiles), and the
// hardware dispatcher balances them as blocks retire: 306 us per step on 512
// grids, against 344 us for 8 persistent blocks per CU striding through the
// bands (their last blocks finished well after the mean) and no better with
// per-range atomic tile queues.
// A tile is 4 waves. A wave covers WX x (64/WX) nodes with WX = 64, 32 or 16,
// or, in the row-major shape, 64 consecutive nodes of the grid in row-major
// order (no lanes lost to a ragged row end). With 64 x 1 waves, a ragged last
// group of up to kTailPack columns is packed row-major into tiles of its
// own (template value 1), instead of a mostly idle wave per row. Per-node arithmetic is the
// single-grid kernel's (stream_node), so batched and single runs agree bit
// for bit.
#include "batch_shape.h"
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

// Node (i, j) of lane `lane` in wave `wave` of tile `local`; false if the
// lane has no node.
template <unsigned WX, class P>
__device__ __forceinline__ bool tile_node(const P &p, unsigned local, unsigned wave,
                                          unsigned lane, int &i, int &j)
{
    const Geom &g = p.g;
    if constexpr (WX == 0u) {
        // row-major: node k = j n0 + i; j from an FP32 estimate of k / n0
        // corrected once (the estimate is off by less than one for every
        // k < 2^31 with j < 2^20)
        const unsigned k = local * 256u + wave * 64u + lane;
        if (k >= unsigned(g.nodes)) return false;
        int jj = int(float(k) * p.inv_n0);
        int ii = int(k) - jj * g.n[0];
        if (ii < 0) { jj--; ii += g.n[0]; }
        else if (ii >= g.n[0]) { jj++; ii -= g.n[0]; }
        i = ii;
        j = jj;
        return true;
    } else if constexpr (WX == 1u) {
        // the packed tail strip of a 64 x 1 grid: its tail columns of every
        // row, row-major (node k = j tail + c at column n0 - tail + c), the
        // same division as above
        const unsigned k = (local & ~kTailTile) * 256u + wave * 64u + lane;
        const int t = int(packed_tail(p));
        if (k >= unsigned(t) * unsigned(g.n[1])) return false;
        int jj = int(float(k) * (1.0f / float(t)));
        int cc = int(k) - jj * t;
        if (cc < 0) { jj--; cc += t; }
        else if (cc >= t) { jj++; cc -= t; }
        i = g.n[0] - t + cc;
        j = jj;
        return true;
    } else {
        constexpr unsigned WY = 64u / WX;  // rows per wave
        const unsigned sh = tile_bits(p);
        const unsigned tx = local & ((1u << sh) - 1u), ty = local >> sh;
        i = int(tx * WX + lane % WX);
        j = int(ty * 4u * WY + wave * WY + lane / WX);
        if constexpr (WY == 1) j = __builtin_amdgcn_readfirstlane(j);
        return j < g.n[1] && i < g.n[0];
    }
}

template <typename T, int MIX, bool TAYLOR, unsigned WX>
__device__ __forceinline__ void batch_tile(const BatchProb<T> &P, unsigned local, const Stage<T> &st,
                                           double dt, const T *__restrict__ tab,
                                           const T *__restrict__ in, T *__restrict__ out)
{
    int i, j;
    if (!tile_node<WX>(P, local, threadIdx.x >> 6, threadIdx.x & 63u, i, j)) return;
    const Geom &g = P.g;
    const T *col = tab + P.tab;
    const T *row = col + int64_t(g.n[0]) * kJet;
    const T *phi = in + P.off;
    T *po = out + P.off;
    stream_node<T, MIX, TAYLOR>(g, P, st, dt, col + int64_t(i) * kJet, row + int64_t(j) * kJet,
                                phi, phi + g.plane, phi + 2 * g.plane, po, po + g.plane,
                                po + 2 * g.plane, i, j);
}

template <typename T, int MIX, bool TAYLOR>
// Eight waves per SIMD in FP32 (at most 64 VGPRs, no spills; the default 73
// left room for seven blocks per CU).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? 8 : 1))) void k_batch_step(const BatchProb<T> *__restrict__ probs,
                                                       const TileRef *__restrict__ tiles,
                                                       unsigned ntiles, Stage<T> st, double dt,
                                                       const T *__restrict__ tab,
                                                       const T *__restrict__ in,
                                                       T *__restrict__ out)
{
    // grid: 8 ceil(ntiles / 8) blocks; block b is tile lb of XCD b % 8's band
    const unsigned xcd = blockIdx.x % 8u, lb = blockIdx.x / 8u;
    const unsigned per = (ntiles + 7u) / 8u;
    const unsigned t = xcd * per + lb;
    if (lb >= per || t >= ntiles) return;
    const TileRef tr = tiles[t];
    const BatchProb<T> &P = probs[tr.prob];
    if (tr.local & kTailTile)
        batch_tile<T, MIX, TAYLOR, 1u>(P, tr.local, st, dt, tab, in, out);
    else if (P.wx == 64u)
        batch_tile<T, MIX, TAYLOR, 64u>(P, tr.local, st, dt, tab, in, out);
    else if (P.wx == 32u)
        batch_tile<T, MIX, TAYLOR, 32u>(P, tr.local, st, dt, tab, in, out);
    else if (P.wx == 16u)
        batch_tile<T, MIX, TAYLOR, 16u>(P, tr.local, st, dt, tab, in, out);
    else
        batch_tile<T, MIX, TAYLOR, 0u>(P, tr.local, st, dt, tab, in, out);
}

// Copy the valid nodes of every problem (phi, psi_x, psi_y) from in to out.
template <typename T, unsigned WX>
__device__ __forceinline__ void copy_tile(const BatchProb<T> &P, unsigned local,
                                          const T *__restrict__ in, T *__restrict__ out)
{
    int i, j;
    if (!tile_node<WX>(P, local, threadIdx.x >> 6, threadIdx.x & 63u, i, j)) return;
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
        if (tr.local & kTailTile) copy_tile<T, 1u>(P, tr.local, in, out);
        else if (P.wx == 64u) copy_tile<T, 64u>(P, tr.local, in, out);
        else if (P.wx == 32u) copy_tile<T, 32u>(P, tr.local, in, out);
        else if (P.wx == 16u) copy_tile<T, 16u>(P, tr.local, in, out);
        else copy_tile<T, 0u>(P, tr.local, in, out);
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
                             const void *tab, const void *in, void *out, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    const unsigned blocks = (ntiles + 7u) / 8u * 8u;  // one per tile, bands of 8 XCDs
    if (prec == GALS_F32) {
        const Stage<float> st = make_stage<float>(dt, c1, c2, c3);
        auto kern = mixed == GALS_MIXED_ZERO   ? k_batch_step<float, GALS_MIXED_ZERO, true>
                    : mixed == GALS_MIXED_CELL ? k_batch_step<float, GALS_MIXED_CELL, true>
                                               : k_batch_step<float, GALS_MIXED_CENTRAL, true>;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s,
                           (const BatchProb<float> *)probs, tiles, ntiles, st, dt,
                           (const float *)tab, (const float *)in, (float *)out);
    } else {
        const Stage<double> st = make_stage<double>(dt, c1, c2, c3);
        auto kern = mixed == GALS_MIXED_ZERO   ? k_batch_step<double, GALS_MIXED_ZERO, false>
                    : mixed == GALS_MIXED_CELL ? k_batch_step<double, GALS_MIXED_CELL, false>
                                               : k_batch_step<double, GALS_MIXED_CENTRAL, false>;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s,
                           (const BatchProb<double> *)probs, tiles, ntiles, st, dt,
                           (const double *)tab, (const double *)in, (double *)out);
    }
    return hipGetLastError();
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
