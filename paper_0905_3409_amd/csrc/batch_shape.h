// Wave shapes of the batched step that the host's tile list and the kernel
// must agree on.
#pragma once

#include "gals_internal.h"

namespace gals {

// With 64 x 1 waves, a ragged last column group of at most kTailPack nodes
// per row is packed row-major into tiles of its own, after the full 64-wide
// columns' tiles: a packed wave, with its row per lane, costs about 1.3 row
// waves, so packing pays while tail / 64 x 1.3 < 1.
constexpr unsigned kTailPack = 48;

// Columns of problem P in the packed tail strip (0: none).
template <typename P>
__host__ __device__ inline unsigned packed_tail(const P &p)
{
    const unsigned rag = unsigned(p.g.n[0]) % 64u;
    return p.wx == 64u && rag <= kTailPack ? rag : 0u;
}

// Tiles of the full columns of problem P (64 x 1 waves: 4 rows per tile);
// the host sets tiles_x to the full 64-wide column groups when it packs.
template <typename P>
__host__ __device__ inline unsigned body_tiles(const P &p)
{
    return p.tiles_x * ((unsigned(p.g.n[1]) + 3u) / 4u);
}

// The tile index a work-list entry carries (TileRef::local). Rectangular
// shapes: the tile's column tx in the low tile_bits bits and its row group
// ty above them, so the kernel splits it with a mask and a shift rather than
// a division by tiles_x. Packed tail tiles: kTailTile | their index in the
// strip. Row-major shape: the tile's index.
constexpr unsigned kTailTile = 0x80000000u;

template <typename P>
__host__ __device__ inline unsigned tile_bits(const P &p)
{
    // bits of tiles_x - 1 (0 for a single tile column)
#ifdef __HIP_DEVICE_COMPILE__
    return p.tiles_x > 1u ? 32u - unsigned(__clz(int(p.tiles_x - 1u))) : 0u;
#else
    return p.tiles_x > 1u ? 32u - unsigned(__builtin_clz(p.tiles_x - 1u)) : 0u;
#endif
}

}  // namespace gals
