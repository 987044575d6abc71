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

}  // namespace gals
