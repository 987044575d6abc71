// GA-CIR step kernels for gfx950: one thread per grid node, wave64, fused
// trace + split + gather + Hermite + gradient update (superconsistent, or
// Heun's method along the characteristic).
//
// Each node reads only the old state (never updated in place) and writes its
// new phi, psi with coalesced SoA stores. The affine 2D step stages its
// tile of the old state through LDS and gathers on-tile feet from there; the
// other steps gather departure cells through the cache hierarchy. Feet any
// number of cells away are gathered from global memory, so every CFL number
// is handled.
#include <type_traits>

#include "stream2d.h"

namespace gals {

// Node index -> (i, j[, k]) with 32-bit arithmetic (the host caps the node
// count below 2^31).
template <typename T, int KIND, int MIX, int PSI>
__global__ __launch_bounds__(kBlock) void k_step2d(Geom g, Vel<T> p, Stage<T> st, double dt,
                                                   const T *__restrict__ phi,
                                                   const T *__restrict__ grad,
                                                   T *__restrict__ phi_o, T *__restrict__ grad_o)
{
    unsigned blk;
    if (!xcd_block(unsigned((g.nodes + kBlock - 1) / kBlock), blk)) return;
    const unsigned id = blk * kBlock + threadIdx.x;
    if (id >= unsigned(g.nodes)) return;
    unsigned ri;
    const int j = int(udiv_magic(id, unsigned(g.n[0]), g.n_magic[0], ri));
    const int i = int(ri);
    const T *gx = grad, *gy = grad + g.plane;

    const double x[2] = {node_coord(g.lo[0], i, g.h[0]), node_coord(g.lo[1], j, g.h[1])};
    double X[2];
    T J[4];  // superconsistent Jacobian, or (Heun) grad v at the node
    trace<T, 2, KIND, PSI == GALS_PSI_SUPERCONSISTENT>(p, st, dt, x, X, J);
    const unsigned out = project_foot<2>(g, X);

    int cell[2];
    double xi[2];
    split<2>(g, X, cell, xi);

    T d[4][4];
    gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(gx, g.plane), plane_rsrc(gy, g.plane),
                     cell[0], cell[1], d);
    Basis<T> bx, by;
    basis<T, false>(T(xi[0]), geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
    basis<T, false>(T(xi[1]), geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
    T H, Hx, Hy;
    hermite2d(d, bx, by, H, Hx, Hy);
    if (out & 1u) Hx = T(0);
    if (out & 2u) Hy = T(0);

    const unsigned o = unsigned(j) * unsigned(g.pitch) + unsigned(i);
    pstore(phi_o, o, H);
    if constexpr (PSI == GALS_PSI_HEUN) {
        T vf[2], Af[4], ps[2];
        const T gH[2] = {Hx, Hy};
        velocity<T, 2, KIND>(p, X, st.c2, vf, Af);
        heun_gradient<T, 2>(Af, J, T(dt), gH, ps);
        pstore(grad_o, o, ps[0]);
        pstore(grad_o + g.plane, o, ps[1]);
    } else {
        pstore(grad_o, o, J[0] * Hx + J[2] * Hy);
        pstore(grad_o + g.plane, o, J[1] * Hx + J[3] * Hy);
    }
}

// ---------------------------------------------------------------------------
// LDS staging of the old state (used by the affine 2D step below). A block
// owns a tile of 64 x TY nodes (four waves, each a row of 64 nodes, TY / 4
// row groups) and stages phi, psi_x, psi_y of the tile and a halo of kHaloX
// columns and kHaloY rows around it: the scheme's stencil is one cell, so a
// foot less than a cell from its node (CFL < 1) reads only the node's
// neighbours, and the cross derivative (A) one column more on each side. The
// staging loads are coalesced and do not depend on the trace, so they are
// issued first and their latency hides behind it. A foot whose stencil leaves
// the staged region (CFL > 1 somewhere) gathers from global memory instead,
// lane by lane, so any CFL number is still handled.
// ---------------------------------------------------------------------------
constexpr int kHaloX = 2, kHaloY = 1;

template <int TY>
struct StageTile {
    static constexpr int W = 64 + 2 * kHaloX;  // staged columns
    static constexpr int H = TY + 2 * kHaloY;  // staged rows
    static constexpr int N = W * H;
    static constexpr int PER = (N + kBlock - 1) / kBlock;  // staged values per thread
};

// The staging of one block's tile: coalesced loads of phi, psi_x, psi_y over
// the tile and its halo into registers (issued before the foot is computed),
// then into LDS. Thread t stages the flattened tile's entries t, t + 256, ...
// Positions outside the grid load nothing (their offset is past the plane:
// the buffer load returns 0) and are never read. (Staging whole rows per
// wave, with one address add per load, cut the vector instructions by 3 % but
// cost FP64 one wave per SIMD and measured no faster in FP32.)
template <typename T, int TY>
struct TileStager {
    using S = StageTile<TY>;
    T sv[3][S::PER];

    __device__ __forceinline__ void load(const Geom &g, const T *phi, const T *gx, const T *gy,
                                         int cx0, int ry0)
    {
        const Rsrc r0 = plane_rsrc(phi, g.plane), r1 = plane_rsrc(gx, g.plane),
                   r2 = plane_rsrc(gy, g.plane);
        const unsigned past = unsigned(g.plane);
        const int tid = int(threadIdx.y) * 64 + int(threadIdx.x);
#pragma unroll
        for (int k = 0; k < S::PER; k++) {
            const int f = tid + k * kBlock;
            const int row = ry0 + f / S::W, col = cx0 + f % S::W;
            const bool in = f < S::N && row >= 0 && row < g.n[1] && col >= 0 && col < g.n[0];
            const unsigned off = in ? unsigned(row) * unsigned(g.pitch) + unsigned(col) : past;
            sv[0][k] = bload(r0, off, T());
            sv[1][k] = bload(r1, off, T());
            sv[2][k] = bload(r2, off, T());
        }
    }

    // Node f's three values sit together at tile[3 f .. 3 f + 2], so that a
    // cell's whole stencil lies within 216 elements of its first value and
    // every read of the gather is an immediate offset from one address.
    __device__ __forceinline__ void store(T *tile) const
    {
        const int tid = int(threadIdx.y) * 64 + int(threadIdx.x);
#pragma unroll
        for (int k = 0; k < S::PER; k++) {
            const int f = tid + k * kBlock;
            if (f < S::N) {
                tile[3 * f] = sv[0][k];
                tile[3 * f + 1] = sv[1][k];
                tile[3 * f + 2] = sv[2][k];
            }
        }
    }
};

// Tiles of 64 x TY nodes, dealt to the XCDs in contiguous bands (as
// xcd_tile does for 64 x 4 tiles of the stream-function step).
struct TileGrid {
    unsigned tiles_x, tiles, magic;  // tiles per row group, in all, floor(2^32 / tiles_x)
};

// Tiles of 64 x rows nodes over the grid.
static TileGrid tile_grid(const Geom &g, int rows)
{
    TileGrid tg;
    tg.tiles_x = unsigned((g.n[0] + 63) / 64);
    tg.tiles = tg.tiles_x * unsigned((g.n[1] + rows - 1) / rows);
    tg.magic = tg.tiles_x > 1 ? unsigned((uint64_t(1) << 32) / tg.tiles_x) : 0xFFFFFFFFu;
    return tg;
}

__device__ __forceinline__ bool xcd_tile_n(const TileGrid &tg, unsigned &tx, unsigned &ty)
{
    const unsigned per = (tg.tiles + 7u) / 8u;
    const unsigned t = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
    unsigned r;
    ty = udiv_magic(t, tg.tiles_x, tg.magic, r);
    tx = r;
    return t < tg.tiles;
}

// Row groups of four per affine tile: 64 x 8 nodes (a 64 x 4 tile stages 1.6
// values per node and field, 64 x 8 1.3; 64 x 16 measured no faster).
constexpr int kAffineRows = 2;

// Non-temporal store of a result the next step reads only after the whole
// launch, from a grid far larger than the caches: the line is not kept in
// them, which leaves the L2 to the tile halos the neighbouring blocks re-read.
template <typename T>
__device__ __forceinline__ void pstore_nt(T *base, unsigned elem, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) +
                                                         elem * unsigned(sizeof(T))));
}

template <typename T>
struct AffineMap {
    double Mc[9], kc[3];  // foot in cell units: s_a = kc_a + sum_b Mc[a][b] idx_b
    double Md[9];         // Mc - I: the displacement in cells s_a - idx_a = kc_a + sum_b Md[a][b] idx_b
    T J[9];               // Jacobian of the foot map (J form), uniform
    T An[9], Af[9];       // Heun: grad v at the node (t + dt) and at the foot (t)
};

template <typename T>
static AffineMap<T> make_affine_map(const gals_ctx *ctx, double dt, double c1, double c2,
                                    double c3)
{
    const int D = ctx->dim;
    const Vel<double> &p = ctx->vd;
    double A[9] = {0}, b[3] = {0}, xc[3] = {0};
    for (int i = 0; i < D; i++) {
        b[i] = p.b[i];
        xc[i] = p.c[i];
        for (int j = 0; j < D; j++) A[i * 3 + j] = p.A[i * 3 + j];
    }
    auto mm = [&](const double *X, const double *Y, double *Z) {  // Z = X Y (3x3)
        double t[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++) acc += X[i * 3 + k] * Y[k * 3 + j];
                t[i * 3 + j] = acc;
            }
        for (int k = 0; k < 9; k++) Z[k] = t[k];
    };
    auto mv = [&](const double *X, const double *y, double *z) {
        double t[3];
        for (int i = 0; i < 3; i++) t[i] = X[i * 3] * y[0] + X[i * 3 + 1] * y[1] + X[i * 3 + 2] * y[2];
        for (int i = 0; i < 3; i++) z[i] = t[i];
    };
    double V0[9], V1[9], V2[9], P[9], w0[3], w1[3], w2[3], q[3];
    for (int k = 0; k < 9; k++) V0[k] = c1 * A[k];
    for (int i = 0; i < 3; i++) w0[i] = c1 * b[i];
    for (int k = 0; k < 9; k++) P[k] = double(k % 4 == 0) - dt * V0[k];  // I - dt V0
    mm(A, P, V1);
    for (int k = 0; k < 9; k++) V1[k] *= c2;
    mv(A, w0, q);
    for (int i = 0; i < 3; i++) w1[i] = c2 * (b[i] - dt * q[i]);
    for (int k = 0; k < 9; k++) P[k] = double(k % 4 == 0) - dt * 0.25 * (V0[k] + V1[k]);
    mm(A, P, V2);
    for (int k = 0; k < 9; k++) V2[k] *= c3;
    double s01[3];
    for (int i = 0; i < 3; i++) s01[i] = w0[i] + w1[i];
    mv(A, s01, q);
    for (int i = 0; i < 3; i++) w2[i] = c3 * (b[i] - dt * 0.25 * q[i]);
    double M[9], m[3];
    for (int k = 0; k < 9; k++)
        M[k] = double(k % 4 == 0) - dt * (V0[k] * (1.0 / 6.0) + V1[k] * (1.0 / 6.0) + V2[k] * (2.0 / 3.0));
    for (int i = 0; i < 3; i++)
        m[i] = -dt * (w0[i] * (1.0 / 6.0) + w1[i] * (1.0 / 6.0) + w2[i] * (2.0 / 3.0));
    // cell units: s_a = (foot_a - lo_a) / h_a with node x_b = lo_b + idx_b h_b
    AffineMap<T> am;
    for (int a = 0; a < 3; a++) {
        am.kc[a] = 0.0;
        for (int j = 0; j < 3; j++) am.Mc[a * 3 + j] = 0.0;
    }
    const Geom &g = ctx->g;
    for (int a = 0; a < D; a++) {
        double k = (xc[a] - g.lo[a]) + m[a];
        for (int j = 0; j < D; j++) {
            am.Mc[a * 3 + j] = M[a * 3 + j] * g.h[j] / g.h[a];
            k += M[a * 3 + j] * (g.lo[j] - xc[j]);
        }
        am.kc[a] = k / g.h[a];
    }
    for (int k = 0; k < 9; k++) am.Md[k] = am.Mc[k] - double(k % 4 == 0);
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++) {
            am.J[i * D + j] = T(M[i * 3 + j]);
            am.An[i * D + j] = T(c1 * A[i * 3 + j]);
            am.Af[i * D + j] = T(c2 * A[i * 3 + j]);
        }
    return am;
}

template <typename T>
__device__ __forceinline__ void split_cell_axis(const Geom &g, int a, double s, int &cell, T &xi,
                                                bool &outb)
{
    const bool below = s < g.lowc[a], above = s > g.outc[a];
    const double fl = fmin(fmax(floor(s), 0.0), g.lastc[a]);
    cell = int(fl);
    T x = T(s - fl);
    x = below ? T(0) : x;
    xi = above ? T(1) : x;
    outb = below || above;
}

// Boundary treatment and split of a foot given in cell units: outside only
// beyond kFootTol cells (then projected: local coordinate 0 or 1 and the
// normal derivative dropped), cell index clamped to [0, nc - 1], local
// coordinate unclamped otherwise (the same rules as project_foot + split).
template <typename T, int D>
__device__ __forceinline__ void split_cells(const Geom &g, const double *s, int *cell, T *xi,
                                            bool *outb)
{
#pragma unroll
    for (int a = 0; a < D; a++) split_cell_axis(g, a, s[a], cell[a], xi[a], outb[a]);
}

// The same for an FP32 state from the displacement in cells e = s - idx
// (FP64, rounded to FP32 here: one rounding, u |e|): with c = floor(e), a
// foot whose cell idx + c lies in [0, nc-1] (not outside, not clamped)
// splits into cell idx + c and local coordinate e - c, both exact in FP32.
// Only the other lanes take the FP64 treatment of split_cells (from
// s = idx + e), and a wave without such lanes skips it; each lane's result
// is the same either way.
template <typename T, int D>
__device__ __forceinline__ void split_disp(const Geom &g, const int *idx, const double *e64,
                                           int *cell, T *xi, bool *outb)
{
    static_assert(sizeof(T) == 4, "FP32 states only");
    float e[D], c[D];
    int cu[D];
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; a++) {
        e[a] = float(e64[a]);
        c[a] = floor(e[a]);
        cu[a] = idx[a] + int(c[a]);
        in = in && unsigned(cu[a]) <= unsigned(g.nc[a] - 1);
    }
    if (__builtin_expect(__all(in), 1)) {
#pragma unroll
        for (int a = 0; a < D; a++) {
            cell[a] = cu[a];
            xi[a] = e[a] - c[a];
            outb[a] = false;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < D; a++) {
        const float fr = e[a] - c[a];
        if (unsigned(cu[a]) <= unsigned(g.nc[a] - 1)) {
            cell[a] = cu[a];
            xi[a] = fr;
            outb[a] = false;
        } else if (cu[a] == g.nc[a] && double(fr) <= g.outc[a] - g.ncd[a]) {
            // at most kFootTol past the last node: the last cell at local
            // coordinate 1 + fr (split_cells' rule, evaluated in FP32)
            cell[a] = g.nc[a] - 1;
            xi[a] = 1.0f + fr;
            outb[a] = false;
        } else {
            split_cell_axis(g, a, double(idx[a]) + e64[a], cell[a], xi[a], outb[a]);
        }
    }
}

// Cell data from the staged tile (node-interleaved: node k's phi, psi_x,
// psi_y at t[3 k], t[3 k + 1], t[3 k + 2]) at index b of the cell's
// lower-left node: every neighbour sits at a fixed offset (one row = W
// nodes). The central cross derivative reads one column beyond each side of
// the cell; at the first and last cell of a row that column lies outside the
// grid, and the one-sided differences used there do not read it (same
// values as gather2d).
template <typename T, int MIX, int W>
__device__ __forceinline__ void gather2d_lds(const Geom &g, const T *tile, int b, int cx,
                                             T d[4][4])
{
    // from node b - 1: offsets up to 3 (W + 2) + 2 elements, within the
    // paired LDS reads' immediate range (255 elements) for W <= 81
    static_assert(3 * (W + 3) + 2 <= 255, "stencil beyond the immediate offsets");
    const T *t = tile + 3 * (b - 1);
    auto at = [&](int k, int f) { return t[3 * (k + 1) + f]; };
    d[0][0] = at(0, 0); d[1][0] = at(1, 0); d[2][0] = at(W, 0); d[3][0] = at(W + 1, 0);
    d[0][1] = at(0, 1); d[1][1] = at(1, 1); d[2][1] = at(W, 1); d[3][1] = at(W + 1, 1);
    if constexpr (MIX == GALS_MIXED_CENTRAL) {
        const T u0[4] = {at(-1, 2), at(0, 2), at(1, 2), at(2, 2)};
        const T u1[4] = {at(W - 1, 2), at(W, 2), at(W + 1, 2), at(W + 2, 2)};
        d[0][2] = u0[1]; d[1][2] = u0[2];
        d[2][2] = u1[1]; d[3][2] = u1[2];
        const T inv2h = geo_i2h<T>(g, 0);
        const bool lo = cx == 0, hi = cx + 1 == g.nc[0];
        diff_pair<T, sizeof(T) == 4>(u0, lo, hi, inv2h, d[0][3], d[1][3]);
        diff_pair<T, sizeof(T) == 4>(u1, lo, hi, inv2h, d[2][3], d[3][3]);
    } else {
        d[0][2] = at(0, 2); d[1][2] = at(1, 2); d[2][2] = at(W, 2); d[3][2] = at(W + 1, 2);
        if constexpr (MIX == GALS_MIXED_CELL) {
            T ga[4], gb[4], out[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                ga[v] = d[v][1];
                gb[v] = d[v][2];
            }
            cell_cross(ga, gb, geo_ih<T>(g, 0), geo_ih<T>(g, 1), out);
#pragma unroll
            for (int v = 0; v < 4; v++) d[v][3] = out[v];
        } else {
            d[0][3] = d[1][3] = d[2][3] = d[3][3] = T(0);
        }
    }
}

// 2D step for an affine field: the foot from the host's map, the old state
// staged in a 64 x 4R node tile with its halo, the gather
// from the tile at fixed offsets, or from global memory for a stencil off
// the tile.
template <typename T, int MIX, int PSI, int R>
__global__ __launch_bounds__(kBlock) void k_step2d_affine(Geom g, TileGrid tg, AffineMap<T> am,
                                                          double dt, const T *__restrict__ phi,
                                                          const T *__restrict__ grad,
                                                          T *__restrict__ phi_o,
                                                          T *__restrict__ grad_o)
{
    using S = StageTile<4 * R>;
    __shared__ T tile[3 * S::N];
    unsigned tx, ty;
    if (!xcd_tile_n(tg, tx, ty)) return;  // whole blocks only: before the barrier
    const int cx0 = int(tx) * 64 - kHaloX, ry0 = int(ty) * (4 * R) - kHaloY;
    const T *gx = grad, *gy = grad + g.plane;
    TileStager<T, 4 * R> stager;
    stager.load(g, phi, gx, gy, cx0, ry0);
    const int i = int(tx) * 64 + int(threadIdx.x);
    int cell[R][2];
    T xi[R][2];
    bool outb[R][2];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = __builtin_amdgcn_readfirstlane(ry0 + kHaloY + int(threadIdx.y) + 4 * r);
        if constexpr (sizeof(T) == 4) {
            const int idx[2] = {i, j};
            double e[2];
#pragma unroll
            for (int a = 0; a < 2; a++)
                e[a] = am.kc[a] + am.Md[a * 3] * double(i) + am.Md[a * 3 + 1] * double(j);
            split_disp<T, 2>(g, idx, e, cell[r], xi[r], outb[r]);
        } else {
            double sc[2];
#pragma unroll
            for (int a = 0; a < 2; a++)
                sc[a] = am.kc[a] + am.Mc[a * 3] * double(i) + am.Mc[a * 3 + 1] * double(j);
            split_cells<T, 2>(g, sc, cell[r], xi[r], outb[r]);
        }
    }
    stager.store(tile);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = __builtin_amdgcn_readfirstlane(ry0 + kHaloY + int(threadIdx.y) + 4 * r);
        const int cx = cell[r][0], cy = cell[r][1];
        const bool on = cx - 1 >= cx0 && cx + 2 < cx0 + S::W && cy >= ry0 && cy + 1 < ry0 + S::H;
        const bool store = i < g.n[0] && j < g.n[1];
        // the Hermite evaluation and the update from the cell data of either
        // source; each source finishes on its own (merging the two sources'
        // cell data before one evaluation cost register moves on every lane)
        auto finish = [&](const T (&d)[4][4]) {
            Basis<T> bx, by;
            basis<T, false>(xi[r][0], geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
            basis<T, false>(xi[r][1], geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
            T H, Hx, Hy;
            hermite2d(d, bx, by, H, Hx, Hy);
            if (outb[r][0]) Hx = T(0);
            if (outb[r][1]) Hy = T(0);
            if (!store) return;
            const unsigned o = unsigned(j) * unsigned(g.pitch) + unsigned(i);
            T g0, g1;
            if constexpr (PSI == GALS_PSI_HEUN) {
                T ps[2];
                const T gH[2] = {Hx, Hy};
                heun_gradient<T, 2>(am.Af, am.An, T(dt), gH, ps);
                g0 = ps[0];
                g1 = ps[1];
            } else {
                g0 = am.J[0] * Hx + am.J[2] * Hy;
                g1 = am.J[1] * Hx + am.J[3] * Hy;
            }
            pstore_nt(phi_o, o, H);
            pstore_nt(grad_o, o, g0);
            pstore_nt(grad_o + g.plane, o, g1);
        };
        if (__builtin_expect(on, 1)) {
            T d[4][4];
            gather2d_lds<T, MIX, S::W>(g, tile, (cy - ry0) * S::W + (cx - cx0), cx, d);
            finish(d);
        } else {
            T d[4][4];
            gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(gx, g.plane),
                             plane_rsrc(gy, g.plane), cx, cy, d);
            finish(d);
        }
    }
}

// Node of this thread in a 3D step. Blocks are dealt to the 8 XCDs
// round-robin by id, and each XCD has its own L2: XCD x takes the nodes of
// every z-plane whose in-plane index (j n0 + i) lies in the x-th eighth of
// the plane, plane after plane in blocks of kBlock. A node gathers from rows
// j - 1 .. j + 2 of planes k and k + 1, so an XCD's gathers stay within its
// eighth of a few planes and the next eighth's first rows, which its L2
// holds (contiguous bands of the flat node order kept a few whole planes of
// every field in each L2, more than it holds in 3D). Returns false past the
// band's last node.
__device__ __forceinline__ bool band_node3d(const Geom &g, int &i, int &j, int &k)
{
    const unsigned x = blockIdx.x & 7u, b = blockIdx.x >> 3;
    const unsigned P = unsigned(g.n[0]) * unsigned(g.n[1]);  // nodes per plane
    const unsigned s0 = unsigned((uint64_t(x) * P) >> 3);
    const unsigned len = unsigned((uint64_t(x + 1u) * P) >> 3) - s0;  // this XCD's nodes per plane
    const unsigned id = b * unsigned(kBlock) + threadIdx.x;
    if (len == 0u || id >= len * unsigned(g.n[2])) return false;
    // plane from an FP32 estimate of id / len, corrected once: a state plane
    // under 2 GiB keeps id < 2^27 and the quotient (a plane index) < 2^21.5,
    // and the estimate's relative error (conversion, reciprocal, product) is
    // under 2^-22, so it is off by less than one
    int kk = int(float(id) * __builtin_amdgcn_rcpf(float(len)));
    int q = int(id) - kk * int(len);
    if (q < 0) { kk--; q += int(len); }
    else if (q >= int(len)) { kk++; q -= int(len); }
    unsigned ri;
    j = int(udiv_magic(s0 + unsigned(q), unsigned(g.n[0]), g.n_magic[0], ri));
    i = int(ri);
    k = kk;
    return true;
}

// Blocks of a 3D step's launch: 8 x the blocks of the largest XCD band.
inline unsigned band_blocks3d(const Geom &g)
{
    const uint64_t P = uint64_t(g.n[0]) * uint64_t(g.n[1]);
    const uint64_t band = (P + 7u) / 8u * uint64_t(g.n[2]);
    return unsigned(8u * ((band + kBlock - 1) / kBlock));
}

// 3D step for an affine field: the foot from the host's map, one thread per
// node, the 64-value gather through the caches.
template <typename T, int MIX, int PSI>
__global__ __launch_bounds__(kBlock) void k_step3d_affine(Geom g, AffineMap<T> am, double dt,
                                                          const T *__restrict__ phi,
                                                          const T *__restrict__ grad,
                                                          T *__restrict__ phi_o,
                                                          T *__restrict__ grad_o)
{
    int i, j, k;
    if (!band_node3d(g, i, j, k)) return;
    double sc[3];
#pragma unroll
    for (int a = 0; a < 3; a++)
        sc[a] = am.kc[a] + am.Mc[a * 3] * double(i) + am.Mc[a * 3 + 1] * double(j) +
                am.Mc[a * 3 + 2] * double(k);
    int cell[3];
    T xi[3];
    bool outb[3];
    split_cells<T, 3>(g, sc, cell, xi, outb);
    const T *gx = grad, *gy = grad + g.plane, *gz = grad + 2 * g.plane;
    T d[8][8];
    gather3d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(gx, g.plane), plane_rsrc(gy, g.plane),
                     plane_rsrc(gz, g.plane), cell[0], cell[1], cell[2], d);
    Basis<T> bx, by, bz;
    basis<T, false>(xi[0], geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
    basis<T, false>(xi[1], geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
    basis<T, false>(xi[2], geo_h<T>(g, 2), geo_ih<T>(g, 2), bz);
    T H, Hx, Hy, Hz;
    hermite3d(d, bx, by, bz, H, Hx, Hy, Hz);
    if (outb[0]) Hx = T(0);
    if (outb[1]) Hy = T(0);
    if (outb[2]) Hz = T(0);
    const unsigned o = (unsigned(k) * unsigned(g.n[1]) + unsigned(j)) * unsigned(g.pitch) +
                       unsigned(i);
    pstore(phi_o, o, H);
    if constexpr (PSI == GALS_PSI_HEUN) {
        T ps[3];
        const T gH[3] = {Hx, Hy, Hz};
        heun_gradient<T, 3>(am.Af, am.An, T(dt), gH, ps);
        pstore(grad_o, o, ps[0]);
        pstore(grad_o + g.plane, o, ps[1]);
        pstore(grad_o + 2 * g.plane, o, ps[2]);
    } else {
        const T *J = am.J;
        pstore(grad_o, o, J[0] * Hx + J[3] * Hy + J[6] * Hz);
        pstore(grad_o + g.plane, o, J[1] * Hx + J[4] * Hy + J[7] * Hz);
        pstore(grad_o + 2 * g.plane, o, J[2] * Hx + J[5] * Hy + J[8] * Hz);
    }
}

// The part of a 3D step after the trace: boundary treatment of the foot,
// split, 64-value gather, tricubic value and gradient, gradient update.
template <typename T, int KIND, int MIX, int PSI>
__device__ __forceinline__ void finish3d(const Geom &g, const Vel<T> &p, const Stage<T> &st,
                                         double dt, int i, int j, int k, double *X, const T *J,
                                         const T *__restrict__ phi, const T *__restrict__ grad,
                                         T *__restrict__ phi_o, T *__restrict__ grad_o)
{
    const T *gx = grad, *gy = grad + g.plane, *gz = grad + 2 * g.plane;
    const unsigned out = project_foot<3>(g, X);

    int cell[3];
    double xi[3];
    split<3>(g, X, cell, xi);

    T d[8][8];
    gather3d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(gx, g.plane), plane_rsrc(gy, g.plane),
                     plane_rsrc(gz, g.plane), cell[0], cell[1], cell[2], d);
    Basis<T> bx, by, bz;
    basis<T, false>(T(xi[0]), geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
    basis<T, false>(T(xi[1]), geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
    basis<T, false>(T(xi[2]), geo_h<T>(g, 2), geo_ih<T>(g, 2), bz);
    T H, Hx, Hy, Hz;
    hermite3d(d, bx, by, bz, H, Hx, Hy, Hz);
    if (out & 1u) Hx = T(0);
    if (out & 2u) Hy = T(0);
    if (out & 4u) Hz = T(0);

    const unsigned o = (unsigned(k) * unsigned(g.n[1]) + unsigned(j)) * unsigned(g.pitch) +
                       unsigned(i);
    pstore(phi_o, o, H);
    if constexpr (PSI == GALS_PSI_HEUN) {
        T vf[3], Af[9], ps[3];
        const T gH[3] = {Hx, Hy, Hz};
        velocity<T, 3, KIND>(p, X, st.c2, vf, Af);
        heun_gradient<T, 3>(Af, J, T(dt), gH, ps);
        pstore(grad_o, o, ps[0]);
        pstore(grad_o + g.plane, o, ps[1]);
        pstore(grad_o + 2 * g.plane, o, ps[2]);
    } else {
        pstore(grad_o, o, J[0] * Hx + J[3] * Hy + J[6] * Hz);
        pstore(grad_o + g.plane, o, J[1] * Hx + J[4] * Hy + J[7] * Hz);
        pstore(grad_o + 2 * g.plane, o, J[2] * Hx + J[5] * Hy + J[8] * Hz);
    }
}

template <typename T, int KIND, int MIX, int PSI>
__global__ __launch_bounds__(kBlock) void k_step3d(Geom g, Vel<T> p, Stage<T> st, double dt,
                                                   const T *__restrict__ phi,
                                                   const T *__restrict__ grad,
                                                   T *__restrict__ phi_o, T *__restrict__ grad_o)
{
    int i, j, k;
    if (!band_node3d(g, i, j, k)) return;

    const double x[3] = {node_coord(g.lo[0], i, g.h[0]), node_coord(g.lo[1], j, g.h[1]),
                         node_coord(g.lo[2], k, g.h[2])};
    double X[3];
    T J[9];
    trace<T, 3, KIND, PSI == GALS_PSI_SUPERCONSISTENT>(p, st, dt, x, X, J);
    finish3d<T, KIND, MIX, PSI>(g, p, st, dt, i, j, k, X, J, phi, grad, phi_o, grad_o);
}

// ---------------------------------------------------------------------------
// Sine vector potentials in 3D: sin(pi x) and cos(pi x) of every node
// coordinate come from per-axis tables (FP64-built, one pair per node along
// each axis); the three stages take the multiples of the node's angles, and
// (SHIFT) the two off-node stages shift them by angle addition whenever
// every offset is small enough for the series of the precision, instead of
// evaluating sin and cos at the stage points. The mode sums are those of
// vel_vecpot.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axis_tables(Geom g, T *__restrict__ tab)
{
    const int id = int(blockIdx.x) * kBlock + int(threadIdx.x);
    int r = id, a = 0;
    while (a < 3 && r >= g.n[a]) r -= g.n[a++];
    if (a >= 3) return;
    double s, c;
    sincospi(node_coord(g.lo[a], r, g.h[a]), &s, &c);
    tab[2 * id] = T(s);
    tab[2 * id + 1] = T(c);
}

// Velocity at one stage point from the multiples of each axis: through LDS
// (LDS, the FP32 kernel) or by per-lane selects.
template <typename T, bool LDS>
__device__ __forceinline__ void modes_at(const Vel<T> &p, T (*tab)[kBlock], const T *sx,
                                         const T *cx, const T *sy, const T *cy, const T *sz,
                                         const T *cz, T cf, T *v, T *A)
{
    if constexpr (LDS) {
        const int tid = int(threadIdx.x);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            tab[r][tid] = sx[r];
            tab[4 + r][tid] = cx[r];
            tab[8 + r][tid] = sy[r];
            tab[12 + r][tid] = cy[r];
            tab[16 + r][tid] = sz[r];
            tab[20 + r][tid] = cz[r];
        }
        vecpot_modes_lds(p, tab, tid, cf, v, A);  // each thread reads only its own column
    } else {
        vecpot_modes(p, sx, cx, sy, cy, sz, cz, cf, v, A);
    }
}

template <typename T, bool SHIFT, bool LDS>
__device__ __forceinline__ void stage_vecpot(const Vel<T> &p, T (*tab)[kBlock], const T *s1,
                                             const T *c1, const double *x, const T *d, T *w,
                                             T *R)
{
    T sx[4], cx[4], sy[4], cy[4], sz[4], cz[4];
    // FP32: the short series up to |pi d| = kShiftMax; FP64: the long one
    constexpr double kMax = sizeof(T) == 4 ? kShiftMax : kShiftMaxLong<T>;
    bool near = SHIFT;
#pragma unroll
    for (int a = 0; a < 3; a++) near = near && fabs(d[a]) <= T(kMax / kPi);
    if (near) {
        T s[3], c[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if constexpr (sizeof(T) == 4)
                shifted_sincos(s1[a], c1[a], d[a], s[a], c[a]);
            else
                shifted_sincos_long(s1[a], c1[a], d[a], s[a], c[a]);
        }
        multiples_from(s[0], c[0], sx, cx);
        multiples_from(s[1], c[1], sy, cy);
        multiples_from(s[2], c[2], sz, cz);
    } else {
        sincos_multiples(T(x[0] + double(d[0])), sx, cx);
        sincos_multiples(T(x[1] + double(d[1])), sy, cy);
        sincos_multiples(T(x[2] + double(d[2])), sz, cz);
    }
    modes_at<T, LDS>(p, tab, sx, cx, sy, cy, sz, cz, T(1), w, R);
}

// Five waves per SIMD for the FP32 superconsistent kernel: about 93 VGPRs
// without spills (six waves would spill); the FP64 and Heun kernels need more
// registers and keep the compiler's choice.
template <typename T, int MIX, bool SHIFT, int PSI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && PSI == GALS_PSI_SUPERCONSISTENT ? 5 : 1))) void k_step3d_vecpot(
    Geom g, Vel<T> p, Stage<T> st,
                                                          double dt, const T *__restrict__ tab,
                                                          const T *__restrict__ phi,
                                                          const T *__restrict__ grad,
                                                          T *__restrict__ phi_o,
                                                          T *__restrict__ grad_o)
{
    constexpr bool LDS = sizeof(T) == 4;
    __shared__ T tab_s[LDS ? 24 : 1][kBlock];
    int i, j, k;
    if (!band_node3d(g, i, j, k)) return;

    const double x[3] = {node_coord(g.lo[0], i, g.h[0]), node_coord(g.lo[1], j, g.h[1]),
                         node_coord(g.lo[2], k, g.h[2])};
    const int64_t ti[3] = {i, int64_t(g.n[0]) + j, int64_t(g.n[0]) + g.n[1] + k};
    T s1[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        s1[a] = tab[2 * ti[a]];
        c1[a] = tab[2 * ti[a] + 1];
    }
    // w_k, R_k: velocity and velocity Jacobian at stage k without the time
    // factor c_k (Stage carries dt c_k in its weights, as in the 2D stream
    // step); the stage offsets and the foot's displacement are summed in T,
    // the foot itself in FP64
    T w0[3], R0[9], w1[3], R1[9], w2[3], R2[9];
    {
        T sx[4], cx[4], sy[4], cy[4], sz[4], cz[4];
        multiples_from(s1[0], c1[0], sx, cx);
        multiples_from(s1[1], c1[1], sy, cy);
        multiples_from(s1[2], c1[2], sz, cz);
        modes_at<T, LDS>(p, tab_s, sx, cx, sy, cy, sz, cz, T(1), w0, R0);  // at x, t + dt
    }
    T d1[3], d2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d1[a] = -st.e1 * w0[a];
    stage_vecpot<T, SHIFT, LDS>(p, tab_s, s1, c1, x, d1, w1, R1);  // at x1 = x + d1, t
#pragma unroll
    for (int a = 0; a < 3; a++) d2[a] = -(st.q1 * w0[a] + st.q2 * w1[a]);
    stage_vecpot<T, SHIFT, LDS>(p, tab_s, s1, c1, x, d2, w2, R2);  // at x2 = x + d2, t + dt/2
    double X[3];
#pragma unroll
    for (int a = 0; a < 3; a++)
        X[a] = x[a] - double(st.f1 * w0[a] + st.f2 * w1[a] + st.f3 * w2[a]);
    T J[9];
    if constexpr (PSI == GALS_PSI_SUPERCONSISTENT) {
        jacobian_chain_w<T, 3>(R0, R1, R2, st, J);
    } else {
#pragma unroll
        for (int q = 0; q < 9; q++) J[q] = st.c1 * R0[q];
    }
    finish3d<T, GALS_VEL_VECPOT_SIN, MIX, PSI>(g, p, st, dt, i, j, k, X, J, phi, grad, phi_o,
                                              grad_o);
}

// ---------------------------------------------------------------------------
// Sine stream-function fields (see stream2d.h).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stream_tables(Geom g, Vel<double> p,
                                                          T *__restrict__ coltab,
                                                          T *__restrict__ rowtab)
{
    stream_table_entry(g, p.S, int(blockIdx.x) * kBlock + int(threadIdx.x), coltab, rowtab);
}

// GA-CIR step for the sine stream-function field. Launch: blocks of 64 x 4
// threads over 64 x 4 node tiles; each wave owns 64 consecutive nodes of one
// row, so the row table is read once per wave through scalar loads. The cell
// data are gathered through the caches after the trace: the kernel is bound
// by its vector ALU, and staging the tile through LDS (as the affine step
// does) measured slower in both precisions (FP32 34.0 -> 39.9 us, FP64 87.2
// -> 102.4 us per 2049^2 step: more instructions, and in FP64 one wave per
// SIMD fewer).
template <typename T, int MIX, bool TAYLOR, int PSI>
__global__ __launch_bounds__(kBlock) void k_step2d_stream(
    Geom g, Vel<T> p, Stage<T> st, double dt, const T *__restrict__ coltab,
    const T *__restrict__ rowtab, const T *__restrict__ phi, const T *__restrict__ grad,
    T *__restrict__ phi_o, T *__restrict__ grad_o)
{
    unsigned tx, ty;
    if (!xcd_tile(g, tx, ty)) return;
    const int i = int(tx) * 64 + int(threadIdx.x);
    const int j = __builtin_amdgcn_readfirstlane(int(ty) * 4 + int(threadIdx.y));
    if (j >= g.n[1] || i >= g.n[0]) return;
    stream_node<T, MIX, TAYLOR, PSI>(g, p, st, dt, coltab + int64_t(i) * kJet,
                                     rowtab + int64_t(j) * kJet, phi, grad, grad + g.plane,
                                     phi_o, grad_o, grad_o + g.plane, i, j);
}

hipError_t launch_stream_tables(const gals_ctx *ctx, void *coltab, void *rowtab, hipStream_t s)
{
    const unsigned blocks = unsigned((ctx->g.n[0] + ctx->g.n[1] + kBlock - 1) / kBlock);
    if (ctx->prec == GALS_F32)
        hipLaunchKernelGGL(k_stream_tables<float>, dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           ctx->vd, (float *)coltab, (float *)rowtab);
    else
        hipLaunchKernelGGL(k_stream_tables<double>, dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           ctx->vd, (double *)coltab, (double *)rowtab);
    return hipGetLastError();
}

template <typename T, int MIX, int PSI>
static hipError_t launch_stream(const gals_ctx *ctx, const Vel<T> &p, const void *phi,
                                const void *grad, void *phi_o, void *grad_o, double dt,
                                double c1, double c2, double c3, const void *coltab,
                                const void *rowtab, hipStream_t s)
{
    const Stage<T> st = make_stage<T>(dt, c1, c2, c3);
    const unsigned tiles = ctx->g.tiles;
    const dim3 grid((tiles + 7u) / 8u * 8u);
    hipLaunchKernelGGL((k_step2d_stream<T, MIX, sizeof(T) == 4, PSI>), grid, dim3(64, 4), 0, s,
                       ctx->g, p, st, dt, (const T *)coltab, (const T *)rowtab, (const T *)phi,
                       (const T *)grad, (T *)phi_o, (T *)grad_o);
    return hipGetLastError();
}

hipError_t launch_axis_tables(const gals_ctx *ctx, void *tab, hipStream_t s)
{
    const int count = ctx->g.n[0] + ctx->g.n[1] + ctx->g.n[2];
    const unsigned blocks = unsigned((count + kBlock - 1) / kBlock);
    if (ctx->prec == GALS_F32)
        hipLaunchKernelGGL(k_axis_tables<float>, dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           (float *)tab);
    else
        hipLaunchKernelGGL(k_axis_tables<double>, dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           (double *)tab);
    return hipGetLastError();
}

template <typename T, int MIX, int PSI>
static hipError_t launch_vecpot(const gals_ctx *ctx, const Vel<T> &p, const void *phi,
                                const void *grad, void *phi_o, void *grad_o, double dt,
                                double c1, double c2, double c3, const void *tab, hipStream_t s)
{
    const Stage<T> st = make_stage<T>(dt, c1, c2, c3);
    const unsigned blocks = band_blocks3d(ctx->g);
    hipLaunchKernelGGL((k_step3d_vecpot<T, MIX, true, PSI>), dim3(blocks),
                       dim3(kBlock), 0, s, ctx->g, p, st, dt, (const T *)tab, (const T *)phi,
                       (const T *)grad, (T *)phi_o, (T *)grad_o);
    return hipGetLastError();
}

template <typename T, int KIND, int MIX, int PSI>
static hipError_t launch_typed(const gals_ctx *ctx, const Vel<T> &p, const void *phi,
                               const void *grad, void *phi_o, void *grad_o, double dt, double c1,
                               double c2, double c3, hipStream_t s)
{
    const Stage<T> st = make_stage<T>(dt, c1, c2, c3);
    // rounded up to a multiple of 8 for the XCD band mapping (xcd_block)
    const unsigned blocks = unsigned((ctx->g.nodes + kBlock - 1) / kBlock + 7) / 8u * 8u;
    if constexpr (KIND == GALS_VEL_AFFINE) {
        const AffineMap<T> am = make_affine_map<T>(ctx, dt, c1, c2, c3);
        if (ctx->dim == 2) {
            const TileGrid tg = tile_grid(ctx->g, 4 * kAffineRows);
            hipLaunchKernelGGL((k_step2d_affine<T, MIX, PSI, kAffineRows>),
                               dim3((tg.tiles + 7u) / 8u * 8u),
                               dim3(64, 4), 0, s, ctx->g, tg, am, dt, (const T *)phi,
                               (const T *)grad, (T *)phi_o, (T *)grad_o);
        } else {
            hipLaunchKernelGGL((k_step3d_affine<T, MIX, PSI>), dim3(band_blocks3d(ctx->g)),
                               dim3(kBlock), 0, s,
                               ctx->g, am, dt, (const T *)phi, (const T *)grad, (T *)phi_o,
                               (T *)grad_o);
        }
        return hipGetLastError();
    }
    if (ctx->dim == 2) {
        if constexpr (KIND == GALS_VEL_STREAM_SIN || KIND == GALS_VEL_VORTEX ||
                      KIND == GALS_VEL_PSEUDO1D) {
            hipLaunchKernelGGL((k_step2d<T, KIND, MIX, PSI>), dim3(blocks), dim3(kBlock), 0, s,
                               ctx->g, p, st, dt, (const T *)phi, (const T *)grad, (T *)phi_o,
                               (T *)grad_o);
            return hipGetLastError();
        }
    } else {
        if constexpr (KIND == GALS_VEL_VECPOT_SIN || KIND == GALS_VEL_LEVEQUE3D) {
            hipLaunchKernelGGL((k_step3d<T, KIND, MIX, PSI>), dim3(band_blocks3d(ctx->g)),
                               dim3(kBlock), 0, s,
                               ctx->g, p, st, dt, (const T *)phi, (const T *)grad, (T *)phi_o,
                               (T *)grad_o);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

template <typename T, int MIX, int PSI>
static hipError_t launch_kind(const gals_ctx *ctx, const Vel<T> &p, const void *phi,
                              const void *grad, void *phi_o, void *grad_o, double dt, double c1,
                              double c2, double c3, hipStream_t s)
{
#define GALS_KIND_CASE(K)                                                                         \
    case K:                                                                                       \
        return launch_typed<T, K, MIX, PSI>(ctx, p, phi, grad, phi_o, grad_o, dt, c1, c2, c3, s);
    switch (ctx->vel_kind) {
        GALS_KIND_CASE(GALS_VEL_AFFINE)
        GALS_KIND_CASE(GALS_VEL_STREAM_SIN)
        GALS_KIND_CASE(GALS_VEL_VECPOT_SIN)
        GALS_KIND_CASE(GALS_VEL_VORTEX)
        GALS_KIND_CASE(GALS_VEL_PSEUDO1D)
        GALS_KIND_CASE(GALS_VEL_LEVEQUE3D)
    default:
        return hipErrorInvalidValue;
    }
#undef GALS_KIND_CASE
}

// Run f with the cross-derivative mode and the gradient update as
// compile-time constants.
template <class F>
static hipError_t with_modes(int mixed, int psi, F &&f)
{
    auto on_psi = [&](auto mix) -> hipError_t {
        if (psi == GALS_PSI_HEUN) return f(mix, std::integral_constant<int, GALS_PSI_HEUN>{});
        return f(mix, std::integral_constant<int, GALS_PSI_SUPERCONSISTENT>{});
    };
    if (mixed == GALS_MIXED_ZERO) return on_psi(std::integral_constant<int, GALS_MIXED_ZERO>{});
    if (mixed == GALS_MIXED_CELL) return on_psi(std::integral_constant<int, GALS_MIXED_CELL>{});
    return on_psi(std::integral_constant<int, GALS_MIXED_CENTRAL>{});
}

hipError_t launch_step(const gals_ctx *ctx, const void *phi, const void *grad, void *phi_o,
                       void *grad_o, double dt, double c1, double c2, double c3,
                       const void *coltab, const void *rowtab, hipStream_t s)
{
    const bool stream = ctx->vel_kind == GALS_VEL_STREAM_SIN && coltab && rowtab;
    const bool vecpot = ctx->dim == 3 && ctx->vel_kind == GALS_VEL_VECPOT_SIN && coltab;
    return with_modes(ctx->mixed, ctx->psi, [&](auto mix, auto psi) -> hipError_t {
        constexpr int MIX = decltype(mix)::value, PSI = decltype(psi)::value;
        if (vecpot)
            return ctx->prec == GALS_F32
                       ? launch_vecpot<float, MIX, PSI>(ctx, ctx->vf, phi, grad, phi_o, grad_o,
                                                        dt, c1, c2, c3, coltab, s)
                       : launch_vecpot<double, MIX, PSI>(ctx, ctx->vd, phi, grad, phi_o, grad_o,
                                                         dt, c1, c2, c3, coltab, s);
        if (stream)
            return ctx->prec == GALS_F32
                       ? launch_stream<float, MIX, PSI>(ctx, ctx->vf, phi, grad, phi_o, grad_o,
                                                        dt, c1, c2, c3, coltab, rowtab, s)
                       : launch_stream<double, MIX, PSI>(ctx, ctx->vd, phi, grad, phi_o, grad_o,
                                                         dt, c1, c2, c3, coltab, rowtab, s);
        return ctx->prec == GALS_F32
                   ? launch_kind<float, MIX, PSI>(ctx, ctx->vf, phi, grad, phi_o, grad_o, dt, c1,
                                                  c2, c3, s)
                   : launch_kind<double, MIX, PSI>(ctx, ctx->vd, phi, grad, phi_o, grad_o, dt, c1,
                                                   c2, c3, s);
    });
}

}  // namespace gals
