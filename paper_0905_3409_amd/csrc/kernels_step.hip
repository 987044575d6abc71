// GA-CIR step kernels for gfx950: one thread per grid node, wave64, fused
// trace + split + gather + Hermite + gradient update (superconsistent, or
// Heun's method along the characteristic).
//
// Each node reads only the old state (never updated in place) and writes its
// new phi, psi with coalesced SoA stores. Departure cells are gathered through
// the cache hierarchy, so any CFL number is handled by the same code path.
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
    unsigned blk;
    if (!xcd_block(unsigned((g.nodes + kBlock - 1) / kBlock), blk)) return;
    const unsigned id = blk * kBlock + threadIdx.x;
    if (id >= unsigned(g.nodes)) return;
    unsigned ri, rj;
    const unsigned row = udiv_magic(id, unsigned(g.n[0]), g.n_magic[0], ri);
    const int k = int(udiv_magic(row, unsigned(g.n[1]), g.n_magic[1], rj));
    const int i = int(ri), j = int(rj);

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
                                             const T *c1, const double *x, const double *xs,
                                             T cf, T *v, T *A)
{
    T sx[4], cx[4], sy[4], cy[4], sz[4], cz[4];
    // FP32: the short series up to |pi d| = kShiftMax; FP64: the long one
    constexpr double kMax = sizeof(T) == 4 ? kShiftMax : kShiftMaxLong<T>;
    bool near = SHIFT;
    T d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        d[a] = T(xs[a] - x[a]);
        near = near && fabs(d[a]) <= T(kMax / kPi);
    }
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
        sincos_multiples(T(xs[0]), sx, cx);
        sincos_multiples(T(xs[1]), sy, cy);
        sincos_multiples(T(xs[2]), sz, cz);
    }
    modes_at<T, LDS>(p, tab, sx, cx, sy, cy, sz, cz, cf, v, A);
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
    unsigned blk;
    if (!xcd_block(unsigned((g.nodes + kBlock - 1) / kBlock), blk)) return;
    const unsigned id = blk * kBlock + threadIdx.x;
    if (id >= unsigned(g.nodes)) return;
    unsigned ri, rj;
    const unsigned row = udiv_magic(id, unsigned(g.n[0]), g.n_magic[0], ri);
    const int k = int(udiv_magic(row, unsigned(g.n[1]), g.n_magic[1], rj));
    const int i = int(ri), j = int(rj);

    const double x[3] = {node_coord(g.lo[0], i, g.h[0]), node_coord(g.lo[1], j, g.h[1]),
                         node_coord(g.lo[2], k, g.h[2])};
    const int64_t ti[3] = {i, int64_t(g.n[0]) + j, int64_t(g.n[0]) + g.n[1] + k};
    T s1[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        s1[a] = tab[2 * ti[a]];
        c1[a] = tab[2 * ti[a] + 1];
    }
    T v0[3], A0[9], v1[3], A1[9], v2[3], A2[9];
    {
        T sx[4], cx[4], sy[4], cy[4], sz[4], cz[4];
        multiples_from(s1[0], c1[0], sx, cx);
        multiples_from(s1[1], c1[1], sy, cy);
        multiples_from(s1[2], c1[2], sz, cz);
        modes_at<T, LDS>(p, tab_s, sx, cx, sy, cy, sz, cz, st.c1, v0, A0);  // v(x, t + dt)
    }
    double x1[3], x2[3], X[3];
#pragma unroll
    for (int a = 0; a < 3; a++) x1[a] = x[a] - dt * double(v0[a]);
    stage_vecpot<T, SHIFT, LDS>(p, tab_s, s1, c1, x, x1, st.c2, v1, A1);  // v(x1, t)
#pragma unroll
    for (int a = 0; a < 3; a++) x2[a] = x[a] - dt * (0.25 * double(v0[a]) + 0.25 * double(v1[a]));
    stage_vecpot<T, SHIFT, LDS>(p, tab_s, s1, c1, x, x2, st.c3, v2, A2);  // v(x2, t + dt/2)
#pragma unroll
    for (int a = 0; a < 3; a++)
        X[a] = x[a] - dt * (double(v0[a]) * (1.0 / 6.0) + double(v1[a]) * (1.0 / 6.0) +
                            double(v2[a]) * (2.0 / 3.0));
    T J[9];
    if constexpr (PSI == GALS_PSI_SUPERCONSISTENT) {
        jacobian_chain<T, 3>(A0, A1, A2, T(dt), J);
    } else {
#pragma unroll
        for (int q = 0; q < 9; q++) J[q] = A0[q];
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
// row, so the row table is read once per wave through scalar loads.
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
    const unsigned blocks = unsigned((ctx->g.nodes + kBlock - 1) / kBlock + 7) / 8u * 8u;
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
    if (ctx->dim == 2) {
        if constexpr (KIND == GALS_VEL_AFFINE || KIND == GALS_VEL_STREAM_SIN ||
                      KIND == GALS_VEL_VORTEX || KIND == GALS_VEL_PSEUDO1D) {
            hipLaunchKernelGGL((k_step2d<T, KIND, MIX, PSI>), dim3(blocks), dim3(kBlock), 0, s,
                               ctx->g, p, st, dt, (const T *)phi, (const T *)grad, (T *)phi_o,
                               (T *)grad_o);
            return hipGetLastError();
        }
    } else {
        if constexpr (KIND == GALS_VEL_AFFINE || KIND == GALS_VEL_VECPOT_SIN ||
                      KIND == GALS_VEL_LEVEQUE3D) {
            hipLaunchKernelGGL((k_step3d<T, KIND, MIX, PSI>), dim3(blocks), dim3(kBlock), 0, s,
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
