// Sine stream-function fields in 2D, s = sum_{m,n} S[m][n] sin(m pi x) sin(n pi y):
// per-column / per-row tables, the per-node jet and its Taylor stages, and the
// whole GA-CIR step for one node. Shared by the single-grid and the batched
// kernels so that both do identical per-node arithmetic.
#pragma once

#include "hermite.h"

namespace gals {

// The field is separable, so every derivative at a node is a short dot
// product of a per-column and a per-row table:
//   coltab[i][a][n] = sum_m S[m][n] (m pi)^a sin^(a)(m pi x_i)
//   rowtab[j][b][n] = (n pi)^b sin^(b)(n pi y_j)
//   d^a/dx^a d^b/dy^b s(x_i, y_j) = sum_n coltab[i][a][n] rowtab[j][b][n]
// with sin^(a) = sin, cos, -sin, -cos, sin for a = 0..4; entries kJetTaylor
// and kJetTaylor + 1 hold sin(pi x_i), cos(pi x_i) (sin(pi y_j), cos(pi y_j)
// in a row), for the stages evaluated by the modal sum. Entries are built in
// FP64 and rounded to T. id < n[0]: column id; n[0] <= id < n[0]+n[1]: row.
template <typename T>
__device__ __forceinline__ void stream_table_entry(const Geom &g, const double (&S)[4][4], int id,
                                                   T *__restrict__ coltab, T *__restrict__ rowtab)
{
    const int nx = g.n[0], ny = g.n[1];
    if (id < nx) {
        const double x = node_coord(g.lo[0], id, g.h[0]);
        double s[4], c[4];
        for (int m = 0; m < 4; m++) sincospi(double(m + 1) * x, &s[m], &c[m]);
        for (int a = 0; a < 5; a++)
            for (int n = 0; n < 4; n++) {
                double u = 0.0;
                for (int m = 0; m < 4; m++) {
                    const double k = (m + 1) * kPi;
                    double f = (a & 1) ? c[m] : s[m];
                    if (a & 2) f = -f;
                    double ka = 1.0;
                    for (int q = 0; q < a; q++) ka *= k;
                    u += S[m][n] * ka * f;
                }
                coltab[int64_t(id) * kJet + 4 * a + n] = T(u);
            }
        T *raw = coltab + int64_t(id) * kJet + kJetTaylor;
        raw[0] = T(s[0]);
        raw[1] = T(c[0]);
        raw[2] = raw[3] = T(0);
    } else if (id < nx + ny) {
        const int j = id - nx;
        const double y = node_coord(g.lo[1], j, g.h[1]);
        for (int n = 0; n < 4; n++) {
            double s, c;
            sincospi(double(n + 1) * y, &s, &c);
            const double k = (n + 1) * kPi;
            double kb = 1.0;
            for (int b = 0; b < 5; b++) {
                double f = (b & 1) ? c : s;
                if (b & 2) f = -f;
                rowtab[int64_t(j) * kJet + 4 * b + n] = T(kb * f);
                kb *= k;
            }
        }
        double s1, c1;
        sincospi(y, &s1, &c1);
        T *raw = rowtab + int64_t(j) * kJet + kJetTaylor;
        raw[0] = T(s1);
        raw[1] = T(c1);
        raw[2] = raw[3] = T(0);
    }
}

template <typename T>
__device__ __forceinline__ T dot4(const T *u, const T *y)
{
    return u[0] * y[0] + u[1] * y[1] + u[2] * y[2] + u[3] * y[3];
}

// The 4-jet of s at a node for Taylor evaluation at an offset (dx, dy):
// degree 3 for the velocity (-s_y, s_x), degree 2 for its derivatives.
template <typename T>
struct StreamJet {
    T d10, d01, d20, d11, d02, d30, d21, d12, d03, d40, d31, d22, d13, d04;
};

// Orders 1..3 of the jet (u, y: a node's column and row table entries of
// orders 0..3), and order 4 (entries of orders 0..4).
template <typename T>
__device__ __forceinline__ void stream_jet3(const T *u, const T *y, StreamJet<T> &J)
{
    J.d10 = dot4(u + 4, y);
    J.d01 = dot4(u, y + 4);
    J.d20 = dot4(u + 8, y);
    J.d11 = dot4(u + 4, y + 4);
    J.d02 = dot4(u, y + 8);
    J.d30 = dot4(u + 12, y);
    J.d21 = dot4(u + 8, y + 4);
    J.d12 = dot4(u + 4, y + 8);
    J.d03 = dot4(u, y + 12);
}

template <typename T>
__device__ __forceinline__ void stream_jet4(const T *u, const T *y, StreamJet<T> &J)
{
    J.d40 = dot4(u + 16, y);
    J.d31 = dot4(u + 12, y + 4);
    J.d22 = dot4(u + 8, y + 8);
    J.d13 = dot4(u + 4, y + 12);
    J.d04 = dot4(u, y + 16);
}

// (s_x, s_y) to degree 2 and (s_xx, s_xy, s_yy) to degree 1 at offset
// (dx, dy): only the jet of order 3 enters. Used while kx |dx| + ky |dy| <=
// kTaylorMax2, where the dropped terms stay below FP32 rounding.
template <typename T>
__device__ __forceinline__ void stream_taylor2(const StreamJet<T> &J, T dx, T dy, T &sx, T &sy,
                                               T &sxx, T &sxy, T &syy)
{
    const T hx = T(0.5) * dx, hy = T(0.5) * dy;
    sx = J.d10 + dx * (J.d20 + hx * J.d30 + dy * J.d21) + dy * (J.d11 + hy * J.d12);
    sy = J.d01 + dx * (J.d11 + hx * J.d21 + dy * J.d12) + dy * (J.d02 + hy * J.d03);
    sxx = J.d20 + dx * J.d30 + dy * J.d21;
    sxy = J.d11 + dx * J.d21 + dy * J.d12;
    syy = J.d02 + dx * J.d12 + dy * J.d03;
}

// (s_x, s_y, s_xx, s_xy, s_yy) at offset (dx, dy) from the node, each
// Taylor polynomial in nested (Horner) form. The factorials go into the
// offsets (hx = dx/2, tx = dx/3, likewise in y), so the jet is used as built:
// e.g. s_x = d10 + dx d20 + dx^2 d30/2 + dx^3 d40/6 + ... with
// dx^2 d30/2 + dx^3 d40/6 = dx hx (d30 + d40 tx).
template <typename T>
__device__ __forceinline__ void stream_taylor(const StreamJet<T> &J, T dx, T dy, T &sx, T &sy,
                                              T &sxx, T &sxy, T &syy)
{
    const T hx = T(0.5) * dx, hy = T(0.5) * dy;
    const T tx = T(1.0 / 3.0) * dx, ty = T(1.0 / 3.0) * dy;
    sx = J.d10 + dx * (J.d20 + hx * (J.d30 + J.d40 * tx + J.d31 * dy)) +
         dy * (J.d11 + dx * (J.d21 + J.d22 * hy) + hy * (J.d12 + J.d13 * ty));
    sy = J.d01 + dx * (J.d11 + hx * (J.d21 + J.d31 * tx + J.d22 * dy)) +
         dy * (J.d02 + dx * (J.d12 + J.d13 * hy) + hy * (J.d03 + J.d04 * ty));
    sxx = J.d20 + dx * (J.d30 + J.d40 * hx + J.d31 * dy) + dy * (J.d21 + J.d22 * hy);
    sxy = J.d11 + dx * (J.d21 + J.d31 * hx + J.d22 * dy) + dy * (J.d12 + J.d13 * hy);
    syy = J.d02 + dx * (J.d12 + J.d22 * hx + J.d13 * dy) + dy * (J.d03 + J.d04 * hy);
}

// Velocity and its Jacobian at node + (dx, dy) without the time factor: the Taylor
// polynomial of the node's jet when its truncation stays below FP32 rounding
// (kx |dx| + ky |dy| <= kTaylorMax), the exact modal sum otherwise (and
// always in FP64). P carries the stream table S and kx, ky. In the modal
// sum, sin and cos of the stage point's angles come from the node's (entries
// kJetTaylor.. of its table rows U, Y) by angle addition with the long series
// when the offset allows (|pi d| <= 0.1 in FP64, 0.25 in FP32: every stage
// of a step at CFL ~1 on grids of 32 or more cells), else from sincospi.
template <typename T, bool TAYLOR, class P>
__device__ __forceinline__ void stream_stage(const P &p, const StreamJet<T> &J,
                                             const T *__restrict__ U, const T *__restrict__ Y,
                                             const Geom &g, int i, int j, double x0,
                                             double y0, T dx, T dy, T *v, T *A)
{
    if (TAYLOR && p.kx * fabs(dx) + p.ky * fabs(dy) <= T(kTaylorMax)) {
        T sx, sy, sxx, sxy, syy;
        stream_taylor(J, dx, dy, sx, sy, sxx, sxy, syy);
        from_stream(sx, sy, sxx, sxy, syy, T(1), v, A);
    } else {
        T s1x, c1x, s1y, c1y;  // sin and cos of pi x and pi y at the stage point
        constexpr T dmax = T(kShiftMaxLong<T> / kPi);
        if (fabs(dx) <= dmax && fabs(dy) <= dmax) {
            shifted_sincos_long(U[kJetTaylor], U[kJetTaylor + 1], dx, s1x, c1x);
            shifted_sincos_long(Y[kJetTaylor], Y[kJetTaylor + 1], dy, s1y, c1y);
        } else {
            // FP32 forms the node's coordinates only here, off the common path
            // (x0, y0 unused); FP64 passes them in (forming them here would
            // cost it scalar-register spills)
            if constexpr (sizeof(T) == 4) {
                x0 = node_coord(g.lo[0], i, g.h[0]);
                y0 = node_coord(g.lo[1], j, g.h[1]);
            }
            sincospi_t(T(x0 + double(dx)), &s1x, &c1x);
            sincospi_t(T(y0 + double(dy)), &s1y, &c1y);
        }
        stream_modes_from(p, s1x, c1x, s1y, c1y, T(1), v, A);
    }
}

// The characteristic trace of node (i, j) for a sine stream-function field
// (the forward step and its adjoint both start from it): the stage
// velocities and velocity Jacobians, the offsets of the stage points from the
// node, the superconsistent Jacobian J of the foot map, and the foot after
// the boundary treatment, split into a cell and a local coordinate.
template <typename T>
struct StreamFoot {
    StreamJet<T> jet;
    T v0[2], v1[2], v2[2], A0[4], A1[4], A2[4], J[4];
    T d1[2], d2[2];  // stage-2 and stage-3 points minus the node
    unsigned out;    // bit a: the foot left the domain along axis a (Neumann)
    bool outb[2];    // the same as flags
    int cell[2];
    T xi[2];         // local coordinate in the cell
    double s[2];     // the foot in cell units, after the boundary treatment
};

// CHAIN = false (Heun's gradient update) skips the Jacobian chain (J unset).
template <typename T, bool TAYLOR, bool CHAIN = true, class P>
__device__ __forceinline__ void stream_trace(const Geom &g, const P &p, const Stage<T> &st,
                                             double dt, const T *__restrict__ U,
                                             const T *__restrict__ Y, int i, int j,
                                             StreamFoot<T> &f)
{
    StreamJet<T> &jet = f.jet;
    {
        T y[16], u[16];
#pragma unroll
        for (int k = 0; k < 16; k++) {
            y[k] = Y[k];
            u[k] = U[k];
        }
        stream_jet3(u, y, jet);
    }
    jet.d40 = jet.d31 = jet.d22 = jet.d13 = jet.d04 = T(0);
    // the order-4 jet, for the lanes whose stages need it
    auto order4 = [&]() {
        T y[kJetTaylor], u[kJetTaylor];
#pragma unroll
        for (int k = 0; k < kJetTaylor; k++) {
            y[k] = Y[k];
            u[k] = U[k];
        }
        stream_jet4(u, y, jet);
    };
    const double x0 = sizeof(T) == 8 ? node_coord(g.lo[0], i, g.h[0]) : 0.0;
    const double y0 = sizeof(T) == 8 ? node_coord(g.lo[1], j, g.h[1]) : 0.0;
    // w_k, R_k: velocity and velocity Jacobian at stage k without the time
    // factor c_k (Stage carries dt c_k in its weights)
    T w0[2], R0[4], w1[2], R1[4], w2[2], R2[4];
    // stage 1 at the node, time t + dt
    from_stream(jet.d10, jet.d01, jet.d20, jet.d11, jet.d02, T(1), w0, R0);
    // stage 2 at x1 = x - dt v0, time t; a lane whose stage offsets are tiny
    // takes the degree-2 polynomial from the order-3 jet, the others the
    // order-4 jet and stream_stage
    f.d1[0] = -st.e1 * w0[0];
    f.d1[1] = -st.e1 * w0[1];
    const bool low1 = TAYLOR && p.kx * fabs(f.d1[0]) + p.ky * fabs(f.d1[1]) <= T(kTaylorMax2);
    if (!low1) order4();
    if (low1) {
        T sx, sy, sxx, sxy, syy;
        stream_taylor2(jet, f.d1[0], f.d1[1], sx, sy, sxx, sxy, syy);
        from_stream(sx, sy, sxx, sxy, syy, T(1), w1, R1);
    } else {
        stream_stage<T, TAYLOR>(p, jet, U, Y, g, i, j, x0, y0, f.d1[0], f.d1[1], w1, R1);
    }
    // stage 3 at x2 = x - dt (v0 + v1) / 4, time t + dt/2
    f.d2[0] = -(st.q1 * w0[0] + st.q2 * w1[0]);
    f.d2[1] = -(st.q1 * w0[1] + st.q2 * w1[1]);
    const bool low2 = TAYLOR && p.kx * fabs(f.d2[0]) + p.ky * fabs(f.d2[1]) <= T(kTaylorMax2);
    if (low1 && !low2) order4();  // the order-4 jet was not needed until now
    if (low2) {
        T sx, sy, sxx, sxy, syy;
        stream_taylor2(jet, f.d2[0], f.d2[1], sx, sy, sxx, sxy, syy);
        from_stream(sx, sy, sxx, sxy, syy, T(1), w2, R2);
    } else {
        stream_stage<T, TAYLOR>(p, jet, U, Y, g, i, j, x0, y0, f.d2[0], f.d2[1], w2, R2);
    }
#pragma unroll
    for (int a = 0; a < 2; a++) {
        f.v0[a] = st.c1 * w0[a];
        f.v1[a] = st.c2 * w1[a];
        f.v2[a] = st.c3 * w2[a];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        f.A0[k] = st.c1 * R0[k];
        f.A1[k] = st.c2 * R1[k];
        f.A2[k] = st.c3 * R2[k];
    }
    if constexpr (CHAIN) jacobian_chain_w<T, 2>(R0, R1, R2, st, f.J);

    // foot in cell units: s = node - dt (v0/6 + v1/6 + 2 v2/3) / h, the
    // displacement summed in T from the T velocities (its rounding is of the
    // order of theirs), the position in FP64
    double s[2];
#pragma unroll
    for (int a = 0; a < 2; a++)
        s[a] = double(a == 0 ? i : j) -
               double(st.f1 * w0[a] + st.f2 * w1[a] + st.f3 * w2[a]) * g.inv_h[a];
    f.out = 0;
#pragma unroll
    for (int a = 0; a < 2; a++) {
        // outside only beyond kFootTol cells (project_foot); the cell index
        // is clamped to [0, nc-1], the local coordinate is not, except for
        // a foot outside, which is projected onto the boundary
        const bool below = s[a] < g.lowc[a], above = s[a] > g.outc[a];
        const double fl = fmin(fmax(floor(s[a]), 0.0), g.lastc[a]);
        f.cell[a] = int(fl);
        T xi = T(s[a] - fl);
        xi = below ? T(0) : xi;
        f.xi[a] = above ? T(1) : xi;
        f.outb[a] = below || above;
        f.out |= unsigned(below || above) << a;
        f.s[a] = below ? 0.0 : above ? g.ncd[a] : s[a];
    }
}

// The part of a stream-function step after the trace and the gather: the
// bicubic, the boundary treatment of its gradient, and the update
// (superconsistent, or Heun's method with grad v at the foot from the node's
// jet) into the output planes.
template <typename T, bool TAYLOR, int PSI, class P>
__device__ __forceinline__ void stream_finish(const Geom &g, const P &p, const Stage<T> &st,
                                              double dt, const T *__restrict__ U,
                                              const T *__restrict__ Y, const StreamFoot<T> &f,
                                              const T (&d)[4][4], T *__restrict__ phi_o,
                                              T *__restrict__ gx_o, T *__restrict__ gy_o, int i,
                                              int j)
{
    Basis<T> bx, by;
    basis<T, false>(T(f.xi[0]), geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
    basis<T, false>(T(f.xi[1]), geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
    T H, Hx, Hy;
    hermite2d(d, bx, by, H, Hx, Hy);
    if (f.outb[0]) Hx = T(0);
    if (f.outb[1]) Hy = T(0);

    const unsigned o = unsigned(j) * unsigned(g.pitch) + unsigned(i);
    pstore(phi_o, o, H);
    if constexpr (PSI == GALS_PSI_HEUN) {
        T vf[2], Af[4], ps[2];
        const T gH[2] = {Hx, Hy};
        stream_stage<T, TAYLOR>(p, f.jet, U, Y, g, i, j, node_coord(g.lo[0], i, g.h[0]),
                                node_coord(g.lo[1], j, g.h[1]), T((f.s[0] - double(i)) * g.h[0]),
                                T((f.s[1] - double(j)) * g.h[1]), vf, Af);
#pragma unroll
        for (int k = 0; k < 4; k++) Af[k] *= st.c2;
        heun_gradient<T, 2>(Af, f.A0, T(dt), gH, ps);
        pstore(gx_o, o, ps[0]);
        pstore(gy_o, o, ps[1]);
    } else {
        pstore(gx_o, o, f.J[0] * Hx + f.J[2] * Hy);
        pstore(gy_o, o, f.J[1] * Hx + f.J[3] * Hy);
    }
}

// One GA-CIR step at node (i, j) of a grid with a sine stream-function field:
// the trace, the gather from global memory and the bicubic update.
template <typename T, int MIX, bool TAYLOR, int PSI = GALS_PSI_SUPERCONSISTENT, class P>
__device__ __forceinline__ void stream_node(const Geom &g, const P &p, const Stage<T> &st,
                                            double dt, const T *__restrict__ U,
                                            const T *__restrict__ Y,
                                            const T *__restrict__ phi, const T *__restrict__ gx,
                                            const T *__restrict__ gy, T *__restrict__ phi_o,
                                            T *__restrict__ gx_o, T *__restrict__ gy_o, int i,
                                            int j)
{
    StreamFoot<T> f;
    stream_trace<T, TAYLOR, PSI == GALS_PSI_SUPERCONSISTENT>(g, p, st, dt, U, Y, i, j, f);
    T d[4][4];
    // buffer resources made here, not before the trace, so that they are not
    // held in scalar registers across it
    gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(gx, g.plane),
                     plane_rsrc(gy, g.plane), f.cell[0], f.cell[1], d);
    stream_finish<T, TAYLOR, PSI>(g, p, st, dt, U, Y, f, d, phi_o, gx_o, gy_o, i, j);
}

// Workgroups are dealt to the 8 XCDs round-robin by id, and each XCD has its
// own L2. Give XCD x a contiguous band of the 64 x 4 node tiles (walked row
// group by row group) so the halo rows a tile gathers were just fetched into
// the same L2 by its neighbours. Returns false for ids past the last tile.
// The division by tiles_x is a scalar multiply-high by the host's
// floor(2^32 / tiles_x) and one correction (exact for every 32-bit t).
__device__ __forceinline__ bool xcd_tile(const Geom &g, unsigned &tx, unsigned &ty)
{
    const unsigned per = (g.tiles + 7u) / 8u;
    const unsigned t = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
    unsigned q = __umulhi(t, g.tiles_x_magic);
    unsigned r = t - q * g.tiles_x;
    if (r >= g.tiles_x) {
        q += 1u;
        r -= g.tiles_x;
    }
    tx = r;
    ty = q;
    return t < g.tiles;
}

// The same for kernels over a flat node range in blocks of kBlock nodes:
// XCD x walks a contiguous band of blocks. The grid is rounded up to a
// multiple of 8; returns false for ids past the last block.
__device__ __forceinline__ bool xcd_block(unsigned blocks, unsigned &b)
{
    const unsigned per = (blocks + 7u) / 8u;
    b = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
    return b < blocks;
}

}  // namespace gals
