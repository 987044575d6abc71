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

// The 4-jet of s at a node, pre-scaled for Taylor evaluation at an offset
// (dx, dy): degree 3 for the velocity (-s_y, s_x), degree 2 for its
// derivatives. a.. = d../2, t.. = d../6.
template <typename T>
struct StreamJet {
    T d10, d01, d20, d11, d02, d30, d21, d12, d03;
    T a30, a12, a21, a03, a40, a31, a22, a13, a04, t40, t13, t31, t04;
};

template <typename T>
__device__ __forceinline__ void stream_jet(const T *u, const T *y, StreamJet<T> &J)
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
    const T d40 = dot4(u + 16, y), d31 = dot4(u + 12, y + 4), d22 = dot4(u + 8, y + 8);
    const T d13 = dot4(u + 4, y + 12), d04 = dot4(u, y + 16);
    const T half = T(0.5), sixth = T(1.0 / 6.0);
    J.a30 = half * J.d30; J.a12 = half * J.d12; J.a21 = half * J.d21; J.a03 = half * J.d03;
    J.a40 = half * d40; J.a31 = half * d31; J.a22 = half * d22; J.a13 = half * d13;
    J.a04 = half * d04;
    J.t40 = sixth * d40; J.t13 = sixth * d13; J.t31 = sixth * d31; J.t04 = sixth * d04;
}

// (s_x, s_y, s_xx, s_xy, s_yy) at offset (dx, dy) from the node, each
// Taylor polynomial in nested (Horner) form.
template <typename T>
__device__ __forceinline__ void stream_taylor(const StreamJet<T> &J, T dx, T dy, T &sx, T &sy,
                                              T &sxx, T &sxy, T &syy)
{
    // s_x: d10 + dx (d20 + dx (a30 + t40 dx + a31 dy)) + dy (d11 + dx (d21 + a22 dy) + dy (a12 + t13 dy))
    sx = J.d10 + dx * (J.d20 + dx * (J.a30 + J.t40 * dx + J.a31 * dy)) +
         dy * (J.d11 + dx * (J.d21 + J.a22 * dy) + dy * (J.a12 + J.t13 * dy));
    // s_y: d01 + dx (d11 + dx (a21 + t31 dx + a22 dy)) + dy (d02 + dx (d12 + a13 dy) + dy (a03 + t04 dy))
    sy = J.d01 + dx * (J.d11 + dx * (J.a21 + J.t31 * dx + J.a22 * dy)) +
         dy * (J.d02 + dx * (J.d12 + J.a13 * dy) + dy * (J.a03 + J.t04 * dy));
    // second derivatives, degree 2: c0 + dx (cx + cxx dx + cxy dy) + dy (cy + cyy dy)
    sxx = J.d20 + dx * (J.d30 + J.a40 * dx + T(2) * J.a31 * dy) + dy * (J.d21 + J.a22 * dy);
    sxy = J.d11 + dx * (J.d21 + J.a31 * dx + T(2) * J.a22 * dy) + dy * (J.d12 + J.a13 * dy);
    syy = J.d02 + dx * (J.d12 + J.a22 * dx + T(2) * J.a13 * dy) + dy * (J.d03 + J.a04 * dy);
}

// Velocity and its Jacobian at node + (dx, dy), stage factor c: the Taylor
// polynomial of the node's jet when its truncation stays below FP32 rounding
// (kx |dx| + ky |dy| <= kTaylorMax), the exact modal sum otherwise (and
// always in FP64). P carries the stream tables S, SQ, SR and kx, ky.
// Otherwise the modal sum; in FP64, sin and cos of the stage point's angles
// come from the node's (entries kJetTaylor.. of its table rows U, Y) by angle
// addition when the offset allows (FP32 keeps sincospi there: the branch is
// rare, and the extra registers would cost the batched kernel a spill).
template <typename T, bool TAYLOR, class P>
__device__ __forceinline__ void stream_stage(const P &p, const StreamJet<T> &J,
                                             const T *__restrict__ U, const T *__restrict__ Y,
                                             double x0, double y0, T dx, T dy, T c, T *v, T *A)
{
    if (TAYLOR && p.kx * fabs(dx) + p.ky * fabs(dy) <= T(kTaylorMax)) {
        T sx, sy, sxx, sxy, syy;
        stream_taylor(J, dx, dy, sx, sy, sxx, sxy, syy);
        from_stream(sx, sy, sxx, sxy, syy, c, v, A);
    } else {
        T sx[4], cx[4], sy[4], cy[4];
        constexpr T dmax = T(kShiftMaxLong<T> / kPi);
        if (sizeof(T) == 8 && fabs(dx) <= dmax && fabs(dy) <= dmax) {
            T s, cs;
            shifted_sincos_long(U[kJetTaylor], U[kJetTaylor + 1], dx, s, cs);
            multiples_from(s, cs, sx, cx);
            shifted_sincos_long(Y[kJetTaylor], Y[kJetTaylor + 1], dy, s, cs);
            multiples_from(s, cs, sy, cy);
        } else {
            sincos_multiples(T(x0 + double(dx)), sx, cx);
            sincos_multiples(T(y0 + double(dy)), sy, cy);
        }
        stream_modes(p, sx, cx, sy, cy, c, v, A);
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
    int cell[2];
    double xi[2];
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
        T y[kJetTaylor], u[kJetTaylor];
#pragma unroll
        for (int k = 0; k < kJetTaylor; k++) {
            y[k] = Y[k];
            u[k] = U[k];
        }
        stream_jet(u, y, jet);
    }
    const double x0 = node_coord(g.lo[0], i, g.h[0]), y0 = node_coord(g.lo[1], j, g.h[1]);
    const T dtT = T(dt);
    // stage 1 at the node, time t + dt
    from_stream(jet.d10, jet.d01, jet.d20, jet.d11, jet.d02, st.c1, f.v0, f.A0);
    // stage 2 at x1 = x - dt v0, time t
    f.d1[0] = -dtT * f.v0[0];
    f.d1[1] = -dtT * f.v0[1];
    stream_stage<T, TAYLOR>(p, jet, U, Y, x0, y0, f.d1[0], f.d1[1], st.c2, f.v1, f.A1);
    // stage 3 at x2 = x - dt (v0 + v1) / 4, time t + dt/2
    f.d2[0] = -dtT * (T(0.25) * f.v0[0] + T(0.25) * f.v1[0]);
    f.d2[1] = -dtT * (T(0.25) * f.v0[1] + T(0.25) * f.v1[1]);
    stream_stage<T, TAYLOR>(p, jet, U, Y, x0, y0, f.d2[0], f.d2[1], st.c3, f.v2, f.A2);
    if constexpr (CHAIN) jacobian_chain<T, 2>(f.A0, f.A1, f.A2, dtT, f.J);

    // foot in cell units, FP64: s = node - dt (v0/6 + v1/6 + 2 v2/3) / h
    double s[2];
    s[0] = double(i) - dt * (double(f.v0[0]) * (1.0 / 6.0) + double(f.v1[0]) * (1.0 / 6.0) +
                             double(f.v2[0]) * (2.0 / 3.0)) * g.inv_h[0];
    s[1] = double(j) - dt * (double(f.v0[1]) * (1.0 / 6.0) + double(f.v1[1]) * (1.0 / 6.0) +
                             double(f.v2[1]) * (2.0 / 3.0)) * g.inv_h[1];
    f.out = 0;
#pragma unroll
    for (int a = 0; a < 2; a++) {
        if (g.bc == GALS_BC_NEUMANN) {
            // outside only beyond kFootTol cells (project_foot)
            if (s[a] < -kFootTol) { s[a] = 0.0; f.out |= 1u << a; }
            else if (s[a] > double(g.nc[a]) + kFootTol) { s[a] = double(g.nc[a]); f.out |= 1u << a; }
        }
        // cell index clamped to [0, nc-1], local coordinate unclamped
        const double fl = fmin(fmax(floor(s[a]), 0.0), double(g.nc[a] - 1));
        f.cell[a] = int(fl);
        f.xi[a] = s[a] - fl;
        f.s[a] = s[a];
    }
}

// One GA-CIR step at node (i, j) of a grid with a sine stream-function field:
// the trace, the gather and the bicubic update (superconsistent, or Heun's
// method with grad v at the foot from the node's jet).
template <typename T, int MIX, bool TAYLOR, int PSI = GALS_PSI_SUPERCONSISTENT, class P>
__device__ __forceinline__ void stream_node(const Geom &g, const P &p, const Stage<T> &st,
                                            double dt, const T *__restrict__ U,
                                            const T *__restrict__ Y, Rsrc rphi, Rsrc rgx,
                                            Rsrc rgy, T *__restrict__ phi_o,
                                            T *__restrict__ gx_o, T *__restrict__ gy_o, int i,
                                            int j)
{
    StreamFoot<T> f;
    stream_trace<T, TAYLOR, PSI == GALS_PSI_SUPERCONSISTENT>(g, p, st, dt, U, Y, i, j, f);
    T d[4][4];
    gather2d<T, MIX>(g, rphi, rgx, rgy, f.cell[0], f.cell[1], d);
    Basis<T> bx, by;
    basis<T, false>(T(f.xi[0]), T(g.h[0]), T(g.inv_h[0]), bx);
    basis<T, false>(T(f.xi[1]), T(g.h[1]), T(g.inv_h[1]), by);
    T H, Hx, Hy;
    hermite2d(d, bx, by, H, Hx, Hy);
    if (f.out & 1u) Hx = T(0);
    if (f.out & 2u) Hy = T(0);

    const int64_t o = int64_t(j) * g.pitch + i;
    phi_o[o] = H;
    if constexpr (PSI == GALS_PSI_HEUN) {
        const double x0 = node_coord(g.lo[0], i, g.h[0]), y0 = node_coord(g.lo[1], j, g.h[1]);
        T vf[2], Af[4], ps[2];
        const T gH[2] = {Hx, Hy};
        stream_stage<T, TAYLOR>(p, f.jet, U, Y, x0, y0, T((f.s[0] - double(i)) * g.h[0]),
                                T((f.s[1] - double(j)) * g.h[1]), st.c2, vf, Af);
        heun_gradient<T, 2>(Af, f.A0, T(dt), gH, ps);
        gx_o[o] = ps[0];
        gy_o[o] = ps[1];
    } else {
        gx_o[o] = f.J[0] * Hx + f.J[2] * Hy;
        gy_o[o] = f.J[1] * Hx + f.J[3] * Hy;
    }
}

// Workgroups are dealt to the 8 XCDs round-robin by id, and each XCD has its
// own L2. Give XCD x a contiguous band of tiles (walked row group by row
// group) so the halo rows a tile gathers were just fetched into the same L2
// by its neighbours. Returns false for ids past the last tile.
__device__ __forceinline__ bool xcd_tile(unsigned tiles_x, unsigned tiles, unsigned &tx,
                                         unsigned &ty)
{
    const unsigned per = (tiles + 7u) / 8u;
    const unsigned t = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
    tx = t % tiles_x;
    ty = t / tiles_x;
    return t < tiles;
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
