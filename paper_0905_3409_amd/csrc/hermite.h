// Device building blocks of one GA-CIR step: the superconsistent Shu-Osher
// trace, the FP64 cell split, the cell gather with on-the-fly central cross
// derivatives, and the bi-/tri-cubic Hermite evaluation.
#pragma once

#include "velocity.h"

namespace gals {

// ---------------------------------------------------------------------------
// Superconsistent Shu-Osher trace (sec. 5.1, Ex. ex:superconsistent_ShuOsher).
// Positions are FP64; velocities and the Jacobian chain are in T. J is the
// Jacobian of the foot map in J form, J[i*D+j] = dX_i/dx_j, so the gradient
// update of eq. (superconsistency) is psi_new = J^T grad H.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void matmul_acc(const T *A, const T *B, T *C)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            T s = A[i * D] * B[j];
#pragma unroll
            for (int k = 1; k < D; k++) s += A[i * D + k] * B[k * D + j];
            C[i * D + j] = s;
        }
}

// Superconsistent Jacobian of the Shu-Osher foot map from the velocity
// Jacobians A0, A1, A2 at the three stage points (J form):
// J1 = I - dt A0; J2 = I - dt (A0/4 + A1 J1 / 4);
// J = I - dt (A0/6 + A1 J1 / 6 + 2 A2 J2 / 3).
template <typename T, int D>
__device__ __forceinline__ void jacobian_chain(const T *A0, const T *A1, const T *A2, T dtT, T *J)
{
    T J1[D * D], B1[D * D], J2[D * D], B2[D * D];
#pragma unroll
    for (int k = 0; k < D * D; k++) J1[k] = T((k % (D + 1)) == 0) - dtT * A0[k];
    matmul_acc<T, D>(A1, J1, B1);
#pragma unroll
    for (int k = 0; k < D * D; k++)
        J2[k] = T((k % (D + 1)) == 0) - dtT * (T(0.25) * A0[k] + T(0.25) * B1[k]);
    matmul_acc<T, D>(A2, J2, B2);
#pragma unroll
    for (int k = 0; k < D * D; k++)
        J[k] = T((k % (D + 1)) == 0) -
               dtT * (A0[k] * T(1.0 / 6.0) + B1[k] * T(1.0 / 6.0) + B2[k] * T(2.0 / 3.0));
}

// The same chain from the stage Jacobians without their time factors,
// R_k = A_k / c_k, with dt c_k folded into the weights of Stage:
// J1 = I - e1 R0; J2 = I - q1 R0 - q2 R1 J1; J = I - f1 R0 - f2 R1 J1 - f3 R2 J2.
template <typename T, int D>
__device__ __forceinline__ void jacobian_chain_w(const T *R0, const T *R1, const T *R2,
                                                 const Stage<T> &st, T *J)
{
    T J1[D * D], P1[D * D], J2[D * D], P2[D * D];
#pragma unroll
    for (int k = 0; k < D * D; k++) J1[k] = T((k % (D + 1)) == 0) - st.e1 * R0[k];
    matmul_acc<T, D>(R1, J1, P1);
#pragma unroll
    for (int k = 0; k < D * D; k++) J2[k] = T((k % (D + 1)) == 0) - st.q1 * R0[k] - st.q2 * P1[k];
    matmul_acc<T, D>(R2, J2, P2);
#pragma unroll
    for (int k = 0; k < D * D; k++)
        J[k] = T((k % (D + 1)) == 0) - st.f1 * R0[k] - st.f2 * P1[k] - st.f3 * P2[k];
}

// CHAIN = false (Heun's gradient update) skips the Jacobian chain; J then
// receives A0, the velocity Jacobian at the node at time t + dt.
template <typename T, int D, int KIND, bool CHAIN = true>
__device__ __forceinline__ void trace(const Vel<T> &p, const Stage<T> &st, double dt,
                                      const double *x, double *X, T *J)
{
    T v0[D], A0[D * D], v1[D], A1[D * D], v2[D], A2[D * D];
    double x1[D], x2[D];
    const T dtT = T(dt);
    // stage 1: v(x, t+dt)
    velocity<T, D, KIND>(p, x, st.c1, v0, A0);
#pragma unroll
    for (int i = 0; i < D; i++) x1[i] = x[i] - dt * double(v0[i]);
    // stage 2: v(x1, t)
    velocity<T, D, KIND>(p, x1, st.c2, v1, A1);
#pragma unroll
    for (int i = 0; i < D; i++) x2[i] = x[i] - dt * (0.25 * double(v0[i]) + 0.25 * double(v1[i]));
    // stage 3: v(x2, t+dt/2)
    velocity<T, D, KIND>(p, x2, st.c3, v2, A2);
#pragma unroll
    for (int i = 0; i < D; i++)
        X[i] = x[i] - dt * (double(v0[i]) * (1.0 / 6.0) + double(v1[i]) * (1.0 / 6.0) +
                            double(v2[i]) * (2.0 / 3.0));
    if constexpr (CHAIN) {
        jacobian_chain<T, D>(A0, A1, A2, dtT, J);
    } else {
#pragma unroll
        for (int k = 0; k < D * D; k++) J[k] = A0[k];
    }
}

// Heun's method for d psi/d tau = -grad v . psi (eq. cir_evolution_psi)
// from the foot (time t, velocity Jacobian Af) to the node (time t + dt,
// An), J form (A[i][j] = dv_i/dx_j, so grad v . psi = A^T psi):
// k1 = -Af^T g, k2 = -An^T (g + dt k1), psi = g + dt (k1 + k2) / 2.
template <typename T, int D>
__device__ __forceinline__ void heun_gradient(const T *Af, const T *An, T dtT, const T *g, T *psi)
{
    T k1[D], pp[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        T s = Af[i] * g[0];
#pragma unroll
        for (int j = 1; j < D; j++) s += Af[j * D + i] * g[j];
        k1[i] = -s;
    }
#pragma unroll
    for (int i = 0; i < D; i++) pp[i] = g[i] + dtT * k1[i];
#pragma unroll
    for (int i = 0; i < D; i++) {
        T s = An[i] * pp[0];
#pragma unroll
        for (int j = 1; j < D; j++) s += An[j * D + i] * pp[j];
        psi[i] = g[i] + T(0.5) * dtT * (k1[i] - s);
    }
}

// ---------------------------------------------------------------------------
// Homogeneous Neumann treatment of a foot outside the domain: project it onto
// the domain and remember the axes whose normal derivative must vanish. A
// foot counts as outside only when it lies more than kFootTol cells beyond
// the boundary; closer, it stays where it is (the boundary cell's cubic is
// evaluated there), so that a foot within rounding of the boundary, e.g. of a
// node on a face the flow runs along, is not decided by that rounding.
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ unsigned project_foot(const Geom &g, double *X)
{
    unsigned out = 0;
    if (g.bc == GALS_BC_NEUMANN) {
#pragma unroll
        for (int a = 0; a < D; a++) {
            const double tol = kFootTol * g.h[a];
            if (X[a] < g.lo[a] - tol) {
                X[a] = g.lo[a];
                out |= 1u << a;
            } else if (X[a] > g.top[a] + tol) {
                X[a] = g.top[a];
                out |= 1u << a;
            }
        }
    }
    return out;
}

// ---------------------------------------------------------------------------
// Cell split in FP64: clamped cell index, unclamped local coordinate (a foot
// outside the grid evaluates the boundary cell's polynomial). Not-a-number
// feet land in cell 0 and propagate.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void split(const Geom &g, const double *X, int *cell, double *xi)
{
#pragma unroll
    for (int a = 0; a < D; a++) {
        const double s = (X[a] - g.lo[a]) * g.inv_h[a];
        const double fl = floor(s);
        const double top = double(g.nc[a] - 1);
        int c;
        if (fl >= 0.0 && fl <= top) c = int(fl);
        else if (fl > top) c = g.nc[a] - 1;
        else c = 0;
        cell[a] = c;
        xi[a] = s - double(c);
    }
}

// ---------------------------------------------------------------------------
// Raw buffer loads: one descriptor per plane (base, size in bytes), 32-bit
// element offsets, reads outside the plane return 0. The host keeps every
// plane below 2 GiB, so its size in bytes and every byte offset into it fit a
// signed 32-bit integer.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t Rsrc;

template <typename T>
__device__ __forceinline__ Rsrc plane_rsrc(const T *base, int64_t elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), 0, int(elems * int64_t(sizeof(T))),
                                             0x00020000);
}

__device__ __forceinline__ float bload(Rsrc r, unsigned elem, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, elem * 4u, 0, 0));
}

__device__ __forceinline__ double bload(Rsrc r, unsigned elem, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, elem * 8u, 0, 0));
}

// Store element `elem` of a plane through a 32-bit byte offset (every plane
// is below 2 GiB), so the address is the plane's scalar base plus one vector
// offset.
template <typename T>
__device__ __forceinline__ void pstore(T *base, unsigned elem, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + elem * unsigned(sizeof(T))) = v;
}

// ---------------------------------------------------------------------------
// Cross derivatives (sec. 2.3, approach (A)) at the two corners c, c+1 of a
// cell from samples u[0..3] at nodes c-1..c+2 (clamped into [0, N]): central
// differences inside, one-sided 3-point differences at node 0 and node N.
// ---------------------------------------------------------------------------
// WAVE: the one-sided forms are evaluated only by waves that hold an edge
// cell (a uniform branch; FP32 2D only: elsewhere the branch costs registers).
template <typename T, bool WAVE = false>
__device__ __forceinline__ void diff_pair(const T *u, bool lo_edge, bool hi_edge, T inv2h,
                                          T &d0, T &d1)
{
    T a = u[2] - u[0], b = u[3] - u[1];
    if (!WAVE || __builtin_amdgcn_ballot_w64(lo_edge || hi_edge)) {
        a = lo_edge ? T(4) * u[2] - T(3) * u[1] - u[3] : a;
        b = hi_edge ? T(3) * u[2] - T(4) * u[1] + u[0] : b;
    }
    d0 = a * inv2h;
    d1 = b * inv2h;
}

// Cross derivative by the cell-based approach (B) (sec. 2.3) on one cell
// facet spanned by axes a, b: ga = phi_a, gb = phi_b at the facet's vertices
// (index bit 0 along a, bit 1 along b). Differences along the four edges
// give the cross derivative at the edge centres; a vertex takes 3/4 of its
// two edges and -1/4 of the two opposite ones (bilinear extrapolation).
template <typename T>
__device__ __forceinline__ void cell_cross(const T *ga, const T *gb, T inv_ha, T inv_hb, T *out)
{
    const T ea0 = (ga[2] - ga[0]) * inv_hb, ea1 = (ga[3] - ga[1]) * inv_hb;  // edges along b
    const T eb0 = (gb[1] - gb[0]) * inv_ha, eb1 = (gb[3] - gb[2]) * inv_ha;  // edges along a
    out[0] = T(0.75) * (ea0 + eb0) - T(0.25) * (ea1 + eb1);
    out[1] = T(0.75) * (ea1 + eb0) - T(0.25) * (ea0 + eb1);
    out[2] = T(0.75) * (ea0 + eb1) - T(0.25) * (ea1 + eb0);
    out[3] = T(0.75) * (ea1 + eb1) - T(0.25) * (ea0 + eb0);
}

// Cell data d[v][alpha]: v = vertex bits (x = bit 0), alpha = derivative bits.
// 2D alpha: 0 phi, 1 psi_x, 2 psi_y, 3 phi_xy.
template <typename T, int MIX>
__device__ __forceinline__ void gather2d(const Geom &g, Rsrc rphi, Rsrc rgx, Rsrc rgy, int cx,
                                         int cy, T d[4][4])
{
    const unsigned r0 = unsigned(cy) * unsigned(g.pitch), r1 = r0 + unsigned(g.pitch);
    const unsigned i0 = unsigned(cx), i1 = unsigned(cx) + 1u;
    d[0][0] = bload(rphi, r0 + i0, T()); d[1][0] = bload(rphi, r0 + i1, T());
    d[2][0] = bload(rphi, r1 + i0, T()); d[3][0] = bload(rphi, r1 + i1, T());
    d[0][1] = bload(rgx, r0 + i0, T()); d[1][1] = bload(rgx, r0 + i1, T());
    d[2][1] = bload(rgx, r1 + i0, T()); d[3][1] = bload(rgx, r1 + i1, T());
    if constexpr (MIX == GALS_MIXED_CELL) {
        d[0][2] = bload(rgy, r0 + i0, T()); d[1][2] = bload(rgy, r0 + i1, T());
        d[2][2] = bload(rgy, r1 + i0, T()); d[3][2] = bload(rgy, r1 + i1, T());
        T ga[4], gb[4], out[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            ga[v] = d[v][1];
            gb[v] = d[v][2];
        }
        cell_cross(ga, gb, geo_ih<T>(g, 0), geo_ih<T>(g, 1), out);
#pragma unroll
        for (int v = 0; v < 4; v++) d[v][3] = out[v];
    } else if constexpr (MIX == GALS_MIXED_CENTRAL) {
        const unsigned im = unsigned(cx > 0 ? cx - 1 : 0);
        const unsigned i2 = unsigned(cx + 2 <= g.nc[0] ? cx + 2 : g.nc[0]);
        const T u0[4] = {bload(rgy, r0 + im, T()), bload(rgy, r0 + i0, T()),
                         bload(rgy, r0 + i1, T()), bload(rgy, r0 + i2, T())};
        const T u1[4] = {bload(rgy, r1 + im, T()), bload(rgy, r1 + i0, T()),
                         bload(rgy, r1 + i1, T()), bload(rgy, r1 + i2, T())};
        d[0][2] = u0[1]; d[1][2] = u0[2];
        d[2][2] = u1[1]; d[3][2] = u1[2];
        const T inv2h = geo_i2h<T>(g, 0);
        const bool lo = cx == 0, hi = cx + 1 == g.nc[0];
        diff_pair<T, sizeof(T) == 4>(u0, lo, hi, inv2h, d[0][3], d[1][3]);
        diff_pair<T, sizeof(T) == 4>(u1, lo, hi, inv2h, d[2][3], d[3][3]);
    } else {
        d[0][2] = bload(rgy, r0 + i0, T()); d[1][2] = bload(rgy, r0 + i1, T());
        d[2][2] = bload(rgy, r1 + i0, T()); d[3][2] = bload(rgy, r1 + i1, T());
        d[0][3] = d[1][3] = d[2][3] = d[3][3] = T(0);
    }
}

// 3D alpha: 0 phi, 1 psi_x, 2 psi_y, 3 phi_xy, 4 psi_z, 5 phi_xz, 6 phi_yz,
// 7 phi_xyz, with phi_xy = D_x psi_y, phi_xz = D_x psi_z, phi_yz = D_y psi_z,
// phi_xyz = D_x D_y psi_z.
template <typename T, int MIX>
__device__ __forceinline__ void gather3d(const Geom &g, Rsrc rphi, Rsrc rgx, Rsrc rgy, Rsrc rgz,
                                         int c0, int c1, int c2, T d[8][8])
{
    if constexpr (MIX == GALS_MIXED_CELL) {
        // the 8 vertices' phi and gradients; cross derivatives per facet
        const unsigned P = unsigned(g.pitch), S = unsigned(g.pitch) * unsigned(g.n[1]);
#pragma unroll
        for (int v = 0; v < 8; v++) {
            const unsigned o = unsigned(c2 + (v >> 2)) * S + unsigned(c1 + ((v >> 1) & 1)) * P +
                               unsigned(c0 + (v & 1));
            d[v][0] = bload(rphi, o, T());
            d[v][1] = bload(rgx, o, T());
            d[v][2] = bload(rgy, o, T());
            d[v][4] = bload(rgz, o, T());
        }
        const T ih[3] = {geo_ih<T>(g, 0), geo_ih<T>(g, 1), geo_ih<T>(g, 2)};
        // (a, b) = (x, y), (x, z), (y, z) into alpha 3, 5, 6; facet level along
        // the third axis c
        constexpr int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2}, pc[3] = {2, 1, 0};
        constexpr int slot[3] = {3, 5, 6};
#pragma unroll
        for (int q = 0; q < 3; q++)
#pragma unroll
            for (int lc = 0; lc < 2; lc++) {
                T ga[4], gb[4], out[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int v = ((k & 1) << pa[q]) | (((k >> 1) & 1) << pb[q]) | (lc << pc[q]);
                    ga[k] = d[v][1 << pa[q]];
                    gb[k] = d[v][1 << pb[q]];
                }
                cell_cross(ga, gb, ih[pa[q]], ih[pb[q]], out);
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int v = ((k & 1) << pa[q]) | (((k >> 1) & 1) << pb[q]) | (lc << pc[q]);
                    d[v][slot[q]] = out[k];
                }
            }
        // phi_xyz, first order, from psi_z on the xy facet of each z level
#pragma unroll
        for (int lz = 0; lz < 2; lz++) {
            const int b = 4 * lz;
            const T xyz = (d[b + 3][4] - d[b + 2][4] - d[b + 1][4] + d[b][4]) * (ih[0] * ih[1]);
#pragma unroll
            for (int k = 0; k < 4; k++) d[b + k][7] = xyz;
        }
        return;
    }
    const unsigned P = unsigned(g.pitch), S = unsigned(g.pitch) * unsigned(g.n[1]);
    const unsigned xs[4] = {unsigned(c0 > 0 ? c0 - 1 : 0), unsigned(c0), unsigned(c0 + 1),
                            unsigned(c0 + 2 <= g.nc[0] ? c0 + 2 : g.nc[0])};
    const unsigned ys[4] = {unsigned(c1 > 0 ? c1 - 1 : 0), unsigned(c1), unsigned(c1 + 1),
                            unsigned(c1 + 2 <= g.nc[1] ? c1 + 2 : g.nc[1])};
    const bool xlo = c0 == 0, xhi = c0 + 1 == g.nc[0];
    const bool ylo = c1 == 0, yhi = c1 + 1 == g.nc[1];
    const T i2hx = geo_i2h<T>(g, 0), i2hy = geo_i2h<T>(g, 1);
#pragma unroll
    for (int vz = 0; vz < 2; vz++) {
        const unsigned zo = unsigned(c2 + vz) * S;
#pragma unroll
        for (int vy = 0; vy < 2; vy++) {
            const unsigned ro = zo + ys[1 + vy] * P;
#pragma unroll
            for (int vx = 0; vx < 2; vx++) {
                const int v = vx + 2 * vy + 4 * vz;
                d[v][0] = bload(rphi, ro + xs[1 + vx], T());
                d[v][1] = bload(rgx, ro + xs[1 + vx], T());
            }
            if constexpr (MIX == GALS_MIXED_CENTRAL) {
                const T u[4] = {bload(rgy, ro + xs[0], T()), bload(rgy, ro + xs[1], T()),
                                bload(rgy, ro + xs[2], T()), bload(rgy, ro + xs[3], T())};
                d[2 * vy + 4 * vz][2] = u[1];
                d[1 + 2 * vy + 4 * vz][2] = u[2];
                diff_pair(u, xlo, xhi, i2hx, d[2 * vy + 4 * vz][3], d[1 + 2 * vy + 4 * vz][3]);
            } else {
                d[2 * vy + 4 * vz][2] = bload(rgy, ro + xs[1], T());
                d[1 + 2 * vy + 4 * vz][2] = bload(rgy, ro + xs[2], T());
                d[2 * vy + 4 * vz][3] = d[1 + 2 * vy + 4 * vz][3] = T(0);
            }
        }
        if constexpr (MIX == GALS_MIXED_CENTRAL) {
            T w[4][4];  // psi_z at (ys[jy], xs[jx])
#pragma unroll
            for (int jy = 0; jy < 4; jy++)
#pragma unroll
                for (int jx = 0; jx < 4; jx++) w[jy][jx] = bload(rgz, zo + ys[jy] * P + xs[jx], T());
            T dy[2][4];  // D_y psi_z at rows c1, c1+1 for each x sample
#pragma unroll
            for (int jx = 0; jx < 4; jx++) {
                const T col[4] = {w[0][jx], w[1][jx], w[2][jx], w[3][jx]};
                diff_pair(col, ylo, yhi, i2hy, dy[0][jx], dy[1][jx]);
            }
#pragma unroll
            for (int vy = 0; vy < 2; vy++) {
                const int b = 2 * vy + 4 * vz;
                d[b][4] = w[1 + vy][1];
                d[b + 1][4] = w[1 + vy][2];
                diff_pair(w[1 + vy], xlo, xhi, i2hx, d[b][5], d[b + 1][5]);  // phi_xz
                d[b][6] = dy[vy][1];                                       // phi_yz
                d[b + 1][6] = dy[vy][2];
                diff_pair(dy[vy], xlo, xhi, i2hx, d[b][7], d[b + 1][7]);    // phi_xyz
            }
        } else {
#pragma unroll
            for (int vy = 0; vy < 2; vy++) {
                const int b = 2 * vy + 4 * vz;
                const unsigned ro = zo + ys[1 + vy] * P;
                d[b][4] = bload(rgz, ro + xs[1], T());
                d[b + 1][4] = bload(rgz, ro + xs[2], T());
                d[b][5] = d[b + 1][5] = d[b][6] = d[b + 1][6] = d[b][7] = d[b + 1][7] = T(0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 1D Hermite factors (sec. 2.3, eq. 1-cubic_basis_functions), with the h^alpha
// scaling of eq. (p-cubic_interpolant) folded in. Index k = v + 2 alpha:
//   k=0 f(t), k=1 f(1-t), k=2 h g(t), k=3 -h g(1-t),
// f = 1 - 3t^2 + 2t^3, g = t (1-t)^2; dw = d/dx, ddw = d2/dx2.
// ---------------------------------------------------------------------------
template <typename T>
struct Basis {
    T w[4], dw[4], ddw[4];
};

template <typename T, bool SECOND>
__device__ __forceinline__ void basis(T t, T h, T inv_h, Basis<T> &b)
{
    const T s = T(1) - t;
    const T t2 = t * t;
    const T f1 = t2 * (T(3) - T(2) * t);  // f(1-t) = 1 - f(t)
    b.w[0] = T(1) - f1;
    b.w[1] = f1;
    b.w[2] = h * t * s * s;
    b.w[3] = -h * s * t2;
    const T df = T(6) * t * s * inv_h;  // d/dx f(1-t)
    b.dw[0] = -df;
    b.dw[1] = df;
    b.dw[2] = s * (T(1) - T(3) * t);
    b.dw[3] = t * (T(3) * t - T(2));
    if constexpr (SECOND) {
        const T ddf = (T(12) * t - T(6)) * inv_h * inv_h;
        b.ddw[0] = ddf;
        b.ddw[1] = -ddf;
        b.ddw[2] = (T(6) * t - T(4)) * inv_h;
        b.ddw[3] = (T(6) * t - T(2)) * inv_h;
    }
}

// Value and gradient of the bicubic (contract y, then x).
template <typename T>
__device__ __forceinline__ void hermite2d(const T d[4][4], const Basis<T> &bx, const Basis<T> &by,
                                          T &H, T &Hx, T &Hy)
{
    H = Hx = Hy = T(0);
#pragma unroll
    for (int vx = 0; vx < 2; vx++)
#pragma unroll
        for (int ax = 0; ax < 2; ax++) {
            T s = T(0), sy = T(0);
#pragma unroll
            for (int vy = 0; vy < 2; vy++)
#pragma unroll
                for (int ay = 0; ay < 2; ay++) {
                    const T dd = d[vx + 2 * vy][ax + 2 * ay];
                    s += dd * by.w[vy + 2 * ay];
                    sy += dd * by.dw[vy + 2 * ay];
                }
            const int k = vx + 2 * ax;
            H += s * bx.w[k];
            Hx += s * bx.dw[k];
            Hy += sy * bx.w[k];
        }
}

// Value, gradient and Hessian of the bicubic.
template <typename T>
__device__ __forceinline__ void hermite2d_full(const T d[4][4], const Basis<T> &bx,
                                               const Basis<T> &by, T &H, T *G, T *Hs)
{
    T h = 0, hx = 0, hy = 0, hxx = 0, hxy = 0, hyy = 0;
#pragma unroll
    for (int vx = 0; vx < 2; vx++)
#pragma unroll
        for (int ax = 0; ax < 2; ax++) {
            T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int vy = 0; vy < 2; vy++)
#pragma unroll
                for (int ay = 0; ay < 2; ay++) {
                    const T dd = d[vx + 2 * vy][ax + 2 * ay];
                    s0 += dd * by.w[vy + 2 * ay];
                    s1 += dd * by.dw[vy + 2 * ay];
                    s2 += dd * by.ddw[vy + 2 * ay];
                }
            const int k = vx + 2 * ax;
            h += s0 * bx.w[k];
            hx += s0 * bx.dw[k];
            hxx += s0 * bx.ddw[k];
            hy += s1 * bx.w[k];
            hxy += s1 * bx.dw[k];
            hyy += s2 * bx.w[k];
        }
    H = h;
    G[0] = hx; G[1] = hy;
    Hs[0] = hxx; Hs[1] = hxy; Hs[2] = hxy; Hs[3] = hyy;
}

// Value and gradient of the tricubic (contract z, then y, then x).
template <typename T>
__device__ __forceinline__ void hermite3d(const T d[8][8], const Basis<T> &bx, const Basis<T> &by,
                                          const Basis<T> &bz, T &H, T &Hx, T &Hy, T &Hz)
{
    H = Hx = Hy = Hz = T(0);
#pragma unroll
    for (int vx = 0; vx < 2; vx++)
#pragma unroll
        for (int ax = 0; ax < 2; ax++) {
            T a0 = 0, ay_ = 0, az_ = 0;
#pragma unroll
            for (int vy = 0; vy < 2; vy++)
#pragma unroll
                for (int ay = 0; ay < 2; ay++) {
                    T z0 = 0, z1 = 0;
#pragma unroll
                    for (int vz = 0; vz < 2; vz++)
#pragma unroll
                        for (int az = 0; az < 2; az++) {
                            const T dd = d[vx + 2 * vy + 4 * vz][ax + 2 * ay + 4 * az];
                            z0 += dd * bz.w[vz + 2 * az];
                            z1 += dd * bz.dw[vz + 2 * az];
                        }
                    const int ky = vy + 2 * ay;
                    a0 += z0 * by.w[ky];
                    ay_ += z0 * by.dw[ky];
                    az_ += z1 * by.w[ky];
                }
            const int k = vx + 2 * ax;
            H += a0 * bx.w[k];
            Hx += a0 * bx.dw[k];
            Hy += ay_ * bx.w[k];
            Hz += az_ * bx.w[k];
        }
}

// Value, gradient and Hessian (row-major 3x3) of the tricubic.
template <typename T>
__device__ __forceinline__ void hermite3d_full(const T d[8][8], const Basis<T> &bx,
                                               const Basis<T> &by, const Basis<T> &bz, T &H,
                                               T *G, T *Hs)
{
    T h = 0, hx = 0, hy = 0, hz = 0, hxx = 0, hyy = 0, hzz = 0, hxy = 0, hxz = 0, hyz = 0;
#pragma unroll
    for (int vx = 0; vx < 2; vx++)
#pragma unroll
        for (int ax = 0; ax < 2; ax++) {
            T a00 = 0, a10 = 0, a20 = 0, a01 = 0, a11 = 0, a02 = 0;
#pragma unroll
            for (int vy = 0; vy < 2; vy++)
#pragma unroll
                for (int ay = 0; ay < 2; ay++) {
                    T z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
                    for (int vz = 0; vz < 2; vz++)
#pragma unroll
                        for (int az = 0; az < 2; az++) {
                            const T dd = d[vx + 2 * vy + 4 * vz][ax + 2 * ay + 4 * az];
                            z0 += dd * bz.w[vz + 2 * az];
                            z1 += dd * bz.dw[vz + 2 * az];
                            z2 += dd * bz.ddw[vz + 2 * az];
                        }
                    const int ky = vy + 2 * ay;
                    a00 += z0 * by.w[ky];
                    a10 += z0 * by.dw[ky];
                    a20 += z0 * by.ddw[ky];
                    a01 += z1 * by.w[ky];
                    a11 += z1 * by.dw[ky];
                    a02 += z2 * by.w[ky];
                }
            const int k = vx + 2 * ax;
            h += a00 * bx.w[k];
            hx += a00 * bx.dw[k];
            hxx += a00 * bx.ddw[k];
            hy += a10 * bx.w[k];
            hxy += a10 * bx.dw[k];
            hyy += a20 * bx.w[k];
            hz += a01 * bx.w[k];
            hxz += a01 * bx.dw[k];
            hyz += a11 * bx.w[k];
            hzz += a02 * bx.w[k];
        }
    H = h;
    G[0] = hx; G[1] = hy; G[2] = hz;
    Hs[0] = hxx; Hs[1] = hxy; Hs[2] = hxz;
    Hs[3] = hxy; Hs[4] = hyy; Hs[5] = hyz;
    Hs[6] = hxz; Hs[7] = hyz; Hs[8] = hzz;
}

}  // namespace gals
