// Discrete adjoint of the GA-CIR step for 2D sine stream-function fields, and
// the smoothed-Heaviside shape loss that seeds it.
//
// One step maps u = (phi, psi_x, psi_y) to M(u; S), where S[m][n] is the
// folded stream-function table (s = sum S[m][n] sin(m pi x) sin(n pi y)).
// For node x with foot X, Jacobian J (J[i][j] = dX_i/dx_j), mask m_a = 0 on
// axes where the foot was projected back onto the domain, and the bicubic H
// of the foot cell built from u (sec. 2.3, eq. p-cubic_interpolant; cross
// derivatives by approach (A)):
//     phi_new = H(X),   psi_new_j = sum_i J[i][j] m_i dH/dx_i(X)
// (sec. 4 steps 1-3, eq. superconsistency). M is linear in u, so with
// lambda = dF/du_new at the node and mu_i = m_i sum_j J[i][j] lambda_j:
//   * the state adjoint scatters lambda_phi W_q + mu . grad W_q onto the 16
//     cell data q (the transpose of the interpolation), and the phi_xy data
//     onto psi_y through the transpose of the central difference D_x;
//   * the parameter derivative seeds the foot with Xbar = m (lambda_phi grad H
//     + Hess H mu) and the Jacobian with Jbar[i][j] = m_i H_i lambda_j, runs
//     both back through the three Shu-Osher stages of
//     Ex. ex:superconsistent_ShuOsher (reverse mode: the stage positions
//     pick up grad v and the third derivatives of s), and reads off
//     dF/dS[m][n] = sum over stages c_k (vbar_k . v_mn(x_k) + Abar_k : grad v_mn(x_k)).
// The state adjoint is accumulated with FP64 atomics (its summation order is
// not fixed); the parameter derivative with a fixed-order block reduction.
// With CLEAR the kernel zeroes lam_in as it reads it, so lam_in can receive
// the next (earlier) step's scatter without a separate fill.
#include "reduce.h"
#include "stream2d.h"

namespace gals {

// Third derivatives (s_xxx, s_xxy, s_xyy, s_yyy) of the whole field from the
// table S, the y factors carrying the wavenumbers (N cos, N^2 sin, N^3 cos).
template <typename T, class P>
__device__ __forceinline__ void third_derivs(const P &p, const T *sx, const T *cx, const T *sy,
                                             const T *cy, T *t)
{
    t[0] = t[1] = t[2] = t[3] = T(0);
    T qy[4], ry[4], ty[4];
#pragma unroll
    for (int n = 0; n < 4; n++) {
        const T N = T((n + 1) * kPi);
        qy[n] = N * cy[n];
        ry[n] = T((n + 1) * (n + 1) * kPi * kPi) * sy[n];
        ty[n] = T((n + 1) * (n + 1) * kPi * kPi) * qy[n];
    }
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const T M = T((m + 1) * kPi);
        T Py = T(0), Qy = T(0), Ry = T(0), Ty = T(0);
#pragma unroll
        for (int n = 0; n < 4; n++) {
            Py += p.S[m][n] * sy[n];
            Qy += p.S[m][n] * qy[n];
            Ry += p.S[m][n] * ry[n];
            Ty += p.S[m][n] * ty[n];
        }
        t[0] -= (M * M * M) * cx[m] * Py;
        t[1] -= (M * M) * sx[m] * Qy;
        t[2] -= M * cx[m] * Ry;
        t[3] -= sx[m] * Ty;
    }
}

// sum_ik Abar[i][k] dG[i][k]/dx and /dy from the third derivatives t.
template <typename T>
__device__ __forceinline__ void grad_v_adj(const T *t, const T *Ab, T &gx, T &gy)
{
    gx = -Ab[0] * t[1] - Ab[1] * t[2] + Ab[2] * t[0] + Ab[3] * t[1];
    gy = -Ab[0] * t[2] - Ab[1] * t[3] + Ab[2] * t[1] + Ab[3] * t[2];
}

// dF/dS[m][n] += c (vbar . v_mn + Abar : G_mn) at one stage point, for all
// 16 (m, n): with a = -vbar_x, b = vbar_y, e = Abar[3] - Abar[0],
// the mode term is sin(Mx) (N a cos(Ny) + (N^2 Abar[1] - M^2 Abar[2]) sin(Ny))
//                + cos(Mx) M (b sin(Ny) + N e cos(Ny)).
// Per n the y factors are formed once (p = N a cos + N^2 d1 sin, q = d2 sin,
// r = b sin + N e cos), per m the product M cos(Mx); then each (m, n) takes
// three multiply-adds: acc += sin(Mx) (p + M^2 q) + M cos(Mx) r.
template <typename T>
__device__ __forceinline__ void mode_terms(T c, const T *vb, const T *Ab, const T *sx,
                                           const T *cx, const T *sy, const T *cy, T (&acc)[16])
{
    const T a = -c * vb[0], b = c * vb[1], e = c * (Ab[3] - Ab[0]);
    const T d1 = c * Ab[1], d2 = -c * Ab[2];
    T p[4], q[4], r[4], mc[4];
#pragma unroll
    for (int n = 0; n < 4; n++) {
        const T N = T((n + 1) * kPi);
        p[n] = (N * a) * cy[n] + (N * N * d1) * sy[n];
        q[n] = d2 * sy[n];
        r[n] = b * sy[n] + (N * e) * cy[n];
    }
#pragma unroll
    for (int m = 0; m < 4; m++) mc[m] = T((m + 1) * kPi) * cx[m];
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const T M2 = T((m + 1) * (m + 1) * kPi * kPi);
#pragma unroll
        for (int n = 0; n < 4; n++) {
            // one multiply-add per statement (as one expression the two
            // products would cost a multiply, a multiply-add and an add)
            acc[4 * m + n] += sx[m] * (p[n] + M2 * q[n]);
            acc[4 * m + n] += mc[m] * r[n];
        }
    }
}

// C = A B^T and C = A^T B for 2 x 2 matrices stored row-major.
template <typename T>
__device__ __forceinline__ void mul2_abt(const T *A, const T *B, T *C)
{
    C[0] = A[0] * B[0] + A[1] * B[1];
    C[1] = A[0] * B[2] + A[1] * B[3];
    C[2] = A[2] * B[0] + A[3] * B[1];
    C[3] = A[2] * B[2] + A[3] * B[3];
}

template <typename T>
__device__ __forceinline__ void mul2_atb(const T *A, const T *B, T *C)
{
    C[0] = A[0] * B[0] + A[2] * B[2];
    C[1] = A[0] * B[1] + A[2] * B[3];
    C[2] = A[1] * B[0] + A[3] * B[2];
    C[3] = A[1] * B[1] + A[3] * B[3];
}

template <typename T>
__device__ __forceinline__ void mul2(const T *A, const T *B, T *C)
{
    C[0] = A[0] * B[0] + A[1] * B[2];
    C[1] = A[0] * B[1] + A[1] * B[3];
    C[2] = A[2] * B[0] + A[3] * B[2];
    C[3] = A[2] * B[1] + A[3] * B[3];
}

__device__ __forceinline__ void scatter(double *p, double v) { unsafeAtomicAdd(p, v); }

// sin(l pi x'), cos(l pi x') for l = 1..4 at x' = x + d from sin and cos of
// pi x (the node's table entries): angle addition when the offset is in the
// series' range (as in the 3D step), sincospi otherwise.
template <typename T>
__device__ __forceinline__ void stage_multiples(T s1, T c1, double x, T d, T *s, T *c)
{
    constexpr double kMax = sizeof(T) == 4 ? kShiftMax : kShiftMaxLong<T>;
    if (fabs(d) <= T(kMax / kPi)) {
        T ss, cc;
        if constexpr (sizeof(T) == 4)
            shifted_sincos(s1, c1, d, ss, cc);
        else
            shifted_sincos_long(s1, c1, d, ss, cc);
        multiples_from(ss, cc, s, c);
    } else {
        sincos_multiples(T(x + double(d)), s, c);
    }
}

// LDS tile of the block's scatter: fields x nodes, nodes per row x rows.
constexpr int kTileW = 96, kTileH = 12;

// The transpose of the gather: dbar[v][alpha] for corner v = vx + 2 vy of
// cell (c0, c1) goes to phi, psi_x, psi_y of that corner and, for the cross
// derivative phi_xy = D_x psi_y, to psi_y of the difference stencil (central
// inside, one-sided 3-point at node 0 and node nc). add(field, x, y, value).
// Per row of the cell the psi_y shares of both corners and of both stencils
// are summed first: four nodes c0 - 1 .. c0 + 2 inside, three at an edge.
template <int MIX, class Add>
__device__ __forceinline__ void emit_scatter(const double (&dbar)[4][4], int c0, int c1, int nc,
                                             double inv2h, Add add)
{
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int x = c0 + (v & 1), y = c1 + (v >> 1);
        add(0, x, y, dbar[v][0]);
        add(1, x, y, dbar[v][1]);
        if constexpr (MIX != GALS_MIXED_CENTRAL) add(2, x, y, dbar[v][2]);
    }
    if constexpr (MIX == GALS_MIXED_CENTRAL) {
        const bool lo = c0 == 0, hi = c0 + 1 == nc;  // nc >= 2: not both
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const int y = c1 + r;
            const double d0 = dbar[2 * r][2], d1 = dbar[2 * r + 1][2];
            const double a = dbar[2 * r][3] * inv2h, b = dbar[2 * r + 1][3] * inv2h;
            // shares of psi_y at nodes c0 - 1, c0, c0 + 1, c0 + 2
            double t0 = -a, t1 = d0 - b, t2 = d1 + a, t3 = b;
            if (lo) {
                t0 = 0.0;
                t1 = d0 - 3.0 * a - b;
                t2 = d1 + 4.0 * a;
                t3 = b - a;
            } else if (hi) {
                t0 = b - a;
                t1 = d0 - 4.0 * b;
                t2 = d1 + a + 3.0 * b;
                t3 = 0.0;
            }
            if (!lo) add(2, c0 - 1, y, t0);
            add(2, c0, y, t1);
            add(2, c0 + 1, y, t2);
            if (!hi) add(2, c0 + 2, y, t3);
        }
    }
}

// Four waves per SIMD in FP32 (at most 128 VGPRs): an earlier form took 134
// and three waves by default, 80 us per step on the 1024^2 gradient workload
// against 68 at four. The FP64 kernel would spill heavily and keeps the
// default.
template <typename T, int MIX, bool TAYLOR, bool CLEAR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? 4 : 1))) void k_adjoint2d_stream(
    Geom g, Vel<T> p, Stage<T> st, double dt, const T *__restrict__ coltab,
    const T *__restrict__ rowtab, const T *__restrict__ phi, const T *__restrict__ grad,
    double *__restrict__ lam_in, double *__restrict__ lam_out, double *__restrict__ partials)
{
    unsigned tx, ty;
    const bool in_grid = xcd_tile(g, tx, ty);
    const int i = int(tx) * 64 + int(threadIdx.x & 63u);
    const int j = __builtin_amdgcn_readfirstlane(int(ty) * 4 + int(threadIdx.x >> 6));
    double gacc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) gacc[q] = 0.0;
    double dbar[4][4];
    int cell0 = 0, cell1 = 0;
    const bool valid = in_grid && i < g.n[0] && j < g.n[1];

    if (valid) {
        StreamFoot<T> f;
        stream_trace<T, TAYLOR>(g, p, st, dt, coltab + int64_t(i) * kJet,
                                rowtab + int64_t(j) * kJet, i, j, f);
        const int64_t o = int64_t(j) * g.pitch + i;
        const double lf = lam_in[o], lx = lam_in[o + g.plane], ly = lam_in[o + 2 * g.plane];
        if constexpr (CLEAR) {
            lam_in[o] = 0.0;
            lam_in[o + g.plane] = 0.0;
            lam_in[o + 2 * g.plane] = 0.0;
        }

        T d[4][4];
        gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(grad, g.plane),
                         plane_rsrc(grad + g.plane, g.plane), f.cell[0], f.cell[1], d);
        Basis<T> bx, by;
        basis<T, true>(T(f.xi[0]), geo_h<T>(g, 0), geo_ih<T>(g, 0), bx);
        basis<T, true>(T(f.xi[1]), geo_h<T>(g, 1), geo_ih<T>(g, 1), by);
        T H, Gr[2], Hs[4];
        hermite2d_full(d, bx, by, H, Gr, Hs);

        const double m0 = (f.out & 1u) ? 0.0 : 1.0, m1 = (f.out & 2u) ? 0.0 : 1.0;
        const double mu0 = m0 * (double(f.J[0]) * lx + double(f.J[1]) * ly);
        const double mu1 = m1 * (double(f.J[2]) * lx + double(f.J[3]) * ly);

        // ---- state adjoint: the cell data's share, dbar[v][alpha] =
        // lambda_phi W + mu . grad W (scattered below)
        cell0 = f.cell[0];
        cell1 = f.cell[1];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int a = 0; a < 4; a++) {
                const int kx = (v & 1) + 2 * (a & 1), ky = (v >> 1) + 2 * (a >> 1);
                dbar[v][a] = lf * double(bx.w[kx]) * double(by.w[ky]) +
                             mu0 * double(bx.dw[kx]) * double(by.w[ky]) +
                             mu1 * double(bx.w[kx]) * double(by.dw[ky]);
            }
        if constexpr (MIX == GALS_MIXED_CELL) {
            // transpose of approach (B): phi_xy[v] = 3/4 (ea[vx] + eb[vy])
            // - 1/4 (ea[1-vx] + eb[1-vy]) with ea[k] = (psi_x[k+2] - psi_x[k]) / hy
            // and eb[k] = (psi_y[2k+1] - psi_y[2k]) / hx, all within the cell
            const double ihx = double(geo_ih<T>(g, 0)), ihy = double(geo_ih<T>(g, 1));
            double ea[2] = {0.0, 0.0}, eb[2] = {0.0, 0.0};
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int vx = v & 1, vy = v >> 1;
                ea[vx] += 0.75 * dbar[v][3];
                ea[1 - vx] -= 0.25 * dbar[v][3];
                eb[vy] += 0.75 * dbar[v][3];
                eb[1 - vy] -= 0.25 * dbar[v][3];
                dbar[v][3] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < 2; k++) {
                dbar[k + 2][1] += ea[k] * ihy;
                dbar[k][1] -= ea[k] * ihy;
                dbar[2 * k + 1][2] += eb[k] * ihx;
                dbar[2 * k][2] -= eb[k] * ihx;
            }
        }

        // ---- parameter derivative, reverse mode through the trace
        // seeds: Xbar = m (lambda_phi grad H + Hess H mu), Jbar[i][j] = m_i H_i lambda_j
        const T dtT = T(dt);
        const T Xb[2] = {T(m0 * (lf * double(Gr[0]) + double(Hs[0]) * mu0 + double(Hs[1]) * mu1)),
                         T(m1 * (lf * double(Gr[1]) + double(Hs[2]) * mu0 + double(Hs[3]) * mu1))};
        const T Jb[4] = {T(m0 * double(Gr[0]) * lx), T(m0 * double(Gr[0]) * ly),
                         T(m1 * double(Gr[1]) * lx), T(m1 * double(Gr[1]) * ly)};
        // forward chain pieces: J1 = I - dt A0, B1 = A1 J1, J2 = I - dt (A0 + B1) / 4
        T J1[4], B1[4], J2[4];
#pragma unroll
        for (int k = 0; k < 4; k++) J1[k] = T((k % 3) == 0) - dtT * f.A0[k];
        mul2(f.A1, J1, B1);
#pragma unroll
        for (int k = 0; k < 4; k++)
            J2[k] = T((k % 3) == 0) - dtT * (T(0.25) * f.A0[k] + T(0.25) * B1[k]);
        // J = I - dt (A0/6 + B1/6 + 2 B2/3), B2 = A2 J2
        T A0b[4], B1b[4], B2b[4], A1b[4], A2b[4], J1b[4], J2b[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            A0b[k] = -dtT * T(1.0 / 6.0) * Jb[k];
            B1b[k] = A0b[k];
            B2b[k] = -dtT * T(2.0 / 3.0) * Jb[k];
        }
        mul2_abt(B2b, J2, A2b);
        mul2_atb(f.A2, B2b, J2b);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            A0b[k] += -dtT * T(0.25) * J2b[k];
            B1b[k] += -dtT * T(0.25) * J2b[k];
        }
        mul2_abt(B1b, J1, A1b);
        mul2_atb(f.A1, B1b, J1b);
#pragma unroll
        for (int k = 0; k < 4; k++) A0b[k] += -dtT * J1b[k];
        // X = x - dt (v0/6 + v1/6 + 2 v2/3)
        T v0b[2], v1b[2], v2b[2];
#pragma unroll
        for (int a = 0; a < 2; a++) {
            v0b[a] = -dtT * T(1.0 / 6.0) * Xb[a];
            v1b[a] = v0b[a];
            v2b[a] = -dtT * T(2.0 / 3.0) * Xb[a];
        }
        const double x0 = node_coord(g.lo[0], i, g.h[0]), y0 = node_coord(g.lo[1], j, g.h[1]);
        T sx[4], cx[4], sy[4], cy[4], t3[4];
        T sb[16];
#pragma unroll
        for (int q = 0; q < 16; q++) sb[q] = T(0);
        // sin and cos of pi x and pi y at the node (table entries kJetTaylor..)
        const T *cr = coltab + int64_t(i) * kJet + kJetTaylor;
        const T *rr = rowtab + int64_t(j) * kJet + kJetTaylor;
        // stage 3 at x2 = x - dt (v0 + v1) / 4: v2 = c3 v(x2), A2 = c3 grad v(x2)
        stage_multiples(cr[0], cr[1], x0, f.d2[0], sx, cx);
        stage_multiples(rr[0], rr[1], y0, f.d2[1], sy, cy);
        mode_terms(st.c3, v2b, A2b, sx, cx, sy, cy, sb);
        third_derivs(p, sx, cx, sy, cy, t3);
        {
            T gx, gy;
            grad_v_adj(t3, A2b, gx, gy);
            const T x2b[2] = {f.A2[0] * v2b[0] + f.A2[2] * v2b[1] + st.c3 * gx,
                              f.A2[1] * v2b[0] + f.A2[3] * v2b[1] + st.c3 * gy};
#pragma unroll
            for (int a = 0; a < 2; a++) {
                v0b[a] += -dtT * T(0.25) * x2b[a];
                v1b[a] += -dtT * T(0.25) * x2b[a];
            }
        }
        // stage 2 at x1 = x - dt v0
        stage_multiples(cr[0], cr[1], x0, f.d1[0], sx, cx);
        stage_multiples(rr[0], rr[1], y0, f.d1[1], sy, cy);
        mode_terms(st.c2, v1b, A1b, sx, cx, sy, cy, sb);
        third_derivs(p, sx, cx, sy, cy, t3);
        {
            T gx, gy;
            grad_v_adj(t3, A1b, gx, gy);
            const T x1b[2] = {f.A1[0] * v1b[0] + f.A1[2] * v1b[1] + st.c2 * gx,
                              f.A1[1] * v1b[0] + f.A1[3] * v1b[1] + st.c2 * gy};
#pragma unroll
            for (int a = 0; a < 2; a++) v0b[a] += -dtT * x1b[a];
        }
        // stage 1 at the node
        multiples_from(cr[0], cr[1], sx, cx);
        multiples_from(rr[0], rr[1], sy, cy);
        mode_terms(st.c1, v0b, A0b, sx, cx, sy, cy, sb);
#pragma unroll
        for (int q = 0; q < 16; q++) gacc[q] += double(sb[q]);
    }

    // ---- scatter the cell data's share onto lam_out. The block's feet lie
    // in a small box of cells (for moderate CFL numbers), so the block sums
    // its contributions in an LDS tile first and adds the tile to lam_out
    // with one global atomic per node and field: about 4x fewer global
    // atomics. Boxes larger than the tile fall back to direct atomics.
    __shared__ double s_tile[3 * kTileH * kTileW];
    __shared__ int s_box[4];
    if (threadIdx.x == 0) {
        s_box[0] = s_box[2] = 0x7fffffff;
        s_box[1] = s_box[3] = -0x7fffffff;
    }
    __syncthreads();
    {
        // min of cell0, -cell0, cell1, -cell1 over the block's nodes (the
        // neutral element of min for lanes without a node)
        int b[4] = {valid ? cell0 : 0x7fffffff, valid ? -cell0 : 0x7fffffff,
                    valid ? cell1 : 0x7fffffff, valid ? -cell1 : 0x7fffffff};
#pragma unroll
        for (int k = 0; k < 4; k++) b[k] = wave_min(b[k]);
        if ((threadIdx.x & 63u) == 0) {
            atomicMin(&s_box[0], b[0]);
            atomicMax(&s_box[1], -b[1]);
            atomicMin(&s_box[2], b[2]);
            atomicMax(&s_box[3], -b[3]);
        }
    }
    __syncthreads();
    // the block has nodes: then all four are cell indices in [0, nc - 1]
    const bool any = s_box[0] <= s_box[1] && s_box[2] <= s_box[3];
    const int bx0 = s_box[0] - 1, by0 = s_box[2];
    const int bw = any ? s_box[1] - s_box[0] + 4 : 0, bh = any ? s_box[3] - s_box[2] + 2 : 0;
    const double inv2h = double(geo_i2h<T>(g, 0));
    if (any && bw <= kTileW && bh <= kTileH) {
        const int area = bw * bh;
        for (int e = threadIdx.x; e < 3 * area; e += kBlock) s_tile[e] = 0.0;
        __syncthreads();
        if (valid)
            emit_scatter<MIX>(dbar, cell0, cell1, g.nc[0], inv2h, [&](int fld, int x, int y, double v) {
                atomicAdd(&s_tile[fld * area + (y - by0) * bw + (x - bx0)], v);
            });
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * area; e += kBlock) {
            const double v = s_tile[e];
            const int fld = e / area, r = e - fld * area;
            const int y = by0 + r / bw, x = bx0 + r % bw;
            if (v != 0.0 && x >= 0 && x < g.n[0] && y < g.n[1])
                scatter(lam_out + fld * g.plane + int64_t(y) * g.pitch + x, v);
        }
    } else if (valid) {
        emit_scatter<MIX>(dbar, cell0, cell1, g.nc[0], inv2h, [&](int fld, int x, int y, double v) {
            scatter(lam_out + fld * g.plane + int64_t(y) * g.pitch + x, v);
        });
    }
    block_sum16<true>(gacc, partials + int64_t(blockIdx.x) * 16);
}

// Parameter-derivative partials: sum over blocks in a fixed order.
__global__ __launch_bounds__(kBlock) void k_fold_grad(const double *__restrict__ partials,
                                                      int nparts, double *__restrict__ out)
{
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
#pragma unroll
        for (int q = 0; q < 16; q++) acc[q] += partials[int64_t(b) * 16 + q];
    }
    block_reduce<16, true>(acc, 0u, out);
}

__global__ __launch_bounds__(kBlock) void k_zero(double *__restrict__ p, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += stride) p[k] = 0.0;
}

// Loss prod(h) sum (H_eps(phi) - H_eps(phi_ref))^2 over the nodes; with lam,
// also its derivative: lam_phi = 2 prod(h) (H_eps(phi) - H_eps(phi_ref))
// H_eps'(phi), lam_psi = 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_heaviside_loss(Geom g, const T *__restrict__ phi,
                                                           const T *__restrict__ phr, double eps,
                                                           double cellvol,
                                                           double *__restrict__ lam,
                                                           double *__restrict__ partials)
{
    double acc[1] = {0.0};
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x; id < g.nodes; id += stride) {
        const int64_t o = (id / g.n[0]) * g.pitch + id % g.n[0];
        const double p = double(phi[o]);
        const double dd = heaviside_eps(p, eps) - heaviside_eps(double(phr[o]), eps);
        acc[0] += dd * dd;
        if (lam) {
            lam[o] = 2.0 * cellvol * dd * heaviside_eps_deriv(p, eps);
            lam[o + g.plane] = 0.0;
            lam[o + 2 * g.plane] = 0.0;
        }
    }
    block_reduce<1>(acc, 0u, partials + int64_t(blockIdx.x) * kRedSlots);
}

unsigned adjoint_blocks(const gals_ctx *ctx)
{
    return (ctx->g.tiles + 7u) / 8u * 8u;
}

template <typename T, int MIX>
static void launch_adj(const gals_ctx *ctx, const Vel<T> &p, const void *phi, const void *grad,
                       double *lam_in, double *lam_out, bool clear, double *partials, double dt,
                       double c1, double c2, double c3, const void *coltab, const void *rowtab,
                       hipStream_t s)
{
    const Stage<T> st = make_stage<T>(dt, c1, c2, c3);
    if (clear)
        hipLaunchKernelGGL((k_adjoint2d_stream<T, MIX, sizeof(T) == 4, true>),
                           dim3(adjoint_blocks(ctx)), dim3(kBlock), 0, s, ctx->g, p, st, dt,
                           (const T *)coltab, (const T *)rowtab, (const T *)phi, (const T *)grad,
                           lam_in, lam_out, partials);
    else
        hipLaunchKernelGGL((k_adjoint2d_stream<T, MIX, sizeof(T) == 4, false>),
                           dim3(adjoint_blocks(ctx)), dim3(kBlock), 0, s, ctx->g, p, st, dt,
                           (const T *)coltab, (const T *)rowtab, (const T *)phi, (const T *)grad,
                           lam_in, lam_out, partials);
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(kBlock), 0, s,
                       p, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const gals_ctx *ctx, const void *phi, const void *grad,
                               double *lam_in, double *lam_out, bool clear, double *partials,
                               double dt, double c1, double c2, double c3, const void *coltab,
                               const void *rowtab, hipStream_t s)
{
#define GALS_ADJ(T, V, M)                                                                   \
    launch_adj<T, M>(ctx, ctx->V, phi, grad, lam_in, lam_out, clear, partials, dt, c1, c2, c3, \
                     coltab, rowtab, s)
    if (ctx->prec == GALS_F32) {
        if (ctx->mixed == GALS_MIXED_ZERO) GALS_ADJ(float, vf, GALS_MIXED_ZERO);
        else if (ctx->mixed == GALS_MIXED_CELL) GALS_ADJ(float, vf, GALS_MIXED_CELL);
        else GALS_ADJ(float, vf, GALS_MIXED_CENTRAL);
    } else {
        if (ctx->mixed == GALS_MIXED_ZERO) GALS_ADJ(double, vd, GALS_MIXED_ZERO);
        else if (ctx->mixed == GALS_MIXED_CELL) GALS_ADJ(double, vd, GALS_MIXED_CELL);
        else GALS_ADJ(double, vd, GALS_MIXED_CENTRAL);
    }
#undef GALS_ADJ
    return hipGetLastError();
}

hipError_t launch_fold_grad(const double *partials, int nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold_grad, dim3(1), dim3(kBlock), 0, s, partials, nparts, out);
    return hipGetLastError();
}

hipError_t launch_heaviside_loss(const gals_ctx *ctx, const void *phi, const void *phi_ref,
                                 double eps, double *lam, double *partials, double *out,
                                 hipStream_t s)
{
    double cellvol = 1.0;
    for (int a = 0; a < ctx->dim; a++) cellvol *= ctx->g.h[a];
    if (ctx->prec == GALS_F32)
        hipLaunchKernelGGL(k_heaviside_loss<float>, dim3(kRedBlocks), dim3(kBlock), 0, s, ctx->g,
                           (const float *)phi, (const float *)phi_ref, eps, cellvol, lam,
                           partials);
    else
        hipLaunchKernelGGL(k_heaviside_loss<double>, dim3(kRedBlocks), dim3(kBlock), 0, s,
                           ctx->g, (const double *)phi, (const double *)phi_ref, eps, cellvol,
                           lam, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold<1>, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks, 0u, out);
    return hipGetLastError();
}

}  // namespace gals
