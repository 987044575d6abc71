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
//   * the parameter derivative adds, per table entry p,
//     (lambda_phi grad H + Hess H mu) . (m X'_p) + sum_ij J'_p[i][j] m_i H_i lambda_j,
//     with X'_p, J'_p the derivatives of the foot and of J along S[m][n]
//     (forward mode through the three Shu-Osher stages of
//     Ex. ex:superconsistent_ShuOsher; the stage Jacobians differentiate into
//     the third derivatives of s).
// The state adjoint is accumulated with FP64 atomics (its summation order is
// not fixed); the parameter derivative with a fixed-order block reduction.
#include "reduce.h"
#include "stream2d.h"

namespace gals {

// v and grad v (J form, G[i][j] = dv_i/dx_j) of the single mode
// sin(M x) sin(N y), M = (m+1) pi, N = (n+1) pi, from sin/cos of k pi x, y.
template <typename T>
__device__ __forceinline__ void mode_field(int m, int n, const T *sx, const T *cx, const T *sy,
                                           const T *cy, T *v, T *G)
{
    const T M = T((m + 1) * kPi), N = T((n + 1) * kPi);
    const T s_x = M * cx[m] * sy[n], s_y = N * sx[m] * cy[n];
    const T s_xx = -M * M * sx[m] * sy[n], s_xy = M * N * cx[m] * cy[n];
    const T s_yy = -N * N * sx[m] * sy[n];
    v[0] = -s_y;
    v[1] = s_x;
    G[0] = -s_xy;
    G[1] = -s_yy;
    G[2] = s_xx;
    G[3] = s_xy;
}

// Third derivatives (s_xxx, s_xxy, s_xyy, s_yyy) of the whole field.
template <typename T>
__device__ __forceinline__ void third_derivs(const T (&S)[4][4], const T *sx, const T *cx,
                                             const T *sy, const T *cy, T *t)
{
    t[0] = t[1] = t[2] = t[3] = T(0);
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const T M = T((m + 1) * kPi);
        T Py = T(0), Qy = T(0), Ry = T(0), Ty = T(0);
#pragma unroll
        for (int n = 0; n < 4; n++) {
            const T N = T((n + 1) * kPi);
            Py += S[m][n] * sy[n];
            Qy += S[m][n] * N * cy[n];
            Ry += S[m][n] * N * N * sy[n];
            Ty += S[m][n] * N * N * N * cy[n];
        }
        t[0] -= M * M * M * cx[m] * Py;
        t[1] -= M * M * sx[m] * Qy;
        t[2] -= M * cx[m] * Ry;
        t[3] -= sx[m] * Ty;
    }
}

// d(grad v)/dx . delta in J form, from the third derivatives t.
template <typename T>
__device__ __forceinline__ void grad_v_dir(const T *t, T dx, T dy, T *D)
{
    D[0] = -(t[1] * dx + t[2] * dy);
    D[1] = -(t[2] * dx + t[3] * dy);
    D[2] = t[0] * dx + t[1] * dy;
    D[3] = t[1] * dx + t[2] * dy;
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

template <typename T, int MIX, bool TAYLOR>
__global__ __launch_bounds__(kBlock) void k_adjoint2d_stream(
    Geom g, Vel<T> p, Stage<T> st, double dt, const T *__restrict__ coltab,
    const T *__restrict__ rowtab, const T *__restrict__ phi, const T *__restrict__ grad,
    const double *__restrict__ lam_in, double *__restrict__ lam_out,
    double *__restrict__ partials)
{
    const unsigned tiles_x = (unsigned(g.n[0]) + 63u) / 64u;
    const unsigned tiles = tiles_x * ((unsigned(g.n[1]) + 3u) / 4u);
    unsigned tx, ty;
    const bool in_grid = xcd_tile(tiles_x, tiles, tx, ty);
    const int i = int(tx) * 64 + int(threadIdx.x & 63u);
    const int j = __builtin_amdgcn_readfirstlane(int(ty) * 4 + int(threadIdx.x >> 6));
    double gacc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) gacc[q] = 0.0;

    if (in_grid && i < g.n[0] && j < g.n[1]) {
        StreamFoot<T> f;
        stream_trace<T, TAYLOR>(g, p, st, dt, coltab + int64_t(i) * kJet,
                                rowtab + int64_t(j) * kJet, i, j, f);
        const int64_t o = int64_t(j) * g.pitch + i;
        const double lf = lam_in[o], lx = lam_in[o + g.plane], ly = lam_in[o + 2 * g.plane];

        T d[4][4];
        gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(grad, g.plane),
                         plane_rsrc(grad + g.plane, g.plane), f.cell[0], f.cell[1], d);
        Basis<T> bx, by;
        basis<T, true>(T(f.xi[0]), T(g.h[0]), T(g.inv_h[0]), bx);
        basis<T, true>(T(f.xi[1]), T(g.h[1]), T(g.inv_h[1]), by);
        T H, Gr[2], Hs[4];
        hermite2d_full(d, bx, by, H, Gr, Hs);

        const double m0 = (f.out & 1u) ? 0.0 : 1.0, m1 = (f.out & 2u) ? 0.0 : 1.0;
        const double mu0 = m0 * (double(f.J[0]) * lx + double(f.J[1]) * ly);
        const double mu1 = m1 * (double(f.J[2]) * lx + double(f.J[3]) * ly);

        // ---- state adjoint: transpose of the gather and the interpolation
        double *Lphi = lam_out, *Lx = lam_out + g.plane, *Ly = lam_out + 2 * g.plane;
        const double inv2h = double(T(0.5 * g.inv_h[0]));
#pragma unroll
        for (int vy = 0; vy < 2; vy++) {
            const int64_t row = int64_t(f.cell[1] + vy) * g.pitch;
#pragma unroll
            for (int vx = 0; vx < 2; vx++) {
                const int ci = f.cell[0] + vx;
                double db[4];
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const int kx = vx + 2 * (a & 1), ky = vy + 2 * (a >> 1);
                    db[a] = lf * double(bx.w[kx]) * double(by.w[ky]) +
                            mu0 * double(bx.dw[kx]) * double(by.w[ky]) +
                            mu1 * double(bx.w[kx]) * double(by.dw[ky]);
                }
                scatter(Lphi + row + ci, db[0]);
                scatter(Lx + row + ci, db[1]);
                scatter(Ly + row + ci, db[2]);
                if constexpr (MIX == GALS_MIXED_CENTRAL) {
                    // phi_xy at node ci = D_x psi_y: central inside, one-sided
                    // 3-point at node 0 and node nc
                    const double c = db[3] * inv2h;
                    if (ci == 0) {
                        scatter(Ly + row + 0, -3.0 * c);
                        scatter(Ly + row + 1, 4.0 * c);
                        scatter(Ly + row + 2, -c);
                    } else if (ci == g.nc[0]) {
                        scatter(Ly + row + ci, 3.0 * c);
                        scatter(Ly + row + ci - 1, -4.0 * c);
                        scatter(Ly + row + ci - 2, c);
                    } else {
                        scatter(Ly + row + ci + 1, c);
                        scatter(Ly + row + ci - 1, -c);
                    }
                }
            }
        }

        // ---- parameter derivative
        // r = lambda_phi grad H + Hess H mu,  P[i][j] = m_i H_i lambda_j
        const double r0 = lf * double(Gr[0]) + double(Hs[0]) * mu0 + double(Hs[1]) * mu1;
        const double r1 = lf * double(Gr[1]) + double(Hs[2]) * mu0 + double(Hs[3]) * mu1;
        const double P[4] = {m0 * double(Gr[0]) * lx, m0 * double(Gr[0]) * ly,
                             m1 * double(Gr[1]) * lx, m1 * double(Gr[1]) * ly};
        const double x0 = g.lo[0] + double(i) * g.h[0], y0 = g.lo[1] + double(j) * g.h[1];
        T sx0[4], cx0[4], sy0[4], cy0[4], sx1[4], cx1[4], sy1[4], cy1[4];
        T sx2[4], cx2[4], sy2[4], cy2[4];
        sincos_multiples(T(x0), sx0, cx0);
        sincos_multiples(T(y0), sy0, cy0);
        sincos_multiples(T(x0 + double(f.d1[0])), sx1, cx1);
        sincos_multiples(T(y0 + double(f.d1[1])), sy1, cy1);
        sincos_multiples(T(x0 + double(f.d2[0])), sx2, cx2);
        sincos_multiples(T(y0 + double(f.d2[1])), sy2, cy2);
        T t1[4], t2[4];
        third_derivs(p.S, sx1, cx1, sy1, cy1, t1);
        third_derivs(p.S, sx2, cx2, sy2, cy2, t2);
        const T dtT = T(dt);
        // the chain of the forward Jacobian: J1 = I - dt A0, B1 = A1 J1,
        // J2 = I - dt (A0 + B1) / 4
        T J1[4], B1[4], J2[4];
#pragma unroll
        for (int k = 0; k < 4; k++) J1[k] = T((k % 3) == 0) - dtT * f.A0[k];
        mul2(f.A1, J1, B1);
#pragma unroll
        for (int k = 0; k < 4; k++)
            J2[k] = T((k % 3) == 0) - dtT * (T(0.25) * f.A0[k] + T(0.25) * B1[k]);
#pragma unroll
        for (int m = 0; m < 4; m++)
#pragma unroll
            for (int n = 0; n < 4; n++) {
                T vp[2], Gp[4];
                // stage 1: v0' = c1 v_p(x), A0' = c1 G_p(x)
                mode_field(m, n, sx0, cx0, sy0, cy0, vp, Gp);
                T v0p[2] = {st.c1 * vp[0], st.c1 * vp[1]};
                T A0p[4] = {st.c1 * Gp[0], st.c1 * Gp[1], st.c1 * Gp[2], st.c1 * Gp[3]};
                const T x1p[2] = {-dtT * v0p[0], -dtT * v0p[1]};
                // stage 2 at x1: v1' = c2 v_p(x1) + A1 x1', A1' = c2 (G_p(x1) + dG(x1) x1')
                mode_field(m, n, sx1, cx1, sy1, cy1, vp, Gp);
                T D[4];
                grad_v_dir(t1, x1p[0], x1p[1], D);
                const T v1p[2] = {st.c2 * vp[0] + f.A1[0] * x1p[0] + f.A1[1] * x1p[1],
                                  st.c2 * vp[1] + f.A1[2] * x1p[0] + f.A1[3] * x1p[1]};
                T A1p[4];
#pragma unroll
                for (int k = 0; k < 4; k++) A1p[k] = st.c2 * (Gp[k] + D[k]);
                const T x2p[2] = {-dtT * (T(0.25) * v0p[0] + T(0.25) * v1p[0]),
                                  -dtT * (T(0.25) * v0p[1] + T(0.25) * v1p[1])};
                // stage 3 at x2
                mode_field(m, n, sx2, cx2, sy2, cy2, vp, Gp);
                grad_v_dir(t2, x2p[0], x2p[1], D);
                const T v2p[2] = {st.c3 * vp[0] + f.A2[0] * x2p[0] + f.A2[1] * x2p[1],
                                  st.c3 * vp[1] + f.A2[2] * x2p[0] + f.A2[3] * x2p[1]};
                T A2p[4];
#pragma unroll
                for (int k = 0; k < 4; k++) A2p[k] = st.c3 * (Gp[k] + D[k]);
                // foot: X' = -dt (v0'/6 + v1'/6 + 2 v2'/3)
                T Xp[2];
#pragma unroll
                for (int a = 0; a < 2; a++)
                    Xp[a] = -dtT * (v0p[a] * T(1.0 / 6.0) + v1p[a] * T(1.0 / 6.0) +
                                    v2p[a] * T(2.0 / 3.0));
                // Jacobian: J1' = -dt A0', B1' = A1' J1 + A1 J1',
                // J2' = -dt (A0' + B1')/4, B2' = A2' J2 + A2 J2',
                // J' = -dt (A0'/6 + B1'/6 + 2 B2'/3)
                T J1p[4], B1p[4], B1q[4], J2p[4], B2p[4], B2q[4];
#pragma unroll
                for (int k = 0; k < 4; k++) J1p[k] = -dtT * A0p[k];
                mul2(A1p, J1, B1p);
                mul2(f.A1, J1p, B1q);
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    B1p[k] += B1q[k];
                    J2p[k] = -dtT * (T(0.25) * A0p[k] + T(0.25) * B1p[k]);
                }
                mul2(A2p, J2, B2p);
                mul2(f.A2, J2p, B2q);
                double acc = r0 * m0 * double(Xp[0]) + r1 * m1 * double(Xp[1]);
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const T Jp = -dtT * (A0p[k] * T(1.0 / 6.0) + B1p[k] * T(1.0 / 6.0) +
                                         (B2p[k] + B2q[k]) * T(2.0 / 3.0));
                    acc += double(Jp) * P[k];
                }
                gacc[4 * m + n] += acc;
            }
    }
    block_reduce<16, true>(gacc, 0u, partials + int64_t(blockIdx.x) * 16);
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
    const unsigned tiles =
        unsigned((ctx->g.n[0] + 63) / 64) * unsigned((ctx->g.n[1] + 3) / 4);
    return (tiles + 7u) / 8u * 8u;
}

template <typename T, int MIX>
static void launch_adj(const gals_ctx *ctx, const Vel<T> &p, const void *phi, const void *grad,
                       const double *lam_in, double *lam_out, double *partials, double dt,
                       double c1, double c2, double c3, const void *coltab, const void *rowtab,
                       hipStream_t s)
{
    const Stage<T> st{T(c1), T(c2), T(c3)};
    hipLaunchKernelGGL((k_adjoint2d_stream<T, MIX, sizeof(T) == 4>), dim3(adjoint_blocks(ctx)),
                       dim3(kBlock), 0, s, ctx->g, p, st, dt, (const T *)coltab,
                       (const T *)rowtab, (const T *)phi, (const T *)grad, lam_in, lam_out,
                       partials);
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
                               const double *lam_in, double *lam_out, double *partials,
                               double dt, double c1, double c2, double c3, const void *coltab,
                               const void *rowtab, hipStream_t s)
{
    hipError_t e = launch_zero(lam_out, 3 * ctx->g.plane, s);
    if (e != hipSuccess) return e;
    if (ctx->prec == GALS_F32) {
        if (ctx->mixed == GALS_MIXED_ZERO)
            launch_adj<float, GALS_MIXED_ZERO>(ctx, ctx->vf, phi, grad, lam_in, lam_out,
                                               partials, dt, c1, c2, c3, coltab, rowtab, s);
        else
            launch_adj<float, GALS_MIXED_CENTRAL>(ctx, ctx->vf, phi, grad, lam_in, lam_out,
                                                  partials, dt, c1, c2, c3, coltab, rowtab, s);
    } else {
        if (ctx->mixed == GALS_MIXED_ZERO)
            launch_adj<double, GALS_MIXED_ZERO>(ctx, ctx->vd, phi, grad, lam_in, lam_out,
                                                partials, dt, c1, c2, c3, coltab, rowtab, s);
        else
            launch_adj<double, GALS_MIXED_CENTRAL>(ctx, ctx->vd, phi, grad, lam_in, lam_out,
                                                   partials, dt, c1, c2, c3, coltab, rowtab, s);
    }
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
