// Inflow boundary conditions (sec. 4.1) for gfx950, applied after a step:
// Dirichlet data with the normal derivative from the equation, and the
// homogeneous Neumann condition of eq. (Neumann_bc_evolution) solved by a
// GA-CIR step of one dimension less on the inflow face. Both kernels run one
// thread per boundary node (each node counted once), a few thousand threads
// against the step's millions of nodes.
#include "hermite.h"

namespace gals {

// ---------------------------------------------------------------------------
// Boundary enumeration: faces in the order (axis 0 low, axis 0 high, axis 1
// low, ...); face (a, side) holds nodes / n[a] nodes, the other axes in
// increasing order, fastest first. A node that also lies on a face of a lower
// axis belongs to that face and is skipped here.
// ---------------------------------------------------------------------------
int64_t boundary_count(const Geom &g)
{
    int64_t c = 0;
    for (int a = 0; a < g.dim; a++) c += 2 * (g.nodes / g.n[a]);
    return c;
}

template <int D>
__device__ __forceinline__ bool boundary_node(const Geom &g, int64_t id, int *ijk)
{
#pragma unroll
    for (int a = 0; a < D; a++) {
        const int64_t cnt = g.nodes / g.n[a];
        if (id < 2 * cnt) {
            const bool high = id >= cnt;
            int64_t r = high ? id - cnt : id;
#pragma unroll
            for (int b = 0; b < D; b++) {
                if (b == a) {
                    ijk[b] = high ? g.nc[a] : 0;
                } else {
                    ijk[b] = int(r % g.n[b]);
                    r /= g.n[b];
                }
            }
#pragma unroll
            for (int b = 0; b < a; b++)
                if (ijk[b] == 0 || ijk[b] == g.nc[b]) return false;
            return true;
        }
        id -= 2 * cnt;
    }
    return false;
}

template <int D>
__device__ __forceinline__ int64_t offset_of(const Geom &g, const int *ijk)
{
    const int64_t row = D == 3 ? int64_t(ijk[2]) * g.n[1] + ijk[1] : int64_t(ijk[1]);
    return row * g.pitch + ijk[0];
}

__device__ __forceinline__ int64_t axis_stride(const Geom &g, int a)
{
    return a == 0 ? 1 : a == 1 ? g.pitch : g.pitch * g.n[1];
}

// Inflow faces of a boundary node from v at the node (time t + dt): the flow
// enters through face a when its inward normal component exceeds
// kInflowTheta max(|v|, h_a / dt). Rounding must not decide on a face that is
// a streamline or at a stagnation point, and the Dirichlet normal derivative,
// which divides by v_n, stays bounded.
template <typename T, int D>
__device__ __forceinline__ unsigned inflow_faces(const Geom &g, const int *ijk, const T *v,
                                                 double dt)
{
    constexpr T kInflowTheta = T(1e-6);
    T speed2 = T(0);
#pragma unroll
    for (int a = 0; a < D; a++) speed2 += v[a] * v[a];
    const T speed = sqrt(speed2);
    unsigned in = 0;
#pragma unroll
    for (int a = 0; a < D; a++) {
        const T vmin = kInflowTheta * fmax(speed, T(g.h[a] / dt));
        // low face: outward normal -e_a, inflow if v_a > 0; high face: v_a < 0
        if ((ijk[a] == 0 && v[a] > vmin) || (ijk[a] == g.nc[a] && v[a] < -vmin)) in |= 1u << a;
    }
    return in;
}

// ---------------------------------------------------------------------------
// Dirichlet inflow data: phi and the tangential gradient prescribed, the
// normal derivative -(phi_t + tangential v . grad phi) / v_n from the
// equation; every gradient component prescribed where the flow enters
// through several faces.
// ---------------------------------------------------------------------------
template <typename T, int D, int KIND>
__global__ __launch_bounds__(kBlock) void k_inflow(Geom g, Vel<T> p, T c, double dt,
                                                   int64_t count, T *__restrict__ phi,
                                                   T *__restrict__ grad,
                                                   const T *__restrict__ phi_b,
                                                   const T *__restrict__ grad_b,
                                                   const T *__restrict__ phit_b)
{
    const int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    int ijk[3] = {0, 0, 0};
    if (id >= count || !boundary_node<D>(g, id, ijk)) return;
    double x[D];
#pragma unroll
    for (int a = 0; a < D; a++) x[a] = node_coord(g.lo[a], ijk[a], g.h[a]);
    T v[D], A[D * D];
    velocity<T, D, KIND>(p, x, c, v, A);
    const unsigned in = inflow_faces<T, D>(g, ijk, v, dt);
    if (!in) return;
    const int64_t o = offset_of<D>(g, ijk);
    phi[o] = phi_b[o];
    T s = phit_b[o];
#pragma unroll
    for (int a = 0; a < D; a++) {
        const T ga = grad_b[a * g.plane + o];
        grad[a * g.plane + o] = ga;
        if (!((in >> a) & 1u)) s += v[a] * ga;
    }
    if (__builtin_popcount(in) == 1) {
        const int axis = __builtin_ctz(in);
        grad[axis * g.plane + o] = -s / v[axis];
    }
}

// ---------------------------------------------------------------------------
// Homogeneous Neumann inflow: on the face, phi_t + v_T . grad_T phi = 0 over
// the K tangential axes T, one GA-CIR step from the state at time t: the
// superconsistent Shu-Osher trace with v_T (positions FP64, as in the full
// step), the foot projected onto the face, the K-cubic Hermite interpolant of
// the face data (cross derivative of the pair by the context's rule:
// approach (A) differences psi_T1 along T0, as the full step's mixed planes
// do), psi_T = J^T grad H; the normal derivatives are the prescribed zeros.
// ---------------------------------------------------------------------------
template <typename T, int D, int K, int KIND, int MIX>
__device__ __forceinline__ void face_update(const Geom &g, const Vel<T> &p, const Stage<T> &st,
                                            double dt, const double *x, const int *ijk,
                                            const int *tax, const T *v0, const T *A0,
                                            const T *__restrict__ sphi,
                                            const T *__restrict__ sgrad, T *__restrict__ dphi,
                                            T *__restrict__ dgrad, int64_t o)
{
    T vs0[K], As0[K * K], vs1[K], As1[K * K], vs2[K], As2[K * K];
#pragma unroll
    for (int i = 0; i < K; i++) {
        vs0[i] = v0[tax[i]];
#pragma unroll
        for (int j = 0; j < K; j++) As0[i * K + j] = A0[tax[i] * D + tax[j]];
    }
    double x1[D], x2[D], X[D];
#pragma unroll
    for (int a = 0; a < D; a++) x1[a] = x2[a] = X[a] = x[a];
    T v[D], A[D * D];
    // stage 2: v(x1, t), x1 = x - dt v0 along the face
#pragma unroll
    for (int i = 0; i < K; i++) x1[tax[i]] = x[tax[i]] - dt * double(vs0[i]);
    velocity<T, D, KIND>(p, x1, st.c2, v, A);
#pragma unroll
    for (int i = 0; i < K; i++) {
        vs1[i] = v[tax[i]];
#pragma unroll
        for (int j = 0; j < K; j++) As1[i * K + j] = A[tax[i] * D + tax[j]];
    }
    // stage 3: v(x2, t + dt/2)
#pragma unroll
    for (int i = 0; i < K; i++)
        x2[tax[i]] = x[tax[i]] - dt * (0.25 * double(vs0[i]) + 0.25 * double(vs1[i]));
    velocity<T, D, KIND>(p, x2, st.c3, v, A);
#pragma unroll
    for (int i = 0; i < K; i++) {
        vs2[i] = v[tax[i]];
#pragma unroll
        for (int j = 0; j < K; j++) As2[i * K + j] = A[tax[i] * D + tax[j]];
    }
#pragma unroll
    for (int i = 0; i < K; i++)
        X[tax[i]] = x[tax[i]] - dt * (double(vs0[i]) * (1.0 / 6.0) + double(vs1[i]) * (1.0 / 6.0) +
                                      double(vs2[i]) * (2.0 / 3.0));
    T J[K * K];
    jacobian_chain<T, K>(As0, As1, As2, T(dt), J);

    // project the foot onto the face and split it into the face's cells
    unsigned out = 0;
    int cell[K];
    double xi[K];
    int64_t oc = o;  // offset of the face cell's first vertex
#pragma unroll
    for (int i = 0; i < K; i++) {
        const int a = tax[i];
        double Xa = X[a];
        const double tol = kFootTol * g.h[a];  // as project_foot
        if (Xa < g.lo[a] - tol) {
            Xa = g.lo[a];
            out |= 1u << i;
        } else if (Xa > g.top[a] + tol) {
            Xa = g.top[a];
            out |= 1u << i;
        }
        const double s = (Xa - g.lo[a]) * g.inv_h[a];
        const double fl = floor(s);
        const double top = double(g.nc[a] - 1);
        int c;
        if (fl >= 0.0 && fl <= top) c = int(fl);
        else if (fl > top) c = g.nc[a] - 1;
        else c = 0;
        cell[i] = c;
        xi[i] = s - double(c);
        oc += int64_t(c - ijk[a]) * axis_stride(g, a);
    }

    T H, G[K];
    if constexpr (K == 1) {
        const int a = tax[0];
        const int64_t s0 = axis_stride(g, a);
        const T *ga = sgrad + a * g.plane;
        const T d[2][2] = {{sphi[oc], ga[oc]}, {sphi[oc + s0], ga[oc + s0]}};
        Basis<T> b;
        basis<T, false>(T(xi[0]), geo_h<T>(g, a), geo_ih<T>(g, a), b);
        H = G[0] = T(0);
#pragma unroll
        for (int vv = 0; vv < 2; vv++)
#pragma unroll
            for (int al = 0; al < 2; al++) {
                H += d[vv][al] * b.w[vv + 2 * al];
                G[0] += d[vv][al] * b.dw[vv + 2 * al];
            }
    } else {
        const int a0 = tax[0], a1 = tax[1];
        const int64_t s0 = axis_stride(g, a0), s1 = axis_stride(g, a1);
        const T *g0 = sgrad + a0 * g.plane, *g1 = sgrad + a1 * g.plane;
        T d[4][4];
#pragma unroll
        for (int vv = 0; vv < 4; vv++) {
            const int64_t ov = oc + (vv & 1) * s0 + (vv >> 1) * s1;
            d[vv][0] = sphi[ov];
            d[vv][1] = g0[ov];
            d[vv][2] = g1[ov];
        }
        if constexpr (MIX == GALS_MIXED_CELL) {
            T ga[4], gb[4], cr[4];
#pragma unroll
            for (int vv = 0; vv < 4; vv++) {
                ga[vv] = d[vv][1];
                gb[vv] = d[vv][2];
            }
            cell_cross(ga, gb, geo_ih<T>(g, a0), geo_ih<T>(g, a1), cr);
#pragma unroll
            for (int vv = 0; vv < 4; vv++) d[vv][3] = cr[vv];
        } else if constexpr (MIX == GALS_MIXED_CENTRAL) {
            // psi_T1 at nodes c0-1 .. c0+2 along T0 (clamped), both rows
            const int c0 = cell[0], n0 = g.nc[a0];
            const int64_t om = oc - (c0 > 0 ? s0 : 0);
            const int64_t o2 = oc + (c0 + 2 <= n0 ? 2 : 1) * s0;
            const T inv2h = geo_i2h<T>(g, a0);
            const bool lo = c0 == 0, hi = c0 + 1 == n0;
#pragma unroll
            for (int row = 0; row < 2; row++) {
                const int64_t sh = row * s1;
                const T u[4] = {g1[om + sh], g1[oc + sh], g1[oc + s0 + sh], g1[o2 + sh]};
                diff_pair(u, lo, hi, inv2h, d[2 * row][3], d[2 * row + 1][3]);
            }
        } else {
#pragma unroll
            for (int vv = 0; vv < 4; vv++) d[vv][3] = T(0);
        }
        Basis<T> b0, b1;
        basis<T, false>(T(xi[0]), geo_h<T>(g, a0), geo_ih<T>(g, a0), b0);
        basis<T, false>(T(xi[1]), geo_h<T>(g, a1), geo_ih<T>(g, a1), b1);
        hermite2d(d, b0, b1, H, G[0], G[1]);
    }
#pragma unroll
    for (int i = 0; i < K; i++)
        if ((out >> i) & 1u) G[i] = T(0);  // the extension is constant across the edge
    dphi[o] = H;
#pragma unroll
    for (int a = 0; a < D; a++) dgrad[a * g.plane + o] = T(0);
#pragma unroll
    for (int i = 0; i < K; i++) {
        T s = J[i] * G[0];
#pragma unroll
        for (int j = 1; j < K; j++) s += J[j * K + i] * G[j];
        dgrad[tax[i] * g.plane + o] = s;
    }
}

template <typename T, int D, int KIND, int MIX>
__global__ __launch_bounds__(kBlock) void k_face(Geom g, Vel<T> p, Stage<T> st, double dt,
                                                 int64_t count, const T *__restrict__ sphi,
                                                 const T *__restrict__ sgrad,
                                                 T *__restrict__ dphi, T *__restrict__ dgrad)
{
    const int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    int ijk[3] = {0, 0, 0};
    if (id >= count || !boundary_node<D>(g, id, ijk)) return;
    double x[D];
#pragma unroll
    for (int a = 0; a < D; a++) x[a] = node_coord(g.lo[a], ijk[a], g.h[a]);
    T v0[D], A0[D * D];
    velocity<T, D, KIND>(p, x, st.c1, v0, A0);
    const unsigned in = inflow_faces<T, D>(g, ijk, v0, dt);
    if (!in) return;
    const int64_t o = offset_of<D>(g, ijk);
    int tax[D] = {}, k = 0;
#pragma unroll
    for (int a = 0; a < D; a++)
        if (!((in >> a) & 1u)) tax[k++] = a;
    if (k == 0) {
        // a corner entered through every face: phi_t = 0, zero gradient
        dphi[o] = sphi[o];
#pragma unroll
        for (int a = 0; a < D; a++) dgrad[a * g.plane + o] = T(0);
        return;
    }
    if constexpr (D == 3) {
        if (k == 2) {
            face_update<T, D, 2, KIND, MIX>(g, p, st, dt, x, ijk, tax, v0, A0, sphi, sgrad, dphi,
                                            dgrad, o);
            return;
        }
    }
    face_update<T, D, 1, KIND, MIX>(g, p, st, dt, x, ijk, tax, v0, A0, sphi, sgrad, dphi, dgrad,
                                    o);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
#define GALS_BOUNDARY_KINDS(X)                                                                    \
    X(2, GALS_VEL_AFFINE)                                                                         \
    X(2, GALS_VEL_STREAM_SIN)                                                                     \
    X(2, GALS_VEL_VORTEX)                                                                         \
    X(2, GALS_VEL_PSEUDO1D)                                                                       \
    X(3, GALS_VEL_AFFINE)                                                                         \
    X(3, GALS_VEL_VECPOT_SIN)                                                                     \
    X(3, GALS_VEL_LEVEQUE3D)

template <typename T>
static hipError_t inflow_typed(const gals_ctx *ctx, const Vel<T> &p, void *phi, void *grad,
                               double c, double dt, hipStream_t s)
{
    const int64_t count = boundary_count(ctx->g);
    const dim3 grid(unsigned((count + kBlock - 1) / kBlock)), block(kBlock);
    const T cc = T(c);
    T *ph = (T *)phi, *gr = (T *)grad;
    const T *pb = (const T *)ctx->inflow_phi, *gb = (const T *)ctx->inflow_grad,
            *tb = (const T *)ctx->inflow_phit;
#define GALS_INFLOW(D, K)                                                                         \
    case D * 16 + K:                                                                              \
        hipLaunchKernelGGL((k_inflow<T, D, K>), grid, block, 0, s, ctx->g, p, cc, dt, count, ph,  \
                           gr, pb, gb, tb);                                                       \
        break;
    switch (ctx->dim * 16 + ctx->vel_kind) {
        GALS_BOUNDARY_KINDS(GALS_INFLOW)
    default:
        return hipErrorInvalidValue;
    }
#undef GALS_INFLOW
    return hipGetLastError();
}

hipError_t launch_inflow(const gals_ctx *ctx, void *phi, void *grad, double c, double dt,
                         hipStream_t s)
{
    return ctx->prec == GALS_F32 ? inflow_typed<float>(ctx, ctx->vf, phi, grad, c, dt, s)
                                 : inflow_typed<double>(ctx, ctx->vd, phi, grad, c, dt, s);
}

template <typename T, int MIX>
static hipError_t face_typed(const gals_ctx *ctx, const Vel<T> &p, const void *sphi,
                             const void *sgrad, void *dphi, void *dgrad, double dt, double c1,
                             double c2, double c3, hipStream_t s)
{
    const int64_t count = boundary_count(ctx->g);
    const dim3 grid(unsigned((count + kBlock - 1) / kBlock)), block(kBlock);
    const Stage<T> st = make_stage<T>(dt, c1, c2, c3);
    const T *sp = (const T *)sphi, *sg = (const T *)sgrad;
    T *dp = (T *)dphi, *dg = (T *)dgrad;
#define GALS_FACE(D, K)                                                                           \
    case D * 16 + K:                                                                              \
        hipLaunchKernelGGL((k_face<T, D, K, MIX>), grid, block, 0, s, ctx->g, p, st, dt, count,   \
                           sp, sg, dp, dg);                                                       \
        break;
    switch (ctx->dim * 16 + ctx->vel_kind) {
        GALS_BOUNDARY_KINDS(GALS_FACE)
    default:
        return hipErrorInvalidValue;
    }
#undef GALS_FACE
    return hipGetLastError();
}

template <typename T>
static hipError_t face_mix(const gals_ctx *ctx, const Vel<T> &p, const void *sphi,
                           const void *sgrad, void *dphi, void *dgrad, double dt, double c1,
                           double c2, double c3, hipStream_t s)
{
    if (ctx->mixed == GALS_MIXED_CELL)
        return face_typed<T, GALS_MIXED_CELL>(ctx, p, sphi, sgrad, dphi, dgrad, dt, c1, c2, c3, s);
    if (ctx->mixed == GALS_MIXED_ZERO)
        return face_typed<T, GALS_MIXED_ZERO>(ctx, p, sphi, sgrad, dphi, dgrad, dt, c1, c2, c3, s);
    return face_typed<T, GALS_MIXED_CENTRAL>(ctx, p, sphi, sgrad, dphi, dgrad, dt, c1, c2, c3, s);
}

hipError_t launch_face(const gals_ctx *ctx, const void *sphi, const void *sgrad, void *dphi,
                       void *dgrad, double dt, double c1, double c2, double c3, hipStream_t s)
{
    return ctx->prec == GALS_F32
               ? face_mix<float>(ctx, ctx->vf, sphi, sgrad, dphi, dgrad, dt, c1, c2, c3, s)
               : face_mix<double>(ctx, ctx->vd, sphi, sgrad, dphi, dgrad, dt, c1, c2, c3, s);
}

}  // namespace gals
