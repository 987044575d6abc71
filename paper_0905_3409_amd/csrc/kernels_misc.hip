// Point evaluation (value, normal, curvature) and deterministic FP64
// reductions (error norms, shape error, volume, max speed) for gfx950.
#include "hermite.h"
#include "reduce.h"

namespace gals {

constexpr int64_t kEvalMaxBlocks = int64_t(1) << 20;

// ---------------------------------------------------------------------------
// Point evaluation (sec. 3.2): n = grad H / |grad H|, and the curvature
// kappa = div n = (|g|^2 tr(Hess) - g^T Hess g) / |g|^3, which is eq.
// (curvature) in 2D and the sum of the principal curvatures in 3D.
// ---------------------------------------------------------------------------
template <typename T, int D, int MIX>
__device__ __forceinline__ void eval_point(const Geom &g, const T *__restrict__ phi,
                                           const T *__restrict__ grad,
                                           const double *__restrict__ pts, int64_t npts,
                                           int64_t id, T *__restrict__ val,
                                           T *__restrict__ normal, T *__restrict__ curv)
{
    double X[D];
#pragma unroll
    for (int a = 0; a < D; a++) X[a] = pts[a * npts + id];
    int cell[D];
    double xi[D];
    split<D>(g, X, cell, xi);
    T H, G[D], Hs[D * D];
    Basis<T> b[D];
#pragma unroll
    for (int a = 0; a < D; a++) basis<T, true>(T(xi[a]), geo_h<T>(g, a), geo_ih<T>(g, a), b[a]);
    if constexpr (D == 2) {
        T d[4][4];
        gather2d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(grad, g.plane),
                         plane_rsrc(grad + g.plane, g.plane), cell[0], cell[1], d);
        hermite2d_full(d, b[0], b[1], H, G, Hs);
    } else {
        T d[8][8];
        gather3d<T, MIX>(g, plane_rsrc(phi, g.plane), plane_rsrc(grad, g.plane),
                         plane_rsrc(grad + g.plane, g.plane), plane_rsrc(grad + 2 * g.plane, g.plane),
                         cell[0], cell[1], cell[2], d);
        hermite3d_full(d, b[0], b[1], b[2], H, G, Hs);
    }
    T g2 = T(0), tr = T(0), gHg = T(0);
#pragma unroll
    for (int a = 0; a < D; a++) {
        g2 += G[a] * G[a];
        tr += Hs[a * D + a];
#pragma unroll
        for (int c = 0; c < D; c++) gHg += G[a] * Hs[a * D + c] * G[c];
    }
    const bool ok = g2 > T(0);
    const T nrm = sqrt(g2);
    if (val) val[id] = H;
    if (normal) {
#pragma unroll
        for (int a = 0; a < D; a++) normal[a * npts + id] = ok ? G[a] / nrm : T(0);
    }
    if (curv) curv[id] = ok ? (g2 * tr - gHg) / (g2 * nrm) : T(0);
}

template <typename T, int D, int MIX>
__global__ __launch_bounds__(kBlock) void k_eval(Geom g, const T *__restrict__ phi,
                                                 const T *__restrict__ grad,
                                                 const double *__restrict__ pts, int64_t npts,
                                                 T *__restrict__ val, T *__restrict__ normal,
                                                 T *__restrict__ curv)
{
    // grid-stride over the points: the launch caps its grid (eval_typed), so
    // any count the entry point accepts fits the launch's work-item count
    for (int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x; id < npts;
         id += int64_t(gridDim.x) * kBlock)
        eval_point<T, D, MIX>(g, phi, grad, pts, npts, id, val, normal, curv);
}

template <typename T, int MIX>
static hipError_t eval_typed(const gals_ctx *ctx, const void *phi, const void *grad,
                             const double *pts, int64_t npts, void *val, void *normal, void *curv,
                             hipStream_t s)
{
    // at most 2^20 blocks of 256 (2^28 work items); larger counts loop
    const int64_t want = (npts + kBlock - 1) / kBlock;
    const unsigned blocks = unsigned(want < kEvalMaxBlocks ? want : kEvalMaxBlocks);
    if (ctx->dim == 2)
        hipLaunchKernelGGL((k_eval<T, 2, MIX>), dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           (const T *)phi, (const T *)grad, pts, npts, (T *)val, (T *)normal,
                           (T *)curv);
    else
        hipLaunchKernelGGL((k_eval<T, 3, MIX>), dim3(blocks), dim3(kBlock), 0, s, ctx->g,
                           (const T *)phi, (const T *)grad, pts, npts, (T *)val, (T *)normal,
                           (T *)curv);
    return hipGetLastError();
}

hipError_t launch_eval(const gals_ctx *ctx, const void *phi, const void *grad, const double *pts,
                       int64_t npts, void *val, void *normal, void *curv, hipStream_t s)
{
    if (npts == 0) return hipSuccess;
#define GALS_EVAL(T, M) eval_typed<T, M>(ctx, phi, grad, pts, npts, val, normal, curv, s)
    if (ctx->prec == GALS_F32)
        return ctx->mixed == GALS_MIXED_ZERO   ? GALS_EVAL(float, GALS_MIXED_ZERO)
               : ctx->mixed == GALS_MIXED_CELL ? GALS_EVAL(float, GALS_MIXED_CELL)
                                               : GALS_EVAL(float, GALS_MIXED_CENTRAL);
    return ctx->mixed == GALS_MIXED_ZERO   ? GALS_EVAL(double, GALS_MIXED_ZERO)
           : ctx->mixed == GALS_MIXED_CELL ? GALS_EVAL(double, GALS_MIXED_CELL)
                                           : GALS_EVAL(double, GALS_MIXED_CENTRAL);
#undef GALS_EVAL
}

__device__ __forceinline__ int64_t node_offset(const Geom &g, int64_t id)
{
    const int64_t i = id % g.n[0];
    const int64_t r = id / g.n[0];
    return r * g.pitch + i;  // rows of 3D planes are contiguous in (j, k)
}

// slots: 0 max|dphi| 1 max|dpsi| 2 sum|dH| 3 max band 4 sum H(-phi)
//        5 sum H(-phi_ref) 6 nonfinite count 7 max|phi_ref|
constexpr unsigned kNormsMax = (1u << 0) | (1u << 1) | (1u << 3) | (1u << 7);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_norms(Geom g, const T *__restrict__ phi,
                                                  const T *__restrict__ grad,
                                                  const T *__restrict__ phr,
                                                  const T *__restrict__ grr, double eps,
                                                  double band, double *__restrict__ partials)
{
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x; id < g.nodes; id += stride) {
        const int64_t o = node_offset(g, id);
        const double p = double(phi[o]), r = double(phr[o]);
        const double e = fabs(p - r);
        acc[0] = fmax(acc[0], e);
        double nf = isfinite(p) ? 0.0 : 1.0;
        for (int a = 0; a < g.dim; a++) {
            const double q = double(grad[a * g.plane + o]);
            acc[1] = fmax(acc[1], fabs(q - double(grr[a * g.plane + o])));
            nf += isfinite(q) ? 0.0 : 1.0;
        }
        acc[2] += fabs(heaviside_eps(p, eps) - heaviside_eps(r, eps));
        if (fabs(r) <= band) acc[3] = fmax(acc[3], e);
        acc[4] += heaviside_eps(-p, eps);
        acc[5] += heaviside_eps(-r, eps);
        acc[6] += nf;
        acc[7] = fmax(acc[7], fabs(r));
    }
    block_reduce<8>(acc, kNormsMax, partials + int64_t(blockIdx.x) * kRedSlots);
}

hipError_t launch_norms(const gals_ctx *ctx, const void *phi, const void *grad,
                        const void *phi_ref, const void *grad_ref, double eps, double band,
                        double *partials, double *out, hipStream_t s)
{
    if (ctx->prec == GALS_F32)
        hipLaunchKernelGGL(k_norms<float>, dim3(kRedBlocks), dim3(kBlock), 0, s, ctx->g,
                           (const float *)phi, (const float *)grad, (const float *)phi_ref,
                           (const float *)grad_ref, eps, band, partials);
    else
        hipLaunchKernelGGL(k_norms<double>, dim3(kRedBlocks), dim3(kBlock), 0, s, ctx->g,
                           (const double *)phi, (const double *)grad, (const double *)phi_ref,
                           (const double *)grad_ref, eps, band, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold<8>, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks, kNormsMax,
                       out);
    return hipGetLastError();
}

// max over nodes of |v(x_node, t)|, c = c(t)
template <typename T, int D, int KIND>
__global__ __launch_bounds__(kBlock) void k_max_speed(Geom g, Vel<T> p, T c,
                                                      double *__restrict__ partials)
{
    double acc[1] = {0.0};
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t id = int64_t(blockIdx.x) * kBlock + threadIdx.x; id < g.nodes; id += stride) {
        int64_t r = id;
        double x[D];
#pragma unroll
        for (int a = 0; a < D; a++) {
            const int64_t ia = r % g.n[a];
            r /= g.n[a];
            x[a] = node_coord(g.lo[a], ia, g.h[a]);
        }
        T v[D], J[D * D];
        velocity<T, D, KIND>(p, x, c, v, J);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < D; a++) s += double(v[a]) * double(v[a]);
        acc[0] = fmax(acc[0], sqrt(s));
    }
    block_reduce<1>(acc, 1u, partials + int64_t(blockIdx.x) * kRedSlots);
}

template <typename T>
static hipError_t max_speed_typed(const gals_ctx *ctx, const Vel<T> &p, double c,
                                  double *partials, hipStream_t s)
{
    const dim3 grid(kRedBlocks), block(kBlock);
    const T cc = T(c);
    switch (ctx->dim * 16 + ctx->vel_kind) {
    case 2 * 16 + GALS_VEL_AFFINE:
        hipLaunchKernelGGL((k_max_speed<T, 2, GALS_VEL_AFFINE>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 2 * 16 + GALS_VEL_STREAM_SIN:
        hipLaunchKernelGGL((k_max_speed<T, 2, GALS_VEL_STREAM_SIN>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 2 * 16 + GALS_VEL_VORTEX:
        hipLaunchKernelGGL((k_max_speed<T, 2, GALS_VEL_VORTEX>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 2 * 16 + GALS_VEL_PSEUDO1D:
        hipLaunchKernelGGL((k_max_speed<T, 2, GALS_VEL_PSEUDO1D>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 3 * 16 + GALS_VEL_AFFINE:
        hipLaunchKernelGGL((k_max_speed<T, 3, GALS_VEL_AFFINE>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 3 * 16 + GALS_VEL_VECPOT_SIN:
        hipLaunchKernelGGL((k_max_speed<T, 3, GALS_VEL_VECPOT_SIN>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    case 3 * 16 + GALS_VEL_LEVEQUE3D:
        hipLaunchKernelGGL((k_max_speed<T, 3, GALS_VEL_LEVEQUE3D>), grid, block, 0, s, ctx->g, p, cc, partials);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_max_speed(const gals_ctx *ctx, double c, double *partials, double *out,
                            hipStream_t s)
{
    hipError_t e = ctx->prec == GALS_F32 ? max_speed_typed<float>(ctx, ctx->vf, c, partials, s)
                                         : max_speed_typed<double>(ctx, ctx->vd, c, partials, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold<1>, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks, 1u, out);
    return hipGetLastError();
}

}  // namespace gals
