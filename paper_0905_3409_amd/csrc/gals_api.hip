// Host runtime of the C ABI declared in include/gals.h: argument validation,
// velocity-parameter preparation, workspace layout and launch sequencing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "gals_internal.h"

using namespace gals;

namespace {
thread_local char g_err[512] = "";
}

void gals::set_error_v(const char *fmt, va_list ap) { vsnprintf(g_err, sizeof(g_err), fmt, ap); }

namespace {

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    gals::set_error_v(fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GALS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t elem_size(const gals_ctx *c) { return c->prec == GALS_F32 ? 4 : 8; }

size_t state_bytes(const gals_ctx *c)
{
    return size_t(1 + c->dim) * size_t(c->g.plane) * elem_size(c);
}

size_t partial_offset(const gals_ctx *c) { return align256(state_bytes(c)); }

size_t coltab_offset(const gals_ctx *c)
{
    return partial_offset(c) + align256(sizeof(double) * size_t(kRedBlocks + 1) * kRedSlots);
}

size_t rowtab_offset(const gals_ctx *c)
{
    return coltab_offset(c) + align256(size_t(kJet) * size_t(c->g.n[0]) * elem_size(c));
}

size_t axistab_offset(const gals_ctx *c)
{
    return rowtab_offset(c) + align256(size_t(kJet) * size_t(c->g.n[1]) * elem_size(c));
}

size_t workspace_bytes(const gals_ctx *c)
{
    const size_t axis = 2 * size_t(c->g.n[0] + c->g.n[1] + c->g.n[2]) * elem_size(c);
    return axistab_offset(c) + align256(axis);
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

bool aligned(const void *p, size_t a) { return (uintptr_t(p) % a) == 0; }

// Make the context's device current for the duration of a call.
struct DeviceGuard {
    int old = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

double time_factor(double period, double t) { return period > 0.0 ? cos(M_PI * t / period) : 1.0; }

// Stream-function tables into the workspace (sine stream functions only).
hipError_t launch_tables(const gals_ctx *ctx, void *workspace, hipStream_t s)
{
    char *ws = (char *)workspace;
    if (ctx->dim == 3 && ctx->vel_kind == GALS_VEL_VECPOT_SIN)
        return launch_axis_tables(ctx, ws + axistab_offset(ctx), s);
    if (ctx->vel_kind != GALS_VEL_STREAM_SIN) return hipSuccess;
    return launch_stream_tables(ctx, ws + coltab_offset(ctx), ws + rowtab_offset(ctx), s);
}

// Steps n_begin .. n_end-1 of an advance from time t0 (step n starts at
// t0 + n dt), ping-ponging through the workspace's state copy; the result
// ends in (phi, grad). The tables must be in the workspace already.
hipError_t advance_core(const gals_ctx *ctx, void *phi, void *grad, double t0, double dt,
                        int64_t n_begin, int64_t n_end, void *workspace, hipStream_t s)
{
    const size_t pb = size_t(ctx->g.plane) * elem_size(ctx);
    char *ws = (char *)workspace;
    void *bufs[2][2] = {{phi, grad}, {ws, ws + pb}};
    void *coltab = nullptr, *rowtab = nullptr;
    if (ctx->vel_kind == GALS_VEL_STREAM_SIN) {
        coltab = ws + coltab_offset(ctx);
        rowtab = ws + rowtab_offset(ctx);
    } else if (ctx->dim == 3 && ctx->vel_kind == GALS_VEL_VECPOT_SIN) {
        coltab = ws + axistab_offset(ctx);  // the per-axis sin/cos table
    }
    hipError_t e = hipSuccess;
    for (int64_t n = n_begin; n < n_end; n++) {
        const double t = t0 + double(n) * dt;
        const double c1 = time_factor(ctx->period, t + dt);
        const double c2 = time_factor(ctx->period, t);
        const double c3 = time_factor(ctx->period, t + 0.5 * dt);
        void **src = bufs[(n - n_begin) & 1], **dst = bufs[(n - n_begin + 1) & 1];
        e = launch_step(ctx, src[0], src[1], dst[0], dst[1], dt, c1, c2, c3, coltab, rowtab, s);
        if (e == hipSuccess && ctx->inflow) e = launch_inflow(ctx, dst[0], dst[1], c1, dt, s);
        if (e == hipSuccess && ctx->face)
            e = launch_face(ctx, src[0], src[1], dst[0], dst[1], dt, c1, c2, c3, s);
        if (e != hipSuccess) return e;
    }
    if ((n_end - n_begin) & 1) {
        // the result sits in the workspace: copy the valid part of each plane back
        const size_t es = elem_size(ctx);
        const size_t w = size_t(ctx->g.n[0]) * es, p = size_t(ctx->g.pitch) * es;
        const size_t rows = size_t(ctx->g.n[1]) * size_t(ctx->g.n[2]);
        for (int a = 0; a <= ctx->dim && e == hipSuccess; a++) {
            char *dstp = a == 0 ? (char *)phi : (char *)grad + size_t(a - 1) * pb;
            e = hipMemcpy2DAsync(dstp, p, ws + size_t(a) * pb, p, w, rows, hipMemcpyDeviceToDevice, s);
        }
    }
    return e;
}

template <typename T>
void fill_vel(Vel<T> &v, int kind, int dim, const double *p, int64_t np)
{
    memset(&v, 0, sizeof(v));
    v.kind = kind;
    if (kind == GALS_VEL_AFFINE) {
        for (int i = 0; i < dim; i++) {
            v.b[i] = T(p[i]);
            v.c[i] = p[dim + i];
            for (int j = 0; j < dim; j++) v.A[i * 3 + j] = T(p[2 * dim + i * dim + j]);
        }
    } else if (kind == GALS_VEL_STREAM_SIN) {
        double S[4][4] = {{0}};
        for (int64_t k = 0; k < np / 3; k++) {
            const int m = int(p[3 * k + 1]), n = int(p[3 * k + 2]);
            S[m - 1][n - 1] += p[3 * k];
        }
        int mmax = 0, nmax = 0;
        for (int m = 0; m < 4; m++)
            for (int n = 0; n < 4; n++) {
                const double kn = (n + 1) * M_PI;
                v.S[m][n] = T(S[m][n]);
                v.SQ[m][n] = T(S[m][n] * kn);
                v.SR[m][n] = T(S[m][n] * kn * kn);
                if (S[m][n] != 0.0) {
                    mmax = m + 1 > mmax ? m + 1 : mmax;
                    nmax = n + 1 > nmax ? n + 1 : nmax;
                }
            }
        v.kx = T(M_PI * mmax);
        v.ky = T(M_PI * nmax);
    } else if (kind == GALS_VEL_VECPOT_SIN) {
        v.nvp = int(np / 6);
        for (int k = 0; k < v.nvp; k++) {
            const double *q = p + 6 * k;
            const double ax = q[0], ay = q[1], az = q[2];
            const double L = q[3] * M_PI, M = q[4] * M_PI, N = q[5] * M_PI;
            for (int a = 0; a < 3; a++) v.vpi[k][a] = int(q[3 + a]);
            const double c[21] = {az * M, ay * N, ax * N, az * L, ay * L, ax * M,
                                  az * L * M, ay * L * N, az * M * M, ay * M * N, az * M * N,
                                  ay * N * N, ax * L * N, az * L * L, ax * M * N, ax * N * N,
                                  az * L * N, ay * L * L, ax * L * M, ay * L * M, ax * M * M};
            for (int i = 0; i < 21; i++) v.vpc[k][i] = T(c[i]);
        }
    }
}

bool is_int_in(double x, int lo, int hi) { return x == floor(x) && x >= lo && x <= hi; }

// Checks shared by the advances: velocity and inflow data set, finite
// positive dt, finite t0, steps >= 0, state pointers aligned to the element.
int check_advance_args(const gals_ctx *ctx, const void *phi, const void *grad, double t0,
                       double dt, int64_t steps, const char *what)
{
    if (!ctx->vel_set) return fail(GALS_EINVAL, "%s: no velocity set", what);
    if (ctx->inflow && !ctx->inflow_phi)
        return fail(GALS_EINVAL, "%s: GALS_BC_INFLOW without gals_set_inflow_data", what);
    if (!isfinite(dt) || !(dt > 0.0)) return fail(GALS_EINVAL, "%s: dt must be finite and > 0", what);
    if (!isfinite(t0)) return fail(GALS_EINVAL, "%s: t0 must be finite", what);
    if (steps < 0) return fail(GALS_EINVAL, "%s: steps < 0", what);
    const size_t es = elem_size(ctx);
    if (!aligned(phi, es) || !aligned(grad, es)) return fail(GALS_EINVAL, "%s: misaligned pointer", what);
    return GALS_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free advance: a static device array, one copy per
// GPU the library runs on, held until the process ends. In host code the
// array's name is only a host-side stand-in; its device address on each GPU
// comes from hipGetSymbolAddress with that GPU current, resolved on the entry
// point's first call there and kept per device. Every call on a GPU shares
// that GPU's copy.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = GALS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxScratchDevices];

// Device address of `scratch` on `dev`, which must be the current device.
hipError_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *gals_last_error(void) { return g_err; }

int gals_create(gals_ctx **out, int dim, const int64_t *ncell, const double *lo, const double *hi,
                int prec, int mixed_mode, int bc, int device)
{
    if (!out) return fail(GALS_EINVAL, "gals_create: out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(GALS_EINVAL, "gals_create: dim must be 2 or 3 (got %d)", dim);
    if (!ncell || !lo || !hi) return fail(GALS_EINVAL, "gals_create: NULL ncell/lo/hi");
    if (prec != GALS_F32 && prec != GALS_F64)
        return fail(GALS_EINVAL, "gals_create: unknown precision %d", prec);
    if (mixed_mode != GALS_MIXED_CENTRAL && mixed_mode != GALS_MIXED_CELL &&
        mixed_mode != GALS_MIXED_ZERO)
        return fail(GALS_EINVAL, "gals_create: unknown mixed-derivative mode %d", mixed_mode);
    if (bc < GALS_BC_NEUMANN || bc > GALS_BC_INFLOW_NEUMANN)
        return fail(GALS_EINVAL, "gals_create: unknown boundary treatment %d", bc);
    Geom g;
    memset(&g, 0, sizeof(g));
    g.dim = dim;
    g.bc = bc == GALS_BC_EXTRAPOLATE ? bc : GALS_BC_NEUMANN;  // feet outside: projected
    int64_t nodes = 1;
    for (int a = 0; a < 3; a++) {
        g.n[a] = 1;
        g.h[a] = g.inv_h[a] = 1.0;
    }
    for (int a = 0; a < dim; a++) {
        if (ncell[a] < 2 || ncell[a] > (int64_t(1) << 30))
            return fail(GALS_EINVAL, "gals_create: ncell[%d] = %lld out of range [2, 2^30]", a,
                        (long long)ncell[a]);
        if (!isfinite(lo[a]) || !isfinite(hi[a]) || !(hi[a] > lo[a]))
            return fail(GALS_EINVAL, "gals_create: bounds of axis %d must be finite with hi > lo", a);
        g.nc[a] = int(ncell[a]);
        g.n[a] = int(ncell[a] + 1);
        g.lo[a] = lo[a];
        g.h[a] = (hi[a] - lo[a]) / double(ncell[a]);
        g.inv_h[a] = 1.0 / g.h[a];
        g.top[a] = node_coord(g.lo[a], g.nc[a], g.h[a]);
        nodes *= g.n[a];
        if (nodes >= (int64_t(1) << 31))
            return fail(GALS_EINVAL, "gals_create: more than 2^31 - 1 nodes");
    }
    g.nodes = nodes;
    geom_finish(g);
    g.pitch = (int64_t(g.n[0]) + 63) / 64 * 64;
    g.plane = g.pitch * g.n[1] * g.n[2];
    if (g.plane * int64_t(prec == GALS_F32 ? 4 : 8) >= (int64_t(1) << 31))
        return fail(GALS_EINVAL, "gals_create: a state plane of 2 GiB or more");
    if (device != -1) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess) return hip_fail(e, "gals_create: hipGetDeviceCount");
        if (device < 0 || device >= count)
            return fail(GALS_EINVAL, "gals_create: device %d not in [0, %d)", device, count);
    }
    gals_ctx *c = new (std::nothrow) gals_ctx;
    if (!c) return fail(GALS_ENOMEM, "gals_create: out of host memory");
    memset(c, 0, sizeof(*c));
    c->dim = dim;
    c->prec = prec;
    c->mixed = mixed_mode;
    c->device = device;
    c->g = g;
    c->vel_set = false;
    c->inflow = bc == GALS_BC_INFLOW;
    c->face = bc == GALS_BC_INFLOW_NEUMANN;
    *out = c;
    return GALS_OK;
}

int gals_destroy(gals_ctx *ctx)
{
    delete ctx;
    return GALS_OK;
}

int gals_layout(const gals_ctx *ctx, int64_t *nodes, int64_t *pitch, int64_t *plane_stride)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_layout: NULL context");
    if (nodes)
        for (int a = 0; a < ctx->dim; a++) nodes[a] = ctx->g.n[a];
    if (pitch) *pitch = ctx->g.pitch;
    if (plane_stride) *plane_stride = ctx->g.plane;
    return GALS_OK;
}

int gals_workspace_bytes(const gals_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return fail(GALS_EINVAL, "gals_workspace_bytes: NULL argument");
    *bytes = workspace_bytes(ctx);
    return GALS_OK;
}

int gals_set_velocity(gals_ctx *ctx, int kind, const double *params, int64_t nparams,
                      double period)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_set_velocity: NULL context");
    if (nparams < 0 || (nparams > 0 && !params))
        return fail(GALS_EINVAL, "gals_set_velocity: bad parameter vector");
    if (!isfinite(period) || period < 0.0)
        return fail(GALS_EINVAL, "gals_set_velocity: period must be finite and >= 0");
    for (int64_t k = 0; k < nparams; k++)
        if (!isfinite(params[k])) return fail(GALS_EINVAL, "gals_set_velocity: non-finite parameter");
    const int d = ctx->dim;
    switch (kind) {
    case GALS_VEL_AFFINE:
        if (nparams != 2 * d + d * d)
            return fail(GALS_EINVAL, "gals_set_velocity: AFFINE needs %d parameters", 2 * d + d * d);
        break;
    case GALS_VEL_STREAM_SIN:
        if (d != 2) return fail(GALS_EINVAL, "gals_set_velocity: STREAM_SIN is 2D");
        if (nparams == 0 || nparams % 3)
            return fail(GALS_EINVAL, "gals_set_velocity: STREAM_SIN needs 3 parameters per mode");
        if (nparams / 3 > kMaxStreamModes)
            return fail(GALS_ENOTSUP, "gals_set_velocity: at most %d stream modes", kMaxStreamModes);
        for (int64_t k = 0; k < nparams / 3; k++)
            if (!is_int_in(params[3 * k + 1], 1, 4) || !is_int_in(params[3 * k + 2], 1, 4))
                return fail(GALS_ENOTSUP, "gals_set_velocity: wavenumbers must be integers in 1..4");
        break;
    case GALS_VEL_VECPOT_SIN:
        if (d != 3) return fail(GALS_EINVAL, "gals_set_velocity: VECPOT_SIN is 3D");
        if (nparams == 0 || nparams % 6)
            return fail(GALS_EINVAL, "gals_set_velocity: VECPOT_SIN needs 6 parameters per mode");
        if (nparams / 6 > kMaxVecpotModes)
            return fail(GALS_ENOTSUP, "gals_set_velocity: at most %d vector-potential modes",
                        kMaxVecpotModes);
        for (int64_t k = 0; k < nparams / 6; k++)
            for (int a = 3; a < 6; a++)
                if (!is_int_in(params[6 * k + a], 1, 4))
                    return fail(GALS_ENOTSUP, "gals_set_velocity: wavenumbers must be integers in 1..4");
        break;
    case GALS_VEL_VORTEX:
    case GALS_VEL_PSEUDO1D:
        if (d != 2) return fail(GALS_EINVAL, "gals_set_velocity: field %d is 2D", kind);
        if (nparams != 0) return fail(GALS_EINVAL, "gals_set_velocity: field %d takes no parameters", kind);
        break;
    case GALS_VEL_LEVEQUE3D:
        if (d != 3) return fail(GALS_EINVAL, "gals_set_velocity: LEVEQUE3D is 3D");
        if (nparams != 0) return fail(GALS_EINVAL, "gals_set_velocity: LEVEQUE3D takes no parameters");
        break;
    default:
        return fail(GALS_EINVAL, "gals_set_velocity: unknown velocity kind %d", kind);
    }
    ctx->vel_kind = kind;
    ctx->period = period;
    fill_vel(ctx->vf, kind, d, params, nparams);
    fill_vel(ctx->vd, kind, d, params, nparams);
    ctx->vel_set = true;
    return GALS_OK;
}

int gals_set_inflow_data(gals_ctx *ctx, const void *phi_b, const void *grad_b,
                         const void *phit_b)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_set_inflow_data: NULL context");
    if (!ctx->inflow)
        return fail(GALS_EINVAL, "gals_set_inflow_data: the context was not created with "
                                 "GALS_BC_INFLOW");
    if (!phi_b || !grad_b || !phit_b) return fail(GALS_EINVAL, "gals_set_inflow_data: NULL array");
    const size_t es = elem_size(ctx);
    if (!aligned(phi_b, es) || !aligned(grad_b, es) || !aligned(phit_b, es))
        return fail(GALS_EINVAL, "gals_set_inflow_data: misaligned array");
    ctx->inflow_phi = phi_b;
    ctx->inflow_grad = grad_b;
    ctx->inflow_phit = phit_b;
    return GALS_OK;
}

int gals_set_psi_update(gals_ctx *ctx, int mode)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_set_psi_update: NULL context");
    if (mode != GALS_PSI_SUPERCONSISTENT && mode != GALS_PSI_HEUN)
        return fail(GALS_EINVAL, "gals_set_psi_update: unknown mode %d", mode);
    ctx->psi = mode;
    return GALS_OK;
}

int gals_advance(gals_ctx *ctx, void *phi, void *grad, double t0, double dt, int64_t steps,
                 void *workspace, size_t workspace_bytes_, void *stream)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_advance: NULL context");
    if (!phi || !grad || !workspace) return fail(GALS_EINVAL, "gals_advance: NULL pointer");
    int rc = check_advance_args(ctx, phi, grad, t0, dt, steps, "gals_advance");
    if (rc != GALS_OK) return rc;
    const size_t es = elem_size(ctx);
    if (!aligned(workspace, 256)) return fail(GALS_EINVAL, "gals_advance: misaligned pointer");
    if (workspace_bytes_ < workspace_bytes(ctx))
        return fail(GALS_EINVAL, "gals_advance: workspace of %zu bytes, %zu needed", workspace_bytes_,
                    workspace_bytes(ctx));
    const size_t pb = size_t(ctx->g.plane) * es;
    const size_t gb = pb * size_t(ctx->dim);
    if (overlap(phi, pb, grad, gb) || overlap(phi, pb, workspace, workspace_bytes_) ||
        overlap(grad, gb, workspace, workspace_bytes_))
        return fail(GALS_EINVAL, "gals_advance: phi, grad and workspace must not overlap");
    if (steps == 0) return GALS_OK;
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_advance: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_advance: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_advance: pending HIP error");
    hipStream_t s = (hipStream_t)stream;
    e = launch_tables(ctx, workspace, s);
    if (e == hipSuccess) e = advance_core(ctx, phi, grad, t0, dt, 0, steps, workspace, s);
    return e == hipSuccess ? GALS_OK : hip_fail(e, "gals_advance: launch");
}

int gals_advance_noalloc(gals_ctx *ctx, void *phi, void *grad, double t0, double dt,
                         int64_t steps, void *stream)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_advance_noalloc: NULL context");
    if (!phi || !grad) return fail(GALS_EINVAL, "gals_advance_noalloc: NULL pointer");
    int rc = check_advance_args(ctx, phi, grad, t0, dt, steps, "gals_advance_noalloc");
    if (rc != GALS_OK) return rc;
    const size_t need = workspace_bytes(ctx);
    if (need > kScratchBytes)
        return fail(GALS_EINVAL,
                    "gals_advance_noalloc: the grid needs %zu bytes of scratch, the library's "
                    "static scratch holds %zu (use gals_advance with a workspace)",
                    need, kScratchBytes);
    const size_t pb = size_t(ctx->g.plane) * elem_size(ctx);
    if (overlap(phi, pb, grad, pb * size_t(ctx->dim)))
        return fail(GALS_EINVAL, "gals_advance_noalloc: phi and grad must not overlap");
    if (steps == 0) return GALS_OK;
    if (ctx->device < 0)
        return fail(GALS_EINVAL, "gals_advance_noalloc: host-only context (device -1)");
    if (ctx->device >= kMaxScratchDevices)
        return fail(GALS_EINVAL, "gals_advance_noalloc: device %d beyond the %d supported",
                    ctx->device, kMaxScratchDevices);
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_advance_noalloc: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_advance_noalloc: pending HIP error");
    void *ws = nullptr;
    e = scratch_address(ctx->device, &ws);
    if (e != hipSuccess) return hip_fail(e, "gals_advance_noalloc: hipGetSymbolAddress");
    hipStream_t s = (hipStream_t)stream;
    e = launch_tables(ctx, ws, s);
    if (e == hipSuccess) e = advance_core(ctx, phi, grad, t0, dt, 0, steps, ws, s);
    return e == hipSuccess ? GALS_OK : hip_fail(e, "gals_advance_noalloc: launch");
}

int gals_eval_points(gals_ctx *ctx, const void *phi, const void *grad, const double *pts,
                     int64_t npts, void *val, void *normal, void *curv, void *stream)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_eval_points: NULL context");
    if (npts < 0) return fail(GALS_EINVAL, "gals_eval_points: npts < 0");
    if (npts == 0) return GALS_OK;
    if (!phi || !grad || !pts) return fail(GALS_EINVAL, "gals_eval_points: NULL pointer");
    if (npts >= (int64_t(1) << 40)) return fail(GALS_EINVAL, "gals_eval_points: too many points");
    const size_t es = elem_size(ctx);
    if (!aligned(phi, es) || !aligned(grad, es) || !aligned(pts, 8) || !aligned(val, es) ||
        !aligned(normal, es) || !aligned(curv, es))
        return fail(GALS_EINVAL, "gals_eval_points: misaligned pointer");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_eval_points: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_eval_points: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_eval_points: pending HIP error");
    e = launch_eval(ctx, phi, grad, pts, npts, val, normal, curv, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gals_eval_points: launch");
    return GALS_OK;
}

static int finish_reduction(const gals_ctx *ctx, const double *dev_out, double *host_out, int n,
                            hipStream_t s, const char *what)
{
    (void)ctx;
    hipError_t e = hipMemcpyAsync(host_out, dev_out, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, what);
    return GALS_OK;
}

int gals_max_speed(gals_ctx *ctx, double t, double *out, void *workspace, size_t workspace_bytes_,
                   void *stream)
{
    if (!ctx || !out || !workspace) return fail(GALS_EINVAL, "gals_max_speed: NULL argument");
    if (!ctx->vel_set) return fail(GALS_EINVAL, "gals_max_speed: no velocity set");
    if (!isfinite(t)) return fail(GALS_EINVAL, "gals_max_speed: t must be finite");
    if (!aligned(workspace, 256) || workspace_bytes_ < workspace_bytes(ctx))
        return fail(GALS_EINVAL, "gals_max_speed: workspace too small or misaligned");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_max_speed: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_max_speed: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_max_speed: pending HIP error");
    double *part = (double *)((char *)workspace + partial_offset(ctx));
    double *res = part + size_t(kRedBlocks) * kRedSlots;
    hipStream_t s = (hipStream_t)stream;
    e = launch_max_speed(ctx, time_factor(ctx->period, t), part, res, s);
    if (e != hipSuccess) return hip_fail(e, "gals_max_speed: launch");
    return finish_reduction(ctx, res, out, 1, s, "gals_max_speed: copy");
}

int gals_norms(gals_ctx *ctx, const void *phi, const void *grad, const void *phi_ref,
               const void *grad_ref, double eps, double band, double *out, void *workspace,
               size_t workspace_bytes_, void *stream)
{
    if (!ctx || !out || !workspace) return fail(GALS_EINVAL, "gals_norms: NULL argument");
    if (!phi || !grad || !phi_ref || !grad_ref) return fail(GALS_EINVAL, "gals_norms: NULL state");
    if (!isfinite(eps) || !(eps > 0.0) || !isfinite(band) || band < 0.0)
        return fail(GALS_EINVAL, "gals_norms: eps must be > 0 and band >= 0");
    if (!aligned(workspace, 256) || workspace_bytes_ < workspace_bytes(ctx))
        return fail(GALS_EINVAL, "gals_norms: workspace too small or misaligned");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_norms: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_norms: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_norms: pending HIP error");
    double *part = (double *)((char *)workspace + partial_offset(ctx));
    double *res = part + size_t(kRedBlocks) * kRedSlots;
    hipStream_t s = (hipStream_t)stream;
    e = launch_norms(ctx, phi, grad, phi_ref, grad_ref, eps, band, part, res, s);
    if (e != hipSuccess) return hip_fail(e, "gals_norms: launch");
    int rc = finish_reduction(ctx, res, out, 8, s, "gals_norms: copy");
    if (rc != GALS_OK) return rc;
    double cellvol = 1.0;
    for (int a = 0; a < ctx->dim; a++) cellvol *= ctx->g.h[a];
    out[2] *= cellvol;
    out[4] *= cellvol;
    out[5] *= cellvol;
    return GALS_OK;
}


/* ---------------------------------------------------------------------------
 * Adjoint of the advance (2D sine stream-function fields).
 * Workspace: [forward workspace | `every` segment states | one adjoint state
 * (3 FP64 planes) | per-block partials of dF/dS (16 FP64 each)].
 * ------------------------------------------------------------------------- */
}  // extern "C"

namespace {

size_t seg_state_bytes(const gals_ctx *c) { return align256(state_bytes(c)); }
size_t lam_bytes(const gals_ctx *c) { return 3 * size_t(c->g.plane) * sizeof(double); }

size_t adj_seg_offset(const gals_ctx *c) { return align256(workspace_bytes(c)); }
size_t adj_lam_offset(const gals_ctx *c, int64_t every)
{
    return adj_seg_offset(c) + size_t(every) * seg_state_bytes(c);
}
size_t adj_part_offset(const gals_ctx *c, int64_t every)
{
    return adj_lam_offset(c, every) + align256(lam_bytes(c));
}
size_t adj_workspace_bytes(const gals_ctx *c, int64_t every)
{
    return adj_part_offset(c, every) +
           align256(sizeof(double) * 16 * size_t(adjoint_blocks(c)));
}

int64_t nsegments(int64_t steps, int64_t every) { return (steps + every - 1) / every; }

int check_adjoint_ctx(const gals_ctx *ctx, const char *what)
{
    if (!ctx) return fail(GALS_EINVAL, "%s: NULL context", what);
    if (!ctx->vel_set) return fail(GALS_EINVAL, "%s: no velocity set", what);
    if (ctx->dim != 2 || ctx->vel_kind != GALS_VEL_STREAM_SIN)
        return fail(GALS_ENOTSUP, "%s: the adjoint covers 2D GALS_VEL_STREAM_SIN fields", what);
    if (ctx->psi != GALS_PSI_SUPERCONSISTENT)
        return fail(GALS_ENOTSUP, "%s: the adjoint covers the superconsistent gradient update",
                    what);
    if (ctx->inflow || ctx->face)
        return fail(GALS_ENOTSUP, "%s: no adjoint of the inflow boundary conditions", what);
    return GALS_OK;
}

// Copy a state (phi plane, then dim gradient planes) to/from one contiguous
// checkpoint slot.
hipError_t copy_state(const gals_ctx *ctx, void *dphi, void *dgrad, const void *sphi,
                      const void *sgrad, hipStream_t s)
{
    const size_t pb = size_t(ctx->g.plane) * elem_size(ctx);
    hipError_t e = hipMemcpyAsync(dphi, sphi, pb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dgrad, sgrad, pb * size_t(ctx->dim), hipMemcpyDeviceToDevice, s);
    return e;
}

}  // namespace

extern "C" {

int gals_checkpoint_bytes(const gals_ctx *ctx, int64_t steps, int64_t every, size_t *bytes)
{
    if (!ctx || !bytes) return fail(GALS_EINVAL, "gals_checkpoint_bytes: NULL argument");
    if (steps < 0 || every < 1) return fail(GALS_EINVAL, "gals_checkpoint_bytes: steps >= 0, every >= 1");
    *bytes = size_t(nsegments(steps, every)) * seg_state_bytes(ctx);
    return GALS_OK;
}

int gals_adjoint_workspace_bytes(const gals_ctx *ctx, int64_t every, size_t *bytes)
{
    if (!ctx || !bytes) return fail(GALS_EINVAL, "gals_adjoint_workspace_bytes: NULL argument");
    if (every < 1 || every > (int64_t(1) << 20))
        return fail(GALS_EINVAL, "gals_adjoint_workspace_bytes: every must be in [1, 2^20]");
    *bytes = adj_workspace_bytes(ctx, every);
    return GALS_OK;
}

int gals_advance_save(gals_ctx *ctx, void *phi, void *grad, double t0, double dt, int64_t steps,
                      int64_t every, void *ckpt, size_t ckpt_bytes, void *workspace,
                      size_t workspace_bytes_, void *stream)
{
    if (!ctx) return fail(GALS_EINVAL, "gals_advance_save: NULL context");
    if (every < 1) return fail(GALS_EINVAL, "gals_advance_save: every must be >= 1");
    if (!ckpt && steps > 0) return fail(GALS_EINVAL, "gals_advance_save: NULL checkpoint store");
    size_t need = 0;
    if (steps >= 0) need = size_t(nsegments(steps, every)) * seg_state_bytes(ctx);
    if (steps > 0 && (ckpt_bytes < need || !aligned(ckpt, 256)))
        return fail(GALS_EINVAL, "gals_advance_save: checkpoint store of %zu bytes, %zu needed "
                                 "(256-byte aligned)", ckpt_bytes, need);
    // the argument checks of gals_advance, without running it
    int rc = gals_advance(ctx, phi, grad, t0, dt, 0, workspace, workspace_bytes_, stream);
    if (rc != GALS_OK) return rc;
    if (steps < 0) return fail(GALS_EINVAL, "gals_advance_save: steps < 0");
    if (steps == 0) return GALS_OK;
    const size_t pb = size_t(ctx->g.plane) * elem_size(ctx);
    if (overlap(ckpt, ckpt_bytes, phi, pb) || overlap(ckpt, ckpt_bytes, grad, pb * ctx->dim) ||
        overlap(ckpt, ckpt_bytes, workspace, workspace_bytes_))
        return fail(GALS_EINVAL, "gals_advance_save: the checkpoint store overlaps another buffer");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_advance_save: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_advance_save: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_advance_save: pending HIP error");
    hipStream_t s = (hipStream_t)stream;
    e = launch_tables(ctx, workspace, s);
    for (int64_t k = 0; k < nsegments(steps, every) && e == hipSuccess; k++) {
        char *slot = (char *)ckpt + size_t(k) * seg_state_bytes(ctx);
        e = copy_state(ctx, slot, slot + pb, phi, grad, s);
        const int64_t n0 = k * every, n1 = n0 + every < steps ? n0 + every : steps;
        if (e == hipSuccess) e = advance_core(ctx, phi, grad, t0, dt, n0, n1, workspace, s);
    }
    return e == hipSuccess ? GALS_OK : hip_fail(e, "gals_advance_save: launch");
}

int gals_adjoint(gals_ctx *ctx, const void *ckpt, size_t ckpt_bytes, double t0, double dt,
                 int64_t steps, int64_t every, double *lam, double *dS, void *workspace,
                 size_t workspace_bytes_, void *stream)
{
    int rc = check_adjoint_ctx(ctx, "gals_adjoint");
    if (rc != GALS_OK) return rc;
    if (!lam || !dS || !workspace) return fail(GALS_EINVAL, "gals_adjoint: NULL pointer");
    if (!isfinite(dt) || !(dt > 0.0) || !isfinite(t0))
        return fail(GALS_EINVAL, "gals_adjoint: dt must be finite and > 0, t0 finite");
    if (steps < 0 || every < 1 || every > (int64_t(1) << 20))
        return fail(GALS_EINVAL, "gals_adjoint: steps >= 0 and every in [1, 2^20]");
    const size_t need_ck = size_t(nsegments(steps, every)) * seg_state_bytes(ctx);
    if (steps > 0 && (!ckpt || ckpt_bytes < need_ck || !aligned(ckpt, 256)))
        return fail(GALS_EINVAL, "gals_adjoint: checkpoint store of %zu bytes, %zu needed",
                    ckpt_bytes, need_ck);
    const size_t need = adj_workspace_bytes(ctx, every);
    if (workspace_bytes_ < need || !aligned(workspace, 256))
        return fail(GALS_EINVAL, "gals_adjoint: workspace of %zu bytes, %zu needed (256-byte aligned)",
                    workspace_bytes_, need);
    if (!aligned(lam, 8) || !aligned(dS, 8)) return fail(GALS_EINVAL, "gals_adjoint: misaligned pointer");
    if (overlap(lam, lam_bytes(ctx), workspace, workspace_bytes_) ||
        overlap(dS, 16 * sizeof(double), workspace, workspace_bytes_) ||
        overlap(lam, lam_bytes(ctx), dS, 16 * sizeof(double)) ||
        (steps > 0 && (overlap(ckpt, ckpt_bytes, workspace, workspace_bytes_) ||
                       overlap(ckpt, ckpt_bytes, lam, lam_bytes(ctx)))))
        return fail(GALS_EINVAL, "gals_adjoint: buffers overlap");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_adjoint: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_adjoint: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_adjoint: pending HIP error");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const size_t pb = size_t(ctx->g.plane) * elem_size(ctx);
    const size_t sb = seg_state_bytes(ctx);
    char *seg = ws + adj_seg_offset(ctx);
    double *lamA = lam, *lamB = (double *)(ws + adj_lam_offset(ctx, every));
    double *part = (double *)(ws + adj_part_offset(ctx, every));
    const int nblocks = int(adjoint_blocks(ctx));
    void *coltab = ws + coltab_offset(ctx), *rowtab = ws + rowtab_offset(ctx);
    e = launch_tables(ctx, workspace, s);
    if (e == hipSuccess) e = launch_zero(part, int64_t(nblocks) * 16, s);
    if (e == hipSuccess) e = launch_zero(dS, 16, s);
    // each adjoint step zeroes the buffer it reads, which then receives the
    // next step's scatter: only the first target needs a fill
    if (e == hipSuccess) e = launch_zero(lamB, 3 * ctx->g.plane, s);
    for (int64_t k = nsegments(steps, every) - 1; k >= 0 && e == hipSuccess; k--) {
        const int64_t n0 = k * every, len = n0 + every < steps ? every : steps - n0;
        // recompute the states of this segment from its checkpoint
        const char *slot = (const char *)ckpt + size_t(k) * sb;
        e = copy_state(ctx, seg, seg + pb, slot, slot + pb, s);
        const void *coltab_c = coltab, *rowtab_c = rowtab;
        for (int64_t q = 1; q < len && e == hipSuccess; q++) {
            const double t = t0 + double(n0 + q - 1) * dt;
            char *src = seg + size_t(q - 1) * sb, *dst = seg + size_t(q) * sb;
            e = launch_step(ctx, src, src + pb, dst, dst + pb, dt,
                            time_factor(ctx->period, t + dt), time_factor(ctx->period, t),
                            time_factor(ctx->period, t + 0.5 * dt), coltab_c, rowtab_c, s);
        }
        // reverse sweep over the segment
        for (int64_t q = len - 1; q >= 0 && e == hipSuccess; q--) {
            const double t = t0 + double(n0 + q) * dt;
            const char *u = seg + size_t(q) * sb;
            e = launch_adjoint_step(ctx, u, u + pb, lamA, lamB, true, part, dt,
                                    time_factor(ctx->period, t + dt), time_factor(ctx->period, t),
                                    time_factor(ctx->period, t + 0.5 * dt), coltab, rowtab, s);
            double *tmp = lamA;
            lamA = lamB;
            lamB = tmp;
        }
    }
    if (e == hipSuccess && lamA != lam)
        e = hipMemcpyAsync(lam, lamA, lam_bytes(ctx), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_fold_grad(part, nblocks, dS, s);
    return e == hipSuccess ? GALS_OK : hip_fail(e, "gals_adjoint: launch");
}

int gals_adjoint_step(gals_ctx *ctx, const void *phi, const void *grad, double t, double dt,
                      const double *lam_in, double *lam_out, double *dS, void *workspace,
                      size_t workspace_bytes_, void *stream)
{
    int rc = check_adjoint_ctx(ctx, "gals_adjoint_step");
    if (rc != GALS_OK) return rc;
    if (!phi || !grad || !lam_in || !lam_out || !dS || !workspace)
        return fail(GALS_EINVAL, "gals_adjoint_step: NULL pointer");
    if (!isfinite(dt) || !(dt > 0.0) || !isfinite(t))
        return fail(GALS_EINVAL, "gals_adjoint_step: dt must be finite and > 0, t finite");
    const size_t need = adj_workspace_bytes(ctx, 1);
    if (workspace_bytes_ < need || !aligned(workspace, 256))
        return fail(GALS_EINVAL, "gals_adjoint_step: workspace of %zu bytes, %zu needed",
                    workspace_bytes_, need);
    const size_t es = elem_size(ctx), pb = size_t(ctx->g.plane) * es;
    if (!aligned(phi, es) || !aligned(grad, es) || !aligned(lam_in, 8) || !aligned(lam_out, 8) ||
        !aligned(dS, 8))
        return fail(GALS_EINVAL, "gals_adjoint_step: misaligned pointer");
    if (overlap(lam_in, lam_bytes(ctx), lam_out, lam_bytes(ctx)) ||
        overlap(lam_out, lam_bytes(ctx), workspace, workspace_bytes_) ||
        overlap(lam_out, lam_bytes(ctx), phi, pb) || overlap(lam_out, lam_bytes(ctx), grad, 2 * pb) ||
        overlap(dS, 16 * sizeof(double), lam_out, lam_bytes(ctx)) ||
        overlap(dS, 16 * sizeof(double), workspace, workspace_bytes_))
        return fail(GALS_EINVAL, "gals_adjoint_step: buffers overlap");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_adjoint_step: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_adjoint_step: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_adjoint_step: pending HIP error");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    double *part = (double *)(ws + adj_part_offset(ctx, 1));
    const int nblocks = int(adjoint_blocks(ctx));
    e = launch_tables(ctx, workspace, s);
    if (e == hipSuccess) e = launch_zero(part, int64_t(nblocks) * 16, s);
    if (e == hipSuccess) e = launch_zero(lam_out, 3 * ctx->g.plane, s);
    if (e == hipSuccess)
        e = launch_adjoint_step(ctx, phi, grad, const_cast<double *>(lam_in), lam_out, false, part, dt,
                                time_factor(ctx->period, t + dt), time_factor(ctx->period, t),
                                time_factor(ctx->period, t + 0.5 * dt), ws + coltab_offset(ctx),
                                ws + rowtab_offset(ctx), s);
    if (e == hipSuccess) e = launch_fold_grad(part, nblocks, dS, s);
    return e == hipSuccess ? GALS_OK : hip_fail(e, "gals_adjoint_step: launch");
}

int gals_shape_loss(gals_ctx *ctx, const void *phi, const void *phi_ref, double eps, double *loss,
                    double *lam, void *workspace, size_t workspace_bytes_, void *stream)
{
    if (!ctx || !phi || !phi_ref || !loss || !workspace)
        return fail(GALS_EINVAL, "gals_shape_loss: NULL argument");
    if (ctx->dim != 2) return fail(GALS_ENOTSUP, "gals_shape_loss: 2D grids only");
    if (!isfinite(eps) || !(eps > 0.0)) return fail(GALS_EINVAL, "gals_shape_loss: eps must be > 0");
    if (!aligned(workspace, 256) || workspace_bytes_ < workspace_bytes(ctx))
        return fail(GALS_EINVAL, "gals_shape_loss: workspace too small or misaligned");
    if (lam && (!aligned(lam, 8) || overlap(lam, lam_bytes(ctx), workspace, workspace_bytes_)))
        return fail(GALS_EINVAL, "gals_shape_loss: lam misaligned or overlapping the workspace");
    if (ctx->device < 0) return fail(GALS_EINVAL, "gals_shape_loss: host-only context (device -1)");
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "gals_shape_loss: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gals_shape_loss: pending HIP error");
    double *part = (double *)((char *)workspace + partial_offset(ctx));
    double *res = part + size_t(kRedBlocks) * kRedSlots;
    hipStream_t s = (hipStream_t)stream;
    e = launch_heaviside_loss(ctx, phi, phi_ref, eps, lam, part, res, s);
    if (e != hipSuccess) return hip_fail(e, "gals_shape_loss: launch");
    const int rc = finish_reduction(ctx, res, loss, 1, s, "gals_shape_loss: copy");
    if (rc != GALS_OK) return rc;
    double cellvol = 1.0;
    for (int a = 0; a < ctx->dim; a++) cellvol *= ctx->g.h[a];
    *loss *= cellvol;
    return GALS_OK;
}

}  // extern "C"
