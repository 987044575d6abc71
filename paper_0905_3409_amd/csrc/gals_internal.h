// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include "../../include/gals.h"

namespace gals {

constexpr int kBlock = 256;          // threads per block of every node/point kernel
constexpr int kMaxStreamModes = 64;  // user modes of GALS_VEL_STREAM_SIN
constexpr int kMaxVecpotModes = 8;   // user modes of GALS_VEL_VECPOT_SIN
constexpr int kRedBlocks = 1024;     // partial sums of the deterministic reductions
constexpr int kRedSlots = 8;         // doubles per partial
constexpr int kJetTaylor = 20;       // stream-function jet entries per column / row
constexpr int kJet = 24;             // table stride: the jet, sin and cos of pi x, 2 unused
// Taylor evaluation of the FP32 stream-function velocity at a stage point is
// used while kx |dx| + ky |dy| stays below kTaylorMax (truncation < FP32
// rounding), and below kTaylorMax2 a degree lower: velocity degree 2 and its
// Jacobian degree 1, whose dropped terms are (k d)^3 / 6 = 1.5e-8 of the
// velocity and, through dt grad v <= k d, (k d)^3 / 2 = 4.6e-8 in the
// superconsistent Jacobian (at most one FP32 ulp).
constexpr float kTaylorMax = 0.03f;
constexpr float kTaylorMax2 = 0.0045f;

// A foot counts as outside the domain only when it lies more than kFootTol
// cells beyond the boundary (see project_foot).
constexpr double kFootTol = 1e-6;

// Grid geometry, passed by value to kernels.
struct Geom {
    int dim;
    int bc;          // GALS_BC_NEUMANN or GALS_BC_EXTRAPOLATE
    double top[3];   // lo + ncell * h: the last node of each axis
    int n[3];        // nodes per axis (1 for unused axes)
    int nc[3];       // cells per axis
    double lo[3];
    double h[3];
    double inv_h[3];
    int64_t pitch;   // row pitch in elements
    int64_t plane;   // plane stride in elements
    int64_t nodes;   // n[0]*n[1]*n[2]
    // derived by geom_finish, so that kernels need no per-wave conversions:
    double ncd[3];   // nc as double
    double lastc[3]; // nc - 1 as double (the last cell)
    // a foot (in cell units) below lowc or above outc is outside the domain:
    // -kFootTol and nc + kFootTol under GALS_BC_NEUMANN, -inf and +inf (never)
    // under GALS_BC_EXTRAPOLATE
    double lowc[3], outc[3];
    float hf[3], ihf[3], i2hf[3];  // h, 1/h, 1/(2h) rounded to FP32
    // 2D node tiles of 64 x 4: per row group, in all, and floor(2^32 /
    // tiles_x) (2^32 - 1 for one tile a row) for the division by tiles_x
    unsigned tiles_x, tiles, tiles_x_magic;
    unsigned n_magic[3];  // floor(2^32 / n[a]) (2^32 - 1 for one node): see udiv_magic
};

// x / d and x % d for 32-bit x from m = floor(2^32 / d) (2^32 - 1 for d = 1):
// floor(x m / 2^32) is the quotient or one less, so a multiply-high and one
// correction give it exactly for every x.
__device__ __forceinline__ unsigned udiv_magic(unsigned x, unsigned d, unsigned m, unsigned &r)
{
    unsigned q = __umulhi(x, m);
    r = x - q * d;
    if (r >= d) {
        q += 1u;
        r -= d;
    }
    return q;
}

// Fill the derived fields of a Geom whose bc, nc, h and inv_h are set.
inline void geom_finish(Geom &g)
{
    for (int a = 0; a < 3; a++) {
        g.ncd[a] = double(g.nc[a]);
        g.lastc[a] = double(g.nc[a] - 1);
        const bool proj = g.bc == GALS_BC_NEUMANN;
        g.lowc[a] = proj ? -kFootTol : -__builtin_inf();
        g.outc[a] = proj ? double(g.nc[a]) + kFootTol : __builtin_inf();
        g.hf[a] = float(g.h[a]);
        g.ihf[a] = float(g.inv_h[a]);
        g.i2hf[a] = float(0.5 * g.inv_h[a]);
    }
    g.tiles_x = unsigned((g.n[0] + 63) / 64);
    g.tiles = g.tiles_x * unsigned((g.n[1] + 3) / 4);
    g.tiles_x_magic = g.tiles_x > 1 ? unsigned((uint64_t(1) << 32) / g.tiles_x) : 0xFFFFFFFFu;
    for (int a = 0; a < 3; a++)
        g.n_magic[a] = g.n[a] > 1 ? unsigned((uint64_t(1) << 32) / unsigned(g.n[a])) : 0xFFFFFFFFu;
}

// h, 1/h and 1/(2h) of axis a in the working precision T.
template <typename T>
__device__ __forceinline__ T geo_h(const Geom &g, int a)
{
    if constexpr (sizeof(T) == 4) return g.hf[a];
    else return g.h[a];
}
template <typename T>
__device__ __forceinline__ T geo_ih(const Geom &g, int a)
{
    if constexpr (sizeof(T) == 4) return g.ihf[a];
    else return g.inv_h[a];
}
template <typename T>
__device__ __forceinline__ T geo_i2h(const Geom &g, int a)
{
    if constexpr (sizeof(T) == 4) return g.i2hf[a];
    else return 0.5 * g.inv_h[a];
}

// Coordinate of node i along an axis: lo + i h with the product rounded before
// the sum, never fused, on the host and in every kernel alike. A fused value
// can land one ulp beyond top (computed the same way), and a foot at that
// node would then count as outside the domain.
__host__ __device__ inline double node_coord(double lo, int64_t i, double h)
{
#pragma clang fp contract(off)
    return lo + double(i) * h;
}

// Velocity parameters in the arithmetic type T, passed by value to kernels.
// Stream-function modes are folded into dense 4x4 tables over (m,n) so that
// every loop is fully unrolled with compile-time wavenumbers.
template <typename T>
struct Vel {
    int kind;
    // AFFINE: v = b + A (x - c); A[i*3+j] = dv_i/dx_j
    T b[3];
    double c[3];
    T A[9];
    // STREAM_SIN: S[m][n] = sum of a over modes with wavenumbers (m+1, n+1);
    // SQ = S * (n+1) pi, SR = S * ((n+1) pi)^2
    T S[4][4], SQ[4][4], SR[4][4];
    T kx, ky;  // pi * largest wavenumber present along x, y
    // VECPOT_SIN, per mode: wavenumber indices (1..4) and 21 coefficients
    // (amplitude times pi-scaled wavenumber products, see vel_vecpot)
    int nvp;
    int vpi[kMaxVecpotModes][3];
    T vpc[kMaxVecpotModes][21];
};

// Per-step factors of the three Shu-Osher stages: the time factors c1, c2,
// c3 = c(t+dt), c(t), c(t+dt/2), and the stage weights with dt and the time
// factors folded in, for traces that carry each stage's field without its
// time factor (w_k = v_k / c_k, R_k = grad v_k / c_k):
//   x1 = x - e1 w0, x2 = x - q1 w0 - q2 w1, foot = x - f1 w0 - f2 w1 - f3 w2
// with e1 = dt c1, q1 = dt c1 / 4, q2 = dt c2 / 4, f1 = dt c1 / 6,
// f2 = dt c2 / 6, f3 = 2 dt c3 / 3, each rounded once to T. Built on the host
// by make_stage, identically for every launcher.
template <typename T>
struct Stage {
    T c1, c2, c3;
    T e1, q1, q2, f1, f2, f3;
};

template <typename T>
inline Stage<T> make_stage(double dt, double c1, double c2, double c3)
{
    Stage<T> s;
    s.c1 = T(c1);
    s.c2 = T(c2);
    s.c3 = T(c3);
    s.e1 = T(dt * c1);
    s.q1 = T(dt * c1 * 0.25);
    s.q2 = T(dt * c2 * 0.25);
    s.f1 = T(dt * c1 / 6.0);
    s.f2 = T(dt * c2 / 6.0);
    s.f3 = T(dt * c3 * 2.0 / 3.0);
    return s;
}

// One problem of a batch (sine stream-function fields only): its geometry,
// its velocity tables, where its state and stream tables live, and the wave
// shape its tiles use (nodes per wave along x: 64, 32 or 16).
template <typename T>
struct BatchProb {
    Geom g;
    T S[4][4], SQ[4][4], SR[4][4];
    T kx, ky;
    int64_t off;       // element offset of this problem's phi plane in the batch state
    int64_t tab;       // element offset of its column table (row table follows)
    unsigned wx;       // nodes per wave along x; 0: row-major (64 consecutive nodes per wave)
    unsigned tiles_x;  // tiles per row group (rectangular shapes)
    float inv_n0;      // 1 / nodes per row (row-major shape)
};


// One tile of the flat work list: problem index and tile index within it.
struct TileRef {
    unsigned prob;
    unsigned local;
};

}  // namespace gals

struct gals_ctx {
    int dim;
    int prec;
    int mixed;
    int psi;  // GALS_PSI_*
    int device;
    gals::Geom g;
    bool vel_set;
    int vel_kind;
    double period;
    gals::Vel<float> vf;
    gals::Vel<double> vd;
    bool inflow;  // GALS_BC_INFLOW: g.bc is GALS_BC_NEUMANN for the feet
    bool face;    // GALS_BC_INFLOW_NEUMANN: likewise, plus the face scheme
    const void *inflow_phi, *inflow_grad, *inflow_phit;
};

namespace gals {

// Thread-local error text returned by gals_last_error() (gals_api.hip).
void set_error_v(const char *fmt, va_list ap);

// Launchers (kernels_*.hip). Each returns a hipError_t of the launch.
hipError_t launch_step(const gals_ctx *ctx, const void *phi, const void *grad, void *phi_o,
                       void *grad_o, double dt, double c1, double c2, double c3,
                       const void *coltab, const void *rowtab, hipStream_t s);
// Per-column / per-row stream-function tables (GALS_VEL_STREAM_SIN only).
hipError_t launch_stream_tables(const gals_ctx *ctx, void *coltab, void *rowtab, hipStream_t s);
// sin(pi x), cos(pi x) at the node coordinates of each axis (x, then y, then
// z; one pair per node) for 3D sine vector potentials (kernels_step.hip).
hipError_t launch_axis_tables(const gals_ctx *ctx, void *tab, hipStream_t s);

// Inflow boundary conditions after a step of size dt (boundary.hip):
// Dirichlet data at time factor c, and homogeneous Neumann inflow by the face
// scheme from the state before the step (sphi, sgrad) into the stepped one.
hipError_t launch_inflow(const gals_ctx *ctx, void *phi, void *grad, double c, double dt,
                         hipStream_t s);
hipError_t launch_face(const gals_ctx *ctx, const void *sphi, const void *sgrad, void *dphi,
                       void *dgrad, double dt, double c1, double c2, double c3, hipStream_t s);

// Adjoint of the stream-function step and the shape loss (adjoint.hip).
// adjoint_blocks: blocks of the adjoint launch (16 partials each).
unsigned adjoint_blocks(const gals_ctx *ctx);
// lam_out must hold zeros; clear: zero lam_in as it is read.
hipError_t launch_adjoint_step(const gals_ctx *ctx, const void *phi, const void *grad,
                               double *lam_in, double *lam_out, bool clear, double *partials,
                               double dt, double c1, double c2, double c3, const void *coltab,
                               const void *rowtab, hipStream_t s);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_fold_grad(const double *partials, int nparts, double *out, hipStream_t s);
hipError_t launch_heaviside_loss(const gals_ctx *ctx, const void *phi, const void *phi_ref,
                                 double eps, double *lam, double *partials, double *out,
                                 hipStream_t s);

// Batched stream-function problems (batch.hip). probs/tiles are device arrays.
hipError_t launch_batch_tables(int prec, const void *probs_f64, int nprob, int max_entries,
                               void *tab, hipStream_t s);
hipError_t launch_batch_step(int prec, int mixed, const void *probs, const TileRef *tiles,
                             unsigned ntiles, double dt, double c1, double c2, double c3,
                             const void *tab, const void *in, void *out, hipStream_t s);
hipError_t launch_batch_copy(int prec, const void *probs, const TileRef *tiles, unsigned ntiles,
                             const void *in, void *out, unsigned blocks, hipStream_t s);
hipError_t launch_eval(const gals_ctx *ctx, const void *phi, const void *grad, const double *pts,
                       int64_t npts, void *val, void *normal, void *curv, hipStream_t s);
hipError_t launch_norms(const gals_ctx *ctx, const void *phi, const void *grad,
                        const void *phi_ref, const void *grad_ref, double eps, double band,
                        double *partials, double *out, hipStream_t s);
hipError_t launch_max_speed(const gals_ctx *ctx, double c, double *partials, double *out,
                            hipStream_t s);

}  // namespace gals
