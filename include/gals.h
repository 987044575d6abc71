/*
 * gals.h - C ABI of the MI355X (gfx950) gradient-augmented level set library.
 *
 * The library advances a level set function phi and its gradient psi =
 * grad phi, both stored on the nodes of a uniform 2D or 3D grid, with the
 * gradient-augmented CIR scheme of Nave, Rosales and Seibold ("A
 * gradient-augmented level set method with an optimally local, coherent
 * advection scheme"): per node, the characteristic is traced backwards with
 * the superconsistent Shu-Osher scheme (sec. 5.1, Ex.
 * ex:superconsistent_ShuOsher), the bi-/tri-cubic Hermite interpolant
 * (sec. 2.3, eq. p-cubic_interpolant) of the cell holding the foot is
 * evaluated, and phi <- H(foot), psi <- (grad foot) . grad H(foot)
 * (eq. superconsistency). Cross derivatives are rebuilt from neighbouring
 * gradients by central differencing (sec. 2.3, approach (A)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: dim in {2,3}; ncell[a] >= 2 cells on [lo[a], hi[a]]; nodes per axis
 *   n[a] = ncell[a] + 1; h[a] = (hi[a]-lo[a]) / ncell[a]; node i sits at
 *   lo + i*h.
 * Device layout (SoA planes): element type float (GALS_F32) or double
 *   (GALS_F64). A plane holds n[1] (2D) or n[1]*n[2] (3D) rows of
 *   `pitch` elements, x fastest: element (i,j,k) at i + pitch*(j + n[1]*k).
 *   pitch = n[0] rounded up to a multiple of 64; `plane_stride` =
 *   pitch*n[1](*n[2]) elements. `phi` points to one plane; `grad` to dim
 *   planes at grad + a*plane_stride (psi_x, psi_y[, psi_z]). Padding
 *   elements are never read or written. Device pointers must be aligned to
 *   their element size.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream). Calls marked "async" only enqueue work on it.
 * Ownership: the caller allocates and owns every device buffer (state,
 *   workspace, points, outputs); the library owns only its context and never
 *   frees caller memory.
 * Errors: every entry point returns GALS_OK (0) or a negative code and never
 *   throws; gals_last_error() returns a thread-local message describing the
 *   last failure. Asynchronous kernel faults surface as GALS_EHIP from a
 *   later call.
 * Threads: a context may be used from one host thread at a time; calls that
 *   share a workspace must be ordered on one stream.
 */
#ifndef GALS_H
#define GALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gals_ctx gals_ctx;

enum { GALS_OK = 0, GALS_EINVAL = -1, GALS_ENOMEM = -2, GALS_EHIP = -3, GALS_ENOTSUP = -4 };

/* State and Hermite arithmetic precision. Foot coordinates, the cell split
 * and all reductions are FP64 in both. */
enum { GALS_F32 = 1, GALS_F64 = 2 };

/* Cross-derivative reconstruction (sec. 2.3): central differencing (A), with
 * one-sided 3-point differences at the first and last node; the cell-based
 * approach (B), from the gradients at the cell's own vertices (edge-centre
 * differences weighted 3/4, 3/4, -1/4, -1/4; in 3D on the facet through the
 * vertex, and the first-order phi_xyz on the xy facet), which leaves the
 * interpolant continuous with O(h^3) gradient jumps; or all zero (the
 * robustness ablation noted at the end of sec. 2.3). */
enum { GALS_MIXED_CENTRAL = 0, GALS_MIXED_CELL = 1, GALS_MIXED_ZERO = 2 };

/* Gradient update (sec. 4 step 3): the superconsistent update psi_new =
 * grad(foot map)^T grad H (eq. superconsistency, the default), or Heun's
 * method for eq. cir_evolution_psi along the characteristic, from grad H at
 * the foot (time t) to the node (time t + dt), with grad v at both ends. */
enum { GALS_PSI_SUPERCONSISTENT = 0, GALS_PSI_HEUN = 1 };

/* Treatment of a departure point (foot) outside the domain. GALS_BC_NEUMANN
 * (the default): homogeneous Neumann, the boundary condition the paper
 * prescribes at inflow edges in its tests (sec. 6.1, 6.2); the foot is
 * projected onto the domain and the extension, constant along the outward
 * normal, has zero normal derivative. GALS_BC_EXTRAPOLATE: the nearest
 * boundary cell's polynomial is evaluated outside its cell (exact for
 * polynomial data, but it amplifies values when feet land more than about one
 * cell out, e.g. a rotation at CFL > 1 in the corners). GALS_BC_INFLOW:
 * Dirichlet inflow data (sec. 4.1) from gals_set_inflow_data at boundary
 * nodes where the flow enters, feet outside the domain projected as with
 * GALS_BC_NEUMANN. GALS_BC_INFLOW_NEUMANN: the homogeneous Neumann inflow
 * condition of sec. 4.1 (eq. Neumann_bc_evolution, zero normal derivative):
 * feet projected as with GALS_BC_NEUMANN, and boundary nodes where the flow
 * enters take phi and the tangential gradient from a GA-CIR step of one
 * dimension less on the face (tangential velocity, face data at the start of
 * the step, the context's cross-derivative rule, superconsistent gradient
 * update), normal derivatives 0; a corner entered through every face keeps
 * its value. Inflow faces as for gals_set_inflow_data. Single grids only. */
enum {
    GALS_BC_NEUMANN = 0,
    GALS_BC_EXTRAPOLATE = 1,
    GALS_BC_INFLOW = 2,
    GALS_BC_INFLOW_NEUMANN = 3
};

/* Velocity fields v(x,t) = c(t) v_s(x), c(t) = cos(pi t / period) when
 * period > 0, else 1. Parameter vectors (FP64):
 *   GALS_VEL_AFFINE     2D/3D  b[d], c[d], A[d*d] row-major, A[i][j] = dv_i/dx_j;
 *                              v_s = b + A (x - c)  (rotation, shear, constant)
 *   GALS_VEL_STREAM_SIN 2D     (a, m, n) per mode, 1..64 modes, m, n integers in
 *                              1..4: stream function s = sum a sin(m pi x) sin(n pi y),
 *                              v_s = (-s_y, s_x)
 *   GALS_VEL_VECPOT_SIN 3D     (ax, ay, az, l, m, n) per mode, 1..8 modes, l, m, n
 *                              integers in 1..4: A = sum (ax,ay,az) sin(l pi x)
 *                              sin(m pi y) sin(n pi z), v_s = curl A
 *   GALS_VEL_VORTEX     2D     none: s = sin^2(pi x) sin^2(pi y) / pi ("vortex in a
 *                              box", sec. 6.1, eq. swirl_2d_velocity_field)
 *   GALS_VEL_PSEUDO1D   2D     none: v_s = exp(e.x) e, e = (sqrt 2, sqrt pi)/sqrt(2+pi)
 *                              (sec. 6.1, eq. velocity_1)
 *   GALS_VEL_LEVEQUE3D  3D     none: the 3D deformation field of sec. 6.2, with the
 *                              first component read as 2 sin^2(pi x) sin(2 pi y)
 *                              sin(2 pi z) so that the field is divergence free
 * The analytic deformation matrix of each field is used (sec. 4 assumes v and
 * grad v exactly accessible). */
enum {
    GALS_VEL_AFFINE = 1,
    GALS_VEL_STREAM_SIN = 2,
    GALS_VEL_VECPOT_SIN = 3,
    GALS_VEL_VORTEX = 4,
    GALS_VEL_PSEUDO1D = 5,
    GALS_VEL_LEVEQUE3D = 6
};

/* Create a context for one grid (the problem statement of sec. 2.1: a
 * surface moved by a given velocity, phi and psi on grid nodes). `device` is
 * the HIP device the context launches on; -1 makes a host-only context that
 * answers layout, workspace and parameter-validation calls and rejects every
 * device call with EINVAL (no HIP call is made). EINVAL on dim not in {2,3},
 * ncell[a] < 2, hi <= lo, non-finite bounds, unknown prec, mixed_mode or bc, a
 * device outside [-1, device count), 2^31 or more nodes, or a padded state
 * plane of 2 GiB or more (the kernels address a plane with 32-bit byte
 * offsets); EHIP if the
 * device count cannot be read. */
int gals_create(gals_ctx **out, int dim, const int64_t *ncell, const double *lo,
                const double *hi, int prec, int mixed_mode, int bc, int device);

/* Release a context (NULL is accepted). */
int gals_destroy(gals_ctx *ctx);

/* Report the device layout: nodes[dim] per axis, row pitch and plane stride
 * in elements. Any output may be NULL. */
int gals_layout(const gals_ctx *ctx, int64_t *nodes, int64_t *pitch,
                int64_t *plane_stride);

/* Workspace bytes every call on this context needs (one ping-pong copy of
 * the state plus reduction partials), aligned to 256 bytes. */
int gals_workspace_bytes(const gals_ctx *ctx, size_t *bytes);

/* Set the velocity field (sec. 4). EINVAL on a wrong parameter count, kind
 * not valid for the grid's dim, non-finite parameters or period < 0;
 * ENOTSUP on sine-mode indices outside 1..4 or too many modes. Host-only. */
int gals_set_velocity(gals_ctx *ctx, int kind, const double *params, int64_t nparams,
                      double period);
/* Gradient update of later advances: GALS_PSI_SUPERCONSISTENT (default) or
 * GALS_PSI_HEUN. Batches and the adjoint use the superconsistent update. */
int gals_set_psi_update(gals_ctx *ctx, int mode);

/* Dirichlet inflow data for a GALS_BC_INFLOW context (sec. 4.1): device
 * arrays in the state layout, phi_b (one plane), grad_b (dim planes) and
 * phit_b (one plane), read at boundary nodes only. After each step (ending
 * at time t), at a boundary node where v(x, t) enters the domain through one
 * face, phi = phi_b, the tangential gradient = grad_b's, and the normal
 * derivative = -(phit_b + tangential v . grad_b) / v_n, from the equation;
 * where the flow enters through several faces (edges, corners) every
 * component comes from grad_b. The data are for the end time of the step
 * (for time-dependent data advance one step at a time and update them).
 * The flow enters through face a where its inward normal component exceeds
 * 1e-6 max(|v|, h_a / dt), so a face that is a streamline (a no-penetration
 * wall) or a stagnation point takes no data whatever the rounding of v.
 * The caller keeps the arrays alive while they are set. EINVAL for a
 * context of another boundary treatment. */
int gals_set_inflow_data(gals_ctx *ctx, const void *phi_b, const void *grad_b,
                         const void *phit_b);

/* Advance phi and grad (device, in place) by `steps` GA-CIR steps of size dt
 * from time t0 (sec. 4, steps 1-3, with the superconsistent update of eq.
 * superconsistency). Step n goes from t0 + n*dt to t0 + (n+1)*dt; times are
 * computed, not accumulated. Departure points may lie any number of cells
 * away (any CFL); feet outside the domain follow the context's boundary
 * treatment. Async: kernel launches and, for an odd step count, one
 * device-to-device copy back from the workspace, all on `stream`; no
 * allocation, fill or synchronisation, so a caller may capture the call in
 * a HIP graph. EINVAL on NULL or overlapping state/workspace
 * pointers, workspace smaller than gals_workspace_bytes, non-finite or
 * non-positive dt, non-finite t0, steps < 0, no velocity set, or a
 * GALS_BC_INFLOW context without inflow data. */
int gals_advance(gals_ctx *ctx, void *phi, void *grad, double t0, double dt, int64_t steps,
                 void *workspace, size_t workspace_bytes, void *stream);

/* Size of the library's static device scratch used by gals_advance_noalloc
 * (64 MiB per GPU the library runs on, held until the process ends). */
#define GALS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * advance as gals_advance (same kernels, same results bit for bit) with no
 * workspace argument. The ping-pong state copy and the velocity tables live
 * in the library's static device scratch of GALS_NOALLOC_SCRATCH_BYTES per
 * GPU; the call allocates and frees nothing. The caller still owns phi and
 * grad. Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents (nothing in it needs to start at zero): calls that overlap
 * on one GPU (different streams, different host threads) race and must be
 * ordered by the caller, e.g. on one stream. EINVAL as gals_advance, and
 * when gals_workspace_bytes of the context exceeds the scratch (2D FP32
 * grids fit up to about 2048^2 cells, FP64 up to about 1440^2). Async. */
int gals_advance_noalloc(gals_ctx *ctx, void *phi, void *grad, double t0, double dt,
                         int64_t steps, void *stream);

/* Value, unit normal and curvature of the Hermite interpolant at npts points
 * (sec. 3.2, eqs. surface_normal and curvature; in 3D the curvature is the
 * divergence of the normal, i.e. the sum of the principal curvatures).
 * pts: device FP64, SoA (x[npts], y[npts][, z[npts]]). Outputs are device
 * arrays of the context's element type: val[npts], normal[dim*npts] (SoA),
 * curv[npts]; any output may be NULL. Where the gradient is exactly zero the
 * normal and curvature are 0. A point outside the domain evaluates the
 * nearest boundary cell's polynomial. Async. EINVAL on NULL state/points,
 * npts < 0 or npts >= 2^40; npts = 0 does nothing. */
int gals_eval_points(gals_ctx *ctx, const void *phi, const void *grad, const double *pts,
                     int64_t npts, void *val, void *normal, void *curv, void *stream);

/* max over nodes of |v(x_node, t)| into *out (host): the largest speed that
 * sets the CFL number v_max dt / h, which the remark on the time step in
 * sec. 4 relates to how far a foot may land from its node (feet a cell or
 * more away are gathered like any other). Uses the workspace for partials,
 * synchronises the stream. */
int gals_max_speed(gals_ctx *ctx, double t, double *out, void *workspace,
                   size_t workspace_bytes, void *stream);

/* Error norms of (phi, grad) against a reference state (sec. 6.1, eq.
 * maximum_norm), FP64 accumulation, deterministic. out[8] (host):
 *   [0] max |phi - phi_ref|              [1] max over components |psi - psi_ref|
 *   [2] prod(h) * sum |H_eps(phi) - H_eps(phi_ref)|  (L1 shape error)
 *   [3] max |phi - phi_ref| over nodes with |phi_ref| <= band
 *   [4] prod(h) * sum H_eps(-phi)        [5] the same for phi_ref (volumes)
 *   [6] count of non-finite entries of phi and grad   [7] max |phi_ref|
 * with H_eps(s) = 0 (s < -eps), 1 (s > eps), (1 + s/eps + sin(pi s/eps)/pi)/2.
 * Uses the workspace for partials, synchronises the stream. */
int gals_norms(gals_ctx *ctx, const void *phi, const void *grad, const void *phi_ref,
               const void *grad_ref, double eps, double band, double *out,
               void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Derivatives (2D grids with GALS_VEL_STREAM_SIN fields). The advance is a
 * chain of steps u_{n+1} = M(u_n; S), u = (phi, psi_x, psi_y), S the folded
 * stream-function table: S[m][n] = sum of the amplitudes of the modes with
 * wavenumbers (m, n), m, n = 1..4, so dF/da_k = dF/dS[m_k][n_k]. Each step is
 * linear in u (sec. 4 steps 1-3, eq. superconsistency); gals_adjoint_step
 * applies its transpose and adds the step's contribution to dF/dS, which
 * differentiates the three Shu-Osher stages of the trace
 * (Ex. ex:superconsistent_ShuOsher) with S. Adjoint states are FP64 and use
 * the state layout (3 planes of plane_stride elements, lam_phi, lam_x,
 * lam_y); dF/dS is 16 FP64 values in device memory, index 4 (m-1) + (n-1).
 * The state adjoint sums with FP64 atomics, so its last bits vary from run to
 * run; dF/dS is reduced in a fixed order. Other fields, 3D grids, Heun's
 * gradient update or GALS_BC_INFLOW contexts: ENOTSUP.
 * ------------------------------------------------------------------------- */

/* Bytes of a checkpoint store for `steps` steps saved every `every` steps:
 * ceil(steps / every) states, each (1 + dim) planes rounded up to 256 B. */
int gals_checkpoint_bytes(const gals_ctx *ctx, int64_t steps, int64_t every, size_t *bytes);
/* As gals_advance (same workspace), and store the state before steps
 * 0, every, 2 every, ... in ckpt (device, 256-byte aligned, caller-owned).
 * Step n starts at t0 + n dt, exactly as in gals_advance. Async. */
int gals_advance_save(gals_ctx *ctx, void *phi, void *grad, double t0, double dt, int64_t steps,
                      int64_t every, void *ckpt, size_t ckpt_bytes, void *workspace,
                      size_t workspace_bytes, void *stream);
/* Workspace bytes of gals_adjoint with checkpoints every `every` steps (and,
 * with every = 1, of gals_adjoint_step): the advance's workspace, `every`
 * recomputed states, one adjoint state and the dF/dS partials. */
int gals_adjoint_workspace_bytes(const gals_ctx *ctx, int64_t every, size_t *bytes);
/* Reverse sweep of the advance stored by gals_advance_save (same t0, dt,
 * steps, every, velocity): lam holds dF/du at the final state on entry and
 * dF/du at the initial state on return; dS receives dF/dS (overwritten).
 * Recomputes each segment of `every` states from its checkpoint. Async. */
int gals_adjoint(gals_ctx *ctx, const void *ckpt, size_t ckpt_bytes, double t0, double dt,
                 int64_t steps, int64_t every, double *lam, double *dS, void *workspace,
                 size_t workspace_bytes, void *stream);
/* One reverse step: (phi, grad) is the state at the start of the step (time
 * t), lam_in = dF/du after the step, lam_out = dF/du before it (overwritten;
 * must not overlap lam_in); dS += the step's dF/dS. Workspace: every = 1. */
int gals_adjoint_step(gals_ctx *ctx, const void *phi, const void *grad, double t, double dt,
                      const double *lam_in, double *lam_out, double *dS, void *workspace,
                      size_t workspace_bytes, void *stream);
/* Shape loss prod(h) sum over nodes (H_eps(phi) - H_eps(phi_ref))^2 with the
 * smoothed Heaviside of gals_norms (2D); *loss on the host. If lam is not
 * NULL it receives dloss/du (3 FP64 planes; psi parts 0), the seed of
 * gals_adjoint. Synchronises the stream. */
int gals_shape_loss(gals_ctx *ctx, const void *phi, const void *phi_ref, double eps, double *loss,
                    double *lam, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent 2D grids, each with its own sine stream-function
 * field (GALS_VEL_STREAM_SIN; all share one period), advanced together by one
 * launch per step over a flat work list of node tiles of every problem. The
 * state of all problems is one buffer: problem p's phi plane starts at
 * element offset[p], followed by its psi_x and
 * psi_y planes (same pitch/plane conventions as a single grid). Throughput
 * layer for the paper's method applied to many small problems; the per-node
 * arithmetic is that of gals_advance, so results agree bit for bit.
 * ------------------------------------------------------------------------- */
typedef struct gals_batch gals_batch;

/* Create a batch of nprob (1..65535) 2D grids: ncell[2p], ncell[2p+1] cells
 * on [lo[2p], hi[2p]] x [lo[2p+1], hi[2p+1]], each plane under 2 GiB.
 * device -1: host-only (layout and validation). The batch owns small device
 * tables (problem descriptors and the tile list) that it uploads before its
 * first advance; EINVAL for invalid sizes, ENOMEM when out of host memory.
 * Its wave shapes start as those recorded for its shape by
 * gals_batch_autotune (see there), else 64 for every class. */
int gals_batch_create(gals_batch **out, int64_t nprob, const int64_t *ncell, const double *lo,
                      const double *hi, int prec, int mixed_mode, int bc, int device);
int gals_batch_destroy(gals_batch *b);
/* offset/pitch/plane: nprob entries each (elements); total_elems: buffer size. */
int gals_batch_layout(const gals_batch *b, int64_t *offset, int64_t *pitch, int64_t *plane,
                      int64_t *total_elems);
int gals_batch_workspace_bytes(const gals_batch *b, size_t *bytes);
/* Velocity of problem p: GALS_VEL_STREAM_SIN parameters as for a single grid
 * (ENOTSUP for other kinds); every problem must use the same period. */
int gals_batch_set_velocity(gals_batch *b, int64_t p, int kind, const double *params,
                            int64_t nparams, double period);
/* Wave shape per grid-size class (nodes per row <= 48, <= 96, <= 192, more):
 * nodes per wave along x, 64, 32 or 16 (a wave covers 64/w rows), or 0 for
 * the row-major shape (a wave takes 64 consecutive nodes of the grid in
 * row-major order). With 64, a ragged last group of at most 48 columns is
 * packed row-major into waves of its own. A tile is 4 waves. Default 64 for
 * every class. The shape changes only the speed: results are the same bit
 * for bit. */
int gals_batch_set_tiles(gals_batch *b, const int *wave_width_per_class);
int gals_batch_get_tiles(const gals_batch *b, int *wave_width_per_class);
/* Advance every problem by `steps` steps (as gals_advance). use_graph != 0
 * captures the whole advance into a hipGraph on first use and replays it
 * while (state, workspace, stream, t0, dt, steps) are unchanged; capture
 * needs a non-null stream. Async. */
int gals_batch_advance(gals_batch *b, void *state, double t0, double dt, int64_t steps,
                       int use_graph, void *workspace, size_t workspace_bytes, void *stream);
/* Choose the wave shape per size class by timing `steps` steps of each
 * candidate on this batch (coordinate descent over the classes); keeps the
 * fastest and returns its time in *best_ms. Advances `state` while timing:
 * pass a scratch copy. Synchronises the stream. The choice is recorded for
 * the batch's shape (precision, cross-derivative rule and every problem's
 * cell counts, in order): a batch of the same shape created later in the
 * process starts with it, and when the environment variable GALS_TUNE_FILE
 * names a file the choice is appended to it as a line "key w0 w1 w2 w3" (key
 * in hex), which gals_batch_create of later processes reads (the last line
 * for a key wins; unreadable or invalid lines are ignored). */
int gals_batch_autotune(gals_batch *b, void *state, double dt, int64_t steps, void *workspace,
                        size_t workspace_bytes, void *stream, double *best_ms);

/* Thread-local text of the last error ("" if none). */
const char *gals_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GALS_H */
