/*
 * Plain FP64 CPU oracle for the gradient-augmented CIR (GA-CIR) level set step
 * of Nave, Rosales and Seibold, "A gradient-augmented level set method with an
 * optimally local, coherent advection scheme".
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table or
 * constant with the GPU library; the two agree only on the public argument
 * conventions (grid geometry, velocity parameter layout), which each side
 * implements on its own.
 *
 * Conventions (all arrays FP64, dense, no padding):
 *   dim in {2,3}; ncell[a] cells along axis a; nodes per axis nn[a] = ncell[a]+1;
 *   h[a] = (hi[a]-lo[a]) / ncell[a]; node (i,j,k) sits at lo + (i,j,k)*h.
 *   A node field is a plane of nn[0]*nn[1]*(nn[2]) doubles, x fastest:
 *   index = i + nn[0]*(j + nn[1]*k).
 *   phi: 1 plane.  psi: dim planes back to back (psi_x, psi_y[, psi_z]).
 *   Points are AoS: pts[p*dim + a].
 *
 * Velocity kinds and their parameter vectors (v(x,t) = c(t) * v_s(x) with
 * c(t) = cos(pi t / period) when period > 0, else 1):
 *   1 AFFINE     (2D/3D)  params = b[d], c[d], A[d*d] (row-major, A[i][j] = dv_i/dx_j):
 *                          v_s = b + A (x - c)
 *   2 STREAM_SIN (2D)     params = (a, m, n) per mode: stream function
 *                          s = sum a sin(m pi x) sin(n pi y), v_s = (-s_y, s_x)
 *   3 VECPOT_SIN (3D)     params = (ax, ay, az, l, m, n) per mode: vector potential
 *                          A = sum (ax,ay,az) sin(l pi x) sin(m pi y) sin(n pi z),
 *                          v_s = curl A
 *   4 VORTEX     (2D)     params = none: stream function (1/pi) sin^2(pi x) sin^2(pi y)
 *                          (the "vortex in a box" field of the accuracy study, sec. 6.1)
 *   5 PSEUDO1D   (2D)     params = none: v_s = exp(e.x) e, e = (sqrt2, sqrtpi)/sqrt(2+pi)
 *                          (eq. velocity_1)
 *   6 LEVEQUE3D  (3D)     params = none: the 3D deformation field of sec. 6.2
 *
 * Mixed-derivative modes (sec. 2.3): 0 central differencing (A), 2 all zero.
 * Boundary treatment of feet outside the domain (bc): 0 homogeneous Neumann
 * (foot projected onto the domain, zero normal derivative), 1 extrapolation
 * of the boundary cell's polynomial, 3 as 0, and inflow boundary nodes
 * follow the homogeneous Neumann condition of sec. 4.1 (eq.
 * Neumann_bc_evolution): a GA-CIR step of one dimension less on the face,
 * normal derivative 0.
 */
#ifndef GALS_ORACLE_H
#define GALS_ORACLE_H

/* A foot counts as outside the domain (bc 0 and 3) only when it lies more
 * than ORC_FOOT_TOL cells beyond the boundary; closer, it stays where it is
 * and the boundary cell's cubic is evaluated there. A foot within rounding
 * of the boundary (a node on a face the flow runs along) must not have its
 * normal derivative zeroed or kept by the sign of that rounding. */
#define ORC_FOOT_TOL 1e-6

#ifdef __cplusplus
extern "C" {
#endif

/* 1D basis w^v_alpha(x) of eq. (1-cubic_basis_functions) and its derivatives
 * of order deriv in {0,1,2}. Returns 0, or -1 on bad arguments. */
int orc_basis(int v, int alpha, int deriv, double x, double *out);

/* p-cubic Hermite interpolant, eq. (p-cubic_interpolant), on one cell with
 * edge lengths h[dim], evaluated at local coordinates xi[dim] (0..1 inside).
 * data[v * 2^dim + alpha]: the derivative d^alpha phi at vertex v, with v and
 * alpha bit masks (bit a = axis a). Outputs (any may be NULL):
 * val, grad[dim], hess[dim*dim]. */
int orc_hermite(int dim, const double *data, const double *h, const double *xi,
                double *val, double *grad, double *hess);

/* Cross derivatives at every node from psi (sec. 2.3). mode 0: central (A)
 * with one-sided 3-point differences at the first and last node; mode 2: zero.
 * Output planes: 2D [phi_xy]; 3D [phi_xy, phi_xz, phi_yz, phi_xyz]. Mode 1,
 * the cell-based approach (B), has no per-node values (-1 here); the step,
 * the evaluation and orc_grad_cs form them per cell. */
int orc_mixed(int dim, const long *ncell, const double *lo, const double *hi,
              int mode, const double *psi, double *mixed);

/* Velocity v(x,t) and the deformation matrix in the paper's convention
 * G[i*dim+j] = d v_j / d x_i (sec. 4). */
int orc_velocity(int dim, int kind, const double *params, long nparams,
                 double period, const double *x, double t, double *v, double *G);

/* Superconsistent Shu-Osher backward trace (Ex. ex:superconsistent_ShuOsher):
 * from node position x at time t+dt back to time t. Returns the foot X[dim]
 * and D[i*dim+j] = d X_j / d x_i. */
int orc_trace(int dim, int kind, const double *params, long nparams, double period,
              const double *x, double t, double dt, double *X, double *D);

/* Advance phi, psi in place by `steps` GA-CIR steps of size dt from time t0.
 * Step n goes from t0 + n dt to t0 + (n+1) dt. mixed_mode 0 (A), 1 (B),
 * 2 zero; psi_update 0 superconsistent (eq. superconsistency), 1 Heun's
 * method for eq. cir_evolution_psi along the characteristic. */
int orc_advance(int dim, const long *ncell, const double *lo, const double *hi,
                int kind, const double *params, long nparams, double period,
                int mixed_mode, int bc, int psi_update, double *phi, double *psi,
                double t0, double dt, long steps);

/* One step from time t to t+dt, evaluated only at the listed node indices.
 * phi_out[count], psi_out[count*dim]. */
int orc_step_nodes(int dim, const long *ncell, const double *lo, const double *hi,
                   int kind, const double *params, long nparams, double period,
                   int mixed_mode, int bc, int psi_update, const double *phi,
                   const double *psi, double t, double dt, const long *nodes, long count,
                   double *phi_out, double *psi_out);

/* Dirichlet inflow data (sec. 4.1) applied after a step of size dt ending
 * at time t: at boundary nodes where v(x, t) enters the domain (inward
 * normal component above 1e-6 max(|v|, h_a / dt)), phi = phi_b, the
 * tangential gradient = grad_b's, and the normal derivative from the
 * equation, -(phit_b + tangential v . grad_b) / v_n (all components from
 * grad_b where the flow enters through several faces). In place. */
int orc_apply_inflow(int dim, const long *ncell, const double *lo, const double *hi,
                     int kind, const double *params, long nparams, double period, double t,
                     double dt, double *phi, double *psi, const double *phi_b,
                     const double *grad_b, const double *phit_b);

/* Value, gradient, Hessian, normal and curvature of the Hermite interpolant at
 * npts points (sec. 3.2, eqs. surface_normal and curvature). Any output may be
 * NULL. grad/normal: npts*dim, hess: npts*dim*dim, kappa: npts. */
int orc_eval_points(int dim, const long *ncell, const double *lo, const double *hi,
                    int mixed_mode, const double *phi, const double *psi,
                    const double *pts, long npts, double *val, double *grad,
                    double *hess, double *normal, double *kappa);

/* Diagnostics over all nodes, compared with a reference state:
 * out[0] e_max(phi), out[1] e_max(psi) (eq. maximum_norm),
 * out[2] L1 shape error  prod(h) * sum |H_eps(phi) - H_eps(phi_ref)|,
 * out[3] max |phi - phi_ref| over nodes with |phi_ref| <= band,
 * out[4] volume prod(h) * sum H_eps(-phi), out[5] the same for phi_ref,
 * out[6] number of non-finite entries in phi and psi, out[7] max |phi_ref|. */
int orc_norms(int dim, const long *ncell, const double *lo, const double *hi,
              const double *phi, const double *psi, const double *phi_ref,
              const double *psi_ref, double eps, double band, double *out);

/* max over nodes of |v(x_node, t)|. */
double orc_max_speed(int dim, const long *ncell, const double *lo, const double *hi,
                     int kind, const double *params, long nparams, double period,
                     double t);

/* Complex-step derivatives (gals_oracle_cs.c) of a functional of the final
 * state of a 2D GALS_VEL_STREAM_SIN advance with respect to the folded
 * stream-function table S[m][n] (m, n = 1..4; grad[4*(m-1) + (n-1)]). The
 * functional is sum(lam . u_T) over the 3 planes of lam (3N values) if lam is
 * not NULL, else prod(h) sum (H_eps(phi_T) - H_eps(phi_target))^2. *value
 * receives the functional. Runs 16 complex advances. */
int orc_grad_cs(const long *ncell, const double *lo, const double *hi, const double *params,
                long nparams, double period, int mixed_mode, int bc, const double *phi0,
                const double *psi0, double t0, double dt, long steps, const double *lam,
                const double *phi_target, double eps, double *value, double *grad);

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
/* Threads of the OpenMP loops from now on (n >= 1). */
int orc_set_threads(int n);
/* Order of the Hermite sums from now on: 0 (default) the literal sum over
 * every (vertex, derivative) pair of eq. (p-cubic_interpolant); 1 the same
 * sum contracted axis by axis (last axis first). Both are exact FP64
 * evaluations of one definition that round in different orders; the second
 * exists to measure that difference. */
int orc_set_sum_order(int order);
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
