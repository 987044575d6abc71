/*
 * Plain FP64 CPU oracle for the gradient-augmented CIR level set step.
 *
 * TEST INFRASTRUCTURE ONLY: the GPU library never links, loads or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do. Every routine follows the paper's statement directly, without blocking,
 * fusion or reordering, so that it can be checked against the text by eye:
 *
 *   basis functions ........ sec. 2.3, eq. (1-cubic_basis_functions)
 *   Hermite interpolant .... sec. 2.3, eq. (p-cubic_interpolant), rectangular
 *                            cells scale the alpha-th datum by prod h_a^alpha_a
 *   cross derivatives ...... sec. 2.3, approach (A) central differencing, or
 *                            approach (B) cell-based (per cell, from the
 *                            gradients at its own vertices)
 *   characteristic trace ... sec. 5.1, Ex. ex:superconsistent_ShuOsher
 *   one step ............... sec. 4 (steps 1-3) with the superconsistent
 *                            gradient update, eq. (superconsistency), or the
 *                            gradient ODE (eq. cir_evolution_psi) integrated
 *                            along the characteristic by Heun's method
 *   normal, curvature ...... sec. 3.2, eqs. (surface_normal), (curvature)
 *   error norms ............ sec. 6.1, eq. (maximum_norm)
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - cross derivatives at the first/last node use one-sided 3-point
 *     differences; phi_xy = D_x psi_y, phi_xz = D_x psi_z, phi_yz = D_y psi_z,
 *     phi_xyz = D_x D_y psi_z (the highest-index gradient component);
 *   - approach (B) in 3D: a vertex takes phi_xy from the cell's xy facet
 *     through it (likewise phi_xz, phi_yz), and phi_xyz from the first-order
 *     formula on that xy facet;
 *   - Heun's method for the gradient runs from the foot (time t, after the
 *     boundary treatment) to the node (time t + dt), starting from grad H;
 *   - a foot outside the domain: with bc = 0 (homogeneous Neumann, as the
 *     paper prescribes at inflow edges in its tests, sec. 6.1 and 6.2) the
 *     foot is projected onto the domain and the extension, constant along
 *     the outward normal, has zero normal derivative; with bc = 1 the
 *     nearest boundary cell's polynomial is extrapolated (clamped cell index,
 *     unclamped local coordinate). Point evaluation always extrapolates;
 *   - a foot exactly on a cell face belongs to the cell on its right,
 *     except at the last node, which belongs to the last cell (xi = 1);
 *   - 3D curvature is the divergence of the unit normal (sum of the principal
 *     curvatures); normal and curvature are 0 where the gradient vanishes;
 *   - shape error and volume use the smoothed Heaviside
 *     H_eps(s) = 0 (s < -eps), 1 (s > eps), (1 + s/eps + sin(pi s/eps)/pi)/2.
 *
 * Built with -ffp-contract=off so that no fused multiply-add changes the
 * rounding of the written expressions.
 */
#include "gals_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 3

/* ---------------------------------------------------------------------------
 * 1D basis (eq. 1-cubic_basis_functions): f(x) = 1 - 3x^2 + 2x^3,
 * g(x) = x (1-x)^2, and w^0_0 = f(x), w^1_0 = f(1-x), w^0_1 = g(x),
 * w^1_1 = -g(1-x).
 * ------------------------------------------------------------------------- */
static double f_d(int d, double x)
{
    if (d == 0) return 1.0 - 3.0 * x * x + 2.0 * x * x * x;
    if (d == 1) return -6.0 * x + 6.0 * x * x;
    return -6.0 + 12.0 * x;
}

static double g_d(int d, double x)
{
    if (d == 0) return x * (1.0 - x) * (1.0 - x);
    if (d == 1) return 1.0 - 4.0 * x + 3.0 * x * x;
    return -4.0 + 6.0 * x;
}

/* d-th derivative of w^v_alpha at x; the chain rule through (1-x) gives a
 * factor (-1)^d for the v = 1 functions. */
static double w_d(int v, int alpha, int d, double x)
{
    double sgn = (d % 2 == 0) ? 1.0 : -1.0;
    if (v == 0 && alpha == 0) return f_d(d, x);
    if (v == 1 && alpha == 0) return sgn * f_d(d, 1.0 - x);
    if (v == 0 && alpha == 1) return g_d(d, x);
    return -sgn * g_d(d, 1.0 - x);
}

int orc_basis(int v, int alpha, int deriv, double x, double *out)
{
    if (v < 0 || v > 1 || alpha < 0 || alpha > 1 || deriv < 0 || deriv > 2 || !out)
        return -1;
    *out = w_d(v, alpha, deriv, x);
    return 0;
}

/* ---------------------------------------------------------------------------
 * p-cubic Hermite interpolant (eq. p-cubic_interpolant):
 *   H(x) = sum_{v,alpha} phi^v_alpha h^alpha W^v_alpha(x/h),
 *   W^v_alpha(u) = prod_a w^{v_a}_{alpha_a}(u_a).
 * A derivative of H of multi-order delta differentiates each factor delta_a
 * times and divides by h_a^delta_a.
 * ------------------------------------------------------------------------- */
static double hermite_derivative(int dim, const double *data, const double *h,
                                 const double *xi, const int *delta)
{
    int nv = 1 << dim;
    double sum = 0.0;
    for (int v = 0; v < nv; v++) {
        for (int alpha = 0; alpha < nv; alpha++) {
            double term = data[v * nv + alpha];
            for (int a = 0; a < dim; a++) {
                int va = (v >> a) & 1;
                int aa = (alpha >> a) & 1;
                if (aa) term *= h[a];
                term *= w_d(va, aa, delta[a], xi[a]);
                for (int k = 0; k < delta[a]; k++) term /= h[a];
            }
            sum += term;
        }
    }
    return sum;
}

/* The same derivative summed in another order, axis by axis: the (v_a,
 * alpha_a) pairs of the last axis are contracted with their 1D factors
 * first, then those of the axis before it, and so on. The definition is the
 * same sum; only the order of the roundings differs. Used solely to measure
 * how far two correct FP64 evaluations of the interpolant lie apart (the
 * scale of the parity tolerance); the default is the literal sum above. */
static double hermite_derivative_axes(int dim, const double *data, const double *h,
                                      const double *xi, const int *delta)
{
    int nv = 1 << dim;
    /* acc[q], q = sum_a q_a 4^a with q_a = v_a + 2 alpha_a */
    double acc[64];
    for (int v = 0; v < nv; v++)
        for (int alpha = 0; alpha < nv; alpha++) {
            int q = 0;
            for (int a = dim - 1; a >= 0; a--)
                q = 4 * q + (((v >> a) & 1) + 2 * ((alpha >> a) & 1));
            acc[q] = data[v * nv + alpha];
        }
    int size = 1;
    for (int a = 0; a < dim; a++) size *= 4;
    for (int a = dim - 1; a >= 0; a--) {
        size /= 4;  /* entries left after contracting axis a */
        for (int r = 0; r < size; r++) {
            double s = 0.0;
            for (int qa = 0; qa < 4; qa++) {
                int va = qa & 1, aa = qa >> 1;
                double f = w_d(va, aa, delta[a], xi[a]);
                if (aa) f *= h[a];
                for (int k = 0; k < delta[a]; k++) f /= h[a];
                s += acc[r + size * qa] * f;
            }
            acc[r] = s;
        }
    }
    return acc[0];
}

static int g_sum_order = 0;

int orc_set_sum_order(int order)
{
    if (order < 0 || order > 1) return -1;
    g_sum_order = order;
    return 0;
}

static double hermite_any(int dim, const double *data, const double *h, const double *xi,
                          const int *delta)
{
    if (g_sum_order == 1) return hermite_derivative_axes(dim, data, h, xi, delta);
    return hermite_derivative(dim, data, h, xi, delta);
}

int orc_hermite(int dim, const double *data, const double *h, const double *xi,
                double *val, double *grad, double *hess)
{
    if (dim < 1 || dim > MAXD || !data || !h || !xi) return -1;
    int delta[MAXD];
    if (val) {
        for (int a = 0; a < dim; a++) delta[a] = 0;
        *val = hermite_any(dim, data, h, xi, delta);
    }
    if (grad) {
        for (int b = 0; b < dim; b++) {
            for (int a = 0; a < dim; a++) delta[a] = (a == b);
            grad[b] = hermite_any(dim, data, h, xi, delta);
        }
    }
    if (hess) {
        for (int b = 0; b < dim; b++)
            for (int c = 0; c < dim; c++) {
                for (int a = 0; a < dim; a++) delta[a] = (a == b) + (a == c);
                hess[b * dim + c] = hermite_any(dim, data, h, xi, delta);
            }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Grid helpers.
 * ------------------------------------------------------------------------- */
typedef struct {
    int dim;
    long nc[MAXD];   /* cells per axis */
    long nn[MAXD];   /* nodes per axis */
    double lo[MAXD], h[MAXD];
    long nodes;      /* total node count */
} grid_t;

static int make_grid(grid_t *g, int dim, const long *ncell, const double *lo,
                     const double *hi)
{
    if ((dim != 2 && dim != 3) || !ncell || !lo || !hi) return -1;
    g->dim = dim;
    g->nodes = 1;
    for (int a = 0; a < MAXD; a++) {
        g->nc[a] = 0; g->nn[a] = 1; g->lo[a] = 0.0; g->h[a] = 1.0;
    }
    for (int a = 0; a < dim; a++) {
        if (ncell[a] < 2 || !(hi[a] > lo[a])) return -1;
        g->nc[a] = ncell[a];
        g->nn[a] = ncell[a] + 1;
        g->lo[a] = lo[a];
        g->h[a] = (hi[a] - lo[a]) / (double)ncell[a];
        g->nodes *= g->nn[a];
    }
    return 0;
}

static long node_index(const grid_t *g, const long *ijk)
{
    long idx = 0, stride = 1;
    for (int a = 0; a < g->dim; a++) {
        idx += ijk[a] * stride;
        stride *= g->nn[a];
    }
    return idx;
}

static void node_coords(const grid_t *g, long idx, long *ijk)
{
    for (int a = 0; a < g->dim; a++) {
        ijk[a] = idx % g->nn[a];
        idx /= g->nn[a];
    }
}

/* ---------------------------------------------------------------------------
 * Cross derivatives, approach (A): central differences of neighbouring
 * gradient values. D_a is the 1D second-order difference along axis a.
 * ------------------------------------------------------------------------- */
static double diff_axis(const grid_t *g, const double *u, const long *ijk, int a)
{
    long p[MAXD], q[MAXD], r[MAXD];
    long n = g->nn[a] - 1; /* last node index */
    for (int b = 0; b < g->dim; b++) p[b] = q[b] = r[b] = ijk[b];
    double h = g->h[a];
    if (ijk[a] == 0) {
        q[a] = 1; r[a] = 2;
        return (-3.0 * u[node_index(g, p)] + 4.0 * u[node_index(g, q)] - u[node_index(g, r)]) / (2.0 * h);
    }
    if (ijk[a] == n) {
        q[a] = n - 1; r[a] = n - 2;
        return (3.0 * u[node_index(g, p)] - 4.0 * u[node_index(g, q)] + u[node_index(g, r)]) / (2.0 * h);
    }
    q[a] = ijk[a] + 1; r[a] = ijk[a] - 1;
    return (u[node_index(g, q)] - u[node_index(g, r)]) / (2.0 * h);
}

static int mixed_planes(const grid_t *g, int mode, const double *psi, double *mixed)
{
    int nm = (g->dim == 2) ? 1 : 4;
    long N = g->nodes;
    if (mode == 2 || mode == 1) {
        /* zero (mode 2); cell-based values are formed per cell (mode 1) */
        memset(mixed, 0, sizeof(double) * (size_t)(nm * N));
        return 0;
    }
    if (mode != 0) return -1;
    const double *psi_y = psi + N;
    if (g->dim == 2) {
#pragma omp parallel for schedule(static)
        for (long idx = 0; idx < N; idx++) {
            long ijk[MAXD];
            node_coords(g, idx, ijk);
            mixed[idx] = diff_axis(g, psi_y, ijk, 0); /* phi_xy = D_x psi_y */
        }
        return 0;
    }
    const double *psi_z = psi + 2 * N;
    double *dyz = (double *)malloc(sizeof(double) * (size_t)N);
    if (!dyz) return -1;
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long ijk[MAXD] = {0, 0, 0};
        node_coords(g, idx, ijk);
        dyz[idx] = diff_axis(g, psi_z, ijk, 1);             /* D_y psi_z */
    }
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long ijk[MAXD] = {0, 0, 0};
        node_coords(g, idx, ijk);
        mixed[idx] = diff_axis(g, psi_y, ijk, 0);           /* phi_xy  = D_x psi_y     */
        mixed[N + idx] = diff_axis(g, psi_z, ijk, 0);       /* phi_xz  = D_x psi_z     */
        mixed[2 * N + idx] = dyz[idx];                      /* phi_yz  = D_y psi_z     */
        mixed[3 * N + idx] = diff_axis(g, dyz, ijk, 0);     /* phi_xyz = D_x D_y psi_z */
    }
    free(dyz);
    return 0;
}

int orc_mixed(int dim, const long *ncell, const double *lo, const double *hi,
              int mode, const double *psi, double *mixed)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !psi || !mixed || mode == 1) return -1;
    return mixed_planes(&g, mode, psi, mixed);
}

/* ---------------------------------------------------------------------------
 * Velocity fields. G[i*dim+j] = d v_j / d x_i (the paper's deformation
 * matrix, rows = derivative direction).
 * ------------------------------------------------------------------------- */
static const double PI = 3.14159265358979323846;

static double time_factor(double period, double t)
{
    return (period > 0.0) ? cos(PI * t / period) : 1.0;
}

/* v = (-s_y, s_x) from a stream function s with first derivatives (sx, sy)
 * and second derivatives (sxx, sxy, syy). */
static void from_stream(double sx, double sy, double sxx, double sxy, double syy,
                        double *v, double *G)
{
    v[0] = -sy;
    v[1] = sx;
    G[0 * 2 + 0] = -sxy; /* d u / dx */
    G[0 * 2 + 1] = sxx;  /* d v / dx */
    G[1 * 2 + 0] = -syy; /* d u / dy */
    G[1 * 2 + 1] = sxy;  /* d v / dy */
}

static int velocity_steady(int dim, int kind, const double *p, long np,
                           const double *x, double *v, double *G)
{
    int d = dim;
    if (kind == 1) { /* AFFINE: v = b + A (x - c) */
        if (np != 2 * d + d * d) return -1;
        const double *b = p, *c = p + d, *A = p + 2 * d;
        for (int i = 0; i < d; i++) {
            v[i] = b[i];
            for (int j = 0; j < d; j++) v[i] += A[i * d + j] * (x[j] - c[j]);
        }
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) G[i * d + j] = A[j * d + i];
        return 0;
    }
    if (kind == 2) { /* STREAM_SIN: s = sum a sin(m pi x) sin(n pi y) */
        if (d != 2 || np % 3 != 0) return -1;
        double sx = 0, sy = 0, sxx = 0, sxy = 0, syy = 0;
        for (long k = 0; k < np / 3; k++) {
            double a = p[3 * k], M = p[3 * k + 1] * PI, N = p[3 * k + 2] * PI;
            double Sx = sin(M * x[0]), Cx = cos(M * x[0]);
            double Sy = sin(N * x[1]), Cy = cos(N * x[1]);
            sx += a * M * Cx * Sy;
            sy += a * N * Sx * Cy;
            sxx += -a * M * M * Sx * Sy;
            syy += -a * N * N * Sx * Sy;
            sxy += a * M * N * Cx * Cy;
        }
        from_stream(sx, sy, sxx, sxy, syy, v, G);
        return 0;
    }
    if (kind == 3) { /* VECPOT_SIN: v = curl A */
        if (d != 3 || np % 6 != 0) return -1;
        double dA[3][3] = {{0}};      /* dA[c][i]    = d A_c / d x_i          */
        double ddA[3][3][3] = {{{0}}}; /* ddA[c][i][j] = d2 A_c / d x_i d x_j */
        for (long k = 0; k < np / 6; k++) {
            const double *a = p + 6 * k;
            double K[3] = {a[3] * PI, a[4] * PI, a[5] * PI};
            double S[3], C[3];
            for (int i = 0; i < 3; i++) { S[i] = sin(K[i] * x[i]); C[i] = cos(K[i] * x[i]); }
            double fg[3], fh[3][3];
            /* gradient and Hessian of f = S0 S1 S2 */
            for (int i = 0; i < 3; i++) {
                double t = K[i] * C[i];
                for (int m = 0; m < 3; m++) if (m != i) t *= S[m];
                fg[i] = t;
                for (int j = 0; j < 3; j++) {
                    double u;
                    if (i == j) {
                        u = -K[i] * K[i] * S[0] * S[1] * S[2];
                    } else {
                        int o = 3 - i - j;
                        u = K[i] * C[i] * K[j] * C[j] * S[o];
                    }
                    fh[i][j] = u;
                }
            }
            for (int c = 0; c < 3; c++)
                for (int i = 0; i < 3; i++) {
                    dA[c][i] += a[c] * fg[i];
                    for (int j = 0; j < 3; j++) ddA[c][i][j] += a[c] * fh[i][j];
                }
        }
        /* v_j = eps_{jab} d_a A_b ; G[i][j] = d_i v_j = eps_{jab} d_i d_a A_b */
        static const int nxt[3] = {1, 2, 0}, prv[3] = {2, 0, 1};
        for (int j = 0; j < 3; j++) {
            int a = nxt[j], b = prv[j];
            v[j] = dA[b][a] - dA[a][b];
            for (int i = 0; i < 3; i++) G[i * 3 + j] = ddA[b][i][a] - ddA[a][i][b];
        }
        return 0;
    }
    if (kind == 4) { /* VORTEX: s = (1/pi) sin^2(pi x) sin^2(pi y) */
        if (d != 2 || np != 0) return -1;
        double sx1 = sin(PI * x[0]), sy1 = sin(PI * x[1]);
        double s2x = sin(2 * PI * x[0]), s2y = sin(2 * PI * x[1]);
        double c2x = cos(2 * PI * x[0]), c2y = cos(2 * PI * x[1]);
        double sx = s2x * sy1 * sy1;
        double sy = sx1 * sx1 * s2y;
        double sxx = 2 * PI * c2x * sy1 * sy1;
        double syy = 2 * PI * sx1 * sx1 * c2y;
        double sxy = PI * s2x * s2y;
        from_stream(sx, sy, sxx, sxy, syy, v, G);
        return 0;
    }
    if (kind == 5) { /* PSEUDO1D: v = exp(e.x) e (eq. velocity_1) */
        if (d != 2 || np != 0) return -1;
        double r = sqrt(2.0 + PI);
        double e[2] = {sqrt(2.0) / r, sqrt(PI) / r};
        double ex = exp(e[0] * x[0] + e[1] * x[1]);
        for (int j = 0; j < 2; j++) v[j] = ex * e[j];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) G[i * 2 + j] = ex * e[i] * e[j];
        return 0;
    }
    if (kind == 6) { /* LEVEQUE3D (sec. 6.2, 3D deformation field) */
        if (d != 3 || np != 0) return -1;
        double s1[3], s2[3], c2[3];
        for (int i = 0; i < 3; i++) {
            s1[i] = sin(PI * x[i]); s2[i] = sin(2 * PI * x[i]); c2[i] = cos(2 * PI * x[i]);
        }
        double q[3] = {s1[0] * s1[0], s1[1] * s1[1], s1[2] * s1[2]}; /* sin^2 */
        v[0] = 2.0 * q[0] * s2[1] * s2[2];
        v[1] = -s2[0] * q[1] * s2[2];
        v[2] = -s2[0] * s2[1] * q[2];
        /* d sin^2(pi x)/dx = pi sin(2 pi x); d sin(2 pi x)/dx = 2 pi cos(2 pi x) */
        G[0 * 3 + 0] = 2.0 * PI * s2[0] * s2[1] * s2[2];
        G[1 * 3 + 0] = 2.0 * q[0] * 2 * PI * c2[1] * s2[2];
        G[2 * 3 + 0] = 2.0 * q[0] * s2[1] * 2 * PI * c2[2];
        G[0 * 3 + 1] = -2 * PI * c2[0] * q[1] * s2[2];
        G[1 * 3 + 1] = -s2[0] * PI * s2[1] * s2[2];
        G[2 * 3 + 1] = -s2[0] * q[1] * 2 * PI * c2[2];
        G[0 * 3 + 2] = -2 * PI * c2[0] * s2[1] * q[2];
        G[1 * 3 + 2] = -s2[0] * 2 * PI * c2[1] * q[2];
        G[2 * 3 + 2] = -s2[0] * s2[1] * PI * s2[2];
        return 0;
    }
    return -1;
}

int orc_velocity(int dim, int kind, const double *params, long nparams,
                 double period, const double *x, double t, double *v, double *G)
{
    double vv[MAXD], GG[MAXD * MAXD];
    if ((dim != 2 && dim != 3) || !x || !v || !G) return -1;
    if (velocity_steady(dim, kind, params, nparams, x, vv, GG)) return -1;
    double c = time_factor(period, t);
    for (int i = 0; i < dim; i++) v[i] = c * vv[i];
    for (int i = 0; i < dim * dim; i++) G[i] = c * GG[i];
    return 0;
}

/* ---------------------------------------------------------------------------
 * Superconsistent Shu-Osher trace (Ex. ex:superconsistent_ShuOsher), written
 * in the paper's convention: D1 = grad x1, D2 = grad x2, D = grad X, and
 * products "grad x1 . grad v(x1)" are matrix products D1 G(x1).
 * ------------------------------------------------------------------------- */
static void matmul(int d, const double *A, const double *B, double *C)
{
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = 0.0;
            for (int k = 0; k < d; k++) s += A[i * d + k] * B[k * d + j];
            C[i * d + j] = s;
        }
}

int orc_trace(int dim, int kind, const double *params, long nparams, double period,
              const double *x, double t, double dt, double *X, double *D)
{
    int d = dim;
    double v0[MAXD], v1[MAXD], v2[MAXD];
    double G0[9], G1[9], G2[9], D1[9], D2[9], P1[9], P2[9];
    double x1[MAXD], x2[MAXD];
    if (!x || !X || !D) return -1;
    /* x1 = x - dt v(x, t+dt);  grad x1 = I - dt grad v(x, t+dt) */
    if (orc_velocity(d, kind, params, nparams, period, x, t + dt, v0, G0)) return -1;
    for (int i = 0; i < d; i++) x1[i] = x[i] - dt * v0[i];
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) D1[i * d + j] = (i == j) - dt * G0[i * d + j];
    /* x2 = x - dt (v(x,t+dt)/4 + v(x1,t)/4) */
    if (orc_velocity(d, kind, params, nparams, period, x1, t, v1, G1)) return -1;
    matmul(d, D1, G1, P1);
    for (int i = 0; i < d; i++) x2[i] = x[i] - dt * (0.25 * v0[i] + 0.25 * v1[i]);
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++)
            D2[i * d + j] = (i == j) - dt * (0.25 * G0[i * d + j] + 0.25 * P1[i * d + j]);
    /* X = x - dt (v(x,t+dt)/6 + v(x1,t)/6 + 2 v(x2,t+dt/2)/3) */
    if (orc_velocity(d, kind, params, nparams, period, x2, t + 0.5 * dt, v2, G2)) return -1;
    matmul(d, D2, G2, P2);
    for (int i = 0; i < d; i++)
        X[i] = x[i] - dt * (v0[i] / 6.0 + v1[i] / 6.0 + 2.0 * v2[i] / 3.0);
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++)
            D[i * d + j] = (i == j) - dt * (G0[i * d + j] / 6.0 + P1[i * d + j] / 6.0 +
                                            2.0 * P2[i * d + j] / 3.0);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Locate a point: cell index clamped to the grid, local coordinate unclamped.
 * ------------------------------------------------------------------------- */
static void locate(const grid_t *g, const double *X, long *cell, double *xi)
{
    for (int a = 0; a < g->dim; a++) {
        double s = (X[a] - g->lo[a]) / g->h[a];
        double fl = floor(s);
        long c;
        if (fl >= 0.0 && fl <= (double)(g->nc[a] - 1)) c = (long)fl;
        else if (fl > (double)(g->nc[a] - 1)) c = g->nc[a] - 1;
        else c = 0; /* below the grid, or not a number */
        cell[a] = c;
        xi[a] = s - (double)c;
    }
}

/* Approach (B) on one facet: the cross derivative u_ab at the four facet
 * vertices (index 0..3, bit 0 along axis a, bit 1 along axis b) from
 * ga = phi_a and gb = phi_b there. Edge-centre differences
 *   (ga(.,1) - ga(.,0)) / hb on the two edges along b,
 *   (gb(1,.) - gb(0,.)) / ha on the two edges along a,
 * then each vertex takes 3/4 of its two edges and -1/4 of the two others. */
static void cell_cross(const double *ga, const double *gb, double ha, double hb, double *out)
{
    double ea[2], eb[2]; /* ea[k]: edge at position k along a; eb[k]: at k along b */
    for (int k = 0; k < 2; k++) {
        ea[k] = (ga[k + 2] - ga[k]) / hb;
        eb[k] = (gb[2 * k + 1] - gb[2 * k]) / ha;
    }
    for (int v = 0; v < 4; v++) {
        int va = v & 1, vb = (v >> 1) & 1;
        out[v] = 0.75 * (ea[va] + eb[vb]) - 0.25 * (ea[1 - va] + eb[1 - vb]);
    }
}

/* Replace the cross derivatives of gathered cell data by approach (B). */
static void cell_based_cross(const grid_t *g, double *data)
{
    int nv = 1 << g->dim;
    if (g->dim == 2) {
        double ga[4], gb[4], out[4];
        for (int v = 0; v < 4; v++) { ga[v] = data[v * 4 + 1]; gb[v] = data[v * 4 + 2]; }
        cell_cross(ga, gb, g->h[0], g->h[1], out);
        for (int v = 0; v < 4; v++) data[v * 4 + 3] = out[v];
        return;
    }
    /* 3D: the facet through vertex v normal to axis c, for the pair (a, b) */
    static const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2}, pc[3] = {2, 1, 0};
    static const int slot[3] = {3, 5, 6}; /* xy, xz, yz */
    for (int q = 0; q < 3; q++) {
        int a = pa[q], b = pb[q], c = pc[q];
        for (int lc = 0; lc < 2; lc++) {
            double ga[4], gb[4], out[4];
            int ids[4];
            for (int k = 0; k < 4; k++) {
                int v = ((k & 1) << a) | (((k >> 1) & 1) << b) | (lc << c);
                ids[k] = v;
                ga[k] = data[v * nv + (1 << a)];
                gb[k] = data[v * nv + (1 << b)];
            }
            cell_cross(ga, gb, g->h[a], g->h[b], out);
            for (int k = 0; k < 4; k++) data[ids[k] * nv + slot[q]] = out[k];
        }
    }
    /* phi_xyz (first order) from psi_z on the xy facet at each z level */
    for (int lz = 0; lz < 2; lz++) {
        int v00 = 4 * lz, v10 = v00 + 1, v01 = v00 + 2, v11 = v00 + 3;
        double val = (data[v11 * nv + 4] - data[v01 * nv + 4] - data[v10 * nv + 4] +
                      data[v00 * nv + 4]) / (g->h[0] * g->h[1]);
        for (int k = 0; k < 4; k++) data[(v00 + k) * nv + 7] = val;
    }
}

/* Gather the 4^p data of a cell: data[v*2^p + alpha]. */
static void gather_cell(const grid_t *g, const long *cell, const double *phi,
                        const double *psi, const double *mixed, double *data)
{
    int nv = 1 << g->dim;
    long N = g->nodes;
    /* plane of the alpha-th datum: 0 phi, single bit -> psi_a, else a mixed plane */
    for (int v = 0; v < nv; v++) {
        long ijk[MAXD] = {0, 0, 0};
        for (int a = 0; a < g->dim; a++) ijk[a] = cell[a] + ((v >> a) & 1);
        long idx = node_index(g, ijk);
        for (int alpha = 0; alpha < nv; alpha++) {
            double val;
            if (alpha == 0) val = phi[idx];
            else if (alpha == 1) val = psi[idx];
            else if (alpha == 2) val = psi[N + idx];
            else if (alpha == 4) val = psi[2 * N + idx];
            else if (alpha == 3) val = mixed[idx];            /* xy  */
            else if (alpha == 5) val = mixed[N + idx];        /* xz  */
            else if (alpha == 6) val = mixed[2 * N + idx];    /* yz  */
            else val = mixed[3 * N + idx];                    /* xyz */
            data[v * nv + alpha] = val;
        }
    }
}

/* One GA-CIR step at node idx (sec. 4, steps 1-3, with the superconsistent
 * gradient update of eq. superconsistency). */
static int step_node(const grid_t *g, int kind, const double *params, long np,
                     double period, int bc, int mixed_mode, int psi_update,
                     const double *phi, const double *psi, const double *mixed, double t,
                     double dt, long idx, double *phi_new, double *psi_new)
{
    int d = g->dim;
    long ijk[MAXD], cell[MAXD];
    double x[MAXD], X[MAXD], D[9], xi[MAXD], data[64], val, grad[MAXD];
    int outside[MAXD] = {0, 0, 0};
    node_coords(g, idx, ijk);
    for (int a = 0; a < d; a++) x[a] = g->lo[a] + (double)ijk[a] * g->h[a];
    if (orc_trace(d, kind, params, np, period, x, t, dt, X, D)) return -1;
    if (bc == 0 || bc == 3) {
        /* homogeneous Neumann: project the foot onto the domain */
        for (int a = 0; a < d; a++) {
            double top = g->lo[a] + (double)g->nc[a] * g->h[a];
            double tol = ORC_FOOT_TOL * g->h[a];
            if (X[a] < g->lo[a] - tol) { X[a] = g->lo[a]; outside[a] = 1; }
            else if (X[a] > top + tol) { X[a] = top; outside[a] = 1; }
        }
    }
    locate(g, X, cell, xi);
    gather_cell(g, cell, phi, psi, mixed, data);
    if (mixed_mode == 1) cell_based_cross(g, data);
    orc_hermite(d, data, g->h, xi, &val, grad, NULL);
    for (int a = 0; a < d; a++)
        if (outside[a]) grad[a] = 0.0; /* the extension is constant along the normal */
    *phi_new = val;
    if (psi_update == 1) {
        /* Heun's method for d psi/d tau = -grad v . psi (eq. cir_evolution_psi)
         * from the foot at time t to the node at time t + dt */
        double v[MAXD], Gf[9], Gn[9], k1[MAXD], k2[MAXD], pp[MAXD];
        if (orc_velocity(d, kind, params, np, period, X, t, v, Gf)) return -1;
        if (orc_velocity(d, kind, params, np, period, x, t + dt, v, Gn)) return -1;
        for (int i = 0; i < d; i++) {
            double s = 0.0;
            for (int j = 0; j < d; j++) s += Gf[i * d + j] * grad[j];
            k1[i] = -s;
        }
        for (int i = 0; i < d; i++) pp[i] = grad[i] + dt * k1[i];
        for (int i = 0; i < d; i++) {
            double s = 0.0;
            for (int j = 0; j < d; j++) s += Gn[i * d + j] * pp[j];
            k2[i] = -s;
        }
        for (int i = 0; i < d; i++) psi_new[i] = grad[i] + 0.5 * dt * (k1[i] + k2[i]);
        return 0;
    }
    for (int i = 0; i < d; i++) {
        double s = 0.0;
        for (int j = 0; j < d; j++) s += D[i * d + j] * grad[j];
        psi_new[i] = s;
    }
    return 0;
}

/* Inflow faces of a boundary node (sec. 4.1: where v . n < 0). The flow
 * enters through face a when its inward normal component exceeds
 * INFLOW_THETA max(|v|, h_a / dt), dt the step: along a face that is a
 * streamline (v_n = 0 analytically) or at a stagnation point the rounding of
 * v must not decide, and the Dirichlet normal derivative, which divides by
 * v_n, stays bounded. Returns the number of inflow faces; in[a] marks them. */
#define INFLOW_THETA 1e-6
static int inflow_axes(const grid_t *g, const long *ijk, const double *v, double dt, int *in)
{
    double speed2 = 0.0;
    int nin = 0;
    for (int a = 0; a < g->dim; a++) speed2 += v[a] * v[a];
    for (int a = 0; a < g->dim; a++) {
        const double vmin = INFLOW_THETA * fmax(sqrt(speed2), g->h[a] / dt);
        /* low face: outward normal -e_a, inflow if v_a > 0; high face: v_a < 0 */
        in[a] = (ijk[a] == 0 && v[a] > vmin) || (ijk[a] == g->nc[a] && v[a] < -vmin);
        nin += in[a];
    }
    return nin;
}

/* Velocity restricted to the axes tax[0..k-1] of a boundary face: the
 * components v_T and their derivatives along T, Gs[i*k+j] = d v_{T_j} / d x_{T_i}
 * (the deformation-matrix convention), at a point whose other coordinates
 * stay on the face. */
static int face_velocity(const grid_t *g, int kind, const double *params, long np,
                         double period, const double *x, double t, const int *tax, int k,
                         double *vs, double *Gs)
{
    double v[MAXD], G[9];
    if (orc_velocity(g->dim, kind, params, np, period, x, t, v, G)) return -1;
    for (int i = 0; i < k; i++) {
        vs[i] = v[tax[i]];
        for (int j = 0; j < k; j++) Gs[i * k + j] = G[tax[i] * g->dim + tax[j]];
    }
    return 0;
}

/* Homogeneous Neumann inflow (sec. 4.1, eq. Neumann_bc_evolution with zero
 * prescribed normal derivative): at a boundary node where the flow enters
 * through the faces marked in[], phi and the gradient along the remaining
 * (tangential) axes T solve phi_t + v_T . grad_T phi = 0 on the face by a
 * GA-CIR step of dimension k = |T| (sec. 4, steps 1-3): the superconsistent
 * Shu-Osher trace with v_T, its foot projected onto the face, the k-cubic
 * Hermite interpolant of the face data at time t (cross derivative of the
 * pair of T axes by the context's rule) and psi_T = D grad H. The normal
 * derivatives are the prescribed zeros. With no tangential axis left (a
 * corner where the flow enters through every face) phi keeps its value. */
static int face_node(const grid_t *g, int kind, const double *params, long np, double period,
                     int mixed_mode, const double *phi, const double *psi, const double *mixed,
                     double t, double dt, const long *ijk, const int *in, double *phi_new,
                     double *psi_new)
{
    int d = g->dim, k = 0, tax[MAXD];
    long N = g->nodes, idx = node_index(g, ijk);
    for (int a = 0; a < d; a++) {
        psi_new[a] = 0.0;
        if (!in[a]) tax[k++] = a;
    }
    if (k == 0) {
        *phi_new = phi[idx];
        return 0;
    }
    /* superconsistent Shu-Osher trace on the face (as orc_trace, axes T only) */
    double x[MAXD], x1[MAXD], x2[MAXD], X[MAXD];
    double v0[2], v1[2], v2[2], G0[4], G1[4], G2[4], D1[4], D2[4], P1[4], P2[4], D[4];
    for (int a = 0; a < d; a++) x[a] = g->lo[a] + (double)ijk[a] * g->h[a];
    for (int a = 0; a < d; a++) x1[a] = x2[a] = X[a] = x[a];
    if (face_velocity(g, kind, params, np, period, x, t + dt, tax, k, v0, G0)) return -1;
    for (int i = 0; i < k; i++) x1[tax[i]] = x[tax[i]] - dt * v0[i];
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++) D1[i * k + j] = (i == j) - dt * G0[i * k + j];
    if (face_velocity(g, kind, params, np, period, x1, t, tax, k, v1, G1)) return -1;
    matmul(k, D1, G1, P1);
    for (int i = 0; i < k; i++) x2[tax[i]] = x[tax[i]] - dt * (0.25 * v0[i] + 0.25 * v1[i]);
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++)
            D2[i * k + j] = (i == j) - dt * (0.25 * G0[i * k + j] + 0.25 * P1[i * k + j]);
    if (face_velocity(g, kind, params, np, period, x2, t + 0.5 * dt, tax, k, v2, G2)) return -1;
    matmul(k, D2, G2, P2);
    for (int i = 0; i < k; i++)
        X[tax[i]] = x[tax[i]] - dt * (v0[i] / 6.0 + v1[i] / 6.0 + 2.0 * v2[i] / 3.0);
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++)
            D[i * k + j] = (i == j) - dt * (G0[i * k + j] / 6.0 + P1[i * k + j] / 6.0 +
                                            2.0 * P2[i * k + j] / 3.0);
    /* project the foot onto the face; locate it in the face's cells */
    long cell[MAXD], fullcell[MAXD];
    double xi_full[MAXD], xi[2], hs[2];
    int outside[2] = {0, 0};
    for (int i = 0; i < k; i++) {
        int a = tax[i];
        double top = g->lo[a] + (double)g->nc[a] * g->h[a];
        double tol = ORC_FOOT_TOL * g->h[a];
        if (X[a] < g->lo[a] - tol) { X[a] = g->lo[a]; outside[i] = 1; }
        else if (X[a] > top + tol) { X[a] = top; outside[i] = 1; }
    }
    locate(g, X, fullcell, xi_full);
    for (int i = 0; i < k; i++) {
        cell[i] = fullcell[tax[i]];
        xi[i] = xi_full[tax[i]];
        hs[i] = g->h[tax[i]];
    }
    /* face cell data, data[v * 2^k + alpha]: vertex bit i and derivative bit
     * i along T_i; alpha 3 (k = 2) is the cross derivative of the pair */
    int nv = 1 << k;
    double data[16], ga[4], gb[4], cr[4];
    long pair_plane = 0;
    if (k == 2) pair_plane = (tax[0] == 0) ? (tax[1] == 1 ? 0 : 1) : 2; /* xy, xz, yz */
    for (int v = 0; v < nv; v++) {
        long vijk[MAXD];
        for (int a = 0; a < d; a++) vijk[a] = ijk[a];
        for (int i = 0; i < k; i++) vijk[tax[i]] = cell[i] + ((v >> i) & 1);
        long vi = node_index(g, vijk);
        data[v * nv + 0] = phi[vi];
        for (int i = 0; i < k; i++) data[v * nv + (1 << i)] = psi[tax[i] * N + vi];
        if (k == 2) {
            ga[v] = psi[tax[0] * N + vi];
            gb[v] = psi[tax[1] * N + vi];
            /* approach (A): the 3D mixed plane of the pair, a difference along
             * the face (2D grids have no pair on a face) */
            data[v * nv + 3] = (mixed_mode == 0) ? mixed[pair_plane * N + vi] : 0.0;
        }
    }
    if (k == 2 && mixed_mode == 1) {
        cell_cross(ga, gb, hs[0], hs[1], cr);
        for (int v = 0; v < 4; v++) data[v * nv + 3] = cr[v];
    }
    double val, grad[2];
    orc_hermite(k, data, hs, xi, &val, grad, NULL);
    for (int i = 0; i < k; i++)
        if (outside[i]) grad[i] = 0.0;
    *phi_new = val;
    for (int i = 0; i < k; i++) {
        double s = 0.0;
        for (int j = 0; j < k; j++) s += D[i * k + j] * grad[j];
        psi_new[tax[i]] = s;
    }
    return 0;
}

/* bc 3: after a step with projected feet, inflow boundary nodes take the
 * face scheme's values, computed from the state at time t. */
static int face_override(const grid_t *g, int kind, const double *params, long np,
                         double period, int mixed_mode, const double *phi, const double *psi,
                         const double *mixed, double t, double dt, long idx, double *phi_new,
                         double *psi_new)
{
    long ijk[MAXD];
    double x[MAXD], v[MAXD], G[9];
    int in[MAXD], on_boundary = 0;
    node_coords(g, idx, ijk);
    for (int a = 0; a < g->dim; a++)
        if (ijk[a] == 0 || ijk[a] == g->nc[a]) on_boundary = 1;
    if (!on_boundary) return 0;
    for (int a = 0; a < g->dim; a++) x[a] = g->lo[a] + (double)ijk[a] * g->h[a];
    if (orc_velocity(g->dim, kind, params, np, period, x, t + dt, v, G)) return -1;
    if (inflow_axes(g, ijk, v, dt, in) == 0) return 0;
    return face_node(g, kind, params, np, period, mixed_mode, phi, psi, mixed, t, dt, ijk, in,
                     phi_new, psi_new);
}

int orc_advance(int dim, const long *ncell, const double *lo, const double *hi,
                int kind, const double *params, long nparams, double period,
                int mixed_mode, int bc, int psi_update, double *phi, double *psi,
                double t0, double dt, long steps)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !phi || !psi || steps < 0 || bc < 0 || bc > 3 ||
        bc == 2 || psi_update < 0 || psi_update > 1)
        return -1;
    long N = g.nodes;
    int nm = (dim == 2) ? 1 : 4;
    double *mixed = (double *)malloc(sizeof(double) * (size_t)(nm * N));
    double *phi2 = (double *)malloc(sizeof(double) * (size_t)N);
    double *psi2 = (double *)malloc(sizeof(double) * (size_t)(dim * N));
    int err = (!mixed || !phi2 || !psi2) ? -1 : 0;
    for (long n = 0; n < steps && !err; n++) {
        double t = t0 + (double)n * dt;
        if (mixed_planes(&g, mixed_mode, psi, mixed)) { err = -1; break; }
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (long idx = 0; idx < N; idx++) {
            double pn, gn[MAXD];
            if (step_node(&g, kind, params, nparams, period, bc, mixed_mode, psi_update, phi,
                          psi, mixed, t, dt, idx, &pn, gn) ||
                (bc == 3 && face_override(&g, kind, params, nparams, period, mixed_mode, phi,
                                          psi, mixed, t, dt, idx, &pn, gn))) {
                bad = 1;
                continue;
            }
            phi2[idx] = pn;
            for (int a = 0; a < dim; a++) psi2[a * N + idx] = gn[a];
        }
        if (bad) { err = -1; break; }
        memcpy(phi, phi2, sizeof(double) * (size_t)N);
        memcpy(psi, psi2, sizeof(double) * (size_t)(dim * N));
    }
    free(mixed); free(phi2); free(psi2);
    return err;
}

/* Dirichlet inflow data (sec. 4.1): at a boundary node where the velocity at
 * time t (the end of the step) points into the domain, phi is prescribed,
 * the tangential gradient components follow from it, and the normal one
 * from the equation, phi_n = -(phi_t + sum of tangential v_a phi_a) / v_n.
 * phi_b, grad_b (dim planes) and phit_b hold the prescribed phi, its
 * gradient and its time derivative at the nodes; where the flow enters
 * through more than one face (edges, corners) every gradient component is
 * taken from grad_b. Other nodes are left as they are. Inflow faces as in
 * inflow_axes. */
int orc_apply_inflow(int dim, const long *ncell, const double *lo, const double *hi,
                     int kind, const double *params, long nparams, double period, double t,
                     double dt, double *phi, double *psi, const double *phi_b,
                     const double *grad_b, const double *phit_b)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !phi || !psi || !phi_b || !grad_b || !phit_b ||
        !(dt > 0.0))
        return -1;
    long N = g.nodes;
    int bad = 0;
    for (long idx = 0; idx < N; idx++) {
        long ijk[MAXD] = {0, 0, 0};
        double x[MAXD], v[MAXD], G[9];
        int in[MAXD], nin = 0, axis = -1;
        node_coords(&g, idx, ijk);
        int on_boundary = 0;
        for (int a = 0; a < dim; a++)
            if (ijk[a] == 0 || ijk[a] == g.nc[a]) on_boundary = 1;
        if (!on_boundary) continue;
        for (int a = 0; a < dim; a++) x[a] = g.lo[a] + (double)ijk[a] * g.h[a];
        if (orc_velocity(dim, kind, params, nparams, period, x, t, v, G)) { bad = 1; break; }
        nin = inflow_axes(&g, ijk, v, dt, in);
        for (int a = 0; a < dim; a++)
            if (in[a]) axis = a;
        if (nin == 0) continue;
        phi[idx] = phi_b[idx];
        for (int a = 0; a < dim; a++) psi[a * N + idx] = grad_b[a * N + idx];
        if (nin == 1) {
            double s = phit_b[idx];
            for (int a = 0; a < dim; a++)
                if (a != axis) s += v[a] * grad_b[a * N + idx];
            psi[axis * N + idx] = -s / v[axis];
        }
    }
    return bad ? -1 : 0;
}

int orc_step_nodes(int dim, const long *ncell, const double *lo, const double *hi,
                   int kind, const double *params, long nparams, double period,
                   int mixed_mode, int bc, int psi_update, const double *phi,
                   const double *psi, double t, double dt, const long *nodes, long count,
                   double *phi_out, double *psi_out)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !phi || !psi || !nodes || count < 0 ||
        bc < 0 || bc > 3 || bc == 2 || psi_update < 0 || psi_update > 1)
        return -1;
    long N = g.nodes;
    int nm = (dim == 2) ? 1 : 4;
    double *mixed = (double *)malloc(sizeof(double) * (size_t)(nm * N));
    if (!mixed) return -1;
    int err = mixed_planes(&g, mixed_mode, psi, mixed);
    for (long k = 0; k < count && !err; k++) {
        if (nodes[k] < 0 || nodes[k] >= N) { err = -1; break; }
        err = step_node(&g, kind, params, nparams, period, bc, mixed_mode, psi_update, phi,
                        psi, mixed, t, dt, nodes[k], &phi_out[k], &psi_out[k * dim]);
        if (!err && bc == 3)
            err = face_override(&g, kind, params, nparams, period, mixed_mode, phi, psi, mixed,
                                t, dt, nodes[k], &phi_out[k], &psi_out[k * dim]);
    }
    free(mixed);
    return err;
}

/* ---------------------------------------------------------------------------
 * Point evaluation: value, gradient, Hessian, normal (eq. surface_normal) and
 * curvature (eq. curvature in 2D; the divergence of the normal in 3D).
 * ------------------------------------------------------------------------- */
int orc_eval_points(int dim, const long *ncell, const double *lo, const double *hi,
                    int mixed_mode, const double *phi, const double *psi,
                    const double *pts, long npts, double *val, double *grad,
                    double *hess, double *normal, double *kappa)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !phi || !psi || (!pts && npts) || npts < 0)
        return -1;
    long N = g.nodes;
    int nm = (dim == 2) ? 1 : 4;
    double *mixed = (double *)malloc(sizeof(double) * (size_t)(nm * N));
    if (!mixed) return -1;
    if (mixed_planes(&g, mixed_mode, psi, mixed)) { free(mixed); return -1; }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npts; p++) {
        long cell[MAXD];
        double xi[MAXD], data[64], H, Gr[MAXD], Hs[9];
        locate(&g, pts + p * dim, cell, xi);
        gather_cell(&g, cell, phi, psi, mixed, data);
        if (mixed_mode == 1) cell_based_cross(&g, data);
        orc_hermite(dim, data, g.h, xi, &H, Gr, Hs);
        if (val) val[p] = H;
        if (grad) for (int a = 0; a < dim; a++) grad[p * dim + a] = Gr[a];
        if (hess) for (int a = 0; a < dim * dim; a++) hess[p * dim * dim + a] = Hs[a];
        double n2 = 0.0;
        for (int a = 0; a < dim; a++) n2 += Gr[a] * Gr[a];
        double nrm = sqrt(n2);
        if (normal)
            for (int a = 0; a < dim; a++) normal[p * dim + a] = (n2 > 0.0) ? Gr[a] / nrm : 0.0;
        if (kappa) {
            double k = 0.0;
            if (n2 > 0.0) {
                if (dim == 2) {
                    double px = Gr[0], py = Gr[1];
                    double pxx = Hs[0], pxy = Hs[1], pyy = Hs[3];
                    k = (pxx * py * py - 2.0 * px * py * pxy + pyy * px * px) / (n2 * nrm);
                } else {
                    double px = Gr[0], py = Gr[1], pz = Gr[2];
                    double pxx = Hs[0], pyy = Hs[4], pzz = Hs[8];
                    double pxy = Hs[1], pxz = Hs[2], pyz = Hs[5];
                    k = (px * px * (pyy + pzz) + py * py * (pxx + pzz) + pz * pz * (pxx + pyy)
                         - 2.0 * (px * py * pxy + px * pz * pxz + py * pz * pyz)) / (n2 * nrm);
                }
            }
            kappa[p] = k;
        }
    }
    free(mixed);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Diagnostics.
 * ------------------------------------------------------------------------- */
static double heaviside_eps(double s, double eps)
{
    if (s < -eps) return 0.0;
    if (s > eps) return 1.0;
    return 0.5 * (1.0 + s / eps + sin(PI * s / eps) / PI);
}

int orc_norms(int dim, const long *ncell, const double *lo, const double *hi,
              const double *phi, const double *psi, const double *phi_ref,
              const double *psi_ref, double eps, double band, double *out)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi) || !phi || !psi || !phi_ref || !psi_ref || !out)
        return -1;
    long N = g.nodes;
    double cellvol = 1.0;
    for (int a = 0; a < dim; a++) cellvol *= g.h[a];
    double emax_phi = 0, emax_psi = 0, l1 = 0, linf_band = 0, vol = 0, vol_ref = 0;
    double nonfinite = 0, max_ref = 0;
    for (long i = 0; i < N; i++) {
        double e = fabs(phi[i] - phi_ref[i]);
        if (e > emax_phi) emax_phi = e;
        for (int a = 0; a < dim; a++) {
            double ea = fabs(psi[a * N + i] - psi_ref[a * N + i]);
            if (ea > emax_psi) emax_psi = ea;
            if (!isfinite(psi[a * N + i])) nonfinite += 1;
        }
        if (!isfinite(phi[i])) nonfinite += 1;
        l1 += fabs(heaviside_eps(phi[i], eps) - heaviside_eps(phi_ref[i], eps));
        if (fabs(phi_ref[i]) <= band && e > linf_band) linf_band = e;
        vol += heaviside_eps(-phi[i], eps);
        vol_ref += heaviside_eps(-phi_ref[i], eps);
        if (fabs(phi_ref[i]) > max_ref) max_ref = fabs(phi_ref[i]);
    }
    out[0] = emax_phi; out[1] = emax_psi; out[2] = l1 * cellvol; out[3] = linf_band;
    out[4] = vol * cellvol; out[5] = vol_ref * cellvol; out[6] = nonfinite; out[7] = max_ref;
    return 0;
}

double orc_max_speed(int dim, const long *ncell, const double *lo, const double *hi,
                     int kind, const double *params, long nparams, double period,
                     double t)
{
    grid_t g;
    if (make_grid(&g, dim, ncell, lo, hi)) return -1.0;
    double best = 0.0;
    for (long idx = 0; idx < g.nodes; idx++) {
        long ijk[MAXD] = {0, 0, 0};
        double x[MAXD], v[MAXD], G[9];
        node_coords(&g, idx, ijk);
        for (int a = 0; a < dim; a++) x[a] = g.lo[a] + (double)ijk[a] * g.h[a];
        if (orc_velocity(dim, kind, params, nparams, period, x, t, v, G)) return -1.0;
        double s = 0.0;
        for (int a = 0; a < dim; a++) s += v[a] * v[a];
        s = sqrt(s);
        if (s > best) best = s;
    }
    return best;
}

/* Threads of the OpenMP loops from now on (n >= 1). */
int orc_set_threads(int n)
{
    if (n < 1) return -1;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
