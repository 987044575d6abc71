/*
 * Parameter derivatives of the 2D GA-CIR advance by complex-step
 * differentiation.
 *
 * TEST INFRASTRUCTURE ONLY (like gals_oracle.c): the GPU library never links,
 * loads or calls this file.
 *
 * For a sine stream function s = sum_k a_k sin(m_k pi x) sin(n_k pi y), the
 * velocity depends on the amplitudes only through the folded table
 * S[m][n] = sum of a_k over the modes with (m_k, n_k) = (m, n). The derivative
 * of a functional F(u_T) of the final state with respect to S[m][n] is
 *     dF/dS[m][n] = Im F(S + i h e_mn) / h,   h = 1e-30,
 * exact to rounding because no difference of nearby numbers is taken. The
 * step is evaluated in complex arithmetic exactly as the paper states it
 * (sec. 4 steps 1-3, the superconsistent trace of Ex.
 * ex:superconsistent_ShuOsher, the Hermite interpolant of eq.
 * p-cubic_interpolant, the cross derivatives of approach (A) or (B), sec.
 * 2.3); the only non-analytic operations are the cell choice and the boundary
 * test, which look at the real part, so the result is the derivative of the
 * discrete advance with its cells held fixed (with (A) the advance is C^1 in
 * S, the interpolant being C^1 across cell faces; with (B) it is C^1 except
 * where a foot crosses a face).
 *
 * Two functionals:
 *   linear:  F = sum over nodes of lam_phi phi_T + lam_x psi_x,T + lam_y psi_y,T
 *   loss:    F = prod(h) sum over nodes of (H_eps(phi_T) - H_eps(phi_target))^2
 * with the smoothed Heaviside H_eps of the diagnostics (gals_oracle.c).
 * Boundary treatment and cross-derivative modes as in orc_advance.
 *
 * Built with -ffp-contract=off, like the rest of the oracle.
 */
#include "gals_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double PI_CS = 3.14159265358979323846;
static const double H_CS = 1e-30;

typedef struct {
    long nc[2], nn[2], N;
    double lo[2], h[2];
} grid2_t;

/* stream-function velocity and deformation matrix G[i*2+j] = d v_j / d x_i
 * (the paper's convention), from the real modes plus one imaginary
 * perturbation of S[pm][pn] (pm, pn in 1..4). */
static void velocity_cs(const double *params, long nmodes, int pm, int pn, double c,
                        const cplx *x, cplx *v, cplx *G)
{
    cplx sx = 0, sy = 0, sxx = 0, sxy = 0, syy = 0;
    for (long k = 0; k <= nmodes; k++) {
        cplx a;
        double M, N;
        if (k < nmodes) {
            a = params[3 * k];
            M = params[3 * k + 1] * PI_CS;
            N = params[3 * k + 2] * PI_CS;
        } else {
            a = I * H_CS;
            M = pm * PI_CS;
            N = pn * PI_CS;
        }
        cplx Sx = csin(M * x[0]), Cx = ccos(M * x[0]);
        cplx Sy = csin(N * x[1]), Cy = ccos(N * x[1]);
        sx += a * M * Cx * Sy;
        sy += a * N * Sx * Cy;
        sxx += -a * M * M * Sx * Sy;
        syy += -a * N * N * Sx * Sy;
        sxy += a * M * N * Cx * Cy;
    }
    /* v = (-s_y, s_x) */
    v[0] = -c * sy;
    v[1] = c * sx;
    G[0] = -c * sxy; /* d u / dx */
    G[1] = c * sxx;  /* d v / dx */
    G[2] = -c * syy; /* d u / dy */
    G[3] = c * sxy;  /* d v / dy */
}

static double tfac(double period, double t)
{
    return (period > 0.0) ? cos(PI_CS * t / period) : 1.0;
}

static void matmul2(const cplx *A, const cplx *B, cplx *C)
{
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) C[i * 2 + j] = A[i * 2] * B[j] + A[i * 2 + 1] * B[2 + j];
}

/* Superconsistent Shu-Osher trace in the paper's convention (D = grad X). */
static void trace_cs(const double *params, long nmodes, int pm, int pn, double period,
                     const double *x, double t, double dt, cplx *X, cplx *D)
{
    cplx xc[2] = {x[0], x[1]}, v0[2], v1[2], v2[2], G0[4], G1[4], G2[4];
    cplx x1[2], x2[2], D1[4], D2[4], P1[4], P2[4];
    velocity_cs(params, nmodes, pm, pn, tfac(period, t + dt), xc, v0, G0);
    for (int i = 0; i < 2; i++) x1[i] = x[i] - dt * v0[i];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) D1[i * 2 + j] = (double)(i == j) - dt * G0[i * 2 + j];
    velocity_cs(params, nmodes, pm, pn, tfac(period, t), x1, v1, G1);
    matmul2(D1, G1, P1);
    for (int i = 0; i < 2; i++) x2[i] = x[i] - dt * (0.25 * v0[i] + 0.25 * v1[i]);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            D2[i * 2 + j] = (double)(i == j) - dt * (0.25 * G0[i * 2 + j] + 0.25 * P1[i * 2 + j]);
    velocity_cs(params, nmodes, pm, pn, tfac(period, t + 0.5 * dt), x2, v2, G2);
    matmul2(D2, G2, P2);
    for (int i = 0; i < 2; i++)
        X[i] = x[i] - dt * (v0[i] / 6.0 + v1[i] / 6.0 + 2.0 * v2[i] / 3.0);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            D[i * 2 + j] = (double)(i == j) - dt * (G0[i * 2 + j] / 6.0 + P1[i * 2 + j] / 6.0 +
                                                   2.0 * P2[i * 2 + j] / 3.0);
}

/* 1D basis of eq. (1-cubic_basis_functions) and derivatives, complex argument:
 * f = 1 - 3x^2 + 2x^3, g = x (1-x)^2, w^0_0 = f(x), w^1_0 = f(1-x),
 * w^0_1 = g(x), w^1_1 = -g(1-x). */
static cplx f_cs(int d, cplx x)
{
    if (d == 0) return 1.0 - 3.0 * x * x + 2.0 * x * x * x;
    return -6.0 * x + 6.0 * x * x;
}

static cplx g_cs(int d, cplx x)
{
    if (d == 0) return x * (1.0 - x) * (1.0 - x);
    return 1.0 - 4.0 * x + 3.0 * x * x;
}

static cplx w_cs(int v, int alpha, int d, cplx x)
{
    double sgn = (d == 0) ? 1.0 : -1.0;
    if (v == 0 && alpha == 0) return f_cs(d, x);
    if (v == 1 && alpha == 0) return sgn * f_cs(d, 1.0 - x);
    if (v == 0 && alpha == 1) return g_cs(d, x);
    return -sgn * g_cs(d, 1.0 - x);
}

/* Value (delta = 0,0) or first derivative of the bicubic interpolant:
 * sum over vertices v and derivative multi-indices alpha of
 * data[v*4 + alpha] prod_a h_a^alpha_a w^{v_a}_{alpha_a}(xi_a) / h_a^delta_a. */
static cplx hermite_cs(const cplx *data, const double *h, const cplx *xi, const int *delta)
{
    cplx sum = 0;
    for (int v = 0; v < 4; v++)
        for (int alpha = 0; alpha < 4; alpha++) {
            cplx term = data[v * 4 + alpha];
            for (int a = 0; a < 2; a++) {
                int va = (v >> a) & 1, aa = (alpha >> a) & 1;
                if (aa) term *= h[a];
                term *= w_cs(va, aa, delta[a], xi[a]);
                if (delta[a]) term /= h[a];
            }
            sum += term;
        }
    return sum;
}

/* D_x at node (i, j) of a node plane (central, one-sided 3-point at the ends). */
static cplx diff_x_cs(const grid2_t *g, const cplx *u, long i, long j)
{
    long n = g->nn[0] - 1, r = j * g->nn[0];
    double h = g->h[0];
    if (i == 0) return (-3.0 * u[r] + 4.0 * u[r + 1] - u[r + 2]) / (2.0 * h);
    if (i == n) return (3.0 * u[r + n] - 4.0 * u[r + n - 1] + u[r + n - 2]) / (2.0 * h);
    return (u[r + i + 1] - u[r + i - 1]) / (2.0 * h);
}

/* Approach (B) (sec. 2.3) on the cell's data: edge-centre differences of
 * psi_x along y and psi_y along x, then 3/4 of a vertex's two edges and -1/4
 * of the two others. */
static void cell_cross_cs(cplx *data, double hx, double hy)
{
    cplx ex[2], ey[2];
    for (int k = 0; k < 2; k++) {
        ex[k] = (data[(k + 2) * 4 + 1] - data[k * 4 + 1]) / hy;
        ey[k] = (data[(2 * k + 1) * 4 + 2] - data[(2 * k) * 4 + 2]) / hx;
    }
    for (int v = 0; v < 4; v++) {
        int vx = v & 1, vy = v >> 1;
        data[v * 4 + 3] = 0.75 * (ex[vx] + ey[vy]) - 0.25 * (ex[1 - vx] + ey[1 - vy]);
    }
}

static void step_cs(const grid2_t *g, const double *params, long nmodes, int pm, int pn,
                    double period, int mixed_mode, int bc, const cplx *phi, const cplx *psi,
                    cplx *mixed, double t, double dt, cplx *phi2, cplx *psi2)
{
    long N = g->N;
    const cplx *psi_y = psi + N;
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long i = idx % g->nn[0], j = idx / g->nn[0];
        mixed[idx] = (mixed_mode == 0) ? diff_x_cs(g, psi_y, i, j) : 0.0; /* phi_xy = D_x psi_y (A) */
    }
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long ij[2] = {idx % g->nn[0], idx / g->nn[0]};
        double x[2];
        cplx X[2], D[4], xi[2], data[16], grad[2];
        long cell[2];
        int outside[2] = {0, 0};
        for (int a = 0; a < 2; a++) x[a] = g->lo[a] + (double)ij[a] * g->h[a];
        trace_cs(params, nmodes, pm, pn, period, x, t, dt, X, D);
        if (bc == 0) { /* homogeneous Neumann: project the foot onto the domain */
            for (int a = 0; a < 2; a++) {
                double top = g->lo[a] + (double)g->nc[a] * g->h[a];
                double tol = ORC_FOOT_TOL * g->h[a];
                if (creal(X[a]) < g->lo[a] - tol) { X[a] = g->lo[a]; outside[a] = 1; }
                else if (creal(X[a]) > top + tol) { X[a] = top; outside[a] = 1; }
            }
        }
        for (int a = 0; a < 2; a++) { /* cell from the real part, xi keeps the imaginary part */
            cplx s = (X[a] - g->lo[a]) / g->h[a];
            double fl = floor(creal(s));
            long c;
            if (fl >= 0.0 && fl <= (double)(g->nc[a] - 1)) c = (long)fl;
            else if (fl > (double)(g->nc[a] - 1)) c = g->nc[a] - 1;
            else c = 0;
            cell[a] = c;
            xi[a] = s - (double)c;
        }
        for (int v = 0; v < 4; v++) {
            long k = (cell[0] + (v & 1)) + g->nn[0] * (cell[1] + (v >> 1));
            data[v * 4 + 0] = phi[k];
            data[v * 4 + 1] = psi[k];
            data[v * 4 + 2] = psi[N + k];
            data[v * 4 + 3] = mixed[k];
        }
        if (mixed_mode == 1) cell_cross_cs(data, g->h[0], g->h[1]);
        int d00[2] = {0, 0}, d10[2] = {1, 0}, d01[2] = {0, 1};
        phi2[idx] = hermite_cs(data, g->h, xi, d00);
        grad[0] = outside[0] ? 0.0 : hermite_cs(data, g->h, xi, d10);
        grad[1] = outside[1] ? 0.0 : hermite_cs(data, g->h, xi, d01);
        for (int a = 0; a < 2; a++) /* psi_new = grad X . grad H */
            psi2[a * N + idx] = D[a * 2 + 0] * grad[0] + D[a * 2 + 1] * grad[1];
    }
}

static cplx heaviside_cs(cplx s, double eps)
{
    if (creal(s) < -eps) return 0.0;
    if (creal(s) > eps) return 1.0;
    return 0.5 * (1.0 + s / eps + csin(PI_CS * s / eps) / PI_CS);
}

int orc_grad_cs(const long *ncell, const double *lo, const double *hi, const double *params,
                long nparams, double period, int mixed_mode, int bc, const double *phi0,
                const double *psi0, double t0, double dt, long steps, const double *lam,
                const double *phi_target, double eps, double *value, double *grad)
{
    grid2_t g;
    if (!ncell || !lo || !hi || !params || nparams % 3 || !phi0 || !psi0 || steps < 0 ||
        !grad || (!lam && !phi_target) || mixed_mode < 0 || mixed_mode > 2 || bc < 0 ||
        bc > 1)
        return -1;
    g.N = 1;
    for (int a = 0; a < 2; a++) {
        if (ncell[a] < 2 || !(hi[a] > lo[a])) return -1;
        g.nc[a] = ncell[a];
        g.nn[a] = ncell[a] + 1;
        g.lo[a] = lo[a];
        g.h[a] = (hi[a] - lo[a]) / (double)ncell[a];
        g.N *= g.nn[a];
    }
    long N = g.N;
    cplx *phi = malloc(sizeof(cplx) * (size_t)N), *psi = malloc(sizeof(cplx) * (size_t)(2 * N));
    cplx *phi2 = malloc(sizeof(cplx) * (size_t)N), *psi2 = malloc(sizeof(cplx) * (size_t)(2 * N));
    cplx *mixed = malloc(sizeof(cplx) * (size_t)N);
    int err = (!phi || !psi || !phi2 || !psi2 || !mixed) ? -1 : 0;
    for (int p = 0; p < 16 && !err; p++) {
        int pm = p / 4 + 1, pn = p % 4 + 1;
        for (long k = 0; k < N; k++) phi[k] = phi0[k];
        for (long k = 0; k < 2 * N; k++) psi[k] = psi0[k];
        for (long n = 0; n < steps; n++) {
            double t = t0 + (double)n * dt;
            step_cs(&g, params, nparams / 3, pm, pn, period, mixed_mode, bc, phi, psi, mixed, t,
                    dt, phi2, psi2);
            cplx *tp = phi; phi = phi2; phi2 = tp;
            cplx *tq = psi; psi = psi2; psi2 = tq;
        }
        cplx F = 0;
        if (lam) {
            for (long k = 0; k < N; k++)
                F += lam[k] * phi[k] + lam[N + k] * psi[k] + lam[2 * N + k] * psi[N + k];
        } else {
            for (long k = 0; k < N; k++) {
                cplx dd = heaviside_cs(phi[k], eps) - heaviside_cs(phi_target[k], eps);
                F += dd * dd;
            }
            F *= g.h[0] * g.h[1];
        }
        grad[p] = cimag(F) / H_CS;
        if (p == 0 && value) *value = creal(F);
    }
    free(phi); free(psi); free(phi2); free(psi2); free(mixed);
    return err;
}
