// Analytic velocity fields and their Jacobians on the device.
//
// Every field returns v(x) scaled by the stage time factor c, and the
// Jacobian in the "J form" J[i*D + j] = d v_i / d x_j (the transpose of the
// paper's deformation matrix of sec. 4). Positions arrive in FP64; the field
// is evaluated in the arithmetic type T.
#pragma once

#include "gals_internal.h"

namespace gals {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void sincospi_t(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_t(double x, double *s, double *c) { sincospi(x, s, c); }
__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }

// sin(k pi x), cos(k pi x) for k = 1..4 (index k-1): one sincospi, then the
// Chebyshev recurrence s_{k+1} = 2 cos(pi x) s_k - s_{k-1}.
template <typename T>
__device__ __forceinline__ void sincos_multiples(T x, T s[4], T c[4])
{
    sincospi_t(x, &s[0], &c[0]);
    const T t = T(2) * c[0];
    s[1] = t * s[0];
    c[1] = t * c[0] - T(1);
    s[2] = t * s[1] - s[0];
    c[2] = t * c[1] - c[0];
    s[3] = t * s[2] - s[1];
    c[3] = t * c[2] - c[1];
}

// The same multiples from sin(pi x), cos(pi x) already known.
template <typename T>
__device__ __forceinline__ void multiples_from(T s1, T c1, T s[4], T c[4])
{
    s[0] = s1;
    c[0] = c1;
    const T t = T(2) * c1;
    s[1] = t * s[0];
    c[1] = t * c[0] - T(1);
    s[2] = t * s[1] - s[0];
    c[2] = t * c[1] - c[0];
    s[3] = t * s[2] - s[1];
    c[3] = t * c[2] - c[1];
}

// sin(pi (x + d)), cos(pi (x + d)) from s1 = sin(pi x), c1 = cos(pi x) by
// angle addition, with sin(pi d) and cos(pi d) from their Taylor series: for
// |pi d| <= kShiftMax the dropped terms are below 3e-9 (sine) and 3e-11
// (cosine), far under FP32 rounding.
constexpr double kShiftMax = 0.05;
template <typename T>
__device__ __forceinline__ void shifted_sincos(T s1, T c1, T d, T &s, T &c)
{
    const T a = T(kPi) * d, a2 = a * a;
    const T sd = a * (T(1) - a2 * T(1.0 / 6.0));
    const T cd = T(1) - a2 * (T(0.5) - a2 * T(1.0 / 24.0));
    s = s1 * cd + c1 * sd;
    c = c1 * cd - s1 * sd;
}

// As shifted_sincos with longer series (to a^9 and a^10): for |pi d| <=
// kShiftMaxLong<T> the dropped terms are below 3e-19 in FP64 (0.1) and
// 4e-15 in FP32 (0.25), under either precision's rounding.
template <typename T>
constexpr double kShiftMaxLong = sizeof(T) == 8 ? 0.1 : 0.25;
template <typename T>
__device__ __forceinline__ void shifted_sincos_long(T s1, T c1, T d, T &s, T &c)
{
    const T a = T(kPi) * d, a2 = a * a;
    const T sd =
        a * (T(1) - a2 * (T(1.0 / 6) - a2 * (T(1.0 / 120) - a2 * (T(1.0 / 5040) -
                                                                   a2 * T(1.0 / 362880)))));
    const T cd =
        T(1) - a2 * (T(0.5) - a2 * (T(1.0 / 24) - a2 * (T(1.0 / 720) -
                                                         a2 * (T(1.0 / 40320) -
                                                               a2 * T(1.0 / 3628800)))));
    s = s1 * cd + c1 * sd;
    c = c1 * cd - s1 * sd;
}

template <typename T>
__device__ __forceinline__ T pick4(const T a[4], int i)
{
    // i is uniform across the wave (a kernel parameter)
    return i == 1 ? a[0] : i == 2 ? a[1] : i == 3 ? a[2] : a[3];
}

// v = (-s_y, s_x) from a stream function's derivatives.
template <typename T>
__device__ __forceinline__ void from_stream(T sx, T sy, T sxx, T sxy, T syy, T c, T *v, T *J)
{
    v[0] = -c * sy;
    v[1] = c * sx;
    J[0] = -c * sxy;  // du/dx
    J[1] = -c * syy;  // du/dy
    J[2] = c * sxx;   // dv/dx
    J[3] = c * sxy;   // dv/dy
}

template <typename T>
__device__ __forceinline__ void vel_affine(const Vel<T> &p, const double *x, int D, T c, T *v,
                                           T *J)
{
    T y[3];
    for (int j = 0; j < D; j++) y[j] = T(x[j] - p.c[j]);
    for (int i = 0; i < D; i++) {
        T s = p.b[i];
        for (int j = 0; j < D; j++) s += p.A[i * 3 + j] * y[j];
        v[i] = c * s;
        for (int j = 0; j < D; j++) J[i * D + j] = c * p.A[i * 3 + j];
    }
}

// Stream function s = sum_{m,n} S[m][n] sin((m+1) pi x) sin((n+1) pi y).
// Params is any parameter block with the table S. The y factors carry the
// wavenumbers (k_n cos, k_n^2 sin), so only S is read: 16 uniform values
// instead of 48 keep the kernels' scalar registers from spilling.
template <typename T, class Params>
__device__ __forceinline__ void stream_modes(const Params &p, const T *sx, const T *cx,
                                             const T *sy, const T *cy, T c, T *v, T *J)
{
    T fx = 0, fy = 0, fxx = 0, fyy = 0, fxy = 0;
    T qy[4], ry[4];
#pragma unroll
    for (int n = 0; n < 4; n++) {
        const T kn = T((n + 1) * kPi);
        qy[n] = kn * cy[n];
        ry[n] = T((n + 1) * (n + 1) * kPi * kPi) * sy[n];
    }
#pragma unroll
    for (int m = 0; m < 4; m++) {
        T P = 0, Q = 0, R = 0;
#pragma unroll
        for (int n = 0; n < 4; n++) {
            P += p.S[m][n] * sy[n];  // sum_n S sin(n pi y)
            Q += p.S[m][n] * qy[n];  // d/dy
            R += p.S[m][n] * ry[n];  // -d2/dy2
        }
        const T km = T((m + 1) * kPi);
        const T kc = km * cx[m];
        fx += kc * P;
        fy += sx[m] * Q;
        fxx -= km * km * sx[m] * P;
        fyy -= sx[m] * R;
        fxy += kc * Q;
    }
    from_stream(fx, fy, fxx, fxy, fyy, c, v, J);
}

// The same five sums from sin and cos of pi x and pi y at the point alone,
// contracted over m first: A_n = sum_m S[m][n] (m pi) cos(m pi x),
// B_n = sum_m S[m][n] sin(m pi x), C_n = sum_m S[m][n] (m pi)^2 sin(m pi x);
// then s_x = sum_n sin(n pi y) A_n, s_xy = sum_n (n pi) cos(n pi y) A_n,
// s_y = sum_n (n pi) cos(n pi y) B_n, s_yy = -sum_n (n pi)^2 sin(n pi y) B_n,
// s_xx = -sum_n sin(n pi y) C_n. The multiples of each angle come from the
// recurrence of multiples_from one at a time, so only the twelve partial sums
// and the recurrence are live (fewer registers than the sums over tabulated
// multiples; the same values up to the order of the additions).
template <typename T, class Params>
__device__ __forceinline__ void stream_modes_from(const Params &p, T s1x, T c1x, T s1y, T c1y,
                                                  T c, T *v, T *J)
{
    T A[4], B[4], C[4];
    {
        const T t = T(2) * c1x;
        T sm = s1x, cm = c1x, sp = T(0), cp = T(1);  // sin, cos of (m+1) pi x and m pi x
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const T km = T((m + 1) * kPi);
            const T kc = km * cm, ks = km * km * sm;
#pragma unroll
            for (int n = 0; n < 4; n++) {
                if (m == 0) {
                    A[n] = p.S[m][n] * kc;
                    B[n] = p.S[m][n] * sm;
                    C[n] = p.S[m][n] * ks;
                } else {
                    A[n] += p.S[m][n] * kc;
                    B[n] += p.S[m][n] * sm;
                    C[n] += p.S[m][n] * ks;
                }
            }
            const T sn = t * sm - sp, cn = t * cm - cp;
            sp = sm;
            cp = cm;
            sm = sn;
            cm = cn;
        }
    }
    T fx = 0, fy = 0, fxx = 0, fyy = 0, fxy = 0;
    const T t = T(2) * c1y;
    T sn = s1y, cn = c1y, sp = T(0), cp = T(1);
#pragma unroll
    for (int n = 0; n < 4; n++) {
        const T kn = T((n + 1) * kPi);
        const T qy = kn * cn, ry = kn * kn * sn;
        fx += sn * A[n];
        fxy += qy * A[n];
        fy += qy * B[n];
        fyy -= ry * B[n];
        fxx -= sn * C[n];
        const T s2 = t * sn - sp, c2 = t * cn - cp;
        sp = sn;
        cp = cn;
        sn = s2;
        cn = c2;
    }
    from_stream(fx, fy, fxx, fxy, fyy, c, v, J);
}

template <typename T, class Params>
__device__ __forceinline__ void vel_stream(const Params &p, const double *x, T c, T *v, T *J)
{
    T sx[4], cx[4], sy[4], cy[4];
    sincos_multiples(T(x[0]), sx, cx);
    sincos_multiples(T(x[1]), sy, cy);
    stream_modes(p, sx, cx, sy, cy, c, v, J);
}

// s = sin^2(pi x) sin^2(pi y) / pi.
template <typename T>
__device__ __forceinline__ void vel_vortex(const double *x, T c, T *v, T *J)
{
    T s1x, c1x, s1y, c1y;
    sincospi_t(T(x[0]), &s1x, &c1x);
    sincospi_t(T(x[1]), &s1y, &c1y);
    const T qx = s1x * s1x, qy = s1y * s1y;             // sin^2
    const T s2x = T(2) * s1x * c1x, s2y = T(2) * s1y * c1y;  // sin(2 pi .)
    const T c2x = T(1) - T(2) * qx, c2y = T(1) - T(2) * qy;  // cos(2 pi .)
    const T pi = T(kPi);
    from_stream(s2x * qy, qx * s2y, T(2) * pi * c2x * qy, pi * s2x * s2y, T(2) * pi * qx * c2y,
                c, v, J);
}

// v = exp(e.x) e, e = (sqrt 2, sqrt pi) / sqrt(2 + pi).
template <typename T>
__device__ __forceinline__ void vel_pseudo1d(const double *x, T c, T *v, T *J)
{
    // e = (sqrt 2, sqrt pi) / sqrt(2 + pi), a unit vector
    const T e0 = T(0.6236862429526107), e1 = T(0.7816747855416966);
    const T E = c * exp_t(T(e0 * T(x[0]) + e1 * T(x[1])));
    v[0] = E * e0;
    v[1] = E * e1;
    J[0] = E * e0 * e0;
    J[1] = E * e0 * e1;
    J[2] = J[1];
    J[3] = E * e1 * e1;
}

// One mode's terms of vecpot_modes added into the sums, one product per
// statement: each is a single multiply-add into its sum (a term pair written
// as one expression would cost a multiply, a multiply-add and an add).
template <typename T>
__device__ __forceinline__ void vecpot_accumulate(const T *q, T SSS, T SCS, T SSC, T SCC, T CSS,
                                                  T CCS, T CSC, T &vx, T &vy, T &vz, T &j00,
                                                  T &j01, T &j02, T &j10, T &j11, T &j12,
                                                  T &j20, T &j21, T &j22)
{
    vx += q[0] * SCS;
    vx -= q[1] * SSC;
    vy += q[2] * SSC;
    vy -= q[3] * CSS;
    vz += q[4] * CSS;
    vz -= q[5] * SCS;
    j00 += q[6] * CCS;
    j00 -= q[7] * CSC;
    j01 -= q[8] * SSS;
    j01 -= q[9] * SCC;
    j02 += q[10] * SCC;
    j02 += q[11] * SSS;
    j10 += q[12] * CSC;
    j10 += q[13] * SSS;
    j11 += q[14] * SCC;
    j11 -= q[6] * CCS;
    j12 -= q[15] * SSS;
    j12 -= q[16] * CSC;
    j20 -= q[17] * SSS;
    j20 -= q[18] * CCS;
    j21 += q[19] * CCS;
    j21 += q[20] * SSS;
    j22 += q[7] * CSC;
    j22 -= q[14] * SCC;
}

// v = curl A, A = sum_k a_k sin(l pi x) sin(m pi y) sin(n pi z). Per mode the
// seven products of sines (S) and cosines (C) in x, y, z are formed once and
// combined with precomputed coefficients a_c K_i (K_j) (K = wavenumber * pi):
//   vpc[0..5]  = az M, ay N, ax N, az L, ay L, ax M
//   vpc[6..20] = az LM, ay LN, az MM, ay MN, az MN, ay NN, ax LN, az LL,
//                ax MN, ax NN, az LN, ay LL, ax LM, ay LM, ax MM
template <typename T>
__device__ __forceinline__ void vecpot_modes(const Vel<T> &p, const T *sx, const T *cx,
                                             const T *sy, const T *cy, const T *sz, const T *cz,
                                             T c, T *v, T *J)
{
    T vx = 0, vy = 0, vz = 0;
    T j00 = 0, j01 = 0, j02 = 0, j10 = 0, j11 = 0, j12 = 0, j20 = 0, j21 = 0, j22 = 0;
    for (int k = 0; k < p.nvp; k++) {
        const T Sx = pick4(sx, p.vpi[k][0]), Cx = pick4(cx, p.vpi[k][0]);
        const T Sy = pick4(sy, p.vpi[k][1]), Cy = pick4(cy, p.vpi[k][1]);
        const T Sz = pick4(sz, p.vpi[k][2]), Cz = pick4(cz, p.vpi[k][2]);
        const T ss = Sy * Sz, cs = Cy * Sz, sc = Sy * Cz, cc = Cy * Cz;
        const T SSS = Sx * ss, SCS = Sx * cs, SSC = Sx * sc, SCC = Sx * cc;
        const T CSS = Cx * ss, CCS = Cx * cs, CSC = Cx * sc;
        vecpot_accumulate(p.vpc[k], SSS, SCS, SSC, SCC, CSS, CCS, CSC, vx, vy, vz, j00, j01,
                          j02, j10, j11, j12, j20, j21, j22);
    }
    v[0] = c * vx; v[1] = c * vy; v[2] = c * vz;
    J[0] = c * j00; J[1] = c * j01; J[2] = c * j02;
    J[3] = c * j10; J[4] = c * j11; J[5] = c * j12;
    J[6] = c * j20; J[7] = c * j21; J[8] = c * j22;
}

// The same sums with the multiples staged in LDS, value-major (row r of
// kBlock entries: 0-3 sin(l pi x), 4-7 cos(l pi x), then y, then z), read at
// each mode's uniform wavenumber rows: a wave-uniform row offset instead of a
// per-lane select of one of four registers.
template <typename T>
__device__ __forceinline__ void vecpot_modes_lds(const Vel<T> &p, const T (*tab)[kBlock],
                                                 int tid, T c, T *v, T *J)
{
    T vx = 0, vy = 0, vz = 0;
    T j00 = 0, j01 = 0, j02 = 0, j10 = 0, j11 = 0, j12 = 0, j20 = 0, j21 = 0, j22 = 0;
#pragma unroll 2
    for (int k = 0; k < p.nvp; k++) {
        const int l = p.vpi[k][0] - 1, m = p.vpi[k][1] - 1, n = p.vpi[k][2] - 1;
        const T Sx = tab[l][tid], Cx = tab[4 + l][tid];
        const T Sy = tab[8 + m][tid], Cy = tab[12 + m][tid];
        const T Sz = tab[16 + n][tid], Cz = tab[20 + n][tid];
        const T ss = Sy * Sz, cs = Cy * Sz, sc = Sy * Cz, cc = Cy * Cz;
        const T SSS = Sx * ss, SCS = Sx * cs, SSC = Sx * sc, SCC = Sx * cc;
        const T CSS = Cx * ss, CCS = Cx * cs, CSC = Cx * sc;
        vecpot_accumulate(p.vpc[k], SSS, SCS, SSC, SCC, CSS, CCS, CSC, vx, vy, vz, j00, j01,
                          j02, j10, j11, j12, j20, j21, j22);
    }
    v[0] = c * vx; v[1] = c * vy; v[2] = c * vz;
    J[0] = c * j00; J[1] = c * j01; J[2] = c * j02;
    J[3] = c * j10; J[4] = c * j11; J[5] = c * j12;
    J[6] = c * j20; J[7] = c * j21; J[8] = c * j22;
}

template <typename T>
__device__ __forceinline__ void vel_vecpot(const Vel<T> &p, const double *x, T c, T *v, T *J)
{
    T sx[4], cx[4], sy[4], cy[4], sz[4], cz[4];
    sincos_multiples(T(x[0]), sx, cx);
    sincos_multiples(T(x[1]), sy, cy);
    sincos_multiples(T(x[2]), sz, cz);
    vecpot_modes(p, sx, cx, sy, cy, sz, cz, c, v, J);
}

// Divergence-free reading of the 3D deformation field of sec. 6.2:
// u = 2 sin^2(pi x) sin(2 pi y) sin(2 pi z), v = -sin(2 pi x) sin^2(pi y) sin(2 pi z),
// w = -sin(2 pi x) sin(2 pi y) sin^2(pi z).
template <typename T>
__device__ __forceinline__ void vel_leveque(const double *x, T c, T *v, T *J)
{
    T s1[3], c1[3], q[3], s2[3], c2[3];
    for (int i = 0; i < 3; i++) {
        sincospi_t(T(x[i]), &s1[i], &c1[i]);
        q[i] = s1[i] * s1[i];
        s2[i] = T(2) * s1[i] * c1[i];
        c2[i] = T(1) - T(2) * q[i];
    }
    const T pi = T(kPi), tpi = T(2 * kPi);
    v[0] = c * T(2) * q[0] * s2[1] * s2[2];
    v[1] = -c * s2[0] * q[1] * s2[2];
    v[2] = -c * s2[0] * s2[1] * q[2];
    J[0] = c * tpi * s2[0] * s2[1] * s2[2];        // du/dx
    J[1] = c * T(2) * q[0] * tpi * c2[1] * s2[2];  // du/dy
    J[2] = c * T(2) * q[0] * s2[1] * tpi * c2[2];  // du/dz
    J[3] = -c * tpi * c2[0] * q[1] * s2[2];        // dv/dx
    J[4] = -c * s2[0] * pi * s2[1] * s2[2];        // dv/dy
    J[5] = -c * s2[0] * q[1] * tpi * c2[2];        // dv/dz
    J[6] = -c * tpi * c2[0] * s2[1] * q[2];        // dw/dx
    J[7] = -c * s2[0] * tpi * c2[1] * q[2];        // dw/dy
    J[8] = -c * s2[0] * s2[1] * pi * s2[2];        // dw/dz
}

// Dispatch on the compile-time field kind (D = space dimension).
template <typename T, int D, int KIND>
__device__ __forceinline__ void velocity(const Vel<T> &p, const double *x, T c, T *v, T *J)
{
    if constexpr (KIND == GALS_VEL_AFFINE) {
        vel_affine(p, x, D, c, v, J);
    } else if constexpr (KIND == GALS_VEL_STREAM_SIN) {
        vel_stream(p, x, c, v, J);
    } else if constexpr (KIND == GALS_VEL_VECPOT_SIN) {
        vel_vecpot(p, x, c, v, J);
    } else if constexpr (KIND == GALS_VEL_VORTEX) {
        vel_vortex(x, c, v, J);
    } else if constexpr (KIND == GALS_VEL_PSEUDO1D) {
        vel_pseudo1d(x, c, v, J);
    } else {
        vel_leveque(x, c, v, J);
    }
}

}  // namespace gals
