// rh_device.hpp -- device arithmetic of one WENO sweep for gfx950.
//
// Per cell: FP64 closed-form primitive recovery for the conformal equation of
// state (p = e/3), the physical flux along the sweep axis (Eq. (1) of
// Sikorski et al., arXiv:1604.03360), global Lax-Friedrichs splitting with
// alpha = 1, and finite-difference WENO5 / WENO7 reconstruction with Jiang-Shu
// smoothness indicators (Sec. 1.2).  Templated on the storage/stencil type T
// (float or double); the primitive recovery is always FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rh {

// Floors of the primitive recovery (they never modify the stored state).
constexpr double kEFloor = 1e-12;   // below this E the cell is treated as at rest
constexpr double kVDelta = 1e-12;   // |M|^2 is capped at (1 - kVDelta) E^2

struct HubbleBC {
    double t;          // stage time
    double t0, e0, n0; // u^mu = x^mu/tau, e = e0 (t0/tau)^4, n = n0 (t0/tau)^3
    double c0[3];      // centre of cell (0,0,0)
    double h[3];       // cell widths
};

// Analytic Hubble-like flow at (x, y, z, t), converted to conserved variables.
__device__ inline void hubble_conserved(const HubbleBC& hb, double x, double y, double z,
                                        double u[5]) {
    const double t = hb.t;
    const double tau = sqrt(t * t - (x * x + y * y + z * z));
    const double s = hb.t0 / tau;
    const double e = hb.e0 * s * s * s * s;
    const double n = hb.n0 * s * s * s;
    const double vx = x / t, vy = y / t, vz = z / t;
    const double p = e / 3.0;
    const double g2 = 1.0 / (1.0 - (vx * vx + vy * vy + vz * vz));
    const double w = e + p;
    u[0] = w * g2 - p;
    u[1] = w * g2 * vx;
    u[2] = w * g2 * vy;
    u[3] = w * g2 * vz;
    u[4] = n * sqrt(g2);
}

// Closed-form primitive recovery for p = e/3 (FP64):
//   M^2 = |M|^2, D = sqrt(4E^2 - 3M^2), v = 3M/(2E + D), p = (E^2 - M^2)/(E + D).
// Only the velocity along the sweep axis and p are needed for the flux.  Both
// divisions share one reciprocal of (2E + D)(E + D).
template <int DIR>
__device__ __forceinline__ void recover_vp(double E, double Mx, double My, double Mz,
                                           double& vd, double& p, unsigned& clamped) {
    double Md = DIR == 0 ? Mx : (DIR == 1 ? My : Mz);
    if (E < kEFloor) {
        vd = 0.0;
        p = (E > 0.0 ? E : 0.0) / 3.0;
        ++clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    const double E2 = E * E;
    const double cap = (1.0 - kVDelta) * E * E;
    if (M2 > cap) {
        Md *= sqrt(cap / M2);
        M2 = cap;
        ++clamped;
    }
    const double D = sqrt(4.0 * E2 - 3.0 * M2);
    const double a = 2.0 * E + D;
    const double b = E + D;
    const double r = 1.0 / (a * b);
    vd = 3.0 * b * r * Md;
    p = (E2 - M2) * a * r;
}

// Split fluxes f+- = (F_d(u) +- u) / 2 of one cell along axis DIR.
template <class T, int DIR>
__device__ __forceinline__ void split_flux(const T u[5], T fp[5], T fm[5], unsigned& clamped) {
    double vd, p;
    recover_vp<DIR>((double)u[0], (double)u[1], (double)u[2], (double)u[3], vd, p, clamped);
    const T v = (T)vd, P = (T)p, half = (T)0.5;
    T f[5];
    f[0] = u[1 + DIR];
    f[1] = u[1] * v + (DIR == 0 ? P : (T)0);
    f[2] = u[2] * v + (DIR == 1 ? P : (T)0);
    f[3] = u[3] * v + (DIR == 2 ? P : (T)0);
    f[4] = u[4] * v;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        fp[c] = half * (f[c] + u[c]);
        fm[c] = half * (f[c] - u[c]);
    }
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// WENO5: s0..s4 = f_{i-2..i+2}; left-biased value at i+1/2.
// Candidates q_k, indicators beta_k (Jiang-Shu), linear weights (1, 6, 3)/10.
// omega_k = alpha_k / sum(alpha), alpha_k = d_k / (eps + beta_k)^2, evaluated with
// one reciprocal as d_k prod_{j != k} g_j / sum_k(...), g_j = (eps + beta_j)^2.
template <class T>
__device__ __forceinline__ T weno5(T s0, T s1, T s2, T s3, T s4, T eps) {
    const T c13 = (T)(1.0 / 3.0), c16 = (T)(1.0 / 6.0), c56 = (T)(5.0 / 6.0);
    const T c76 = (T)(7.0 / 6.0), c116 = (T)(11.0 / 6.0), c1312 = (T)(13.0 / 12.0), q4 = (T)0.25;
    const T q0 = c13 * s0 - c76 * s1 + c116 * s2;
    const T q1 = -c16 * s1 + c56 * s2 + c13 * s3;
    const T q2 = c13 * s2 + c56 * s3 - c16 * s4;
    const T a0 = s0 - (T)2 * s1 + s2, b0 = s0 - (T)4 * s1 + (T)3 * s2;
    const T a1 = s1 - (T)2 * s2 + s3, b1 = s1 - s3;
    const T a2 = s2 - (T)2 * s3 + s4, b2 = (T)3 * s2 - (T)4 * s3 + s4;
    T g0 = eps + (c1312 * a0 * a0 + q4 * b0 * b0);
    T g1 = eps + (c1312 * a1 * a1 + q4 * b1 * b1);
    T g2 = eps + (c1312 * a2 * a2 + q4 * b2 * b2);
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
    const T w0 = (T)0.1 * (g1 * g2);
    const T w1 = (T)0.6 * (g0 * g2);
    const T w2 = (T)0.3 * (g0 * g1);
    return (w0 * q0 + w1 * q1 + w2 * q2) * fast_rcp(w0 + w1 + w2);
}

// WENO7 smoothness indicators beta_k = sum_{l=1..3} int_cell (d^l p_k/dx^l)^2 of
// the cubic candidate p_k = a0 + a1 x + a2 x^2 + a3 x^3 (x in cells):
// beta_k = a1^2 + a1 a3 / 2 + 13/3 a2^2 + 3129/80 a3^2, with a1..a3 difference
// combinations of the stencil (well conditioned in FP32 as well as FP64).
template <class T>
__device__ __forceinline__ void weno7_beta(T m3, T m2, T m1, T z0, T p1, T p2, T p3, T b[4]) {
    const T c24 = (T)(1.0 / 24.0), c6 = (T)(1.0 / 6.0), h = (T)0.5;
    const T k2 = (T)(13.0 / 3.0), k3 = (T)(3129.0 / 80.0);
    T a1[4], a2[4], a3[4];
    a1[0] = c24 * (-(T)7 * m3 + (T)33 * m2 - (T)69 * m1 + (T)43 * z0);
    a2[0] = h * (-m3 + (T)4 * m2 - (T)5 * m1 + (T)2 * z0);
    a3[0] = c6 * (-m3 + (T)3 * (m2 - m1) + z0);
    a1[1] = c24 * ((T)5 * m2 - (T)27 * m1 + (T)15 * z0 + (T)7 * p1);
    a2[1] = h * (m1 - (T)2 * z0 + p1);
    a3[1] = c6 * (-m2 + (T)3 * (m1 - z0) + p1);
    a1[2] = c24 * (-(T)7 * m1 - (T)15 * z0 + (T)27 * p1 - (T)5 * p2);
    a2[2] = a2[1];
    a3[2] = c6 * (-m1 + (T)3 * (z0 - p1) + p2);
    a1[3] = c24 * (-(T)43 * z0 + (T)69 * p1 - (T)33 * p2 + (T)7 * p3);
    a2[3] = h * ((T)2 * z0 - (T)5 * p1 + (T)4 * p2 - p3);
    a3[3] = c6 * (-z0 + (T)3 * (p1 - p2) + p3);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        b[k] = a1[k] * (a1[k] + h * a3[k]) + k2 * a2[k] * a2[k] + k3 * a3[k] * a3[k];
}

// WENO7: s0..s6 = f_{i-3..i+3}; linear weights (1, 12, 18, 4)/35.
template <class T>
__device__ __forceinline__ T weno7(T s0, T s1, T s2, T s3, T s4, T s5, T s6, T eps) {
    const T c12 = (T)(1.0 / 12.0);
    const T q0 = c12 * (-(T)3 * s0 + (T)13 * s1 - (T)23 * s2 + (T)25 * s3);
    const T q1 = c12 * (s1 - (T)5 * s2 + (T)13 * s3 + (T)3 * s4);
    const T q2 = c12 * (-s2 + (T)7 * s3 + (T)7 * s4 - s5);
    const T q3 = c12 * ((T)3 * s3 + (T)13 * s4 - (T)5 * s5 + s6);
    T b[4];
    weno7_beta(s0, s1, s2, s3, s4, s5, s6, b);
    T g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g[k] = eps + b[k];
        g[k] *= g[k];
    }
    T w0, w1, w2, w3;
    if constexpr (sizeof(T) == 8) {
        // FP64: one division via products of the other three squared terms
        const T g01 = g[0] * g[1], g23 = g[2] * g[3];
        w0 = (T)(1.0 / 35.0) * (g[1] * g23);
        w1 = (T)(12.0 / 35.0) * (g[0] * g23);
        w2 = (T)(18.0 / 35.0) * (g01 * g[3]);
        w3 = (T)(4.0 / 35.0) * (g01 * g[2]);
    } else {
        // FP32: products of three squared terms can overflow; use reciprocals
        w0 = (T)(1.0 / 35.0) * fast_rcp(g[0]);
        w1 = (T)(12.0 / 35.0) * fast_rcp(g[1]);
        w2 = (T)(18.0 / 35.0) * fast_rcp(g[2]);
        w3 = (T)(4.0 / 35.0) * fast_rcp(g[3]);
    }
    return (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) * fast_rcp(w0 + w1 + w2 + w3);
}

// Numerical flux at an interface from a window of 2R cells: w[j] holds the
// split fluxes of cell (i - R + 1 + j), j = 0 .. 2R-1, for the interface i+1/2.
// F = fhat+ (left-biased on f+) + fhat- (mirrored, right-biased on f-).
template <class T, int ORDER>
__device__ __forceinline__ T interface_flux(const T* wp, const T* wm, T eps) {
    if constexpr (ORDER == 5) {
        return weno5<T>(wp[0], wp[1], wp[2], wp[3], wp[4], eps)
             + weno5<T>(wm[5], wm[4], wm[3], wm[2], wm[1], eps);
    } else {
        return weno7<T>(wp[0], wp[1], wp[2], wp[3], wp[4], wp[5], wp[6], eps)
             + weno7<T>(wm[7], wm[6], wm[5], wm[4], wm[3], wm[2], wm[1], eps);
    }
}

}  // namespace rh
