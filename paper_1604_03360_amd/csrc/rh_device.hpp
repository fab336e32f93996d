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

// Last SSP-RK3 stage, u^n / 3 + 2/3 (u2 + dt L(u2)) with v = u2 + dt L(u2),
// evaluated in increment form u^n + 2/3 (v - u^n).  The plain form's rounded
// weights sum to 1 + 3e-8 in FP32, which scales every state (and the totals of
// a periodic grid) by that factor each step; in increment form the rounding of
// 2/3 multiplies only the increment and a uniform state stays exactly uniform.
template <class T>
__device__ __forceinline__ T rk3_last(T un, T v) { return un + (T)(2.0 / 3.0) * (v - un); }

// Reciprocals.  FP32: the hardware reciprocal (about 1 ulp).  FP64: the
// hardware estimate refined by two Newton-Raphson steps r <- r + r (1 - x r),
// which carries the estimate to full double precision for the normal-range
// arguments used here (weight sums, (2E + D)(E + D)).
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Square root of a positive normal double (no rescaling of tiny or huge
// arguments, no special cases): the hardware reciprocal square root y refined
// by one coupled Goldschmidt step on (g, h) ~ (sqrt(x), 1/(2 sqrt(x))) and two
// Newton corrections g <- g + (x - g^2) h.  Used for 4E^2 - 3M^2 >= E^2 with E
// above the floor, which is always in the normal range.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// Closed-form primitive recovery for p = e/3 (FP64):
//   M^2 = |M|^2, D = sqrt(4E^2 - 3M^2), v = 3M/(2E + D), p = (E^2 - M^2)/(E + D).
// Only the velocity along the sweep axis and p are needed for the flux.  Both
// divisions share one (Newton-refined) reciprocal of (2E + D)(E + D).
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
    const double D = sqrt_pos(4.0 * E2 - 3.0 * M2);
    const double a = 2.0 * E + D;
    const double b = E + D;
    const double r = fast_rcp(a * b);
    vd = 3.0 * b * r * Md;
    p = (E2 - M2) * a * r;
}

// The same recovery for two sweep axes at once: kap and the (capped) momenta
// such that v_d = kap * Ms_d for every axis d, with the arithmetic of
// recover_vp (so v_d is bitwise the value recover_vp<d> returns).
__device__ __forceinline__ void recover_kp(double E, double Mx, double My, double Mz, double& kap,
                                           double& Mxs, double& Mys, double& p, unsigned& clamped) {
    if (E < kEFloor) {
        kap = 0.0;
        Mxs = 0.0;
        Mys = 0.0;
        p = (E > 0.0 ? E : 0.0) / 3.0;
        ++clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    const double E2 = E * E;
    const double cap = (1.0 - kVDelta) * E * E;
    Mxs = Mx;
    Mys = My;
    if (M2 > cap) {
        const double sc = sqrt(cap / M2);
        Mxs *= sc;
        Mys *= sc;
        M2 = cap;
        ++clamped;
    }
    const double D = sqrt_pos(4.0 * E2 - 3.0 * M2);
    const double a = 2.0 * E + D;
    const double b = E + D;
    const double r = fast_rcp(a * b);
    kap = 3.0 * b * r;
    p = (E2 - M2) * a * r;
}

// The recovery for all three axes (v_d = kap * Ms_d), with the arithmetic of
// recover_vp, so each v_d is bitwise the value recover_vp<d> returns.
__device__ __forceinline__ void recover_kp3(double E, double Mx, double My, double Mz, double& kap,
                                            double& Mxs, double& Mys, double& Mzs, double& p,
                                            unsigned& clamped) {
    if (E < kEFloor) {
        kap = 0.0;
        Mxs = 0.0;
        Mys = 0.0;
        Mzs = 0.0;
        p = (E > 0.0 ? E : 0.0) / 3.0;
        ++clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    const double E2 = E * E;
    const double cap = (1.0 - kVDelta) * E * E;
    Mxs = Mx;
    Mys = My;
    Mzs = Mz;
    if (M2 > cap) {
        const double sc = sqrt(cap / M2);
        Mxs *= sc;
        Mys *= sc;
        Mzs *= sc;
        M2 = cap;
        ++clamped;
    }
    const double D = sqrt_pos(4.0 * E2 - 3.0 * M2);
    const double a = 2.0 * E + D;
    const double b = E + D;
    const double r = fast_rcp(a * b);
    kap = 3.0 * b * r;
    p = (E2 - M2) * a * r;
}

// Ideal-gas equation of state (unit rest mass per unit charge):
// p = (gamma - 1)(e - n), cut off at zero pressure; c_s^2 = gamma p / (e + p).
__device__ __forceinline__ double ideal_p(double gm1, double e, double n) {
    const double p = gm1 * (e - n);
    return p > 0.0 ? p : 0.0;
}

// Ideal-gas primitive recovery (FP64), in the form of recover_kp3: v_d =
// kap * Ms_d, with e and p.  The speed v along M solves
//   g(v) = v (E + p(E - |M| v, N sqrt(1 - v^2))) - |M| = 0,
// g increasing on [0, 1) (dg/dv >= E - (gamma - 1)|M| > 0 for gamma <= 2), with
// the root inside [|M| / (gamma E), |M| / E] because 0 <= p <= (gamma - 1) E.
// Newton steps, kept inside the shrinking bracket (a step leaving it is
// replaced by bisection), stop at a relative step of at most 1e-15.  They start from
// the root for the same fluid without rest mass (n = 0, p = (gamma - 1) e), the
// smaller root of (gamma - 1)|M| v^2 - gamma E v + |M| = 0, which lies in the
// bracket and is exact when N = 0.
// Floors as the closed form: E below the floor -> at rest; |M|^2 capped.
__device__ inline void recover_ideal(double E, double Mx, double My, double Mz, double N, double gm1,
                                     double& kap, double& Mxs, double& Mys, double& Mzs, double& p,
                                     double& e, unsigned& clamped) {
    if (E < kEFloor) {
        kap = 0.0;
        Mxs = Mys = Mzs = 0.0;
        e = E > 0.0 ? E : 0.0;
        p = ideal_p(gm1, e, N);
        ++clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    const double cap = (1.0 - kVDelta) * E * E;
    Mxs = Mx;
    Mys = My;
    Mzs = Mz;
    if (M2 > cap) {
        const double sc = sqrt(cap / M2);
        Mxs *= sc;
        Mys *= sc;
        Mzs *= sc;
        M2 = cap;
        ++clamped;
    }
    if (!(M2 > 0.0)) {
        kap = 0.0;
        e = E;
        p = ideal_p(gm1, E, N);
        return;
    }
    const double M = sqrt(M2);
    const double ge = (gm1 + 1.0) * E;
    double lo = M / ge, hi = M / E;
    // 2|M| / (gamma E + sqrt(gamma^2 E^2 - 4 (gamma - 1) M^2)); the radicand is at
    // least (2 - gamma)^2 E^2 >= 0
    const double rad = ge * ge - 4.0 * gm1 * M2;
    double v = 2.0 * M / (ge + sqrt(rad > 0.0 ? rad : 0.0));
    v = v < lo ? lo : (v > hi ? hi : v);
#pragma unroll 1
    for (int it = 0; it < 80; ++it) {
        const double w = sqrt_pos(1.0 - v * v);
        const double pr = gm1 * ((E - M * v) - N * w);
        double g, dg;
        if (pr > 0.0) {
            g = v * (E + pr) - M;
            dg = (E + pr) + v * gm1 * (N * v * fast_rcp(w) - M);
        } else {
            g = v * E - M;
            dg = E;
        }
        if (g == 0.0) break;
        if (g > 0.0) hi = v;
        else lo = v;
        const double vn = v - g * fast_rcp(dg);
        // converged: tested before the bracket, since a step below the rounding
        // of v lands on v itself, the end of the bracket just moved there
        if (fabs(vn - v) <= 1e-15 * v) {
            v = vn;
            break;
        }
        v = vn > lo && vn < hi ? vn : 0.5 * (lo + hi);
    }
    kap = v / M;
    e = E - M * v;
    p = ideal_p(gm1, e, N * sqrt(1.0 - v * v));
}

// Largest characteristic speed along an axis, from the velocity along it, v^2
// and c_s^2: the acoustic eigenvalues
//   (v_d (1 - c^2) +- c sqrt((1 - v^2)(1 - v^2 c^2 - v_d^2 (1 - c^2)))) / (1 - v^2 c^2)
// bracket v_d, so the larger magnitude of the two bounds every wave.
__device__ __forceinline__ double max_char_speed(double vd, double v2, double cs2) {
    const double disc = cs2 * (1.0 - v2) * (1.0 - v2 * cs2 - vd * vd * (1.0 - cs2));
    const double root = sqrt(disc > 0.0 ? disc : 0.0);
    const double a = vd * (1.0 - cs2);
    return (fabs(a) + root) / (1.0 - v2 * cs2);
}

// Split fluxes f+- = (F_d(u) +- u) / 2 of one cell along axis DIR, given the
// velocity along DIR and the pressure, returned doubled (F_d +- u).
//
// The forward sweeps work with twice the split fluxes, F +- u: the WENO
// reconstruction is homogeneous of degree one when eps scales with the square
// of the data, so reconstructing F +- u with 4 eps gives exactly (all scalings
// are powers of two) twice the face flux, and the factor 1/2 is folded into
// the flux difference.
template <class T, int DIR>
__device__ __forceinline__ void split_flux_vp(const T u[5], T v, T P, T fp[5], T fm[5]) {
    T f[5];
    f[0] = u[1 + DIR];
    f[1] = u[1] * v + (DIR == 0 ? P : (T)0);
    f[2] = u[2] * v + (DIR == 1 ? P : (T)0);
    f[3] = u[3] * v + (DIR == 2 ? P : (T)0);
    f[4] = u[4] * v;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        fp[c] = f[c] + u[c];
        fm[c] = f[c] - u[c];
    }
}

template <class T, int DIR>
__device__ __forceinline__ void split_flux(const T u[5], T fp[5], T fm[5], unsigned& clamped) {
    double vd, p;
    recover_vp<DIR>((double)u[0], (double)u[1], (double)u[2], (double)u[3], vd, p, clamped);
    split_flux_vp<T, DIR>(u, (T)vd, (T)p, fp, fm);
}

// WENO5: s0..s4 = f_{i-2..i+2}; left-biased value at i+1/2 (Jiang-Shu).
// Written in the differences E_j = s_j - s_{j-1} about the centre c = s2:
//   q_k - c:  (-E1/3 + 5 E2/6), (E2/6 + E3/3), (2 E3/3 - E4/6)
//   beta_k = 13/12 A_k^2 + 1/4 B_k^2 with A = (E2-E1, E3-E2, E4-E3),
//            B = (3E2-E1, E2+E3, E4-3E3).
// Expanded in the E's, 4 beta_k = 16/3 h_k with
//   h0 = E1^2 - 11/4 E1 E2 + 5/2 E2^2,  h1 = E2^2 - 5/4 E2 E3 + E3^2,
//   h2 = E4^2 - 11/4 E3 E4 + 5/2 E3^2
// (positive definite), so g_k = (h_k + 3/16 (4 eps))^2 is (3/16)^2 (4 eps +
// 4 beta_k)^2 and the common factor cancels in the weights
// alpha_k = d_k / (eps + beta_k)^2, d = (1, 6, 3)/10, which are evaluated with
// one reciprocal and carried as 10 w = (g1 g2, 6 g0 g2, 3 g0 g1), the factors 6
// and 3 folded into the candidates of the numerator:
//   num = g2 (g1 dq0 + g0 (6 dq1)) + g0 g1 (3 dq2),  den = g2 (g1 + 6 g0) + 3 g0 g1.
template <class T>
__device__ __forceinline__ T weno5(T s0, T s1, T s2, T s3, T s4, T eps4) {
    const T E1 = s1 - s0, E2 = s2 - s1, E3 = s3 - s2, E4 = s4 - s3;
    const T dq0 = (T)(5.0 / 6.0) * E2 - (T)(1.0 / 3.0) * E1;   // q0 - c
    const T dq1s = E2 + (T)2 * E3;                              // 6 (q1 - c)
    const T dq2s = (T)2 * E3 - (T)0.5 * E4;                     // 3 (q2 - c)
    const T e = (T)0.1875 * eps4;
    T g0 = E1 * (E1 - (T)2.75 * E2) + ((T)2.5 * E2 * E2 + e);
    T g1 = E2 * (E2 - (T)1.25 * E3) + (E3 * E3 + e);
    T g2 = E4 * (E4 - (T)2.75 * E3) + ((T)2.5 * E3 * E3 + e);
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
    const T a = g0 * g1;
    const T num = g2 * (g1 * dq0 + g0 * dq1s) + a * dq2s;
    const T den = g2 * ((T)6 * g0 + g1) + (T)3 * a;
    return s2 + num * fast_rcp(den);
}

// WENO7: s0..s6 = f_{i-3..i+3}; linear weights (1, 12, 18, 4)/35.  With
// D_j = s_j - s_{j-1} and c = s3, the candidates are c + dq_k and the cubic
// candidate p_k = a0 + a1 x + a2 x^2 + a3 x^3 gives
// beta_k = a1^2 + a1 a3 / 2 + 13/3 a2^2 + 3129/80 a3^2 (the sum of the cell
// integrals of its squared first three derivatives).  a2 and a3 are carried
// pre-scaled by sqrt(13/3) and sqrt(3129/80).
template <class T>
__device__ __forceinline__ T weno7(T s0, T s1, T s2, T s3, T s4, T s5, T s6, T eps) {
    const T D1 = s1 - s0, D2 = s2 - s1, D3 = s3 - s2, D4 = s4 - s3, D5 = s5 - s4, D6 = s6 - s5;
    const T dq0 = (T)0.25 * D1 - (T)(5.0 / 6.0) * D2 + (T)(13.0 / 12.0) * D3;
    const T dq1 = (T)(1.0 / 3.0) * D3 - (T)(1.0 / 12.0) * D2 + (T)0.25 * D4;
    const T dq2 = (T)(1.0 / 12.0) * (D3 - D5) + (T)0.5 * D4;
    const T dq3 = (T)0.75 * D4 - (T)(1.0 / 3.0) * D5 + (T)(1.0 / 12.0) * D6;
    const T r2 = (T)2.0816659994661326;    // sqrt(13/3)
    const T kk = (T)(0.5 / 6.253998720818545);   // 1 / (2 sqrt(3129/80))
    const T a1_0 = (T)(7.0 / 24.0) * D1 - (T)(13.0 / 12.0) * D2 + (T)(43.0 / 24.0) * D3;
    const T a1_1 = (T)(11.0 / 12.0) * D3 - (T)(5.0 / 24.0) * D2 + (T)(7.0 / 24.0) * D4;
    const T a1_2 = (T)(7.0 / 24.0) * D3 + (T)(11.0 / 12.0) * D4 - (T)(5.0 / 24.0) * D5;
    const T a1_3 = (T)(43.0 / 24.0) * D4 - (T)(13.0 / 12.0) * D5 + (T)(7.0 / 24.0) * D6;
    const T a2_0 = (T)(0.5 * 2.0816659994661326) * D1 - (T)(1.5 * 2.0816659994661326) * D2 + r2 * D3;
    const T a2_1 = (T)(0.5 * 2.0816659994661326) * (D4 - D3);
    const T a2_3 = (T)(1.5 * 2.0816659994661326) * D5 - r2 * D4 - (T)(0.5 * 2.0816659994661326) * D6;
    const T c6 = (T)(6.253998720818545 / 6.0);
    const T a3_0 = c6 * ((D1 + D3) - (T)2 * D2);
    const T a3_1 = c6 * ((D2 + D4) - (T)2 * D3);
    const T a3_2 = c6 * ((D3 + D5) - (T)2 * D4);
    const T a3_3 = c6 * ((D4 + D6) - (T)2 * D5);
    T g0, g1, g2, g3;
    if constexpr (sizeof(T) == 4) {
        // FP32: 240 beta_k as quadratic forms in its three differences
        // (x, y, z) = (D_{k+1}, D_{k+2}, D_{k+3}); the factor 240 (on eps too)
        // cancels in the weights.  Fewer operations than the derivative form.
        // Rounding in the terms grows by at most the ratio of the summed
        // absolute coefficients to 240 (68 for the outer stencils): a few 1e-6
        // relative in beta at FP32, far below the parity bar.
        const T e = (T)240 * eps;
        auto q = [e](T x, T y, T z, T cxx, T cxy, T cxz, T cyy, T cyz, T czz) {
            return x * (cxx * x + cxy * y + cxz * z) + (y * (cyy * y + cyz * z) + (czz * z * z + e));
        };
        g0 = q(D1, D2, D3, (T)547, (T)-2788, (T)1854, (T)3708, (T)-5188, (T)2107);
        g1 = q(D2, D3, D4, (T)267, (T)-1108, (T)494, (T)1468, (T)-1428, (T)547);
        g2 = q(D3, D4, D5, (T)547, (T)-1428, (T)494, (T)1468, (T)-1108, (T)267);
        g3 = q(D4, D5, D6, (T)2107, (T)-5188, (T)1854, (T)3708, (T)-2788, (T)547);
    } else {
        // FP64: the sum-of-squares form (no cancellation)
        g0 = a1_0 * (a1_0 + kk * a3_0) + (a2_0 * a2_0 + (a3_0 * a3_0 + eps));
        g1 = a1_1 * (a1_1 + kk * a3_1) + (a2_1 * a2_1 + (a3_1 * a3_1 + eps));
        g2 = a1_2 * (a1_2 + kk * a3_2) + (a2_1 * a2_1 + (a3_2 * a3_2 + eps));
        g3 = a1_3 * (a1_3 + kk * a3_3) + (a2_3 * a2_3 + (a3_3 * a3_3 + eps));
    }
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
    g3 *= g3;
    if constexpr (sizeof(T) == 8) {
        // FP64: one reciprocal via products of the other three squared terms
        const T g01 = g0 * g1, g23 = g2 * g3;
        const T w0 = (T)(1.0 / 35.0) * (g1 * g23);
        const T w1 = (T)(12.0 / 35.0) * (g0 * g23);
        const T w2 = (T)(18.0 / 35.0) * (g01 * g3);
        const T w3 = (T)(4.0 / 35.0) * (g01 * g2);
        const T num = (w0 * dq0 + w1 * dq1) + (w2 * dq2 + w3 * dq3);
        const T den = (w0 + w1) + (w2 + w3);
        return s3 + num * fast_rcp(den);
    } else {
        // FP32: products of three squared terms can overflow, so one reciprocal
        // per weight; the linear weights 35 d = (1, 12, 18, 4) are folded into
        // the candidates (12 dq1 = 4 D3 - D2 + 3 D4, 18 dq2 = 3/2 (D3 - D5) + 9 D4,
        // 4 dq3 = 3 D4 - 4/3 D5 + 1/3 D6) and the weight sum, the 1/35 cancels
        const T r0 = fast_rcp(g0), r1 = fast_rcp(g1), r2 = fast_rcp(g2), r3 = fast_rcp(g3);
        const T q1 = ((T)4 * D3 - D2) + (T)3 * D4;
        const T q2 = (T)1.5 * (D3 - D5) + (T)9 * D4;
        const T q3 = ((T)3 * D4 - (T)(4.0 / 3.0) * D5) + (T)(1.0 / 3.0) * D6;
        const T num = (r0 * dq0 + r1 * q1) + (r2 * q2 + r3 * q3);
        const T den = (r0 + (T)12 * r1) + ((T)18 * r2 + (T)4 * r3);
        return s3 + num * fast_rcp(den);
    }
}

}  // namespace rh
