// rh_adjoint.hpp -- device arithmetic of the hand-written adjoint of L.
//
// With w a field of weights, sum_i w_i . L_i (Eq. (2) of Sikorski et al.,
// arXiv:1604.03360) equals the sum over faces of Fhat(i+1/2) . g(i+1/2) with
// g = (w_{i+1} - w_i) / h; its gradient with respect to the state is therefore
// built face by face: the gradient of each WENO reconstruction (Sec. 1.2) with
// respect to its stencil, scaled by g, is accumulated on the stencil cells, and
// each cell's accumulated split-flux adjoints a+- are mapped through the split
// f+- = (F(u) +- u)/2 and the flux Jacobian of F, whose primitive-recovery part
// comes from the per-cell pack below.
#pragma once
#include "rh_device.hpp"

namespace rh {

// Gradient of weno5 (difference form, see weno5) times gbar, added to out[0..4].
// With omega_k the nonlinear weights, dq_k the candidates minus the centre and
// G_k = 13/3 A_k^2 + B_k^2 + 4 eps:
//   d fhat / d s = e_2 + sum_k omega_k grad(dq_k)
//                  - 2 sum_k omega_k (dq_k - fhat + s2) / G_k grad(G_k),
//   grad(G_k) = 26/3 A_k grad(A_k) + 2 B_k grad(B_k).
template <class T>
__device__ __forceinline__ void weno5_grad_acc(T s0, T s1, T s2, T s3, T s4, T eps4, T gbar,
                                               T& o0, T& o1, T& o2, T& o3, T& o4) {
    const T E1 = s1 - s0, E2 = s2 - s1, E3 = s3 - s2, E4 = s4 - s3;
    const T dq0 = (T)(5.0 / 6.0) * E2 - (T)(1.0 / 3.0) * E1;
    const T dq1 = (T)(1.0 / 6.0) * E2 + (T)(1.0 / 3.0) * E3;
    const T dq2 = (T)(2.0 / 3.0) * E3 - (T)(1.0 / 6.0) * E4;
    const T A0 = E2 - E1, A1 = E3 - E2, A2 = E4 - E3;
    const T B0 = (T)3 * E2 - E1, B1 = E2 + E3, B2 = E4 - (T)3 * E3;
    const T c133 = (T)(13.0 / 3.0);
    const T G0 = (c133 * A0) * A0 + (B0 * B0 + eps4);
    const T G1 = (c133 * A1) * A1 + (B1 * B1 + eps4);
    const T G2 = (c133 * A2) * A2 + (B2 * B2 + eps4);
    const T g0 = G0 * G0, g1 = G1 * G1, g2 = G2 * G2;
    const T w0 = (T)0.1 * (g1 * g2), w1 = (T)0.6 * (g0 * g2), w2 = (T)0.3 * (g0 * g1);
    const T rs = fast_rcp(w0 + w1 + w2);
    const T om0 = w0 * rs, om1 = w1 * rs, om2 = w2 * rs;
    const T fd = om0 * dq0 + om1 * dq1 + om2 * dq2;
    const T c0 = (T)(-2.0) * om0 * (dq0 - fd) * fast_rcp(G0);
    const T c1 = (T)(-2.0) * om1 * (dq1 - fd) * fast_rcp(G1);
    const T c2 = (T)(-2.0) * om2 * (dq2 - fd) * fast_rcp(G2);
    const T pA0 = (T)(26.0 / 3.0) * c0 * A0, pA1 = (T)(26.0 / 3.0) * c1 * A1, pA2 = (T)(26.0 / 3.0) * c2 * A2;
    const T pB0 = (T)2 * c0 * B0, pB1 = (T)2 * c1 * B1, pB2 = (T)2 * c2 * B2;
    // grad(dq): (1/3, -7/6, 5/6, 0, 0), (0, -1/6, -1/6, 1/3, 0), (0, 0, -2/3, 5/6, -1/6)
    // grad(A):  (1, -2, 1, 0, 0), (0, 1, -2, 1, 0), (0, 0, 1, -2, 1)
    // grad(B):  (1, -4, 3, 0, 0), (0, -1, 0, 1, 0), (0, 0, 3, -4, 1)
    const T d0 = (T)(1.0 / 3.0) * om0 + pA0 + pB0;
    const T d1 = (T)(-7.0 / 6.0) * om0 - (T)(1.0 / 6.0) * om1 - (T)2 * pA0 + pA1 - (T)4 * pB0 - pB1;
    const T d2 = (T)1 + (T)(5.0 / 6.0) * om0 - (T)(1.0 / 6.0) * om1 - (T)(2.0 / 3.0) * om2 + pA0
               - (T)2 * pA1 + pA2 + (T)3 * pB0 + (T)3 * pB2;
    const T d3 = (T)(1.0 / 3.0) * om1 + (T)(5.0 / 6.0) * om2 + pA1 - (T)2 * pA2 + pB1 - (T)4 * pB2;
    const T d4 = (T)(-1.0 / 6.0) * om2 + pA2 + pB2;
    o0 += gbar * d0;
    o1 += gbar * d1;
    o2 += gbar * d2;
    o3 += gbar * d3;
    o4 += gbar * d4;
}

// The same gradient written in the first differences E_j (the smoothness
// indicators in the expanded form h_k of weno5): fewer instructions, more live
// values; used where registers are plentiful (the LDS-tiled x adjoint).  With omega_k the
// nonlinear weights, dq_k the candidates minus the centre and G_k = h_k + e:
//   d fhat / d E_j = sum_k omega_k d dq_k/d E_j + sum_k c_k d h_k/d E_j,
//   c_k = -2 omega_k (dq_k - sum_m omega_m dq_m) / G_k,
// and d/d s follows from E_j = s_j - s_{j-1} (plus 1 on the centre s2).
template <class T>
__device__ __forceinline__ void weno5_grad_acc_e(T s0, T s1, T s2, T s3, T s4, T eps4, T gbar,
                                                 T& o0, T& o1, T& o2, T& o3, T& o4) {
    const T E1 = s1 - s0, E2 = s2 - s1, E3 = s3 - s2, E4 = s4 - s3;
    const T dq0 = (T)(5.0 / 6.0) * E2 - (T)(1.0 / 3.0) * E1;
    const T dq1 = (T)(1.0 / 6.0) * E2 + (T)(1.0 / 3.0) * E3;
    const T dq2 = (T)(2.0 / 3.0) * E3 - (T)(1.0 / 6.0) * E4;
    const T e = (T)0.1875 * eps4;
    const T t0 = E1 - (T)2.75 * E2, t1 = E2 - (T)1.25 * E3, t2 = E4 - (T)2.75 * E3;
    const T u0 = (T)2.5 * E2, u2 = (T)2.5 * E3;
    const T G0 = E1 * t0 + (u0 * E2 + e);
    const T G1 = E2 * t1 + (E3 * E3 + e);
    const T G2 = E4 * t2 + (u2 * E3 + e);
    const T g0 = G0 * G0, g1 = G1 * G1, g2 = G2 * G2;
    // 10 w = (g1 g2, 6 g0 g2, 3 g0 g1)
    const T p12 = g1 * g2, p02 = g0 * g2, p01 = g0 * g1;
    const T rs = fast_rcp((T)3 * p01 + ((T)6 * p02 + p12));
    const T om0 = p12 * rs, om1 = p02 * ((T)6 * rs), om2 = p01 * ((T)3 * rs);
    const T fd = om0 * dq0 + om1 * dq1 + om2 * dq2;
    const T gb2 = (T)(-2.0) * gbar;
    const T c0 = (gb2 * om0) * (dq0 - fd) * fast_rcp(G0);
    const T c1 = (gb2 * om1) * (dq1 - fd) * fast_rcp(G1);
    const T c2 = (gb2 * om2) * (dq2 - fd) * fast_rcp(G2);
    const T wb0 = gbar * om0, wb1 = gbar * om1, wb2 = gbar * om2;
    // d h_k / d E_j
    const T h0_1 = t0 + E1, h0_2 = (u0 + u0) - (T)2.75 * E1;
    const T h1_2 = t1 + E2, h1_3 = (E3 + E3) - (T)1.25 * E2;
    const T h2_3 = (u2 + u2) - (T)2.75 * E4, h2_4 = t2 + E4;
    const T gE1 = c0 * h0_1 - (T)(1.0 / 3.0) * wb0;
    const T gE2 = (c0 * h0_2 + c1 * h1_2) + ((T)(5.0 / 6.0) * wb0 + (T)(1.0 / 6.0) * wb1);
    const T gE3 = (c1 * h1_3 + c2 * h2_3) + ((T)(1.0 / 3.0) * wb1 + (T)(2.0 / 3.0) * wb2);
    const T gE4 = c2 * h2_4 - (T)(1.0 / 6.0) * wb2;
    o0 -= gE1;
    o1 += gE1 - gE2;
    o2 += gbar + (gE2 - gE3);
    o3 += gE3 - gE4;
    o4 += gE4;
}

// Gradient of weno7 (see weno7) times gbar, added to o[0..6].  With
// G_k = a1 (a1 + kk a3h) + a2h^2 + a3h^2 + eps (a2h = r2 a2, a3h = r3 a3,
// kk = 1/(2 r3)):
//   grad(G_k) = (2 a1 + kk a3h) grad(a1) + 2 r2 a2h grad(a2) + (a1/2 + 2 r3 a3h) grad(a3).
template <class T>
__device__ __forceinline__ void weno7_grad_acc(const T s[7], T eps, T gbar, T o[7]) {
    const T D1 = s[1] - s[0], D2 = s[2] - s[1], D3 = s[3] - s[2], D4 = s[4] - s[3];
    const T D5 = s[5] - s[4], D6 = s[6] - s[5];
    T dq[4], a1[4], a2h[4], a3h[4];
    dq[0] = (T)0.25 * D1 - (T)(5.0 / 6.0) * D2 + (T)(13.0 / 12.0) * D3;
    dq[1] = (T)(1.0 / 3.0) * D3 - (T)(1.0 / 12.0) * D2 + (T)0.25 * D4;
    dq[2] = (T)(1.0 / 12.0) * (D3 - D5) + (T)0.5 * D4;
    dq[3] = (T)0.75 * D4 - (T)(1.0 / 3.0) * D5 + (T)(1.0 / 12.0) * D6;
    const T r2 = (T)2.0816659994661326, r3 = (T)6.253998720818545, kk = (T)(0.5 / 6.253998720818545);
    a1[0] = (T)(7.0 / 24.0) * D1 - (T)(13.0 / 12.0) * D2 + (T)(43.0 / 24.0) * D3;
    a1[1] = (T)(11.0 / 12.0) * D3 - (T)(5.0 / 24.0) * D2 + (T)(7.0 / 24.0) * D4;
    a1[2] = (T)(7.0 / 24.0) * D3 + (T)(11.0 / 12.0) * D4 - (T)(5.0 / 24.0) * D5;
    a1[3] = (T)(43.0 / 24.0) * D4 - (T)(13.0 / 12.0) * D5 + (T)(7.0 / 24.0) * D6;
    a2h[0] = r2 * ((T)0.5 * D1 - (T)1.5 * D2 + D3);
    a2h[1] = r2 * ((T)0.5 * (D4 - D3));
    a2h[2] = a2h[1];
    a2h[3] = r2 * ((T)1.5 * D5 - D4 - (T)0.5 * D6);
    a3h[0] = (r3 / (T)6) * ((D1 + D3) - (T)2 * D2);
    a3h[1] = (r3 / (T)6) * ((D2 + D4) - (T)2 * D3);
    a3h[2] = (r3 / (T)6) * ((D3 + D5) - (T)2 * D4);
    a3h[3] = (r3 / (T)6) * ((D4 + D6) - (T)2 * D5);
    T G[4], al[4];
    T sum = (T)0;
    const T dk[4] = {(T)(1.0 / 35.0), (T)(12.0 / 35.0), (T)(18.0 / 35.0), (T)(4.0 / 35.0)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        G[k] = a1[k] * (a1[k] + kk * a3h[k]) + (a2h[k] * a2h[k] + (a3h[k] * a3h[k] + eps));
        const T rg = fast_rcp(G[k]);
        al[k] = dk[k] * rg * rg;
        sum += al[k];
    }
    const T rs = fast_rcp(sum);
    T om[4], fd = (T)0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        om[k] = al[k] * rs;
        fd += om[k] * dq[k];
    }
    // gradient tables in s0..s6 (a2, a3 unscaled)
    const T gdq[4][7] = {{(T)(-0.25), (T)(13.0 / 12), (T)(-23.0 / 12), (T)(13.0 / 12), 0, 0, 0},
                         {0, (T)(1.0 / 12), (T)(-5.0 / 12), (T)(1.0 / 12), (T)0.25, 0, 0},
                         {0, 0, (T)(-1.0 / 12), (T)(-5.0 / 12), (T)(7.0 / 12), (T)(-1.0 / 12), 0},
                         {0, 0, 0, (T)(-0.75), (T)(13.0 / 12), (T)(-5.0 / 12), (T)(1.0 / 12)}};
    const T ga1[4][7] = {{(T)(-7.0 / 24), (T)(11.0 / 8), (T)(-23.0 / 8), (T)(43.0 / 24), 0, 0, 0},
                         {0, (T)(5.0 / 24), (T)(-9.0 / 8), (T)(5.0 / 8), (T)(7.0 / 24), 0, 0},
                         {0, 0, (T)(-7.0 / 24), (T)(-5.0 / 8), (T)(9.0 / 8), (T)(-5.0 / 24), 0},
                         {0, 0, 0, (T)(-43.0 / 24), (T)(23.0 / 8), (T)(-11.0 / 8), (T)(7.0 / 24)}};
    const T ga2[4][7] = {{(T)(-0.5), (T)2, (T)(-2.5), (T)1, 0, 0, 0},
                         {0, 0, (T)0.5, (T)(-1), (T)0.5, 0, 0},
                         {0, 0, (T)0.5, (T)(-1), (T)0.5, 0, 0},
                         {0, 0, 0, (T)1, (T)(-2.5), (T)2, (T)(-0.5)}};
    const T ga3[4][7] = {{(T)(-1.0 / 6), (T)0.5, (T)(-0.5), (T)(1.0 / 6), 0, 0, 0},
                         {0, (T)(-1.0 / 6), (T)0.5, (T)(-0.5), (T)(1.0 / 6), 0, 0},
                         {0, 0, (T)(-1.0 / 6), (T)0.5, (T)(-0.5), (T)(1.0 / 6), 0},
                         {0, 0, 0, (T)(-1.0 / 6), (T)0.5, (T)(-0.5), (T)(1.0 / 6)}};
    T d[7] = {0, 0, 0, (T)1, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T c = (T)(-2.0) * om[k] * (dq[k] - fd) * fast_rcp(G[k]);
        const T p1 = c * ((T)2 * a1[k] + kk * a3h[k]);
        const T p2 = c * ((T)2 * r2 * a2h[k]);
        const T p3 = c * ((T)0.5 * a1[k] + (T)2 * r3 * a3h[k]);
#pragma unroll
        for (int j = 0; j < 7; ++j) d[j] += om[k] * gdq[k][j] + p1 * ga1[k][j] + p2 * ga2[k][j] + p3 * ga3[k][j];
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) o[j] += gbar * d[j];
}

// Primitive recovery written as v = kappa(E, M^2) M and p = P(E, M^2), with the
// four partial derivatives of kappa and P (FP64).  This covers the floors: below
// the energy floor kappa = 0 and P = max(E, 0)/3; above the velocity cap M is
// rescaled to |v| = 1 - delta, which makes kappa = K0/|M| and P = E delta/(1 +
// sqrt(1 + 3 delta)) with constants from the closed form.
struct RecoveryPack {
    double kap, p, kap_E, kap_M2, p_E, p_M2;
};

__device__ __forceinline__ RecoveryPack recovery_pack(double E, double Mx, double My, double Mz) {
    RecoveryPack o;
    if (E < kEFloor) {
        o.kap = 0.0;
        o.p = (E > 0.0 ? E : 0.0) / 3.0;
        o.kap_E = o.kap_M2 = o.p_M2 = 0.0;
        o.p_E = E > 0.0 ? 1.0 / 3.0 : 0.0;
        return o;
    }
    const double M2 = Mx * Mx + My * My + Mz * Mz;
    const double cap = (1.0 - kVDelta) * E * E;
    if (M2 > cap) {
        const double q = sqrt(1.0 + 3.0 * kVDelta);
        o.kap = 3.0 * sqrt(1.0 - kVDelta) / ((2.0 + q) * sqrt(M2));
        o.p = E * kVDelta / (1.0 + q);
        o.kap_E = 0.0;
        o.kap_M2 = -0.5 * o.kap / M2;
        o.p_E = kVDelta / (1.0 + q);
        o.p_M2 = 0.0;
        return o;
    }
    const double D = sqrt(4.0 * E * E - 3.0 * M2);
    const double a = 2.0 * E + D, b = E + D;
    const double r = fast_rcp(a * b * D);
    const double ra = b * D * r, rb = a * D * r, rD = a * b * r;
    o.kap = 3.0 * ra;
    o.p = (E * E - M2) * rb;
    o.kap_E = -(o.kap * o.kap / 3.0) * (2.0 + 4.0 * E * rD);
    o.kap_M2 = 0.5 * o.kap * o.kap * rD;
    o.p_E = (2.0 * E - o.p * (1.0 + 4.0 * E * rD)) * rb;
    o.p_M2 = (1.5 * o.p * rD - 1.0) * rb;
    return o;
}

}  // namespace rh
