// rh_oracle.cpp -- plain FP64 CPU oracle for 3+1D ideal relativistic hydrodynamics
// discretised with finite-difference WENO5/WENO7 and third-order SSP Runge-Kutta.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU path is checked against.  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
// table or helper with the GPU library, and it never calls into it.
//
// What it follows (Sikorski et al., "Relativistic hydrodynamics on graphics
// processing units", arXiv:1604.03360):
//   * Sec. 1, Eq. (1): conservation laws du/dt + sum_i d f_i(u)/dx_i = 0 for the
//     energy, momentum and charge densities u = (E, Mx, My, Mz, N).
//   * Sec. 1, Eq. (2): semi-discrete operator on a Cartesian grid,
//     L(u) = sum_i (F_i(x - e_i/2) - F_i(x + e_i/2)) / |e_i|, where F_i at a half
//     cell is read as the finite-difference WENO numerical flux (Sec. 1.2).
//   * Sec. 1: the ODE is integrated by a third-order Runge-Kutta method, read as the
//     Shu-Osher strong-stability-preserving variant.
//   * Sec. 1.2: finite-difference WENO of fifth and seventh order (Jiang-Shu
//     smoothness indicators, nonlinear weights, component-wise, global
//     Lax-Friedrichs splitting with alpha = 1).
//   * Sec. 1.1: the MUSTA-FORCE scheme -- MUSCL reconstruction with a slope
//     limiter, then a multi-stage predictor-corrector on the first-order
//     centred (FORCE) flux at every interface.
// Readings where the paper is silent (equation of state p = e/3, closed-form
// primitive recovery, floors, boundary conditions, epsilon = 1e-6, the MUSTA
// stage count and local Courant number, the limiters offered) are listed with
// the design notes of the repository.  Two generalisations of the flux step
// are also implemented: local Lax-Friedrichs splitting (alpha per interface
// from the characteristic speeds) and an ideal-gas equation of state whose
// primitive recovery is a bisection for the speed.
//
// Everything is templated on the scalar type so that T = std::complex<double>
// evaluates the same arithmetic in complex-step mode (directional derivatives for
// the adjoint checks).  Branches compare real parts only.
//
// Parity status: every function here is pinned by CPU tests against closed forms,
// definitions derived symbolically at test time, exact solutions or invariants.
// The hand-written VJP is pinned against the complex-step JVP (dot-product test).

#include <cmath>
#include <complex>
#include <vector>
#include <cstring>
#include <cstdint>
#include <algorithm>
#include <type_traits>

using cplx = std::complex<double>;

namespace {

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

// ---------------------------------------------------------------------------
// Grid description (the oracle's own; mirrors nothing outside this file).
// ---------------------------------------------------------------------------
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_HUBBLE = 2 };
enum { SCHEME_MUSTA = 2 };   // order field: 5 or 7 select WENO, 2 MUSTA-FORCE
enum { EOS_CONFORMAL = 0, EOS_IDEAL = 1 };
enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_VANLEER = 2, LIM_SUPERBEE = 3, LIM_NONE = 4 };

// Floors applied to the primitive recovery only (never to the stored state).
const double E_FLOOR = 1e-12;      // below this energy density the cell is treated as at rest
const double V_DELTA = 1e-12;      // momentum squared capped at (1 - V_DELTA) E^2

}  // namespace

extern "C" {

struct orc_grid {
    int n[3];          // cells along x, y, z
    double h[3];       // cell widths dx, dy, dz
    double c0[3];      // centre of cell (0,0,0)
    int order;         // 5 (WENO5) or 7 (WENO7)
    int bc[3];         // per axis: 0 periodic, 1 outflow (zero gradient), 2 analytic Hubble flow
    double eps;        // WENO epsilon
    double hub[3];     // Hubble flow: t0, e0, n0
    int limiter;       // MUSTA-FORCE: MUSCL slope limiter (LIM_*)
    int musta_k;       // MUSTA-FORCE: FORCE evaluations per interface (>= 1)
    double musta_cfl;  // MUSTA-FORCE: dt/dx of the local predictor-corrector
    int lf_local;      // WENO: 0 global Lax-Friedrichs (alpha = 1), 1 alpha per interface
    int eos;           // 0 conformal p = e/3, 1 ideal gas p = (gamma - 1)(e - n), p >= 0
    double gamma;      // ideal gas: adiabatic index
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Equation of state and the state <-> primitive maps (Sec. 1, Eq. (1) variables)
// Conformal EOS p = e/3.  Conserved: E = T^00, M_i = T^0i, N = n gamma.
// ---------------------------------------------------------------------------
template <class T>
void prim2con(const T pr[5], T u[5]) {
    // pr = (e, vx, vy, vz, n)
    T e = pr[0], vx = pr[1], vy = pr[2], vz = pr[3], n = pr[4];
    T p = e / 3.0;
    T v2 = vx * vx + vy * vy + vz * vz;
    T g2 = 1.0 / (1.0 - v2);
    T w = e + p;
    u[0] = w * g2 - p;
    u[1] = w * g2 * vx;
    u[2] = w * g2 * vy;
    u[3] = w * g2 * vz;
    u[4] = n * std::sqrt(g2);
}

// Closed-form inversion for p = e/3: with M^2 = |M|^2 and D = sqrt(4E^2 - 3M^2),
// v = 3 M / (2E + D), p = (E^2 - M^2) / (E + D), n = N sqrt(1 - v^2).
// Returns the velocity and pressure; *clamped is incremented when a floor acts.
template <class T>
void con2prim(const T u[5], T v[3], T& p, T& nden, long* clamped) {
    T E = u[0], Mx = u[1], My = u[2], Mz = u[3], N = u[4];
    if (re(E) < E_FLOOR) {
        v[0] = v[1] = v[2] = T(0.0);
        p = (re(E) > 0.0 ? E : T(0.0)) / 3.0;
        nden = N;
        if (clamped) ++*clamped;
        return;
    }
    T M2 = Mx * Mx + My * My + Mz * Mz;
    T cap = (1.0 - V_DELTA) * E * E;
    if (re(M2) > re(cap)) {
        T s = std::sqrt(cap / M2);
        Mx = Mx * s; My = My * s; Mz = Mz * s;
        M2 = cap;
        if (clamped) ++*clamped;
    }
    T D = std::sqrt(4.0 * E * E - 3.0 * M2);
    T k = 3.0 / (2.0 * E + D);
    v[0] = k * Mx;
    v[1] = k * My;
    v[2] = k * Mz;
    p = (E * E - M2) / (E + D);
    nden = N * std::sqrt(1.0 - k * k * M2);
}

// Physical flux along axis d of Eq. (1): F_d = (M_d, M_x v_d + p delta_xd,
// M_y v_d + p delta_yd, M_z v_d + p delta_zd, N v_d).
template <class T>
void flux(int d, const T u[5], const T v[3], T p, T f[5]) {
    f[0] = u[1 + d];
    f[1] = u[1] * v[d] + (d == 0 ? p : T(0.0));
    f[2] = u[2] * v[d] + (d == 1 ? p : T(0.0));
    f[3] = u[3] * v[d] + (d == 2 ? p : T(0.0));
    f[4] = u[4] * v[d];
}

// ---------------------------------------------------------------------------
// Generalised equation of state (beyond the paper's test fluids).  The ideal
// gas has unit rest mass per unit of the conserved charge: e = n + n eps_int,
// p = (gamma - 1) n eps_int = (gamma - 1)(e - n), cut off at zero pressure.
// Its sound speed is c_s^2 = gamma p / (e + p) (relativistic enthalpy
// e + p); the conformal fluid has c_s^2 = 1/3.
// ---------------------------------------------------------------------------
double ideal_pressure(double gamma, double e, double n) {
    double p = (gamma - 1.0) * (e - n);
    return p > 0.0 ? p : 0.0;
}

double eos_pressure(const orc_grid& g, double e, double n) {
    return g.eos == EOS_IDEAL ? ideal_pressure(g.gamma, e, n) : e / 3.0;
}

double sound_speed2(const orc_grid& g, double e, double p) {
    if (g.eos != EOS_IDEAL) return 1.0 / 3.0;
    return e + p > 0.0 ? g.gamma * p / (e + p) : 0.0;
}

// (e, vx, vy, vz, n) -> (E, Mx, My, Mz, N) for the grid's equation of state:
// E = (e + p) W^2 - p, M = (e + p) W^2 v, N = n W, W^2 = 1 / (1 - v^2).
void prim2con_eos(const orc_grid& g, const double pr[5], double u[5]) {
    double e = pr[0], vx = pr[1], vy = pr[2], vz = pr[3], n = pr[4];
    double p = eos_pressure(g, e, n);
    double v2 = vx * vx + vy * vy + vz * vz;
    double W2 = 1.0 / (1.0 - v2);
    double w = e + p;
    u[0] = w * W2 - p;
    u[1] = w * W2 * vx;
    u[2] = w * W2 * vy;
    u[3] = w * W2 * vz;
    u[4] = n * std::sqrt(W2);
}

// Ideal-gas recovery.  With the velocity v along M, E + p = (e + p) W^2 and
// M = (E + p) v, so e = E - |M| v and n = N sqrt(1 - v^2); the speed is the
// root in [0, 1) of g(v) = v (E + p(e(v), n(v))) - |M|.  g(0) = -|M| <= 0,
// g(1) = E + p - |M| > 0 below the cap, and g is increasing (dg/dv >=
// E - (gamma - 1)|M| > 0 for gamma <= 2), so plain bisection finds it; it stops
// when the bracket is below one part in 1e16 of the speed.  Same floors as the
// closed form: E below the floor -> at rest; |M|^2 capped at (1 - delta) E^2.
void con2prim_ideal(const orc_grid& g, const double u[5], double v[3], double& p, double& e,
                    double& n, long* clamped) {
    double E = u[0], Mx = u[1], My = u[2], Mz = u[3], N = u[4];
    if (E < E_FLOOR) {
        v[0] = v[1] = v[2] = 0.0;
        e = E > 0.0 ? E : 0.0;
        n = N;
        p = ideal_pressure(g.gamma, e, n);
        if (clamped) ++*clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    double cap = (1.0 - V_DELTA) * E * E;
    if (M2 > cap) {
        double s = std::sqrt(cap / M2);
        Mx *= s; My *= s; Mz *= s;
        M2 = cap;
        if (clamped) ++*clamped;
    }
    double M = std::sqrt(M2);
    double speed = 0.0;
    if (M > 0.0) {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 400; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double pm = ideal_pressure(g.gamma, E - M * mid, N * std::sqrt(1.0 - mid * mid));
            if (mid * (E + pm) - M < 0.0) lo = mid; else hi = mid;
            if (hi - lo <= 1e-16 * hi) break;
        }
        speed = 0.5 * (lo + hi);
    }
    e = E - M * speed;
    n = N * std::sqrt(1.0 - speed * speed);
    p = ideal_pressure(g.gamma, e, n);
    double k = M > 0.0 ? speed / M : 0.0;
    v[0] = k * Mx;
    v[1] = k * My;
    v[2] = k * Mz;
}

// Primitive recovery for the grid's equation of state; T = double only for the
// ideal gas (the complex-step paths are conformal).
template <class T>
void recover(const orc_grid& g, const T u[5], T v[3], T& p, T& e, T& n, long* clamped) {
    if constexpr (std::is_same<T, double>::value) {
        if (g.eos == EOS_IDEAL) {
            con2prim_ideal(g, u, v, p, e, n, clamped);
            return;
        }
    }
    con2prim(u, v, p, n, clamped);
    e = 3.0 * p;
}

// Largest characteristic speed |lambda| of the flux along axis d: the
// acoustic eigenvalues
//   lambda+- = (v_d (1 - c_s^2) +- c_s sqrt((1 - v^2)(1 - v^2 c_s^2 - v_d^2 (1 - c_s^2))))
//              / (1 - v^2 c_s^2)
// bracket the material speed v_d, so the larger magnitude of the two is the
// bound.
double max_speed(const orc_grid& g, int d, const double v[3], double p, double e) {
    double cs2 = sound_speed2(g, e, p);
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double vd = v[d];
    double disc = cs2 * (1.0 - v2) * (1.0 - v2 * cs2 - vd * vd * (1.0 - cs2));
    double root = std::sqrt(disc > 0.0 ? disc : 0.0);
    double den = 1.0 - v2 * cs2;
    double lp = (vd * (1.0 - cs2) + root) / den, lm = (vd * (1.0 - cs2) - root) / den;
    return std::max(std::fabs(lp), std::fabs(lm));
}

// ---------------------------------------------------------------------------
// MUSTA-FORCE (Sec. 1.1).
// MUSCL: limited slope of cell j from a = u_j - u_{j-1}, b = u_{j+1} - u_j,
// component-wise on the conserved variables; zero where a and b do not share a
// sign.  minmod: the smaller magnitude; MC: min(2|a|, 2|b|, |a + b|/2); van
// Leer: 2ab/(a + b); superbee: max(min(2|a|, |b|), min(|a|, 2|b|)); NONE: no
// slope (first order).
// ---------------------------------------------------------------------------
double limited_slope(int lim, double a, double b) {
    if (lim == LIM_NONE) return 0.0;
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    double sg = a > 0.0 ? 1.0 : -1.0, aa = std::fabs(a), ab = std::fabs(b);
    if (lim == LIM_MINMOD) return sg * std::min(aa, ab);
    if (lim == LIM_MC) return sg * std::min(std::min(2.0 * aa, 2.0 * ab), 0.5 * (aa + ab));
    if (lim == LIM_VANLEER) return 2.0 * a * b / (a + b);
    return sg * std::max(std::min(2.0 * aa, ab), std::min(aa, 2.0 * ab));
}

// physical flux along d of a state, through the grid's recovery
void state_flux(const orc_grid& g, int d, const double u[5], double f[5], long* clamped) {
    double v[3], p, e, n;
    recover(g, u, v, p, e, n, clamped);
    flux(d, u, v, p, f);
}

// The MUSTA flux at one interface from the reconstructed states uL | uR,
// with lam = dt/dx of the local solver.  Each stage evaluates the FORCE flux,
// the mean of the Lax-Friedrichs flux and the flux of the two-step
// Lax-Wendroff (Richtmyer) state,
//   uM = (uL + uR)/2 - lam/2 (fR - fL),
//   F  = (fL + 2 f(uM) + fR)/4 - (uR - uL)/(4 lam),
// and, before every stage but the last, opens the local Riemann fan by one
// local time step of each side's cell: uL -= lam (F - fL), uR -= lam (fR - F).
void musta_flux(const orc_grid& g, int d, const double uL0[5], const double uR0[5], double F[5],
                long* clamped) {
    double uL[5], uR[5];
    for (int c = 0; c < 5; ++c) { uL[c] = uL0[c]; uR[c] = uR0[c]; }
    const double lam = g.musta_cfl;
    for (int stage = 1; stage <= g.musta_k; ++stage) {
        double fL[5], fR[5], uM[5], fM[5];
        state_flux(g, d, uL, fL, clamped);
        state_flux(g, d, uR, fR, clamped);
        for (int c = 0; c < 5; ++c) uM[c] = 0.5 * (uL[c] + uR[c]) - 0.5 * lam * (fR[c] - fL[c]);
        state_flux(g, d, uM, fM, clamped);
        for (int c = 0; c < 5; ++c)
            F[c] = 0.25 * (fL[c] + 2.0 * fM[c] + fR[c]) - (uR[c] - uL[c]) / (4.0 * lam);
        if (stage < g.musta_k) {
            for (int c = 0; c < 5; ++c) {
                uL[c] = uL[c] - lam * (F[c] - fL[c]);
                uR[c] = uR[c] - lam * (fR[c] - F[c]);
            }
        }
    }
}

// Face i+1/2 from the four cells i-1 .. i+2 along the line (s[0..3]): MUSCL
// states uL = u_i + slope_i / 2, uR = u_{i+1} - slope_{i+1} / 2, then MUSTA.
void musta_face(const orc_grid& g, int d, const double s[4][5], double F[5], long* clamped) {
    double uL[5], uR[5];
    for (int c = 0; c < 5; ++c) {
        double si = limited_slope(g.limiter, s[1][c] - s[0][c], s[2][c] - s[1][c]);
        double sj = limited_slope(g.limiter, s[2][c] - s[1][c], s[3][c] - s[2][c]);
        uL[c] = s[1][c] + 0.5 * si;
        uR[c] = s[2][c] - 0.5 * sj;
    }
    musta_flux(g, d, uL, uR, F, clamped);
}

// ---------------------------------------------------------------------------
// WENO reconstruction (Sec. 1.2).  Finite-difference form: the point values f_j
// are treated as cell averages of a function h whose value at x_{i+1/2} is the
// numerical flux.  s[0 .. 2r-2] holds f_{i-r+1} .. f_{i+r-1}; the result is the
// left-biased reconstruction at i+1/2.
// Candidate interpolants q_k, linear weights d_k and smoothness indicators beta_k
// follow Jiang & Shu; beta_k = sum_{l=1}^{r-1} int_{cell} (d^l p_k / dx^l)^2 dx
// with dx = 1, written as squares of difference combinations (WENO5) or from
// the derivative coefficients of the cubic candidate polynomial (WENO7).
// ---------------------------------------------------------------------------
template <class T>
void weno5_parts(const T s[5], T q[3], T b[3]) {
    const T &fm2 = s[0], &fm1 = s[1], &f0 = s[2], &fp1 = s[3], &fp2 = s[4];
    q[0] = (2.0 * fm2 - 7.0 * fm1 + 11.0 * f0) / 6.0;
    q[1] = (-fm1 + 5.0 * f0 + 2.0 * fp1) / 6.0;
    q[2] = (2.0 * f0 + 5.0 * fp1 - fp2) / 6.0;
    T a0 = fm2 - 2.0 * fm1 + f0, c0 = fm2 - 4.0 * fm1 + 3.0 * f0;
    T a1 = fm1 - 2.0 * f0 + fp1, c1 = fm1 - fp1;
    T a2 = f0 - 2.0 * fp1 + fp2, c2 = 3.0 * f0 - 4.0 * fp1 + fp2;
    b[0] = 13.0 / 12.0 * a0 * a0 + 0.25 * c0 * c0;
    b[1] = 13.0 / 12.0 * a1 * a1 + 0.25 * c1 * c1;
    b[2] = 13.0 / 12.0 * a2 * a2 + 0.25 * c2 * c2;
}

template <class T>
void weno7_parts(const T s[7], T q[4], T b[4]) {
    const T &m3 = s[0], &m2 = s[1], &m1 = s[2], &z0 = s[3], &p1 = s[4], &p2 = s[5], &p3 = s[6];
    q[0] = (-3.0 * m3 + 13.0 * m2 - 23.0 * m1 + 25.0 * z0) / 12.0;
    q[1] = (m2 - 5.0 * m1 + 13.0 * z0 + 3.0 * p1) / 12.0;
    q[2] = (-m1 + 7.0 * z0 + 7.0 * p1 - p2) / 12.0;
    q[3] = (3.0 * z0 + 13.0 * p1 - 5.0 * p2 + p3) / 12.0;
    // beta_k = int_cell (p')^2 + (p'')^2 + (p''')^2 for the cubic candidate
    // p_k(x) = a0 + a1 x + a2 x^2 + a3 x^3 (x in cells from the centre of cell i):
    // beta_k = a1^2 + a1 a3 / 2 + 13/3 a2^2 + 3129/80 a3^2.
    T a1[4], a2[4], a3[4];
    a1[0] = (-7.0 * m3 + 33.0 * m2 - 69.0 * m1 + 43.0 * z0) / 24.0;
    a2[0] = (-m3 + 4.0 * m2 - 5.0 * m1 + 2.0 * z0) / 2.0;
    a3[0] = (-m3 + 3.0 * m2 - 3.0 * m1 + z0) / 6.0;
    a1[1] = (5.0 * m2 - 27.0 * m1 + 15.0 * z0 + 7.0 * p1) / 24.0;
    a2[1] = (m1 - 2.0 * z0 + p1) / 2.0;
    a3[1] = (-m2 + 3.0 * m1 - 3.0 * z0 + p1) / 6.0;
    a1[2] = (-7.0 * m1 - 15.0 * z0 + 27.0 * p1 - 5.0 * p2) / 24.0;
    a2[2] = (m1 - 2.0 * z0 + p1) / 2.0;
    a3[2] = (-m1 + 3.0 * z0 - 3.0 * p1 + p2) / 6.0;
    a1[3] = (-43.0 * z0 + 69.0 * p1 - 33.0 * p2 + 7.0 * p3) / 24.0;
    a2[3] = (2.0 * z0 - 5.0 * p1 + 4.0 * p2 - p3) / 2.0;
    a3[3] = (-z0 + 3.0 * p1 - 3.0 * p2 + p3) / 6.0;
    for (int k = 0; k < 4; ++k)
        b[k] = a1[k] * a1[k] + 0.5 * a1[k] * a3[k] + 13.0 / 3.0 * a2[k] * a2[k]
             + 3129.0 / 80.0 * a3[k] * a3[k];
}

const double D5[3] = {1.0 / 10.0, 6.0 / 10.0, 3.0 / 10.0};
const double D7[4] = {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0};

// Nonlinear weights alpha_k = d_k / (eps + beta_k)^2, omega_k = alpha_k / sum(alpha).
// linear != 0 replaces omega by d (used only by tests of the linear scheme).
template <class T>
T weno(int order, const T* s, double eps, int linear) {
    int r = order == 5 ? 3 : 4;
    T q[4], b[4];
    const double* d;
    if (order == 5) { weno5_parts(s, q, b); d = D5; }
    else            { weno7_parts(s, q, b); d = D7; }
    if (linear) {
        T acc = 0.0;
        for (int k = 0; k < r; ++k) acc += d[k] * q[k];
        return acc;
    }
    T alpha[4], sum = 0.0;
    for (int k = 0; k < r; ++k) {
        T g = eps + b[k];
        alpha[k] = d[k] / (g * g);
        sum += alpha[k];
    }
    T acc = 0.0;
    for (int k = 0; k < r; ++k) acc += (alpha[k] / sum) * q[k];
    return acc;
}

// ---------------------------------------------------------------------------
// Analytic Hubble-like flow: u^mu = x^mu / tau, tau = sqrt(t^2 - r^2),
// e = e0 (t0/tau)^4, n = n0 (t0/tau)^3, v = x/t.
// ---------------------------------------------------------------------------
void hubble_prim(const double hub[3], double t, double x, double y, double z, double pr[5]) {
    double tau = std::sqrt(t * t - (x * x + y * y + z * z));
    double s = hub[0] / tau;
    pr[0] = hub[1] * s * s * s * s;
    pr[1] = x / t;
    pr[2] = y / t;
    pr[3] = z / t;
    pr[4] = hub[2] * s * s * s;
}

inline size_t cidx(const orc_grid& g, int i, int j, int k) {
    return (size_t)i + (size_t)g.n[0] * ((size_t)j + (size_t)g.n[1] * (size_t)k);
}

// State of cell m along axis d on the line through (i, j, k), m may lie in the
// ghost region; ghosts follow the axis boundary condition.
template <class T>
void line_cell(const orc_grid& g, double t, const T* u, int d, int ijk[3], int m, T out[5]) {
    int nd = g.n[d];
    int c[3] = {ijk[0], ijk[1], ijk[2]};
    if (m >= 0 && m < nd) {
        c[d] = m;
    } else if (g.bc[d] == BC_PERIODIC) {
        c[d] = ((m % nd) + nd) % nd;
    } else if (g.bc[d] == BC_OUTFLOW) {
        c[d] = m < 0 ? 0 : nd - 1;
    } else {  // analytic Hubble flow at the ghost centre
        c[d] = m;
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = g.c0[a] + c[a] * g.h[a];
        double pr[5], uc[5];
        hubble_prim(g.hub, t, x[0], x[1], x[2], pr);
        prim2con(pr, uc);
        for (int f = 0; f < 5; ++f) out[f] = T(uc[f]);
        return;
    }
    size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
    size_t id = cidx(g, c[0], c[1], c[2]);
    for (int f = 0; f < 5; ++f) out[f] = u[f * ncell + id];
}

// MUSTA-FORCE form of Eq. (2): the face fluxes of every axis longer than one
// cell (an axis of one cell contributes nothing), accumulated x, y, z.  Two
// ghost cells per side feed the MUSCL slopes of the faces at the line ends.
// Floors are counted per recovery of a face state (three per MUSTA stage),
// each face of the grid once.
void apply_L_musta(const orc_grid& g, double t, const double* u, double* L, long* clamps) {
    const int G = 2;
    size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
    long clamp_total = 0;
    for (int d = 0; d < 3; ++d) {
        if (g.n[d] == 1) continue;
        int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        int nd = g.n[d];
        long nlines = (long)g.n[a1] * g.n[a2];
#pragma omp parallel for schedule(static) reduction(+ : clamp_total)
        for (long line = 0; line < nlines; ++line) {
            int ijk[3];
            ijk[d] = 0;
            ijk[a1] = (int)(line % g.n[a1]);
            ijk[a2] = (int)(line / g.n[a1]);
            int len = nd + 2 * G;
            std::vector<double> uu(5 * len), Fh(5 * (nd + 1));
            for (int m = -G; m < nd + G; ++m) {
                double uc[5];
                line_cell(g, t, u, d, ijk, m, uc);
                for (int c = 0; c < 5; ++c) uu[c * len + m + G] = uc[c];
            }
            for (int i = -1; i < nd; ++i) {
                double st[4][5], F[5];
                for (int o = 0; o < 4; ++o)
                    for (int c = 0; c < 5; ++c) st[o][c] = uu[c * len + (i - 1 + o) + G];
                long cl = 0;
                musta_face(g, d, st, F, &cl);
                clamp_total += cl;
                for (int c = 0; c < 5; ++c) Fh[c * (nd + 1) + i + 1] = F[c];
            }
            for (int i = 0; i < nd; ++i) {
                int cc[3] = {ijk[0], ijk[1], ijk[2]};
                cc[d] = i;
                size_t id = cidx(g, cc[0], cc[1], cc[2]);
                for (int c = 0; c < 5; ++c) {
                    const double* Fc = &Fh[c * (nd + 1)];   // faces -1/2 .. nd-1/2 of component c
                    L[c * ncell + id] += (Fc[i] - Fc[i + 1]) / g.h[d];
                }
            }
        }
    }
    if (clamps) *clamps += clamp_total;
}

// Eq. (2): L(u) = sum_d (Fhat_d(i-1/2) - Fhat_d(i+1/2)) / h_d, directions in the
// order x, y, z, accumulated into a zeroed array.  WENO face fluxes from
// Lax-Friedrichs-split fluxes f+- = (F +- alpha u)/2: alpha = 1 (global), or,
// with lf_local, the largest characteristic speed over the 2r cells of the
// interface's stencil.
template <class T>
void apply_L(const orc_grid& g, double t, const T* u, T* L, long* clamps) {
    size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
    for (size_t q = 0; q < 5 * ncell; ++q) L[q] = T(0.0);
    if constexpr (std::is_same<T, double>::value) {
        if (g.order == SCHEME_MUSTA) {
            apply_L_musta(g, t, u, L, clamps);
            return;
        }
    }
    const int r = g.order == 5 ? 3 : 4;
    const int G = r;  // ghost cells per side
    const bool local = g.lf_local != 0;
    long clamp_total = 0;
    for (int d = 0; d < 3; ++d) {
        int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        int nd = g.n[d];
        long nlines = (long)g.n[a1] * g.n[a2];
#pragma omp parallel for schedule(static) reduction(+ : clamp_total)
        for (long line = 0; line < nlines; ++line) {
            int ijk[3];
            ijk[d] = 0;
            ijk[a1] = (int)(line % g.n[a1]);
            ijk[a2] = (int)(line / g.n[a1]);
            int len = nd + 2 * G;
            std::vector<T> ff(5 * len), uu(5 * len), Fh(5 * (nd + 1));
            std::vector<double> spd(len, 1.0);
            for (int m = -G; m < nd + G; ++m) {
                T uc[5], v[3], p, e, nden, f[5];
                line_cell(g, t, u, d, ijk, m, uc);
                long cl = 0;
                recover(g, uc, v, p, e, nden, &cl);
                if (m >= 0 && m < nd) clamp_total += cl;
                flux(d, uc, v, p, f);
                for (int c = 0; c < 5; ++c) {
                    ff[c * len + m + G] = f[c];
                    uu[c * len + m + G] = uc[c];
                }
                if constexpr (std::is_same<T, double>::value) {
                    if (local) spd[m + G] = max_speed(g, d, v, p, e);
                }
            }
            // interfaces i+1/2 for i = -1 .. nd-1 stored at Fh[i+1]
            for (int i = -1; i < nd; ++i) {
                double alpha = 1.0;
                if (local) {
                    alpha = 0.0;
                    for (int o = 0; o < 2 * r; ++o) alpha = std::max(alpha, spd[(i - r + 1 + o) + G]);
                }
                for (int c = 0; c < 5; ++c) {
                    T sp[7], sm[7];
                    for (int o = 0; o < 2 * r - 1; ++o) {
                        const int jp = c * len + (i - r + 1 + o) + G;   // f+_{i-r+1+o}
                        const int jm = c * len + (i + r - o) + G;       // mirrored: f-_{i+r-o}
                        if (local) {
                            sp[o] = 0.5 * (ff[jp] + alpha * uu[jp]);
                            sm[o] = 0.5 * (ff[jm] - alpha * uu[jm]);
                        } else {
                            sp[o] = 0.5 * (ff[jp] + uu[jp]);
                            sm[o] = 0.5 * (ff[jm] - uu[jm]);
                        }
                    }
                    Fh[c * (nd + 1) + i + 1] = weno(g.order, sp, g.eps, 0) + weno(g.order, sm, g.eps, 0);
                }
            }
            for (int i = 0; i < nd; ++i) {
                int cc[3] = {ijk[0], ijk[1], ijk[2]};
                cc[d] = i;
                size_t id = cidx(g, cc[0], cc[1], cc[2]);
                for (int c = 0; c < 5; ++c)
                    L[c * ncell + id] += (Fh[c * (nd + 1) + i] - Fh[c * (nd + 1) + i + 1]) / g.h[d];
            }
        }
    }
    if (clamps) *clamps += clamp_total;
}

// Shu-Osher SSP-RK3 (Sec. 1, third-order Runge-Kutta), stage times t, t+dt, t+dt/2.
template <class T>
void rk3_step(const orc_grid& g, double t, double dt, T* u, long* clamps) {
    size_t N = 5 * (size_t)g.n[0] * g.n[1] * g.n[2];
    std::vector<T> L(N), u1(N), u2(N);
    apply_L(g, t, u, L.data(), clamps);
    for (size_t q = 0; q < N; ++q) u1[q] = u[q] + dt * L[q];
    apply_L(g, t + dt, u1.data(), L.data(), clamps);
    for (size_t q = 0; q < N; ++q) u2[q] = 0.75 * u[q] + 0.25 * (u1[q] + dt * L[q]);
    apply_L(g, t + 0.5 * dt, u2.data(), L.data(), clamps);
    for (size_t q = 0; q < N; ++q) u[q] = (1.0 / 3.0) * u[q] + (2.0 / 3.0) * (u2[q] + dt * L[q]);
}

bool grid_ok(const orc_grid* g) {
    if (!g) return false;
    if (g->order != 5 && g->order != 7 && g->order != SCHEME_MUSTA) return false;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || !(g->h[a] > 0.0)) return false;
        if (g->bc[a] < 0 || g->bc[a] > 2) return false;
        // the analytic boundary is the conformal fluid's Hubble flow
        if (g->bc[a] == BC_HUBBLE && g->eos != EOS_CONFORMAL) return false;
    }
    if (g->eos != EOS_CONFORMAL && g->eos != EOS_IDEAL) return false;
    if (g->eos == EOS_IDEAL && !(g->gamma > 1.0 && g->gamma <= 2.0)) return false;
    if (g->lf_local != 0 && g->lf_local != 1) return false;
    if (g->order == SCHEME_MUSTA) {
        if (g->limiter < LIM_MINMOD || g->limiter > LIM_NONE) return false;
        if (g->musta_k < 1 || !(g->musta_cfl > 0.0 && g->musta_cfl <= 1.0)) return false;
    }
    return true;
}

// The complex-step derivatives and the hand-written adjoint cover the paper's
// WENO scheme with the conformal fluid and global splitting.
bool grid_ok_adjoint(const orc_grid* g) {
    return grid_ok(g) && g->order != SCHEME_MUSTA && g->eos == EOS_CONFORMAL && g->lf_local == 0;
}

}  // namespace

extern "C" {

// Primitive (e, vx, vy, vz, n) -> conserved (E, Mx, My, Mz, N), SoA [5][n].
int orc_prim2con(long n, const double* prim, double* con) {
    for (long i = 0; i < n; ++i) {
        double pr[5], u[5];
        for (int f = 0; f < 5; ++f) pr[f] = prim[f * n + i];
        prim2con(pr, u);
        for (int f = 0; f < 5; ++f) con[f * n + i] = u[f];
    }
    return 0;
}

// Conserved -> primitive (e, vx, vy, vz, n) with floors; SoA [5][n].
int orc_con2prim(long n, const double* con, double* prim, long* clamps) {
    long cl = 0;
    for (long i = 0; i < n; ++i) {
        double u[5], v[3], p, nd;
        for (int f = 0; f < 5; ++f) u[f] = con[f * n + i];
        con2prim(u, v, p, nd, &cl);
        prim[0 * n + i] = 3.0 * p;
        prim[1 * n + i] = v[0];
        prim[2 * n + i] = v[1];
        prim[3 * n + i] = v[2];
        prim[4 * n + i] = nd;
    }
    if (clamps) *clamps = cl;
    return 0;
}

// Physical flux along axis d for n states (SoA [5][n]).
int orc_flux(int d, long n, const double* con, double* f_out) {
    if (d < 0 || d > 2) return -1;
    for (long i = 0; i < n; ++i) {
        double u[5], v[3], p, nd, f[5];
        for (int c = 0; c < 5; ++c) u[c] = con[c * n + i];
        con2prim(u, v, p, nd, (long*)nullptr);
        flux(d, u, v, p, f);
        for (int c = 0; c < 5; ++c) f_out[c * n + i] = f[c];
    }
    return 0;
}

// One WENO reconstruction from 2r-1 values (left-biased, at i+1/2).
double orc_weno(int order, const double* s, double eps, int linear) {
    return weno(order, s, eps, linear);
}

// Candidate values q_k and smoothness indicators beta_k of one stencil.
int orc_weno_parts(int order, const double* s, double* q, double* b) {
    if (order == 5) weno5_parts(s, q, b);
    else if (order == 7) weno7_parts(s, q, b);
    else return -1;
    return 0;
}

// Primitive <-> conserved maps and characteristic speeds for the equation of
// state of grid g (conformal or ideal gas); SoA [5][n].
int orc_prim2con_eos(const orc_grid* g, long n, const double* prim, double* con) {
    if (!grid_ok(g)) return -1;
    for (long i = 0; i < n; ++i) {
        double pr[5], u[5];
        for (int f = 0; f < 5; ++f) pr[f] = prim[f * n + i];
        prim2con_eos(*g, pr, u);
        for (int f = 0; f < 5; ++f) con[f * n + i] = u[f];
    }
    return 0;
}

int orc_con2prim_eos(const orc_grid* g, long n, const double* con, double* prim, long* clamps) {
    if (!grid_ok(g)) return -1;
    long cl = 0;
    for (long i = 0; i < n; ++i) {
        double u[5], v[3], p, e, nd;
        for (int f = 0; f < 5; ++f) u[f] = con[f * n + i];
        recover(*g, u, v, p, e, nd, &cl);
        prim[0 * n + i] = e;
        prim[1 * n + i] = v[0];
        prim[2 * n + i] = v[1];
        prim[3 * n + i] = v[2];
        prim[4 * n + i] = nd;
    }
    if (clamps) *clamps = cl;
    return 0;
}

// Largest characteristic speed along axis d of n conserved states.
int orc_max_speed(const orc_grid* g, int d, long n, const double* con, double* out) {
    if (!grid_ok(g) || d < 0 || d > 2) return -1;
    for (long i = 0; i < n; ++i) {
        double u[5], v[3], p, e, nd;
        for (int f = 0; f < 5; ++f) u[f] = con[f * n + i];
        recover(*g, u, v, p, e, nd, (long*)nullptr);
        out[i] = max_speed(*g, d, v, p, e);
    }
    return 0;
}

// Limited MUSCL slope from the backward and forward differences a, b.
double orc_limited_slope(int limiter, double a, double b) { return limited_slope(limiter, a, b); }

// MUSTA flux along d between the states uL | uR (5 values each), and the face
// flux from the four cells around the face (s[4][5], cell-major).
int orc_musta_flux(const orc_grid* g, int d, const double* uL, const double* uR, double* F, long* clamps) {
    if (!grid_ok(g) || g->order != SCHEME_MUSTA || d < 0 || d > 2) return -1;
    long cl = 0;
    musta_flux(*g, d, uL, uR, F, &cl);
    if (clamps) *clamps = cl;
    return 0;
}

int orc_musta_face(const orc_grid* g, int d, const double* s, double* F) {
    if (!grid_ok(g) || g->order != SCHEME_MUSTA || d < 0 || d > 2) return -1;
    double st[4][5];
    for (int o = 0; o < 4; ++o)
        for (int c = 0; c < 5; ++c) st[o][c] = s[o * 5 + c];
    musta_face(*g, d, st, F, (long*)nullptr);
    return 0;
}

// L(u) at time t (t only matters for analytic boundaries).  u, L: [5][nz][ny][nx].
int orc_L(const orc_grid* g, double t, const double* u, double* L, long* clamps) {
    if (!grid_ok(g)) return -1;
    apply_L(*g, t, u, L, clamps);
    return 0;
}

// n SSP-RK3 steps of size dt, in place; *t is advanced.
int orc_step(const orc_grid* g, double* t, double dt, int nsteps, double* u, long* clamps) {
    if (!grid_ok(g) || !(dt > 0.0) || nsteps < 0) return -1;
    for (int s = 0; s < nsteps; ++s) {
        rk3_step(*g, *t, dt, u, clamps);
        *t += dt;
    }
    return 0;
}

// Compensated (Kahan) FP64 sums of the five conserved fields over all cells.
int orc_totals(const orc_grid* g, const double* u, double out[5]) {
    if (!grid_ok(g)) return -1;
    size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    for (int f = 0; f < 5; ++f) {
        double s = 0.0, c = 0.0;
        for (size_t i = 0; i < ncell; ++i) {
            double y = u[f * ncell + i] - c;
            double tt = s + y;
            c = (tt - s) - y;
            s = tt;
        }
        out[f] = s;
    }
    return 0;
}

// Analytic Hubble-like flow primitives at n points xyz[3][n] at time t.
int orc_hubble_prim(const double hub[3], double t, long n, const double* xyz, double* prim) {
    for (long i = 0; i < n; ++i) {
        double pr[5];
        hubble_prim(hub, t, xyz[i], xyz[n + i], xyz[2 * n + i], pr);
        for (int f = 0; f < 5; ++f) prim[f * n + i] = pr[f];
    }
    return 0;
}

// Directional derivative J(u) v of L at u by the complex step:
// Jv = Im L(u + i h v) / h with h = 1e-30 (no subtractive cancellation).
int orc_jvp_L(const orc_grid* g, double t, const double* u, const double* v, double* jv) {
    if (!grid_ok_adjoint(g)) return -1;
    const double h = 1e-30;
    size_t N = 5 * (size_t)g->n[0] * g->n[1] * g->n[2];
    std::vector<cplx> uc(N), Lc(N);
    for (size_t q = 0; q < N; ++q) uc[q] = cplx(u[q], h * v[q]);
    apply_L(*g, t, uc.data(), Lc.data(), (long*)nullptr);
    for (size_t q = 0; q < N; ++q) jv[q] = Lc[q].imag() / h;
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Exact Riemann solution for the conformal fluid (p = e/3) with both initial
// states at rest and e_L > e_R: a left-moving rarefaction, a contact and a
// right-moving shock.  This is the analytic reference of the shock-tube test
// (Sec. 3, Fig. 1).
//   * Rarefaction: the Riemann invariant artanh(v) + (sqrt(3)/4) ln e is constant
//     across the fan; inside it xi = (v - c_s) / (1 - v c_s), c_s = 1/sqrt(3);
//     the flow is isentropic, so n / e^(3/4) is constant.
//   * Shock: in the shock frame the normal velocities obey v_a v_b = 1/3 and the
//     energy densities e_b / e_a = (9 v_a^2 - 1) / (3 (1 - v_a^2)); the charge
//     flux n gamma v is continuous.
// ---------------------------------------------------------------------------
namespace {

struct RiemannStar {
    double e_star, v_star, n_left_star, n_right_star, v_shock, xi_tail;
};

double shock_post_velocity(double vs) {
    // lab-frame velocity behind a shock moving at vs into fluid at rest
    double vb = 1.0 / (3.0 * vs);
    return (vs - vb) / (1.0 - vs * vb);
}
double shock_energy_ratio(double vs) { return (9.0 * vs * vs - 1.0) / (3.0 * (1.0 - vs * vs)); }

RiemannStar riemann_star(double eL, double nL, double eR, double nR) {
    const double sq3 = std::sqrt(3.0);
    // residual in the shock speed: velocity behind the shock minus velocity at the
    // same energy density on the rarefaction branch
    auto resid = [&](double vs) {
        double es = eR * shock_energy_ratio(vs);
        double v_rare = std::tanh(0.25 * sq3 * std::log(eL / es));
        return shock_post_velocity(vs) - v_rare;
    };
    double lo = 1.0 / sq3, hi = 1.0;
    // resid(lo) < 0 (no shock, rarefaction still accelerates), resid(hi) > 0
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (resid(mid) < 0.0) lo = mid; else hi = mid;
    }
    RiemannStar s;
    s.v_shock = 0.5 * (lo + hi);
    s.e_star = eR * shock_energy_ratio(s.v_shock);
    s.v_star = shock_post_velocity(s.v_shock);
    s.n_left_star = nL * std::pow(s.e_star / eL, 0.75);
    // charge flux continuity in the shock frame: n_a gamma_a v_a = n_b gamma_b v_b
    double va = s.v_shock, vb = 1.0 / (3.0 * s.v_shock);
    double ga = 1.0 / std::sqrt(1.0 - va * va), gb = 1.0 / std::sqrt(1.0 - vb * vb);
    s.n_right_star = nR * ga * va / (gb * vb);
    double cs = 1.0 / sq3;
    s.xi_tail = (s.v_star - cs) / (1.0 - s.v_star * cs);
    return s;
}

}  // namespace

extern "C" {

// prim_out[5][n] = (e, v, 0, 0, n) at similarity coordinates xi[i] = x/t.
// star_out (6 doubles, may be null): e*, v*, n* left of contact, n* right of
// contact, shock speed, rarefaction tail speed.
int orc_riemann_conformal(double eL, double nL, double eR, double nR, long n, const double* xi,
                          double* prim_out, double* star_out) {
    if (!(eL > eR) || !(eR > 0.0)) return -1;
    RiemannStar s = riemann_star(eL, nL, eR, nR);
    const double cs = 1.0 / std::sqrt(3.0);
    for (long i = 0; i < n; ++i) {
        double x = xi[i], e, v, nn;
        if (x < -cs) { e = eL; v = 0.0; nn = nL; }
        else if (x < s.xi_tail) {
            v = (x + cs) / (1.0 + x * cs);
            e = eL * std::exp(-(4.0 / std::sqrt(3.0)) * std::atanh(v));
            nn = nL * std::pow(e / eL, 0.75);
        }
        else if (x < s.v_star) { e = s.e_star; v = s.v_star; nn = s.n_left_star; }
        else if (x < s.v_shock) { e = s.e_star; v = s.v_star; nn = s.n_right_star; }
        else { e = eR; v = 0.0; nn = nR; }
        prim_out[0 * n + i] = e;
        prim_out[1 * n + i] = v;
        prim_out[2 * n + i] = 0.0;
        prim_out[3 * n + i] = 0.0;
        prim_out[4 * n + i] = nn;
    }
    if (star_out) {
        star_out[0] = s.e_star; star_out[1] = s.v_star; star_out[2] = s.n_left_star;
        star_out[3] = s.n_right_star; star_out[4] = s.v_shock; star_out[5] = s.xi_tail;
    }
    return 0;
}

}  // extern "C"

#ifdef _OPENMP
#include <omp.h>
#endif

// Thread count of the OpenMP loops over grid lines (n >= 1); used only to time
// the oracle single-threaded.
extern "C" void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

extern "C" int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// ---------------------------------------------------------------------------
// Adjoint (vector-Jacobian products) of L and of one SSP-RK3 step.
//
// With w a field of weights, sum_i w_i . L_i = sum over every interface i+1/2
// of Fhat(i+1/2) . (w_{i+1} - w_i) / h (summation by parts of Eq. (2), with w
// zero outside the grid).  Each face flux depends on the split fluxes of its
// stencil cells, each split flux f+- = (F(u) +- u)/2 on the state of its cell,
// and ghost cells are copies of interior cells (periodic, outflow) or
// constants (analytic boundaries).  The chain rule is applied in that order:
//   * d fhat / d s_j from the WENO formula: omega-weighted candidate
//     coefficients plus the weight sensitivities,
//     d fhat/d s_j = sum_k omega_k dq_k/ds_j
//                    - 2 sum_k omega_k (q_k - fhat)/(eps + beta_k) dbeta_k/ds_j;
//     the linear and quadratic forms q_k(s), beta_k(s) are read off the forward
//     formulas at unit vectors (beta_k by polarization), so no coefficient is
//     typed twice;
//   * d F / d u per cell by the complex step of the forward flux (exact to
//     rounding);
//   * contributions to ghost cells are sent back to the interior cell they copy.
// ---------------------------------------------------------------------------
namespace {

struct WenoForms {
    int r = 0;
    double Q[4][7];       // q_k = sum_j Q[k][j] s_j
    double B[4][7][7];    // beta_k = s^T B_k s (symmetric)
};

WenoForms weno_forms(int order) {
    WenoForms F;
    F.r = order == 5 ? 3 : 4;
    const int m = 2 * F.r - 1;
    double e[7], q[4], b[4];
    double bd[7][4];
    for (int j = 0; j < m; ++j) {
        for (int i = 0; i < m; ++i) e[i] = i == j ? 1.0 : 0.0;
        if (order == 5) weno5_parts(e, q, b); else weno7_parts(e, q, b);
        for (int k = 0; k < F.r; ++k) {
            F.Q[k][j] = q[k];
            F.B[k][j][j] = b[k];
            bd[j][k] = b[k];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            for (int t = 0; t < m; ++t) e[t] = (t == i || t == j) ? 1.0 : 0.0;
            if (order == 5) weno5_parts(e, q, b); else weno7_parts(e, q, b);
            for (int k = 0; k < F.r; ++k) {
                const double off = 0.5 * (b[k] - bd[i][k] - bd[j][k]);
                F.B[k][i][j] = off;
                F.B[k][j][i] = off;
            }
        }
    return F;
}

const WenoForms& forms(int order) {
    static const WenoForms f5 = weno_forms(5), f7 = weno_forms(7);
    return order == 5 ? f5 : f7;
}

// gradient of the left-biased reconstruction with respect to its 2r-1 inputs
void weno_grad(int order, const double* s, double eps, double* grad) {
    const WenoForms& F = forms(order);
    const int r = F.r, m = 2 * r - 1;
    const double* d = order == 5 ? D5 : D7;
    double q[4], b[4];
    if (order == 5) weno5_parts(s, q, b); else weno7_parts(s, q, b);
    double alpha[4], sum = 0.0;
    for (int k = 0; k < r; ++k) {
        const double gk = eps + b[k];
        alpha[k] = d[k] / (gk * gk);
        sum += alpha[k];
    }
    double omega[4], fhat = 0.0;
    for (int k = 0; k < r; ++k) {
        omega[k] = alpha[k] / sum;
        fhat += omega[k] * q[k];
    }
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int k = 0; k < r; ++k) {
            double dbeta = 0.0;
            for (int i = 0; i < m; ++i) dbeta += 2.0 * F.B[k][j][i] * s[i];
            acc += omega[k] * F.Q[k][j] - 2.0 * omega[k] * (q[k] - fhat) / (eps + b[k]) * dbeta;
        }
        grad[j] = acc;
    }
}

// J[c][q] = d F_{d,c} / d u_q for one cell (complex step of the forward flux)
void flux_jacobian(int d, const double u[5], double J[5][5]) {
    const double h = 1e-30;
    for (int q = 0; q < 5; ++q) {
        cplx uc[5], v[3], p, nd, f[5];
        for (int c = 0; c < 5; ++c) uc[c] = cplx(u[c], c == q ? h : 0.0);
        con2prim(uc, v, p, nd, (long*)nullptr);
        flux(d, uc, v, p, f);
        for (int c = 0; c < 5; ++c) J[c][q] = f[c].imag() / h;
    }
}

// interior index of line position m along axis d (or -1 for analytic ghosts)
long line_target(const orc_grid& g, int d, const int ijk[3], int m) {
    const int nd = g.n[d];
    int c[3] = {ijk[0], ijk[1], ijk[2]};
    if (m >= 0 && m < nd) c[d] = m;
    else if (g.bc[d] == BC_PERIODIC) c[d] = ((m % nd) + nd) % nd;
    else if (g.bc[d] == BC_OUTFLOW) c[d] = m < 0 ? 0 : nd - 1;
    else return -1;
    return (long)cidx(g, c[0], c[1], c[2]);
}

// ubar += J(u)^T w at time t
void vjp_L(const orc_grid& g, double t, const double* u, const double* w, double* ubar) {
    const int r = g.order == 5 ? 3 : 4, G = r, m = 2 * r - 1;
    const size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
    for (int d = 0; d < 3; ++d) {
        const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        const int nd = g.n[d];
        const long nlines = (long)g.n[a1] * g.n[a2];
        // lines are independent except for periodic wrap onto themselves, so a
        // line's scatter stays inside the line: parallel over lines is safe
#pragma omp parallel for schedule(static)
        for (long line = 0; line < nlines; ++line) {
            int ijk[3];
            ijk[d] = 0;
            ijk[a1] = (int)(line % g.n[a1]);
            ijk[a2] = (int)(line / g.n[a1]);
            const int len = nd + 2 * G;
            std::vector<double> uc(5 * len), fp(5 * len), fm(5 * len), ap(5 * len, 0.0), am(5 * len, 0.0);
            for (int mm = -G; mm < nd + G; ++mm) {
                double ul[5], v[3], p, nden, f[5];
                line_cell(g, t, u, d, ijk, mm, ul);
                con2prim(ul, v, p, nden, (long*)nullptr);
                flux(d, ul, v, p, f);
                for (int c = 0; c < 5; ++c) {
                    uc[c * len + mm + G] = ul[c];
                    fp[c * len + mm + G] = 0.5 * (f[c] + ul[c]);
                    fm[c * len + mm + G] = 0.5 * (f[c] - ul[c]);
                }
            }
            for (int i = -1; i < nd; ++i) {
                for (int c = 0; c < 5; ++c) {
                    const double wr = i + 1 < nd ? w[c * ncell + line_target(g, d, ijk, i + 1)] : 0.0;
                    const double wl = i >= 0 ? w[c * ncell + line_target(g, d, ijk, i)] : 0.0;
                    const double gi = (wr - wl) / g.h[d];
                    double sp[7], sm[7], gp[7], gm[7];
                    for (int o = 0; o < m; ++o) {
                        sp[o] = fp[c * len + (i - r + 1 + o) + G];
                        sm[o] = fm[c * len + (i + r - o) + G];
                    }
                    weno_grad(g.order, sp, g.eps, gp);
                    weno_grad(g.order, sm, g.eps, gm);
                    for (int o = 0; o < m; ++o) {
                        ap[c * len + (i - r + 1 + o) + G] += gi * gp[o];
                        am[c * len + (i + r - o) + G] += gi * gm[o];
                    }
                }
            }
            for (int mm = -G; mm < nd + G; ++mm) {
                const long tgt = line_target(g, d, ijk, mm);
                if (tgt < 0) continue;
                double ul[5], J[5][5];
                for (int c = 0; c < 5; ++c) ul[c] = uc[c * len + mm + G];
                flux_jacobian(d, ul, J);
                for (int q = 0; q < 5; ++q) {
                    double acc = 0.5 * (ap[q * len + mm + G] - am[q * len + mm + G]);
                    for (int c = 0; c < 5; ++c)
                        acc += 0.5 * (ap[c * len + mm + G] + am[c * len + mm + G]) * J[c][q];
                    ubar[q * ncell + tgt] += acc;
                }
            }
        }
    }
}

}  // namespace

extern "C" {

// out = J(u)^T w for L at time t (fields [5][nz][ny][nx]).
int orc_vjp_L(const orc_grid* g, double t, const double* u, const double* w, double* out) {
    if (!grid_ok_adjoint(g)) return -1;
    const size_t N = 5 * (size_t)g->n[0] * g->n[1] * g->n[2];
    for (size_t q = 0; q < N; ++q) out[q] = 0.0;
    vjp_L(*g, t, u, w, out);
    return 0;
}

// Adjoint of one SSP-RK3 step from u (time t): ubar_out = (d u_{n+1} / d u_n)^T ubar_in.
// Stage states are recomputed; the stage adjoints are
//   b2 = 2/3 b3 + 2/3 dt J(u2)^T b3,  b1 = 1/4 b2 + 1/4 dt J(u1)^T b2,
//   b0 = 1/3 b3 + 3/4 b2 + b1 + dt J(u)^T b1,  with b3 = ubar_in.
int orc_vjp_step(const orc_grid* g, double t, double dt, const double* u, const double* ubar_in,
                 double* ubar_out) {
    if (!grid_ok_adjoint(g)) return -1;
    const size_t N = 5 * (size_t)g->n[0] * g->n[1] * g->n[2];
    std::vector<double> L(N), u1(N), u2(N), b2(N), b1(N), tmp(N);
    apply_L(*g, t, u, L.data(), (long*)nullptr);
    for (size_t q = 0; q < N; ++q) u1[q] = u[q] + dt * L[q];
    apply_L(*g, t + dt, u1.data(), L.data(), (long*)nullptr);
    for (size_t q = 0; q < N; ++q) u2[q] = 0.75 * u[q] + 0.25 * (u1[q] + dt * L[q]);
    std::fill(tmp.begin(), tmp.end(), 0.0);
    vjp_L(*g, t + 0.5 * dt, u2.data(), ubar_in, tmp.data());
    for (size_t q = 0; q < N; ++q) b2[q] = (2.0 / 3.0) * ubar_in[q] + (2.0 / 3.0) * dt * tmp[q];
    std::fill(tmp.begin(), tmp.end(), 0.0);
    vjp_L(*g, t + dt, u1.data(), b2.data(), tmp.data());
    for (size_t q = 0; q < N; ++q) b1[q] = 0.25 * b2[q] + 0.25 * dt * tmp[q];
    std::fill(tmp.begin(), tmp.end(), 0.0);
    vjp_L(*g, t, u, b1.data(), tmp.data());
    for (size_t q = 0; q < N; ++q)
        ubar_out[q] = (1.0 / 3.0) * ubar_in[q] + 0.75 * b2[q] + b1[q] + dt * tmp[q];
    return 0;
}

// Directional derivative of one SSP-RK3 step by the complex step.
int orc_jvp_step(const orc_grid* g, double t, double dt, const double* u, const double* v,
                 double* jv) {
    if (!grid_ok_adjoint(g)) return -1;
    const double h = 1e-30;
    const size_t N = 5 * (size_t)g->n[0] * g->n[1] * g->n[2];
    std::vector<cplx> uc(N);
    for (size_t q = 0; q < N; ++q) uc[q] = cplx(u[q], h * v[q]);
    rk3_step(*g, t, dt, uc.data(), (long*)nullptr);
    for (size_t q = 0; q < N; ++q) jv[q] = uc[q].imag() / h;
    return 0;
}

}  // extern "C"
