"""Exact solution of the relativistic shock tube of an ideal gas, for the
tests (independent of the oracle and of the GPU code).

Fluid: p = (gamma - 1)(e - n) with unit rest mass per charge n, enthalpy per
charge h = (e + p) / n, sound speed c_s^2 = gamma p / (e + p).  Both states at
rest, left pressure above right: a rarefaction moves left, then a contact, then
a shock moves right.  Derived here from the conservation laws of E, M and N:

* rarefaction: the entropy p n^-gamma and the Riemann invariant
  atanh(v) + int c_s dn / n are constant across it (characteristic form of the
  isentropic equations, dp = c_s^2 (e + p) dn / n); inside the fan x / t equals
  the left-going characteristic speed (v - c_s) / (1 - v c_s);
* shock: the jump conditions F(U_b) - F(U_a) = V_s (U_b - U_a) for
  U = (E, M, N), F = (M, M v + p, N v).  Their combination without the
  velocities (the relativistic Hugoniot, h_b^2 - h_a^2 = (h_b / n_b + h_a / n_a)
  (p_b - p_a)) gives n_b, the N and M conditions then give v_b (a quadratic
  in its Lorentz factor) and V_s, and the E condition is left as a check of the
  solution (energy_residual);
* the star pressure makes the two velocities equal.
"""
import numpy as np
from scipy import integrate, optimize


def state(n, p, v, gam):
    """Conserved (E, M, N) and fluxes (M, M v + p, N v) of a state."""
    e = n + p / (gam - 1.0)
    w2 = 1.0 / (1.0 - v * v)
    M = (e + p) * w2 * v
    U = np.array([(e + p) * w2 - p, M, n * np.sqrt(w2)])
    F = np.array([M, M * v + p, U[2] * v])
    return U, F


def sound_speed(n, p, gam):
    e = n + p / (gam - 1.0)
    return np.sqrt(gam * p / (e + p))


def rarefaction(nL, pL, p, gam):
    """(n, v) reached from the left state at rest by the left-moving rarefaction
    down to pressure p."""
    K = pL / nL ** gam
    n = nL * (p / pL) ** (1.0 / gam)
    G, _ = integrate.quad(lambda m: sound_speed(m, K * m ** gam, gam) / m, n, nL, epsabs=0.0,
                          epsrel=1e-13, limit=400)
    return n, np.tanh(G)


def shock(nR, pR, p, gam):
    """(n_b, v_b, V_s) behind the right-moving shock into the right state at rest
    that raises the pressure to p."""
    ha = 1.0 + gam / (gam - 1.0) * pR / nR

    def hugoniot(nb):
        hb = 1.0 + gam / (gam - 1.0) * p / nb
        return (hb * hb - ha * ha) - (hb / nb + ha / nR) * (p - pR)

    lo, hi = nR * (1.0 + 1e-12), nR * 2.0
    while hugoniot(hi) * hugoniot(lo) > 0.0:
        hi *= 2.0
        if hi > 1e12 * nR:
            raise RuntimeError("no compression on the Hugoniot")
    nb = optimize.brentq(hugoniot, lo, hi, xtol=1e-15 * nR, rtol=1e-15, maxiter=500)
    # N and M conditions with the state ahead at rest: V_s = N_b v_b / (N_b - N_a)
    # and w_b (W^2 - 1) n_a = (p - pR)(n_b W - n_a), w = e + p, a quadratic in the
    # Lorentz factor W of the state behind with exactly one positive root
    wb = nb + p / (gam - 1.0) + p
    dp = p - pR
    W = (dp * nb + np.sqrt(dp * dp * nb * nb + 4.0 * wb * nR * nR * (wb - dp))) / (2.0 * wb * nR)
    vb = np.sqrt(1.0 - 1.0 / (W * W))
    Vs = nb * W * vb / (nb * W - nR)
    return nb, vb, Vs


def energy_residual(nR, pR, p, nb, vb, Vs, gam):
    """Relative residual of the E jump condition (not used to build the shock)."""
    Ua, Fa = state(nR, pR, 0.0, gam)
    Ub, Fb = state(nb, p, vb, gam)
    return abs((Fb[0] - Fa[0]) - Vs * (Ub[0] - Ua[0])) / max(abs(Fb[0]), abs(Ub[0]))


def star_state(nL, pL, nR, pR, gam):
    """Star pressure and velocity, densities on both sides of the contact, shock
    speed and the rarefaction tail speed."""
    def mismatch(p):
        return rarefaction(nL, pL, p, gam)[1] - shock(nR, pR, p, gam)[1]

    ps = optimize.brentq(mismatch, pR * (1.0 + 1e-9), pL * (1.0 - 1e-9), xtol=1e-16 * pL, rtol=1e-15,
                         maxiter=500)
    nl, vs = rarefaction(nL, pL, ps, gam)
    nr, vr, Vs = shock(nR, pR, ps, gam)
    cs = sound_speed(nl, ps, gam)
    return {"p": ps, "v": 0.5 * (vs + vr), "n_left": nl, "n_right": nr, "v_shock": Vs,
            "xi_tail": (vs - cs) / (1.0 - vs * cs), "xi_head": -sound_speed(nL, pL, gam)}


def sample(nL, pL, nR, pR, gam, xi):
    """(n, p, v) of the exact solution at x / t = xi (an array)."""
    s = star_state(nL, pL, nR, pR, gam)
    K = pL / nL ** gam
    out = np.empty((3, len(xi)))
    for i, q in enumerate(xi):
        if q < s["xi_head"]:
            out[:, i] = nL, pL, 0.0
        elif q < s["xi_tail"]:
            def fan(n):
                n0, v = rarefaction(nL, pL, K * n ** gam, gam)
                c = sound_speed(n, K * n ** gam, gam)
                return (v - c) / (1.0 - v * c) - q
            n = optimize.brentq(fan, s["n_left"], nL, xtol=1e-15, rtol=1e-13)
            out[:, i] = n, K * n ** gam, rarefaction(nL, pL, K * n ** gam, gam)[1]
        elif q < s["v"]:
            out[:, i] = s["n_left"], s["p"], s["v"]
        elif q < s["v_shock"]:
            out[:, i] = s["n_right"], s["p"], s["v"]
        else:
            out[:, i] = nR, pR, 0.0
    return out
