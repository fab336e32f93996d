"""Exact ellipsoidal solution of the conformal fluid (p = e/3) with a passive
charge, for the tests (independent of the oracle and of the GPU code).

Velocity u^mu = x^mu / tau (tau^2 = t^2 - r^2, so v = x / t) and energy density
e = e0 (t0 / tau)^4: the Hubble-like flow.  Its flow lines are x = v t with v
fixed, so s = (x^2/a^2 + y^2/b^2 + z^2/c^2) / t^2 is constant along them
(u.d s = 0, s being homogeneous of degree zero in (t, x)); with d_mu u^mu = 3/tau
and u.d tau = 1, any n = (t0 / tau)^3 F(s) satisfies d_mu (n u^mu) = 0.  The
stress tensor of the conformal fluid does not depend on n, so e and v are
unchanged.  Here F(s) = n0 + n1 exp(-s/2): an ellipsoidal charge on the uniform
background that the analytic (Hubble) ghost cells carry, which is exact there
wherever n1 exp(-s/2) is negligible.
"""
import numpy as np


def cell_centres(spec):
    """(X, Y, Z) of the cell centres, arrays of shape (nz, ny, nx)."""
    nx, ny, nz = spec["shape"]
    axes = [spec["c0"][d] + spec["h"][d] * np.arange(m) for d, m in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return X, Y, Z


def primitives(spec, t, xyz=None):
    """(e, vx, vy, vz, n) of the exact solution at time t (shape (5, nz, ny, nx))."""
    t0, e0, n0 = spec["hub"]
    n1, a, b, c = spec["ellipsoid"]
    X, Y, Z = cell_centres(spec) if xyz is None else xyz
    tau = np.sqrt(t * t - (X * X + Y * Y + Z * Z))
    s = (X * X / (a * a) + Y * Y / (b * b) + Z * Z / (c * c)) / (t * t)
    out = np.empty((5,) + X.shape)
    out[0] = e0 * (t0 / tau) ** 4
    out[1], out[2], out[3] = X / t, Y / t, Z / t
    out[4] = (t0 / tau) ** 3 * (n0 + n1 * np.exp(-0.5 * s))
    return out


def ghost_mismatch(spec, t_end):
    """Largest n1 exp(-s/2) over the ghost cells for times up to t_end: what the
    Hubble ghost cells, which carry n0 only, leave out.  s grows outwards and
    falls with t, so the first ghost layer at t_end is the worst case."""
    n1, a, b, c = spec["ellipsoid"]
    nx, ny, nz = spec["shape"]
    worst = 0.0
    for d, (m, w) in enumerate(zip((nx, ny, nz), (a, b, c))):
        lo = abs(spec["c0"][d] - spec["h"][d])                  # first ghost centre below
        hi = abs(spec["c0"][d] + m * spec["h"][d])              # first ghost centre above
        x = min(lo, hi)
        worst = max(worst, n1 * np.exp(-0.5 * (x / (w * t_end)) ** 2))
    return worst
