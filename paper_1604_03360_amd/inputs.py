"""Seeded synthetic workloads (initial primitive fields and grid descriptions).

This module holds no arithmetic of the numerical method: it only samples the
initial primitive fields (e, vx, vy, vz, n) of the test problems on cell centres
and describes the grids.  The GPU library and the CPU oracle each convert these
primitives to conserved variables themselves, so both sides start from the same
numbers and share nothing else.

Workloads (sizes, steps and boundary conditions are readings of the paper's
Sec. 3 test problems, which it gives without numbers):
  * ``sod``       1+1D shock tube on x in [-1, 1] (Sec. 3, Fig. 1).
  * ``hubble``    3+1D Hubble-like expansion on [-5, 5]^3 (Sec. 3, Fig. 3).
  * ``blob``      3+1D ellipsoidal Gaussian energy blob at rest, periodic; a
                  synthetic stand-in for the ellipsoidal-flow run (Sec. 3, Fig. 2).
  * ``hotspots``  event-by-event initial states: Poisson-many Gaussian hot spots
                  on a dilute background (motivation of Sec. 1's introduction).
"""
import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_HUBBLE = 0, 1, 2
CFL = 0.4


def _centres(n, h, c0):
    return c0 + h * np.arange(n, dtype=np.float64)


def _spec(name, shape, h, c0, bc, prim, order=5, t0=0.0, nsteps=1, hub=(10.0, 1.0, 0.5)):
    nx, ny, nz = shape
    assert prim.shape == (5, nz, ny, nx)
    live = [h[a] for a in range(3) if shape[a] > 1] or [h[0]]
    return {
        "name": name, "shape": tuple(int(s) for s in shape), "h": tuple(float(v) for v in h),
        "c0": tuple(float(v) for v in c0), "bc": tuple(int(b) for b in bc), "order": int(order),
        "eps": 1e-6, "hub": tuple(float(v) for v in hub), "t0": float(t0),
        "dt": CFL * min(live), "nsteps": int(nsteps), "prim": np.ascontiguousarray(prim),
    }


def sod(nx=400, order=5, nsteps=None):
    """Relativistic Sod tube: e=1, n=1 for x<0; e=0.1, n=0.125 for x>0; at rest."""
    h = 2.0 / nx
    x = _centres(nx, h, -1.0 + 0.5 * h)
    prim = np.zeros((5, 1, 1, nx))
    left = x < 0.0
    prim[0, 0, 0] = np.where(left, 1.0, 0.1)
    prim[4, 0, 0] = np.where(left, 1.0, 0.125)
    steps = nsteps if nsteps is not None else int(round(0.4 / (CFL * h)))
    return _spec("sod", (nx, 1, 1), (h, h, h), (-1.0 + 0.5 * h, 0.0, 0.0),
                 (BC_OUTFLOW,) * 3, prim, order=order, nsteps=steps)


def hubble(n=128, order=5, t0=10.0, half_width=5.0, nsteps=100, e0=1.0, n0=0.5, shape=None):
    """Hubble-like flow u^mu = x^mu/tau at t0 with e = e0 (t0/tau)^4, n = n0 (t0/tau)^3."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    h = 2.0 * half_width / shape[0]
    c0 = -half_width + 0.5 * h
    x = _centres(shape[0], h, c0)
    y = _centres(shape[1], h, c0)
    z = _centres(shape[2], h, c0)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    tau = np.sqrt(t0 * t0 - (X * X + Y * Y + Z * Z))
    prim = np.empty((5,) + X.shape)
    prim[0] = e0 * (t0 / tau) ** 4
    prim[1] = X / t0
    prim[2] = Y / t0
    prim[3] = Z / t0
    prim[4] = n0 * (t0 / tau) ** 3
    return _spec("hubble", shape, (h, h, h), (c0, c0, c0), (BC_HUBBLE,) * 3, prim,
                 order=order, t0=t0, nsteps=nsteps, hub=(t0, e0, n0))


def ellipsoidal(n=128, order=5, t0=10.0, half_width=5.0, nsteps=100, e0=1.0, n0=0.5, n1=1.0,
                axes=(0.03, 0.04, 0.05), shape=None):
    """Hubble-like flow carrying an ellipsoidal charge: e and v as in hubble(), and
    n = (t0/tau)^3 (n0 + n1 exp(-s/2)), s = (x^2/a^2 + y^2/b^2 + z^2/c^2) / t^2 at
    t = t0, with (a, b, c) = axes (speeds: the ellipsoid's semi-axes grow as a t)."""
    spec = hubble(n=n, order=order, t0=t0, half_width=half_width, nsteps=nsteps, e0=e0, n0=n0,
                  shape=shape)
    nx, ny, nz = spec["shape"]
    h, c0 = spec["h"][0], spec["c0"][0]
    Z, Y, X = np.meshgrid(_centres(nz, h, c0), _centres(ny, h, c0), _centres(nx, h, c0), indexing="ij")
    a, b, c = axes
    tau = np.sqrt(t0 * t0 - (X * X + Y * Y + Z * Z))
    s = (X * X / (a * a) + Y * Y / (b * b) + Z * Z / (c * c)) / (t0 * t0)
    spec["prim"][4] = (t0 / tau) ** 3 * (n0 + n1 * np.exp(-0.5 * s))
    spec["name"] = "ellipsoidal"
    spec["ellipsoid"] = (float(n1), float(a), float(b), float(c))
    return spec


def _centred_axis(n, h):
    return _centres(n, h, -(0.5 * n - 0.5) * h)


def blob(n=256, h=0.1, order=5, nsteps=200, shape=None):
    """Ellipsoidal Gaussian at rest: e = 1e-3 + 20 exp(-x^2/8 - y^2/18 - z^2/32), n = e^(3/4)."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    x = _centred_axis(shape[0], h)
    y = _centred_axis(shape[1], h)
    z = _centred_axis(shape[2], h)
    gx = np.exp(-x * x / (2 * 2.0 ** 2))
    gy = np.exp(-y * y / (2 * 3.0 ** 2))
    gz = np.exp(-z * z / (2 * 4.0 ** 2))
    prim = np.zeros((5, shape[2], shape[1], shape[0]))
    prim[0] = 1e-3 + 20.0 * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    prim[4] = prim[0] ** 0.75
    c0 = tuple(-(0.5 * s - 0.5) * h for s in shape)
    return _spec("blob", shape, (h, h, h), c0, (BC_PERIODIC,) * 3, prim, order=order,
                 nsteps=nsteps)


HOTSPOT_SIZES = (64, 96, 128, 160)


def hotspots(event, size=None, h=0.15, order=5, nsteps=100, mean_spots=50, sigma=0.5,
             mean_amp=5.0, centre_sd=3.0, seed_base=1604):
    """One event: K ~ Poisson(50) Gaussian hot spots (sigma 0.5, amplitude ~ Exp(mean 5),
    centres ~ N(0, 3^2) per axis) on e = 1e-3, at rest, n = e^(3/4), periodic cube.

    Draw order from ``np.random.default_rng([seed_base, event])``: cube size (uniform
    over 64, 96, 128, 160 unless given), K, then per spot its amplitude and centre.
    Distances use the minimum image so that the field is periodic."""
    rng = np.random.default_rng([seed_base, int(event)])
    drawn = int(rng.choice(HOTSPOT_SIZES))
    n = int(size) if size is not None else drawn
    K = int(rng.poisson(mean_spots))
    amps = rng.exponential(mean_amp, K)
    centres = rng.normal(0.0, centre_sd, (K, 3))
    box = n * h
    x = _centred_axis(n, h)
    e = np.full((n, n, n), 1e-3)

    def g1(c):
        d = x - c
        d = d - box * np.round(d / box)
        return np.exp(-d * d / (2.0 * sigma * sigma))

    if K:
        # sum of K separable Gaussians as one (n x K) @ (K x n^2) product
        gx = np.stack([g1(c) for c in centres[:, 0]])
        gy = np.stack([g1(c) for c in centres[:, 1]])
        gz = np.stack([g1(c) for c in centres[:, 2]])
        zk = (gz * amps[:, None]).T                        # (n, K)
        kyx = (gy[:, :, None] * gx[:, None, :]).reshape(K, n * n)
        e += (zk @ kyx).reshape(n, n, n)
    prim = np.zeros((5, n, n, n))
    prim[0] = e
    prim[4] = e ** 0.75
    c0 = -(0.5 * n - 0.5) * h
    spec = _spec("hotspots", (n, n, n), (h, h, h), (c0, c0, c0), (BC_PERIODIC,) * 3, prim,
                 order=order, nsteps=nsteps)
    spec["event"] = int(event)
    spec["n_spots"] = K
    return spec


def batch(n_events=64, **kw):
    """The event-by-event ensemble: events 0 .. n_events-1, sizes drawn per event."""
    return [hotspots(k, **kw) for k in range(n_events)]


def batch_sizes(n_events=64, seed_base=1604):
    """Cube sizes of the ensemble without building the fields."""
    out = []
    for k in range(n_events):
        rng = np.random.default_rng([seed_base, k])
        out.append(int(rng.choice(HOTSPOT_SIZES)))
    return out


def diff_event(n=96, **kw):
    """Single seeded event for the differentiable run (seed 1000, fixed size 96)."""
    return hotspots(1000, size=n, nsteps=50, **kw)


def random_smooth(shape, h=0.1, seed=0, amp_v=0.3, bc=(BC_PERIODIC,) * 3, order=5):
    """Smooth random periodic primitive field (sums of low Fourier modes); used for
    parity cases that exercise all three velocity components."""
    rng = np.random.default_rng([seed, 77])
    nx, ny, nz = shape
    prim = np.zeros((5, nz, ny, nx))
    ax = [2 * np.pi * np.arange(s) / s for s in shape]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")

    def field():
        acc = np.zeros_like(X)
        for _ in range(3):
            kx, ky, kz = rng.integers(0, 3, 3)
            acc += rng.normal() * np.sin(kx * X + ky * Y + kz * Z + rng.uniform(0, 2 * np.pi))
        return acc / 3.0

    prim[0] = 1.0 + 0.5 * np.tanh(field())
    vx, vy, vz = field(), field(), field()
    vmag = np.sqrt(vx * vx + vy * vy + vz * vz) + 1e-12
    scale = amp_v * np.tanh(vmag) / vmag
    prim[1], prim[2], prim[3] = vx * scale, vy * scale, vz * scale
    prim[4] = 0.5 + 0.25 * np.tanh(field())
    c0 = tuple(-(0.5 * s - 0.5) * h for s in shape)
    return _spec("random_smooth", shape, (h, h, h), c0, bc, prim, order=order)


def with_scheme(spec, **opts):
    """A copy of a workload spec with scheme options attached: order (5, 7, or 2 for
    MUSTA-FORCE), limiter, musta_k, musta_cfl, lf_local, eos, gamma."""
    out = dict(spec)
    out.update(opts)
    return out


def hot_gas(spec):
    """A copy of a workload spec whose energy density is raised by twice the charge
    density (e -> e + 2n), so that an ideal gas of unit rest mass per charge has
    positive pressure everywhere."""
    out = dict(spec)
    prim = spec["prim"].copy()
    prim[0] = prim[0] + 2.0 * prim[4]
    out["prim"] = prim
    return out


def sod_ideal(nx=400, nsteps=None):
    """Relativistic shock tube of an ideal gas (gamma = 5/3) on x in [-1, 1], at rest:
    x < 0: e = 29.995, n = 10; x > 0: e = 1.0000015, n = 1 (pressures 13.33 and 1e-6
    for gamma = 5/3, the first relativistic shock tube of Marti and Mueller).
    Outflow boundaries; t = 0.4 after the default number of steps."""
    h = 2.0 / nx
    x = _centres(nx, h, -1.0 + 0.5 * h)
    prim = np.zeros((5, 1, 1, nx))
    left = x < 0.0
    prim[0, 0, 0] = np.where(left, 29.995, 1.0000015)
    prim[4, 0, 0] = np.where(left, 10.0, 1.0)
    steps = nsteps if nsteps is not None else int(round(0.4 / (CFL * h)))
    spec = _spec("sod_ideal", (nx, 1, 1), (h, h, h), (-1.0 + 0.5 * h, 0.0, 0.0),
                 (BC_OUTFLOW,) * 3, prim, nsteps=steps)
    spec["eos"] = 1
    spec["gamma"] = 5.0 / 3.0
    return spec
