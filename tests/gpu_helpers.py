"""Shared helpers of the GPU tests: run a workload through the C ABI and
through the oracle on identical inputs, and compare per field."""
import numpy as np

import oracle
from paper_1604_03360_amd import inputs


def rh_module():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU visible")
    from paper_1604_03360_amd import rh
    rh.library()   # raises ImportError if the HIP library is missing
    return rh


def gpu_hydro(spec, precision, order=None):
    rh = rh_module()
    h = rh.Hydro.from_spec(spec, precision=precision, scheme=order or spec["order"])
    h.set_primitive(spec["prim"])
    return h


def gpu_L(spec, precision, order=None, t=None):
    h = gpu_hydro(spec, precision, order)
    L = h.apply_L(spec["t0"] if t is None else t).double().cpu().numpy()
    h.close()
    return L


def gpu_steps(spec, precision, nsteps, order=None, dt=None):
    h = gpu_hydro(spec, precision, order)
    t = h.step(dt or spec["dt"], nsteps)
    u = h.get()
    tot, cnt = h.totals()
    h.close()
    return u, t, np.array(tot), cnt


def oracle_L(spec, order=None, t=None):
    g = oracle.grid_from_spec(spec, order=order)
    return oracle.apply_L(g, oracle.prim2con(spec["prim"]), spec["t0"] if t is None else t)


def oracle_steps(spec, nsteps, order=None, dt=None):
    g = oracle.grid_from_spec(spec, order=order)
    u, t = oracle.step(g, oracle.prim2con(spec["prim"]), dt or spec["dt"], nsteps, t=spec["t0"])
    return u, t


def field_errors(got, ref):
    """Per-field normalised L-infinity error max|got - ref| / max|ref| (fields whose
    reference is identically zero report the plain max|got|)."""
    got = np.asarray(got, dtype=np.float64).reshape(5, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(5, -1)
    out = []
    for f in range(5):
        scale = np.abs(ref[f]).max()
        diff = np.abs(got[f] - ref[f]).max()
        out.append(diff / scale if scale > 0 else diff)
    return np.array(out)


def L_errors(got, ref, u, h_min):
    """Errors of L(u) per field, normalised by max(max|L_ref|, max|u|/h): L is a
    difference of face fluxes whose size is set by |u| (|f+-| <= |u| + p), so
    max|u|/h bounds what rounding can leave in L even where L itself cancels to
    nearly zero (e.g. the pure dissipation term of a fluid at rest)."""
    got = np.asarray(got, dtype=np.float64).reshape(5, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(5, -1)
    u = np.asarray(u, dtype=np.float64).reshape(5, -1)
    out = []
    for f in range(5):
        scale = max(np.abs(ref[f]).max(), np.abs(u[f]).max() / h_min)
        out.append(np.abs(got[f] - ref[f]).max() / scale if scale > 0 else np.abs(got[f]).max())
    return np.array(out)


def assert_fields_close(got, ref, tol, what=""):
    err = field_errors(got, ref)
    assert np.all(np.isfinite(got)), what + ": non-finite values"
    assert np.all(err <= tol), "%s: normalised L-inf errors %s exceed %g" % (what, err, tol)
    return err


SMALL_CASES = {
    # ragged shapes spanning several tiles and segments on every axis
    "smooth_periodic": lambda o: inputs.random_smooth((70, 37, 23), h=0.1, seed=1, order=o),
    "smooth_outflow": lambda o: inputs.random_smooth((33, 20, 45), h=0.07, seed=2, order=o,
                                                     bc=(inputs.BC_OUTFLOW,) * 3),
    "hubble": lambda o: inputs.hubble(n=24, order=o, half_width=3.0),
    "blob": lambda o: inputs.blob(h=0.25, order=o, shape=(64, 48, 40)),
    "sod": lambda o: inputs.sod(nx=400, order=o),
    "hotspots": lambda o: inputs.hotspots(3, size=48, order=o),
}
