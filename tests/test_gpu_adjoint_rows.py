"""The whole-row x adjoint (periodic x rows of 32, 64, 96, 128, 192 or 256
cells) against the FP64 oracle's adjoint: FP64 (1e-12) and FP32 (5e-5), WENO5
and WENO7, row counts that leave part of the last block empty, non-periodic and
analytic y/z boundaries; the adjoint of a step; and bitwise equality with the
tiled x adjoint (forced in a child process with RH_ADJ_XROW=0)."""
import numpy as np
import pytest

import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import rh_module

pytestmark = pytest.mark.gpu

P, O, H = inputs.BC_PERIODIC, inputs.BC_OUTFLOW, inputs.BC_HUBBLE


def hubble_periodic_x(o):
    spec = inputs.hubble(n=32, order=o, half_width=3.0)
    spec["bc"] = (P, H, H)
    return spec


CASES = {
    # 15 rows: the second block of eight rows holds one empty row
    "rows_32_hubble_yz": hubble_periodic_x,
    "rows_64_outflow_yz": lambda o: inputs.random_smooth((64, 7, 3), h=0.1, seed=91, bc=(P, O, O), order=o),
    "rows_96": lambda o: inputs.random_smooth((96, 5, 3), h=0.1, seed=92, order=o),
    "rows_128_outflow_z": lambda o: inputs.random_smooth((128, 3, 3), h=0.05, seed=93, bc=(P, P, O), order=o),
    "rows_192_one_row": lambda o: inputs.random_smooth((192, 1, 1), h=0.05, seed=94, order=o),
    "rows_256": lambda o: inputs.random_smooth((256, 3, 2), h=0.05, seed=95, order=o),
}


def vjp_errors(got, ref, w, h):
    """Per-field max|got - ref| normalised by max(max|ref|, max|w|/h)."""
    got = np.asarray(got, np.float64).reshape(5, -1)
    ref = np.asarray(ref, np.float64).reshape(5, -1)
    scale = max(np.abs(ref).max(), np.abs(w).max() / h)
    return np.abs(got - ref).max(axis=1) / scale


def _setup(rh, spec, prec, seed=7):
    h = rh.Hydro.from_spec(spec, precision=prec)
    u = oracle.prim2con(spec["prim"])
    w = np.random.default_rng(seed).normal(size=u.shape)
    return h, u, w


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_row_vjp_fp64_matches_oracle(case, order):
    rh = rh_module()
    spec = CASES[case](order)
    assert spec["bc"][0] == P
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    t = spec["t0"] + 0.2
    got = h.vjp(u, w, t=t).cpu().numpy()
    h.close()
    ref = oracle.vjp_L(oracle.grid_from_spec(spec), u, w, t=t)
    err = vjp_errors(got, ref, w, min(spec["h"]))
    print(case, order, err, flush=True)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_row_vjp_fp32_close_to_oracle(case, order):
    rh = rh_module()
    spec = CASES[case](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP32)
    t = spec["t0"] + 0.2
    got = h.vjp(u, w, t=t).double().cpu().numpy()
    h.close()
    u32 = u.astype(np.float32).astype(np.float64)
    w32 = w.astype(np.float32).astype(np.float64)
    ref = oracle.vjp_L(oracle.grid_from_spec(spec), u32, w32, t=t)
    err = vjp_errors(got, ref, w32, min(spec["h"]))
    print(case, order, "fp32", err, flush=True)
    assert np.all(err <= 5e-5), err


@pytest.mark.parametrize("order", [5, 7])
def test_row_step_vjp_fp64_matches_oracle(order):
    rh = rh_module()
    spec = CASES["rows_64_outflow_yz"](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    dt, t = spec["dt"], spec["t0"]
    got = h.step_vjp(u, w, dt, t=t).cpu().numpy()
    h.close()
    ref = oracle.vjp_step(oracle.grid_from_spec(spec), u, w, dt, t=t)
    err = np.abs(got - ref).reshape(5, -1).max(axis=1) / np.abs(ref).max()
    print(order, err, flush=True)
    assert np.all(err <= 1e-12), err


TILED_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import rh_module
rh = rh_module()
for o in (5, 7):
    for shape in ((64, 11, 5), (96, 7, 3)):
        spec = inputs.random_smooth(shape, h=0.1, seed=96, bc=(0, 1, 0), order=o)
        u = oracle.prim2con(spec["prim"])
        w = np.random.default_rng(9).normal(size=u.shape)
        for name, prec in (("fp64", rh.RH_PREC_FP64), ("fp32", rh.RH_PREC_FP32)):
            h = rh.Hydro.from_spec(spec, precision=prec)
            got = h.vjp(u, w, t=0.1).cpu().numpy()
            h.close()
            np.save("%s_%s_%d_%d.npy" % (sys.argv[2], name, o, shape[0]), got)
"""


def test_row_vjp_is_bitwise_the_tiled_kernel(tmp_path):
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "tiled")
    env = dict(os.environ, RH_ADJ_XROW="0")
    r = subprocess.run([sys.executable, "-c", TILED_SCRIPT, root, out], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    rh = rh_module()
    for o in (5, 7):
        for shape in ((64, 11, 5), (96, 7, 3)):
            spec = inputs.random_smooth(shape, h=0.1, seed=96, bc=(P, O, P), order=o)
            u = oracle.prim2con(spec["prim"])
            w = np.random.default_rng(9).normal(size=u.shape)
            for name, prec in (("fp64", rh.RH_PREC_FP64), ("fp32", rh.RH_PREC_FP32)):
                h = rh.Hydro.from_spec(spec, precision=prec)
                got = h.vjp(u, w, t=0.1).cpu().numpy()
                h.close()
                tiled = np.load("%s_%s_%d_%d.npy" % (out, name, o, shape[0]))
                assert np.array_equal(got, tiled), (name, o, shape, np.abs(got - tiled).max())
