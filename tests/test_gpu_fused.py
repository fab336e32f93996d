"""The fused x-y sweep (WENO5 and WENO7 grids with a periodic x
axis of 64..256 cells, a multiple of 64) against the FP64 oracle: non-periodic
and analytic y boundaries, a grid with one z plane (the fused launch then
applies the stage combine), every admissible row length, FP64 (1e-12) and FP32
(2e-5); graph replays; bitwise equality with the separate sweeps."""
import numpy as np
import pytest

from paper_1604_03360_amd import inputs
from gpu_helpers import assert_fields_close, field_errors, gpu_steps, oracle_steps, rh_module

pytestmark = pytest.mark.gpu

P, O, H = inputs.BC_PERIODIC, inputs.BC_OUTFLOW, inputs.BC_HUBBLE


def hubble_periodic_x(o=5):
    spec = inputs.hubble(n=64, order=o, half_width=3.0)
    spec["bc"] = (P, H, H)
    return spec


CASES = {
    "outflow_yz": lambda o=5: inputs.random_smooth((64, 27, 13), h=0.1, seed=81, bc=(P, O, O), order=o),
    "one_z_plane": lambda o=5: inputs.random_smooth((128, 20, 1), h=0.1, seed=82, order=o),
    "rows_of_192": lambda o=5: inputs.random_smooth((192, 17, 5), h=0.05, seed=83, bc=(P, P, O), order=o),
    "rows_of_256": lambda o=5: inputs.random_smooth((256, 9, 3), h=0.05, seed=84, order=o),
    "hubble_y": hubble_periodic_x,
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision,tol,order", [("fp64", 1e-12, 5), ("fp64", 1e-12, 7), ("fp32", 2e-5, 5),
                                                 ("fp32", 2e-5, 7)])
def test_fused_xy_matches_oracle(case, precision, tol, order):
    rh = rh_module()
    spec = CASES[case](order)
    assert spec["shape"][0] % 64 == 0 and spec["bc"][0] == P
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    nsteps = 3
    got, tg, _, cnt = gpu_steps(spec, prec, nsteps)
    ref, tr = oracle_steps(spec, nsteps)
    assert tg == pytest.approx(tr, abs=1e-12)
    print(case, precision, order, field_errors(got, ref), flush=True)
    assert_fields_close(got, ref, tol, "%s %s WENO%d" % (case, precision, order))
    assert cnt[1] == 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_xy_graph_replay_matches_eager(precision):
    """Steps replayed from the captured step graph (which holds the fused launch)
    equal eager steps bitwise, with eager work between the replays."""
    import torch
    from gpu_helpers import gpu_hydro
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    spec = CASES["outflow_yz"]()
    dt = spec["dt"]
    eager = gpu_hydro(spec, prec)
    for _ in range(3):
        eager.step(dt, 2)
    graphed = gpu_hydro(spec, prec)
    rh.rh_set_graph(graphed.plan, True)
    for _ in range(3):
        graphed.step(dt, 2)
        scratch = torch.randn(1 << 18, device="cuda")
        scratch.mul_(3.0).sum().item()
        torch.cuda.synchronize()
    assert np.array_equal(graphed.get(), eager.get())
    eager.close()
    graphed.close()


SPLIT_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
from paper_1604_03360_amd import inputs
from gpu_helpers import gpu_steps, rh_module
rh = rh_module()
for o in (5, 7):
    spec = inputs.random_smooth((128, 27, 11), h=0.1, seed=85, bc=(0, 1, 0), order=o)
    for name, prec in (("fp64", rh.RH_PREC_FP64), ("fp32", rh.RH_PREC_FP32)):
        got, _, _, _ = gpu_steps(spec, prec, 3)
        np.save("%s_%s_%d.npy" % (sys.argv[2], name, o), got)
"""


def test_fused_xy_is_bitwise_the_split_sweeps(tmp_path):
    """The fused launch gives bitwise the state of the separate x and y sweeps
    (forced in a child process with RH_FUSE_XY=0)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "split")
    env = dict(os.environ, RH_FUSE_XY="0")
    r = subprocess.run([sys.executable, "-c", SPLIT_SCRIPT, root, out], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    rh = rh_module()
    for o in (5, 7):
        spec = inputs.random_smooth((128, 27, 11), h=0.1, seed=85, bc=(P, O, P), order=o)
        for name, prec in (("fp64", rh.RH_PREC_FP64), ("fp32", rh.RH_PREC_FP32)):
            got, _, _, _ = gpu_steps(spec, prec, 3)
            split = np.load("%s_%s_%d.npy" % (out, name, o))
            assert np.array_equal(got, split), (name, o, np.abs(got - split).max())
