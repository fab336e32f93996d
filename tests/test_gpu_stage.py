"""The fused stage (one launch per Runge-Kutta stage: L along x, y and z and the
stage combine) on single grids.

It must give bitwise the results of the directional sweeps (which are held to
the oracle by the other parity files) for every boundary kind, both orders,
both precisions, both tile shapes, ragged tiles and segments of any length,
and it is also compared with the FP64 oracle directly: L and three SSP-RK3
steps (FP64 1e-12, FP32 2e-5 after the steps and 1e-5 on L, normalised as in
the other parity files), the floor counter with planted unphysical cells,
graph replays, and the error paths of the path / tuning calls.
"""
import numpy as np
import pytest

import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import L_errors, assert_fields_close, field_errors, rh_module

pytestmark = pytest.mark.gpu

P, O, H = inputs.BC_PERIODIC, inputs.BC_OUTFLOW, inputs.BC_HUBBLE

CASES = {
    # ragged in x and y for both tile shapes, several z segments
    "periodic_ragged": lambda o: inputs.random_smooth((70, 37, 23), h=0.1, seed=101, order=o),
    "outflow_ragged": lambda o: inputs.random_smooth((33, 20, 45), h=0.07, seed=102, order=o,
                                                     bc=(O, O, O)),
    "mixed_bc": lambda o: inputs.random_smooth((48, 19, 30), h=0.08, seed=103, order=o, bc=(O, P, O)),
    # axes shorter than the stencil halo
    "tiny_axes": lambda o: inputs.random_smooth((5, 3, 2), h=0.1, seed=104, order=o, bc=(P, O, P)),
    "hubble": lambda o: inputs.hubble(n=24, order=o, half_width=3.0),
    "blob": lambda o: inputs.blob(h=0.25, order=o, shape=(64, 48, 40)),
}

TILES = {5: (16, 32), 7: (16,)}


def _prec(rh, name):
    return rh.RH_PREC_FP64 if name == "fp64" else rh.RH_PREC_FP32


def _hydro(rh, spec, prec, path, tile=None, seg=0):
    h = rh.Hydro.from_spec(spec, precision=prec)
    rh.rh_set_path(h.plan, path)
    if tile:
        rh.rh_set_stage_tuning(h.plan, tile, seg)
    h.set_primitive(spec["prim"])
    return h


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_stage_L_bitwise_sweeps_and_oracle(case, order, precision):
    rh = rh_module()
    prec = _prec(rh, precision)
    spec = CASES[case](order)
    ref_h = _hydro(rh, spec, prec, rh.RH_PATH_SWEEPS)
    ref = ref_h.apply_L().double().cpu().numpy()
    ref_h.close()
    orc = oracle.apply_L(oracle.grid_from_spec(spec), oracle.prim2con(spec["prim"]), spec["t0"])
    for tile in TILES[order]:
        for seg in (0, 1, 7):
            h = _hydro(rh, spec, prec, rh.RH_PATH_STAGE, tile, seg)
            assert rh.rh_get_path(h.plan) == rh.RH_PATH_STAGE
            got = h.apply_L().double().cpu().numpy()
            h.close()
            assert np.array_equal(got, ref), (case, order, precision, tile, seg)
    err = L_errors(ref, orc, oracle.prim2con(spec["prim"]), min(spec["h"]))
    print(case, order, precision, "L vs oracle", err, flush=True)
    assert np.all(err <= (1e-12 if precision == "fp64" else 1e-5)), err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_stage_steps_bitwise_sweeps_and_oracle(case, order, precision):
    rh = rh_module()
    prec = _prec(rh, precision)
    spec = CASES[case](order)
    nsteps, dt = 3, spec["dt"]
    ref_h = _hydro(rh, spec, prec, rh.RH_PATH_SWEEPS)
    ref_h.step(dt, nsteps)
    ref = ref_h.get()
    tref, cref = ref_h.totals()
    ref_h.close()
    for tile in TILES[order]:
        h = _hydro(rh, spec, prec, rh.RH_PATH_STAGE, tile, 0)
        h.step(dt, nsteps)
        got = h.get()
        tot, cnt = h.totals()
        h.close()
        assert np.array_equal(got, ref), (case, order, precision, tile)
        assert list(cnt) == list(cref)
    orc, _ = oracle.step(oracle.grid_from_spec(spec), oracle.prim2con(spec["prim"]), dt, nsteps,
                         t=spec["t0"])
    print(case, order, precision, "steps vs oracle", field_errors(ref, orc), flush=True)
    assert_fields_close(ref, orc, 1e-12 if precision == "fp64" else 2e-5, case)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stage_floor_counter_and_values(precision):
    """Planted unphysical cells (energy floor, velocity cap): the fused stage
    gives the sweeps' L bitwise and counts each floored cell once."""
    from test_gpu_floors import CASES as FCASES, planted_state
    rh = rh_module()
    prec = _prec(rh, precision)
    for case in sorted(FCASES):
        spec = FCASES[case](5)
        u, planted = planted_state(spec, 11)
        if prec == rh.RH_PREC_FP32:
            u = u.astype(np.float32).astype(np.float64)
        out = {}
        for path in (rh.RH_PATH_SWEEPS, rh.RH_PATH_STAGE):
            h = rh.Hydro.from_spec(spec, precision=prec)
            rh.rh_set_path(h.plan, path)
            h.set_conserved(u)
            rh.rh_reset_counters(h.plan)
            L = h.apply_L().double().cpu().numpy()
            _, cnt = h.totals()
            h.close()
            out[path] = (L, cnt[0])
        assert np.array_equal(out[rh.RH_PATH_SWEEPS][0], out[rh.RH_PATH_STAGE][0]), case
        assert out[rh.RH_PATH_STAGE][1] == len(planted) == out[rh.RH_PATH_SWEEPS][1], case


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_stage_graph_replay_matches_eager(precision):
    import torch
    rh = rh_module()
    prec = _prec(rh, precision)
    spec = CASES["periodic_ragged"](5)
    dt = spec["dt"]
    eager = _hydro(rh, spec, prec, rh.RH_PATH_STAGE)
    for _ in range(3):
        eager.step(dt, 2)
    graphed = _hydro(rh, spec, prec, rh.RH_PATH_STAGE)
    rh.rh_set_graph(graphed.plan, True)
    for _ in range(3):
        graphed.step(dt, 2)
        scratch = torch.randn(1 << 18, device="cuda")
        scratch.mul_(3.0).sum().item()
        torch.cuda.synchronize()
    assert np.array_equal(graphed.get(), eager.get())
    eager.close()
    graphed.close()


def test_stage_kernel_class_and_errors():
    rh = rh_module()
    spec = CASES["periodic_ragged"](5)
    h = _hydro(rh, spec, rh.RH_PREC_FP32, rh.RH_PATH_STAGE)
    rh.rh_set_timing(h.plan, True)
    h.step(spec["dt"], 2)
    times = rh.rh_kernel_times(h.plan)
    assert times["stage"][1] == 6 and times["stage"][0] > 0.0
    for k in ("sweep_x", "sweep_y", "sweep_z", "sweep_xy"):
        assert times[k][1] == 0
    with pytest.raises(rh.RHError) as e:
        rh.rh_set_stage_tuning(h.plan, 64, 0)
    assert e.value.status == rh.RH_E_INVAL
    with pytest.raises(rh.RHError) as e:
        rh.rh_set_path(h.plan, 9)
    assert e.value.status == rh.RH_E_INVAL
    h.close()
    spec7 = CASES["periodic_ragged"](7)
    h = _hydro(rh, spec7, rh.RH_PREC_FP32, rh.RH_PATH_STAGE)
    with pytest.raises(rh.RHError) as e:
        rh.rh_set_stage_tuning(h.plan, 32, 0)
    assert e.value.status == rh.RH_E_NOTSUP
    h.close()
    # an axis of one cell: the default path stays the sweeps, the fused stage
    # can be selected (it leaves that axis out, as the sweeps do)
    flat = inputs.random_smooth((40, 30, 1), h=0.1, seed=105)
    h = rh.Hydro.from_spec(flat, precision=rh.RH_PREC_FP32)
    assert rh.rh_get_path(h.plan) == rh.RH_PATH_SWEEPS
    rh.rh_set_path(h.plan, rh.RH_PATH_STAGE)
    assert rh.rh_get_path(h.plan) == rh.RH_PATH_STAGE
    h.close()
