"""MUSTA-FORCE, local Lax-Friedrichs splitting and the ideal gas on the GPU
(through the C ABI) against the FP64 oracle, element by element.

Bars as for the WENO path: FP64 plans 1e-12 (normalised L-infinity per field;
L normalised by max(max|L|, max|u|/h)); FP32 plans 1e-5 on L and 2e-5 after a
few steps.  Shapes are ragged and span several 16 x 15 (MUSTA-FORCE) or 16 x 16
(WENO) tiles and z segments; axes of one cell are included.
"""
import numpy as np
import pytest

import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import L_errors, field_errors, rh_module

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
OUT = inputs.BC_OUTFLOW
MUSTA = 2


def _cases():
    return {
        "smooth_periodic": lambda: inputs.random_smooth((37, 33, 21), h=0.1, seed=1),
        "smooth_outflow": lambda: inputs.random_smooth((33, 20, 45), h=0.07, seed=2, bc=(OUT,) * 3),
        "hubble": lambda: inputs.hubble(n=24, half_width=3.0),
        "hotspots": lambda: inputs.hotspots(3, size=40),
        "sod": lambda: inputs.sod(nx=400),
        "line_y": lambda: inputs.random_smooth((1, 47, 1), h=0.1, seed=3),
        "plane_xz": lambda: inputs.random_smooth((35, 1, 19), h=0.1, seed=4, bc=(OUT, 0, 0)),
    }


def _con(spec):
    return oracle.prim2con_eos(oracle.grid_from_spec(spec), spec["prim"])


def _hydro(rh, spec, precision, **kw):
    h = rh.Hydro.from_spec(spec, precision=precision, **kw)
    h.set_primitive(spec["prim"])
    return h


def _L_pair(rh, spec, precision, t=None):
    t = spec["t0"] + (0.3 if spec["name"] == "hubble" else 0.0) if t is None else t
    h = _hydro(rh, spec, precision)
    got = h.apply_L(t).double().cpu().numpy()
    _, cnt = h.totals()
    h.close()
    ref, clamps = oracle.apply_L(oracle.grid_from_spec(spec), _con(spec), t, return_clamps=True)
    return got, ref, cnt, clamps


def _steps_pair(rh, spec, precision, nsteps):
    h = _hydro(rh, spec, precision)
    h.step(spec["dt"], nsteps)
    got = h.get()
    _, cnt = h.totals()
    h.close()
    ref, _, clamps = oracle.step(oracle.grid_from_spec(spec), _con(spec), spec["dt"], nsteps,
                                 t=spec["t0"], return_clamps=True)
    return got, ref, cnt, clamps


# ---------------------------------------------------------------------------
# MUSTA-FORCE
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("limiter", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("case", sorted(_cases()))
def test_musta_L_fp64(case, limiter):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=MUSTA, limiter=limiter, musta_k=2, musta_cfl=0.9)
    got, ref, cnt, clamps = _L_pair(rh, spec, rh.RH_PREC_FP64)
    err = L_errors(got, ref, _con(spec), min(spec["h"]))
    print(case, limiter, err, flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(err <= FP64_TOL), err
    assert cnt[0] == clamps


@pytest.mark.parametrize("k,cfl", [(1, 0.9), (3, 0.9), (4, 0.5), (8, 1.0)])
def test_musta_stage_counts_fp64(k, cfl):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()["smooth_outflow"](), order=MUSTA, limiter=1, musta_k=k, musta_cfl=cfl)
    got, ref, _, _ = _L_pair(rh, spec, rh.RH_PREC_FP64)
    err = L_errors(got, ref, _con(spec), min(spec["h"]))
    print(k, cfl, err, flush=True)
    assert np.all(err <= FP64_TOL), err


@pytest.mark.parametrize("limiter", [0, 3])
@pytest.mark.parametrize("case,nsteps", [("smooth_periodic", 4), ("hubble", 4), ("hotspots", 3),
                                         ("plane_xz", 5)])
def test_musta_steps_fp64(case, nsteps, limiter):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=MUSTA, limiter=limiter)
    got, ref, cnt, clamps = _steps_pair(rh, spec, rh.RH_PREC_FP64, nsteps)
    err = field_errors(got, ref)
    print(case, limiter, err, flush=True)
    assert np.all(err <= FP64_TOL), err
    assert cnt[0] == clamps


def test_musta_sod_full_run_fp64():
    rh = rh_module()
    spec = inputs.with_scheme(inputs.sod(nx=400), order=MUSTA, limiter=1, musta_k=2)
    got, ref, cnt, clamps = _steps_pair(rh, spec, rh.RH_PREC_FP64, spec["nsteps"])
    err = field_errors(got, ref)
    print("musta sod", err, flush=True)
    assert np.all(err <= FP64_TOL), err
    assert cnt[0] == clamps == 0


@pytest.mark.parametrize("case", ["smooth_periodic", "hubble", "hotspots"])
def test_musta_fp32(case):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=MUSTA, limiter=2)
    got, ref, _, _ = _L_pair(rh, spec, rh.RH_PREC_FP32)
    errL = L_errors(got, ref, _con(spec), min(spec["h"]))
    got, ref, _, _ = _steps_pair(rh, spec, rh.RH_PREC_FP32, 4)
    err = field_errors(got, ref)
    print(case, "fp32", errL, err, flush=True)
    assert np.all(errL <= 1e-5), errL
    assert np.all(err <= 2e-5), err


def test_musta_floors_counted_per_face_state():
    """Cells below the energy floor and beyond the velocity cap: L and the floor
    count (per recovery of a face state, each face once) against the oracle."""
    rh = rh_module()
    spec = inputs.with_scheme(inputs.random_smooth((29, 31, 17), h=0.1, seed=6), order=MUSTA, limiter=0)
    con = _con(spec)
    rng = np.random.default_rng(13)
    cells = rng.choice(con[0].size, 40, replace=False)
    flat = con.reshape(5, -1)
    flat[0, cells[:20]] = 1e-14                     # below the energy floor
    flat[1, cells[20:]] = 1.5 * flat[0, cells[20:]]  # beyond the velocity cap
    h = rh.Hydro.from_spec(spec, precision=rh.RH_PREC_FP64)
    h.set_conserved(con)
    got = h.apply_L(0.0).double().cpu().numpy()
    _, cnt = h.totals()
    h.close()
    ref, clamps = oracle.apply_L(oracle.grid_from_spec(spec), con, 0.0, return_clamps=True)
    err = L_errors(got, ref, con, min(spec["h"]))
    print("floors", err, cnt, clamps, flush=True)
    assert clamps > 0 and cnt[0] == clamps
    assert np.all(err <= FP64_TOL), err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_musta_batch_equals_single_grids(precision):
    import torch
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    specs = [inputs.with_scheme(inputs.hotspots(k, size=s), order=MUSTA, limiter=3, musta_k=2)
             for k, s in ((0, 24), (1, 40), (2, 17))]
    b = rh.Batch(specs, precision=prec)
    b.set_primitive([sp["prim"] for sp in specs])
    rh.rh_batch_set_graph(b.batch, 1)
    b.step(specs[0]["dt"], 3)
    got = b.get()
    b.close()
    for sp, g in zip(specs, got):
        h = _hydro(rh, sp, prec)
        h.step(sp["dt"], 3)
        single = h.get()
        h.close()
        assert np.array_equal(g, single)
    torch.cuda.synchronize()


def test_musta_graph_replays_match_eager():
    rh = rh_module()
    spec = inputs.with_scheme(_cases()["smooth_periodic"](), order=MUSTA, limiter=1)
    a = _hydro(rh, spec, rh.RH_PREC_FP32)
    b = _hydro(rh, spec, rh.RH_PREC_FP32)
    rh.rh_set_graph(b.plan, 1)
    for _ in range(3):
        a.step(spec["dt"], 2)
        b.step(spec["dt"], 2)
        assert np.array_equal(a.get(), b.get())
    a.close()
    b.close()


# ---------------------------------------------------------------------------
# Local Lax-Friedrichs splitting (WENO)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(_cases()))
def test_local_split_L_fp64(case, order):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=order, lf_local=True)
    got, ref, cnt, clamps = _L_pair(rh, spec, rh.RH_PREC_FP64)
    err = L_errors(got, ref, _con(spec), min(spec["h"]))
    print(case, order, err, flush=True)
    assert np.all(err <= FP64_TOL), err


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case,nsteps", [("smooth_periodic", 4), ("hubble", 4), ("hotspots", 3)])
def test_local_split_steps(case, nsteps, order):
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=order, lf_local=True)
    got, ref, _, _ = _steps_pair(rh, spec, rh.RH_PREC_FP64, nsteps)
    err = field_errors(got, ref)
    got32, _, _, _ = _steps_pair(rh, spec, rh.RH_PREC_FP32, nsteps)
    err32 = field_errors(got32, ref)
    print(case, order, err, err32, flush=True)
    assert np.all(err <= FP64_TOL), err
    assert np.all(err32 <= 2e-5), err32


@pytest.mark.parametrize("order", [5, 7])
def test_local_split_sod_full_run_fp64(order):
    rh = rh_module()
    spec = inputs.with_scheme(inputs.sod(nx=400), order=order, lf_local=True)
    got, ref, _, _ = _steps_pair(rh, spec, rh.RH_PREC_FP64, spec["nsteps"])
    err = field_errors(got, ref)
    print("llf sod", order, err, flush=True)
    assert np.all(err <= FP64_TOL), err


# ---------------------------------------------------------------------------
# Ideal gas
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gamma", [4.0 / 3.0, 5.0 / 3.0, 2.0])
def test_ideal_gas_field_conversion(gamma):
    rh = rh_module()
    spec = inputs.with_scheme(inputs.hot_gas(inputs.random_smooth((21, 19, 17), seed=7, amp_v=0.9)),
                              eos=1, gamma=gamma)
    h = _hydro(rh, spec, rh.RH_PREC_FP64)
    con = h.get(rh.RH_FIELDS_CONSERVED)
    prim = h.get(rh.RH_FIELDS_PRIMITIVE)
    h.close()
    g = oracle.grid_from_spec(spec)
    ref_con = oracle.prim2con_eos(g, spec["prim"])
    ref_prim = oracle.con2prim_eos(g, ref_con)
    assert np.all(field_errors(con, ref_con) <= 1e-14)
    err = field_errors(prim, ref_prim)
    print("ideal prim", gamma, err, flush=True)
    assert np.all(err <= 1e-13), err


@pytest.mark.parametrize("scheme", ["weno5", "weno5_local", "weno7_local", "musta"])
@pytest.mark.parametrize("case", ["smooth_periodic", "smooth_outflow", "hotspots", "plane_xz"])
def test_ideal_gas_L_fp64(case, scheme):
    rh = rh_module()
    opts = {"weno5": dict(order=5), "weno5_local": dict(order=5, lf_local=True),
            "weno7_local": dict(order=7, lf_local=True), "musta": dict(order=MUSTA, limiter=1)}[scheme]
    spec = inputs.with_scheme(inputs.hot_gas(_cases()[case]()), eos=1, gamma=5.0 / 3.0, **opts)
    got, ref, _, _ = _L_pair(rh, spec, rh.RH_PREC_FP64)
    err = L_errors(got, ref, _con(spec), min(spec["h"]))
    print(case, scheme, err, flush=True)
    assert np.all(err <= FP64_TOL), err


@pytest.mark.parametrize("scheme", ["weno5_local", "musta"])
def test_ideal_gas_shock_tube(scheme):
    """The gamma = 5/3 shock tube, 100 steps, FP64 against the oracle; FP32 after
    a few steps."""
    rh = rh_module()
    opts = dict(order=5, lf_local=True) if scheme == "weno5_local" else dict(order=MUSTA, limiter=1)
    spec = inputs.with_scheme(inputs.sod_ideal(nx=400), **opts)
    got, ref, cnt, clamps = _steps_pair(rh, spec, rh.RH_PREC_FP64, 100)
    err = field_errors(got, ref)
    got32, ref32, _, _ = _steps_pair(rh, spec, rh.RH_PREC_FP32, 5)
    err32 = field_errors(got32, ref32)
    print("ideal sod", scheme, err, err32, cnt, clamps, flush=True)
    assert np.all(err <= FP64_TOL), err
    assert np.all(err32 <= 2e-5), err32


@pytest.mark.parametrize("split", ["global", "local"])
def test_ideal_gas_floors_counted_once_per_cell(split):
    """Ideal gas, WENO5: cells below the energy floor and beyond the velocity cap.
    L against the oracle; the floor counter counts each floored cell once per
    evaluation of L (the recovery pass solves every cell once), as the oracle's
    primitive recovery of the state does (its L recovers each cell once per axis)."""
    rh = rh_module()
    spec = inputs.with_scheme(inputs.hot_gas(inputs.random_smooth((29, 31, 17), h=0.1, seed=6)), eos=1,
                              gamma=5.0 / 3.0, order=5, lf_local=split == "local")
    con = _con(spec)
    rng = np.random.default_rng(17)
    cells = rng.choice(con[0].size, 40, replace=False)
    flat = con.reshape(5, -1)
    flat[0, cells[:20]] = 1e-14                     # below the energy floor
    flat[1, cells[20:]] = 1.5 * flat[0, cells[20:]]  # beyond the velocity cap
    h = rh.Hydro.from_spec(spec, precision=rh.RH_PREC_FP64)
    h.set_conserved(con)
    got = h.apply_L(0.0).double().cpu().numpy()
    _, cnt = h.totals()
    h.close()
    grid = oracle.grid_from_spec(spec)
    ref, clamps = oracle.apply_L(grid, con, 0.0, return_clamps=True)
    _, floored = oracle.con2prim_eos(grid, con, return_clamps=True)
    err = L_errors(got, ref, con, min(spec["h"]))
    print("ideal floors", split, err, cnt, floored, clamps, flush=True)
    assert floored == 40 and clamps == 3 * floored and cnt[0] == floored
    assert np.all(err <= FP64_TOL), err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ideal_gas_batch_equals_single_grids(precision):
    """Grids of different sizes in one batch: the recovery pass finds each block's
    grid in its own block table; three steps bitwise equal to single-grid runs,
    also after autotuning the batch (the tuning runs the recovery pass too)."""
    import torch
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    for lf_local in (False, True):
        specs = [inputs.with_scheme(inputs.hot_gas(inputs.hotspots(k, size=s)), eos=1, gamma=5.0 / 3.0,
                                    lf_local=lf_local) for k, s in ((0, 24), (1, 40), (2, 17))]
        b = rh.Batch(specs, precision=prec)
        b.set_primitive([sp["prim"] for sp in specs])
        if lf_local:
            rh.rh_batch_autotune(b.batch, 1)
        rh.rh_batch_set_graph(b.batch, 1)
        b.step(specs[0]["dt"], 3)
        got = b.get()
        b.close()
        for sp, g in zip(specs, got):
            h = _hydro(rh, sp, prec)
            h.step(sp["dt"], 3)
            single = h.get()
            h.close()
            assert np.array_equal(g, single)
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ideal_gas_shock_tube_full_run_against_exact_solution(precision):
    """The gamma = 5/3 shock tube to t = 0.4 on 800 cells (WENO5, local
    splitting) on the GPU against the exact solution of tests/ideal_riemann.py:
    the same L1 bars as the oracle's own run (n 0.06, p 0.045, v 0.006) and the
    star plateau within 0.5%."""
    import ideal_riemann as ir
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    gam = 5.0 / 3.0
    pL, pR = (gam - 1.0) * (29.995 - 10.0), (gam - 1.0) * (1.0000015 - 1.0)
    spec = inputs.with_scheme(inputs.sod_ideal(nx=800), order=5, lf_local=True)
    h = _hydro(rh, spec, prec)
    t = h.step(spec["dt"], spec["nsteps"])
    prim = h.get(rh.RH_FIELDS_PRIMITIVE).reshape(5, 800)
    h.close()
    x = spec["c0"][0] + spec["h"][0] * np.arange(800)
    ex = ir.sample(10.0, pL, 1.0, pR, gam, x / t)
    got = np.array([prim[4], (gam - 1.0) * (prim[0] - prim[4]), prim[1]])
    err = np.abs(got - ex).sum(axis=1) * spec["h"][0]
    s = ir.star_state(10.0, pL, 1.0, pR, gam)
    i = np.argmin(np.abs(x - 0.5 * (s["xi_tail"] + s["v"]) * t))
    print("ideal tube exact", precision, err, got[1, i] / s["p"] - 1.0, flush=True)
    assert t == pytest.approx(0.4, abs=1e-12)
    assert np.all(err < [0.06, 0.045, 0.006]), err
    assert got[1, i] == pytest.approx(s["p"], rel=5e-3) and got[2, i] == pytest.approx(s["v"], rel=5e-3)


# ---------------------------------------------------------------------------
# Paths and errors
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", ["sod", "line_y", "plane_xz"])
def test_stage_path_with_single_cell_axes_equals_sweeps(case, order):
    """The fused stage on grids with axes of one cell gives the sweeps' bits."""
    rh = rh_module()
    spec = inputs.with_scheme(_cases()[case](), order=order)
    out = []
    for path in (rh.RH_PATH_SWEEPS, rh.RH_PATH_STAGE):
        h = _hydro(rh, spec, rh.RH_PREC_FP32)
        rh.rh_set_path(h.plan, path)
        h.step(spec["dt"], 3)
        out.append(h.get())
        h.close()
    assert np.array_equal(out[0], out[1])


def test_scheme_errors():
    rh = rh_module()
    for opts in (dict(order=MUSTA), dict(order=5, lf_local=True), dict(order=5, eos=1, gamma=1.4)):
        spec = inputs.with_scheme(inputs.random_smooth((16, 16, 16), seed=8), **opts)
        h = _hydro(rh, spec, rh.RH_PREC_FP32)
        with pytest.raises(rh.RHError) as ei:
            rh.rh_set_path(h.plan, rh.RH_PATH_SWEEPS)
        assert ei.value.status == rh.RH_E_NOTSUP
        with pytest.raises(rh.RHError) as ei:
            h.vjp(h.state, h.state)
        assert ei.value.status == rh.RH_E_NOTSUP
        with pytest.raises(rh.RHError) as ei:
            h.step_vjp(h.state, h.state, 0.01)
        assert ei.value.status == rh.RH_E_NOTSUP
        h.close()
    spec = inputs.with_scheme(inputs.hubble(n=16, half_width=3.0), eos=1)
    with pytest.raises(rh.RHError) as ei:
        rh.Hydro.from_spec(spec)
    assert ei.value.status == rh.RH_E_NOTSUP
