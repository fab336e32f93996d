"""Hand-written adjoint on the GPU against the oracle's adjoint and against the
oracle's complex-step directional derivatives (dot-product test)."""
import numpy as np
import pytest

import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import rh_module

pytestmark = pytest.mark.gpu

CASES = {
    "smooth_periodic": lambda o: inputs.random_smooth((37, 29, 23), h=0.1, seed=61, order=o),
    "smooth_outflow": lambda o: inputs.random_smooth((26, 33, 19), h=0.08, seed=62, order=o,
                                                     bc=(inputs.BC_OUTFLOW,) * 3),
    "hubble": lambda o: inputs.hubble(n=20, order=o, half_width=3.0),
    "hotspots": lambda o: inputs.hotspots(9, size=32, order=o),
    "tiny_periodic": lambda o: inputs.random_smooth((6, 5, 4), h=0.2, seed=63, order=o),
    # degenerate axes: a line along x, planes without x and without y
    "line_x_outflow": lambda o: inputs.random_smooth((90, 1, 1), h=0.05, seed=64, order=o,
                                                     bc=(inputs.BC_OUTFLOW,) * 3),
    "plane_yz": lambda o: inputs.random_smooth((1, 27, 21), h=0.1, seed=65, order=o),
    "plane_xz_outflow": lambda o: inputs.random_smooth((35, 1, 18), h=0.1, seed=66, order=o,
                                                       bc=(inputs.BC_OUTFLOW,) * 3),
}


def vjp_errors(got, ref, w, h):
    """Per-field max|got - ref| normalised by max(max|ref|, max|w|/h): the adjoint
    is a sum of face weights (w_{i+1} - w_i)/h times O(1) derivatives."""
    got = np.asarray(got, np.float64).reshape(5, -1)
    ref = np.asarray(ref, np.float64).reshape(5, -1)
    scale = max(np.abs(ref).max(), np.abs(w).max() / h)
    return np.abs(got - ref).max(axis=1) / scale


def _setup(rh, spec, prec):
    h = rh.Hydro.from_spec(spec, precision=prec)
    u = oracle.prim2con(spec["prim"])
    w = np.random.default_rng(7).normal(size=u.shape)
    return h, u, w


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_vjp_L_fp64_matches_oracle(case, order):
    rh = rh_module()
    spec = CASES[case](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    t = spec["t0"] + 0.2
    got = h.vjp(u, w, t=t).cpu().numpy()
    h.close()
    ref = oracle.vjp_L(oracle.grid_from_spec(spec), u, w, t=t)
    err = vjp_errors(got, ref, w, min(spec["h"]))
    print(case, order, err, flush=True)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("order", [5, 7])
def test_vjp_L_dot_product_with_oracle_jvp(order):
    rh = rh_module()
    spec = CASES["smooth_periodic"](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    v = np.random.default_rng(8).normal(size=u.shape)
    got = h.vjp(u, w).cpu().numpy()
    h.close()
    jv = oracle.jvp_L(oracle.grid_from_spec(spec), u, v)
    assert np.vdot(got, v) == pytest.approx(np.vdot(w, jv), rel=1e-11)


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("case", ["smooth_periodic", "smooth_outflow", "hubble", "hotspots", "line_x_outflow",
                                  "plane_yz"])
def test_step_vjp_fp64_matches_oracle(case, order):
    rh = rh_module()
    spec = CASES[case](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    dt, t = spec["dt"], spec["t0"]
    got = h.step_vjp(u, w, dt, t=t).cpu().numpy()
    h.close()
    ref = oracle.vjp_step(oracle.grid_from_spec(spec), u, w, dt, t=t)
    err = np.abs(got - ref).reshape(5, -1).max(axis=1) / np.abs(ref).max()
    print(case, order, err, flush=True)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("case,order", [("smooth_periodic", 5), ("hotspots", 5), ("smooth_outflow", 5),
                                        ("hubble", 5), ("smooth_periodic", 7), ("hubble", 7)])
def test_vjp_fp32_close_to_oracle(case, order):
    """FP32 adjoint (both WENO5 gradient forms: the analytic-ghost build keeps the
    compact one) against the FP64 oracle on the FP32-rounded inputs."""
    rh = rh_module()
    spec = CASES[case](order)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP32)
    dt, t0 = spec["dt"], spec["t0"]
    got = h.vjp(u, w, t=t0 + 0.2).double().cpu().numpy()
    gs = h.step_vjp(u, w, dt, t=t0).double().cpu().numpy()
    h.close()
    u32 = u.astype(np.float32).astype(np.float64)
    w32 = w.astype(np.float32).astype(np.float64)
    g = oracle.grid_from_spec(spec)
    err = vjp_errors(got, oracle.vjp_L(g, u32, w32, t=t0 + 0.2), w32, min(spec["h"]))
    ref_s = oracle.vjp_step(g, u32, w32, dt, t=t0)
    err_s = np.abs(gs - ref_s).max() / np.abs(ref_s).max()
    print(case, order, "fp32", err, err_s, flush=True)
    assert np.all(err <= 5e-5) and err_s <= 5e-5, (err, err_s)


def test_charge_adjoint_is_zero_for_energy_momentum_weights():
    rh = rh_module()
    spec = CASES["hotspots"](5)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    w[4] = 0.0
    got = h.vjp(u, w).cpu().numpy()
    h.close()
    assert np.all(got[4] == 0.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["smooth_outflow", "hubble", "hotspots"])
def test_stored_stages_give_the_recomputed_adjoint(case, precision):
    """rh_step_store advances the state exactly as rh_step and records the two
    stage states, which equal the oracle's (FP64); the adjoint from the stored
    stages equals the recomputing adjoint bitwise (same kernels, same inputs)."""
    rh = rh_module()
    import torch
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    spec = CASES[case](5)
    dt, t0 = spec["dt"], spec["t0"]
    h, u, w = _setup(rh, spec, prec)
    h.set_primitive(spec["prim"])
    u_n = h.state.clone()
    stages = h.step_store(dt)
    after_store = h.state.clone()
    assert h.t == pytest.approx(t0 + dt, abs=1e-12)
    h.state.copy_(u_n)
    h.t = t0
    h.step(dt, 1)
    assert torch.equal(h.state, after_store)
    wd = torch.tensor(w, dtype=h.dtype, device="cuda")
    a = h.step_vjp(u_n, wd, dt, t=t0)
    b = h.step_vjp_stored(u_n, stages, wd, dt, t=t0)
    assert torch.equal(a, b)
    if precision == "fp64":
        g = oracle.grid_from_spec(spec)
        un = u_n.cpu().numpy()
        u1 = un + dt * oracle.apply_L(g, un, t0)
        u2 = 0.75 * un + 0.25 * (u1 + dt * oracle.apply_L(g, u1, t0 + dt))
        st = stages.cpu().numpy()
        for got, ref in ((st[0], u1), (st[1], u2)):
            err = np.abs(got - ref).reshape(5, -1).max(axis=1) / np.abs(ref).max()
            assert np.all(err <= 1e-12), err
    h.close()


def test_stored_adjoint_rejects_aliasing():
    rh = rh_module()
    import torch
    spec = CASES["tiny_periodic"](5)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    stages = h.step_store(spec["dt"])
    u_n = h.state.clone()
    ubar = torch.ones_like(u_n)
    # scratch overlapping the stages, and an output overlapping the stages
    with pytest.raises(rh.RHError) as e:
        rh.rh_step_vjp_stored(h.plan, 0.0, spec["dt"], u_n.data_ptr(), stages.data_ptr(), ubar.data_ptr(),
                              torch.empty_like(u_n).data_ptr(), stages.data_ptr())
    assert e.value.status == rh.RH_E_INVAL
    with pytest.raises(rh.RHError) as e:
        rh.rh_step_vjp_stored(h.plan, 0.0, spec["dt"], u_n.data_ptr(), stages.data_ptr(), ubar.data_ptr(),
                              stages[1].data_ptr(), torch.empty((2,) + tuple(u_n.shape), dtype=u_n.dtype,
                                                                device="cuda").data_ptr())
    assert e.value.status == rh.RH_E_INVAL
    with pytest.raises(rh.RHError) as e:
        rh.rh_step_store(h.plan, spec["dt"], 0.0, h.workspace.data_ptr())
    assert e.value.status == rh.RH_E_INVAL
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["hubble", "hotspots"])
def test_store_n_steps_and_their_adjoint(case, precision):
    """rh_step_store_n over three steps: the final state and time are those of
    rh_step(3) (bitwise; the step graph replays are bitwise the eager steps), the
    store holds each step's start state and the stage states rh_step_store gives
    from it, and the adjoint chained backward through the stored steps equals the
    chain of recomputing adjoints bitwise."""
    rh = rh_module()
    import torch
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    spec = CASES[case](5)
    dt, t0, n = spec["dt"], spec["t0"], 3
    h, u, w = _setup(rh, spec, prec)
    h.set_primitive(spec["prim"])
    u0 = h.state.clone()
    store = h.step_store_n(dt, n)
    final, t_end = h.state.clone(), h.t
    h.state.copy_(u0)
    h.t = t0
    h.step(dt, n)
    assert torch.equal(h.state, final) and h.t == t_end
    h.state.copy_(u0)
    h.t = t0
    times = []
    for k in range(n):
        times.append(h.t)
        assert torch.equal(store[k, 0], h.state)
        stages = h.step_store(dt)
        assert torch.equal(store[k, 1:], stages)
    wd = torch.tensor(w, dtype=h.dtype, device="cuda")
    a, b = wd.clone(), wd.clone()
    for k in reversed(range(n)):
        a = h.step_vjp_stored(store[k, 0], store[k, 1:], a, dt, t=times[k])
        b = h.step_vjp(store[k, 0].clone(), b, dt, t=times[k])
    assert torch.equal(a, b) and bool(torch.isfinite(a).all())
    h.close()


def test_store_n_rejects_bad_arguments():
    rh = rh_module()
    import torch
    spec = CASES["tiny_periodic"](5)
    h, u, w = _setup(rh, spec, rh.RH_PREC_FP64)
    store = torch.empty((2, 3) + tuple(h.state.shape), dtype=h.dtype, device="cuda")
    for bad in (dict(n=-1, ptr=store.data_ptr()), dict(n=1, ptr=0), dict(n=1, ptr=h.state.data_ptr()),
                dict(n=1, ptr=h.workspace.data_ptr())):
        with pytest.raises(rh.RHError) as e:
            rh.rh_step_store_n(h.plan, spec["dt"], bad["n"], 0.0, bad["ptr"])
        assert e.value.status == rh.RH_E_INVAL
    with pytest.raises(rh.RHError) as e:
        rh.rh_step_store_n(h.plan, 0.0, 1, 0.0, store.data_ptr())
    assert e.value.status == rh.RH_E_INVAL
    assert rh.rh_step_store_n(h.plan, spec["dt"], 0, 1.5, store.data_ptr()) == 1.5
    assert rh.rh_step_store_n(h.plan, spec["dt"], 0, 1.5, 0) == 1.5
    h.close()
