"""Differentiable run (hot-spot event at rest, WENO5, SSP-RK3, checkpoints every
10 steps): the gradient of the energy-weighted momentum anisotropy
sum(Mx^2 - My^2) / sum(E) at the final time with respect to the initial energy
density, through the hand-written adjoint, against central finite differences of
the FP64 forward run on 32 random cells."""
import numpy as np
import pytest
import torch

from paper_1604_03360_amd import inputs
from gpu_helpers import rh_module

pytestmark = pytest.mark.gpu


def anisotropy(u):
    u = u.double()
    return (u[1] ** 2 - u[2] ** 2).sum() / u[0].sum()


def initial_state(e0):
    # at rest E = e, M = 0, N = n = e^(3/4) (the conformal state map at v = 0)
    z = torch.zeros_like(e0)
    return torch.stack([e0, z, z, z, e0 ** 0.75])


def gradient(rh, spec, precision, n_steps, every=10):
    from paper_1604_03360_amd import autograd
    h = rh.Hydro.from_spec(spec, precision=precision)
    dtype = h.dtype
    e0 = torch.tensor(spec["prim"][0], dtype=torch.float64, device="cuda").requires_grad_(True)
    u0 = initial_state(e0).to(dtype)
    uT = autograd.run(u0, h, spec["dt"], n_steps, every)
    loss = anisotropy(uT)
    loss.backward()
    g = e0.grad.detach().cpu().numpy()
    h.close()
    return loss.item(), g


def loss_fd(rh, spec, e0, n_steps):
    h = rh.Hydro.from_spec(spec, precision=rh.RH_PREC_FP64)
    with torch.no_grad():
        h.state.copy_(initial_state(torch.tensor(e0, device="cuda")))
    h.step(spec["dt"], n_steps)
    val = anisotropy(h.state).item()
    h.close()
    return val


@pytest.mark.parametrize("n,n_steps", [(32, 12), (96, 50)])
def test_adjoint_gradient_against_finite_differences(n, n_steps):
    rh = rh_module()
    spec = inputs.diff_event(n=n)
    loss64, g64 = gradient(rh, spec, rh.RH_PREC_FP64, n_steps)
    loss32, g32 = gradient(rh, spec, rh.RH_PREC_FP32, n_steps)
    assert loss32 == pytest.approx(loss64, rel=1e-4)
    e0 = spec["prim"][0]
    cells = np.random.default_rng([1604, 2000]).choice(e0.size, 32, replace=False)
    # add the cells where the gradient is largest, so the check sees real signal
    cells = np.concatenate([cells, np.argsort(np.abs(g64).ravel())[-8:]])
    gmax = np.abs(g64).max()
    for c in cells:
        idx = np.unravel_index(c, e0.shape)

        def central(hstep):
            ep, em = e0.copy(), e0.copy()
            ep[idx] += hstep
            em[idx] -= hstep
            return (loss_fd(rh, spec, ep, n_steps) - loss_fd(rh, spec, em, n_steps)) / (2 * hstep)

        # Richardson-extrapolated central difference (truncation O(h^4)) from steps of
        # 2e-4 and 1e-4 relative; the rounding noise of the FP64 runs, about
        # eps |loss| / h per difference, is amplified by (4 + 1/2) / 3 and added to the bound
        hstep = 1e-4 * e0[idx]
        fd = (4.0 * central(hstep) - central(2.0 * hstep)) / 3.0
        noise = 100 * np.finfo(float).eps * abs(loss64) / hstep * 1.5
        assert abs(g64[idx] - fd) <= 1e-6 * gmax + noise + 1e-6 * abs(fd), (idx, g64[idx], fd)
        assert abs(g32[idx] - fd) <= 1e-3 * gmax, (idx, g32[idx], fd)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_step_after_backward_continues_the_forward_run(precision):
    """backward replays checkpointed segments on the plan's own buffers; afterwards
    the plan holds the forward's final state and time again, so further steps
    equal those of an uninterrupted run, bitwise."""
    from paper_1604_03360_amd import autograd
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    spec = inputs.diff_event(n=32)
    dt = spec["dt"]
    h = rh.Hydro.from_spec(spec, precision=prec)
    e0 = torch.tensor(spec["prim"][0], dtype=torch.float64, device="cuda").requires_grad_(True)
    uT = autograd.run(initial_state(e0).to(h.dtype), h, dt, 7, every=3)
    anisotropy(uT).backward()
    assert h.t == pytest.approx(spec["t0"] + 7 * dt, abs=1e-12)
    assert torch.equal(h.state, uT.detach())
    h.step(dt, 4)
    after = h.state.clone()
    h.close()
    ref = rh.Hydro.from_spec(spec, precision=prec)
    with torch.no_grad():
        ref.state.copy_(initial_state(e0.detach()).to(ref.dtype))
    ref.step(dt, 11)
    assert torch.equal(after, ref.state)
    ref.close()
