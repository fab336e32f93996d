"""Differentiable SSP-RK3 runs: a torch.autograd.Function over the C ABI.

``HydroRun.apply(u0, hydro, dt, n_steps, every)`` advances the conserved state
u0 (a device tensor of the plan's dtype and layout [5][nz][ny][nx]) by n_steps
steps of the library's SSP-RK3 scheme and returns the final state.  The forward
pass keeps a checkpoint of the state every ``every`` steps; the backward pass
replays each checkpointed segment forward, keeping every step's input and its
two Runge-Kutta stage states (``rh_step_store_n``), and then applies the
hand-written adjoint of one step (``rh_step_vjp_stored``) in reverse.  The
replays run on the plan's own state buffer; backward restores that buffer and
the plan's time to what they held when it was called, so stepping the plan
after backward continues from there.
All arithmetic runs in the library's kernels; this module only sequences calls
and keeps the checkpoints.
"""
import torch

from . import rh


class HydroRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, hydro, dt, n_steps, every):
        if u0.dtype != hydro.dtype or tuple(u0.shape) != tuple(hydro.state.shape):
            raise ValueError("u0 must match the plan's dtype and [5][nz][ny][nx] shape")
        every = max(1, int(every))
        t0 = hydro.t
        hydro.state.copy_(u0.detach())
        checkpoints = []
        for s in range(int(n_steps)):
            if s % every == 0:
                checkpoints.append((hydro.state.clone(), hydro.t))
            hydro.step(dt, 1)
        ctx.hydro = hydro
        ctx.dt = float(dt)
        ctx.n_steps = int(n_steps)
        ctx.every = every
        ctx.checkpoints = checkpoints
        ctx.t0 = t0
        return hydro.state.clone()

    @staticmethod
    def backward(ctx, grad_out):
        hydro, dt, every = ctx.hydro, ctx.dt, ctx.every
        ubar = grad_out.detach().to(hydro.dtype).contiguous()
        # the replays below overwrite the plan's state: keep what it holds now
        resume_state, resume_t = hydro.state.clone(), hydro.t
        for seg in reversed(range(len(ctx.checkpoints))):
            u_c, t_c = ctx.checkpoints[seg]
            steps = min(every, ctx.n_steps - seg * every)
            hydro.state.copy_(u_c)
            hydro.t = t_c
            # [steps][3]: each step's input and its two stage states
            store = hydro.step_store_n(dt, steps)
            times = [t_c]
            for _ in range(steps - 1):
                times.append(times[-1] + dt)   # the step times the replay took
            for j in reversed(range(steps)):
                ubar = hydro.step_vjp_stored(store[j, 0], store[j, 1:], ubar, dt, t=times[j])
            del store
        hydro.state.copy_(resume_state)
        hydro.t = resume_t
        return ubar, None, None, None, None


def run(u0, hydro, dt, n_steps, every=10):
    """Differentiable n_steps SSP-RK3 run from u0 (see HydroRun)."""
    return HydroRun.apply(u0, hydro, dt, n_steps, every)
