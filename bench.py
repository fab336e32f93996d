"""Benchmark of the WENO5 / SSP-RK3 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 3+1D ellipsoidal Gaussian energy blob at rest on a periodic
256^3 grid (dx = 0.1, dt = 0.04, WENO5, conformal EOS), the synthetic stand-in
for the paper's ellipsoidal-flow run.  One step is one full SSP-RK3 step
(three evaluations of L, nine directional sweeps).  The state is resident in
HBM before the timed region; K steps are timed between stream synchronisations.

Prints ONE JSON line.  `value` is FP32 cell-updates/s (storage, stencil and
Runge-Kutta in FP32, primitive recovery in FP64); the FP64 run is reported
beside it.  The roofline block is for the dominant sweep kernel, timed live
with HIP events on the library's stream; the CPU baseline is the FP64 oracle on
the host cores over a bounded sample (whole-grid steps of the same workload).
Side blocks: WENO7, the adjoint, the differentiable run, the 64-event ensemble,
the other schemes (MUSTA-FORCE, local splitting, ideal gas) on the same blob,
and the per-field error of the 128^3 Hubble-like flow after 100 steps against
the FP64 oracle.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WENO5-RK3 cell-updates/s @256^3 FP32 vs FP64, %HBM peak; adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0
SETTLE_S = 0.3
# MI355X vector peaks (256 CUs, 2.4 GHz): FP32 157.3 TFLOP/s (packed), FP64 78.6 TFLOP/s
ALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

# Algorithmic FP operations per cell for one directional sweep (textbook formulas,
# add/mul/div/sqrt = 1): 10 WENO reconstructions (WENO5: 69 each; WENO7: 194 each)
# + 5 face sums + flux and Lax-Friedrichs split (25) + flux difference (10) + one
# third of the primitive recovery (20 / 3) + accumulation of L (5).
WENO_FLOPS = {5: 69, 7: 194}


def sweep_flops_per_cell(order):
    return 10 * WENO_FLOPS[order] + 5 + 25 + 10 + 20.0 / 3.0 + 5


# MUSTA-FORCE (same counting rules), per face: MUSCL states 5 x (2 slopes of 6
# operations + 2 half-slope updates of 2) = 80; per stage three physical fluxes,
# each a recovery (about 20) and the flux (8), the Richtmyer state (5 x 4), the
# FORCE flux (5 x 7) and, between stages, the corrector (5 x 4); per cell and axis
# one face, the flux difference (10) and the accumulation of L (5).
def musta_flops_per_cell_axis(k):
    per_stage = 3 * (20 + 8) + 20 + 35
    return 80 + k * per_stage + (k - 1) * 20 + 10 + 5


# HBM values per cell that each sweep class must move in this split-sweep design:
# x sweep reads u (5) and writes L (5); y sweep reads u, L and writes L (15);
# z sweep reads u, L, u^n and writes the new state (20; 15 in stage 1); the
# fused x-y sweep reads u and writes L (10).
SWEEP_VALUES = {"sweep_x": 10.0, "sweep_y": 15.0, "sweep_z": (15.0 + 20.0 + 20.0) / 3.0, "sweep_xy": 10.0}
# directional sweeps per launch of each class (the fused class does two)
SWEEP_AXES = {"sweep_x": 1, "sweep_y": 1, "sweep_z": 1, "sweep_xy": 2}


def source_hash():
    h = hashlib.sha256()
    for name in ("rh_device.hpp", "rh_internal.hpp", "rh_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1604_03360_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_profile(precision, order=5):
    """Per-kernel counters of the committed rocprofv3 PMC summary of the scheme
    (HBM bytes and VALU wave instructions per launch), if it was taken on the
    current kernel sources (else {})."""
    name = "pmc_traffic_blob256.json" if order == 5 else "pmc_traffic_blob256_weno7.json"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    try:
        rec = json.load(open(path))
    except ValueError:
        return {}
    if rec.get("source_hash") != source_hash() or rec.get("order", 5) != order:
        return {}
    return rec.get("kernels", {}).get(precision, {})


def load_traffic(kernel, precision, order=5):
    """HBM traffic per launch of one sweep class from the PMC summary, or None."""
    ent = load_profile(precision, order).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


def load_trace_avg(kernel, precision, order=5):
    """Average launch time (ms) of one kernel class at 256^3 in the committed
    kernel trace of the default benchmark command, if taken on the current
    kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "bench_default_kernel_trace.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != source_hash():
        return None
    ent = rec.get("kernels", {}).get("%s|%s|%d" % (precision, kernel, order))
    return None if ent is None else ent.get("avg_ms_settled")


# one VALU wave instruction per CU per cycle is the nominal unpacked issue rate
# (4 SIMDs, a wave64 instruction every 4 cycles each): 256 CUs x 2.4 GHz
VALU_WAVE_ISSUE_PER_S = 256 * 2.4e9


def run_gpu(spec, precision, steps, warmup, path=None):
    import torch
    from paper_1604_03360_amd import rh
    prec = rh.RH_PREC_FP32 if precision == "fp32" else rh.RH_PREC_FP64
    h = rh.Hydro.from_spec(spec, precision=prec)
    if path is not None:
        rh.rh_set_path(h.plan, path)
    h.set_primitive(spec["prim"])
    u_init = h.state.clone()     # device copy of the initial state
    rh.rh_set_graph(h.plan, 1)   # steps replayed from one captured graph
    dt = spec["dt"]
    # Untimed clock settling before the warm-up steps: the GPU raises its clock
    # over the first few hundred milliseconds of sustained work (the same kernel
    # ran 10-40% longer in the first 50 ms of a run than after 0.3 s), so steps
    # are replayed until at least SETTLE_S seconds of them have run.
    settle_steps = 0
    s0 = time.perf_counter()
    while time.perf_counter() - s0 < SETTLE_S:
        h.step(dt, 4)
        torch.cuda.synchronize()
        settle_steps += 4
    # back to the initial state, so that the warm-up and timed steps are the
    # first steps of the run (the settling replays would otherwise carry the blob
    # to the end of its 200 steps, where the recovery's velocity cap acts); the
    # copy runs on the device, since an upload from the host would leave the GPU
    # idle long enough to lower its clock again
    h.state.copy_(u_init)
    del u_init
    h.t = spec["t0"]
    rh.rh_reset_counters(h.plan)
    if warmup:
        h.step(dt, warmup)
    stream = torch.cuda.current_stream()
    stream.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    h.step(dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    # per-kernel times from events the library records around each launch, in a
    # second run of the same length (the events themselves add a little time,
    # so the headline figure above is taken without them)
    rh.rh_set_timing(h.plan, 1)
    h.step(dt, steps)
    ktimes = rh.rh_kernel_times(h.plan)
    rh.rh_set_timing(h.plan, 0)
    tot, cnt = h.totals()
    h.close()
    del h
    torch.cuda.empty_cache()
    ncell = spec["shape"][0] * spec["shape"][1] * spec["shape"][2]
    return {"ms_per_step": ms_total / steps, "wall_s": wall, "value": ncell * steps / (ms_total * 1e-3),
            "kernels": ktimes, "totals": tot, "counters": cnt, "settle_steps": settle_steps}


def run_adjoint(spec, precision, reps, repeats=5):
    """Time the adjoint of one SSP-RK3 step with its stage states resident in HBM
    (recorded by rh_step_store), the same adjoint with the stage states
    recomputed (rh_step_vjp), and one forward step, all on the same plan with
    eager launches and no per-launch timing events: each figure is the median
    over `repeats` runs of `reps` calls.  The per-kernel adjoint times come from
    a separate pass with the library's per-launch events on."""
    import statistics

    import torch
    from paper_1604_03360_amd import rh
    prec = rh.RH_PREC_FP32 if precision == "fp32" else rh.RH_PREC_FP64
    h = rh.Hydro.from_spec(spec, precision=prec)
    h.set_primitive(spec["prim"])
    dt = spec["dt"]
    h.step(dt, 1)
    u_n = h.state.clone()
    t_n = h.t
    stages = h.step_store(dt)
    ubar = torch.randn_like(u_n)
    out = h.step_vjp_stored(u_n, stages, ubar, dt, t=t_n)     # warm-up, allocates scratch
    out = h.step_vjp(u_n, ubar, dt, t=t_n)
    stream = torch.cuda.current_stream()

    def per_call_ms(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {"stored": [], "recompute": [], "forward": []}
    for _ in range(repeats):
        res["stored"].append(per_call_ms(lambda: h.step_vjp_stored(u_n, stages, ubar, dt, t=t_n)))
        res["recompute"].append(per_call_ms(lambda: h.step_vjp(u_n, ubar, dt, t=t_n)))
        res["forward"].append(per_call_ms(lambda: h.step(dt, 1)))
    adj_ms = statistics.median(res["stored"])
    rec_ms = statistics.median(res["recompute"])
    fwd_ms = statistics.median(res["forward"])
    rh.rh_set_timing(h.plan, 1)
    for _ in range(reps):
        out = h.step_vjp_stored(u_n, stages, ubar, dt, t=t_n)
    kt = rh.rh_kernel_times(h.plan)
    rh.rh_set_timing(h.plan, 0)
    finite = bool(torch.isfinite(out).all().item())
    h.close()
    del h, u_n, ubar, out, stages
    torch.cuda.empty_cache()
    return {"step_vjp_ms": adj_ms, "step_ms": fwd_ms, "ratio": adj_ms / fwd_ms,
            "step_vjp_recompute_ms": rec_ms, "ratio_with_recompute": rec_ms / fwd_ms, "finite": finite,
            "ratio_range": [min(res["stored"]) / max(res["forward"]), max(res["stored"]) / min(res["forward"])],
            "timing": "median of %d runs of %d calls each, eager launches, no per-launch events" % (repeats, reps),
            "adjoint_sweeps_ms_per_step_vjp": kt["adjoint"][0] / reps}


def run_diff(n_steps=50, every=10):
    """The differentiable run: one 96^3 hot-spot event (FP32, WENO5), 50 steps with
    a checkpoint every 10, the anisotropy loss and its gradient with respect to the
    initial energy density through the autograd function.  Reports the forward
    time, the backward time (replays plus adjoint steps) and the adjoint of one
    step from stored stages against one forward step on this grid."""
    import torch
    from paper_1604_03360_amd import autograd, inputs, rh
    spec = inputs.diff_event(n=96)
    adj = run_adjoint(spec, "fp32", 10)
    h = rh.Hydro.from_spec(spec, precision=rh.RH_PREC_FP32)
    e0 = torch.tensor(spec["prim"][0], dtype=torch.float64, device="cuda").requires_grad_(True)
    z = torch.zeros_like(e0)

    def loss_and_grad():
        u0 = torch.stack([e0, z, z, z, e0 ** 0.75]).to(torch.float32)
        h.t = 0.0
        t0 = time.perf_counter()
        uT = autograd.run(u0, h, spec["dt"], n_steps, every)
        uT = uT.double()
        loss = (uT[1] ** 2 - uT[2] ** 2).sum() / uT[0].sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e0.grad = None
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    loss_and_grad()                    # warm-up
    fwd_s, bwd_s = loss_and_grad()
    h.close()
    del h, e0
    torch.cuda.empty_cache()
    return {"grid": [96, 96, 96], "steps": n_steps, "checkpoint_every": every,
            "forward_s": fwd_s, "backward_s": bwd_s, "backward_over_forward": bwd_s / fwd_s,
            "adjoint_step_ratio": adj["ratio"], "adjoint_step_ratio_with_recompute": adj["ratio_with_recompute"],
            "step_vjp_ms": adj["step_vjp_ms"], "step_ms": adj["step_ms"],
            "workload": "one 96^3 hot-spot event, FP32, WENO5, dt=0.06, gradient of sum(Mx^2-My^2)/sum(E) "
                        "at the final time with respect to the initial e"}


def run_batch(steps, warmup):
    """The 64-event hot-spot ensemble (FP32, WENO5): autotuned launch shapes,
    graph-captured steps; after the warm-up steps the events are reset to their
    initial state, resident in HBM, so that the timed steps are the ensemble's
    run (100 steps by default)."""
    import torch
    from paper_1604_03360_amd import inputs, rh
    specs = inputs.batch()
    b = rh.Batch(specs, precision=rh.RH_PREC_FP32)
    b.set_primitive([sp["prim"] for sp in specs])
    u_init = b.state.clone()     # device copy of the initial states
    ncell = sum(sp["shape"][0] * sp["shape"][1] * sp["shape"][2] for sp in specs)
    t0 = specs[0]["t0"]
    del specs
    tuning = rh.rh_batch_autotune(b.batch, 2)
    rh.rh_batch_set_graph(b.batch, True)
    dt = inputs.CFL * 0.15
    b.step(dt, warmup)
    # the timed steps are the ensemble's run from its initial state (restored on
    # the device, without an idle gap before the timed region)
    b.state.copy_(u_init)
    b.t = t0
    del u_init
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, cnt = b.totals()
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"value": ncell * steps / (ms * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms / steps,
            "steps": steps, "events": 64, "cells": ncell, "tuning": list(tuning), "graph": True,
            "counters": cnt,
            "workload": "64 hot-spot events, cubes of 64..160 cells, FP32, WENO5, periodic, "
                        "dx=0.15, dt=0.06, one batch"}


def run_schemes(n, steps, warmup):
    """The 256^3 blob with the other schemes of the library, each one fused launch
    per stage: MUSTA-FORCE (minmod, two stages, the paper's other scheme) in FP32
    and FP64, WENO5 with local Lax-Friedrichs splitting (FP32), and WENO5 with the
    ideal gas (gamma 5/3, FP32; the blob heated so that e > n).  The fused WENO5
    stage with global splitting is timed beside them for reference."""
    from paper_1604_03360_amd import inputs, rh
    base = inputs.blob(n=n, order=5)
    ncell = n ** 3
    legs = {
        "musta_fp32": (inputs.with_scheme(base, order=2, limiter=0, musta_k=2), "fp32"),
        "musta_fp64": (inputs.with_scheme(base, order=2, limiter=0, musta_k=2), "fp64"),
        "weno5_stage_fp32": (base, "fp32"),
        "weno5_local_split_fp32": (inputs.with_scheme(base, lf_local=True), "fp32"),
        "weno5_ideal_gas_fp32": (inputs.with_scheme(inputs.hot_gas(base), eos=1, gamma=5.0 / 3.0), "fp32"),
    }
    out = {}
    for name, (sp, prec) in legs.items():
        r = run_gpu(sp, prec, steps, warmup, path=rh.RH_PATH_STAGE)
        ms, launches = r["kernels"]["stage"]
        ent = {"value": r["value"], "unit": "cell-updates/s", "ms_per_step": r["ms_per_step"],
               "stage_launch_ms": ms / launches, "counters": r["counters"]}
        oms, olaunches = r["kernels"]["other"]
        if "ideal" in name and olaunches > 0:
            ent["recovery_launch_ms"] = oms / olaunches   # the per-cell Newton pass before each stage
        if name.startswith("musta"):
            flops = 3 * musta_flops_per_cell_axis(2) * ncell
            achieved = flops / (ms / launches * 1e-3) / 1e12
            ent["roofline"] = {"bound": "alu", "kernel": "stage_musta", "achieved": round(achieved, 3),
                               "peak": ALU_PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                               "frac": round(achieved / ALU_PEAK_TFLOPS[prec], 4),
                               "flops_per_cell_launch": 3 * musta_flops_per_cell_axis(2)}
        out[name] = ent
        print("bench: %s %.4g cell-updates/s (%.3f ms/step)" % (name, r["value"], r["ms_per_step"]),
              file=sys.stderr, flush=True)
    out["musta_over_weno5_time"] = out["weno5_stage_fp32"]["value"] / out["musta_fp32"]["value"]
    out["workload"] = "%d^3 blob, %d steps each, fused stage; MUSTA-FORCE minmod, 2 stages, local dt/dx 0.9" % (n, steps)
    return out


def musta_cpu_sample(gpu_value):
    """The paper's only speed figure compares its MUSTA-FORCE GPU program with a
    single-threaded CPU one.  For context: the oracle's MUSTA-FORCE, one thread,
    one step of the blob at 64^3, against the FP32 GPU figure of the leg above."""
    import oracle
    from paper_1604_03360_amd import inputs
    sp = inputs.with_scheme(inputs.blob(n=64, order=5), order=2, limiter=0, musta_k=2)
    g = oracle.grid_from_spec(sp)
    u = oracle.prim2con(sp["prim"])
    cores = oracle.num_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step(g, u, sp["dt"], 1)
        el = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    v = 64 ** 3 / el
    return {"value": v, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "1 MUSTA-FORCE SSP-RK3 step of the blob at 64^3 (dx 0.1), FP64, %.1f s" % el,
            "gpu_fp32_over_this": gpu_value / v}


def hubble_field_errors(n=128, nsteps=100):
    """Per-field error of the 128^3 Hubble-like flow after its 100 steps: the FP32
    and FP64 GPU states against the FP64 oracle (normalised L-infinity,
    max|gpu - oracle| / max|oracle| per field), and the energy density of each
    against the closed form on interior cells."""
    import numpy as np
    import torch
    import oracle
    from paper_1604_03360_amd import inputs, rh
    spec = inputs.hubble(n=n)
    g = oracle.grid_from_spec(spec)
    t0 = time.perf_counter()
    ref, t_end = oracle.step(g, oracle.prim2con(spec["prim"]), spec["dt"], nsteps, t=spec["t0"])
    cpu_s = time.perf_counter() - t0
    names = ("E", "Mx", "My", "Mz", "N")
    out = {"grid": [n] * 3, "steps": nsteps, "t_end": t_end, "oracle_s": round(cpu_s, 1),
           "norm": "max|gpu - oracle| / max|oracle| per field"}
    for prec, code in (("fp32", rh.RH_PREC_FP32), ("fp64", rh.RH_PREC_FP64)):
        h = rh.Hydro.from_spec(spec, precision=code)
        h.set_primitive(spec["prim"])
        h.step(spec["dt"], nsteps)
        got = h.get()
        h.close()
        del h
        torch.cuda.empty_cache()
        d = np.abs(got - ref).reshape(5, -1).max(1) / np.abs(ref).reshape(5, -1).max(1)
        out[prec] = {k: float(v) for k, v in zip(names, d)}
    return out


def copy_rate(nbytes=1 << 30, reps=20):
    """Rate (GB/s, bytes read plus bytes written) of a plain device-to-device copy
    of 1 GiB, timed with events after the same clock settling as the timed runs:
    the rate the part streams half reads, half writes with no arithmetic, a
    reference for the HBM-bound sweeps (streams with fewer writes can exceed it)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s0 = time.perf_counter()
    while time.perf_counter() - s0 < SETTLE_S:
        b.copy_(a)
        torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def roofline(run, precision, order, ncell, copy_GBps=None):
    elem = 4 if precision == "fp32" else 8
    kern = {k: v for k, v in run["kernels"].items() if k.startswith("sweep") and v[1] > 0}
    dom = max(kern, key=lambda k: kern[k][0])
    ms, launches = kern[dom]
    avg_s = ms / launches * 1e-3
    flops_cell = SWEEP_AXES[dom] * sweep_flops_per_cell(order)
    flops = flops_cell * ncell
    achieved = flops / avg_s / 1e12
    peak = ALU_PEAK_TFLOPS[precision]
    alg_bytes = SWEEP_VALUES[dom] * elem * ncell
    traffic = load_traffic(dom, precision, order)
    hbm = {
        "kernel": dom, "design_bytes_per_launch": alg_bytes,
        "achieved_GBps": round(alg_bytes / avg_s / 1e9, 1), "peak_GBps": HBM_PEAK_GBS,
        "frac": round(alg_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4),
    }
    if traffic:
        # counted HBM bytes (copy-calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE) over
        # the same live launch time
        hbm["counted_bytes_per_launch"] = traffic
        hbm["counted_GBps"] = round(traffic / avg_s / 1e9, 1)
        hbm["counted_frac"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    # whole step: algorithmic bytes (read the stage input in all three stages and
    # u^n in stages 2 and 3, write each stage's output: 40 values per cell-update)
    # and, from the PMC summary, the counted bytes of all sweep launches
    step_s = run["ms_per_step"] * 1e-3
    alg_step = 40.0 * elem * ncell
    hbm["step_alg"] = {"bytes": alg_step, "GBps": round(alg_step / step_s / 1e9, 1),
                       "frac": round(alg_step / step_s / 1e9 / HBM_PEAK_GBS, 4)}
    prof = load_profile(precision, order)
    if copy_GBps:
        hbm["copy_GBps"] = round(copy_GBps, 1)
        hbm["copy_frac_of_peak"] = round(copy_GBps / HBM_PEAK_GBS, 4)
    # every sweep class of the step: counted bytes over its live launch time, against
    # the peak and against the plain copy's rate
    per_class = {}
    for k, (kms, kl) in kern.items():
        if k in prof and "bytes_per_launch" in prof[k]:
            gbps = prof[k]["bytes_per_launch"] / (kms / kl * 1e-3) / 1e9
            ent = {"ms_per_launch": round(kms / kl, 4), "counted_bytes_per_launch": prof[k]["bytes_per_launch"],
                   "counted_GBps": round(gbps, 1), "counted_frac": round(gbps / HBM_PEAK_GBS, 4)}
            if copy_GBps:
                ent["of_copy_rate"] = round(gbps / copy_GBps, 4)
            per_class[k] = ent
    if per_class:
        hbm["sweeps"] = per_class
    if all(k in prof and "bytes_per_launch" in prof[k] for k in kern):
        # every sweep class of the step, three launches each (one per stage)
        counted = 3.0 * sum(prof[k]["bytes_per_launch"] for k in kern)
        hbm["step_counted"] = {"bytes": counted, "GBps": round(counted / step_s / 1e9, 1),
                               "frac": round(counted / step_s / 1e9 / HBM_PEAK_GBS, 4)}
    valu = None
    if dom in prof and "SQ_INSTS_VALU" in prof[dom] and prof[dom].get("_dur_valu_run"):
        # counted VALU wave instructions over the duration of the same counter
        # pass's dispatch (not this run's event time), per CU and clock cycle
        ent = prof[dom]
        wi, dur = ent["SQ_INSTS_VALU"], ent["_dur_valu_run"]
        rate = wi / dur / VALU_WAVE_ISSUE_PER_S
        valu = {"kernel": dom, "wave_instr_per_launch": wi, "instr_per_cell": round(wi * 64 / ncell, 1),
                "time_base": "dispatch duration in the counter pass (%.1f us)" % (dur * 1e6),
                "wave_instr_per_cu_cycle_at_2.4GHz": round(rate, 4)}
        if ent.get("clock_ghz"):
            valu["clock_ghz_measured"] = round(ent["clock_ghz"], 3)
            valu["wave_instr_per_cu_cycle"] = round(wi / dur / (256 * ent["clock_ghz"] * 1e9), 4)
        if ent.get("valu_busy") is not None:
            valu["valu_busy"] = round(ent["valu_busy"], 4)
    out = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4), "traffic": traffic,
        "kernel": dom, "avg_launch_ms": round(ms / launches, 4),
        "flops_per_cell": flops_cell, "valu": valu,
    }
    tr = load_trace_avg(dom, precision, order)
    if tr:
        # the same figure from the committed kernel trace of the default command
        out["trace_avg_launch_ms"] = round(tr, 4)
        out["frac_trace"] = round(flops / (tr * 1e-3) / 1e12 / peak, 4)
    return dom, out, hbm


def cpu_baseline(spec, nsteps):
    import oracle
    oracle.build()
    g = oracle.grid_from_spec(spec)
    u = oracle.prim2con(spec["prim"])
    t0 = time.perf_counter()
    oracle.step(g, u, spec["dt"], nsteps)
    el = time.perf_counter() - t0
    ncell = spec["shape"][0] * spec["shape"][1] * spec["shape"][2]
    cores = oracle.num_threads()
    out = {"value": ncell * nsteps / el, "unit": "cell-updates/s", "cores": cores,
           "kind": "oracle",
           "sample": "%d whole-grid SSP-RK3 step(s) of the same %d^3 WENO%d blob, FP64, %.1f s"
                     % (nsteps, spec["shape"][0], spec["order"], el)}
    # single-threaded, as the paper's CPU comparison: one step of the blob at 96^3
    from paper_1604_03360_amd import inputs
    small = inputs.blob(n=96, order=spec["order"])
    g1 = oracle.grid_from_spec(small)
    u1 = oracle.prim2con(small["prim"])
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step(g1, u1, small["dt"], 1)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    out["single_thread"] = {"value": 96 ** 3 / el1, "unit": "cell-updates/s", "cores": 1,
                            "sample": "1 SSP-RK3 step of the blob at 96^3 (dx 0.1), FP64, %.1f s" % el1}
    # the whole 200-step blob run at these rates, and the host it was measured on
    out["full_run_200_steps_s"] = {"all_cores": 200 * ncell / out["value"],
                                   "one_thread": 200 * ncell / out["single_thread"]["value"]}
    out["host"] = {"nproc": os.cpu_count(), "cpu_model": cpu_model()}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--scheme", type=int, default=5, choices=(5, 7))
    ap.add_argument("--cpu-steps", type=int, default=5,
                    help="whole-grid oracle steps timed for cpu_baseline (about 12 s on 16 host cores)")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="timed steps of the 64-event ensemble (its configured run length)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-weno7", action="store_true")
    ap.add_argument("--no-schemes", action="store_true")
    ap.add_argument("--no-hubble", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy three times (reference "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this benchmark measures one GPU only (the path has no multi-GPU mode); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1604_03360_amd import inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    spec = inputs.blob(n=args.n, order=args.scheme)
    ncell = args.n ** 3
    print("bench: blob %d^3 WENO%d, %d warmup + %d timed steps" % (args.n, args.scheme, args.warmup,
                                                                  args.steps), file=sys.stderr, flush=True)
    copy_GBps = copy_rate()
    r32 = run_gpu(spec, "fp32", args.steps, args.warmup)
    print("bench: fp32 %.4g cell-updates/s (%.3f ms/step)" % (r32["value"], r32["ms_per_step"]),
          file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(spec, "fp64", args.steps, args.warmup)
        print("bench: fp64 %.4g cell-updates/s (%.3f ms/step)" % (r64["value"], r64["ms_per_step"]),
              file=sys.stderr, flush=True)
    def side_leg(name, fn):
        # the side legs add context to the headline figure; a failure in one of
        # them (an error status from the library, say) is reported in its block
        # instead of losing the whole line
        try:
            return fn()
        except Exception as e:  # noqa: BLE001
            import traceback
            traceback.print_exc()
            print("bench: %s leg failed: %s" % (name, e), file=sys.stderr, flush=True)
            return {"error": "%s: %s" % (type(e).__name__, e)}

    def weno7_leg():
        # the same blob with WENO7, FP32 and FP64 (steps replayed from the graph)
        spec7 = inputs.blob(n=args.n, order=7)
        w = {}
        for prec in ("fp32", "fp64"):
            r = run_gpu(spec7, prec, min(args.steps, 10), min(args.warmup, 2))
            _, roof7, hbm7 = roofline(r, prec, 7, ncell)
            w[prec] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "roofline": roof7, "hbm": hbm7,
                       "kernels_ms_per_step": {k: v[0] / min(args.steps, 10) for k, v in r["kernels"].items()}}
        w["fp32_over_fp64"] = w["fp32"]["value"] / w["fp64"]["value"]
        print("bench: WENO7 fp32 %.4g, fp64 %.4g cell-updates/s" % (w["fp32"]["value"], w["fp64"]["value"]),
              file=sys.stderr, flush=True)
        return w

    def adjoint_leg():
        a = run_adjoint(spec, "fp32", 3)
        print("bench: adjoint step %.3f ms (%.3f ms with recomputation) vs forward step %.3f ms "
              "(ratio %.2f, %.2f)" % (a["step_vjp_ms"], a["step_vjp_recompute_ms"], a["step_ms"],
                                      a["ratio"], a["ratio_with_recompute"]), file=sys.stderr, flush=True)
        return a

    def diff_leg():
        d = run_diff()
        print("bench: 96^3 differentiable run: forward %.3f s, backward %.3f s; adjoint step ratio %.2f"
              % (d["forward_s"], d["backward_s"], d["adjoint_step_ratio"]), file=sys.stderr, flush=True)
        return d

    def batch_leg():
        b = run_batch(args.batch_steps, 2)
        print("bench: batch %.4g cell-updates/s (%.3f ms/step)" % (b["value"], b["ms_per_step"]),
              file=sys.stderr, flush=True)
        return b

    def schemes_leg():
        sc = run_schemes(args.n, min(args.steps, 10), min(args.warmup, 2))
        if not args.no_cpu_baseline:
            sc["musta_cpu_single_thread"] = side_leg("MUSTA CPU sample",
                                                     lambda: musta_cpu_sample(sc["musta_fp32"]["value"]))
        return sc

    def hubble_leg():
        hf = hubble_field_errors()
        print("bench: Hubble 128^3 after 100 steps, FP32 per-field error vs the FP64 oracle %s"
              % hf["fp32"], file=sys.stderr, flush=True)
        return hf

    # the configured workloads first (the ensemble, the adjoint and the
    # differentiable run), then the other schemes: a long run heats the part,
    # and later legs run at a somewhat lower clock
    bat = side_leg("batch", batch_leg) if not args.no_batch else None
    adj = side_leg("adjoint", adjoint_leg) if not args.no_adjoint else None
    diff = side_leg("differentiable run", diff_leg) if not args.no_adjoint else None
    w7 = side_leg("WENO7", weno7_leg) if args.scheme == 5 and not args.no_weno7 else None
    sch = side_leg("schemes", schemes_leg) if not args.no_schemes else None
    hub = side_leg("Hubble per-field errors", hubble_leg) if not args.no_hubble else None
    dom, roof, hbm = roofline(r32, "fp32", args.scheme, ncell, copy_GBps)
    out = {
        "metric": METRIC, "value": r32["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ellipsoidal Gaussian blob at rest, %d^3 periodic, dx=0.1, dt=0.04, "
                               "WENO%d + global Lax-Friedrichs, SSP-RK3, p=e/3" % (args.n, args.scheme),
                   "grid": [args.n] * 3, "precision": "FP32 storage/stencil/RK, FP64 primitive recovery",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "hbm": hbm,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in r32["kernels"].items()},
        "counters": r32["counters"],
    }
    if w7 is not None:
        out["weno7"] = w7
    if adj is not None:
        out["adjoint"] = dict(adj, workload="same grid, FP32: adjoint of one SSP-RK3 step with its "
                                           "stage states resident / one forward step; with the stage "
                                           "states recomputed in ratio_with_recompute")
    if diff is not None:
        out["differentiable_run"] = diff
    if bat is not None:
        out["batch"] = bat
    if sch is not None:
        out["schemes"] = sch
    if hub is not None:
        out["fp32_error_per_field"] = hub
    if r64 is not None:
        _, roof64, hbm64 = roofline(r64, "fp64", args.scheme, ncell, copy_GBps)
        out["fp64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                       "fp32_over_fp64": r32["value"] / r64["value"], "roofline": roof64, "hbm": hbm64,
                       "kernels_ms_per_step": {k: v[0] / args.steps for k, v in r64["kernels"].items()}}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = side_leg("CPU baseline", lambda: cpu_baseline(spec, args.cpu_steps))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
