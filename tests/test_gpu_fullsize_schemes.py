"""Parity of the other schemes at the benchmark's full size, in the launch
configuration it times (the fused stage with its default tile and segment):
the 256^3 blob, one SSP-RK3 step, every cell of every field against the FP64
oracle's step.

* MUSTA-FORCE (minmod, two stages, local dt/dx 0.9), FP64 and FP32;
* WENO5 with local Lax-Friedrichs splitting, FP32;
* WENO5 with the ideal gas (gamma 5/3, the blob heated so that e > n), FP32.

Bars: 1e-12 (FP64) and 2e-5 (FP32), normalised L-infinity per field.
"""
import numpy as np
import pytest

import oracle
from paper_1604_03360_amd import inputs
from gpu_helpers import field_errors, rh_module

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _workload(name):
    base = inputs.blob(n=256, order=5)
    if name == "musta":
        return inputs.with_scheme(base, order=2, limiter=0, musta_k=2, musta_cfl=0.9)
    if name == "local_split":
        return inputs.with_scheme(base, lf_local=True)
    return inputs.with_scheme(inputs.hot_gas(base), eos=1, gamma=5.0 / 3.0)


@pytest.mark.parametrize("name,precision,tol", [("musta", "fp64", 1e-12), ("musta", "fp32", 2e-5),
                                                ("local_split", "fp32", 2e-5),
                                                ("ideal_gas", "fp32", 2e-5)])
def test_blob_256_one_step(name, precision, tol):
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    spec = _workload(name)
    print("blob 256^3 %s %s" % (name, precision), flush=True)
    h = rh.Hydro.from_spec(spec, precision=prec)
    assert rh.rh_get_path(h.plan) == rh.RH_PATH_STAGE
    h.set_primitive(spec["prim"])
    h.step(spec["dt"], 1)
    got = h.get()
    _, cnt = h.totals()
    h.close()
    g = oracle.grid_from_spec(spec)
    print("oracle ...", flush=True)
    ref, _ = oracle.step(g, oracle.prim2con_eos(g, spec["prim"]), spec["dt"], 1)
    err = field_errors(got, ref)
    print(err, cnt, flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(err <= tol), err
    assert cnt[1] == 0
