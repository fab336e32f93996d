"""The largest grids the boundary accepts, on the path the benchmark times.

A plan takes a grid whose every field is below 4 GiB (the kernels address a
field with 32-bit byte offsets from its base).  The grids here come within 2% of
that: 256 x 2048 x 2016 cells in FP32 and 256 x 2048 x 1008 in FP64 (about 85 GB
of state and workspace on the device), stepped on the default path (fused x-y
sweep, z roll, graph replays).

The oracle cannot step a billion cells, so the initial data repeat with a period
of 16 cells along every axis (a smooth periodic field on one 16^3 tile, copied)
and the grid is periodic with a multiple of that period.  Every cell then runs
the same arithmetic on the same neighbourhood, so every 16^3 tile of the result
must equal every other one bit for bit -- a wrong offset anywhere in the far
reaches of a field breaks this -- and tile 0 must match the FP64 oracle run on a
single 16^3 periodic tile (1e-12 FP64, 2e-5 FP32 per field).  A small grid takes
the same checks.
"""
import numpy as np
import pytest
import torch

from paper_1604_03360_amd import inputs
from gpu_helpers import field_errors, oracle_steps, rh_module

pytestmark = pytest.mark.gpu

P = 16        # period of the initial data, cells per axis
STEPS = 2

FIELD_LIMIT = 1 << 32


def tile_spec(order):
    return inputs.random_smooth((P, P, P), h=0.1, seed=11, order=order)


def run_tiled(shape, precision, order):
    """Steps the grid `shape` filled with copies of the 16^3 tile; returns whether
    all tiles are bitwise equal, tile 0 (FP64 host copy) and the counters."""
    rh = rh_module()
    nx, ny, nz = shape
    assert nx % P == 0 and ny % P == 0 and nz % P == 0
    tile = tile_spec(order)
    spec = dict(tile, shape=tuple(shape), prim=None)
    h = rh.Hydro.from_spec(spec, precision=precision)
    try:
        prim = torch.as_tensor(tile["prim"], device="cuda").repeat(1, nz // P, ny // P, nx // P)
        h.set_primitive(prim)
        del prim
        rh.rh_set_graph(h.plan, 1)
        h.step(tile["dt"], STEPS)
        _, cnt = h.totals()
        st = h.state.view(5, nz // P, P, ny // P, P, nx // P, P)
        ref = st[:, :1, :, :1, :, :1, :]
        same = all(torch.equal(st[f], ref[f].expand_as(st[f])) for f in range(5))
        tile0 = st[:, 0, :, 0, :, 0, :].double().cpu().numpy()
        del st, ref
    finally:
        h.close()
        del h
        torch.cuda.empty_cache()
    return same, tile0, cnt


CASES = [
    # shape, precision, order, tolerance against the oracle
    ((64, 48, 32), "fp32", 5, 2e-5),
    ((64, 48, 32), "fp64", 7, 1e-12),
    ((256, 2048, 2016), "fp32", 5, 2e-5),
    ((256, 2048, 1008), "fp64", 5, 1e-12),
    ((256, 2048, 2016), "fp32", 7, 2e-5),
]


@pytest.mark.parametrize("shape,precision,order,tol", CASES)
def test_tiled_grid_matches_one_tile(shape, precision, order, tol):
    rh = rh_module()
    prec = rh.RH_PREC_FP32 if precision == "fp32" else rh.RH_PREC_FP64
    field_bytes = shape[0] * shape[1] * shape[2] * (4 if precision == "fp32" else 8)
    assert field_bytes < FIELD_LIMIT
    print("grid %s %s WENO%d, %.3f of the field limit" % (shape, precision, order, field_bytes / FIELD_LIMIT),
          flush=True)
    same, tile0, cnt = run_tiled(shape, prec, order)
    assert same
    assert cnt == [0, 0]
    ref, _ = oracle_steps(tile_spec(order), STEPS)
    err = field_errors(tile0, ref)
    print("tile 0 against the oracle", err, flush=True)
    assert np.all(err <= tol), err
