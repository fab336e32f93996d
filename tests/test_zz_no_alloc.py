"""The allocation-free totals entry point (rh_totals_noalloc) against rh_totals,
which computes the same reduction with plan-owned partials.  Two calls in a
row on one device share the library's static scratch array; the second has a
smaller input, so a stale partial of the first call would show."""
import numpy as np
import pytest

from gpu_helpers import rh_module
from paper_1604_03360_amd import inputs


def _totals_both(rh, torch, shape, precision, seed, poison=None):
    spec = inputs.random_smooth(shape, h=0.1, seed=seed)
    h = rh.Hydro.from_spec(spec, precision=precision)
    h.set_primitive(spec["prim"])
    h.step(spec["dt"], 1)
    if poison is not None:
        h.state.view(5, -1)[poison] = float("nan")
        torch.cuda.current_stream().synchronize()
    ref, cnt = h.totals()
    ncell = int(np.prod(shape))
    out = torch.full((6,), -1.0, dtype=torch.float64, device="cuda")
    rh.rh_totals_noalloc(h.state.data_ptr(), precision, ncell, out.data_ptr(), h.stream_ptr())
    got = out.cpu().numpy()
    h.close()
    return np.array(ref), cnt, got


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_totals_noalloc_equals_rh_totals(precision):
    import torch
    rh = rh_module()
    prec = rh.RH_PREC_FP64 if precision == "fp64" else rh.RH_PREC_FP32
    # larger input first, then a smaller one (fewer cells than reduction blocks
    # times 256 lanes, so most partial slots of the second call are sums over
    # empty ranges), then one with non-finite cells
    for shape, seed, poison in (((61, 37, 29), 3, None), ((9, 7, 5), 4, None),
                                ((23, 11, 13), 5, (2, slice(100, 107)))):
        ref, cnt, got = _totals_both(rh, torch, shape, prec, seed, poison)
        print("noalloc totals", precision, shape, got, flush=True)
        if poison is None:
            assert np.array_equal(got[:5], ref), (got, ref)   # same kernels, same bits
        else:
            assert np.array_equal(got[:5], ref, equal_nan=True), (got, ref)
        assert got[5] == cnt[1]


@pytest.mark.gpu
def test_totals_noalloc_rejects_bad_arguments():
    import torch
    rh = rh_module()
    buf = torch.zeros((5, 8), dtype=torch.float64, device="cuda")
    out = torch.zeros(6, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for args in ((0, rh.RH_PREC_FP64, 8, out.data_ptr()), (buf.data_ptr(), 7, 8, out.data_ptr()),
                 (buf.data_ptr(), rh.RH_PREC_FP64, 0, out.data_ptr()),
                 (buf.data_ptr(), rh.RH_PREC_FP64, rh.RH_NOALLOC_MAX_BYTES // 8 + 1, out.data_ptr()),
                 (buf.data_ptr(), rh.RH_PREC_FP64, 8, 0)):
        with pytest.raises(rh.RHError) as ei:
            rh.rh_totals_noalloc(*args, s)
        assert ei.value.status == rh.RH_E_INVAL
