"""The entry point that allocates nothing (sscg_apply_A_noalloc) against sscg_apply_A,
called through the C-ABI on the same inputs: two calls in a row on one context, the
second with a smaller input (fewer sources), in FP64 and FP32; the array it stages in
is shared, so the second call must not see the first one's data. Bars: FP64 1e-14 and
FP32 2e-6 per vector (max-abs, relative to the vector's largest entry), as for apply_A
against the oracle; bitwise once sscg_apply_A has tuned the launch shape the no-alloc
call then reuses. Requests beyond the 16 MiB staging are refused on the host."""
import numpy as np
import pytest

import synth
from tests.helpers import case, to_dev, to_host, vec_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name,bar", [("fp64", 1e-14), ("fp32", 2e-6)])
def test_apply_A_noalloc_matches_apply_A(sscg, prec_name, bar):
    prec = sscg.FP64 if prec_name == "fp64" else sscg.MIXED
    dims, kappa = (8, 8, 8, 8), 0.125
    case(f"apply_A_noalloc {prec_name} {dims}: nsrc 4 then 1")
    U = synth.gauge_field(dims, 0.5, 21)
    c = sscg.Context(dims, kappa)
    c.set_gauge(U, 12 if prec_name == "fp32" else 18)
    V = int(np.prod(dims))
    for call, nsrc, seed in ((1, 4, 31), (2, 1, 32)):
        x = to_dev(synth.sources(V, nsrc, seed))
        y0 = to_dev(np.zeros((nsrc, V, 4, 3)))
        y1 = to_dev(np.zeros((nsrc, V, 4, 3)))
        c.apply_A_noalloc(x, y0, prec)        # before any tuning: the default launch shape
        c.apply_A(x, y1, prec)                # tunes (prec, nsrc)
        a, b = to_host(y0).reshape(nsrc, -1), to_host(y1).reshape(nsrc, -1)
        assert vec_err(a, b) <= bar, (call, vec_err(a, b))
        y2 = to_dev(np.zeros((nsrc, V, 4, 3)))
        c.apply_A_noalloc(x, y2, prec)        # the shape just tuned: the same kernels
        assert np.array_equal(to_host(y2), to_host(y1)), call
    c.close()


def test_apply_A_noalloc_rejects_oversize(sscg):
    case("apply_A_noalloc oversize request")
    dims = (16, 16, 16, 16)                   # 786432 entries per vector
    c = sscg.Context(dims, 0.13)
    c.set_gauge(synth.unit_gauge(dims))
    V = int(np.prod(dims))
    x = to_dev(np.zeros((2, V, 4, 3)))
    y = to_dev(np.zeros((2, V, 4, 3)))
    with pytest.raises(sscg.SSCGError) as e:
        c.apply_A_noalloc(x, y, sscg.FP64)    # 2 x 786432 > 1048576 FP64 entries
    assert e.value.code == sscg.EINVAL
    c.apply_A_noalloc(x[:1].contiguous(), y[:1].contiguous(), sscg.FP64)   # one source fits
    c.close()
