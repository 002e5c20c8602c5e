"""Gauge covariance of the library's update (the symmetry of Sec. 2), on the GPU
through the C ABI: evolving the gauge-transformed state gives the transformed
evolved state, and the measured observables do not change.  A property that
holds at any size, checked here at a size of several tiles with ragged tails, in
both plane layouts (single steps; pairs of steps) and both precisions."""
import math

import numpy as np
import pytest

from tests import inputs as I

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import fields_np, group_errors, upload  # noqa: E402

SHAPE = (128, 12, 10)


@pytest.mark.parametrize("layout", [AH.AH_LAYOUT_15, AH.AH_LAYOUT_20], ids=["l15", "l20"])
@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32], ids=["fp64", "fp32"])
def test_update_is_gauge_covariant(prec, layout):
    print("CASE test=gauge_covariance prec", prec, "layout", layout, flush=True)
    st = I.random_state(SHAPE, seed=41)
    alpha = I.gauge_function(SHAPE, seed=42)
    gst = I.gauge_transform(st, alpha)
    if prec == AH.AH_FP32:
        st, gst = (x.astype(np.float32).astype(np.float64) for x in (st, gst))
    p = AH.Params(*SHAPE, precision=prec, tau0=2.0, tau_ref=4.0, era_p=1.0, s=1.0,
                  init=AH.AH_INIT_NONE, layout=layout)
    out, obs = [], []
    for s0 in (st, gst):
        with AH.Context([p], [upload(p, s0)]) as c:
            c.step(8)
            (o,) = c.measure()
            out.append(fields_np(c))
            obs.append(o)
    err = group_errors(out[1], I.gauge_transform(out[0], alpha))
    print("  max rel err per group", {k: f"{v:.1e}" for k, v in err.items()}, flush=True)
    assert max(err.values()) < (1e-12 if prec == AH.AH_FP64 else 1e-5), err
    a, b = obs
    rel = 1e-10 if prec == AH.AH_FP64 else 1e-4
    scale = abs(a.energy)   # sums with cancellations (sum_lag) are compared on the energy's scale
    for k in ("kin", "grad", "elec", "mag", "pot", "energy", "sum_lag"):
        assert getattr(b, k) == pytest.approx(getattr(a, k), rel=rel, abs=rel * scale), k
    for gv, av in zip(b.v2, a.v2):
        assert (math.isnan(gv) and math.isnan(av)) or gv == pytest.approx(av, rel=rel, abs=1e-12)
    # windings: integers, equal unless a phase difference sits within rounding of pi
    assert b.net_wind_dir == a.net_wind_dir == [0, 0, 0]
    assert abs(b.n_wind - a.n_wind) <= (0 if prec == AH.AH_FP64 else 4), (a.n_wind, b.n_wind)
