"""ah_measure_noalloc (no context, no allocation: the library's static device
scratch) against ah_measure on the same states, through the C ABI.

Two calls in a row, the second with fewer and smaller realizations, in both
precisions: every count and the winding map equal ah_measure's exactly, every
FP64 sum to 1e-12 relative (only the order of the per-block atomic additions
differs).  The second call also leaves the free device memory unchanged.
"""
import dataclasses

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from paper_1809_00995_amd import ah as B  # noqa: E402

SUMS = ("sum_lag", "kin", "grad", "elec", "mag", "pot", "energy", "pres", "pres_lag", "rho_lag",
        "v2_eos", "xi_l")


def _compare(got, ref):
    for r, (g, o) in enumerate(zip(got, ref)):
        assert (g.step, g.n_wind, g.n_wind_dir, g.net_wind_dir, g.n_pierced, g.nonfinite) == \
            (o.step, o.n_wind, o.n_wind_dir, o.net_wind_dir, o.n_pierced, o.nonfinite), r
        assert (g.tau, g.a, g.length, g.xi_w) == (o.tau, o.a, o.length, o.xi_w), r
        for k in SUMS:
            assert getattr(g, k) == pytest.approx(getattr(o, k), rel=1e-12, abs=0, nan_ok=True), \
                (r, k)
        for k in ("num", "den", "v2"):
            assert np.allclose(getattr(g, k), getattr(o, k), rtol=1e-11, atol=0), (r, k)


def _reference(shapes, prec, steps):
    """Realizations from the seeded random phase advanced `steps` single steps
    (even: the state is back in planes 0-9), and ah_measure of them."""
    ps = [AH.Params(nx, ny, nz, precision=prec, tau0=0.0, tau_ref=4.0, era_p=1.0 + (k % 2),
                    s=1.0 - (k % 2), seed=50 + k, layout=AH.AH_LAYOUT_15)
          for k, (nx, ny, nz) in enumerate(shapes)]
    planes = [AH.alloc_planes(p) for p in ps]
    ctx = AH.Context(ps, planes)
    ctx.step(steps)
    for r in range(len(ps)):
        assert ctx.current_planes(r) == list(range(10))
    ref, maps = ctx.measure(wind=True)
    qs = [dataclasses.replace(p, step0=ctx.current_step(r), init=AH.AH_INIT_NONE)
          for r, p in enumerate(ps)]
    ctx.close()
    return qs, planes, ref, maps


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_noalloc_measure_equals_measure_on_two_calls(prec):
    # tiled shapes with ragged y and z tails and a plain-kernel shape; then one smaller lattice
    calls = [[(128, 12, 10), (64, 16, 12), (40, 12, 10)], [(64, 8, 6)]]
    stream = torch.cuda.Stream()
    for k, shapes in enumerate(calls):
        print(f"CASE test=noalloc prec={prec} call={k} shapes={shapes}", flush=True)
        qs, planes, ref, maps = _reference(shapes, prec, steps=6)
        n = len(qs)
        out = torch.full((n * B.OBS_BYTES,), 0xAB, dtype=torch.uint8, device="cuda")
        wind = torch.full((sum(3 * q.sites for q in qs),), 7, dtype=torch.int8, device="cuda")
        torch.cuda.synchronize()
        free_before = torch.cuda.mem_get_info()[0]
        AH.measure_noalloc(qs, planes, out, wind, stream=stream)
        stream.synchronize()
        if k > 0:
            assert torch.cuda.mem_get_info()[0] == free_before
        _compare(AH.obs_from_bytes(out.cpu(), n), ref)
        off = 0
        for q, m in zip(qs, maps):
            got = wind[off:off + 3 * q.sites].view(3, q.nz, q.ny, q.nx)
            assert torch.equal(got, m)
            off += 3 * q.sites


def test_noalloc_measure_rejects_sizes_beyond_its_scratch():
    p = AH.Params(64, 8, 8)
    t = AH.alloc_planes(p)
    out = torch.zeros(B.OBS_BYTES * (B.AH_NOALLOC_MAX_REAL + 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(AH.AHError) as e:
        AH.measure_noalloc([p] * (B.AH_NOALLOC_MAX_REAL + 1), [t] * (B.AH_NOALLOC_MAX_REAL + 1), out)
    assert e.value.code == B.AH_E_INVALID and "static scratch" in str(e.value)
