"""GPU parity of z-slabs (one GPU's share of a z-decomposed lattice).

A slab whose halo planes are filled, before every pass, from its own opposite
faces is a periodic lattice: the fields of its slab planes must equal a
periodic run of the same state bit for bit, through single steps, two-step
passes and fused measurements, and its observables and winding map must equal
the periodic ones.  The periodic runs are pinned to the oracle elsewhere.
"""
import numpy as np
import pytest
import torch

from tests import inputs as I

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import fields_np, upload  # noqa: E402

L15, L20 = AH.AH_LAYOUT_15, AH.AH_LAYOUT_20


def _print_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _params(shape, prec, layout, z_halo=0, **kw):
    base = dict(precision=prec, tau0=1.0, tau_ref=3.0, era_p=1.0, s=1.0, init=AH.AH_INIT_NONE)
    base.update(kw)
    return AH.Params(*shape, layout=layout, z_halo=z_halo, **base)


def _close_halo(c, p):
    """Fill the halo planes of the current copy from the slab's own opposite faces."""
    t, H, nz = c.planes[0], p.z_halo, p.nz
    for f in c.current_planes(0):
        t[f, :H] = t[f, nz:nz + H]
        t[f, H + nz:] = t[f, H:2 * H]


def _slab_ctx(p, st, kernel, tile_y=0):
    t = AH.alloc_planes(p)
    t.zero_()
    H = p.z_halo
    t[:10, H:H + p.nz] = torch.from_numpy(st).to(dtype=p.dtype, device=t.device)
    c = AH.Context([p], [t])
    c.set_kernel(kernel, tile_y, 0)
    _close_halo(c, p)
    return c


def _slab_fields(c, p):
    H = p.z_halo
    return c.fields()[:, H:H + p.nz]


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
@pytest.mark.parametrize("layout,z_halo,kernel", [(L15, 1, AH.AH_KERNEL_TILED),
                                                  (L15, 2, AH.AH_KERNEL_TILED),
                                                  (L20, 2, AH.AH_KERNEL_TILED2)],
                         ids=["l15h1", "l15h2", "l20h2_pairs"])
def test_closed_slab_equals_periodic_lattice(prec, layout, z_halo, kernel):
    """Passes of 1 and 2 steps (pairs where the kernel takes them), with a fused
    measurement in between, on a slab closed on itself: bitwise the periodic run."""
    shape = (128, 12, 16)
    _print_case(test="closed_slab", prec=prec, layout=layout, z_halo=z_halo)
    st = I.random_state(shape, seed=919, amp_a=1.5)
    ref_p = _params(shape, prec, layout)
    slab_p = _params(shape, prec, layout, z_halo)
    ref = AH.Context([ref_p], [upload(ref_p, st)])
    ref.set_kernel(kernel)
    slab = _slab_ctx(slab_p, st, kernel)
    two = kernel == AH.AH_KERNEL_TILED2
    with ref, slab:
        # pass sizes: pairs when available, a measured step, odd steps
        plan = [(2 if two else 1, 0), (1, 1), (1, 0), (2 if two else 1, 0), (1, 1)]
        for k, meas in plan:
            if meas:
                (g,), = ref.step(k, measure_every=1)
                (h,), = slab.step(k, measure_every=1)
                assert h.step == g.step
                assert h.n_wind_dir == g.n_wind_dir and h.net_wind_dir == g.net_wind_dir
                assert h.n_pierced == g.n_pierced
                for name in ("energy", "sum_lag", "kin", "grad", "elec", "mag", "pot", "pres",
                             "xi_w"):
                    assert getattr(h, name) == pytest.approx(getattr(g, name), rel=1e-12), name
            else:
                ref.step(k)
                slab.step(k)
            _close_halo(slab, slab_p)
            assert slab.current_step() == ref.current_step()
            assert torch.equal(_slab_fields(slab, slab_p), ref.fields()), (k, meas)
        # standalone measurement and winding map of the slab planes
        (g,), (wg,) = ref.measure(wind=True)
        (h,), (wh,) = slab.measure(wind=True)
        assert torch.equal(wh[:, z_halo:z_halo + shape[2]], wg)
        assert h.n_wind == g.n_wind and h.energy == pytest.approx(g.energy, rel=1e-12)


def test_slab_halo_planes_are_read_not_written():
    """The kernels never write a halo plane, and a slab's result depends on its halo
    (an open slab, halo zero, differs from the closed one next to the faces only)."""
    shape = (64, 8, 12)
    _print_case(test="slab_halo_untouched")
    p = _params(shape, AH.AH_FP32, L20, 2)
    st = I.random_state(shape, seed=920)
    with _slab_ctx(p, st, AH.AH_KERNEL_TILED2) as c:
        t = c.planes[0]
        t[:, :2] = 7.0
        t[:, 2 + shape[2]:] = -7.0
        c.step(2)
        assert bool((t[:, :2] == 7.0).all()) and bool((t[:, 2 + shape[2]:] == -7.0).all())
    with _slab_ctx(p, st, AH.AH_KERNEL_TILED2) as a, _slab_ctx(p, st, AH.AH_KERNEL_TILED2) as b:
        b.planes[0][:, :2] = 0
        b.planes[0][:, 2 + shape[2]:] = 0
        a.step(2)
        b.step(2)
        fa, fb = _slab_fields(a, p), _slab_fields(b, p)
        # two steps reach two planes in from each face; the middle is unaffected
        assert torch.equal(fa[:, 2:-2], fb[:, 2:-2])
        assert not torch.equal(fa[:, :2], fb[:, :2])


def test_slab_call_rules():
    """One pass per call; no pairs with one halo plane; the unsupported entry points
    refuse slabs."""
    shape = (64, 8, 8)
    _print_case(test="slab_rules")
    p2 = _params(shape, AH.AH_FP32, L20, 2)
    st = I.random_state(shape, seed=921)
    with _slab_ctx(p2, st, AH.AH_KERNEL_TILED2) as c:
        with pytest.raises(AH.AHError):
            c.step(3)                       # a pair and a single step: two passes
        with pytest.raises(AH.AHError):
            c.step(2, measure_every=1)      # measured state: single-step pass first
        with pytest.raises(AH.AHError):
            c.gauss_residual()
        with pytest.raises(AH.AHError):
            c.set_launch(1, 0)
        with pytest.raises(AH.AHError):
            c.set_kernel(AH.AH_KERNEL_PLAIN)
        with pytest.raises(AH.AHError):
            c.autotune()
        assert c.current_step() == 0        # nothing ran
        c.step(2)
        assert c.current_step() == 2
    p1 = _params(shape, AH.AH_FP32, L20, 1)
    with _slab_ctx(p1, st, AH.AH_KERNEL_TILED2) as c:
        with pytest.raises(AH.AHError):
            c.step(2)                       # one halo plane: no pairs
        c.step(1)
        assert c.current_step() == 1
