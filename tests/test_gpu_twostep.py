"""GPU parity of the 20-plane layout and of the two-steps-per-pass kernel.

The two-step kernel forms every site update with the same arithmetic (same
rounding) as the single-step tiled kernel, so its runs agree bit for bit with
runs of single steps, in either layout; the single-step kernels are pinned to
the FP64 oracle elsewhere, and the oracle bars here are the single-step ones
(1e-12 FP64, 1e-5 FP32, max-norm relative per field group).
"""
import numpy as np
import pytest
import torch

from tests import inputs as I

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import fields_np, group_errors, oracle_params, upload  # noqa: E402

L15, L20 = AH.AH_LAYOUT_15, AH.AH_LAYOUT_20
# ragged in y and z, a tile taller than the lattice, the smallest lattice, odd sizes
SHAPES = [(64, 12, 10), (128, 6, 5), (64, 4, 4), (192, 9, 37)]


def _print_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _params(shape, prec, layout, **kw):
    base = dict(precision=prec, tau0=1.0, tau_ref=3.0, era_p=1.0, s=1.0, init=AH.AH_INIT_NONE)
    base.update(kw)
    return AH.Params(*shape, layout=layout, **base)


def _ctx(p, planes, kernel=AH.AH_KERNEL_AUTO, tile_y=0, chunk_z=0):
    c = AH.Context([p], [planes])
    if kernel != AH.AH_KERNEL_AUTO:
        c.set_kernel(kernel, tile_y, chunk_z)
    return c


@pytest.mark.parametrize("kernel", [AH.AH_KERNEL_PLAIN, AH.AH_KERNEL_TILED], ids=["plain", "tiled"])
def test_layout20_single_steps_match_oracle(O, kernel):
    """Single-step kernels in the 20-plane layout (Pi, E written to the other
    copy) against the oracle, FP64, 9 steps."""
    shape = (64, 12, 10)
    _print_case(test="layout20_single", kernel=kernel)
    p = _params(shape, AH.AH_FP64, L20, era_p=2.0, s=0.0)
    st = I.random_state(shape, seed=707)
    with _ctx(p, upload(p, st), kernel) as c:
        c.step(9)
        got = fields_np(c)
        assert c.current_planes() == ([10 + f for f in range(10)])
    ref, _ = O.run(oracle_params(O, p), st, 0, 9)
    assert max(group_errors(got, ref).values()) < 1e-12


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
@pytest.mark.parametrize("shape", SHAPES)
def test_two_step_bitwise_equals_single_steps(prec, shape):
    """Runs of 1, 4 and 7 steps (pairs and an odd step left over) through the
    two-step kernel equal single-step tiled runs in the 15-plane layout bit for
    bit, for every tile height and a few z-chunks (one plane, ragged, whole)."""
    st = I.random_state(shape, seed=808)
    tys = [4, 5] if prec == AH.AH_FP64 else [4, 8, 9]
    ref_p = _params(shape, prec, L15)
    with _ctx(ref_p, upload(ref_p, st), AH.AH_KERNEL_TILED) as c:
        refs = []
        for k in (1, 4, 7):
            c.step(k)
            refs.append((c.current_step(), c.fields().clone()))
    for ty in tys:
        for cz in (0, 1, 3, shape[2]):
            _print_case(test="two_step_bitwise", prec=prec, shape=shape, ty=ty, cz=cz)
            p = _params(shape, prec, L20)
            with _ctx(p, upload(p, st), AH.AH_KERNEL_TILED2, ty, cz) as c:
                for k, (n_ref, f_ref) in zip((1, 4, 7), refs):
                    c.step(k)
                    assert c.current_step() == n_ref
                    assert torch.equal(c.fields(), f_ref), (ty, cz, n_ref)


@pytest.mark.parametrize("era,s", [(0.0, 0.0), (1.0, 1.0), (2.0, 0.0), (1.0, 0.5)])
def test_two_step_matches_oracle_fp64(O, era, s):
    shape = (64, 12, 10)
    _print_case(test="two_step_oracle", era=era, s=s)
    p = _params(shape, AH.AH_FP64, L20, era_p=era, s=s)
    st = I.random_state(shape, seed=909)
    with _ctx(p, upload(p, st), AH.AH_KERNEL_TILED2) as c:
        c.step(10)
        got = fields_np(c)
    ref, _ = O.run(oracle_params(O, p), st, 0, 10)
    assert max(group_errors(got, ref).values()) < 1e-12


def test_two_step_matches_oracle_fp32(O):
    """FP32 storage and arithmetic vs the FP64 oracle from the FP32-rounded
    input: 1e-5 after 10 steps, as for the single-step kernels."""
    shape = (128, 6, 5)
    _print_case(test="two_step_fp32")
    p = _params(shape, AH.AH_FP32, L20)
    st = I.random_state(shape, seed=910).astype(np.float32).astype(np.float64)
    with _ctx(p, upload(p, st), AH.AH_KERNEL_TILED2) as c:
        c.step(10)
        got = fields_np(c)
    ref, _ = O.run(oracle_params(O, p), st, 0, 10)
    assert max(group_errors(got, ref).values()) < 1e-5


def test_two_step_core_growth_switch(O):
    """A pair of steps straddling the end of core growth (s = -1 -> 1 at
    tau_s) uses each step's own couplings."""
    shape = (64, 12, 10)
    _print_case(test="two_step_core_growth")
    p = AH.Params(*shape, precision=AH.AH_FP64, tau0=0.5, tau_ref=1.5, era_p=1.0, s=-1.0,
                  s_late=1.0, tau_s=1.55, seed=61, layout=L20)
    op = oracle_params(O, p)
    with _ctx(p, AH.alloc_planes(p), AH.AH_KERNEL_TILED2) as c:
        obs = c.step(20, measure_every=5)
        got = fields_np(c)
        mx, _ = c.gauss_residual()
    ref, oobs = O.run(op, O.init_random_phase(op), 0, 20, measure_every=5)
    assert max(group_errors(got, ref).values()) < 1e-12
    assert [o[0].step for o in obs] == [o.step for o in oobs]
    for (g,), o in zip(obs, oobs):
        assert g.n_wind == o.n_wind
        assert g.energy == pytest.approx(o.energy, rel=1e-9)
    assert mx[0] < 1e-12


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
def test_two_step_measurements_graphs_and_n_end(prec):
    """Measured steps, odd leftovers, graph replay of pairs and a realization
    that stops at an odd n_end: fields bit-identical and the same observations
    as single steps in the 15-plane layout."""
    _print_case(test="two_step_schedule", prec=prec)
    ps = [AH.Params(64, 8, 8, precision=prec, tau_ref=2.0, era_p=1.0, s=1.0, seed=41),
          AH.Params(128, 16, 12, precision=prec, tau_ref=3.0, era_p=2.0, s=0.0, seed=42,
                    n_end=13),
          AH.Params(64, 24, 20, precision=prec, tau_ref=2.5, era_p=1.0, s=0.0, seed=43)]

    def run(layout, kernel, graph_steps):
        qs = [AH.Params(**{**p.__dict__, "layout": layout}) for p in ps]
        with AH.Context(qs, [AH.alloc_planes(q) for q in qs]) as c:
            c.set_kernel(kernel)
            c.set_launch(False, graph_steps)
            obs = c.step(23, measure_every=6)
            obs += [c.measure()]
            return [c.fields(r).clone() for r in range(3)], obs, \
                [c.current_step(r) for r in range(3)], c.gauss_residual()

    ref_f, ref_o, ref_s, ref_g = run(L15, AH.AH_KERNEL_TILED, 0)
    assert ref_s == [23, 13, 23]
    for g in (0, 5, 4):
        f, o, s, gs = run(L20, AH.AH_KERNEL_TILED2, g)
        assert s == ref_s
        for r in range(3):
            assert torch.equal(f[r], ref_f[r]), (g, r)
        assert len(o) == len(ref_o)
        for row, ref_row in zip(o, ref_o):
            for a, b in zip(row, ref_row):
                assert a.step == b.step and a.n_wind_dir == b.n_wind_dir
                if a.step >= 0:
                    assert a.energy == pytest.approx(b.energy, rel=1e-12)
                    assert a.v2 == pytest.approx(b.v2, rel=1e-12, nan_ok=True)
        assert gs[0] == pytest.approx(ref_g[0], rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
@pytest.mark.parametrize("batched", [False, True], ids=["solo", "batched"])
def test_two_step_autotune_keeps_results(prec, batched):
    """The autotuner (for one launch per realization, or for the batched form, where it
    times a tall scratch lattice) leaves the fields alone and installs tiles that give
    the same fields bit for bit as untuned single steps."""
    _print_case(test="two_step_autotune", prec=prec, batched=batched)
    ps = [AH.Params(128, 16, 40, precision=prec, tau_ref=2.0, era_p=1.0, s=1.0, seed=51,
                    layout=L20)]
    if batched:
        ps.append(AH.Params(64, 24, 20, precision=prec, tau_ref=2.5, era_p=2.0, s=0.0, seed=52,
                            layout=L20))
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.set_launch(batched, 0)
        c.step(3)
        before = [c.fields(r).clone() for r in range(len(ps))]
        ty, cz = c.autotune()
        assert ty in ((4, 5) if prec == AH.AH_FP64 else (4, 8, 9))
        assert len(cz) == len(ps) and all(z >= 1 for z in cz)
        for r in range(len(ps)):
            assert torch.equal(c.fields(r), before[r])
        c.step(8)
        tuned = [c.fields(r).clone() for r in range(len(ps))]
    qs = [AH.Params(**{**p.__dict__, "layout": L15}) for p in ps]
    with AH.Context(qs, [AH.alloc_planes(q) for q in qs]) as c:
        c.step(11)
        for r in range(len(ps)):
            assert torch.equal(c.fields(r), tuned[r]), r


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
def test_two_step_batched_ensemble(prec):
    """The ensemble form with two-step passes: one persistent launch per pair
    (eager and replayed from graphs) over realizations of uneven size, one
    stopping at an odd n_end, equals single steps launched per realization."""
    _print_case(test="two_step_batched", prec=prec)
    ps = [AH.Params(64, 8, 8, precision=prec, tau_ref=2.0, era_p=1.0, s=1.0, seed=71),
          AH.Params(128, 16, 12, precision=prec, tau_ref=3.0, era_p=2.0, s=0.0, seed=72),
          AH.Params(64, 24, 20, precision=prec, tau_ref=2.5, era_p=1.0, s=0.0, seed=73, n_end=9),
          AH.Params(192, 6, 5, precision=prec, tau_ref=1.5, era_p=2.0, s=0.0, seed=74)]

    def run(layout, kernel, batched, graph_steps):
        qs = [AH.Params(**{**p.__dict__, "layout": layout}) for p in ps]
        with AH.Context(qs, [AH.alloc_planes(q) for q in qs]) as c:
            c.set_kernel(kernel)
            c.set_launch(batched, graph_steps)
            obs = c.step(17, measure_every=5)
            return ([c.fields(r).clone() for r in range(len(qs))], obs,
                    [c.current_step(r) for r in range(len(qs))])

    ref_f, ref_o, ref_s = run(L15, AH.AH_KERNEL_TILED, False, 0)
    assert ref_s == [17, 17, 9, 17]
    for g in (0, 3, 4):
        f, o, s = run(L20, AH.AH_KERNEL_TILED2, True, g)
        assert s == ref_s
        for r in range(len(ps)):
            assert torch.equal(f[r], ref_f[r]), (g, r)
        assert len(o) == len(ref_o)
        for row, ref_row in zip(o, ref_o):
            for a, b in zip(row, ref_row):
                assert a.step == b.step and a.n_wind_dir == b.n_wind_dir
                if a.step >= 0:
                    assert a.energy == pytest.approx(b.energy, rel=1e-12)


@pytest.mark.parametrize("layout", [L15, L20])
def test_degenerate_calls(layout):
    """Zero steps change nothing and measure nothing; a cadence longer than the call
    measures only the states it meets (here the first); a frozen realization (n_end
    reached) stays bitwise unchanged under further steps; ah_measure on a fresh
    context sees the initial state."""
    _print_case(test="degenerate", layout=layout)
    p = AH.Params(64, 8, 6, precision=AH.AH_FP32, tau_ref=2.0, era_p=1.0, s=1.0, seed=81,
                  layout=layout, n_end=5)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        (m0,) = c.measure()
        f0 = c.fields().clone()
        assert c.step(0) == [] and c.current_step() == 0
        assert c.step(0, measure_every=3) == []
        assert torch.equal(c.fields(), f0)
        obs = c.step(3, measure_every=100)
        assert [o[0].step for o in obs] == [0]
        assert obs[0][0].n_wind == m0.n_wind and obs[0][0].energy == pytest.approx(m0.energy, rel=1e-12)
        c.step(10)
        assert c.current_step() == 5
        f5 = c.fields().clone()
        obs = c.step(4, measure_every=1)
        assert all(o[0].step == -1 for o in obs)   # frozen: slots left unmeasured
        assert torch.equal(c.fields(), f5)
