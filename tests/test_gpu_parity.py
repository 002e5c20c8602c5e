"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances: FP64 kernels 1e-12 (max-norm relative per field group) after tens
of steps -- the two sides evaluate the same formulas in a different order and
with different libm implementations, so they differ by rounding only.  FP32
kernels: 1e-5 on fields after 10 steps, 1e-3 on string length and <v^2> at
the end, windings compared plaquette by plaquette with mismatches allowed only
on plaquettes with a link whose phase argument lies within 1e-6 of pi.

These tests hold the 15-plane layout (one step per pass, Pi and E updated in
place) unless they say otherwise; the 20-plane layout, the library's default
through the binding, is covered by the two-step, full-size and ensemble tests.
"""
import functools
import math

import numpy as np
import pytest
import torch

from tests import inputs as I

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import (ambiguous_links, fields_np, group_errors, oracle_params,  # noqa: E402
                            plaquette_touches, upload)

P15 = functools.partial(AH.Params, layout=AH.AH_LAYOUT_15)
KERNELS = [AH.AH_KERNEL_PLAIN, AH.AH_KERNEL_TILED]
SHAPES = [(64, 12, 10), (128, 6, 5)]


def _ctx(p, planes, kernel=AH.AH_KERNEL_AUTO, tile_y=0, chunk_z=0):
    c = AH.Context([p], [planes])
    if kernel != AH.AH_KERNEL_AUTO:
        c.set_kernel(kernel, tile_y, chunk_z)
    return c


def _print_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_init_random_phase_matches_oracle(O, prec):
    _print_case(test="init", prec=prec)
    p = P15(32, 32, 32, precision=prec, seed=12345)
    t = AH.alloc_planes(p)
    with AH.Context([p], [t]) as c:
        got = fields_np(c)
    ref = O.init_random_phase(oracle_params(O, p))
    if prec == AH.AH_FP64:
        assert np.abs(got - ref).max() < 1e-15
    else:
        ref32 = ref.astype(np.float32).astype(np.float64)
        ulp = np.spacing(np.abs(ref32).astype(np.float32)).astype(np.float64)
        assert (np.abs(got - ref32) <= ulp).all()
        assert (got == ref32).mean() > 0.999


@pytest.mark.parametrize("kernel", KERNELS, ids=["plain", "tiled"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("era,s", [(0.0, 0.0), (1.0, 1.0), (2.0, 0.0), (1.0, 0.5)])
def test_step_fp64_random_state(O, kernel, shape, era, s):
    _print_case(test="step_fp64", kernel=kernel, shape=shape, era=era, s=s)
    nx, ny, nz = shape
    p = P15(nx, ny, nz, precision=AH.AH_FP64, tau0=1.0, tau_ref=2.0, era_p=era, s=s,
                  init=AH.AH_INIT_NONE)
    st = I.random_state(shape, seed=101)
    op = oracle_params(O, p)
    with _ctx(p, upload(p, st), kernel) as c:
        ref = st
        for n_done, k in ((1, 1), (10, 9)):
            c.step(k)
            ref, _ = O.run(op, ref, n_done - k, k)
            err = group_errors(fields_np(c), ref)
            assert max(err.values()) < 1e-12, (n_done, err)


@pytest.mark.parametrize("kernel", KERNELS, ids=["plain", "tiled"])
def test_step_fp32_random_state(O, kernel):
    """FP32 storage and arithmetic vs the FP64 oracle from the FP32-rounded input:
    1e-5 relative per field group after 10 steps."""
    shape = (64, 12, 10)
    _print_case(test="step_fp32", kernel=kernel, shape=shape)
    p = P15(*shape, precision=AH.AH_FP32, tau0=2.0, tau_ref=4.0, era_p=1.0, s=1.0,
                  init=AH.AH_INIT_NONE)
    st = I.random_state(shape, seed=202).astype(np.float32).astype(np.float64)
    with _ctx(p, upload(p, st), kernel) as c:
        c.step(10)
        got = fields_np(c)
    ref, _ = O.run(oracle_params(O, p), st, 0, 10)
    err = group_errors(got, ref)
    assert max(err.values()) < 1e-5, err


def _compare_obs(g, o, rel):
    assert g.step == o.step
    assert g.n_wind_dir == o.n_wind_dir and g.net_wind_dir == o.net_wind_dir
    assert g.n_pierced == o.n_pierced and g.nonfinite == o.nonfinite == 0
    for k in ("length", "sum_lag", "kin", "grad", "elec", "mag", "pot", "energy", "xi_w",
              "pres", "pres_lag", "rho_lag"):
        # abs: sums of roundoff-sized terms (e.g. the potential at |phi| = sigma) carry no digits
        assert getattr(g, k) == pytest.approx(getattr(o, k), rel=rel, abs=1e-20), k
    for k in ("num", "den"):
        # atol: sums of roundoff-sized terms (e.g. sum G V at |phi| = sigma) carry no digits
        assert np.allclose(getattr(g, k), getattr(o, k), rtol=rel, atol=1e-20), k
    for gv, ov in zip(g.v2, o.v2):
        assert (math.isnan(gv) and math.isnan(ov)) or gv == pytest.approx(ov, rel=rel, abs=1e-14)
    assert (math.isnan(g.v2_eos) and math.isnan(o.v2_eos)) or \
        g.v2_eos == pytest.approx(o.v2_eos, rel=rel, abs=1e-14)
    if math.isnan(o.xi_l):
        assert math.isnan(g.xi_l)
    else:
        assert g.xi_l == pytest.approx(o.xi_l, rel=rel)


def test_config_32cubed_fp64_run(O):
    """32^3, FP64, radiation, s = 1, random phase, 80 steps to tau = 8 with
    string length and <v^2> every 10 steps: every observable vs the oracle."""
    _print_case(test="c1_run")
    p = P15(32, 32, 32, precision=AH.AH_FP64, tau0=0.0, tau_ref=8.0, era_p=1.0, s=1.0,
                  seed=1)
    op = oracle_params(O, p)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        obs = c.step(80, measure_every=10)
        mx, _ = c.gauss_residual()
        got = fields_np(c)
    st, oobs = O.run(op, O.init_random_phase(op), 0, 80, measure_every=10)
    assert len(obs) == len(oobs) == 8
    for (g,), o in zip(obs, oobs):
        _compare_obs(g, o, 1e-9)
    assert mx[0] < 1e-12
    assert max(group_errors(got, st).values()) < 1e-10


@pytest.mark.parametrize("kernel", KERNELS, ids=["plain", "tiled"])
@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_measure_and_wind_map_match_oracle(O, prec, kernel):
    """Standalone measurement of a generic state, and the winding map plaquette
    by plaquette on identical input fields."""
    shape = (64, 10, 9)
    _print_case(test="measure", prec=prec, kernel=kernel)
    p = P15(*shape, precision=prec, tau0=3.0, tau_ref=4.0, era_p=2.0, s=0.0,
                  init=AH.AH_INIT_NONE, step0=7)
    st = I.random_state(shape, seed=303, amp_a=2.5)
    if prec == AH.AH_FP32:
        st = st.astype(np.float32).astype(np.float64)
    with _ctx(p, upload(p, st), kernel) as c:
        (g,), (w,) = c.measure(wind=True)
        w = w.cpu().numpy().astype(np.int64)
    o = O.measure(oracle_params(O, p), 7, st, wind_map=True)
    diff = w != o.wind
    allowed = plaquette_touches(ambiguous_links(st))
    assert not (diff & ~allowed).any()
    print("winding mismatches (all at ambiguous links):", int(diff.sum()))
    # the plain kernel forms every density in FP64; the tiled kernel in the
    # storage precision (FP32 rounding, ~1e-7 per term), accumulating in FP64
    rel = 1e-6 if (prec == AH.AH_FP32 and kernel == AH.AH_KERNEL_TILED) else 1e-10
    if not diff.any():
        _compare_obs(g, o, rel)
    else:
        assert g.energy == pytest.approx(o.energy, rel=rel)


def _plant_near_boundaries(st, prec, seed, frac=0.4, spread=3e-5):
    """Set the angle of a fraction of the links so that the winding argument
    theta^{x+i} - theta^x + A_i of Eq. (11) lies within +-spread of an odd
    multiple of pi (shifted by -2 pi, 0 or 2 pi), rounded to the storage
    precision; returns the number of links within 2.6e-5 of a boundary."""
    rng = np.random.default_rng(seed)
    th = np.arctan2(st[1], st[0])
    near = 0
    for i, axis in enumerate((2, 1, 0)):
        u0 = np.roll(th, -1, axis=axis) - th
        pick = rng.random(th.shape) < frac
        k = rng.integers(-1, 2, size=th.shape)
        a = np.pi - u0 + rng.uniform(-spread, spread, size=th.shape) + 2 * np.pi * k
        if prec == AH.AH_FP32:
            a = a.astype(np.float32).astype(np.float64)
        st[4 + i] = np.where(pick, a, st[4 + i])
        r = np.mod(u0 + st[4 + i] + np.pi, 2 * np.pi)
        near += int((np.minimum(r, 2 * np.pi - r) < 2.6e-5).sum())
    return near


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_winding_near_link_boundaries(O, prec):
    """Links planted around the branch points of [.]_pi (Eq. (11)), within and
    beyond the band where the measuring kernels decide wrap counts from FP64
    instead of FP32 phases: winding map (read-only measurement, tiled and
    plain kernels) and the counts of the fused step measurement equal the
    oracle's at every plaquette whose links are not within 1e-9 of a tie."""
    shape = (64, 10, 9)
    _print_case(test="wind_near_boundaries", prec=prec)
    p = P15(*shape, precision=prec, tau0=3.0, tau_ref=4.0, era_p=2.0, s=0.0,
                  init=AH.AH_INIT_NONE, step0=7)
    st = I.random_state(shape, seed=515, amp_a=2.5)
    if prec == AH.AH_FP32:
        st = st.astype(np.float32).astype(np.float64)
    near = _plant_near_boundaries(st, prec, seed=516)
    assert near > 1000   # the FP64 fallback is exercised at many sites
    o = O.measure(oracle_params(O, p), 7, st, wind_map=True)
    allowed = plaquette_touches(ambiguous_links(st, tol=1e-9))
    for kernel in (AH.AH_KERNEL_TILED, AH.AH_KERNEL_PLAIN):
        with _ctx(p, upload(p, st), kernel) as c:
            (g,), (w,) = c.measure(wind=True)
            w = w.cpu().numpy().astype(np.int64)
            (f,), = c.step(1, measure_every=1)
        diff = w != o.wind
        assert not (diff & ~allowed).any(), (kernel, int((diff & ~allowed).sum()))
        if not allowed.any():
            for obs in (g, f):
                assert obs.step == 7
                assert obs.n_wind_dir == o.n_wind_dir and obs.net_wind_dir == o.net_wind_dir
                assert obs.n_pierced == o.n_pierced


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_gauss_residual_matches_oracle(O, prec):
    shape = (64, 7, 6)
    _print_case(test="gauss", prec=prec)
    p = P15(*shape, precision=prec, tau0=2.0, tau_ref=3.0, era_p=1.0, s=0.5,
                  init=AH.AH_INIT_NONE, step0=4)
    st = I.random_state(shape, seed=404)
    if prec == AH.AH_FP32:
        st = st.astype(np.float32).astype(np.float64)
    with AH.Context([p], [upload(p, st)]) as c:
        mx, rms = c.gauss_residual()
    omx, orms = O.gauss(oracle_params(O, p), 4, st)
    assert mx[0] == pytest.approx(omx, rel=1e-12)
    assert rms[0] == pytest.approx(orms, rel=1e-12)


def test_nonfinite_is_reported():
    _print_case(test="nonfinite")
    p = P15(64, 8, 8, precision=AH.AH_FP32, init=AH.AH_INIT_VACUUM, tau0=1.0)
    t = AH.alloc_planes(p)
    with AH.Context([p], [t]) as c:
        t[8, 3, 4, 5] = float("nan")
        with pytest.raises(AH.AHError) as e:
            c.measure()
        assert e.value.code == AH.ah.AH_E_NONFINITE


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_vacuum_stays_bitwise(prec):
    _print_case(test="vacuum", prec=prec)
    p = P15(64, 8, 8, precision=prec, init=AH.AH_INIT_VACUUM, tau0=0.0, tau_ref=2.0)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        c.step(25)
        got = c.fields()
    ref = torch.zeros_like(got)
    ref[0] = 1.0
    assert torch.equal(got, ref)


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_checkpoint_resume_is_bitwise(prec):
    """Copy the state out at step 12, resume it in a fresh context with
    AH_INIT_NONE and step0 = 12: identical to the uninterrupted run."""
    _print_case(test="resume", prec=prec)
    p = P15(64, 16, 8, precision=prec, tau0=0.0, tau_ref=4.0, era_p=2.0, s=0.0, seed=9)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        c.step(12)
        mid = c.fields().clone()
        c.step(9)
        full = c.fields().clone()
    q = P15(**{**p.__dict__, "init": AH.AH_INIT_NONE, "step0": 12})
    t = AH.alloc_planes(q)
    t[:10] = mid
    with AH.Context([q], [t]) as c:
        c.step(9)
        assert c.current_step() == 21
        assert torch.equal(c.fields(), full)


def test_context_on_its_own_stream():
    """A context on a stream of its own (default priority) gives the same fields,
    observations and winding map as one on the current stream; fields() and
    measure() order their copies after the library's work on that stream."""
    _print_case(test="own_stream")
    p = P15(128, 12, 10, precision=AH.AH_FP32, tau0=0.0, tau_ref=4.0, era_p=1.0, s=1.0,
                  seed=19, layout=AH.AH_LAYOUT_20)
    side = torch.cuda.Stream()
    res = []
    for stream in (None, side):
        with AH.Context([p], [AH.alloc_planes(p)], stream=stream) as c:
            obs = c.step(11, measure_every=5)
            (m,), (w,) = c.measure(wind=True)
            f = c.fields()
            res.append((f.clone(), w.clone(), [o[0].n_wind for o in obs], m.n_wind, m.energy))
    torch.cuda.synchronize()
    (f0, w0, n0, m0, e0), (f1, w1, n1, m1, e1) = res
    assert torch.equal(f0, f1) and torch.equal(w0, w1)
    assert n0 == n1 and m0 == m1 and e1 == pytest.approx(e0, rel=1e-12)


def test_batch_equals_solo_and_n_end():
    """Realizations of different sizes and eras in one context advance exactly
    as they do alone; a realization stops at its n_end."""
    _print_case(test="batch")
    ps = [P15(64, 8, 8, precision=AH.AH_FP32, tau_ref=2.0, era_p=1.0, s=1.0, seed=1),
          P15(64, 16, 4, precision=AH.AH_FP32, tau_ref=3.0, era_p=2.0, s=0.0, seed=2,
                    n_end=7),
          P15(128, 4, 6, precision=AH.AH_FP32, tau_ref=1.0, era_p=1.0, s=0.0, seed=3)]
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.step(11)
        batch = [c.fields(r).clone() for r in range(3)]
        steps = [c.current_step(r) for r in range(3)]
    assert steps == [11, 7, 11]
    for r, p in enumerate(ps):
        with AH.Context([p], [AH.alloc_planes(p)]) as c:
            c.step(11)
            assert torch.equal(c.fields(), batch[r]), r


def test_fused_schedule_matches_separate_measure(O):
    """ah_step's measurements equal ah_measure on the same states."""
    _print_case(test="fused_schedule")
    p = P15(64, 8, 8, precision=AH.AH_FP64, tau_ref=2.0, seed=4)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        c.step(5)
        obs = c.step(10, measure_every=5)
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        c.step(5)
        (m5,) = c.measure()
        c.step(5)
        (m10,) = c.measure()
    assert [o[0].step for o in obs] == [5, 10]
    for (g,), m in zip(obs, (m5, m10)):
        assert g.n_wind == m.n_wind and g.energy == pytest.approx(m.energy, rel=1e-13)


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_tiling_invariance_is_bitwise(prec):
    """Race and halo detector: the tiled kernel under different tile heights
    and z-chunks (ragged in y and z, one chunk, one plane per chunk) gives
    bit-identical fields after several steps."""
    shape = (128, 20, 13)
    _print_case(test="tiling", prec=prec, shape=shape)
    tys = [2, 4, 8] + ([16] if prec == AH.AH_FP32 else [])
    configs = [(ty, cz) for ty in tys for cz in (0, 1, 5, 13)]
    p = P15(*shape, precision=prec, tau0=1.0, tau_ref=3.0, era_p=1.0, s=1.0,
                  init=AH.AH_INIT_NONE)
    st = I.random_state(shape, seed=505)
    ref = None
    for ty, cz in configs:
        with _ctx(p, upload(p, st), AH.AH_KERNEL_TILED, ty, cz) as c:
            c.step(7)
            got = c.fields().clone()
        if ref is None:
            ref = got
        else:
            assert torch.equal(got, ref), (ty, cz)


def test_fused_measurement_run_matches_oracle(O):
    """FP64, 64x24x20, radiation s=1 from the random-phase start: 40 steps with
    the diagnostics fused into the tiled step kernel every 10 steps."""
    _print_case(test="fused_run")
    p = P15(64, 24, 20, precision=AH.AH_FP64, tau0=0.0, tau_ref=5.0, era_p=1.0, s=1.0,
                  seed=11)
    op = oracle_params(O, p)
    with _ctx(p, AH.alloc_planes(p), AH.AH_KERNEL_TILED) as c:
        obs = c.step(40, measure_every=10)
        got = fields_np(c)
    st, oobs = O.run(op, O.init_random_phase(op), 0, 40, measure_every=10)
    assert [o[0].step for o in obs] == [0, 10, 20, 30]
    for (g,), o in zip(obs, oobs):
        _compare_obs(g, o, 1e-9)
    assert max(group_errors(got, st).values()) < 1e-11


@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32])
def test_fused_measurement_on_identical_input(O, prec):
    """The fused FP32/FP64 measurement of a state against the oracle's
    measurement of the same (widened) state."""
    shape = (128, 12, 10)
    _print_case(test="fused_identical", prec=prec)
    p = P15(*shape, precision=prec, tau0=1.0, tau_ref=3.0, era_p=2.0, s=0.0, seed=21)
    with _ctx(p, AH.alloc_planes(p), AH.AH_KERNEL_TILED) as c:
        c.step(10)
        st = fields_np(c)
        (g,), = c.step(1, measure_every=10)
    o = O.measure(oracle_params(O, p), 10, st, wind_map=True)
    rel = 1e-10 if prec == AH.AH_FP64 else 2e-5
    assert g.step == 10
    amb = plaquette_touches(ambiguous_links(st)).sum()
    assert abs(g.n_wind - o.n_wind) <= amb
    if amb == 0:
        assert g.n_wind_dir == o.n_wind_dir
    for k in ("kin", "grad", "elec", "mag", "pot", "energy", "sum_lag", "pres", "pres_lag",
              "rho_lag", "v2_eos"):
        assert getattr(g, k) == pytest.approx(getattr(o, k), rel=rel), k
    for k in ("num", "den", "v2"):
        assert np.allclose(getattr(g, k), getattr(o, k), rtol=rel * 10, atol=1e-20), k


def _ensemble(prec=AH.AH_FP32):
    """Uneven realizations, mixed eras and s, one stopping early (n_end)."""
    return [P15(64, 8, 8, precision=prec, tau_ref=2.0, era_p=1.0, s=1.0, seed=31),
            P15(128, 16, 12, precision=prec, tau_ref=3.0, era_p=2.0, s=0.0, seed=32),
            P15(64, 24, 20, precision=prec, tau_ref=2.5, era_p=1.0, s=0.0, seed=33, n_end=9),
            P15(192, 6, 5, precision=prec, tau_ref=1.5, era_p=2.0, s=0.0, seed=34)]


def _run_ensemble(ps, batched, graph_steps, nsteps=17, measure_every=5):
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.set_launch(batched, graph_steps)
        obs = c.step(nsteps, measure_every=measure_every)
        fields = [c.fields(r).clone() for r in range(len(ps))]
        steps = [c.current_step(r) for r in range(len(ps))]
    return fields, obs, steps


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
def test_batched_and_graph_launches_equal_per_realization(prec):
    """One persistent launch per step (and graph replay) gives bit-identical
    fields and the same observations as one launch per realization."""
    _print_case(test="batched", prec=prec)
    ps = _ensemble(prec)
    ref_f, ref_o, ref_s = _run_ensemble(ps, False, 0)
    assert ref_s == [17, 17, 9, 17]
    for batched, g in ((True, 0), (True, 3), (False, 4)):
        f, o, s = _run_ensemble(ps, batched, g)
        assert s == ref_s
        for r in range(len(ps)):
            assert torch.equal(f[r], ref_f[r]), (batched, g, r)
        assert len(o) == len(ref_o)
        for row, ref_row in zip(o, ref_o):
            for a, b in zip(row, ref_row):
                assert a.step == b.step and a.n_wind_dir == b.n_wind_dir
                if a.step >= 0:
                    assert a.energy == pytest.approx(b.energy, rel=1e-12)
                    assert a.sum_lag == pytest.approx(b.sum_lag, rel=1e-12)
    # the early-stopping realization reports no measurement after its n_end
    assert [row[2].step for row in ref_o] == [0, 5, -1, -1]


def test_graph_replay_repeats_with_eager_work_between():
    """The captured graph is replayed over several calls, with the program's
    own eager work and synchronisation between them; every replay matches the
    eager run."""
    _print_case(test="graph_replay")
    ps = _ensemble(AH.AH_FP32)[:2]
    eager = AH.Context(ps, [AH.alloc_planes(p) for p in ps])
    graph = AH.Context(ps, [AH.alloc_planes(p) for p in ps])
    graph.set_launch(True, 4)
    try:
        for k in range(4):
            eager.step(9)
            graph.step(9)
            scratch = torch.randn(1 << 20, device="cuda")
            _ = float(scratch.sum())                    # eager library work between replays
            graph.measure()
            torch.cuda.synchronize()
            for r in range(2):
                assert torch.equal(graph.fields(r), eager.fields(r)), (k, r)
    finally:
        eager.close()
        graph.close()


def test_autotune_keeps_fields_and_results():
    _print_case(test="autotune")
    ps = _ensemble(AH.AH_FP32)
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.step(3)
        before = [c.fields(r).clone() for r in range(len(ps))]
        ty, cz = c.autotune()
        assert ty in (4, 8, 16) and len(cz) == len(ps) and all(z >= 1 for z in cz)
        for r in range(len(ps)):
            assert torch.equal(c.fields(r), before[r])
        c.set_launch(True, 2)
        c.step(6)
        tuned = [c.fields(r).clone() for r in range(len(ps))]
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.step(9)
        for r in range(len(ps)):
            assert torch.equal(c.fields(r), tuned[r]), r


@pytest.mark.parametrize("kernel", KERNELS, ids=["plain", "tiled"])
def test_core_growth_switch_matches_oracle(O, kernel):
    """s = -1 (core growth) until tau_s, then s = 1 (Sec. 2 after Eq. (8)):
    fields and measurements across the switch against the oracle."""
    shape = (64, 12, 10)
    _print_case(test="core_growth", kernel=kernel)
    p = P15(*shape, precision=AH.AH_FP64, tau0=0.5, tau_ref=1.5, era_p=1.0, s=-1.0,
                  s_late=1.0, tau_s=1.5, seed=61)
    op = oracle_params(O, p)
    with _ctx(p, AH.alloc_planes(p), kernel) as c:
        obs = c.step(20, measure_every=5)
        got = fields_np(c)
        mx, _ = c.gauss_residual()
    ref, oobs = O.run(op, O.init_random_phase(op), 0, 20, measure_every=5)
    assert max(group_errors(got, ref).values()) < 1e-12
    for (g,), o in zip(obs, oobs):
        _compare_obs(g, o, 1e-9)
    assert mx[0] < 1e-12
