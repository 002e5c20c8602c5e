"""Full-size GPU checks, in the launch configuration bench.py times.

- 512^3 (the benchmark workload): one step of the library against the oracle
  evaluated site by site on sampled sites (tile edges in x and y, z-chunk
  edges, lattice boundaries, random interior sites), FP32 and FP64; and the
  two-steps-per-pass kernel against single steps, bit for bit.
- 1024 x 1024 x 128 (one GPU's share of 1024^3 over 8 GPUs, bench.py's slab
  form): the slab with halo planes closed on itself against the periodic
  lattice, bit for bit.
- 48 x 128^3 + 16 x 64^3 + 4 x 256^3 (bench.py's ensemble): autotuned tiles, one
  persistent launch per pair, 10-step graphs, diagnostics every 20 steps, against
  one launch per realization, bit for bit, past the 64^3 realizations' n_end.
- 256^3 radiation era, s = 1, to tau = 64 (640 steps, diagnostics every 10):
  fields after 10 steps against the oracle (FP64: 1e-12; FP32 from the
  FP32-rounded start: 1e-5 per field group), diagnostics at step 10 against
  the oracle, and string length, xi and <v^2> at the end for FP32 against
  FP64 (1e-3), with Gauss's law and the zero net winding held throughout.
"""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import (fields_np, group_errors, oracle_params)  # noqa: E402


def _edge_coords(n, period):
    """Coordinates next to every tile / chunk edge of the given period, plus the lattice ends."""
    c = {0, 1, n - 2, n - 1}
    for e in range(period, n, period):
        c.update({e - 1, e})
    return sorted(x for x in c if 0 <= x < n)


def _sample_sites(n, rng, k_random=4000):
    xs = _edge_coords(n, 64)                 # tile edges in x
    ys = _edge_coords(n, 4)[:32]             # tile edges in y (heights 4 and 8)
    zs = _edge_coords(n, 64)                 # z-chunk edges of the default chunking
    pts = [(x, y, z) for x in xs[::2] for y in ys[::2] for z in zs[::2]]
    pts += [tuple(v) for v in rng.integers(0, n, size=(k_random, 3))]
    return np.unique(np.array([x + n * (y + n * z) for x, y, z in pts], dtype=np.int64))


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
def test_512cubed_one_step_on_sampled_sites(O, prec):
    n = 512
    print(f"CASE test=512_sampled prec={prec}", flush=True)
    p = AH.Params(n, n, n, precision=prec, dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2,
                  era_p=2.0, s=0.0, seed=2024)
    planes = AH.alloc_planes(p)
    with AH.Context([p], [planes]) as c:
        c.step(30)
        torch.cuda.synchronize()
        idx = _sample_sites(n, np.random.default_rng(7))
        state = c.fields().double().cpu().numpy()          # S_30, widened to FP64
        c.step(1)
        got = c.fields().reshape(10, -1)[:, torch.from_numpy(idx).cuda()].double().cpu().numpy().T
    ref = O.step_sites(oracle_params(O, p), 30, state, idx)
    del state
    tol = 1e-12 if prec == AH.AH_FP64 else 1e-5
    for g, cols in (("phi", [0, 1]), ("pi", [2, 3]), ("a", [4, 5, 6]), ("e", [7, 8, 9])):
        scale = np.abs(ref[:, cols]).max()
        err = np.abs(got[:, cols] - ref[:, cols]).max() / scale
        print(f"  {g}: max rel err {err:.2e} over {idx.size} sites", flush=True)
        assert err < tol, g


@pytest.mark.parametrize("prec", [AH.AH_FP32, AH.AH_FP64])
def test_512cubed_two_step_pass_equals_single_steps(prec):
    """The two-steps-per-pass kernel at 512^3 in its default launch shape (20-plane
    layout): 31 steps with diagnostics every 20 from the random-phase start are
    bit-identical to single steps in the 15-plane layout, whose one-step result is
    checked against the oracle site by site above."""
    n = 512
    print(f"CASE test=512_two_step prec={prec}", flush=True)
    base = dict(precision=prec, dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2, era_p=2.0,
                s=0.0, seed=2024)
    runs = []
    for layout in (AH.AH_LAYOUT_15, AH.AH_LAYOUT_20):
        p = AH.Params(n, n, n, layout=layout, **base)
        planes = AH.alloc_planes(p)
        with AH.Context([p], [planes]) as c:
            obs = c.step(31, measure_every=20)
            runs.append((c.fields().clone(), [o[0] for o in obs]))
        del planes
        torch.cuda.empty_cache()
    (f15, o15), (f20, o20) = runs
    assert torch.equal(f15, f20)
    for a, b in zip(o15, o20):
        assert a.step == b.step and a.n_wind == b.n_wind
        assert a.energy == pytest.approx(b.energy, rel=1e-12)


def test_planes_above_4gib_two_step_pass():
    """Planes above 4 GiB (FP64, 1024 x 1024 x 520: 4.36 GB per plane) take the two-step
    kernel's 64-bit addressing: three steps (a pair and a single step) equal single steps
    in the 15-plane layout bit for bit."""
    print("CASE test=large_planes", flush=True)
    base = dict(precision=AH.AH_FP64, dx=0.5, dt=0.1, tau0=1.0, tau_ref=256.0, era_p=1.0,
                s=1.0, seed=77)
    runs = []
    for layout in (AH.AH_LAYOUT_15, AH.AH_LAYOUT_20):
        p = AH.Params(1024, 1024, 520, layout=layout, **base)
        planes = AH.alloc_planes(p)
        with AH.Context([p], [planes]) as c:
            c.step(3)
            runs.append(c.fields().clone())
        del planes
        torch.cuda.empty_cache()
    assert torch.equal(runs[0], runs[1])


def test_slab_1024x1024x128_equals_periodic():
    """One GPU's share of 1024^3 over 8 GPUs, as bench.py times it: a 1024 x 1024 x 128
    FP32 slab with two halo planes a side, refilled before every pass from its own faces,
    equals the periodic 1024 x 1024 x 128 lattice bit for bit through pairs, a fused
    measured step and a single step (the periodic kernels are pinned to the oracle above)."""
    print("CASE test=slab_1024", flush=True)
    nxy, nz, H = 1024, 128, 2
    base = dict(precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=1.0, tau_ref=256.0, era_p=1.0,
                s=1.0, layout=AH.AH_LAYOUT_20)
    pp = AH.Params(nxy, nxy, nz, seed=99, **base)
    ps = AH.Params(nxy, nxy, nz, init=AH.AH_INIT_NONE, z_halo=H, **base)
    tp, ts = AH.alloc_planes(pp), AH.alloc_planes(ps)
    with AH.Context([pp], [tp]) as ref:
        ts.zero_()
        ts[:10, H:H + nz] = ref.fields()
        with AH.Context([ps], [ts]) as slab:
            def refill():
                c0 = slab.current_planes(0)[0]
                cur = ts[c0:c0 + 10]
                cur[:, :H] = cur[:, nz:nz + H]
                cur[:, H + nz:] = cur[:, H:2 * H]
            refill()
            for k, meas in ((2, 0), (1, 1), (1, 0), (2, 0)):
                if meas:
                    (g,), = ref.step(k, measure_every=1)
                    (h,), = slab.step(k, measure_every=1)
                    assert h.n_wind_dir == g.n_wind_dir and h.n_pierced == g.n_pierced
                    assert h.energy == pytest.approx(g.energy, rel=1e-12)
                    assert h.v2[0] == pytest.approx(g.v2[0], rel=1e-10)
                else:
                    ref.step(k)
                    slab.step(k)
                refill()
            assert slab.current_step() == ref.current_step() == 6
            assert torch.equal(slab.fields()[:, H:H + nz], ref.fields())
    del tp, ts
    torch.cuda.empty_cache()


def _full_ensemble():
    """48 x 128^3 + 16 x 64^3 + 4 x 256^3 FP32 in the 20-plane layout; realization r:
    radiation s = 1 if r is even, matter s = 0 if odd, seed 1000 + r, each to its own
    tau_end = N dx / 2 (n_end = 320, 160, 640 steps)."""
    ps = []
    for n, count in ((256, 4), (128, 48), (64, 16)):
        for _ in range(count):
            r = len(ps)
            rad = r % 2 == 0
            tau_end = n * 0.5 / 2.0
            ps.append(AH.Params(n, n, n, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0,
                                tau_ref=tau_end, era_p=1.0 if rad else 2.0,
                                s=1.0 if rad else 0.0, seed=1000 + r,
                                n_end=int(round(tau_end / 0.1)), layout=AH.AH_LAYOUT_20))
    return ps


def test_full_ensemble_in_benchmark_launch_configuration():
    """The ensemble form as bench.py times it (autotuned tiles, one persistent launch
    per pair, 10-step graphs, diagnostics every 20 steps) equals one launch per
    realization bit for bit over 170 steps, past the n_end = 160 of the 64^3
    realizations (frozen since), with the same winding counts and energies."""
    print("CASE test=full_ensemble", flush=True)
    ps = _full_ensemble()
    nsteps = 170

    def run(tuned):
        planes = [AH.alloc_planes(p) for p in ps]
        c = AH.Context(ps, planes)
        try:
            if tuned:
                c.set_launch(True, 10)
                c.autotune()
            else:
                c.set_launch(False, 0)
            obs = c.step(nsteps, measure_every=20)
            steps = [c.current_step(r) for r in range(len(ps))]
            return c, planes, obs, steps
        except BaseException:
            c.close()
            raise

    ref, ref_planes, ref_obs, ref_steps = run(False)
    try:
        got, got_planes, got_obs, got_steps = run(True)
        try:
            assert ref_steps == got_steps == [min(nsteps, p.n_end) for p in ps]
            for r in range(len(ps)):
                assert torch.equal(got.fields(r), ref.fields(r)), r
            assert len(got_obs) == len(ref_obs) == nsteps // 20 + 1
            for row, ref_row in zip(got_obs, ref_obs):
                for r, (a, b) in enumerate(zip(row, ref_row)):
                    assert a.step == b.step, r
                    if b.step >= 0:
                        assert a.n_wind_dir == b.n_wind_dir and a.net_wind_dir == b.net_wind_dir
                        assert a.energy == pytest.approx(b.energy, rel=1e-12), r
                        assert a.sum_lag == pytest.approx(b.sum_lag, rel=1e-12), r
            # the 64^3 realizations measure up to step 140 and not at 160 (their n_end)
            small = [r for r, p in enumerate(ps) if p.nx == 64]
            assert [got_obs[j][small[0]].step for j in range(len(got_obs))] == \
                [0, 20, 40, 60, 80, 100, 120, 140, -1]
        finally:
            got.close()
            del got_planes
    finally:
        ref.close()
        del ref_planes
        torch.cuda.empty_cache()


def test_config_256cubed_radiation_run(O):
    n, steps, every = 256, 640, 10
    print("CASE test=config_256", flush=True)
    base = dict(dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2, era_p=1.0, s=1.0, seed=1)
    res = {}
    for prec in (AH.AH_FP64, AH.AH_FP32):
        p = AH.Params(n, n, n, precision=prec, **base)
        with AH.Context([p], [AH.alloc_planes(p)]) as c:
            c.step(10)
            f10 = fields_np(c)
            obs = c.step(steps - 10, measure_every=every)
            (last,) = c.measure()                   # S_640, tau = 64
            mx, _ = c.gauss_residual()
        res[prec] = (p, f10, [o[0] for o in obs] + [last], mx[0])
    op = oracle_params(O, res[AH.AH_FP64][0])
    init = O.init_random_phase(op)
    ref10, oobs = O.run(op, init, 0, 10, measure_every=10)
    e64 = group_errors(res[AH.AH_FP64][1], ref10)
    init32 = init.astype(np.float32).astype(np.float64)
    ref10_32, _ = O.run(op, init32, 0, 10)
    e32 = group_errors(res[AH.AH_FP32][1], ref10_32)
    print("  step-10 field errors FP64:", e64, " FP32:", e32, flush=True)
    assert max(e64.values()) < 1e-12
    assert max(e32.values()) < 1e-5

    o64, o32 = res[AH.AH_FP64][2], res[AH.AH_FP32][2]
    assert [o.step for o in o64] == list(range(10, steps, every)) + [steps]
    # diagnostics of S_10 (first measurement of the call) against the oracle
    ref_m = O.measure(op, 10, ref10)
    g = o64[0]
    assert g.n_wind == ref_m.n_wind
    for k in ("energy", "sum_lag"):
        assert getattr(g, k) == pytest.approx(getattr(ref_m, k), rel=1e-9), k
    assert np.allclose(g.v2, ref_m.v2, rtol=1e-9)
    # properties held at every measurement
    for o in o64 + o32:
        assert o.net_wind_dir == [0, 0, 0] and o.nonfinite == 0
    assert res[AH.AH_FP64][3] < 1e-12
    # end time: FP32 against FP64
    a, b = o32[-1], o64[-1]
    print(f"  end step {b.step}: n_wind fp64 {b.n_wind} fp32 {a.n_wind}; "
          f"v2_L {b.v2[0]:.6f} {a.v2[0]:.6f}; v2_V {b.v2[1]:.6f} {a.v2[1]:.6f}; "
          f"xi_L {b.xi_l:.5f} {a.xi_l:.5f}", flush=True)
    curve = [(x.step, abs(x.length - y.length) / y.length, abs(x.v2[0] - y.v2[0]) / abs(y.v2[0]))
             for x, y in zip(o32, o64)]
    print("  FP32-FP64 relative divergence (step, length, v2_L):",
          [(s_, f"{l:.1e}", f"{v:.1e}") for s_, l, v in curve[::8]], flush=True)
    assert a.length == pytest.approx(b.length, rel=1e-3)
    assert a.xi_w == pytest.approx(b.xi_w, rel=1e-3)
    for k in range(3):
        assert a.v2[k] == pytest.approx(b.v2[k], rel=1e-3), k
    assert a.v2_eos == pytest.approx(b.v2_eos, rel=1e-3)
    assert not math.isnan(b.xi_l) and a.xi_l == pytest.approx(b.xi_l, rel=1e-3)
