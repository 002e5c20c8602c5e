"""Full-size GPU checks, in the launch configuration bench.py times.

- 512^3 (the benchmark workload): one step of the library against the oracle
  evaluated site by site on sampled sites (tile edges in x and y, z-chunk
  edges, lattice boundaries, random interior sites), FP32 and FP64; the
  two-steps-per-pass kernel against single steps, bit for bit; and the whole
  1280-step run (s = 0 and s = 1) against Gauss's law and zero net winding.
- 1024^3 FP32, radiation era, s = 1 (the largest configuration) in its
  production launch shape: the read-only pass's windings, one pair and one
  single step against the oracle on sampled sites, each evaluated on a small
  periodic lattice holding the site's neighbourhood.
- 1024 x 1024 x 128 (one GPU's share of 1024^3 over 8 GPUs, bench.py's slab
  form): the slab with halo planes closed on itself against the periodic
  lattice, bit for bit.
- 48 x 128^3 + 16 x 64^3 + 4 x 256^3 (bench.py's ensemble): autotuned tiles, one
  persistent launch per pair, 10-step graphs, diagnostics every 20 steps, against
  one launch per realization, bit for bit, past the 64^3 realizations' n_end.
- 256^3 radiation era, s = 1, to tau = 64 (640 steps, diagnostics every 10) in
  the production path: fields after 10 steps against the oracle (FP64: 1e-12;
  FP32 from the FP32-rounded start: 1e-5 per field group), and the whole
  observation series, end state and winding map (FP64) or the end-time string
  length, xi and <v^2> (FP32, 1e-3) against the oracle's stored run of the
  same workload, with Gauss's law and the zero net winding held throughout.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import (ambiguous_links, fields_np, group_errors,  # noqa: E402
                            neighbourhoods, oracle_params, plaquette_touches, site_values,
                            small_params)


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


@pytest.mark.parametrize("s", [0.0, 1.0])
def test_512cubed_full_run_keeps_gauss_law_and_zero_net_winding(s):
    """The benchmark's workload at its full length: 512^3 FP32, matter era, from the
    random-phase start to tau_end = 128 (1280 steps) with diagnostics every 20 steps, in
    the production path (pairs, the read-only measuring pass), for both values of s.
    Properties that hold at any size: every measurement finite with zero net winding in
    each orientation (strings present at the start), and Gauss's law (Sec. 4) kept to the
    FP32 rounding of the updates: each step rounds the E and Pi updates about ten times
    at unit roundoff 6e-8 on terms of order one, so after 1280 steps the residual is below
    10 x 6e-8 x 1280 = 7.7e-4 even if every rounding adds up (checked at 1e-3)."""
    n, steps, every = 512, 1280, 20
    print(f"CASE test=512_full_run s={s}", flush=True)
    p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2,
                  era_p=2.0, s=s, seed=2024)
    planes = AH.alloc_planes(p)
    with AH.Context([p], [planes]) as c:
        obs = [o[0] for o in c.step(steps, measure_every=every)]
        gmax, grms = c.gauss_residual()
    del planes
    torch.cuda.empty_cache()
    assert [o.step for o in obs] == list(range(0, steps, every))
    assert obs[0].n_wind > 0
    for o in obs:
        assert o.nonfinite == 0 and o.net_wind_dir == [0, 0, 0], o.step
        assert math.isfinite(o.energy) and math.isfinite(o.length), o.step
    print(f"  end: n_wind {obs[-1].n_wind}, xi_w {obs[-1].xi_w:.3f}; Gauss residual max "
          f"{gmax[0]:.2e}, rms {grms[0]:.2e}", flush=True)
    assert gmax[0] < 1e-3


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


def test_planes_above_4gib_two_step_pass(O):
    """Planes above 4 GiB (FP64, 1024 x 1024 x 520: 4.36 GB per plane) take the two-step
    kernel's 64-bit addressing: three steps (a pair and a single step) equal single steps
    in the 15-plane layout bit for bit, and one more pair matches the oracle (1e-12 per
    field group) on sampled sites, among them sites past the 4 GiB offset (z >= 512),
    each evaluated on its neighbourhood.  The read-only measuring pass also addresses
    them in 64 bits: its windings equal those of the plain measuring kernel plaquette
    by plaquette, and its sums agree to FP64 rounding."""
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
            if layout == AH.AH_LAYOUT_20:
                (ot,), (wt,) = c.measure(wind=True)
                c.set_kernel(AH.AH_KERNEL_PLAIN)
                (op,), (wp,) = c.measure(wind=True)
                assert torch.equal(wt, wp)
                assert ot.n_wind == op.n_wind and ot.n_wind > 0
                assert ot.length == op.length
                # the parts of the energy, against the total
                for k in ("energy", "kin", "grad", "elec", "mag", "pot"):
                    assert abs(getattr(ot, k) - getattr(op, k)) <= 1e-12 * op.energy, k
                assert list(ot.v2) == pytest.approx(list(op.v2), abs=1e-9)
                del wt, wp
                c.set_kernel(AH.AH_KERNEL_AUTO)
                rng = np.random.default_rng(13)
                xyz = np.concatenate([rng.integers(0, 1024, size=(60, 2)),
                                      rng.integers(0, 520, size=(60, 1))], axis=1)
                edge = [[0, 0, 511], [1023, 1023, 512], [64, 5, 519], [63, 1023, 0],
                        [512, 512, 513], [1, 2, 518]]
                xyz = np.unique(np.concatenate([xyz, edge]), axis=0)
                nb = neighbourhoods(c.fields(), xyz, 2)
                n0 = c.current_step(0)
                c.step(2)
                got = site_values(c.fields(), xyz)
                sp6, mid6 = small_params(O, p, 6), 2 + 6 * (2 + 6 * 2)
                ref = np.stack([O.step_sites(sp6, n0 + 1, O.step(sp6, n0, nb[k]), [mid6])[0]
                                for k in range(len(xyz))])
                _check_groups(got, ref, 1e-12, "pair past 4 GiB")
        del planes
        torch.cuda.empty_cache()
    assert torch.equal(runs[0], runs[1])


def _sample_xyz(n, rng, periods_xy, periods_z, k_random):
    xs = _edge_coords(n, 64)
    ys = sorted({c for per in periods_xy for c in _edge_coords(n, per)})
    zs = sorted({c for per in periods_z for c in _edge_coords(n, per)})
    pts = [(int(rng.choice(xs)), int(rng.choice(ys)), int(rng.choice(zs))) for _ in range(k_random)]
    pts += [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(k_random)]
    return np.unique(np.array(pts, dtype=np.int64), axis=0)


def _check_groups(got, ref, tol, what):
    for g, cols in (("phi", [0, 1]), ("pi", [2, 3]), ("a", [4, 5, 6]), ("e", [7, 8, 9])):
        scale = np.abs(ref[:, cols]).max()
        err = np.abs(got[:, cols] - ref[:, cols]).max() / scale
        print(f"  {what} {g}: max rel err {err:.2e} over {len(got)} sites", flush=True)
        assert err < tol, (what, g)


def test_1024cubed_fp32_production_path(O):
    """The largest configuration, 1024^3 FP32 in the radiation era with s = 1 (85.9 GB in
    the 20-plane layout), in the launch shape the library takes for it: pairs of steps in
    z-chunks of at most 192 planes, the read-only measuring pass on 4 GiB planes (32-bit
    offsets), odd steps by the single-step kernel.  From the random-phase start, 64 steps
    with diagnostics every 64 steps; then, on sampled sites next to every tile and chunk
    edge and at random, each against the oracle evaluated on the site's neighbourhood:
    - the windings of the read-only pass at S_64 (plaquettes with a link within 1e-6 of
      the branch cut aside), whose whole map also equals the plain measuring kernel's
      and nets to zero in every orientation, and whose sums agree with that kernel's
      FP64 densities to 1e-6 of the energy (<v^2> to 1e-5);
    - one pair (S_64 -> S_66) and one single step (S_66 -> S_67), to 1e-5 per field
      group (FP32 arithmetic from FP32 states against FP64)."""
    n = 1024
    print("CASE test=1024_fp32", flush=True)
    p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0, tau_ref=256.0,
                  era_p=1.0, s=1.0, seed=1025)
    planes = AH.alloc_planes(p)
    rng = np.random.default_rng(11)
    with AH.Context([p], [planes]) as c:
        obs = c.step(64, measure_every=64)
        assert len(obs) == 1 and obs[0][0].step == 0
        # the read-only pass at S_64 against the plain kernel and the oracle
        (ot,), (wt,) = c.measure(wind=True)
        c.set_kernel(AH.AH_KERNEL_PLAIN)
        (op,), (wp,) = c.measure(wind=True)
        c.set_kernel(AH.AH_KERNEL_AUTO)
        assert torch.equal(wt, wp)
        assert ot.n_wind == op.n_wind and ot.n_wind > 0
        assert list(ot.net_wind_dir) == [0, 0, 0]
        # the sums: FP32 densities (read-only pass) against FP64 ones (plain kernel) on
        # the same state, 1e-6 of the total energy
        for k in ("energy", "kin", "grad", "elec", "mag", "pot", "sum_lag"):
            assert abs(getattr(ot, k) - getattr(op, k)) <= 1e-6 * op.energy, k
        assert list(ot.v2) == pytest.approx(list(op.v2), abs=1e-5)
        assert ot.v2_eos == pytest.approx(op.v2_eos, abs=1e-5)
        F = c.fields()
        xyz_w = _sample_xyz(n, rng, (4, 8, 9), (128, 171, 192, 205, 512), 300)
        nb = neighbourhoods(F, xyz_w, 1)
        t = torch.as_tensor(xyz_w, device=wt.device)
        w_gpu = wt[:, t[:, 2], t[:, 1], t[:, 0]].T.cpu().numpy()
        del wt, wp
        sp4 = small_params(O, p, 4)
        checked = 0
        for k in range(len(xyz_w)):
            ref = O.measure(sp4, 64, nb[k], wind_map=True).wind[:, 1, 1, 1]
            amb = plaquette_touches(ambiguous_links(nb[k]))[:, 1, 1, 1]
            ok = ~amb
            assert np.array_equal(w_gpu[k][ok], ref[ok]), (xyz_w[k], w_gpu[k], ref)
            checked += int(ok.sum())
        print(f"  windings: {checked} sampled plaquettes equal the oracle's", flush=True)
        # one pair, S_64 -> S_66
        xyz_2 = _sample_xyz(n, rng, (9,), (128, 171, 192, 205), 250)
        nb2 = neighbourhoods(F, xyz_2, 2)
        del F
        c.step(2)
        F = c.fields()
        got2 = site_values(F, xyz_2)
        sp6 = small_params(O, p, 6)
        mid = 2 + 6 * (2 + 6 * 2)
        ref2 = np.stack([O.step_sites(sp6, 65, O.step(sp6, 64, nb2[k]), [mid])[0]
                         for k in range(len(xyz_2))])
        _check_groups(got2, ref2, 1e-5, "pair")
        # one single step, S_66 -> S_67
        xyz_1 = _sample_xyz(n, rng, (8,), (512, 128), 250)
        nb1 = neighbourhoods(F, xyz_1, 1)
        del F
        c.step(1)
        F = c.fields()
        got1 = site_values(F, xyz_1)
        del F
        mid = 1 + 4 * (1 + 4 * 1)
        ref1 = np.stack([O.step_sites(sp4, 66, nb1[k], [mid])[0] for k in range(len(xyz_1))])
        _check_groups(got1, ref1, 1e-5, "single step")
    del planes
    torch.cuda.empty_cache()


def test_slab_1024x1024x128_equals_periodic(O):
    """One GPU's share of 1024^3 over 8 GPUs, as bench.py times it: a 1024 x 1024 x 128
    FP32 slab with two halo planes a side, refilled before every pass from its own faces,
    equals the periodic 1024 x 1024 x 128 lattice bit for bit through pairs, a fused
    measured step and a single step; one more pair of the slab (8-row tiles, the halo
    read through the refilled planes) matches the oracle on sampled sites, among them
    sites next to the slab's faces (1e-5 per field group)."""
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
            rng = np.random.default_rng(17)
            xyz = np.concatenate([rng.integers(0, nxy, size=(60, 2)),
                                  rng.integers(0, nz, size=(60, 1))], axis=1)
            edge = [[0, 0, 0], [nxy - 1, nxy - 1, nz - 1], [64, 8, 0], [63, 7, nz - 1],
                    [500, nxy - 8, 1], [700, 16, nz - 2]]
            xyz = np.unique(np.concatenate([xyz, edge]), axis=0)
            nb = neighbourhoods(ref.fields(), xyz, 2)
            n0 = slab.current_step()
            slab.step(2)
            got = site_values(slab.fields()[:, H:H + nz], xyz)
            sp6, mid6 = small_params(O, pp, 6), 2 + 6 * (2 + 6 * 2)
            want = np.stack([O.step_sites(sp6, n0 + 1, O.step(sp6, n0, nb[k]), [mid6])[0]
                             for k in range(len(xyz))])
            _check_groups(got, want, 1e-5, "slab pair")
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


def test_full_ensemble_in_benchmark_launch_configuration(O):
    """The ensemble form as bench.py times it (autotuned tiles, one persistent launch
    per pair, 10-step graphs, diagnostics every 20 steps) equals one launch per
    realization bit for bit over 170 steps, past the n_end = 160 of the 64^3
    realizations (frozen since), with the same winding counts and energies.  One more
    batched pair then matches the oracle on sampled sites of a 128^3 matter-era and a
    256^3 radiation-era realization (each site's neighbourhood on a 6^3 lattice, FP32
    against FP64 from the same state: 1e-5 per field group)."""
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
            # one more batched pair against the oracle, on sampled sites (tile and
            # lattice edges, random sites) of one active realization of each size
            picks = [next(r for r, p in enumerate(ps) if p.nx == 128 and p.era_p == 2.0),
                     next(r for r, p in enumerate(ps) if p.nx == 256 and p.era_p == 1.0)]
            rng = np.random.default_rng(5)
            cut = {}
            for r in picks:
                m = ps[r].nx
                xyz = np.concatenate([rng.integers(0, m, size=(80, 3)),
                                      [[0, 0, 0], [m - 1, m - 1, m - 1], [63, 64, m // 2],
                                       [64, 7, 63], [m - 1, 8, 64]]])
                xyz = np.unique(xyz, axis=0)
                cut[r] = (xyz, neighbourhoods(got.fields(r), xyz, 2), got.current_step(r))
            got.step(2)
            mid6 = 2 + 6 * (2 + 6 * 2)
            for r in picks:
                xyz, nb, n0 = cut[r]
                sp6 = small_params(O, ps[r], 6)
                ref2 = np.stack([O.step_sites(sp6, n0 + 1, O.step(sp6, n0, nb[k]), [mid6])[0]
                                 for k in range(len(xyz))])
                _check_groups(site_values(got.fields(r), xyz), ref2, 1e-5,
                              f"ensemble {ps[r].nx}^3")
        finally:
            got.close()
            del got_planes
    finally:
        ref.close()
        del ref_planes
        torch.cuda.empty_cache()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else abs(a - b)


def test_config_256cubed_radiation_run(O):
    """256^3 radiation era, s = 1, to tau = 64 in the production path (20-plane
    layout: pairs, FP32 read-only measuring passes, FP64 fused measuring steps),
    diagnostics every 10 steps, against the oracle's run of the same workload
    (tests/golden/make_config2_golden.py): the fields after 10 steps (FP64 1e-12;
    FP32 from the FP32-rounded start 1e-5 per field group); for FP64 every
    observation of the series, the end state on 256 sampled sites and the winding
    map plaquette by plaquette (mismatches only where a link argument lies within
    1e-6 of pi); for FP32 string length, xi_W, xi_L, <v^2>_X and <v^2>_w at the
    end within 1e-3 of the oracle's run from the FP32-rounded start, with the
    divergence along the run printed; Gauss's law and zero net winding held."""
    n, steps, every = 256, 640, 10
    print("CASE test=config_256", flush=True)
    with open(os.path.join(GOLDEN, "config2_256cubed_radiation_s1.json")) as f:
        gold = json.load(f)
    wz = np.load(os.path.join(GOLDEN, "config2_256cubed_radiation_s1_wind640.npz"))
    base = dict(dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2, era_p=1.0, s=1.0, seed=1,
                layout=AH.AH_LAYOUT_20)
    res = {}
    for prec in (AH.AH_FP64, AH.AH_FP32):
        p = AH.Params(n, n, n, precision=prec, **base)
        with AH.Context([p], [AH.alloc_planes(p)]) as c:
            c.step(10)
            f10 = fields_np(c)
            obs = c.step(steps - 10, measure_every=every)
            (last,), (wmap,) = c.measure(wind=True)          # S_640, tau = 64
            mx, _ = c.gauss_residual()
            end = c.fields().reshape(10, -1)
            idx = torch.tensor(gold["runs"]["fp64"]["end"]["sample_sites"], device=end.device)
            sample = end[:, idx].double().cpu().numpy().T
            wmap = wmap.cpu().numpy()
            state = end.view(10, n, n, n).double().cpu().numpy() if prec == AH.AH_FP64 else None
        res[prec] = (p, f10, [o[0] for o in obs] + [last], mx[0], sample, wmap, state)
        torch.cuda.empty_cache()

    # fields after 10 steps against the oracle run here
    op = oracle_params(O, res[AH.AH_FP64][0])
    init = O.init_random_phase(op)
    ref10, _ = O.run(op, init, 0, 10)
    ref10_32, _ = O.run(op, init.astype(np.float32).astype(np.float64), 0, 10)
    e64 = group_errors(res[AH.AH_FP64][1], ref10)
    e32 = group_errors(res[AH.AH_FP32][1], ref10_32)
    print("  step-10 field errors FP64:", e64, " FP32:", e32, flush=True)
    assert max(e64.values()) < 1e-12
    assert max(e32.values()) < 1e-5

    # FP64: the whole series against the oracle's
    g64 = {o["step"]: o for o in gold["runs"]["fp64"]["series"]}
    o64 = res[AH.AH_FP64][2]
    assert [o.step for o in o64] == list(range(10, steps + 1, every))
    worst = {}
    for o in o64:
        r = g64[o.step]
        assert o.net_wind_dir == [0, 0, 0] and o.nonfinite == 0
        assert abs(o.n_wind - r["n_wind"]) <= 2, (o.step, o.n_wind, r["n_wind"])
        for k in ("length", "energy", "sum_lag"):
            worst[k] = max(worst.get(k, 0.0), _rel(getattr(o, k), r[k]))
        # the parts of the energy relative to the whole: the oracle forms
        # 1 - cos(Xi) directly, which carries only ~1e-16 / Xi^2 relative digits
        # while the plaquettes are small (early times)
        for k in ("kin", "grad", "elec", "mag", "pot"):
            worst[k] = max(worst.get(k, 0.0), abs(getattr(o, k) - r[k]) / r["energy"])
        for k in range(3):
            worst[f"v2_{k}"] = max(worst.get(f"v2_{k}", 0.0), _rel(o.v2[k], r["v2"][k]))
    print("  FP64 series, worst relative deviation from the oracle:",
          {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
    for k, v in worst.items():
        assert v < 1e-8, k
    # FP64 end state on sampled sites, Gauss's law, and the winding map
    ref_s = np.array(gold["runs"]["fp64"]["end"]["sample_fields"])
    es = group_errors(res[AH.AH_FP64][4].T, ref_s.T)
    print("  FP64 end fields on 256 sampled sites:", es, flush=True)
    assert max(es.values()) < 1e-9
    assert res[AH.AH_FP64][3] < 1e-12 and gold["runs"]["fp64"]["end"]["gauss_max"] < 1e-12
    ref_w = np.zeros((3, n * n * n), dtype=np.int8)
    ref_w[wz["orientation"].astype(np.int64), wz["site"].astype(np.int64)] = wz["w"]
    diff = res[AH.AH_FP64][5].reshape(3, -1) != ref_w
    allowed = plaquette_touches(ambiguous_links(res[AH.AH_FP64][6])).reshape(3, -1)
    print(f"  FP64 end winding map: {int(np.count_nonzero(ref_w))} pierced plaquettes, "
          f"{int(diff.sum())} differ (all must touch a link within 1e-6 of pi)", flush=True)
    assert not (diff & ~allowed).any()

    # FP32 against the oracle from the FP32-rounded start
    g32 = {o["step"]: o for o in gold["runs"]["fp32_start"]["series"]}
    o32 = res[AH.AH_FP32][2]
    curve = [(o.step, _rel(o.length, g32[o.step]["length"]),
              _rel(o.v2[0], g32[o.step]["v2"][0])) for o in o32]
    print("  FP32 vs oracle relative divergence (step, length, v2_L):",
          [(s_, f"{l:.1e}", f"{v:.1e}") for s_, l, v in curve[::8] + curve[-1:]], flush=True)
    for o in o32:
        assert o.net_wind_dir == [0, 0, 0] and o.nonfinite == 0
    a, b = o32[-1], g32[steps]
    print(f"  end: n_wind oracle {b['n_wind']} fp32 {a.n_wind}; v2 {b['v2']} {a.v2}; "
          f"xi_L {b['xi_l']:.5f} {a.xi_l:.5f}", flush=True)
    for k in ("length", "xi_w", "v2_eos"):
        assert _rel(getattr(a, k), b[k]) < 1e-3, k
    for k in range(3):
        assert _rel(a.v2[k], b["v2"][k]) < 1e-3, k
    assert not math.isnan(b["xi_l"]) and _rel(a.xi_l, b["xi_l"]) < 1e-3
    print(f"  Gauss residual at the end: FP64 {res[AH.AH_FP64][3]:.1e}, "
          f"FP32 {res[AH.AH_FP32][3]:.1e}", flush=True)
