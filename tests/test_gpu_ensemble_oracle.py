"""The batched ensemble form against the FP64 oracle, realization by realization.

Four realizations of uneven size (ragged tiles in y and z), radiation and
matter eras, s = 1, 0 and 1/2, one of them stopping early at an odd n_end
(the ensembles of independent realizations motivated in Sec. 1 and Sec. 5 of
arXiv:1809.00995): one persistent launch per pass (pairs of steps through the
two-step kernel in the 20-plane layout), unmeasured runs of steps replayed from
hipGraphs, tiles from the autotuner, diagnostics every 5 steps.  After 17 steps
every realization's fields must match the oracle's (FP64 1e-12, FP32 from the
FP32-rounded start 1e-5 per field group), every measured state's diagnostics the
oracle's measurement of the same step, and the frozen realization must report
its later slots as unmeasured (step = -1).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import (ambiguous_links, group_errors, oracle_params,  # noqa: E402
                            plaquette_touches)

NSTEPS, EVERY, GRAPH = 17, 5, 4


def _ensemble(prec, layout):
    kw = dict(precision=prec, layout=layout, tau0=0.0)
    return [AH.Params(64, 8, 8, tau_ref=2.0, era_p=1.0, s=1.0, seed=41, **kw),
            AH.Params(128, 16, 12, tau_ref=3.0, era_p=2.0, s=0.0, seed=42, **kw),
            AH.Params(64, 24, 20, tau_ref=2.5, era_p=1.0, s=0.5, seed=43, n_end=13, **kw),
            AH.Params(192, 6, 5, tau_ref=1.5, era_p=2.0, s=1.0, seed=44, **kw)]


def _oracle_run(O, p, fp32_start):
    """The oracle from the seeded start (rounded to FP32 if asked) to
    min(NSTEPS, n_end), measuring every EVERY steps; also the measured states."""
    op = oracle_params(O, p)
    st = O.init_random_phase(op)
    if fp32_start:
        st = st.astype(np.float32).astype(np.float64)
    last = min(NSTEPS, p.n_end) if p.n_end else NSTEPS
    meas = {}
    for n in range(last):
        if n % EVERY == 0:
            meas[n] = (O.measure(op, n, st), st)
        st = O.step(op, n, st)
    return st, meas


def _compare(g, o, state, fp64):
    if fp64:
        assert g.n_wind_dir == o.n_wind_dir and g.net_wind_dir == o.net_wind_dir
        assert g.n_pierced == o.n_pierced
        rel = 1e-9
    else:
        # FP32 fields differ from the oracle's by ~1e-6: a plaquette may only
        # change its winding where a link argument lies that close to +-pi
        amb = int(plaquette_touches(ambiguous_links(state, tol=1e-4)).sum())
        assert abs(g.n_wind - o.n_wind) <= amb and g.net_wind_dir == [0, 0, 0]
        rel = 1e-4
    assert g.nonfinite == o.nonfinite == 0
    for k in ("sum_lag", "kin", "grad", "elec", "mag", "pot", "energy", "pres", "pres_lag",
              "rho_lag"):
        assert getattr(g, k) == pytest.approx(getattr(o, k), rel=rel, abs=1e-20), k
    for k in ("num", "den"):
        assert np.allclose(getattr(g, k), getattr(o, k), rtol=rel, atol=1e-20), k
    for gv, ov in list(zip(g.v2, o.v2)) + [(g.v2_eos, o.v2_eos), (g.xi_l, o.xi_l)]:
        assert (math.isnan(gv) and math.isnan(ov)) or gv == pytest.approx(ov, rel=rel, abs=1e-12)


@pytest.mark.parametrize("layout", [AH.AH_LAYOUT_20, AH.AH_LAYOUT_15], ids=["pairs", "single"])
@pytest.mark.parametrize("prec", [AH.AH_FP64, AH.AH_FP32], ids=["fp64", "fp32"])
def test_batched_ensemble_matches_oracle(O, prec, layout):
    print(f"CASE test=ensemble_oracle prec={prec} layout={layout}", flush=True)
    ps = _ensemble(prec, layout)
    fp64 = prec == AH.AH_FP64
    with AH.Context(ps, [AH.alloc_planes(p) for p in ps]) as c:
        c.set_launch(True, GRAPH)
        ty, cz = c.autotune()
        print(f"  autotuned tile_y {ty}, chunks {cz}", flush=True)
        obs = c.step(NSTEPS, measure_every=EVERY)
        got = [c.fields(r).double().cpu().numpy() for r in range(len(ps))]
        steps = [c.current_step(r) for r in range(len(ps))]
    assert steps == [NSTEPS, NSTEPS, 13, NSTEPS]
    assert [row[0].step for row in obs] == [0, 5, 10, 15]
    for r, p in enumerate(ps):
        ref, meas = _oracle_run(O, p, fp32_start=not fp64)
        err = group_errors(got[r], ref)
        print(f"  realization {r} {p.nx}x{p.ny}x{p.nz}: field errors {err}", flush=True)
        assert max(err.values()) < (1e-12 if fp64 else 1e-5), (r, err)
        for row in obs:
            g = row[r]
            if g.step < 0:
                # frozen at n_end: not measured
                assert p.n_end and g.step == -1 and row[0].step >= p.n_end
                continue
            o, state = meas[g.step]
            _compare(g, o, state, fp64)
        measured = [row[r].step for row in obs if row[r].step >= 0]
        assert measured == sorted(meas)
