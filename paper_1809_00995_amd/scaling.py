"""Scaling validation of string networks (Sec. 4 and Table 3 of arXiv:1809.00995).

Evolves seeded random-phase lattices to half a light-crossing time with the
HIP library (FP32 fields, FP64 diagnostics, unmeasured steps two per pass)
and reports, per case, the slopes
dxi/dtau of the Lagrangian and winding string separations and the mean of
the velocity estimators over the late, scaling part of the run, averaged
over seeds with their standard error.  Cases follow Table 3: radiation era
with s = 1 and s = 0, matter era with s = 0, radiation with a core-growth
period (s = -1) before the true equations of motion (s = 1), and either era
with fixed comoving width (s = 0) before them.

    python -m paper_1809_00995_amd.scaling --n 512 --seeds 5 --out scaling.json
    python -m paper_1809_00995_amd.scaling --cases radiation_s0,matter_s0 --window2 0.75
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch

from . import ah as AH

# name: (era p, s, core growth).  Without core growth a(tau_end) = 1 and the runs start
# at tau = 0.  With core growth s = -1 until tau_cg = tau_end / 2 and s afterwards, with
# a(tau_cg) = 1 so that the couplings e0 a^(s-1), lambda0 a^(2(s-1)) are continuous there;
# the comoving core width (e0 sigma)^-1 a^(-s) then grows as a until tau_cg and shrinks
# as 1/a after it.  The run starts at tau0 = tau_end / 4, where the width is half its
# peak, so that it stays within [dx, 2 dx] for dx = 0.5 in radiation (p = 1).  With
# "fixed" s = 0 until tau_s = tau_end / 2 and s afterwards, from tau = 0.
CASES = {"radiation_s1": (1.0, 1.0, False), "radiation_s0": (1.0, 0.0, False),
         "matter_s0": (2.0, 0.0, False), "radiation_s1_core_growth": (1.0, 1.0, True),
         "radiation_s0_then_s1": (1.0, 1.0, "fixed"), "matter_s0_then_s1": (2.0, 1.0, "fixed")}
DEFAULT_CASES = ("radiation_s0", "matter_s0", "radiation_s1_core_growth")


def evolve(n: int, era: float, s: float, seed: int, measure_every: int = 10, dx: float = 0.5,
           dt: float = 0.1, core_growth=False):
    """One run to tau_end = n dx / 2; returns the observation series."""
    tau_end = n * dx / 2.0
    if core_growth == "fixed":
        # fixed comoving width (s = 0) until tau_s = tau_end / 2, then the true
        # equations of motion (s = 1), with a(tau_s) = 1: the width is 1/(e0 sigma)
        # until tau_s and shrinks as 1/a after it, to 2^-p/(e0 sigma) at tau_end
        p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=dx, dt=dt, tau0=0.0,
                      tau_ref=tau_end / 2, era_p=era, s=0.0, s_late=s, tau_s=tau_end / 2,
                      seed=seed, layout=AH.AH_LAYOUT_20)
        tau0 = 0.0
    elif core_growth:
        tau0 = round(0.25 * tau_end / dt) * dt
        p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=dx, dt=dt, tau0=tau0,
                      tau_ref=tau_end / 2, era_p=era, s=-1.0, s_late=s, tau_s=tau_end / 2,
                      seed=seed, layout=AH.AH_LAYOUT_20)
    else:
        tau0 = 0.0
        p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=dx, dt=dt, tau0=0.0, tau_ref=tau_end,
                      era_p=era, s=s, seed=seed, layout=AH.AH_LAYOUT_20)
    steps = int(round((tau_end - tau0) / dt))
    with AH.Context([p], [AH.alloc_planes(p)]) as c:
        obs = [o[0] for o in c.step(steps, measure_every=measure_every)]
        obs += c.measure()
    torch.cuda.empty_cache()
    return obs


def series(obs, n: int, dx: float = 0.5):
    """Observation series of one run: tau, l / V_box, xi_L, xi_W, <v^2>_{L,V,rho,omega}."""
    vbox = float(n) ** 3 * dx ** 3
    return {"tau": [o.tau for o in obs], "l_over_v": [o.length / vbox for o in obs],
            "xi_l": [o.xi_l for o in obs], "xi_w": [o.xi_w for o in obs],
            "v2_l": [o.v2[0] for o in obs], "v2_v": [o.v2[1] for o in obs],
            "v2_rho": [o.v2[2] for o in obs], "v2_w": [o.v2_eos for o in obs]}


def fit(obs, frac_start: float = 0.5):
    """Slopes of xi_L and xi_W against tau, and mean velocity estimators, over
    tau >= frac_start * tau_end."""
    tau_end = obs[-1].tau
    late = [o for o in obs if o.tau >= frac_start * tau_end]
    tau = np.array([o.tau for o in late])
    out = {}
    for key in ("xi_l", "xi_w"):
        xi = np.array([getattr(o, key) for o in late])
        ok = np.isfinite(xi)
        out["dxi_" + key[3:]] = float(np.polyfit(tau[ok], xi[ok], 1)[0]) if ok.sum() > 2 else math.nan
    out["v2_V"] = float(np.mean([o.v2[1] for o in late]))
    out["v2_L"] = float(np.mean([o.v2[0] for o in late]))
    out["v2_rho"] = float(np.mean([o.v2[2] for o in late]))
    out["v2_w"] = float(np.mean([o.v2_eos for o in late]))
    # the spread of the Lagrangian-weighted estimator between measurements
    out["v2_L_sd"] = float(np.std([o.v2[0] for o in late]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seeds", type=int, default=5)
    ap.add_argument("--first-seed", type=int, default=100, help="seeds first-seed, first-seed + 1, ...")
    ap.add_argument("--cases", default=",".join(DEFAULT_CASES))
    ap.add_argument("--measure-every", type=int, default=10)
    ap.add_argument("--window", type=float, default=0.5,
                    help="fit and average over tau >= window * tau_end")
    ap.add_argument("--window2", type=float, default=0.0,
                    help="also report the fit over tau >= window2 * tau_end")
    ap.add_argument("--out", default=None)
    ap.add_argument("--series", action="store_true", help="also store each run's observation series")
    args = ap.parse_args(argv)
    result = {"n": args.n, "seeds": args.seeds, "first_seed": args.first_seed, "cases": {}}
    for name in args.cases.split(","):
        era, s, cg = CASES[name]
        runs = []
        for k in range(args.seeds):
            seed = args.first_seed + k
            obs = evolve(args.n, era, s, seed=seed, measure_every=args.measure_every,
                         core_growth=cg)
            runs.append(fit(obs, args.window))
            if args.window2:
                runs[-1].update({f"{k}@{args.window2:g}": v
                                 for k, v in fit(obs, args.window2).items()})
            if args.series:
                runs[-1]["series"] = series(obs, args.n)
            runs[-1]["seed"] = seed
            print(f"{name} seed {seed}: " + ", ".join(f"{a}={b:.4f}" for a, b in runs[-1].items()
                                                      if a not in ("series", "seed")), flush=True)
        summary = {}
        for key in (k for k in runs[0] if k not in ("series", "seed")):
            vals = np.array([r[key] for r in runs])
            summary[key] = {"mean": float(np.mean(vals)),
                            "stderr": float(np.std(vals, ddof=1) / math.sqrt(len(vals)))
                            if len(vals) > 1 else math.nan}
        result["cases"][name] = {"runs": runs, "summary": summary}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(result, f, indent=1)
    print(json.dumps({k: {q: round(v["mean"], 4) for q, v in c["summary"].items()}
                      for k, c in result["cases"].items()}), flush=True)
    return result


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
