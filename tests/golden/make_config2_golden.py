"""Write the oracle's reference for the 256^3 radiation-era run to tau = 64.

Calls only the FP64 CPU oracle (``oracle/``).  The workload: a 256^3 periodic
lattice, dx = 0.5, dt = 0.1, lambda0 = 2, e0 = 1, sigma = 1, radiation era
(a = tau / 64), s = 1, the seeded random-phase start of Sec. 2 (seed 1), 640
leapfrog steps (Eqs. (4)-(7)) with the diagnostics of Eqs. (9)-(12) every 10
steps.  Two runs:

- ``fp64``: from the FP64 start;
- ``fp32_start``: from the same start rounded to FP32 (the state an FP32 field
  store begins from), so that an FP32 run can be compared with exact
  arithmetic on identical input.

For each run the file keeps the observation series (steps 0, 10, ..., 640),
the Gauss-law residual and 256 seeded sample sites of the end state; for the
``fp64`` run also every pierced plaquette of the end state (orientation, site,
W) in a compressed numpy file.  On 8 threads the two runs take about 45
minutes.

    python tests/golden/make_config2_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

N, STEPS, EVERY, SEED = 256, 640, 10, 1
OUT_JSON = os.path.join(HERE, "config2_256cubed_radiation_s1.json")
OUT_WIND = os.path.join(HERE, "config2_256cubed_radiation_s1_wind640.npz")
OBS_KEYS = ("step", "tau", "a", "n_wind", "n_wind_dir", "net_wind_dir", "n_pierced", "length",
            "xi_w", "sum_lag", "xi_l", "num", "den", "v2", "kin", "grad", "elec", "mag", "pot",
            "energy", "pres", "pres_lag", "rho_lag", "v2_eos", "nonfinite")


def params() -> O.Params:
    return O.Params(N, N, N, dx=0.5, dt=0.1, tau0=0.0, tau_ref=N * 0.5 / 2, era_p=1.0, s=1.0,
                    lambda0=2.0, e0=1.0, sigma=1.0, seed=SEED)


def sample_sites() -> np.ndarray:
    return np.sort(np.random.default_rng(2019).choice(N**3, size=256, replace=False))


def run(p: O.Params, st: np.ndarray, label: str, keep_wind: bool):
    series = []
    t0 = time.time()
    for n in range(STEPS + 1):
        if n % EVERY == 0:
            last = n == STEPS
            m = O.measure(p, n, st, wind_map=last and keep_wind)
            series.append({k: getattr(m, k) for k in OBS_KEYS})
            print(f"{label}: step {n} n_wind {m.n_wind} v2_L {m.v2[0]:.6f} "
                  f"({time.time() - t0:.0f} s)", flush=True)
        if n < STEPS:
            st = O.step(p, n, st)
    gmax, grms = O.gauss(p, STEPS, st)
    idx = sample_sites()
    flat = st.reshape(10, -1)
    end = {"gauss_max": gmax, "gauss_rms": grms, "sample_sites": idx.tolist(),
           "sample_fields": flat[:, idx].T.tolist()}
    return series, end, (m.wind if keep_wind else None)


def main() -> None:
    p = params()
    init = O.init_random_phase(p)
    out = {"workload": "256^3 periodic lattice, radiation era a = tau/64, s = 1, lambda0 = 2, "
                       "e0 = 1, sigma = 1, dx = 0.5, dt = 0.1, random-phase start seed 1, "
                       "640 steps to tau = 64, diagnostics every 10 steps",
           "made_by": "python tests/golden/make_config2_golden.py (FP64 CPU oracle, "
                      f"{O.threads()} threads)",
           "runs": {}}
    for label, start, wind in (("fp64", init, True),
                               ("fp32_start", init.astype(np.float32).astype(np.float64), False)):
        series, end, wmap = run(p, start, label, wind)
        out["runs"][label] = {"series": series, "end": end}
        if wmap is not None:
            k, z, y, x = np.nonzero(wmap)
            np.savez_compressed(OUT_WIND, orientation=k.astype(np.int8),
                                site=(x + N * (y + N * z)).astype(np.int32),
                                w=wmap[k, z, y, x].astype(np.int8))
    with open(OUT_JSON, "w") as f:
        json.dump(out, f, indent=0, separators=(",", ":"))
        f.write("\n")
    print("wrote", OUT_JSON, OUT_WIND, flush=True)


if __name__ == "__main__":
    main()
