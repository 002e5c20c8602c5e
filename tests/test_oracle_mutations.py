"""The oracle's pins catch plausible mistakes: each case plants one in a copy of
the oracle's C source (a dropped factor, a wrong power of a, a flipped sign, a
swapped index) and runs the pin suite on the copy, which must fail.  CPU only;
the product library is not involved.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what is wrong, text of the oracle, text planted in its place)
MUT = [
 ("c3 missing a^2s", "c->c3 = p->dt * 0.5 * p->lambda0 * r * r * pow(a0, 2.0 * s0);", "c->c3 = p->dt * 0.5 * p->lambda0 * r * r;"),
 ("d1 wrong power", "c->d1 = sm == sp ? pow(q, 2.0 * (1.0 - sp))", "c->d1 = sm == sp ? pow(q, 2.0 * sp)"),
 ("d3 no factor 2", "c->d3 = 2.0 * p->dt", "c->d3 = 1.0 * p->dt"),
 ("d3 wrong power", "r * r * pow(ap, 2.0 * sp);", "r * r * pow(a0, 2.0 * sp);"),
 ("c2 missing r^2", "c->c2 = h * r * r;", "c->c2 = h * r;"),
 ("d2 wrong power", "c->d2 = h * (s0 == sp ? pow(r, 2.0 * (1.0 - sp))", "c->d2 = h * (s0 == sp ? pow(r, 2.0)"),
 ("link sign fwd", "lr += cos(ajp) * qr - sin(ajp) * qi;\n        li += cos(ajp) * qi + sin(ajp) * qr;", "lr += cos(ajp) * qr + sin(ajp) * qi;\n        li += cos(ajp) * qi - sin(ajp) * qr;"),
 ("curl sign", "curl -= sin(plaquette(", "curl += sin(plaquette("),
 ("current sign", "double cur = qr * wi - qi * wr;", "double cur = qi * wr - qr * wi;"),
 ("plaquette index", "return Ai[o] + Aj[pi] - Ai[pj] - Aj[o];", "return Ai[o] + Aj[pj] - Ai[pi] - Aj[o];"),
 ("BB factor", "BB *= 2.0 * idx2 * idx2;", "BB *= idx2 * idx2;"),
 ("g power", "double g = pow(a, 2.0 * (1.0 - sn)) / (2.0 * p->e0 * p->e0);", "double g = pow(a, 2.0 * sn) / (2.0 * p->e0 * p->e0);"),
 ("h power", "double h = p->lambda0 * pow(a, 2.0 + 2.0 * sn);", "double h = p->lambda0 * pow(a, 2.0 * sn);"),
 ("winding Y index", "double loop = Y[i * N + o] + Y[j * N + fi] - Y[i * N + fj]", "double loop = Y[i * N + o] + Y[j * N + fj] - Y[i * N + fi]"),
 ("wrap offset", "return u - OR_TWO_PI * floor((u + OR_PI) / OR_TWO_PI);", "return u - OR_TWO_PI * floor(u / OR_TWO_PI);"),
 ("gauss a_p", "double am = or_scale_factor(p, tau - 0.5 * p->dt);\n    double fe", "double am = or_scale_factor(p, tau + 0.5 * p->dt);\n    double fe"),
 ("gauss sign", "double G = fe * div + fp * charge;", "double G = fe * div - fp * charge;"),
 ("potential sign", "- c->c3 * v * pr;", "+ c->c3 * v * pr;"),
 ("drift uses old Pi", "out10[PHR] = pr + p->dt * pinr;", "out10[PHR] = pr + p->dt * in[PIR * N + o];"),
 ("G uses e^-iA", "double dr = cos(ai) * qr - sin(ai) * qi - pr;\n                    double di = cos(ai) * qi + sin(ai) * qr - pim;", "double dr = cos(ai) * qr + sin(ai) * qi - pr;\n                    double di = cos(ai) * qi - sin(ai) * qr - pim;"),
 ("pressure gauge sign", "double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 - h * V;", "double pres = a2 * K - a2 * G / 3.0 - g * (EE + BB) / 3.0 - h * V;"),
 ("pressure grad 1/3", "double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 - h * V;", "double pres = a2 * K - a2 * G + g * (EE + BB) / 3.0 - h * V;"),
 ("pressure pot sign", "double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 - h * V;", "double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 + h * V;"),
 ("init phase offset", "double theta = OR_TWO_PI * u - OR_PI;", "double theta = OR_PI * u - OR_PI;"),
 # the Lagrangian density, the weights of <v^2>_X and xi_L (Eqs. (9)-(10), (12))
 ("L weight of num is rho", "acc[S_NUM_L] += K * lag;", "acc[S_NUM_L] += K * rho;"),
 ("V weight of den is L", "acc[S_DEN_V] += G * V;", "acc[S_DEN_V] += G * lag;"),
 ("L gradient sign", "double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;", "double lag = a2 * K + a2 * G + g * (EE - BB) - h * V;"),
 ("L magnetic sign", "double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;", "double lag = a2 * K - a2 * G + g * (EE + BB) - h * V;"),
 ("L electric sign", "double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;", "double lag = a2 * K - a2 * G + g * (-EE - BB) - h * V;"),
 ("L potential sign", "double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;", "double lag = a2 * K - a2 * G + g * (EE - BB) + h * V;"),
 ("v2 is R/(1+R)", "obs->v2[k] = 2.0 * R / (1.0 + R);", "obs->v2[k] = R / (1.0 + R);"),
 ("mu is pi sigma^2", "? a * sqrt(-(OR_TWO_PI * s2) * vbox / obs->sum_lag)", "? a * sqrt(-(OR_PI * s2) * vbox / obs->sum_lag)"),
 ("mu is 2 pi sigma", "? a * sqrt(-(OR_TWO_PI * s2) * vbox / obs->sum_lag)", "? a * sqrt(-(OR_TWO_PI * p->sigma) * vbox / obs->sum_lag)"),
 ("xi_L without a", "? a * sqrt(-(OR_TWO_PI * s2) * vbox / obs->sum_lag)", "? sqrt(-(OR_TWO_PI * s2) * vbox / obs->sum_lag)"),
 ("eos without 3", "obs->v2_eos = 0.5 * (1.0 + 3.0 * obs->pres_lag / obs->rho_lag);", "obs->v2_eos = 0.5 * (1.0 + obs->pres_lag / obs->rho_lag);"),
 ("eos density weight", "acc[S_RHO_L] += rho * lag;", "acc[S_RHO_L] += rho * rho;"),
]


@pytest.mark.parametrize("name,orig,planted", MUT, ids=[m[0] for m in MUT])
def test_pins_catch_planted_mistake(tmp_path, name, orig, planted):
    shutil.copytree(os.path.join(ROOT, "oracle"), tmp_path / "oracle",
                    ignore=shutil.ignore_patterns("*.so", "*.tmp", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), tmp_path / "tests",
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path)
    path = tmp_path / "oracle" / "ah_oracle.c"
    src = path.read_text()
    assert src.count(orig) == 1, f"{name}: the oracle text to mutate is not unique or gone"
    path.write_text(src.replace(orig, planted))
    # copies run side by side under a parallel test runner share the cores
    # (OpenMP threads that spin on a shared core slow the pins a hundredfold)
    env = dict(os.environ)
    workers = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1"))
    if workers > 1:
        env["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // workers))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_pins_strings.py"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode != 0, f"{name}: no pin failed\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "error" in r.stdout.lower(), r.stdout[-2000:]
