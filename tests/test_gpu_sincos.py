"""The device sine and cosine of the link phasors in FP32, read back through one
step of the library (through the C ABI) against the FP64 oracle.

The states used here have |phi| = 1, Pi = 0, E = 0, A_y = A_z = 0 everywhere,
A_x = theta on sites with even x and 0 on sites with odd x.  The imaginary part
of the covariant Laplacian (Eq. (4)) at a site with even x then has a single
non-zero term:
- phi = 1 everywhere: Im[e^{i theta} phi(x + 1)] = sin(theta);
- phi = 1 on even x, i on odd x: Im[e^{i theta} phi(x + 1)] + Im[phi(x - 1)]
  = cos(theta) + 1, the one rounded sum of the Laplacian (at most 6e-8);
the potential term vanishes at |phi| = sigma, so after one step Im Pi = c g(theta)
at those sites, g = sin or cos + 1, with one coefficient c for all of them.

The bound: the device's stated sin/cos error (4.3e-7 absolute), the rounding of
cos + 1, and four FP32 roundings of the products that scale the Laplacian.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AH = pytest.importorskip("paper_1809_00995_amd")
from tests.gpu_util import fields_np, oracle_params, upload  # noqa: E402

SHAPE = (64, 12, 10)


def _link_state(lim, seed, odd_phi_imag):
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(seed)
    st = np.zeros((10, nz, ny, nx))
    st[0] = 1.0
    if odd_phi_imag:
        st[0, :, :, 1::2] = 0.0
        st[1, :, :, 1::2] = 1.0
    theta = rng.uniform(-lim, lim, (nz, ny, nx // 2))
    theta[0, 0, :4] = [0.0, np.pi / 2, -np.pi, 2 * np.pi]
    theta = theta.astype(np.float32).astype(np.float64)
    st[4, :, :, 0::2] = theta
    return st, theta


@pytest.mark.parametrize("kernel", [AH.AH_KERNEL_PLAIN, AH.AH_KERNEL_TILED], ids=["plain", "tiled"])
@pytest.mark.parametrize("lim", [4.0, 100.0, 1e4])
@pytest.mark.parametrize("fn", ["sin", "cos"])
def test_link_phasors_within_stated_error(O, kernel, lim, fn):
    print("CASE test=link_phasors kernel", kernel, "lim", lim, "fn", fn, flush=True)
    p = AH.Params(*SHAPE, precision=AH.AH_FP32, tau0=2.0, tau_ref=4.0, era_p=1.0, s=1.0,
                  init=AH.AH_INIT_NONE, layout=AH.AH_LAYOUT_15)
    st, theta = _link_state(lim, seed=31, odd_phi_imag=(fn == "cos"))
    with AH.Context([p], [upload(p, st)]) as c:
        c.set_kernel(kernel)
        c.step(1)
        got = fields_np(c)[3][:, :, 0::2]
    ref = O.run(oracle_params(O, p), st, 0, 1)[0][3][:, :, 0::2]
    g = np.sin(theta) if fn == "sin" else np.cos(theta) + 1.0
    coef = (ref * g).sum() / (g * g).sum()
    # the construction: the oracle's Im Pi at even x is c g(theta)
    assert abs(coef) > 0.1
    assert np.abs(ref - coef * g).max() < 1e-12 * abs(coef)
    bound = (4.3e-7 + 6e-8) * abs(coef) + 4 * 2.0 ** -24 * np.abs(ref)
    err = np.abs(got - ref)
    print(f"max err {err.max() / abs(coef):.3e} (units of c), worst err/bound "
          f"{(err / bound).max():.3f}", flush=True)
    assert np.all(err < bound), (err / bound).max()
