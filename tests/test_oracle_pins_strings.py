"""Pins of the oracle's Lagrangian density, string separation xi_L and velocity
estimators (arXiv:1809.00995, Sec. 2, Eqs. (9)-(10) and (12)) against exact
solutions of the continuum theory.

With lambda = 2 e^2 the straight Nielsen-Olesen string is the BPS vortex: its
profile solves two first-order radial equations (solved here with scipy), its
energy per unit length is exactly 2 pi sigma^2 (this fixes the tension mu in
xi_L), and its Lagrangian density is minus its energy density.  A Lorentz
boost with velocity v along x gives an exact moving string; for it the
weighted estimator 2R/(1+R) equals v^2 for every weight that is a Lorentz
scalar (the Lagrangian, the potential) and, because the transverse stresses
of a BPS vortex vanish pointwise, also for the energy-density weight and for
the equation-of-state estimator.  The lattice samples these continuum fields,
so every lattice value must approach the exact one as dx^2: the tests check
the Richardson extrapolation from dx = 0.5 and 0.25 and the convergence.

On the expanding lattice at conformal time tau the theory at fixed a is a
flat Abelian-Higgs model with couplings e0 a^s and lambda0 a^(2s) (still BPS)
times an overall a^2, so the same string with comoving inverse width
m = e0 sigma a^s pins the a-dependence of the measured densities and of the
prefactor of xi_L.

Field states are built here, in unitary gauge (phi real), from the continuum
solution: |phi| and Pi = D_t phi at the sites, the link angles as line
integrals of the gauge field along each link, E_y as the line integral of the
electric field F_ty = -gamma v B'.  Nothing here calls the HIP library.
"""
import functools

import numpy as np
import pytest
from scipy.integrate import solve_bvp

from tests import inputs as I

R0, R1 = 1e-6, 16.0          # radial range of the profile in units of 1/m


@functools.lru_cache(maxsize=1)
def bps_profile():
    """The unit-winding BPS vortex (lambda = 2 e^2), in r~ = m r with m = e sigma:
    f' = f (1 - a) / r~,  a' = r~ (1 - f^2),  f(0) = a(0) = 0, f, a -> 1.
    phi = sigma f e^{i theta}; the gauge field is a(r~)/r~ (azimuthal, units of 1/e)."""
    def rhs(r, y):
        f, a = y
        return np.vstack([f * (1 - a) / r, r * (1 - f * f)])

    def bc(ya, yb):      # a ~ r^2/2 at the centre, f -> 1 far away
        return np.array([ya[1] - 0.5 * R0**2, yb[0] - 1.0])

    r = np.concatenate([np.geomspace(R0, 1.0, 200), np.linspace(1.0, R1, 400)[1:]])
    sol = solve_bvp(rhs, bc, r, np.vstack([np.tanh(r), 1 - np.exp(-r * r / 2)]),
                    tol=1e-10, max_nodes=200000)
    assert sol.status == 0, sol.message

    def prof(rt):
        rt = np.asarray(rt, dtype=float)
        f, a = np.ones_like(rt), np.ones_like(rt)
        m = rt < R1
        f[m], a[m] = sol.sol(np.maximum(rt[m], R0))
        return f, a
    return prof


def test_bps_profile_has_unit_tension():
    """The continuum energy per unit length of the solved profile,
    2 pi int r dr [f'^2 + f^2 (1-a)^2/r^2 + a'^2/(2 r^2) + (1 - f^2)^2/2],
    is 2 pi (sigma = e = 1): the Bogomolny bound, saturated."""
    prof = bps_profile()
    r = np.linspace(R0, R1, 400001)
    f, a = prof(r)
    fp = f * (1 - a) / r
    ap = r * (1 - f * f)
    dens = fp**2 + f**2 * (1 - a) ** 2 / r**2 + ap**2 / (2 * r**2) + 0.5 * (1 - f * f) ** 2
    e = 2 * np.pi * np.sum(0.5 * (dens[1:] * r[1:] + dens[:-1] * r[:-1]) * np.diff(r))
    assert e == pytest.approx(2 * np.pi, rel=1e-7)


_GX, _GW = np.polynomial.legendre.leggauss(16)
_GX, _GW = 0.5 * (_GX + 1.0), 0.5 * _GW


def string_pair(n, dx, nz, m, sigma, v, t_mom=0.0):
    """A straight string (winding +1) and anti-string (-1) along z, at
    x = L/2 + 0.3 dx and y = L/4 + dx/2, 3L/4 + dx/2 (L = n dx), both moving with
    velocity v along x.  phi and A are taken at time 0, Pi and E at time t_mom.
    Each string's fields are those of the nearest periodic image (the profile
    reaches its vacuum to exp(-m L/2 sqrt 2)).  Returns the (10, nz, n, n) state."""
    prof = bps_profile()
    gam = 1.0 / np.sqrt(1.0 - v * v)
    L = n * dx
    xs = np.arange(n) * dx
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    cores0 = [(L / 2 + 0.3 * dx, L / 4 + 0.5 * dx, 1), (L / 2 + 0.3 * dx, 3 * L / 4 + 0.5 * dx, -1)]

    def rel(px, py, cx, cy):          # displacement from a core, nearest image
        return (px - cx + L / 2) % L - L / 2, (py - cy + L / 2) % L - L / 2

    def scalar(t):
        """|phi|/sigma, its x-derivative in the string frame (x' = gamma x) and
        the unitary-gauge A_x (the winding's 2 pi moved into the links)."""
        mod, dmod, ax = np.ones_like(X), np.zeros_like(X), np.zeros_like(X)
        parts = []
        for cx, cy, w in cores0:
            x0, y0 = rel(X, Y, cx + v * t, cy)
            xp = gam * x0
            rr = np.hypot(xp, y0)
            f, a = prof(m * rr)
            parts.append((f, a, xp, y0, rr, w))
            mod = mod * f
        for f, a, xp, y0, rr, w in parts:
            dmod += (mod / f) * (f * (1 - a) / (m * rr)) * m * xp / rr
            ax += w * (1 - a) * (-y0) / rr**2
        return mod, dmod, ax

    # link angles: line integrals of w (1 - a) d theta in the string frame, the
    # d theta part exactly, the a d theta part by Gauss-Legendre quadrature
    links = []
    for ddx, ddy in ((dx, 0.0), (0.0, dx)):
        tot = np.zeros_like(X)
        for cx, cy, w in cores0:
            x0, y0 = rel(X, Y, cx, cy)
            x0p, dxp = gam * x0, gam * ddx
            dth = np.arctan2(y0 + ddy, x0p + dxp) - np.arctan2(y0, x0p)
            dth = (dth + np.pi) % (2 * np.pi) - np.pi
            acc = np.zeros_like(X)
            for t_, w_ in zip(_GX, _GW):
                xx, yy = x0p + t_ * dxp, y0 + t_ * ddy
                r2 = xx * xx + yy * yy
                _, aa = prof(m * np.sqrt(r2))
                acc += w_ * aa * (xx * ddy - yy * dxp) / r2
            tot += w * (dth - acc)
        links.append(tot)

    mod, _, _ = scalar(0.0)
    modm, dmodm, axm = scalar(t_mom)
    pi = -gam * v * sigma * (dmodm + 1j * axm * modm)      # D_t phi = -gamma v D'_x phi
    ey = np.zeros_like(X)                                  # int F_ty dy, F_ty = -gamma v B'
    for t_, w_ in zip(_GX, _GW):
        b = np.zeros_like(X)
        for cx, cy, w in cores0:
            x0, y0 = rel(X, Y + t_ * dx, cx + v * t_mom, cy)
            f, _ = prof(m * np.hypot(gam * x0, y0))
            b += -w * m * m * (1 - f * f)
        ey += w_ * dx * b
    ey *= -gam * v
    st = np.zeros((10, nz, n, n))
    st[I.PHR] = sigma * mod
    st[I.PIR], st[I.PII] = pi.real, pi.imag
    st[I.AX], st[I.AY] = links
    st[I.EY] = ey
    return st


# (era_p, s, a at the measurement, e0, sigma): flat space, and expanding
# backgrounds where the measured densities carry different powers of a
CASES = [(0.0, 1.0, 1.0, 1.0, 1.0),
         (0.0, 1.0, 1.0, 0.8, 1.25),
         (1.0, 1.0, 0.8, 1.0, 1.0),
         (2.0, 0.0, 0.5, 1.0, 1.0),
         (1.0, 0.5, 0.64, 0.9, 1.1)]
SPACINGS = ((0.5, 40), (0.25, 80))       # box L = 20 in both
NZ = 4


def _measure_pair(O, case, v, dx, n):
    era, s, a, e0, sigma = case
    tau_ref = 10.0
    tau0 = tau_ref * a ** (1.0 / era) if era > 0 else 1.0
    m = e0 * sigma * a**s
    p = O.Params(n, n, NZ, dx=dx, dt=0.05, tau0=tau0, tau_ref=tau_ref, era_p=era, s=s,
                 lambda0=2 * e0 * e0, e0=e0, sigma=sigma)
    assert O.scale_factor(p, tau0) == pytest.approx(a, rel=1e-14)
    return p, O.measure(p, 0, string_pair(n, dx, NZ, m, sigma, v))


def _richardson(values):
    """Extrapolate Q(dx) = Q0 + c dx^2 from dx = 0.5 and 0.25."""
    return (4.0 * values[1] - values[0]) / 3.0


def _check_converges(values, exact, tol_extrap, what):
    err = [v_ - exact for v_ in values]
    q0 = _richardson(values)
    assert abs(q0 - exact) <= tol_extrap, f"{what}: extrapolated {q0} vs exact {exact} ({values})"
    # second order: halving dx divides the error by about four
    assert abs(err[1]) <= 0.4 * abs(err[0]) + 1e-6, f"{what}: no dx^2 convergence ({values})"


@pytest.mark.parametrize("case", CASES, ids=lambda c: "era%g-s%g-a%g-e%g-sig%g" % c)
def test_static_bps_strings_fix_lagrangian_and_xi_l(O, case):
    """Static BPS pair (Pi = E = 0): dx^3 sum L per unit length -> -2 (2 pi sigma^2) a^2
    (L = -rho for a static field; rho integrates to the BPS tension), and
    xi_L -> sqrt(V_box / length) with length = 2 L_z, the true string length:
    this fixes mu = 2 pi sigma^2 and the prefactor a of xi_L (Eq. (9))."""
    era, s, a, e0, sigma = case
    lag, xi, ratio = [], [], []
    for dx, n in SPACINGS:
        p, ob = _measure_pair(O, case, 0.0, dx, n)
        lz = NZ * dx
        lag.append(ob.sum_lag / lz / (-4 * np.pi * sigma**2 * a * a))
        xi.append(ob.xi_l / np.sqrt((n * dx) ** 2 / 2))
        ratio.append(ob.sum_lag / ob.energy)
        assert np.all(np.array(ob.v2) == 0.0)
    _check_converges(lag, 1.0, 5e-4, "sum L per length")
    _check_converges(xi, 1.0, 5e-4, "xi_L")
    assert np.allclose(ratio, -1.0, rtol=1e-13, atol=0)


@pytest.mark.parametrize("v", [0.3, 0.6])
@pytest.mark.parametrize("case", CASES[0:1] + CASES[2:5], ids=lambda c: "era%g-s%g-a%g-e%g-sig%g" % c)
def test_boosted_bps_strings_fix_velocity_estimators(O, case, v):
    """BPS pair boosted to velocity v along x: <v^2>_X = 2R/(1+R) (Eq. (10))
    -> v^2 for X = L, V and rho, and <v^2>_w (Eq. (12)) -> v^2; dx^3 sum L per
    unit length -> -2 (2 pi sigma^2) a^2 / gamma (L is a Lorentz scalar, the
    string is contracted), xi_L -> sqrt(gamma V_box / (2 L_z))."""
    era, s, a, e0, sigma = case
    gam = 1.0 / np.sqrt(1.0 - v * v)
    v2 = {k: [] for k in ("L", "V", "rho", "w")}
    lag, xi = [], []
    for dx, n in SPACINGS:
        _, ob = _measure_pair(O, case, v, dx, n)
        for k, val in zip(("L", "V", "rho"), ob.v2):
            v2[k].append(val)
        v2["w"].append(ob.v2_eos)
        lz = NZ * dx
        lag.append(ob.sum_lag / lz / (-4 * np.pi * sigma**2 * a * a / gam))
        xi.append(ob.xi_l / np.sqrt(gam * (n * dx) ** 2 / 2))
        assert ob.num[0] * ob.den[0] > 0
    for k, vals in v2.items():
        _check_converges(vals, v * v, 5e-4, f"<v^2>_{k}")
        assert abs(vals[1] - v * v) < 0.02 * v * v, (k, vals)
    _check_converges(lag, 1.0, 5e-4, "sum L per length")
    _check_converges(xi, 1.0, 5e-4, "xi_L")


def test_boosted_string_moves_rigidly(O):
    """Evolved with Eqs. (4)-(7) in flat space, the boosted BPS pair (momenta
    sampled at t = -dt/2, the time level they are stored at) moves at v: the
    potential-weighted centre of each string advances v T, its energy is kept
    and <v^2> stays v^2.  Lattice dispersion slows it at O(dx^2)."""
    v, T = 0.5, 6.0
    rel = []
    for (dx, n), dt in zip(SPACINGS, (0.1, 0.05)):
        p = O.Params(n, n, NZ, dx=dx, dt=dt, tau0=0.0, tau_ref=1.0, era_p=0.0, s=1.0)
        st = string_pair(n, dx, NZ, 1.0, 1.0, v, t_mom=-dt / 2)
        nsteps = int(round(T / dt))

        def centres(state):
            pot = (0.25 * (state[I.PHR] ** 2 + state[I.PHI] ** 2 - 1.0) ** 2).sum(axis=0)
            ang = 2 * np.pi * np.arange(n) / n
            out = []
            for rows in (slice(0, n // 2), slice(n // 2, n)):
                w = pot[rows].sum(axis=0)
                out.append(np.arctan2((w * np.sin(ang)).sum(), (w * np.cos(ang)).sum()))
            return np.array(out) * n * dx / (2 * np.pi)

        m0 = O.measure(p, 0, st)
        c0 = centres(st)
        st1, _ = O.run(p, st, 0, nsteps)
        m1 = O.measure(p, nsteps, st1)
        moved = (centres(st1) - c0) % (n * dx)
        rel.append(moved / (v * T) - 1.0)
        assert m1.energy == pytest.approx(m0.energy, rel=2e-4)
        assert m1.v2[0] == pytest.approx(v * v, rel=0.02)
    assert np.abs(rel[1]).max() < 0.01, rel
    assert np.abs(rel[1]).max() < 0.4 * np.abs(rel[0]).min(), rel


@pytest.mark.parametrize("era,s", [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (2.0, 0.0), (2.0, 1.0), (1.0, 0.5)])
def test_lagrangian_terms_match_energy_terms(O, era, s):
    """The Lagrangian density is kinetic minus potential energy, term by term
    with the same powers of a as the energy density (whose terms the FRW energy
    balance pins): a static field has sum L = -sum rho, a field with only
    scalar momentum or only electric field has sum L = +sum rho."""
    n = 6
    p = O.Params(n, n, n, tau0=1.5, tau_ref=2.0, era_p=era, s=s)
    base = I.random_state(n, seed=31)
    static = base.copy()
    static[I.PIR:I.PII + 1] = 0.0
    static[I.EX:I.EZ + 1] = 0.0
    m = O.measure(p, 0, static)
    assert m.grad > 0 and m.mag > 0 and m.pot > 0
    assert m.sum_lag == pytest.approx(-m.energy, rel=1e-13)

    uniform = np.zeros_like(base)
    uniform[I.PHR], uniform[I.PHI] = np.cos(0.7), np.sin(0.7)
    kinetic = uniform.copy()
    kinetic[I.PIR:I.PII + 1] = base[I.PIR:I.PII + 1]
    m = O.measure(p, 0, kinetic)
    assert m.kin > 0 and m.sum_lag == pytest.approx(m.energy, rel=1e-13)
    assert m.energy == pytest.approx(m.kin, rel=1e-13)

    electric = uniform.copy()
    electric[I.EX:I.EZ + 1] = base[I.EX:I.EZ + 1]
    m = O.measure(p, 0, electric)
    assert m.elec > 0 and m.sum_lag == pytest.approx(m.energy, rel=1e-13)
    assert m.energy == pytest.approx(m.elec, rel=1e-13)
