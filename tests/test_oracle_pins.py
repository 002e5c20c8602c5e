"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a
published number, a closed form, an exact invariant of the discrete system, an
independent ODE integration (scipy) of the same lattice model, or a special
case with a known answer.  Each test names the passage of arXiv:1809.00995 it
pins.  All tests run on the CPU in seconds.
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from tests import inputs as I
from tests.inputs import gauge_transform

HERE = os.path.dirname(os.path.abspath(__file__))
ERAS = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (2.0, 0.0), (2.0, 1.0), (1.0, 0.5)]


def khat2(k, n, dx):
    """Eigenvalue of minus the lattice Laplacian for wave number 2 pi k / (n dx)."""
    return 4.0 / dx**2 * np.sin(np.pi * k / n) ** 2


# --------------------------------------------------------------------------
# initial conditions (Sec. 2, text after Eq. (8))

def test_splitmix64_published_vector(O):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    for k, val in rows:
        assert O.splitmix64(1234567, int(k)) == int(val)


def test_random_phase_init(O):
    p = O.Params(16, 16, 16, seed=77)
    st = O.init_random_phase(p)
    assert np.allclose(st[I.PHR] ** 2 + st[I.PHI] ** 2, p.sigma**2, atol=1e-15, rtol=0)
    assert not st[I.PIR:].any()
    th = np.arctan2(st[I.PHI], st[I.PHR]).ravel()
    hist, _ = np.histogram(th, bins=16, range=(-np.pi, np.pi))
    expected = th.size / 16
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert chi2 < 40.0          # 15 dof: p ~ 5e-4
    # different seeds give different fields
    st2 = O.init_random_phase(O.Params(16, 16, 16, seed=78))
    assert np.abs(st2[0] - st[0]).max() > 0.5
    # Gauss's law holds exactly at the start (all momenta zero)
    assert O.gauss(p, 0, st) == (0.0, 0.0)


# --------------------------------------------------------------------------
# the update, Eqs. (4)-(8)

@pytest.mark.parametrize("era,s", ERAS)
def test_vacuum_is_bitwise_stationary(O, era, s):
    p = O.Params(6, 6, 6, tau0=0.0, tau_ref=3.0, era_p=era, s=s)
    st0 = O.vacuum(p)
    st, _ = O.run(p, st0, 0, 30)
    assert np.array_equal(st, st0)


@pytest.mark.parametrize("era,s", [(0.0, 0.0), (1.0, 1.0), (2.0, 0.0)])
def test_pure_gauge_vacuum_is_stationary(O, era, s):
    p = O.Params(6, 5, 7, tau0=1.0, tau_ref=3.0, era_p=era, s=s)
    alpha = I.gauge_function((6, 5, 7), seed=5)
    st0 = gauge_transform(O.vacuum(p), alpha)
    st, _ = O.run(p, st0, 0, 30)
    assert np.abs(st - st0).max() < 1e-12


@pytest.mark.parametrize("era,s", ERAS)
def test_gauss_law_conserved_site_by_site(O, era, s):
    """Sec. 4: Gauss's law is preserved to machine precision.  Here the stronger
    statement: for an arbitrary state the residual G_x is constant in time."""
    p = O.Params(7, 6, 5, tau0=1.0, tau_ref=2.0, era_p=era, s=s)
    st = I.random_state((7, 6, 5), seed=11)
    _, _, g0 = O.gauss(p, 0, st, site_map=True)
    assert np.abs(g0).max() > 0.01              # genuinely violated initially
    for n in range(40):
        st = O.step(p, n, st)
        _, _, g = O.gauss(p, n + 1, st, site_map=True)
        assert np.abs(g - g0).max() < 1e-12 * max(1.0, np.abs(g0).max())


def test_gauss_law_random_phase_run(O):
    """32^3 random-phase run from tau = 0 to 8 (80 steps, radiation, s = 1)."""
    p = O.Params(32, 32, 32, tau0=0.0, tau_ref=8.0, era_p=1.0, s=1.0, seed=1)
    st = O.init_random_phase(p)
    for n in range(80):
        st = O.step(p, n, st)
        if (n + 1) % 20 == 0:
            mx, _ = O.gauss(p, n + 1, st)
            assert mx < 1e-12


@pytest.mark.parametrize("era,s", [(0.0, 0.0), (1.0, 1.0), (2.0, 0.5)])
def test_gauge_covariance_of_the_update(O, era, s):
    p = O.Params(6, 7, 5, tau0=1.0, tau_ref=2.0, era_p=era, s=s)
    st = I.random_state((6, 7, 5), seed=3)
    alpha = I.gauge_function((6, 7, 5), seed=4)
    a, _ = O.run(p, gauge_transform(st, alpha), 0, 6)
    b, _ = O.run(p, st, 0, 6)
    assert np.abs(a - gauge_transform(b, alpha)).max() < 1e-12


def test_time_reversibility_flat(O):
    p = O.Params(8, 8, 8, era_p=0.0)
    st0 = I.smooth_state(8, seed=9)
    n = 30
    sn, _ = O.run(p, st0, 0, n)
    sn1 = O.step(p, n, sn)
    rev = sn.copy()
    rev[I.PIR:I.PII + 1] = -sn1[I.PIR:I.PII + 1]
    rev[I.EX:] = -sn1[I.EX:]
    back, _ = O.run(p, rev, 0, n)
    s1 = O.step(p, 0, st0)
    assert np.abs(back[[0, 1, 4, 5, 6]] - st0[[0, 1, 4, 5, 6]]).max() < 1e-12
    assert np.abs(back[[2, 3, 7, 8, 9]] + s1[[2, 3, 7, 8, 9]]).max() < 1e-12


def _leapfrog_mode_check(O, p, st0, field, shape_fn, omega2, eps, nsteps):
    """Compare with the exact solution of the linearised leapfrog:
    d_n = eps cos(w n dt) shape, with sin(w dt / 2) = (dt/2) sqrt(omega2)."""
    w = 2.0 / p.dt * np.arcsin(0.5 * p.dt * np.sqrt(omega2))
    st = st0.copy()
    st[field] += eps * shape_fn
    mom = I.PIR if field in (I.PHR, I.PHI) else I.EX + (field - I.AX)
    if field == I.PHI:
        mom = I.PII
    st[mom] = eps * (1.0 - np.cos(w * p.dt)) / p.dt * shape_fn
    ref = st0[field]
    for n in range(nsteps):
        st = O.step(p, n, st)
        if (n + 1) % 25 == 0:
            expect = ref + eps * np.cos(w * (n + 1) * p.dt) * shape_fn
            assert np.abs(st[field] - expect).max() < 2e-3 * eps, n


def test_dispersion_higgs_mode_flat(O):
    """Radial mode about the vacuum: omega^2 = khat^2 + lambda0 sigma^2
    (m_phi = sqrt(lambda) sigma, Sec. 2 after Eq. (1))."""
    n = 16
    p = O.Params(n, n, n, era_p=0.0)
    x = np.arange(n)[None, None, :] * np.ones((n, n, n))
    _leapfrog_mode_check(O, p, O.vacuum(p), I.PHR, np.cos(2 * np.pi * 2 * x / n),
                         khat2(2, n, p.dx) + p.lambda0 * p.sigma**2, 1e-6, 200)


def test_dispersion_photon_flat(O):
    """Transverse gauge mode about the vacuum: omega^2 = khat^2 + 2 e0^2 sigma^2
    (equal to the Higgs mass at e0 = 1, lambda0 = 2, Sec. 2 after Eq. (8))."""
    n = 16
    p = O.Params(n, n, n, era_p=0.0)
    z = np.arange(n)[:, None, None] * np.ones((n, n, n))
    _leapfrog_mode_check(O, p, O.vacuum(p), I.AX, np.cos(2 * np.pi * 3 * z / n),
                         khat2(3, n, p.dx) + 2 * p.e0**2 * p.sigma**2, 1e-6, 200)


def test_energy_conservation_flat(O):
    """Flat space (a = 1): the leapfrog conserves the energy to O(dt^2).
    Energy is measured with the momenta averaged over the two half steps around
    tau_n; the measured parts (kin, grad, elec, mag, pot) are those of rho."""
    def max_dev(dt):
        p = O.Params(8, 8, 8, era_p=0.0, dt=dt)
        st = I.smooth_state(8, seed=21, amp=0.5)
        nsteps = int(round(4.0 / dt))
        obs = []
        for n in range(nsteps + 1):
            obs.append(O.measure(p, n, st))
            st = O.step(p, n, st)
        en = []
        for n in range(nsteps):
            a, b = obs[n], obs[n + 1]
            en.append(0.5 * (a.kin + b.kin) + a.grad + 0.5 * (a.elec + b.elec) + a.mag + a.pot)
        en = np.array(en)
        share = max(o.mag for o in obs) / en[0]
        assert share > 0.02                     # magnetic term is exercised
        return np.abs(en - en[0]).max() / en[0]

    d1, d2, d3 = max_dev(0.1), max_dev(0.05), max_dev(0.025)
    assert d1 < 4e-2
    assert 0.15 < d2 / d1 < 0.35 and 0.15 < d3 / d2 < 0.35


# ------------------------- FRW coefficients against an ODE integration -----

def _a(p, tau):
    return (max(tau, 0.0) / p.tau_ref) ** p.era_p


@pytest.mark.parametrize("era,s", [(1.0, 0.0), (1.0, 1.0), (2.0, 0.0), (2.0, 1.0), (1.0, 0.5)])
def test_frw_uniform_fields_match_ode(O, era, s):
    """Spatially uniform phi = f (real) and A_j: the lattice equations reduce to
        (a^2 f')'            = a^2 (2f/dx^2) sum_j (cos A_j - 1)
                               - (lambda0/2) a^(2+2s) (f^2 - sigma^2) f
        (a^(2(1-s)) A_j')'   = -2 e0^2 a^2 f^2 sin A_j
    (action of Sec. 2 with the couplings of Eq. (8)), integrated here with an
    adaptive RK method.  Pins c1, c3, d1, d3 and their powers of a."""
    p = O.Params(4, 4, 4, dt=0.002, tau0=2.0, tau_ref=2.0, era_p=era, s=s)

    def rhs(tau, y):
        f, u = y[0], y[1]
        A, w = y[2:5], y[5:8]
        a = _a(p, tau)
        hub = era / tau
        du = (-2 * hub * u + 2 * f / p.dx**2 * np.sum(np.cos(A) - 1)
              - 0.5 * p.lambda0 * a ** (2 * s) * (f * f - p.sigma**2) * f)
        dw = -2 * (1 - s) * hub * w - 2 * p.e0**2 * a ** (2 * s) * f * f * np.sin(A)
        return np.concatenate(([u, du], w, dw))

    y0 = np.array([1.2, 0.1, 0.3, -0.5, 0.8, 0.2, 0.1, -0.3])
    back = solve_ivp(rhs, (p.tau0, p.tau0 - 0.5 * p.dt), y0, rtol=1e-12, atol=1e-13).y[:, -1]
    st = np.zeros(p.shape)
    st[I.PHR] = y0[0]
    st[I.PIR] = back[1]
    for j in range(3):
        st[I.AX + j] = y0[2 + j]
        st[I.EX + j] = back[5 + j]
    nsteps = 500
    st, _ = O.run(p, st, 0, nsteps)
    tau_end = p.tau0 + nsteps * p.dt
    fwd = solve_ivp(rhs, (p.tau0, tau_end), y0, rtol=1e-12, atol=1e-13).y[:, -1]
    assert abs(st[I.PHR, 0, 0, 0] - fwd[0]) < 1e-4
    assert np.abs(st[I.PHI]).max() < 1e-14
    for j in range(3):
        assert abs(st[I.AX + j, 0, 0, 0] - fwd[2 + j]) < 1e-4
    # uniformity is preserved exactly up to rounding
    assert np.ptp(st[I.PHR]) < 1e-13


@pytest.mark.parametrize("era,s", [(1.0, 0.0), (1.0, 1.0), (2.0, 0.0), (2.0, 1.0), (1.0, 0.5)])
def test_frw_fourier_modes_match_ode(O, era, s):
    """A single lattice Fourier mode, amplitude g(tau):
      scalar (lambda0 = 0, A = 0):   (a^2 g')' = -a^2 khat^2 g        -> c1, c2
      gauge  (phi = 0, A_x(z)):      (a^(2(1-s)) g')' = -a^(2(1-s)) khat^2 g -> d1, d2."""
    n = 8
    p = O.Params(n, n, n, dt=0.002, tau0=2.0, tau_ref=2.0, era_p=era, s=s, lambda0=0.0)
    kh2 = khat2(1, n, p.dx)
    nsteps = 500
    tau_end = p.tau0 + nsteps * p.dt

    for kind in ("scalar", "gauge"):
        damp = 2.0 if kind == "scalar" else 2.0 * (1.0 - s)

        def rhs(tau, y):
            return [y[1], -damp * era / tau * y[1] - kh2 * y[0]]

        eps = 1.0 if kind == "scalar" else 1e-5
        y0 = [eps, 0.3 * eps]
        back = solve_ivp(rhs, (p.tau0, p.tau0 - 0.5 * p.dt), y0, rtol=1e-12, atol=1e-16).y[:, -1]
        fwd = solve_ivp(rhs, (p.tau0, tau_end), y0, rtol=1e-12, atol=1e-16).y[:, -1]
        st = np.zeros(p.shape)
        if kind == "scalar":
            shape = np.cos(2 * np.pi * np.arange(n) / n)[None, None, :] * np.ones((n, n, n))
            st[I.PHR], st[I.PIR] = y0[0] * shape, back[1] * shape
            field = I.PHR
        else:
            shape = np.cos(2 * np.pi * np.arange(n) / n)[:, None, None] * np.ones((n, n, n))
            st[I.AX], st[I.EX] = y0[0] * shape, back[1] * shape
            field = I.AX
        st, _ = O.run(p, st, 0, nsteps)
        assert np.abs(st[field] - fwd[0] * shape).max() < 1e-4 * eps, kind


@pytest.mark.parametrize("era,s", [(1.0, 0.0), (1.0, 1.0), (2.0, 0.5)])
def test_frw_energy_balance_pins_measured_densities(O, era, s):
    """For L(tau) = a^2 (K - G) + g(a) (EE - BB) - h(a) V the energy function
    rho obeys d(sum rho)/dtau = -dL/dtau|explicit
      = -(a'/a) [2 a^2 (K - G) + 2(1-s) g (EE - BB) - (2+2s) h V],
    with g = a^(2(1-s))/(2 e0^2), h = lambda0 a^(2+2s).  Checked on the
    measured component sums: pins the a-dependence of the densities against
    the a-dependence of the update."""
    p = O.Params(8, 8, 8, dt=0.005, tau0=4.0, tau_ref=4.0, era_p=era, s=s)
    st = I.smooth_state(8, seed=31, amp=0.4)
    nsteps = 120
    obs = []
    for n in range(nsteps + 2):
        obs.append(O.measure(p, n, st))
        st = O.step(p, n, st)
    tau = np.array([o.tau for o in obs])
    a = np.array([_a(p, t) for t in tau])
    g = a ** (2 * (1 - s)) / (2 * p.e0**2)
    kin_raw = np.array([o.kin for o in obs]) / a**2       # sum |Pi|^2 at n - 1/2
    ee_raw = np.array([o.elec for o in obs]) / g          # sum E^2 / dx^2 at n - 1/2
    grad = np.array([o.grad for o in obs])
    mag = np.array([o.mag for o in obs])
    pot = np.array([o.pot for o in obs])
    kin = a[:-1] ** 2 * 0.5 * (kin_raw[:-1] + kin_raw[1:])   # at integer time n
    elec = g[:-1] * 0.5 * (ee_raw[:-1] + ee_raw[1:])
    rho = kin + grad[:-1] + elec + mag[:-1] + pot[:-1]
    lhs = (rho[2:] - rho[:-2]) / (2 * p.dt)
    t = tau[1:-2]
    X = (2 * (kin - grad[:-1]) + 2 * (1 - s) * (elec - mag[:-1]) - (2 + 2 * s) * pot[:-1])[1:-1]
    rhs = -(era / t) * X
    assert np.abs(lhs - rhs).max() < 2e-3 * np.abs(rhs).max()


# --------------------------------------------------------------------------
# diagnostics, Eqs. (9)-(11)

def _vortex_pair(n, x1, y1, x2, y2):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    th = np.arctan2(y - y1, x - x1) - np.arctan2(y - y2, x - x2)
    st = np.zeros((10, n, n, n))
    st[I.PHR], st[I.PHI] = np.cos(th), np.sin(th)
    return st


def test_winding_straight_string_pair(O):
    """A straight vortex-antivortex pair along z pierces exactly one xy
    plaquette per z-slice each, with W = +1 and W = -1 (Eq. (11)); nothing in
    the yz and zx planes.  Also with a compensating (pure-gauge) A."""
    n = 16
    p = O.Params(n, n, n, era_p=0.0)
    st = _vortex_pair(n, n / 4 + 0.5, n / 2 + 0.5, 3 * n / 4 + 0.5, n / 2 + 0.5)
    for s in (st, gauge_transform(st, I.gauge_function(n, seed=8))):
        m = O.measure(p, 0, s, wind_map=True)
        w = m.wind
        assert m.n_wind == 2 * n and m.n_pierced == 2 * n
        assert m.n_wind_dir == [2 * n, 0, 0] and m.net_wind_dir == [0, 0, 0]
        assert (w[0, :, n // 2, n // 4] == 1).all()
        assert (w[0, :, n // 2, 3 * n // 4] == -1).all()
        assert np.abs(w).sum() == 2 * n
        assert m.length == pytest.approx(np.pi / 6 * p.dx * 2 * n, rel=1e-15)


def test_winding_random_phase_statistics(O):
    """Uniform random phases at the corners of a plaquette wind with
    probability exactly 1/3; the winding sums to zero over every closed
    surface, hence per orientation over the periodic lattice."""
    p = O.Params(24, 24, 24, seed=5)
    m = O.measure(p, 0, O.init_random_phase(p), wind_map=True)
    frac = m.n_pierced / (3 * 24**3)
    assert abs(frac - 1 / 3) < 0.012
    assert m.net_wind_dir == [0, 0, 0]
    w = m.wind.astype(np.int64)
    # per slice: xy windings summed over each z plane vanish
    assert not w[0].sum(axis=(1, 2)).any()
    assert not w[1].sum(axis=(0, 1)).any()      # yz plaquettes, per x slice
    assert not w[2].sum(axis=(0, 2)).any()      # zx plaquettes, per y slice


def test_observables_are_gauge_invariant(O):
    p = O.Params(8, 8, 8, tau0=2.0, tau_ref=4.0, era_p=1.0, s=1.0)
    st = I.random_state(8, seed=12)
    alpha = I.gauge_function(8, seed=13)
    m1 = O.measure(p, 3, st, wind_map=True)
    m2 = O.measure(p, 3, gauge_transform(st, alpha), wind_map=True)
    assert np.array_equal(m1.wind, m2.wind)
    for k in ("sum_lag", "energy", "kin", "grad", "elec", "mag", "pot"):
        assert getattr(m2, k) == pytest.approx(getattr(m1, k), rel=1e-12)
    for k in ("num", "den", "v2"):
        assert np.allclose(getattr(m2, k), getattr(m1, k), rtol=1e-11)
    g1 = O.gauss(p, 3, st, site_map=True)[2]
    g2 = O.gauss(p, 3, gauge_transform(st, alpha), site_map=True)[2]
    assert np.abs(g1 - g2).max() < 1e-12


def test_velocity_zero_at_rest_and_vacuum_energy(O):
    """Pi = 0 gives <v^2>_X = 0 exactly (Eq. (10)); the vacuum has zero energy
    density and no strings."""
    p = O.Params(8, 8, 8, tau0=1.0, tau_ref=1.0)
    m = O.measure(p, 0, O.init_random_phase(p))
    assert m.v2[1] == 0.0 and m.num == [0.0, 0.0, 0.0]
    v = O.measure(p, 0, O.vacuum(p))
    assert v.energy == 0.0 and v.n_wind == 0 and v.nonfinite == 0


def test_nonfinite_detection(O):
    p = O.Params(6, 6, 6)
    st = O.vacuum(p)
    st[I.EY, 2, 3, 4] = np.nan
    st[I.PHR, 0, 0, 1] = np.inf
    assert O.measure(p, 0, st).nonfinite == 2


@pytest.mark.parametrize("era", [1.0, 2.0])
def test_frw_continuity_pins_pressure(O, era):
    """With the true equations of motion (s = 1) the box-averaged physical
    energy density obeys the FRW continuity equation d(rho/a^4)/dtau =
    -3 (a'/a) (rho + p)/a^4, i.e. for the conformal sums
    d(sum rho)/dtau = (a'/a) sum (rho - 3 p).  Checked on the measured energy
    and pressure (Eq. (12)); the half-step offset of the momenta gives an
    O(dt) error, so dt is small."""
    p = O.Params(8, 8, 8, dt=0.002, tau0=4.0, tau_ref=4.0, era_p=era, s=1.0)
    st = I.smooth_state(8, seed=41, amp=0.4)
    nsteps = 200
    obs = []
    for n in range(nsteps + 1):
        obs.append(O.measure(p, n, st))
        st = O.step(p, n, st)
    tau = np.array([o.tau for o in obs])
    a = np.array([_a(p, t) for t in tau])
    rho = np.array([o.energy for o in obs])
    pres = np.array([o.pres for o in obs])
    kin = np.array([o.kin for o in obs])
    elec = np.array([o.elec for o in obs])
    # momenta averaged over the half steps around tau_n (second order in dt);
    # the kinetic parts enter rho as kin + elec and p as kin + elec / 3
    kraw = kin / a**2
    kmid = a[:-1] ** 2 * 0.5 * (kraw[:-1] + kraw[1:])
    emid = 0.5 * (elec[:-1] + elec[1:])          # g is constant for s = 1
    rho_m = rho[:-1] - kin[:-1] - elec[:-1] + kmid + emid
    pres_m = pres[:-1] - kin[:-1] - elec[:-1] / 3 + kmid + emid / 3
    lhs = (rho_m[2:] - rho_m[:-2]) / (2 * p.dt)
    rhs = era / tau[1:-2] * (rho_m[1:-1] - 3 * pres_m[1:-1])
    assert np.abs(lhs - rhs).max() < 2e-3 * np.abs(rhs).max()
    # the estimator of Eq. (12) as defined from the weighted sums
    o = obs[-1]
    assert o.v2_eos == pytest.approx(0.5 * (1 + 3 * o.pres_lag / o.rho_lag), rel=1e-14)


# ------------------------- core growth: s changes at tau_s (Sec. 2, after Eq. (8)) ----

@pytest.mark.parametrize("era", [1.0, 2.0])
def test_core_growth_switch_keeps_gauss_law(O, era):
    """s = -1 (core growth) until tau_s, then s = 1: the Gauss residual of an
    arbitrary state stays constant site by site through the switch."""
    p = O.Params(7, 6, 5, tau0=1.0, tau_ref=3.0, era_p=era, s=-1.0, s_late=1.0, tau_s=2.0)
    st = I.random_state((7, 6, 5), seed=17)
    _, _, g0 = O.gauss(p, 0, st, site_map=True)
    assert np.abs(g0).max() > 1e-3
    for n in range(25):                       # tau from 1.0 to 3.5 crosses tau_s = 2
        st = O.step(p, n, st)
        _, _, g = O.gauss(p, n + 1, st, site_map=True)
        assert np.abs(g - g0).max() < 1e-12 * max(1.0, np.abs(g0).max())


def test_core_growth_uniform_fields_match_ode(O):
    """Uniform phi = f and A_j across the switch of s at tau_s.  In canonical
    momenta P_f = a^2 f' and P_A = A'/e^2, which stay continuous when the
    couplings e = e0 a^(s-1), lambda = lambda0 a^(2(s-1)) jump:
        f' = P_f / a^2,   P_f' = a^2 (2f/dx^2) sum (cos A - 1) - (lambda0/2) a^(2+2s) (f^2 - 1) f
        A' = e0^2 a^(2(s-1)) P_A,   P_A' = -2 a^2 f^2 sin A
    integrated piecewise by RK; the leapfrog agrees to O(dt)."""
    p = O.Params(4, 4, 4, dt=0.001, tau0=2.0, tau_ref=2.0, era_p=1.0, s=-1.0, s_late=1.0,
                 tau_s=2.25)
    e0 = p.e0

    def rhs_for(s):
        def rhs(tau, y):
            f, pf, A, pA = y[0], y[1], y[2:5], y[5:8]
            a = _a(p, tau)
            df = pf / a**2
            dpf = (a**2 * 2 * f / p.dx**2 * np.sum(np.cos(A) - 1)
                   - 0.5 * p.lambda0 * a ** (2 + 2 * s) * (f * f - p.sigma**2) * f)
            dA = e0**2 * a ** (2 * (s - 1)) * pA
            dpA = -2 * a**2 * f * f * np.sin(A)
            return np.concatenate(([df, dpf], dA, dpA))
        return rhs

    f0, u0 = 1.2, 0.1
    A0 = np.array([0.3, -0.5, 0.8])
    w0 = np.array([0.2, 0.1, -0.3])
    a0 = _a(p, p.tau0)
    e_0 = e0 * a0 ** (p.s - 1)
    y0 = np.concatenate(([f0, a0**2 * u0], A0, w0 / e_0**2))
    # momenta at tau0 - dt/2 for the staggered start
    back = solve_ivp(rhs_for(p.s), (p.tau0, p.tau0 - 0.5 * p.dt), y0, rtol=1e-12, atol=1e-14).y[:, -1]
    am = _a(p, p.tau0 - 0.5 * p.dt)
    em = e0 * am ** (p.s - 1)
    st = np.zeros(p.shape)
    st[I.PHR] = f0
    st[I.PIR] = back[1] / am**2
    for j in range(3):
        st[I.AX + j] = A0[j]
        st[I.EX + j] = back[5 + j] * em**2
    nsteps = 500                              # tau 2.0 -> 2.5 across tau_s = 2.25
    st, _ = O.run(p, st, 0, nsteps)
    tau_end = p.tau0 + nsteps * p.dt
    mid = solve_ivp(rhs_for(p.s), (p.tau0, p.tau_s), y0, rtol=1e-12, atol=1e-14).y[:, -1]
    fin = solve_ivp(rhs_for(p.s_late), (p.tau_s, tau_end), mid, rtol=1e-12, atol=1e-14).y[:, -1]
    assert abs(st[I.PHR, 0, 0, 0] - fin[0]) < 2e-3
    for j in range(3):
        assert abs(st[I.AX + j, 0, 0, 0] - fin[2 + j]) < 2e-3
    # and the switch matters at this size: the constant-s solution is far away
    const = solve_ivp(rhs_for(p.s), (p.tau0, tau_end), y0, rtol=1e-12, atol=1e-14).y[:, -1]
    assert max(abs(const[2 + j] - fin[2 + j]) for j in range(3)) > 2e-2
