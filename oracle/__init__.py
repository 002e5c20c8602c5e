"""Plain FP64 CPU oracle for the Abelian-Higgs lattice leapfrog (arXiv:1809.00995, Sec. 2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls it and it never calls the HIP library.

The arithmetic lives in ``ah_oracle.c`` (plain C, FP64); this module only
marshals numpy arrays of shape ``(10, nz, ny, nx)`` in the plane order
``phi_re, phi_im, Pi_re, Pi_im, A_x, A_y, A_z, E_x, E_y, E_z``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

FIELDS = ("phi_re", "phi_im", "pi_re", "pi_im", "ax", "ay", "az", "ex", "ey", "ez")


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double),
                ("tau0", C.c_double), ("tau_ref", C.c_double),
                ("era_p", C.c_double), ("s", C.c_double),
                ("lambda0", C.c_double), ("e0", C.c_double), ("sigma", C.c_double),
                ("seed", C.c_uint64), ("s_late", C.c_double), ("tau_s", C.c_double)]


class _Coeffs(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("tau", "a_m", "a_0", "a_p", "c1", "c2", "c3", "d1", "d2", "d3")]


class _Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("tau", C.c_double), ("a", C.c_double),
                ("n_wind", C.c_int64), ("n_wind_dir", C.c_int64 * 3),
                ("net_wind_dir", C.c_int64 * 3), ("n_pierced", C.c_int64),
                ("length", C.c_double), ("xi_w", C.c_double),
                ("sum_lag", C.c_double), ("xi_l", C.c_double),
                ("num", C.c_double * 3), ("den", C.c_double * 3), ("v2", C.c_double * 3),
                ("kin", C.c_double), ("grad", C.c_double), ("elec", C.c_double),
                ("mag", C.c_double), ("pot", C.c_double), ("energy", C.c_double),
                ("pres", C.c_double), ("pres_lag", C.c_double), ("rho_lag", C.c_double),
                ("v2_eos", C.c_double), ("nonfinite", C.c_int64)]


@dataclass
class Params:
    """Problem statement of Sec. 2: lattice, spacings, era, s and couplings."""
    nx: int
    ny: int
    nz: int
    dx: float = 0.5
    dt: float = 0.1
    tau0: float = 0.0
    tau_ref: float = 1.0
    era_p: float = 1.0
    s: float = 1.0
    lambda0: float = 2.0
    e0: float = 1.0
    sigma: float = 1.0
    seed: int = 1
    s_late: float = 1.0
    tau_s: float = 0.0

    def _c(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.dx, self.dt, self.tau0,
                       self.tau_ref, self.era_p, self.s, self.lambda0, self.e0,
                       self.sigma, self.seed & 0xFFFFFFFFFFFFFFFF, self.s_late, self.tau_s)

    @property
    def shape(self):
        return (10, self.nz, self.ny, self.nx)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = C.CDLL(_build.LIB)
        P, D = C.POINTER, C.POINTER(C.c_double)
        lib.or_scale_factor.restype = C.c_double
        lib.or_scale_factor.argtypes = [P(_Params), C.c_double]
        lib.or_coefficients.argtypes = [P(_Params), C.c_int64, P(_Coeffs)]
        lib.or_splitmix64.restype = C.c_uint64
        lib.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        lib.or_init_random_phase.argtypes = [P(_Params), D]
        lib.or_step.argtypes = [P(_Params), C.c_int64, D, D]
        lib.or_measure.argtypes = [P(_Params), C.c_int64, D, P(_Obs), C.c_void_p]
        lib.or_gauss.argtypes = [P(_Params), C.c_int64, D, D, D, C.c_void_p]
        lib.or_threads.restype = C.c_int
        lib.or_step_sites.argtypes = [P(_Params), C.c_int64, D, C.c_int64, C.c_void_p, D]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _state(p: Params, st) -> np.ndarray:
    st = np.ascontiguousarray(st, dtype=np.float64)
    if st.shape != p.shape:
        raise ValueError(f"state shape {st.shape} != {p.shape}")
    return st


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().or_threads())


def scale_factor(p: Params, tau: float) -> float:
    return _load().or_scale_factor(C.byref(p._c()), tau)


def coefficients(p: Params, n: int) -> dict:
    c = _Coeffs()
    _load().or_coefficients(C.byref(p._c()), n, C.byref(c))
    return {k: getattr(c, k) for k, _ in _Coeffs._fields_}


def splitmix64(seed: int, k: int) -> int:
    return int(_load().or_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, k))


def init_random_phase(p: Params) -> np.ndarray:
    st = np.empty(p.shape, dtype=np.float64)
    _load().or_init_random_phase(C.byref(p._c()), _dptr(st))
    return st


def vacuum(p: Params) -> np.ndarray:
    st = np.zeros(p.shape, dtype=np.float64)
    st[0] = p.sigma
    return st


def step(p: Params, n: int, st) -> np.ndarray:
    """S_n -> S_{n+1}."""
    st = _state(p, st)
    out = np.empty_like(st)
    _load().or_step(C.byref(p._c()), n, _dptr(st), _dptr(out))
    return out


def step_sites(p: Params, n: int, st, idx) -> np.ndarray:
    """S_{n+1} at the given flat site indices only: array (len(idx), 10)."""
    st = _state(p, st)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 10), dtype=np.float64)
    _load().or_step_sites(C.byref(p._c()), n, _dptr(st), idx.size, idx.ctypes.data, _dptr(out))
    return out


def run(p: Params, st, n0: int, nsteps: int, measure_every: int = 0):
    """Advance nsteps from S_{n0}; optionally measure S_n whenever n % k == 0."""
    st = _state(p, st)
    obs = []
    for n in range(n0, n0 + nsteps):
        if measure_every and n % measure_every == 0:
            obs.append(measure(p, n, st))
        st = step(p, n, st)
    return st, obs


@dataclass
class Obs:
    step: int
    tau: float
    a: float
    n_wind: int
    n_wind_dir: list
    net_wind_dir: list
    n_pierced: int
    length: float
    xi_w: float
    sum_lag: float
    xi_l: float
    num: list
    den: list
    v2: list
    kin: float
    grad: float
    elec: float
    mag: float
    pot: float
    energy: float
    pres: float
    pres_lag: float
    rho_lag: float
    v2_eos: float
    nonfinite: int
    wind: np.ndarray | None = field(default=None, repr=False)


def measure(p: Params, n: int, st, wind_map: bool = False) -> Obs:
    st = _state(p, st)
    o = _Obs()
    wm = np.zeros((3, p.nz, p.ny, p.nx), dtype=np.int8) if wind_map else None
    _load().or_measure(C.byref(p._c()), n, _dptr(st), C.byref(o),
                       wm.ctypes.data if wm is not None else None)
    d = {}
    for k, _ in _Obs._fields_:
        v = getattr(o, k)
        d[k] = list(v) if not isinstance(v, (int, float)) else v
    return Obs(wind=wm, **d)


def gauss(p: Params, n: int, st, site_map: bool = False):
    """Gauss-law residual of S_n: (max |G|, rms G[, per-site map])."""
    st = _state(p, st)
    mx, rms = C.c_double(), C.c_double()
    gm = np.zeros((p.nz, p.ny, p.nx), dtype=np.float64) if site_map else None
    _load().or_gauss(C.byref(p._c()), n, _dptr(st), C.byref(mx), C.byref(rms),
                     gm.ctypes.data if gm is not None else None)
    if site_map:
        return mx.value, rms.value, gm
    return mx.value, rms.value
