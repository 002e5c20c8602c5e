"""Seeded synthetic field states shared by the oracle tests and the GPU parity tests.

This module draws numbers and maps a state through a lattice gauge
transformation (a symmetry the tests check, not a step of the method): it holds
none of the method's arithmetic (no update, no diagnostic).  Arrays have shape (10, nz, ny, nx) in the plane order
phi_re, phi_im, Pi_re, Pi_im, A_x, A_y, A_z, E_x, E_y, E_z.
"""
from __future__ import annotations

import numpy as np

PHR, PHI, PIR, PII, AX, AY, AZ, EX, EY, EZ = range(10)


def random_state(n: int | tuple, seed: int, amp_phi=1.0, amp_pi=0.3, amp_a=0.4,
                 amp_e=0.3, dtype=np.float64) -> np.ndarray:
    """Generic non-trivial state: every field non-zero, uniform noise.

    phi has modulus in [0.5, 1.5] * amp_phi and a uniform phase; Pi, A, E are
    uniform in [-amp, amp].  Such a state does not satisfy Gauss's law, which
    makes it a sharper test of the update (the residual must be conserved
    site by site, not just stay zero).
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    rng = np.random.default_rng(seed)
    st = np.empty((10, nz, ny, nx), dtype=np.float64)
    mod = amp_phi * rng.uniform(0.5, 1.5, size=(nz, ny, nx))
    th = rng.uniform(-np.pi, np.pi, size=(nz, ny, nx))
    st[PHR] = mod * np.cos(th)
    st[PHI] = mod * np.sin(th)
    st[PIR:PII + 1] = rng.uniform(-amp_pi, amp_pi, size=(2, nz, ny, nx))
    st[AX:AZ + 1] = rng.uniform(-amp_a, amp_a, size=(3, nz, ny, nx))
    st[EX:EZ + 1] = rng.uniform(-amp_e, amp_e, size=(3, nz, ny, nx))
    return st.astype(dtype)


def smooth_state(n: int, seed: int, modes: int = 2, amp=0.3) -> np.ndarray:
    """Long-wavelength state: a few low Fourier modes per field around phi = 1.

    Used where a smooth solution is needed (time-step convergence).
    """
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    st = np.zeros((10, n, n, n))
    for f in range(10):
        acc = np.zeros((n, n, n))
        for _ in range(modes):
            k = rng.integers(-1, 2, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            acc += rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) / n + ph)
        st[f] = amp * acc / modes
    st[PHR] += 1.0
    return st


def gauge_transform(st: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """A state's image under the lattice gauge transformation alpha_x (the symmetry
    of Sec. 2): phi, Pi -> e^{i alpha} phi, e^{i alpha} Pi;  A_i -> A_i + alpha_x -
    alpha_{x+i};  E unchanged."""
    out = st.copy()
    c, s = np.cos(alpha), np.sin(alpha)
    for re, im in ((PHR, PHI), (PIR, PII)):
        out[re] = c * st[re] - s * st[im]
        out[im] = s * st[re] + c * st[im]
    for i, axis in enumerate((2, 1, 0)):          # x, y, z are array axes 2, 1, 0
        out[AX + i] = st[AX + i] + alpha - np.roll(alpha, -1, axis=axis)
    return out


def gauge_function(n: int | tuple, seed: int, amp=np.pi) -> np.ndarray:
    """Random lattice gauge function alpha_x, uniform in [-amp, amp]."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return np.random.default_rng(seed).uniform(-amp, amp, size=(nz, ny, nx))
