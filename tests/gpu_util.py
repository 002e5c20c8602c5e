"""Helpers of the tests that compare the library with the oracle: move seeded
states in and out of the library's buffers, and cut a site's neighbourhood out
of a state for the oracle.  No GPU call is made by importing it."""
from __future__ import annotations

import numpy as np
import torch

import paper_1809_00995_amd as AH

GROUPS = {"phi": [0, 1], "pi": [2, 3], "a": [4, 5, 6], "e": [7, 8, 9]}


def oracle_params(O, p: "AH.Params"):
    return O.Params(p.nx, p.ny, p.nz, dx=p.dx, dt=p.dt, tau0=p.tau0, tau_ref=p.tau_ref,
                    era_p=p.era_p, s=p.s, lambda0=p.lambda0, e0=p.e0, sigma=p.sigma, seed=p.seed,
                    s_late=p.s_late, tau_s=p.tau_s)


def upload(p: "AH.Params", st: np.ndarray) -> torch.Tensor:
    """Planes tensor whose current copy (planes 0-9) holds st; p.init must be AH_INIT_NONE."""
    t = AH.alloc_planes(p)
    t.zero_()
    t[:10] = torch.from_numpy(np.ascontiguousarray(st)).to(device=t.device, dtype=t.dtype)
    return t


def fields_np(ctx: "AH.Context", r: int = 0) -> np.ndarray:
    torch.cuda.synchronize()
    return ctx.fields(r).double().cpu().numpy()


def group_errors(got: np.ndarray, ref: np.ndarray) -> dict:
    """Per field group: max |got - ref| / max |ref| (max-norm relative error)."""
    out = {}
    for g, idx in GROUPS.items():
        scale = np.abs(ref[idx]).max()
        diff = np.abs(got[idx] - ref[idx]).max()
        out[g] = diff / scale if scale > 0 else diff
    return out


def ambiguous_links(st: np.ndarray, tol: float = 1e-6) -> np.ndarray:
    """(3, nz, ny, nx) bool: links whose winding argument theta^{x+i} - theta^x + A_i lies
    within tol of +-pi (mod 2 pi), where the [.]_pi of Eq. (11) is decided by rounding."""
    th = np.arctan2(st[1], st[0])
    out = np.zeros((3,) + th.shape, dtype=bool)
    for i, axis in enumerate((2, 1, 0)):
        u = np.roll(th, -1, axis=axis) - th + st[4 + i]
        r = np.mod(u + np.pi, 2 * np.pi)          # in [0, 2 pi); pi is at 0 and 2 pi
        out[i] = np.minimum(r, 2 * np.pi - r) < tol
    return out


def plaquette_touches(amb: np.ndarray) -> np.ndarray:
    """(3, ...) bool: plaquettes xy, yz, zx at x having an ambiguous link among their four."""
    def sh(a, axis):
        return np.roll(a, -1, axis=axis)
    lx, ly, lz = amb
    xy = lx | ly | sh(ly, 2) | sh(lx, 1)
    yz = ly | lz | sh(lz, 1) | sh(ly, 0)
    zx = lz | lx | sh(lx, 0) | sh(lz, 2)
    return np.stack([xy, yz, zx])


def small_params(O, p, L):
    """The oracle's parameters of p on an L^3 periodic lattice."""
    return O.Params(L, L, L, dx=p.dx, dt=p.dt, tau0=p.tau0, tau_ref=p.tau_ref, era_p=p.era_p,
                    s=p.s, lambda0=p.lambda0, e0=p.e0, sigma=p.sigma, seed=p.seed,
                    s_late=p.s_late, tau_s=p.tau_s)


def neighbourhoods(F, xyz, r):
    """For each site (x, y, z) of xyz, the state within r sites of it (Chebyshev) and one
    more layer, as an L^3 periodic lattice with L = 2r + 2 and the site at (r, r, r):
    array (k, 10, L, L, L) in FP64.  A site's update depends on its neighbours and the
    other corners of its plaquettes only, so on this lattice the oracle advances the
    site by one step exactly as on the whole lattice for r = 1, and by two for r = 2."""
    ext = (F.shape[-1], F.shape[-2], F.shape[-3])      # nx, ny, nz
    off = torch.arange(-r, r + 2, device=F.device)
    t = torch.as_tensor(xyz, device=F.device)
    X, Y, Z = [(t[:, k, None] + off) % ext[k] for k in range(3)]
    g = F[:, Z[:, :, None, None], Y[:, None, :, None], X[:, None, None, :]]
    return g.permute(1, 0, 2, 3, 4).double().cpu().numpy()


def site_values(F, xyz):
    """(k, 10) FP64: the state at the given sites."""
    t = torch.as_tensor(xyz, device=F.device)
    return F[:, t[:, 2], t[:, 1], t[:, 0]].T.double().cpu().numpy()
