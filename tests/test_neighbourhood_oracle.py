"""The sampled-site checks of the largest lattices hand the oracle each site's
neighbourhood on a small periodic lattice instead of the whole state
(tests/gpu_util.py: neighbourhoods).  This pins that reduction against the oracle
on whole 16^3 and 16 x 12 x 10 lattices: one step on 4^3, two steps on 6^3 and
the three plaquette windings at the site on 4^3 equal the whole lattice's bit for
bit, at random sites and at the lattice's corners, where the neighbourhood wraps
(each axis by its own extent)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1809_00995_amd as AH
from tests.gpu_util import neighbourhoods, site_values, small_params


@pytest.mark.parametrize("shape", [(16, 16, 16), (16, 12, 10)])
def test_neighbourhood_lattices_reproduce_the_whole_lattice(shape):
    nx, ny, nz = shape
    p = AH.Params(nx, ny, nz, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0, tau_ref=8.0,
                  era_p=1.0, s=1.0, seed=1025)
    op = O.Params(nx, ny, nz, dx=p.dx, dt=p.dt, tau0=p.tau0, tau_ref=p.tau_ref,
                  era_p=p.era_p, s=p.s, seed=p.seed)
    st, _ = O.run(op, O.init_random_phase(op), 0, 30)
    F = torch.from_numpy(st)
    rng = np.random.default_rng(1)
    xyz = np.concatenate([np.stack([rng.integers(0, e, size=40) for e in shape], axis=1),
                          [[0, 0, 0], [nx - 1, ny - 1, nz - 1], [0, ny - 1, 5]]])
    s31 = O.step(op, 30, st)
    s32 = O.step(op, 31, s31)
    sp4, sp6 = small_params(O, p, 4), small_params(O, p, 6)
    nb1, nb2 = neighbourhoods(F, xyz, 1), neighbourhoods(F, xyz, 2)
    mid4, mid6 = 1 + 4 * (1 + 4 * 1), 2 + 6 * (2 + 6 * 2)
    one = np.stack([O.step_sites(sp4, 30, nb1[k], [mid4])[0] for k in range(len(xyz))])
    two = np.stack([O.step_sites(sp6, 31, O.step(sp6, 30, nb2[k]), [mid6])[0]
                    for k in range(len(xyz))])
    assert np.array_equal(one, site_values(torch.from_numpy(s31), xyz))
    assert np.array_equal(two, site_values(torch.from_numpy(s32), xyz))
    wind = O.measure(op, 30, st, wind_map=True).wind
    ref = np.stack([wind[:, z, y, x] for x, y, z in xyz])
    got = np.stack([O.measure(sp4, 30, nb1[k], wind_map=True).wind[:, 1, 1, 1]
                    for k in range(len(xyz))])
    assert np.array_equal(got, ref)
    assert np.abs(ref).sum() > 0       # the sample holds strings
