"""The sampled-site checks of the largest lattices hand the oracle each site's
neighbourhood on a small periodic lattice instead of the whole state
(tests/gpu_util.py: neighbourhoods).  This pins that reduction against the oracle
on a whole 16^3 lattice: one step on 4^3, two steps on 6^3 and the three
plaquette windings at the site on 4^3 equal the whole lattice's bit for bit,
at random sites and at the lattice's corners, where the neighbourhood wraps."""
import numpy as np
import torch

import oracle as O
import paper_1809_00995_amd as AH
from tests.gpu_util import neighbourhoods, site_values, small_params


def test_neighbourhood_lattices_reproduce_the_whole_lattice():
    n = 16
    p = AH.Params(n, n, n, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0, tau_ref=8.0,
                  era_p=1.0, s=1.0, seed=1025)
    op = small_params(O, p, n)
    st, _ = O.run(op, O.init_random_phase(op), 0, 30)
    F = torch.from_numpy(st)
    rng = np.random.default_rng(1)
    xyz = np.concatenate([rng.integers(0, n, size=(40, 3)),
                          [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 5]]])
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
