"""CPU pins of the light-cone helper that FP32 parity tests use to exclude
the links downstream of a flipped accept decision: a link perturbed before
a sweep changes, after the sweep, exactly the links the helper says the
sweep computes from it (checked with the FP64 oracle), and planted
mistakes in the dependence (a dropped backward term, a missing own link,
a wrong parity order) fail."""
import numpy as np
import pytest

import oracle as O
import lightcone as LC


def changed_links(group, dims, beta, sweep, site, mu, seed=3):
    o = O.Lattice(group, dims, beta, seed=seed, start=O.HOT)
    o.sweep(2, 2)
    links = o.get_links()
    a = O.Lattice(group, dims, beta, seed=seed + 2, start=O.COLD)
    b = O.Lattice(group, dims, beta, seed=seed + 2, start=O.COLD)
    a.set_links(links)
    pert = links.copy()
    pert[site, mu] *= 1 + 1e-7
    b.set_links(pert)
    a.sweep(*sweep)
    b.sweep(*sweep)
    return np.abs(a.get_links() - b.get_links()).max(axis=2) > 1e-13


@pytest.mark.parametrize("group,dims,beta,sweep,site,mu", [
    (2, (8, 8, 8, 8), 2.3, (0, 1), 1234, 2),
    (2, (8, 8, 8, 8), 2.3, (1, 0), 77, 0),
    (3, (8, 8, 4, 4), 5.7, (1, 1), 300, 3),
    (3, (6, 4, 4, 2), 5.7, (0, 1), 5, 1)])
def test_cone_equals_changed_links(group, dims, beta, sweep, site, mu):
    changed = changed_links(group, dims, beta, sweep, site, mu)
    init = np.zeros(changed.shape, bool)
    init[site, mu] = True
    cone = LC.downstream(dims, sweep[0], sweep[1], initial=init)
    assert not (changed & ~cone).any()           # nothing changes outside the cone
    assert (cone & ~changed).sum() <= 2          # and the cone is not larger than what changes
    assert 20 < cone.sum() < cone.size           # a real, partial cone


def test_flip_enters_at_its_own_pass():
    dims = (4, 4, 4, 4)
    V = 256
    flips = np.zeros((1, 4, V), bool)
    site = 0  # parity 0, updated in pass (mu = 2, parity 0)
    flips[0, 2, site] = True
    cone = LC.downstream(dims, 1, 0, flips=flips)
    assert cone[site, 2]
    # nothing of direction 0 or 1 depends on it (their passes come earlier)
    assert not cone[:, :2].any()
    # the opposite-parity links of direction 2 read it through the staple
    par = LC.parity(dims)
    assert cone[par == 1, 2].sum() == 6  # x +- nu for nu = 0, 1, 3


def test_planted_mistakes_fail():
    dims, sweep, site, mu = (8, 8, 4, 4), (1, 1), 300, 3
    changed = changed_links(3, dims, 5.7, sweep, site, mu)
    init = np.zeros(changed.shape, bool)
    init[site, mu] = True
    orig_shift = LC._shift

    def forward_only(d, m, s):  # dropped backward term: x - nu maps to x
        return orig_shift(d, m, s) if s > 0 else np.arange(int(np.prod(d)))
    LC._shift = forward_only
    try:
        cone = LC.downstream(dims, *sweep, initial=init)
    finally:
        LC._shift = orig_shift
    assert (changed & ~cone).any()
