"""Frozen external field in the oracle: with frozen = 1 the spatial links of
the time slice t = 0 are held at the background W = B (U = 1) and never
updated, which makes the lambda_3 background of the paper's external-field
simulations (Sec. 1, the flux of Sec. 3.2) impossible to remove by a change
of variables (a reading; the paper names the field only by its flux)."""
import math

import numpy as np
import pytest

import oracle as O
from helpers import neighbour, to_matrices


def plane_traces(links, group, dims, mu, nu):
    """(1/N) Re Tr P_{mu nu}(x) at every site, from W-frame links."""
    m = to_matrices(links, group).reshape(-1, 4, group, group)
    a = m[:, mu]
    b = m[neighbour(dims, mu), nu]
    c = np.conj(np.swapaxes(m[neighbour(dims, nu), mu], -1, -2))
    d = np.conj(np.swapaxes(m[:, nu], -1, -2))
    return np.trace(a @ b @ c @ d, axis1=-2, axis2=-1).real / group


def time_slice(dims):
    nx, ny, nz, nt = dims
    return np.arange(nx * ny * nz * nt) // (nx * ny * nz)  # canonical order: t outermost


@pytest.mark.parametrize("group,n,rng", [(2, 3, O.RNG_MRG32K3A), (3, 2, O.RNG_PHILOX)])
def test_frozen_slice_keeps_the_background(group, n, rng):
    dims = (6, 4, 4, 4)
    beta = 2.3 if group == 2 else 5.7
    background = O.Lattice(group, dims, beta, flux=n, start=O.COLD).get_links()  # W = B everywhere
    L = O.Lattice(group, dims, beta, flux=n, rng=rng, seed=5, start=O.HOT, frozen=1)
    L.sweep(2, 3)
    L.sweep(1, 2)
    w = L.get_links()
    t0 = time_slice(dims) == 0
    assert np.array_equal(w[t0, :3], background[t0, :3])      # held exactly
    assert np.abs(w[t0, 3] - background[t0, 3]).max() > 0.1     # temporal links at t = 0 move
    assert np.abs(w[~t0, :3] - background[~t0, :3]).max() > 0.1
    # so every x-y plaquette of the slice t = 0 keeps its closed form
    phi = 2 * math.pi * n / (dims[0] * dims[1])
    pxy = math.cos(phi) if group == 2 else (1 + 2 * math.cos(phi)) / 3
    assert np.abs(plane_traces(w, group, dims, 0, 1)[t0] - pxy).max() < 1e-13


def test_frozen_field_is_not_removable():
    """Without frozen links the flux is a change of variables and the
    equilibrium plaquette does not depend on it; with the slice t = 0 frozen
    the dynamical spatial plaquettes (t != 0) feel it: SU(2) 4^4, beta 2.3,
    n = 0 against n = 8 (half a flux quantum per x-y plaquette, cos phi = -1
    on the frozen slice), 150 measured (1 HB + 2 OR) sweeps each."""
    dims = (4, 4, 4, 4)
    t = time_slice(dims)

    def dynamical_ps(n):
        L = O.Lattice(2, dims, 2.3, flux=n, seed=3, start=O.COLD, frozen=1)
        xs = []
        for k in range(200):
            L.sweep(1, 2)
            if k >= 50:
                w = L.get_links()
                xs.append(np.mean([plane_traces(w, 2, dims, mu, nu)[t != 0].mean()
                                   for mu, nu in ((0, 1), (0, 2), (1, 2))]))
        b = np.array(xs).reshape(10, -1).mean(axis=1)
        return b.mean(), b.std(ddof=1) / math.sqrt(10)

    (m0, e0), (m8, e8) = dynamical_ps(0), dynamical_ps(8)
    assert m0 - m8 > 8 * math.hypot(e0, e8), (m0, e0, m8, e8)


def test_frozen_rejects_unknown_mode():
    with pytest.raises(ValueError):
        O.Lattice(3, (4, 4, 4, 4), 5.7, frozen=2)
