"""Pins of the oracle's lattice-level steps: initial configurations, the
background flux, unitarity, gauge invariance, overrelaxation invariants and
the staple's plaquette bookkeeping.

The paper prints no physics values, so every pin here is a closed form, an
exact distribution or an invariant that the mathematics fixes."""
import math

import numpy as np
import pytest

import oracle as O
from helpers import (det_error, gauge_transform, haar_su, plaquette_numpy, polyakov_numpy,
                     to_matrices, from_matrices, unitarity_error)


@pytest.mark.parametrize("group", [2, 3])
def test_cold_start_is_unity(group):
    L = O.Lattice(group, (4, 4, 4, 6), 2.3, start=O.COLD)
    p, l = L.measure()
    assert np.all(p == 1.0) and l[0] == 1.0 and l[1] == 0.0


@pytest.mark.parametrize("group,dims,n", [(2, (8, 6, 4, 4), 1), (3, (8, 6, 4, 4), 3),
                                          (3, (32, 32, 4, 2), 4)])
def test_cold_start_flux_closed_form(group, dims, n):
    # every x-y plaquette carries exp(i phi T), phi = 2 pi n / (Nx Ny)
    L = O.Lattice(group, dims, 5.9, flux=n, start=O.COLD)
    p, l = L.measure()
    phi = 2 * math.pi * n / (dims[0] * dims[1])
    pxy = math.cos(phi) if group == 2 else (1 + 2 * math.cos(phi)) / 3
    assert p[1] == pytest.approx((2 + pxy) / 3, abs=1e-14)
    assert p[2] == pytest.approx(1.0, abs=1e-14)
    assert p[0] == pytest.approx((5 + pxy) / 6, abs=1e-14)
    assert l[0] == pytest.approx(1.0, abs=1e-14) and abs(l[1]) < 1e-14


def test_flux_32x8_n4_value():
    # 32^3x8, n = 4: P_xy = (1 + 2 cos(2 pi 4/1024))/3
    L = O.Lattice(3, (32, 32, 2, 2), 5.9, flux=4, start=O.COLD)
    p, _ = L.measure()
    pxy = 3 * p[1] - 2
    assert pxy == pytest.approx(0.99979921246, abs=1e-11)


@pytest.mark.parametrize("group", [2, 3])
def test_hot_start_haar_moments(group):
    L = O.Lattice(group, (8, 8, 8, 8), 5.0, start=O.HOT, seed=7)
    m = to_matrices(L.get_links(), group).reshape(-1, group, group)
    tr = np.trace(m, axis1=-2, axis2=-1)
    n = len(tr)
    assert unitarity_error(m) < 1e-14 and det_error(m) < 1e-14
    assert abs(tr.mean()) < 5 / math.sqrt(n)
    assert abs((np.abs(tr) ** 2).mean() - 1.0) < 5 * math.sqrt(1.0 / n) * 1.5
    p, l = L.measure()
    assert abs(p[0]) < 5 * 0.5 / math.sqrt(6 * L.V)
    assert abs(l[0]) < 5 / math.sqrt(L.V / 8)


@pytest.mark.parametrize("group,rng", [(2, O.RNG_MRG32K3A), (3, O.RNG_PHILOX), (3, O.RNG_MRG32K3A)])
def test_unitarity_after_sweeps(group, rng):
    L = O.Lattice(group, (4, 4, 4, 4), 2.3 if group == 2 else 5.7, rng=rng, seed=3, start=O.HOT)
    L.sweep(2, 3)
    m = to_matrices(L.get_links(), group)
    assert unitarity_error(m) < 1e-13 and det_error(m) < 1e-13


@pytest.mark.parametrize("group,flux", [(2, 0), (3, 0), (3, 2)])
def test_gauge_invariance(group, flux):
    dims = (4, 4, 4, 6)
    L = O.Lattice(group, dims, 5.7, flux=flux, seed=5, start=O.HOT)
    L.sweep(1, 1)
    p0, l0 = L.measure()
    links = to_matrices(L.get_links(), group)
    g = haar_su(group, L.V, np.random.default_rng(9))
    L.set_links(from_matrices(gauge_transform(links, g, dims), group))
    p1, l1 = L.measure()
    assert np.abs(p1 - p0).max() < 1e-13
    assert np.abs(l1 - l0).max() < 1e-13


@pytest.mark.parametrize("group", [2, 3])
def test_measure_matches_independent_numpy(group):
    dims = (4, 6, 4, 4)
    L = O.Lattice(group, dims, 5.7, flux=1, seed=2, start=O.HOT)
    L.sweep(1, 0)
    m = to_matrices(L.get_links(), group)
    p, l = L.measure()
    assert np.abs(p - plaquette_numpy(m, dims)).max() < 1e-13
    assert np.abs(l - polyakov_numpy(m, dims)).max() < 1e-13


@pytest.mark.parametrize("group,flux", [(2, 0), (3, 0), (3, 1)])
def test_staple_counts_every_plaquette_four_times(group, flux):
    # sum over links of Re Tr(W A) = 4 * N * 6V * <P>: each plaquette is
    # reached once from each of its four links.
    dims = (4, 4, 2, 4)
    L = O.Lattice(group, dims, 5.7, flux=flux, seed=8, start=O.HOT)
    L.sweep(1, 0)
    m = to_matrices(L.get_links(), group)
    s = 0.0
    for i in range(L.V):
        for mu in range(4):
            s += np.trace(m[i, mu] @ L.staple(i, mu)).real
    p, _ = L.measure()
    assert s == pytest.approx(4 * group * 6 * L.V * p[0], abs=1e-10)


@pytest.mark.parametrize("group", [2, 3])
def test_overrelaxation_invariants_single_link(group):
    rng = np.random.default_rng(21)
    U = haar_su(group, 1, rng)[0]
    A = sum(haar_su(group, 6, rng))
    Uc = from_matrices(U, group)
    U1, used = O.update_link(group, 5.0, 10, 1, 0, Uc, A, None)
    assert used == 0
    U2, _ = O.update_link(group, 5.0, 10, 1, 0, U1, A, None)
    m1 = to_matrices(U1, group)
    before = np.trace(U @ A).real
    after = np.trace(m1 @ A).real
    assert abs(after - before) <= 1e-14 * abs(before) + 1e-14
    if group == 2:
        assert np.abs(U2 - Uc).max() < 1e-14  # a reflection: OR o OR = identity
    assert not np.allclose(U1, Uc)


@pytest.mark.parametrize("group,flux", [(2, 0), (3, 0), (3, 2)])
def test_overrelaxation_sweep_keeps_action(group, flux):
    L = O.Lattice(group, (4, 4, 4, 4), 5.7, flux=flux, seed=11, start=O.HOT)
    L.sweep(2, 0)
    p0, _ = L.measure()
    before = L.get_links()
    L.sweep(0, 3)
    p1, _ = L.measure()
    assert abs(p1[0] - p0[0]) < 1e-13
    assert np.abs(L.get_links() - before).max() > 1e-2  # links did move


def test_reunitarisation_idempotent_and_projects():
    rng = np.random.default_rng(2)
    U = haar_su(3, 1, rng)[0] + 1e-6 * (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
    Uc = from_matrices(U, 3)
    zero = np.zeros((3, 3))
    # overrelaxation with a zero staple leaves the link; reunit = 1 projects it
    R1, _ = O.update_link(3, 1.0, 10, 1, 1, Uc, zero, None)
    R2, _ = O.update_link(3, 1.0, 10, 1, 1, R1, zero, None)
    m = to_matrices(R1, 3)
    assert unitarity_error(m) < 1e-15 * 10 and det_error(m) < 1e-14
    assert np.abs(R2 - R1).max() < 1e-15 * 10
    assert np.abs(R1 - Uc).max() < 1e-5


def test_set_get_links_roundtrip_with_flux():
    L = O.Lattice(3, (4, 4, 2, 2), 5.7, flux=3, seed=1, start=O.HOT)
    a = L.get_links()
    L.set_links(a)
    assert np.abs(L.get_links() - a).max() < 1e-14


def test_invalid_parameters_rejected():
    for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 4, 1)]:
        with pytest.raises(ValueError):
            O.Lattice(3, dims, 5.7)
    with pytest.raises(ValueError):
        O.Lattice(4, (4, 4, 4, 4), 5.7)
    with pytest.raises(ValueError):
        O.Lattice(3, (4, 4, 4, 4), -1.0)


def test_philox_sweep_is_thread_count_independent():
    a = O.Lattice(3, (4, 4, 4, 4), 5.7, seed=3, start=O.HOT)
    b = O.Lattice(3, (4, 4, 4, 4), 5.7, seed=3, start=O.HOT)
    n = O.get_threads()
    O.set_threads(1)
    a.sweep(1, 2)
    O.set_threads(max(2, n))
    b.sweep(1, 2)
    O.set_threads(n)
    assert np.array_equal(a.get_links(), b.get_links())
