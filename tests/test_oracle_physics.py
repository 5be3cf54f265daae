"""Statistical pins of the oracle's Markov chain: the strong-coupling limit,
heat bath alone versus heat bath plus overrelaxation, and the removability
of the lambda_3 background by the Haar measure (the reading of the external
field adopted for the paper's "magnetic field flux" parameter)."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O


def binned_mean_err(x, nbins=10):
    x = np.asarray(x)
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


def su3_strong_coupling_u(beta, n=96):
    """<(1/3) Re Tr U> for the one-plaquette weight exp((beta/3) Re Tr U),
    by Weyl's integration formula over the SU(3) eigenvalue angles."""
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    z = [np.exp(1j * t1), np.exp(1j * t2), np.exp(-1j * (t1 + t2))]
    vd = np.abs((z[0] - z[1]) * (z[0] - z[2]) * (z[1] - z[2])) ** 2
    rt = (z[0] + z[1] + z[2]).real
    w = vd * np.exp(beta / 3 * rt)
    return float((w * rt / 3).sum() / w.sum())


def test_weyl_quadrature_leading_terms():
    # u(beta) = beta/18 + beta^2/216 + O(beta^3)
    b = 0.05
    assert su3_strong_coupling_u(b) == pytest.approx(b / 18 + b * b / 216, rel=1e-4)


def test_su2_strong_coupling():
    beta = 0.3
    L = O.Lattice(2, (8, 8, 8, 8), beta, seed=31, nhit=120, start=O.HOT)
    for _ in range(5):
        L.sweep(1, 0)
    ps = []
    for _ in range(300):
        L.sweep(1, 0)
        ps.append(L.measure()[0][0])
    m, e = binned_mean_err(ps, 20)
    u = special.iv(2, beta) / special.iv(1, beta)  # leading order; corrections O(u^5) ~ 1e-5
    assert abs(m - u) < 4 * e + 2e-5, (m, e, u)


def test_su3_strong_coupling():
    beta = 0.3
    L = O.Lattice(3, (6, 6, 6, 6), beta, seed=32, nhit=120, start=O.HOT)
    for _ in range(5):
        L.sweep(1, 0)
    ps = []
    for _ in range(400):
        L.sweep(1, 0)
        ps.append(L.measure()[0][0])
    m, e = binned_mean_err(ps, 20)
    u = su3_strong_coupling_u(beta)
    assert u == pytest.approx(0.0170829, abs=2e-7)
    assert abs(m - u) < 4 * e, (m, e, u)


@pytest.mark.parametrize("group,beta", [(2, 2.3), (3, 5.69)])
def test_heat_bath_and_overrelaxation_agree(group, beta):
    dims = (4, 4, 4, 4)
    a = O.Lattice(group, dims, beta, seed=41, start=O.HOT)
    b = O.Lattice(group, dims, beta, seed=42, start=O.HOT)
    for _ in range(20):
        a.sweep(1, 0)
        b.sweep(1, 3)
    pa, pb = [], []
    for _ in range(200 if group == 2 else 150):
        a.sweep(1, 0)
        b.sweep(1, 3)
        pa.append(a.measure()[0][0])
        pb.append(b.measure()[0][0])
    ma, ea = binned_mean_err(pa)
    mb, eb = binned_mean_err(pb)
    assert abs(ma - mb) < 4 * math.hypot(ea, eb), (ma, ea, mb, eb)


def test_flux_is_removable_in_equilibrium():
    # U -> U B is a change of variables under the Haar measure: the
    # equilibrium plaquette cannot depend on the number of flux quanta.
    dims = (4, 4, 4, 4)
    res = []
    for n in (0, 3):
        L = O.Lattice(2, dims, 2.3, flux=n, seed=50 + n, start=O.HOT)
        for _ in range(20):
            L.sweep(1, 1)
        ps = []
        for _ in range(200):
            L.sweep(1, 1)
            ps.append(L.measure()[0][0])
        res.append(binned_mean_err(ps))
    (m0, e0), (m1, e1) = res
    assert abs(m0 - m1) < 4 * math.hypot(e0, e1)
