"""Pins of the oracle's O(N) phi^4 model (the paper's second model family,
Sec. 3.3 and 5), none of which re-types the oracle's arithmetic:

* worked examples with the constant generator, derived by hand;
* kappa = 0: sites decouple and each samples the one-site density
  exp(-phi^2 - lambda (phi^2-1)^2 + h phi_0) on R^N, whose moments come from
  an independent quadrature;
* lambda = 0: the free (Gaussian) lattice field, whose propagator
  1 / (2 (1 - 2 kappa sum_mu cos p_mu)) on the finite periodic lattice gives
  <phi^2> and the nearest-neighbour product exactly (a wrong neighbour index
  or a wrong factor of kappa fails it); an anisotropic lattice with an
  extent of 2 checks the neighbour structure;
* the RANLUX block rule against the raw generator output;
* the hot start's uniform distribution."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O


def binned(x, nbins=20):
    x = np.asarray(x)
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


def series(f, nsweeps, ntherm):
    f.sweep(ntherm)
    out = []
    for _ in range(nsweeps):
        f.sweep(1)
        out.append(f.measure())
    return np.array(out)


# ---- worked examples (constant generator) ----------------------------------

@pytest.mark.parametrize("nhit", [5, 10, 100])
def test_constant_generator_walk_n4(nhit):
    """kappa = lambda = h = 0, delta = 1/2, every uniform 1/4: each hit
    proposes phi - 1/4 (1,1,1,1).  From the cold start the k-th step changes
    phi^2 by (2k-1)/4; exp(-(2k-1)/4) exceeds 1/4 for k <= 3 only, so four
    hits are accepted and every site ends at (0, -1, -1, -1)."""
    f = O.ONField(4, (4, 4, 2, 2), 0.0, 0.0, 0.0, 0.5, rng=O.RNG_CONST, rng_const=0.25, nhit=nhit,
                  start=O.COLD)
    f.sweep(1)
    assert np.array_equal(f.get_field(), np.tile([0.0, -1.0, -1.0, -1.0], (f.V, 1)))
    assert f.acceptance() == pytest.approx(4 / nhit, abs=0)


def test_constant_generator_walk_n1():
    """N = 1, same setting: step k changes phi^2 by (2k-7)/16, and
    exp(-(2k-7)/16) > 1/4 holds up to k = 14: fifteen accepted hits take phi
    from 1 to 1 - 15/4."""
    f = O.ONField(1, (2, 2, 2, 2), 0.0, 0.0, 0.0, 0.5, rng=O.RNG_CONST, rng_const=0.25, nhit=100,
                  start=O.COLD)
    f.sweep(1)
    assert np.array_equal(f.get_field(), np.full((16, 1), -2.75))
    assert f.acceptance() == 0.15


def test_constant_generator_source_and_coupling():
    """kappa and h enter with the signs and factors of the action.  N = 2,
    cold start, lambda = 0, kappa = 1/16, h = 1/2, delta = 1/2, uniforms 3/4:
    each hit proposes phi + (1/4, 1/4).  Parity 0 (all 8 neighbours (1,0)):
    s = phi^2 - (3/2) phi_0, so (1,0) -> (5/4,1/4) changes s by 1/4 and
    exp(-1/4) = 0.779 > 3/4 accepts it; the next step changes s by 1/2 and is
    rejected (exp(-1/2) = 0.607).  Parity 1 then sees neighbours (5/4,1/4):
    s = phi^2 - (7/4) phi_0 - (1/4) phi_1, steps of 1/8 (accepted) and 3/8
    (rejected).  A flipped sign of kappa or h, a dropped factor 2 or only
    forward neighbours would each reject the first step."""
    f = O.ONField(2, (2, 2, 2, 2), 1 / 16, 0.0, 0.5, 0.5, rng=O.RNG_CONST, rng_const=0.75, nhit=3,
                  start=O.COLD)
    f.sweep(1)
    assert np.array_equal(f.get_field(), np.tile([1.25, 0.25], (16, 1)))
    assert f.acceptance() == pytest.approx(1 / 3, abs=1e-15)


@pytest.mark.parametrize("nhit", [11, 40])
def test_constant_generator_quartic_term(nhit):
    """N = 1, kappa = h = 0, lambda = 1/4, delta = 1/2, uniforms 1/4: steps of
    -1/4 from phi = 1 change s = phi^2 + (phi^2-1)^2/4 by -0.390, -0.220,
    -0.108, -0.032, 0.032, 0.108, 0.220, 0.390, 0.642, 0.999 (all accepted:
    exp(-0.999) = 0.368 > 1/4) and then 1.485 (exp = 0.226, rejected): phi
    stops at -3/2 after ten hits, where lambda = 0 would reach -11/4."""
    f = O.ONField(1, (2, 2, 2, 4), 0.0, 0.25, 0.0, 0.5, rng=O.RNG_CONST, rng_const=0.25, nhit=nhit,
                  start=O.COLD)
    f.sweep(1)
    assert np.array_equal(f.get_field(), np.full((32, 1), -1.5))
    assert f.acceptance() == pytest.approx(10 / nhit, abs=1e-15)


# ---- kappa = 0: one-site density ---------------------------------------------

def one_site_moments(n, lam, h):
    """<phi^2>, <(phi^2-1)^2>, <phi_0> for the density
    exp(-r^2 - lam (r^2-1)^2 + h r cos(theta)) on R^n."""
    def w(r, th):
        return math.exp(-r * r - lam * (r * r - 1) ** 2 + h * r * math.cos(th))

    if n == 1:
        def m(f):
            return integrate.quad(lambda x: f(x * x, x) * math.exp(-x * x - lam * (x * x - 1) ** 2 + h * x),
                                  -8, 8, limit=200)[0]
    else:
        def m(f):
            return integrate.dblquad(
                lambda th, r: f(r * r, r * math.cos(th)) * r ** (n - 1) * math.sin(th) ** (n - 2) * w(r, th),
                0, 8, 0, math.pi)[0]
    z = m(lambda r2, x0: 1.0)
    return (m(lambda r2, x0: r2) / z, m(lambda r2, x0: (r2 - 1) ** 2) / z, m(lambda r2, x0: x0) / z)


def test_quadrature_gaussian_limit():
    # lam = 0, h = 0: phi_a ~ N(0, 1/2) so <phi^2> = n/2 and <(phi^2-1)^2> = n/2 + (n/2-1)^2
    for n in (1, 2, 4):
        p2, q, m0 = one_site_moments(n, 0.0, 0.0)
        assert p2 == pytest.approx(n / 2, rel=1e-6)
        assert q == pytest.approx(n / 2 + (n / 2 - 1) ** 2, rel=1e-6)
        assert abs(m0) < 1e-9


@pytest.mark.parametrize("n,lam,h,rng", [(4, 0.5, 0.3, O.RNG_PHILOX), (1, 1.0, 0.4, O.RNG_PHILOX),
                                         (2, 0.2, 0.0, O.RNG_PHILOX), (3, 0.7, 0.5, O.RNG_RANLUX),
                                         (4, 0.3, 0.2, O.RNG_MRG32K3A)])
def test_decoupled_sites_sample_the_one_site_density(n, lam, h, rng):
    f = O.ONField(n, (4, 4, 4, 4), 0.0, lam, h, 1.4, rng=rng, seed=17, nhit=6, start=O.HOT)
    s = series(f, 3000, 50)
    p2, q, m0 = one_site_moments(n, lam, h)
    for col, want in ((0, p2), (2, q), (3, m0)):
        got, err = binned(s[:, col])
        assert abs(got - want) < 4.5 * err + 1e-4, (col, got, want, err)
    assert np.all(s[:, 4 + (n - 1):] == 0.0) or n == 4


# ---- lambda = 0: free field ----------------------------------------------------

def free_field(dims, n, kappa, h):
    ps = np.meshgrid(*[2 * np.pi * np.arange(L) / L for L in dims], indexing="ij")
    cos = sum(np.cos(p) for p in ps)
    g = 1.0 / (2.0 * (1.0 - 2.0 * kappa * cos))
    m = h / (2.0 * (1.0 - 8.0 * kappa))
    phi2 = n * g.mean() + m * m
    link = n * (g * cos / 4.0).mean() + m * m
    return phi2, link, m


@pytest.mark.parametrize("dims,n,kappa,h", [((4, 4, 4, 4), 4, 0.1, 0.0), ((4, 2, 6, 4), 2, 0.1, 0.2),
                                             ((6, 4, 2, 2), 1, 0.08, -0.3)])
def test_free_field_propagator(dims, n, kappa, h):
    f = O.ONField(n, dims, kappa, 0.0, h, 1.3, seed=5, nhit=8, start=O.HOT)
    s = series(f, 4000, 200)
    phi2, link, m = free_field(dims, n, kappa, h)
    for col, want in ((0, phi2), (1, link), (3, m)):
        got, err = binned(s[:, col])
        assert abs(got - want) < 4.5 * err + 1e-4, (col, got, want, err)


def test_free_field_formula_reduces_to_one_site():
    # kappa = 0: every mode has G = 1/2, so <phi^2> = n/2 and no link correlation
    phi2, link, m = free_field((4, 4, 4, 4), 3, 0.0, 0.0)
    assert phi2 == pytest.approx(1.5) and abs(link) < 1e-15 and m == 0


# ---- generators and starts ------------------------------------------------------

def test_ranlux_block_rule():
    """Hot start takes the first N values of a site's first block; the
    sweep's update of that site begins the next block: N values for the
    proposal, then the acceptance value."""
    n, seed = 3, 9
    f = O.ONField(n, (2, 2, 2, 2), 0.0, 0.0, 0.0, 0.8, rng=O.RNG_RANLUX, seed=seed, nhit=1, start=O.HOT)
    phi0 = f.get_field().copy()
    f.sweep(1)
    phi1 = f.get_field()
    for i in range(16):
        raw = O.ranlux_raw(O.ranlux_site_seed(seed, i), 48)
        u = (raw.astype(np.float64) + 0.5) / 2 ** 24
        assert np.array_equal(phi0[i], 2 * u[:n] - 1)
        trial = phi0[i] + 0.8 * (2 * u[24:24 + n] - 1)
        accept = u[24 + n] < math.exp(-(trial @ trial - phi0[i] @ phi0[i]))
        assert np.array_equal(phi1[i], trial if accept else phi0[i])


def test_mrg_stream_layout():
    """MRG32k3a: each site draws sequentially from its own stream (2^127
    apart): the hot start takes N values, each hit N then the acceptance
    value; reproduced from the raw generator at kappa = lambda = h = 0."""
    seed, n, nhit = 77, 3, 2
    f = O.ONField(n, (2, 2, 2, 2), 0.0, 0.0, 0.0, 0.7, rng=O.RNG_MRG32K3A, seed=seed, nhit=nhit, start=O.HOT)
    phi0 = f.get_field().copy()
    f.sweep(1)
    phi1 = f.get_field()
    for i in range(16):
        st = O.mrg_site_state(seed, i)
        u = [O.uniform24(O.mrg_next(st)) for _ in range(n + nhit * (n + 1))]
        cur = 2 * np.array(u[:n]) - 1
        assert np.array_equal(phi0[i], cur)
        for k in range(nhit):
            r = np.array(u[n + k * (n + 1): n + k * (n + 1) + n])
            trial = cur + 0.7 * (2 * r - 1)
            if u[n + k * (n + 1) + n] < math.exp(-(trial @ trial - cur @ cur)):
                cur = trial
        assert np.allclose(phi1[i], cur, rtol=0, atol=1e-15)
        assert np.array_equal(f.mrg_states()[i], st)


def test_hot_start_is_uniform_in_the_cube():
    f = O.ONField(4, (8, 8, 8, 8), 0.3, 1.0, start=O.HOT, seed=3)
    phi = f.get_field()
    assert np.all(np.abs(phi) < 1)
    assert abs(phi.mean()) < 0.01 and phi.var() == pytest.approx(1 / 3, rel=0.02)


def test_philox_counter_layout():
    """Hit k of sweep w at site i uses Philox(i, lattice_id, w, k): one hit
    per sweep at kappa = lambda = h = 0 is reproduced from the raw generator."""
    seed, lid, n = 0x1234_5678_9ABC, 7, 4
    f = O.ONField(n, (2, 2, 2, 2), 0.0, 0.0, 0.0, 0.6, seed=seed, nhit=1, lattice_id=lid, start=O.COLD)
    f.sweep(1)
    phi = f.get_field()
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(16):
        w = O.philox4x32_10([i, lid, 0, 0], key)
        u = ((w >> 8).astype(np.float64) + 0.5) / 2 ** 24
        acc_word = ((int(w[0]) & 0xFF) << 16) | ((int(w[1]) & 0xFF) << 8) | (int(w[2]) & 0xFF)
        ua = (acc_word + 0.5) / 2 ** 24
        old = np.array([1.0, 0, 0, 0])
        trial = old + 0.6 * (2 * u - 1)
        accept = ua < math.exp(-(trial @ trial - 1.0))
        assert np.array_equal(phi[i], trial if accept else old)


def test_rejects_bad_parameters():
    for args in ((5, (4, 4, 4, 4), 0.1, 0.1), (4, (3, 4, 4, 4), 0.1, 0.1), (4, (4, 4, 4, 4), 0.1, -1.0)):
        with pytest.raises(ValueError):
            O.ONField(*args)
    with pytest.raises(ValueError):
        O.ONField(4, (4, 4, 4, 4), 0.1, 0.1, delta=0.0)
    with pytest.raises(ValueError):
        O.ONField(4, (4, 4, 4, 4), 0.1, 0.1, rng=O.RNG_MRG32K3A, seed=0)
    with pytest.raises(ValueError):
        O.ONField(4, (4, 4, 4, 4), 0.1, 0.1, rng=5)
