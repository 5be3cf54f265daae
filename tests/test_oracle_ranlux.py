"""RANLUX luxury level 3 (the paper's generator for its benchmark runs,
Sec. 5) in the oracle: the subtract-with-borrow generator
x_n = x_{n-10} - x_{n-24} - c mod 2^24, of which the first r = 24 of every
p = 223 outputs are used."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O


def test_library_generator_has_the_standard_values():
    # the C++ standard fixes the 10000th output of default-seeded
    # ranlux24_base and ranlux24 (p = 223, r = 23)
    assert O.ranlux_standard_values() == (7937952, 9901578)


def swb_reference(seed: int, n: int) -> np.ndarray:
    """The subtract-with-borrow generator and its seeding written out: a
    Lehmer generator x -> 40014 x mod 2147483563 started at the seed gives the
    24 initial words (mod 2^24, oldest first); the carry starts at 1 if the
    newest word is 0."""
    e = seed % 2147483563 or 1
    x = []
    for _ in range(24):
        e = (40014 * e) % 2147483563
        x.append(e % (1 << 24))
    c = 1 if x[-1] == 0 else 0
    out = []
    for _ in range(n):
        y = x[-10] - x[-24] - c
        c = 1 if y < 0 else 0
        y %= 1 << 24
        x = x[1:] + [y]
        out.append(y)
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("seed", [1, 19780503, 2147483560])
def test_base_generator_written_out(seed):
    assert np.array_equal(O.ranlux_raw(seed, 500, luxury=False), swb_reference(seed, 500))


def test_luxury_blocks():
    base = O.ranlux_raw(12345, 3 * 223, luxury=False)
    lux = O.ranlux_raw(12345, 72)
    for b in range(3):
        assert np.array_equal(lux[24 * b:24 * b + 24], base[223 * b:223 * b + 24])


def test_site_seeds_are_distinct_and_in_range():
    seeds = [O.ranlux_site_seed(7, i, 0) for i in range(4096)] + [O.ranlux_site_seed(7, i, 1) for i in range(4096)]
    assert len(set(seeds)) == len(seeds)
    assert all(1 <= s < 2147483563 for s in seeds)
    assert O.ranlux_site_seed(7, 5, 0) == 1 + (7 + 1000003 * 5) % 2147483561


def binned_mean_err(x, nb):
    x = np.asarray(x)
    b = x[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


def test_su2_strong_coupling_with_ranlux_streams():
    """Generator independence: the SU(2) strong-coupling plaquette
    I_2(beta)/I_1(beta) with RANLUX streams, as with Philox."""
    beta = 0.3
    L = O.Lattice(2, (8, 8, 8, 8), beta, rng=O.RNG_RANLUX, seed=31, nhit=120, start=O.HOT)
    for _ in range(5):
        L.sweep(1, 0)
    ps = []
    for _ in range(300):
        L.sweep(1, 0)
        ps.append(L.measure()[0][0])
    m, e = binned_mean_err(ps, 20)
    u = special.iv(2, beta) / special.iv(1, beta)
    assert abs(m - u) < 4 * e + 2e-5, (m, e, u)


def test_hot_start_with_ranlux_is_haar():
    from helpers import to_matrices
    L = O.Lattice(3, (8, 8, 8, 8), 5.0, rng=O.RNG_RANLUX, seed=7, start=O.HOT)
    m = to_matrices(L.get_links(), 3).reshape(-1, 3, 3)
    tr = np.trace(m, axis1=-2, axis2=-1)
    n = len(tr)
    assert abs(tr.mean()) < 5 / math.sqrt(n)
    assert abs((np.abs(tr) ** 2).mean() - 1.0) < 7.5 / math.sqrt(n)
