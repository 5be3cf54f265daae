"""Pins of the oracle's draw layout: single link updates of a lattice sweep
rebuilt by hand from raw generator outputs.

Each test runs an oracle sweep with the accept log on, then, for sample links,
feeds `update_link` (one link update with a given staple and a plain list of
uniforms) the uniforms that the documented layout prescribes, taken from the
raw generators (Philox4x32-10 words, MRG32k3a outputs, RANLUX luxury-3
blocks), with the staple the link saw at its update (the links of earlier
passes after their update, the others before).  The rebuilt link must equal
the lattice's.  A planted wrong convention (counter not advanced across the
heat-bath sweeps of a compound sweep, direction slot next to the accepted
try, per-link MRG streams, RANLUX blocks not restarted per update) is fed the
same way and must not.

Layout (a reading; the paper's generator library hands out numbers from
buffers, Sec. 3.4): uniform u = ((w >> 8) + 1/2) 2^-24 of a 32-bit word w;
per SU(N) (sub)group g of a heat-bath update, tries t = 0, 1, ... draw four
uniforms and an accepted try two more for the direction.  Philox counter of
try t: (site, lattice id, 4 (h + k) + mu, g (NHIT + 1) + t) with h the
heat-bath sweeps done before the compound sweep and k the heat-bath sweep
within it; the direction uses slot t = NHIT.  MRG32k3a: the site's stream in
order over the site's updates.  RANLUX: each update begins a new block of 24.
"""
import numpy as np
import pytest

import oracle as O

NHIT = 10
U24 = 2.0 ** -24


def u24(w):
    return ((int(w) >> 8) + 0.5) * U24


def parity_of(dims, i):
    nx, ny, nz, _ = dims
    x, y, z, t = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)
    return (x + y + z + t) & 1


def staple_at_update(group, dims, before, after, i, mu):
    """Staple of link (i, mu) at its update in a sweep that took the links from
    `before` to `after`: passes run mu' = 0..3, parity 0 then 1, so links of
    earlier passes are taken after their update."""
    V = int(np.prod(dims))
    par = np.array([parity_of(dims, j) for j in range(V)])
    order = 2 * np.arange(4)[None, :] + par[:, None]  # pass index of every link
    mine = 2 * mu + parity_of(dims, i)
    mixed = np.where((order < mine)[:, :, None], after, before)
    L = O.Lattice(group, dims, 1.0, start=O.COLD)
    L.set_links(mixed)
    return L.staple(i, mu)


def nsub(group):
    return 3 if group == 3 else 1


def tries_of(log_entry):
    """Tries consumed by a (sub)group update with logged outcome t (-1: all rejected)."""
    return NHIT if log_entry < 0 else log_entry + 1


def philox_uniforms(seed, lat, site, word2, accepts, dir_slot=None, packed=False):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = []
    for g, t_acc in enumerate(accepts):
        base = g * NHIT if packed else g * (NHIT + 1)
        for t in range(tries_of(t_acc)):
            w = O.philox4x32_10([site, lat, word2, base + t], key)
            out += [u24(x) for x in w]
        if t_acc >= 0:
            slot = base + (NHIT if dir_slot is None else dir_slot(t_acc))
            w = O.philox4x32_10([site, lat, word2, slot], key)
            out += [u24(w[0]), u24(w[1])]
    return np.array(out)


def test_philox_layout_across_two_heat_bath_sweeps():
    """SU(3) 4^4 from a Haar start after one heat-bath sweep (h = 1): a
    (2 HB) compound sweep.  Sweep k uses counter word 2 = 4 (h + k) + mu."""
    dims, beta, seed, lat = (4, 4, 4, 4), 5.7, 0x9E3779B97F4A7C15, 3
    mk = lambda: O.Lattice(3, dims, beta, seed=seed, lattice_id=lat, start=O.HOT, nhit=NHIT)
    L = mk()
    L.sweep(1, 0)
    s0 = L.get_links()
    ref = mk()  # the state after the first heat-bath sweep of the compound sweep
    ref.sweep(1, 0)
    ref.sweep(1, 0)
    s1 = ref.get_links()  # (differs from it only by the rounding of a reunitarisation)
    L.enable_accept_log(True)
    L.sweep(2, 0)
    s2 = L.get_links()
    V = int(np.prod(dims))
    log = L.accept_log().reshape(2, 4, V, 3).astype(int)
    assert (log >= 1).any() and (log == 0).any()  # both first-try and later acceptances occur
    checked = wrong_h = wrong_slot = wrong_pack = 0
    for i in (0, 1, 5, 22, 63, 64, 200, 255):
        for mu in range(4):
            # k = 0
            A0 = staple_at_update(3, dims, s0, s1, i, mu)
            u = philox_uniforms(seed, lat, i, 4 * (1 + 0) + mu, log[0, mu, i])
            U1, used = rebuild(3, beta, 0, s0[i, mu], A0, u)
            assert used == len(u)
            assert np.abs(U1 - s1[i, mu]).max() < 1e-12, (i, mu)
            # k = 1, reunitarised as the last sweep of the compound sweep
            A1 = staple_at_update(3, dims, s1, s2, i, mu)
            u = philox_uniforms(seed, lat, i, 4 * (1 + 1) + mu, log[1, mu, i])
            U2, used = rebuild(3, beta, 1, U1, A1, u)
            assert used == len(u)
            assert np.abs(U2 - s2[i, mu]).max() < 1e-12, (i, mu)
            checked += 1
            # planted mistakes must not reproduce the lattice's link
            bad = philox_uniforms(seed, lat, i, 4 * 1 + mu, log[1, mu, i])  # h + k not advanced
            wrong_h += differs(3, beta, 1, U1, A1, bad, s2[i, mu])
            bad = philox_uniforms(seed, lat, i, 4 * 2 + mu, log[1, mu, i], dir_slot=lambda t: t + 1)
            wrong_slot += differs(3, beta, 1, U1, A1, bad, s2[i, mu])
            bad = philox_uniforms(seed, lat, i, 4 * 2 + mu, log[1, mu, i], packed=True)
            wrong_pack += differs(3, beta, 1, U1, A1, bad, s2[i, mu])
    assert checked == 32
    # a planted layout coincides with the true one only where it reads the same
    # slots (a packed layout for a link whose later subgroups all rejected, a
    # direction slot t + 1 after an acceptance at the last try)
    assert wrong_h == checked and wrong_slot >= checked - 2 and wrong_pack >= checked - 2, \
        (wrong_h, wrong_slot, wrong_pack)


def test_philox_layout_su2_and_lattice_id():
    """SU(2) 4^4 hot start, one heat-bath sweep: the lattice id is counter
    word 1 and the 64-bit seed is the key (low word first)."""
    dims, beta, seed, lat = (4, 4, 4, 4), 2.3, (5 << 32) | 77, 9
    L = O.Lattice(2, dims, beta, seed=seed, lattice_id=lat, start=O.HOT, nhit=NHIT)
    s0 = L.get_links()
    L.enable_accept_log(True)
    L.sweep(1, 0)
    s1 = L.get_links()
    V = int(np.prod(dims))
    log = L.accept_log().reshape(1, 4, V, 3).astype(int)
    for i in (0, 3, 17, 100, 255):
        for mu in range(4):
            A = staple_at_update(2, dims, s0, s1, i, mu)
            u = philox_uniforms(seed, lat, i, mu, log[0, mu, i, :1])
            U, used = rebuild(2, beta, 1, s0[i, mu], A, u)
            assert used == len(u) and np.abs(U - s1[i, mu]).max() < 1e-13, (i, mu)
            bad = philox_uniforms(seed, 0, i, mu, log[0, mu, i, :1])  # lattice id ignored
            assert differs(2, beta, 1, s0[i, mu], A, bad, s1[i, mu])
            bad = philox_uniforms(seed & 0xFFFFFFFF, lat, i, mu, log[0, mu, i, :1])  # key high word dropped
            assert differs(2, beta, 1, s0[i, mu], A, bad, s1[i, mu])


def rebuild(group, beta, reunit, U, A, u):
    """One heat-bath link update fed the uniforms u; NaN padding behind them
    makes an update that reads more than the layout prescribes visible."""
    out, used = O.update_link(group, beta, NHIT, 0, reunit, U, A,
                              np.concatenate([u, np.full(8 * NHIT * 3, np.nan)]))
    return out, used


def differs(group, beta, reunit, U, A, u, target):
    """True if a link update fed the uniforms u (padded, so that a planted
    layout that needs more tries reads defined values) misses target."""
    u = np.concatenate([u, np.full(8 * NHIT * 3, 0.5)])
    out, _ = O.update_link(group, beta, NHIT, 0, reunit, U, A, u)
    return bool(np.abs(out - target).max() > 1e-3)


def mrg_take(st, n):
    return [O.mrg_next(st) for _ in range(n)]


def draws_needed(accepts):
    return sum(4 * tries_of(t) + (2 if t >= 0 else 0) for t in accepts)


@pytest.mark.parametrize("group", [2, 3])
def test_mrg_draw_order(group):
    """MRG32k3a: the hot start draws 4 (SU(2)) or 12 (SU(3)) uniforms per link
    in mu order from the site's stream, then the heat-bath updates of the
    site's links, mu = 0..3, continue the same stream; the final generator
    state is the stream advanced by every draw."""
    dims, seed = (4, 4, 4, 2), 1234
    beta = 5.7 if group == 3 else 2.3
    L = O.Lattice(group, dims, beta, rng=O.RNG_MRG32K3A, seed=seed, start=O.HOT, nhit=NHIT)
    s0 = L.get_links()
    L.enable_accept_log(True)
    L.sweep(1, 0)
    s1 = L.get_links()
    V = int(np.prod(dims))
    log = L.accept_log().reshape(1, 4, V, 3)[:, :, :, :nsub(group)].astype(int)
    states = L.mrg_states()
    per_link_init = 12 if group == 3 else 4
    for i in (0, 1, 9, 40, V - 1):
        st = O.mrg_site_state(seed, i)
        mrg_take(st, 4 * per_link_init)
        for mu in range(4):
            A = staple_at_update(group, dims, s0, s1, i, mu)
            n = draws_needed(log[0, mu, i])
            u = np.array([((z >> 8) + 0.5) * U24 for z in mrg_take(st, n)])
            U, used = rebuild(group, beta, 1, s0[i, mu], A, u)
            assert used == n and np.abs(U - s1[i, mu]).max() < 1e-13, (i, mu)
            if mu == 1:
                # planted: every link restarting the site's stream after the hot start
                fresh = O.mrg_site_state(seed, i)
                mrg_take(fresh, 4 * per_link_init)
                bad = np.array([((z >> 8) + 0.5) * U24 for z in mrg_take(fresh, n)])
                assert differs(group, beta, 1, s0[i, mu], A, bad, s1[i, mu])
        assert np.array_equal(st, states[i])


def test_ranlux_block_rule():
    """RANLUX luxury 3: the hot start begins one block per link (12 of its 24
    values used), every heat-bath update begins a new block, and an update
    that needs more than 24 values runs on into the next block, after which
    the site's next update begins the block after that."""
    dims, beta, seed = (4, 4, 4, 2), 2.0, 77  # strong coupling: frequent retries
    L = O.Lattice(3, dims, beta, rng=O.RNG_RANLUX, seed=seed, start=O.HOT, nhit=NHIT)
    s0 = L.get_links()
    L.enable_accept_log(True)
    L.sweep(1, 0)
    s1 = L.get_links()
    V = int(np.prod(dims))
    log = L.accept_log().reshape(1, 4, V, 3).astype(int)
    need = np.array([[draws_needed(log[0, mu, i]) for mu in range(4)] for i in range(V)])
    long_sites = [i for i in range(V) if (need[i] > 24).any()]
    assert long_sites, "no update needed more than one block"
    spill = restart = 0
    for i in long_sites[:6] + [0, 5]:
        raw = O.ranlux_raw(O.ranlux_site_seed(seed, i, 0), 24 * 16)
        block = 4  # blocks 0..3 went to the hot start
        seq_block = 4 * 24  # planted: values taken in sequence, blocks not restarted
        for mu in range(4):
            n = need[i, mu]
            take = raw[24 * block: 24 * block + n]
            u = (take + 0.5) * U24
            A = staple_at_update(3, dims, s0, s1, i, mu)
            U, used = rebuild(3, beta, 1, s0[i, mu], A, u)
            assert used == n and np.abs(U - s1[i, mu]).max() < 1e-13, (i, mu, n)
            spill += n > 24
            bad = (raw[seq_block: seq_block + n] + 0.5) * U24
            if mu > 0:
                restart += differs(3, beta, 1, s0[i, mu], A, bad, s1[i, mu])
            seq_block += n
            block += (n + 23) // 24
    assert spill >= 1 and restart >= 1
