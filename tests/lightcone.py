"""Light cone of a checkerboard compound sweep (test-side host logic).

A link update reads its own link and the 18 links of its staple.  When one
update comes out differently on two sides (an accept decision that rounding
flipped), every later update of the same compound sweep that reads a link
already affected is affected too.  ``downstream`` follows that dependence
pass by pass, in the schedule of the sweep (n_hb heat-bath sweeps, then
n_or overrelaxation sweeps; each sweep mu = 0..3, parity 0 then 1), and
returns the links that may differ at the end; parity tests compare every
other link at the full bar.  Shares nothing with the oracle or the library.
"""
from __future__ import annotations

import numpy as np


def _shift(dims, mu, d):
    """Index map i -> i + d * mu-hat in the canonical site order."""
    nx, ny, nz, nt = dims
    idx = np.arange(nx * ny * nz * nt).reshape(nt, nz, ny, nx)
    return np.roll(idx, -d, axis=3 - mu).reshape(-1)


def parity(dims) -> np.ndarray:
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def downstream(dims, n_hb, n_or, flips=None, initial=None) -> np.ndarray:
    """Links [V, 4] (bool) that may differ after one compound sweep.

    flips: bool [n_hb, 4, V], the heat-bath updates whose decision differed
    (heat-bath sweep k, direction mu, canonical site); initial: bool [V, 4],
    links that already differ before the sweep."""
    V = int(np.prod(dims))
    taint = np.zeros((V, 4), bool) if initial is None else initial.astype(bool).copy()
    par = parity(dims)
    plus = [_shift(dims, m, +1) for m in range(4)]
    minus = [_shift(dims, m, -1) for m in range(4)]
    for s in range(n_hb + n_or):
        for mu in range(4):
            for p in (0, 1):
                dep = taint[:, mu].copy()
                for nu in range(4):
                    if nu == mu:
                        continue
                    # forward term U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
                    dep |= taint[plus[mu], nu] | taint[plus[nu], mu] | taint[:, nu]
                    # backward term U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
                    dep |= taint[minus[nu][plus[mu]], nu] | taint[minus[nu], mu] | taint[minus[nu], nu]
                if s < n_hb and flips is not None:
                    dep |= flips[s, mu]
                sel = par == p
                taint[sel, mu] |= dep[sel]
    return taint


def flipped_updates(log_a: np.ndarray, log_b: np.ndarray, n_hb: int, V: int) -> np.ndarray:
    """bool [n_hb, 4, V] from two accept logs [n_hb][mu][site][subgroup]."""
    a = np.asarray(log_a).reshape(n_hb, 4, V, -1)
    b = np.asarray(log_b).reshape(n_hb, 4, V, -1)
    return (a != b).any(axis=3)
