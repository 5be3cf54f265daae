"""Test-side numpy helpers: canonical link format <-> complex matrices and
simple checks.  Not shared with the oracle or the HIP library."""
from __future__ import annotations

import numpy as np


def to_matrices(links: np.ndarray, group: int) -> np.ndarray:
    """Canonical [..., comp] -> [..., N, N] complex."""
    if group == 3:
        c = links[..., 0::2] + 1j * links[..., 1::2]
        return c.reshape(links.shape[:-1] + (3, 3))
    a0, a1, a2, a3 = (links[..., k] for k in range(4))
    m = np.empty(links.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = a0 + 1j * a3
    m[..., 0, 1] = a2 + 1j * a1
    m[..., 1, 0] = -a2 + 1j * a1
    m[..., 1, 1] = a0 - 1j * a3
    return m


def from_matrices(m: np.ndarray, group: int) -> np.ndarray:
    if group == 3:
        out = np.empty(m.shape[:-2] + (18,))
        f = m.reshape(m.shape[:-2] + (9,))
        out[..., 0::2] = f.real
        out[..., 1::2] = f.imag
        return out
    out = np.empty(m.shape[:-2] + (4,))
    out[..., 0] = 0.5 * (m[..., 0, 0] + m[..., 1, 1]).real
    out[..., 1] = 0.5 * (m[..., 0, 1] + m[..., 1, 0]).imag
    out[..., 2] = 0.5 * (m[..., 0, 1] - m[..., 1, 0]).real
    out[..., 3] = 0.5 * (m[..., 0, 0] - m[..., 1, 1]).imag
    return out


def unitarity_error(m: np.ndarray) -> float:
    n = m.shape[-1]
    e = m @ np.conj(np.swapaxes(m, -1, -2)) - np.eye(n)
    return float(np.abs(e).max())


def det_error(m: np.ndarray) -> float:
    return float(np.abs(np.linalg.det(m) - 1.0).max())


def haar_su(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(n) by QR of a complex Ginibre matrix with the phase fix."""
    z = (rng.standard_normal((count, n, n)) + 1j * rng.standard_normal((count, n, n))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / n))[:, None, None]
    return q


def neighbour(dims, mu):
    """Index map i -> i + mu-hat for the canonical site order."""
    nx, ny, nz, nt = dims
    idx = np.arange(nx * ny * nz * nt).reshape(nt, nz, ny, nx)
    axis = 3 - mu
    return np.roll(idx, -1, axis=axis).reshape(-1)


def gauge_transform(links_m: np.ndarray, g: np.ndarray, dims) -> np.ndarray:
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger on [V,4,N,N] matrices."""
    out = np.empty_like(links_m)
    for mu in range(4):
        nb = neighbour(dims, mu)
        out[:, mu] = g @ links_m[:, mu] @ np.conj(np.swapaxes(g[nb], -1, -2))
    return out


def plaquette_numpy(links_m: np.ndarray, dims):
    """Independent numpy plaquette (P, P_s, P_t) on W-frame matrices [V,4,N,N]."""
    n = links_m.shape[-1]
    V = links_m.shape[0]
    sp = tp = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = links_m[:, mu]
            b = links_m[neighbour(dims, mu), nu]
            c = np.conj(np.swapaxes(links_m[neighbour(dims, nu), mu], -1, -2))
            d = np.conj(np.swapaxes(links_m[:, nu], -1, -2))
            tr = np.trace(a @ b @ c @ d, axis1=-2, axis2=-1).real.sum() / n
            if nu == 3:
                tp += tr
            else:
                sp += tr
    ps, pt = sp / (3 * V), tp / (3 * V)
    return np.array([(ps + pt) / 2, ps, pt])


def polyakov_numpy(links_m: np.ndarray, dims):
    nx, ny, nz, nt = dims
    vs = nx * ny * nz
    n = links_m.shape[-1]
    P = np.broadcast_to(np.eye(n, dtype=np.complex128), (vs, n, n)).copy()
    for t in range(nt):
        P = P @ links_m[t * vs:(t + 1) * vs, 3]
    tr = np.trace(P, axis1=-2, axis2=-1) / n
    return np.array([tr.real.mean(), tr.imag.mean()])
