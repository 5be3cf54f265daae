"""Plain FP64 CPU oracle for the checkerboard SU(2)/SU(3) Wilson-action sweep.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product package never imports
it.  The C++ source (``oracle.cpp``) shares no code with the HIP library.

Parity with the paper itself is unpinned (the paper prints no physics
values); each function is pinned by the CPU tests against closed forms,
exact distributions, invariants and an independent PRNG implementation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

RNG_MRG32K3A, RNG_PHILOX, RNG_CONST, RNG_RANLUX = 0, 1, 2, 3
COLD, HOT = 0, 1

_lib = None


def build() -> str:
    """Compile liboracle.so with g++ (FP64, OpenMP, no FP contraction)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off",
           "-fcx-limited-range", "-fPIC", "-shared", "-o", tmp, _SRC]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, d, i, u32, u64, i64 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i, i, i, i, i, d, i, i, d, u64, i, u32, i, i]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_threads.argtypes = [i]
        L.orc_get_threads.restype = i
        L.orc_sweep.argtypes = [vp, i, i]
        L.orc_measure.argtypes = [vp, vp, vp]
        L.orc_get_links.argtypes = [vp, vp]
        L.orc_set_links.argtypes = [vp, vp]
        L.orc_hb_sweeps.argtypes = [vp]
        L.orc_hb_sweeps.restype = u64
        L.orc_get_mrg_states.argtypes = [vp, vp]
        L.orc_get_mrg_states.restype = i
        L.orc_enable_accept_log.argtypes = [vp, i]
        L.orc_get_accept_log.argtypes = [vp, vp, i64]
        L.orc_get_accept_log.restype = i64
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_mrg_site_state.argtypes = [u64, u64, vp]
        L.orc_mrg_site_state.restype = i
        L.orc_mrg_next.argtypes = [vp]
        L.orc_mrg_next.restype = u32
        L.orc_mrg_advance_pow2.argtypes = [vp, i]
        L.orc_uniform24.argtypes = [u32]
        L.orc_uniform24.restype = d
        L.orc_kp_sample.argtypes = [d, i, vp, vp, vp]
        L.orc_kp_sample.restype = i
        L.orc_update_link.argtypes = [i, d, i, i, i, vp, vp, vp, vp]
        L.orc_update_link.restype = i
        L.orc_staple.argtypes = [vp, i64, i, vp]
        L.orc_ranlux_raw.argtypes = [u32, i, i, vp]
        L.orc_ranlux_standard_values.argtypes = [vp]
        L.orc_ranlux_site_seed.argtypes = [u64, i64, u32]
        L.orc_ranlux_site_seed.restype = u32
        L.orc_on_create.restype = vp
        L.orc_on_create.argtypes = [i, i, i, i, i, d, d, d, d, i, d, u64, i, u32, i]
        L.orc_on_destroy.argtypes = [vp]
        L.orc_on_sweep.argtypes = [vp, i]
        L.orc_on_measure.argtypes = [vp, vp]
        L.orc_on_get_field.argtypes = [vp, vp]
        L.orc_on_set_field.argtypes = [vp, vp]
        L.orc_on_sweeps.argtypes = [vp]
        L.orc_on_sweeps.restype = u64
        L.orc_on_get_mrg_states.argtypes = [vp, vp]
        L.orc_on_get_mrg_states.restype = i
        L.orc_on_acceptance.argtypes = [vp]
        L.orc_on_acceptance.restype = d
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def ncomp(group: int) -> int:
    return 18 if group == 3 else 4


class Lattice:
    """One lattice in the oracle.  Links are exchanged in the canonical FP64
    W-frame layout ``[site][mu][comp]``."""

    def __init__(self, group, dims, beta, flux=0, rng=RNG_PHILOX, rng_const=0.5,
                 seed=1, nhit=10, lattice_id=0, start=HOT, frozen=0):
        self.group = int(group)
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        self.rng = rng
        h = lib().orc_create(self.group, *self.dims, float(beta), int(flux), int(rng),
                             float(rng_const), int(seed), int(nhit), int(lattice_id), int(start),
                             int(frozen))
        if not h:
            raise ValueError("oracle rejected the lattice parameters")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def sweep(self, n_hb=1, n_or=0):
        lib().orc_sweep(self._h, int(n_hb), int(n_or))

    def measure(self):
        p = np.zeros(3)
        l = np.zeros(2)
        lib().orc_measure(self._h, _ptr(p), _ptr(l))
        return p, l

    def get_links(self) -> np.ndarray:
        out = np.empty((self.V, 4, ncomp(self.group)))
        lib().orc_get_links(self._h, _ptr(out))
        return out

    def set_links(self, links: np.ndarray) -> None:
        a = np.ascontiguousarray(links, dtype=np.float64).reshape(self.V, 4, ncomp(self.group))
        lib().orc_set_links(self._h, _ptr(a))

    def hb_sweeps(self) -> int:
        return int(lib().orc_hb_sweeps(self._h))

    def mrg_states(self) -> np.ndarray:
        out = np.empty((self.V, 6), dtype=np.uint32)
        if lib().orc_get_mrg_states(self._h, _ptr(out)) != 0:
            raise ValueError("not an MRG32k3a lattice")
        return out

    def enable_accept_log(self, on=True):
        lib().orc_enable_accept_log(self._h, int(bool(on)))

    def accept_log(self) -> np.ndarray:
        n = lib().orc_get_accept_log(self._h, None, 0)
        out = np.empty(n, dtype=np.int8)
        lib().orc_get_accept_log(self._h, _ptr(out), n)
        return out

    def staple(self, site: int, mu: int) -> np.ndarray:
        n = self.group
        out = np.empty(2 * n * n)
        lib().orc_staple(self._h, int(site), int(mu), _ptr(out))
        return (out[0::2] + 1j * out[1::2]).reshape(n, n)


def ranlux_raw(seed: int, n: int, luxury: bool = True) -> np.ndarray:
    """First n 24-bit outputs of RANLUX luxury level 3 (p = 223, r = 24), or of
    the bare subtract-with-borrow generator if luxury is False."""
    out = np.empty(n, dtype=np.uint32)
    lib().orc_ranlux_raw(int(seed), int(n), int(bool(luxury)), _ptr(out))
    return out


def ranlux_standard_values() -> tuple:
    out = np.empty(2, dtype=np.uint32)
    lib().orc_ranlux_standard_values(_ptr(out))
    return int(out[0]), int(out[1])


def ranlux_site_seed(seed: int, site: int, lattice_id: int = 0) -> int:
    return int(lib().orc_ranlux_site_seed(int(seed), int(site), int(lattice_id)))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def mrg_site_state(seed: int, site: int) -> np.ndarray:
    st = np.empty(6, dtype=np.uint32)
    if lib().orc_mrg_site_state(int(seed), int(site), _ptr(st)) != 0:
        raise ValueError("MRG32k3a seed out of range")
    return st


def mrg_next(st: np.ndarray) -> int:
    assert st.dtype == np.uint32 and st.flags.c_contiguous
    return int(lib().orc_mrg_next(_ptr(st)))


def mrg_advance_pow2(st: np.ndarray, e: int) -> None:
    lib().orc_mrg_advance_pow2(_ptr(st), int(e))


def uniform24(w: int) -> float:
    return float(lib().orc_uniform24(int(w) & 0xFFFFFFFF))


def kp_sample(alpha: float, nhit: int, u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float64)
    x = np.empty(4)
    used = ctypes.c_int(0)
    t = lib().orc_kp_sample(float(alpha), int(nhit), _ptr(u), _ptr(x), ctypes.byref(used))
    return t, x, used.value


def update_link(group, beta, nhit, kind, reunit, U, A, u):
    """Update one link U (canonical) with staple A (N x N complex)."""
    n = int(group)
    Uc = np.ascontiguousarray(U, dtype=np.float64)
    Am = np.ascontiguousarray(A, dtype=np.complex128).reshape(n, n)
    Ar = np.empty(2 * n * n)
    Ar[0::2] = Am.real.ravel()
    Ar[1::2] = Am.imag.ravel()
    uu = np.ascontiguousarray(u if u is not None else np.zeros(1), dtype=np.float64)
    out = np.empty(ncomp(n))
    used = lib().orc_update_link(n, float(beta), int(nhit), int(kind), int(reunit),
                                 _ptr(Uc), _ptr(Ar), _ptr(uu), _ptr(out))
    return out, used


class ONField:
    """O(N) phi^4 model in the oracle: an N-vector per site (N = 1..4),
    multi-hit Metropolis with NHIT hits per site and sweep.  The field is
    exchanged as FP64 ``[site][component]``.  ``measure()`` returns
    (<phi^2>, <phi(x).phi(x+mu)>, <(phi^2-1)^2>, <phi_0>, .., <phi_3>)."""

    def __init__(self, ncomp, dims, kappa, lam, h=0.0, delta=1.0, rng=RNG_PHILOX, rng_const=0.5,
                 seed=1, nhit=100, lattice_id=0, start=HOT):
        self.n = int(ncomp)
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        h_ = lib().orc_on_create(self.n, *self.dims, float(kappa), float(lam), float(h), float(delta),
                                 int(rng), float(rng_const), int(seed), int(nhit), int(lattice_id), int(start))
        if not h_:
            raise ValueError("oracle rejected the O(N) parameters")
        self._h = h_

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_on_destroy(h)
            self._h = None

    def sweep(self, n=1):
        lib().orc_on_sweep(self._h, int(n))

    def measure(self) -> np.ndarray:
        out = np.zeros(7)
        lib().orc_on_measure(self._h, _ptr(out))
        return out

    def get_field(self) -> np.ndarray:
        out = np.empty((self.V, self.n))
        lib().orc_on_get_field(self._h, _ptr(out))
        return out

    def set_field(self, phi: np.ndarray) -> None:
        a = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.V, self.n)
        lib().orc_on_set_field(self._h, _ptr(a))

    def sweeps(self) -> int:
        return int(lib().orc_on_sweeps(self._h))

    def acceptance(self) -> float:
        return float(lib().orc_on_acceptance(self._h))

    def mrg_states(self) -> np.ndarray:
        out = np.empty((self.V, 6), dtype=np.uint32)
        if lib().orc_on_get_mrg_states(self._h, _ptr(out)) != 0:
            raise ValueError("not an MRG32k3a field")
        return out
