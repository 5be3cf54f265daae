"""Python binding of liblat.so: the MI355X checkerboard SU(2)/SU(3)
Wilson-action Monte Carlo (see include/lat.h for the C ABI).

Argument marshalling only: every step of the sweep and of the measurements
runs in the HIP kernels of the library.  PyTorch is optional plumbing for
device memory (a caller-owned buffer) and streams.  Importing this module
fails loudly if the compiled library is missing.
"""
from __future__ import annotations

import ctypes
import os
import struct

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblat.so")

OK, EINVAL, ENOMEM, EDEVICE, EIO, ECORRUPT, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32, F32_C12, F64_C12 = 0, 1, 2, 3
RNG_MRG32K3A, RNG_PHILOX, RNG_CONST, RNG_RANLUX = 0, 1, 2, 3
COLD, HOT = 0, 1
FROZEN_NONE, FROZEN_T0 = 0, 1

STORAGE_NAMES = {F64: "f64", F32: "f32", F32_C12: "f32c12", F64_C12: "f64c12"}
NOALLOC_SCRATCH_BYTES = 16 << 20  # LAT_NOALLOC_SCRATCH_BYTES of lat.h


class LatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("storage", ctypes.c_int),
        ("rng", ctypes.c_int),
        ("rng_const", ctypes.c_double),
        ("start", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("nhit", ctypes.c_int),
        ("lattice_id", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("device_buffer", ctypes.c_void_p),
        ("device_bytes", ctypes.c_size_t),
        ("block_size", ctypes.c_int),
        ("tile_order", ctypes.c_int),
        ("layout", ctypes.c_int),
        ("tile", ctypes.c_int * 4),
        ("max_waves_per_simd", ctypes.c_int),
        ("frozen", ctypes.c_int),
        ("stage_lds", ctypes.c_int),
    ]


class Desc(ctypes.Structure):
    _fields_ = [
        ("group", ctypes.c_int), ("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("Nz", ctypes.c_int),
        ("Nt", ctypes.c_int), ("beta", ctypes.c_double), ("field_flux", ctypes.c_int),
        ("seed", ctypes.c_uint64), ("start", ctypes.c_int), ("lattice_id", ctypes.c_uint32),
    ]


def _load():
    # PyTorch ships its own HIP runtime under the same soname as the system's
    # (libamdhip64.so.7); a process can hold only one.  If torch is installed
    # it is loaded first, so that the library and torch share torch's runtime
    # (torch does not start on a runtime other than its own).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1310_7087_amd/build.py` "
            "(the HIP library is the only implementation; there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz, u64, i64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t,
                              ctypes.c_uint64, ctypes.c_int64)
    P = ctypes.POINTER
    L.lat_default_options.argtypes = [P(Options)]
    L.lat_default_options.restype = None
    L.lat_device_bytes.argtypes = [i, i, i, i, i, P(Options)]
    L.lat_device_bytes.restype = sz
    L.lat_create.argtypes = [P(vp), i, i, i, i, i, d, i, P(Options)]
    L.lat_sweep.argtypes = [vp, i, i]
    L.lat_run.argtypes = [vp, i, i, i, i, vp, vp]
    L.lat_measure.argtypes = [vp, vp, vp]
    L.lat_get_links.argtypes = [vp, vp, sz]
    L.lat_get_links_noalloc.argtypes = [vp, vp, sz]
    L.lat_set_links.argtypes = [vp, vp, sz]
    L.lat_get_rng_state.argtypes = [vp, vp, sz]
    L.lat_get_info.argtypes = [vp, P(u64), P(u64), P(u64)]
    L.lat_profile_passes.argtypes = [vp, i, i, i, P(d), P(d)]
    L.lat_autotune.argtypes = [vp, i, i, vp]
    L.lat_get_launch_shape.argtypes = [vp, i, vp]
    L.lat_set_accept_log.argtypes = [vp, i]
    L.lat_get_accept_log.argtypes = [vp, vp, sz]
    L.lat_get_accept_log.restype = i64
    L.lat_save.argtypes = [vp, ctypes.c_char_p]
    L.lat_load.argtypes = [P(vp), ctypes.c_char_p, P(Options)]
    L.lat_destroy.argtypes = [vp]
    L.lat_last_error.argtypes = []
    L.lat_last_error.restype = ctypes.c_char_p
    L.lat_philox4x32_10.argtypes = [vp, vp, vp, sz]
    L.lat_batch_create.argtypes = [P(vp), i, P(Desc), P(Options)]
    L.lat_batch_run.argtypes = [vp, i, i, i, vp, vp]
    L.lat_batch_configure.argtypes = [vp, i, i, i, i]
    L.lat_batch_autotune.argtypes = [vp, i, i, vp]
    L.lat_batch_get_shape.argtypes = [vp, vp]
    L.lat_batch_get_links.argtypes = [vp, i, vp, sz]
    L.lat_batch_set_links.argtypes = [vp, i, vp, sz]
    L.lat_batch_destroy.argtypes = [vp]
    L.lat_on_device_bytes.argtypes = [i, i, i, i, i, P(Options)]
    L.lat_on_device_bytes.restype = sz
    L.lat_on_create.argtypes = [P(vp), i, i, i, i, i, d, d, d, d, P(Options)]
    L.lat_on_sweep.argtypes = [vp, i]
    L.lat_on_measure.argtypes = [vp, vp]
    L.lat_on_run.argtypes = [vp, i, i, vp]
    L.lat_on_acceptance.argtypes = [vp, P(d)]
    L.lat_on_get_field.argtypes = [vp, vp, sz]
    L.lat_on_set_field.argtypes = [vp, vp, sz]
    L.lat_on_get_info.argtypes = [vp, P(u64), P(u64)]
    L.lat_on_profile.argtypes = [vp, i, P(d)]
    L.lat_on_destroy.argtypes = [vp]
    L.lat_on_save.argtypes = [vp, ctypes.c_char_p]
    L.lat_on_load.argtypes = [P(vp), ctypes.c_char_p, P(Options)]
    for name in ("lat_on_save", "lat_on_load", "lat_on_create", "lat_on_sweep", "lat_on_measure", "lat_on_run", "lat_on_acceptance",
                 "lat_on_get_field", "lat_on_set_field", "lat_on_get_info", "lat_on_profile", "lat_on_destroy"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("lat_create", "lat_sweep", "lat_run", "lat_measure", "lat_get_links", "lat_get_links_noalloc", "lat_set_links",
                 "lat_get_rng_state", "lat_get_info", "lat_profile_passes", "lat_autotune", "lat_get_launch_shape", "lat_set_accept_log", "lat_save", "lat_load",
                 "lat_destroy", "lat_philox4x32_10", "lat_batch_create", "lat_batch_run",
                 "lat_batch_get_links", "lat_batch_set_links", "lat_batch_destroy", "lat_batch_configure",
                 "lat_batch_autotune", "lat_batch_get_shape"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(rc: int) -> None:
    if rc != OK:
        raise LatError(rc, lib.lat_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def ncomp(group: int) -> int:
    return 18 if group == 3 else 4


def default_options() -> Options:
    o = Options()
    lib.lat_default_options(ctypes.byref(o))
    return o


def make_options(storage=F64, rng=RNG_PHILOX, rng_const=0.5, start=HOT, seed=1, nhit=10,
                 lattice_id=0, stream=None, device_buffer=None, block_size=0, tile_order=0,
                 layout=0, tile=None, max_waves_per_simd=0, frozen=0, stage_lds=0) -> Options:
    o = default_options()
    o.storage = storage
    o.rng = rng
    o.rng_const = rng_const
    o.start = start
    o.seed = seed
    o.nhit = nhit
    o.lattice_id = lattice_id
    o.block_size = block_size
    o.tile_order = tile_order
    o.layout = layout
    o.max_waves_per_simd = max_waves_per_simd
    o.frozen = frozen
    o.stage_lds = stage_lds
    if tile is not None:
        for k in range(4):
            o.tile[k] = int(tile[k])
    if stream is not None:
        o.stream = stream if isinstance(stream, int) else int(stream.cuda_stream)
    if device_buffer is not None:  # a torch tensor (or any object with data_ptr/nbytes)
        o.device_buffer = int(device_buffer.data_ptr())
        o.device_bytes = int(device_buffer.numel() * device_buffer.element_size())
    return o


def device_bytes(group, dims, **kw) -> int:
    o = make_options(**kw)
    return int(lib.lat_device_bytes(int(group), *map(int, dims), ctypes.byref(o)))


class Lattice:
    """One lattice resident on the GPU.

    Links are exchanged in the canonical FP64 W-frame layout [site][mu][comp]
    (site = x + Nx*(y + Ny*(z + Nz*t)))."""

    def __init__(self, group, dims, beta, flux=0, *, _handle=None, keepalive=None, **opts):
        self.group = int(group)
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        self._keep = keepalive
        self.rng = RNG_PHILOX
        if _handle is not None:
            self._h = _handle
            return
        o = make_options(**opts)
        self.rng = int(o.rng)
        if "device_buffer" in opts and opts["device_buffer"] is not None:
            self._keep = opts["device_buffer"]
        h = ctypes.c_void_p()
        _check(lib.lat_create(ctypes.byref(h), self.group, *self.dims, float(beta), int(flux),
                              ctypes.byref(o)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib.lat_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n_hb=1, n_or=0):
        _check(lib.lat_sweep(self._h, int(n_hb), int(n_or)))

    def run(self, n_sweeps, n_hb=1, n_or=0, measure_every=1):
        k = n_sweeps // measure_every if measure_every > 0 else 0
        p = np.zeros((max(k, 1), 3))
        l = np.zeros((max(k, 1), 2))
        _check(lib.lat_run(self._h, int(n_sweeps), int(n_hb), int(n_or), int(measure_every),
                           _ptr(p), _ptr(l)))
        return p[:k], l[:k]

    def measure(self):
        p = np.zeros(3)
        l = np.zeros(2)
        _check(lib.lat_measure(self._h, _ptr(p), _ptr(l)))
        return p, l

    def get_links(self) -> np.ndarray:
        out = np.empty((self.V, 4, ncomp(self.group)))
        _check(lib.lat_get_links(self._h, _ptr(out), out.size))
        return out

    def get_links_noalloc(self) -> np.ndarray:
        """The same links as get_links, read through the library's fixed
        per-GPU scratch array (no device allocation)."""
        out = np.empty((self.V, 4, ncomp(self.group)))
        _check(lib.lat_get_links_noalloc(self._h, _ptr(out), out.size))
        return out

    def set_links(self, links: np.ndarray) -> None:
        a = np.ascontiguousarray(links, dtype=np.float64)
        _check(lib.lat_set_links(self._h, _ptr(a), a.size))

    def rng_state(self) -> np.ndarray:
        """Per-site generator state words (MRG32k3a: 6, RANLUX: 25)."""
        words = {RNG_MRG32K3A: 6, RNG_RANLUX: 25}.get(self.rng, 6)
        out = np.empty((self.V, words), dtype=np.uint32)
        _check(lib.lat_get_rng_state(self._h, _ptr(out), out.size))
        return out

    def info(self):
        s, hb, sw = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib.lat_get_info(self._h, ctypes.byref(s), ctypes.byref(hb), ctypes.byref(sw)))
        return {"seed": s.value, "hb_sweeps": hb.value, "sweeps": sw.value}

    def profile_passes(self, n_hb=1, n_or=4, reps=3):
        """Average (heat-bath pass ms, overrelaxation pass ms), event-timed."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib.lat_profile_passes(self._h, int(n_hb), int(n_or), int(reps), ctypes.byref(a),
                                      ctypes.byref(b)))
        return a.value, b.value

    def autotune(self, n_hb=1, n_or=4) -> dict:
        """Pick the fastest launch shape for this lattice; the lattice state is
        restored afterwards."""
        r = np.zeros(3, dtype=np.int32)
        _check(lib.lat_autotune(self._h, int(n_hb), int(n_or), _ptr(r)))
        return {"block_size": int(r[0]), "tile_order": int(r[1]), "max_waves_per_simd": int(r[2])}

    def launch_shapes(self) -> dict:
        """Launch shapes of the heat-bath and overrelaxation passes."""
        out = {}
        for kind, name in ((0, "heat_bath"), (1, "overrelaxation")):
            v = np.zeros(8, dtype=np.int32)
            _check(lib.lat_get_launch_shape(self._h, kind, _ptr(v)))
            out[name] = {"block_size": int(v[0]), "tile_order": int(v[1]), "max_waves_per_simd": int(v[2]),
                         "tile": [int(x) for x in v[3:7]], "stage_lds": int(v[7])}
        return out

    def set_accept_log(self, on=True):
        _check(lib.lat_set_accept_log(self._h, int(bool(on))))

    def accept_log(self, max_hb: int = 8) -> np.ndarray:
        out = np.empty(12 * self.V * max_hb, dtype=np.int8)
        n = lib.lat_get_accept_log(self._h, _ptr(out), out.size)
        if n < 0:
            _check(int(n))
        return out[:n].copy()

    def save(self, path: str):
        _check(lib.lat_save(self._h, str(path).encode()))

def load_lattice(path: str, group: int, dims, **opts) -> Lattice:
    h = ctypes.c_void_p()
    o = make_options(**opts) if opts else None
    _check(lib.lat_load(ctypes.byref(h), str(path).encode(), ctypes.byref(o) if o is not None else None))
    return Lattice(group, dims, 0.0, _handle=h)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(c)
    _check(lib.lat_philox4x32_10(_ptr(c), _ptr(k), _ptr(out), c.shape[0]))
    return out


class Batch:
    """Independent lattices advanced together (a coupling or flux scan)."""

    def __init__(self, descs, **common):
        arr = (Desc * len(descs))()
        for k, d in enumerate(descs):
            arr[k].group = int(d["group"])
            arr[k].Nx, arr[k].Ny, arr[k].Nz, arr[k].Nt = map(int, d["dims"])
            arr[k].beta = float(d["beta"])
            arr[k].field_flux = int(d.get("flux", 0))
            arr[k].seed = int(d.get("seed", 1))
            arr[k].start = int(d.get("start", HOT))
            arr[k].lattice_id = int(d.get("lattice_id", k))
        self.descs = list(descs)
        o = make_options(**common)
        h = ctypes.c_void_p()
        _check(lib.lat_batch_create(ctypes.byref(h), len(descs), arr, ctypes.byref(o)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib.lat_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_sweeps, n_hb=1, n_or=0, measure=True):
        n = len(self.descs)
        p = np.zeros((n, 3))
        l = np.zeros((n, 2))
        _check(lib.lat_batch_run(self._h, int(n_sweeps), int(n_hb), int(n_or),
                                 _ptr(p) if measure else None, _ptr(l) if measure else None))
        return p, l

    def configure(self, mode=0, block_size=256, sites_per_thread=1, grid=0):
        """mode 0: one launch per pass over all members, each member whole on
        one XCD; 2: the same with the members' tiles dealt round the XCDs;
        1 (persistent work list) is refused with LAT_EUNSUPPORTED."""
        _check(lib.lat_batch_configure(self._h, int(mode), int(block_size), int(sites_per_thread), int(grid)))

    def autotune(self, n_hb=1, n_or=4) -> dict:
        r = np.zeros(2, dtype=np.int32)
        _check(lib.lat_batch_autotune(self._h, int(n_hb), int(n_or), _ptr(r)))
        return {"block_size": int(r[0]), "sites_per_thread": int(r[1]), "xcd_map": self.shape()["xcd_map"]}

    def shape(self) -> dict:
        r = np.zeros(3, dtype=np.int32)
        _check(lib.lat_batch_get_shape(self._h, _ptr(r)))
        return {"block_size": int(r[0]), "sites_per_thread": int(r[1]), "xcd_map": int(r[2])}

    def get_links(self, i) -> np.ndarray:
        d = self.descs[i]
        V = int(np.prod(d["dims"]))
        out = np.empty((V, 4, ncomp(d["group"])))
        _check(lib.lat_batch_get_links(self._h, int(i), _ptr(out), out.size))
        return out

    def set_links(self, i, links) -> None:
        a = np.ascontiguousarray(links, dtype=np.float64)
        _check(lib.lat_batch_set_links(self._h, int(i), _ptr(a), a.size))


def on_device_bytes(ncomp, dims, **kw) -> int:
    kw.setdefault("nhit", 100)
    o = make_options(**kw)
    return int(lib.lat_on_device_bytes(int(ncomp), *[int(x) for x in dims], ctypes.byref(o)))


class ONField:
    """An O(N) phi^4 field (N = 1..4) on the GPU: ``lat_on_*`` of the C ABI.
    The field is exchanged as FP64 ``[site][component]``; ``measure()``
    returns (<phi^2>, <phi(x).phi(x+mu)>, <(phi^2-1)^2>, <phi_0>, .., <phi_3>)."""

    def __init__(self, ncomp, dims, kappa, lam, h=0.0, delta=1.0, storage=F64, rng=RNG_PHILOX,
                 rng_const=0.5, seed=1, nhit=100, lattice_id=0, start=HOT, stream=None, block_size=0):
        self.n = int(ncomp)
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        o = make_options(storage=storage, rng=rng, rng_const=rng_const, start=start, seed=seed, nhit=nhit,
                         lattice_id=lattice_id, stream=stream, block_size=block_size)
        h_ = ctypes.c_void_p()
        _check(lib.lat_on_create(ctypes.byref(h_), self.n, *self.dims, float(kappa), float(lam), float(h),
                                 float(delta), ctypes.byref(o)))
        self._h = h_

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.lat_on_destroy(self._h)
            self._h = None

    __del__ = close

    def sweep(self, n=1):
        _check(lib.lat_on_sweep(self._h, int(n)))

    def measure(self) -> np.ndarray:
        out = np.zeros(7)
        _check(lib.lat_on_measure(self._h, _ptr(out)))
        return out

    def run(self, n_sweeps, measure_every=1) -> np.ndarray:
        k = n_sweeps // measure_every if measure_every else 0
        out = np.zeros((max(k, 1), 7))
        _check(lib.lat_on_run(self._h, int(n_sweeps), int(measure_every), _ptr(out)))
        return out[:k]

    def acceptance(self) -> float:
        r = ctypes.c_double()
        _check(lib.lat_on_acceptance(self._h, ctypes.byref(r)))
        return r.value

    def get_field(self) -> np.ndarray:
        out = np.empty((self.V, self.n))
        _check(lib.lat_on_get_field(self._h, _ptr(out), out.size))
        return out

    def set_field(self, phi) -> None:
        a = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.V, self.n)
        _check(lib.lat_on_set_field(self._h, _ptr(a), a.size))

    def info(self):
        s, w = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib.lat_on_get_info(self._h, ctypes.byref(s), ctypes.byref(w)))
        return {"seed": s.value, "sweeps": w.value}

    def save(self, path) -> None:
        _check(lib.lat_on_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path, storage=None, stream=None):
        """Continue a saved O(N) chain (storage from the file unless given)."""
        with open(path, "rb") as fh:
            head = struct.unpack("<8s12I", fh.read(8 + 4 * 12))
        self = cls.__new__(cls)
        self.n = int(head[2])
        self.dims = tuple(int(x) for x in head[3:7])
        self.V = int(np.prod(self.dims))
        h_ = ctypes.c_void_p()
        if storage is None and stream is None:
            _check(lib.lat_on_load(ctypes.byref(h_), os.fsencode(path), None))
        else:
            o = make_options(storage=F64 if storage is None else storage, stream=stream)
            _check(lib.lat_on_load(ctypes.byref(h_), os.fsencode(path), ctypes.byref(o)))
        self._h = h_
        return self

    def profile(self, reps) -> float:
        """Average milliseconds per pass (half a sweep) over `reps` sweeps."""
        ms = ctypes.c_double()
        _check(lib.lat_on_profile(self._h, int(reps), ctypes.byref(ms)))
        return ms.value
