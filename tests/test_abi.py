"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lat_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lat_create", "lat_sweep", "lat_measure", "lat_run", "lat_get_links", "lat_set_links",
                 "lat_save", "lat_load", "lat_destroy", "lat_last_error", "lat_batch_create",
                 "lat_batch_run", "lat_batch_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1310_7087_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options():
    import paper_1310_7087_amd as P
    o = P.default_options()
    assert (o.storage, o.rng, o.start, o.nhit, o.seed) == (P.F64, P.RNG_PHILOX, P.HOT, 10, 0)
    assert o.rng_const == 0.5 and o.stream is None and o.device_buffer is None


def test_device_bytes_layout():
    import paper_1310_7087_amd as P
    # 32^3 x 8 SU(3): links are 4 V * (144 | 72 | 48) bytes plus small scratch
    V = 32 ** 3 * 8
    for st, b in ((P.F64, 144), (P.F32, 72), (P.F32_C12, 48), (P.F64_C12, 96)):
        n = P.device_bytes(3, (32, 32, 32, 8), storage=st)
        assert 4 * V * b <= n < 4 * V * b + (1 << 20)
    # MRG state adds 24 bytes per site
    a = P.device_bytes(2, (4, 4, 4, 4), rng=P.RNG_PHILOX)
    b = P.device_bytes(2, (4, 4, 4, 4), rng=P.RNG_MRG32K3A)
    assert b - a >= 24 * 256
    assert P.device_bytes(3, (3, 4, 4, 4)) == 0
    assert P.device_bytes(2, (4, 4, 4, 4), storage=P.F32_C12) == 0


@pytest.mark.parametrize("group,dims,beta,kw,code", [
    (3, (3, 4, 4, 4), 5.7, {}, -1),
    (3, (4, 4, 4, 0), 5.7, {}, -1),
    (4, (4, 4, 4, 4), 5.7, {}, -1),
    (3, (4, 4, 4, 4), -1.0, {}, -1),
    (3, (4, 4, 4, 4), float("nan"), {}, -1),
    (3, (4, 4, 4, 4), 5.7, {"nhit": 0}, -1),
    (3, (4, 4, 4, 4), 5.7, {"nhit": 128}, -1),
    (3, (4, 4, 4, 4), 5.7, {"rng": 7}, -1),
    (3, (4, 4, 4, 4), 5.7, {"rng": 2, "rng_const": 1.0}, -1),
    (3, (4, 4, 4, 4), 5.7, {"rng": 2, "start": 1}, -1),
    (3, (4, 4, 4, 4), 5.7, {"block_size": 100}, -1),
    (2, (4, 4, 4, 4), 2.3, {"storage": 2}, -7),
    (2, (4, 4, 4, 4), 2.3, {"storage": 3}, -7),
    (3, (4, 4, 4, 4), 5.7, {"storage": 4}, -1),
    (3, (4, 4, 4, 4), 5.7, {"frozen": 2}, -1),
    (2, (4, 4, 4, 4), 2.3, {"rng": 0, "seed": 4294944443}, -1),
])
def test_create_rejects_bad_arguments_without_a_device(group, dims, beta, kw, code):
    import paper_1310_7087_amd as P
    with pytest.raises(P.LatError) as e:
        P.Lattice(group, dims, beta, **kw)
    assert e.value.code == code
    assert P.lib.lat_last_error().decode()


def test_null_handles_are_errors_or_noops():
    import paper_1310_7087_amd as P
    assert P.lib.lat_destroy(None) == 0
    assert P.lib.lat_batch_destroy(None) == 0
    assert P.lib.lat_sweep(None, 1, 0) == -1
    assert P.lib.lat_measure(None, None, None) == -1


def test_load_rejects_missing_and_corrupt_files(tmp_path):
    import paper_1310_7087_amd as P
    h = ctypes.c_void_p()
    assert P.lib.lat_load(ctypes.byref(h), str(tmp_path / "none").encode(), None) == P.EIO
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"NOTACKPT" + b"\0" * 200)
    assert P.lib.lat_load(ctypes.byref(h), str(bad).encode(), None) == P.ECORRUPT


def test_maximum_sizes():
    """Per-thread link addresses are 32-bit byte offsets within one plane of
    the half lattice: the largest accepted lattice keeps a plane below 4 GiB
    (SU(3) FP64 128^4 = 154 GB of links, within one GPU's 288 GB); one step
    beyond is rejected before any device call."""
    import paper_1310_7087_amd as P
    V = 128 ** 4
    n = P.device_bytes(3, (128, 128, 128, 128))
    assert 4 * V * 144 <= n < 4 * V * 144 + (1 << 30)
    assert P.device_bytes(3, (256, 128, 128, 128)) == 0
    assert P.device_bytes(3, (256, 128, 128, 128), storage=P.F32_C12) == 0
    assert P.device_bytes(3, (256, 128, 128, 128), storage=P.F32) > 0
    with pytest.raises(P.LatError) as e:
        P.Lattice(3, (256, 128, 128, 128), 6.0)
    assert e.value.code == P.EINVAL and "32-bit" in P.lib.lat_last_error().decode()


@pytest.mark.parametrize("descs,kw,code", [
    ([], {}, -1),
    ([dict(group=3, dims=(4, 4, 4, 4), beta=5.7), dict(group=3, dims=(4, 5, 4, 4), beta=5.7)], {}, -1),
    ([dict(group=4, dims=(4, 4, 4, 4), beta=5.7)], {}, -1),
    ([dict(group=2, dims=(4, 4, 4, 4), beta=float("nan"))], {}, -1),
    ([dict(group=3, dims=(4, 4, 4, 0), beta=5.7)], {}, -1),
    ([dict(group=3, dims=(4, 4, 4, 4), beta=5.7)], {"rng": 0}, -7),
])
def test_batch_rejects_bad_members_without_a_device(descs, kw, code):
    """An empty batch, a member with an odd or zero extent, a bad group or
    coupling, or a generator other than Philox is refused before any device
    call (this host has no GPU)."""
    import paper_1310_7087_amd as P
    with pytest.raises(P.LatError) as e:
        P.Batch(descs, **kw)
    assert e.value.code == code


def test_batch_rejects_frozen_links_without_a_device():
    import paper_1310_7087_amd as P
    with pytest.raises(P.LatError) as e:
        P.Batch([dict(group=3, dims=(4, 4, 4, 4), beta=5.7)], frozen=P.FROZEN_T0)
    assert e.value.code == P.EUNSUPPORTED


def test_o_n_layout_and_rejections_without_a_device():
    import paper_1310_7087_amd as P
    V = 32 ** 4
    for st, b in ((P.F64, 8), (P.F32, 4)):
        n = P.on_device_bytes(4, (32, 32, 32, 32), storage=st)
        assert 4 * V * b <= n < 4 * V * b + (1 << 20)
    # RANLUX keeps 25 words per site
    assert P.on_device_bytes(4, (8, 8, 8, 8), rng=P.RNG_RANLUX) - P.on_device_bytes(4, (8, 8, 8, 8)) >= 100 * 8 ** 4
    assert P.on_device_bytes(5, (4, 4, 4, 4)) == 0
    assert P.on_device_bytes(4, (3, 4, 4, 4)) == 0
    assert P.on_device_bytes(4, (4, 4, 4, 4), storage=P.F32_C12) == 0
    # MRG32k3a keeps 6 words per site
    assert P.on_device_bytes(4, (8, 8, 8, 8), rng=P.RNG_MRG32K3A) - P.on_device_bytes(4, (8, 8, 8, 8)) >= 24 * 8 ** 4
    assert P.on_device_bytes(4, (4, 4, 4, 4), nhit=1001) == 0
    for kw, code in (({"ncomp": 0}, P.EINVAL), ({"dims": (4, 4, 4, 5)}, P.EINVAL), ({"lam": -0.1}, P.EINVAL),
                     ({"delta": 0.0}, P.EINVAL), ({"kappa": float("nan")}, P.EINVAL),
                     ({"storage": P.F64_C12}, P.EUNSUPPORTED), ({"rng": 7}, P.EINVAL),
                     ({"rng": P.RNG_MRG32K3A, "seed": 4294944443}, P.EINVAL),
                     ({"nhit": 0}, P.EINVAL)):
        args = dict(ncomp=4, dims=(4, 4, 4, 4), kappa=0.1, lam=0.1, delta=1.0)
        args.update(kw)
        with pytest.raises(P.LatError) as e:
            P.ONField(args.pop("ncomp"), args.pop("dims"), args.pop("kappa"), args.pop("lam"), **args)
        assert e.value.code == code, kw


def test_loaders_reject_corrupt_files_without_a_device(tmp_path):
    """Checkpoint readers check header, size and checksum before any device
    call: garbage, an empty file and a truncated header give LAT_ECORRUPT,
    a missing file LAT_EIO."""
    import ctypes
    import paper_1310_7087_amd as P
    bad = tmp_path / "bad.ckpt"
    cases = [(b"", P.ECORRUPT), (b"LATCKPT1" + b"\x02\x00\x00\x00", P.ECORRUPT),
             (bytes(range(256)) * 4, P.ECORRUPT)]
    for raw, code in cases:
        bad.write_bytes(raw)
        h = ctypes.c_void_p()
        assert P.lib.lat_load(ctypes.byref(h), str(bad).encode(), None) == code
        assert P.lib.lat_on_load(ctypes.byref(h), str(bad).encode(), None) == code
        assert not h.value
    h = ctypes.c_void_p()
    assert P.lib.lat_load(ctypes.byref(h), str(tmp_path / "missing").encode(), None) == P.EIO
    assert P.lib.lat_on_load(ctypes.byref(h), str(tmp_path / "missing").encode(), None) == P.EIO
