"""The allocation-free link read-out (lat_get_links_noalloc) against the
ordinary one (lat_get_links), through the C ABI: bit-identical links on two
calls in a row, the second on a smaller lattice, plus a lattice that needs
more than one chunk of the fixed scratch array and the rejected sizes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")


def _case(group, dims, storage, beta):
    print(f"no-alloc read-out: SU({group}) {dims} storage {P.STORAGE_NAMES[storage]}", flush=True)
    g = P.Lattice(group, dims, beta, 1, storage=storage, seed=13, start=P.HOT)
    g.sweep(1, 1)
    want = g.get_links()
    got = g.get_links_noalloc()
    assert np.array_equal(got, want)
    g.close()


def test_noalloc_read_out_equals_get_links():
    # 16^3x8 SU(3): 32768 sites of 576 B, more than one 16 MiB chunk
    assert 16 ** 3 * 8 * 4 * 18 * 8 > P.NOALLOC_SCRATCH_BYTES
    _case(3, (16, 16, 16, 8), P.F64, 5.9)
    # a second call, smaller lattice, other group and storage
    _case(2, (6, 4, 4, 2), P.F32, 2.3)
    _case(3, (4, 4, 4, 2), P.F32_C12, 5.7)


def test_noalloc_read_out_rejects_wrong_sizes():
    g = P.Lattice(3, (4, 4, 4, 2), 5.7, seed=1)
    out = np.empty(g.V * 4 * 18 - 1)
    rc = P.lib.lat_get_links_noalloc(g._h, out.ctypes.data, out.size)
    assert rc == P.EINVAL and b"need" in P.lib.lat_last_error()
    assert P.lib.lat_get_links_noalloc(g._h, None, g.V * 4 * 18) == P.EINVAL
    g.close()
