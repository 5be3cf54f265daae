"""GPU tests of the LDS-staged pass (the opposite-parity U_mu links of each
4-D work-group tile copied to LDS first): bit-identical links to the plain
pass for every storage form, tile shape and work-group order, including
tiles at the periodic boundaries, and refusal of tiles that do not divide
the lattice."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")


@pytest.mark.parametrize("storage", [P.F64, P.F32, P.F32_C12, P.F64_C12])
@pytest.mark.parametrize("dims,tile,order", [
    ((16, 8, 8, 4), (8, 4, 4, 2), 4), ((16, 8, 8, 4), (4, 4, 4, 4), 1), ((8, 8, 16, 8), (4, 4, 2, 8), 4),
    ((4, 16, 4, 8), (2, 8, 2, 8), 1), ((16, 16, 16, 4), (8, 4, 2, 4), 4)])
def test_staged_pass_equals_plain_pass(storage, dims, tile, order):
    print(f"LDS-staged pass: SU(3) {dims} tile {tile} order {order} storage {P.STORAGE_NAMES[storage]}",
          flush=True)
    a = P.Lattice(3, dims, 5.8, 1, storage=storage, seed=31, start=P.HOT)
    b = P.Lattice(3, dims, 5.8, 1, storage=storage, seed=31, start=P.HOT, tile=tile, tile_order=order,
                  stage_lds=1)
    for _ in range(2):
        a.sweep(1, 4)
        b.sweep(1, 4)
    assert np.array_equal(a.get_links(), b.get_links())
    pa, la = a.measure()
    pb, lb = b.measure()
    assert np.array_equal(pa, pb) and np.array_equal(la, lb)


def test_staged_pass_accept_log_and_mrg():
    a = P.Lattice(3, (8, 8, 8, 4), 5.7, 0, rng=P.RNG_MRG32K3A, seed=5, start=P.HOT)
    b = P.Lattice(3, (8, 8, 8, 4), 5.7, 0, rng=P.RNG_MRG32K3A, seed=5, start=P.HOT, tile=(4, 4, 4, 4),
                  tile_order=1, stage_lds=1)
    a.set_accept_log(True)
    b.set_accept_log(True)
    a.sweep(2, 1)
    b.sweep(2, 1)
    assert np.array_equal(a.accept_log(), b.accept_log())
    assert np.array_equal(a.rng_state(), b.rng_state())
    assert np.array_equal(a.get_links(), b.get_links())


def test_staged_pass_refuses_tiles_that_do_not_divide():
    with pytest.raises(P.LatError) as e:
        P.Lattice(3, (12, 8, 8, 4), 5.7, 0, tile=(4, 4, 4, 4), stage_lds=1)
    assert e.value.code == P.EINVAL
    with pytest.raises(P.LatError):
        P.Lattice(3, (8, 8, 8, 4), 5.7, 0, stage_lds=1)  # no tile
    with pytest.raises(P.LatError):
        P.Lattice(2, (8, 8, 8, 4), 2.3, 0, tile=(4, 4, 4, 4), stage_lds=1)  # SU(2)
