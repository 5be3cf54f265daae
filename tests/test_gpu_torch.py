"""PyTorch as the provider of device memory and streams: a lattice whose
whole device state lives in a torch tensor and whose work is queued on
torch's current stream runs the same Markov chain, bit for bit, as a lattice
that owns its memory and stream; torch work queued after the sweeps on the
same stream sees the finished links."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("storage", [P.F64, P.F32_C12])
def test_torch_buffer_and_stream_equal_library_owned(storage):
    dims, beta = (8, 8, 8, 4), 5.8
    print(f"torch-owned lattice: SU(3) {dims} storage {P.STORAGE_NAMES[storage]}", flush=True)
    nbytes = P.device_bytes(3, dims, storage=storage)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    off = (-buf.data_ptr()) % 256  # the library needs 256-byte alignment
    view = buf[off:off + nbytes]
    side = torch.cuda.Stream()  # default priority
    with torch.cuda.stream(side):
        stream = torch.cuda.current_stream()
        assert stream.cuda_stream != 0  # a real stream, not the null stream
        a = P.Lattice(3, dims, beta, 1, storage=storage, seed=21, start=P.HOT, stream=stream,
                      device_buffer=view)
        b = P.Lattice(3, dims, beta, 1, storage=storage, seed=21, start=P.HOT)
        # torch work on the same stream between the library's graph launches
        scratch = torch.zeros(1 << 20, device="cuda:0")
        for k in range(3):
            a.sweep(1, 4)
            scratch.add_(1.0)
            b.sweep(1, 4)
        pa, la = a.run(4, 1, 4, measure_every=2)
        pb, lb = b.run(4, 1, 4, measure_every=2)
        assert np.array_equal(pa, pb) and np.array_equal(la, lb)
        assert np.array_equal(a.get_links(), b.get_links())
        assert float(scratch[0]) == 3.0
        # the link planes are in the tensor: a checksum taken by torch on the
        # stream changes when the library sweeps
        before = view.to(torch.int64).sum().item()
        a.sweep(1, 0)
        after = view.to(torch.int64).sum().item()
        assert before != after
    torch.cuda.synchronize()
    a.close()
    b.close()
    del view, buf
