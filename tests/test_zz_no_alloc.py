"""ebc_compress_async_noalloc (the entry point whose workspace is the
library's fixed device array) against ebc_compress_async with a caller
workspace and against the oracle: archive bytes equal on consecutive calls,
the later ones on smaller fields (the array keeps the earlier call's
contents), and a field too large for the array refused before any device
work."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    from paper_2105_12912_amd import ebc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ebc.lib()
    return ebc


def result_of(res):
    """(size, status) from the 16-byte device result of the async calls."""
    h = res.cpu().numpy()
    size = int(h[0])
    status = int(np.array([h[1]], np.int64).view(np.int32)[0])
    return size, status


def compress_both(E, x, eb):
    """The same field through both entry points on the current stream;
    returns the two archives as bytes."""
    rank, dims = E.field_rank_dims(x)
    p = E.make_params(eb, dtype=E._dtype_code(x))
    bound = E.ebc_compress_bound(rank, dims, p)
    stream = E._stream_handle()
    out_a = torch.empty(bound, dtype=torch.uint8, device=x.device)
    res_a = torch.zeros(2, dtype=torch.int64, device=x.device)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    st = E.ebc_compress_async_noalloc(x.data_ptr(), rank, dims, p, out_a.data_ptr(), bound,
                                      res_a.data_ptr(), stream)
    assert st == 0, E.ebc_last_error()
    assert torch.cuda.memory_allocated() == before
    size_a, st_a = result_of(res_a)
    assert st_a == 0 and size_a > 0

    wsz = E.ebc_compress_workspace_size(rank, dims, p)
    ws = torch.empty(wsz, dtype=torch.uint8, device=x.device)
    out_b = torch.empty(bound, dtype=torch.uint8, device=x.device)
    res_b = torch.zeros(2, dtype=torch.int64, device=x.device)
    st = E.ebc_compress_async(x.data_ptr(), rank, dims, p, out_b.data_ptr(), bound,
                              res_b.data_ptr(), ws.data_ptr(), wsz, stream)
    assert st == 0, E.ebc_last_error()
    size_b, st_b = result_of(res_b)
    assert st_b == 0
    return out_a[:size_a].cpu().numpy().tobytes(), out_b[:size_b].cpu().numpy().tobytes()


def test_noalloc_matches_workspace_entry_point(E):
    fields = [
        ("2D 1800x3600 rel 1e-4", synth.climate_2d(), 1e-4),
        ("3D 96^3 lognormal rel 1e-3", synth.lognormal_3d((96, 96, 96), 31), 1e-3),
        ("2D 256x256 rel 1e-4", synth.smooth_2d(256, 256, 1), 1e-4),
        ("2D 128x160 fp64 rel 1e-7", synth.smooth_2d(128, 160, 2).astype(np.float64) * 1e3, 1e-7),
    ]
    sizes = [x.nbytes for _, x, _ in fields]
    assert sizes == sorted(sizes, reverse=True)  # each call smaller than the one before
    for label, x, eb in fields:
        print(f"[noalloc] {label}", flush=True)
        xm = torch.empty(x.shape, dtype=torch.float64 if x.dtype == np.float64 else torch.float32,
                         device="meta")
        rank, dims = E.field_rank_dims(xm)
        need = E.ebc_compress_workspace_size(rank, dims, E.make_params(eb, dtype=E._dtype_code(xm)))
        assert need <= E.EBC_NOALLOC_SCRATCH_BYTES
        a, b = compress_both(E, torch.from_numpy(x).cuda(), eb)
        assert a == b
        assert a == O.compress(x, eb)


def test_noalloc_refuses_a_field_beyond_the_array(E):
    p = E.make_params(1e-4)
    n = 12_000_000
    dims = (n, 1, 1)
    need = E.ebc_compress_workspace_size(1, dims, p)
    assert need > E.EBC_NOALLOC_SCRATCH_BYTES
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    bound = E.ebc_compress_bound(1, dims, p)
    out = torch.full((bound,), 7, dtype=torch.uint8, device="cuda")
    res = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    st = E.ebc_compress_async_noalloc(x.data_ptr(), 1, dims, p, out.data_ptr(), bound,
                                      res.data_ptr(), E._stream_handle())
    assert st == E.EBC_ERR_WS_TOO_SMALL
    assert "fixed array" in E.ebc_last_error()
    torch.cuda.synchronize()
    # nothing ran on the device
    assert int(res[0]) == -1 and int(out[:128].sum()) == 7 * 128
