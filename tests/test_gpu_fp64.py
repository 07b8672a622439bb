"""GPU parity of fp64 fields (Sec. III: fp64 through the same integer core):
archive bytes and reconstructed doubles (as bit patterns) equal to the
oracle's, every element within the bound, for every rank, ragged and
unaligned shapes, outlier-heavy fields (the 3D fix-up path), constant
fields and the error paths."""
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def field64(shape, seed, kind="smooth"):
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.standard_normal(shape)
    x = synth.grf_field(shape, seed).astype(np.float64) if len(shape) > 1 else \
        synth.random_walk_1d(shape[0], seed).astype(np.float64)
    return x * 1e3 + rng.standard_normal(shape) * 1e-6  # fp64 detail below fp32 resolution


CASES = [
    ("1d", (100_003,), "smooth", 1e-7, 1024),
    ("2d", (300, 257), "smooth", 1e-6, 1024),
    ("2d_narrow", (500, 6), "smooth", 1e-5, 1024),
    ("3d", (40, 48, 64), "smooth", 1e-6, 1024),
    ("3d_ragged", (9, 10, 11), "smooth", 1e-4, 1024),
    ("3d_noise", (24, 40, 33), "noise", 1e-4, 64),
    ("2d_noise", (70, 90), "noise", 1e-7, 4096),
    # above 4096 bins: histogram window, codebook and tables in HBM
    ("2d_noise_65536", (200, 150), "noise", 1e-7, 65536),
    ("3d_smooth_16384", (24, 40, 33), "smooth", 1e-8, 16384),
]


@pytest.mark.parametrize("name,shape,kind,eb,nb", CASES, ids=[c[0] for c in CASES])
def test_fp64_bytes_and_roundtrip(E, name, shape, kind, eb, nb):
    x = field64(shape, 5, kind)
    ref = O.compress(x, eb, n_bins=nb)
    assert O.archive_info(ref)["dtype"] == O.DT_F64
    a = E.compress(dev(x), eb, n_bins=nb)
    assert a.cpu().numpy().tobytes() == ref
    y = E.decompress(a)
    assert y.dtype == torch.float64
    yh = y.cpu().numpy()
    np.testing.assert_array_equal(yh.view(np.uint64), O.decompress(ref).view(np.uint64))
    assert float(np.abs(yh - x).max()) <= eb * (float(x.max()) - float(x.min()))


def test_fp64_unaligned_rows(E):
    """Rows whose start is not 16-byte aligned take the element-wise paths."""
    x = field64((33, 45, 27), 6)
    buf = torch.empty(x.size + 1, dtype=torch.float64, device="cuda")
    v = buf[1:].view(x.shape)
    v.copy_(dev(x))
    ref = O.compress(x, 1e-6)
    a = E.compress(v, 1e-6)
    assert a.cpu().numpy().tobytes() == ref
    out = torch.empty(x.size + 1, dtype=torch.float64, device="cuda")[1:].view(x.shape)
    y = E.decompress(a, out=out)
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint64), O.decompress(ref).view(np.uint64))


def test_fp64_codecs(E):
    x = synth.lognormal_3d((32, 40, 48), 7).astype(np.float64)
    for codec in ("rle", "rle_vle", "huffman"):
        ref = O.compress(x, 3e-2, codec=codec)
        a = E.compress(dev(x), 3e-2, codec=codec)
        assert a.cpu().numpy().tobytes() == ref, codec
        np.testing.assert_array_equal(E.decompress(a).cpu().numpy().view(np.uint64),
                                      O.decompress(ref).view(np.uint64))


def test_fp64_constant_and_errors(E):
    c = np.full((20, 30), np.pi)
    a = E.compress(dev(c), 1e-3)
    assert a.cpu().numpy().tobytes() == O.compress(c, 1e-3)
    y = E.decompress(a)
    assert y.dtype == torch.float64 and bool((y == np.pi).all())
    z = np.linspace(-1, 1, 1000)
    z[7] = np.inf
    with pytest.raises(E.EbcError) as ei:
        E.compress(dev(z), 1e-3)
    assert ei.value.status == E.EBC_ERR_NONFINITE
    # codes beyond the int32 range of the Lorenzo arithmetic
    with pytest.raises(E.EbcError) as ei:
        E.compress(dev(np.linspace(-1, 1, 1000)), 2.0 ** -40, "abs")
    assert ei.value.status == E.EBC_ERR_EB_TOO_SMALL
    assert O.compress_status(np.linspace(-1, 1, 1000), 2.0 ** -40, "abs") == -4


def test_fp64_batch(E):
    from paper_2105_12912_amd import batch

    xs = [field64((50_000,), 8), field64((90, 120), 9), field64((20, 24, 28), 10)]
    B = batch.BatchCompress([dev(x) for x in xs], 1e-6)
    B.launch()
    torch.cuda.synchronize()
    arcs = B.archives()
    for x, a in zip(xs, arcs):
        assert a.cpu().numpy().tobytes() == O.compress(x, 1e-6)
    D = batch.BatchDecompress(arcs)
    D.launch()
    torch.cuda.synchronize()
    assert D.statuses() == [0, 0, 0]
    for x, y, a in zip(xs, D.outs, arcs):
        assert y.dtype == torch.float64
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint64),
                                      O.decompress(a.cpu().numpy().tobytes()).view(np.uint64))
