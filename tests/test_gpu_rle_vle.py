"""GPU parity of the RLE+VLE workflow: run-length coding whose run values are
Huffman-coded with a codebook of their own (Sec. III-A, "RLE with optional
VLE"), forced or chosen by the 1.09-bit rule.  Archive bytes and
reconstructed floats must equal the oracle's exactly."""
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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def check(E, x, eb, codec, hc=1024, n_bins=1024, want_codec=None):
    ref = O.compress(x, eb, codec=codec, hc=hc, n_bins=n_bins)
    if want_codec is not None:
        assert O.archive_info(ref)["codec"] == want_codec
    a = E.compress(dev(x), eb, codec=codec, huff_chunk=hc, n_bins=n_bins)
    assert a.cpu().numpy().tobytes() == ref
    y = E.decompress(a)
    np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(O.decompress(ref)))
    return ref


CASES = [
    ("3d_lognormal", lambda: synth.lognormal_3d((48, 64, 80), 3), 3e-2),
    ("2d_smooth", lambda: synth.smooth_2d(300, 200, 5), 1e-3),
    ("1d_walk", lambda: synth.random_walk_1d(300_001, 6), 1e-3),
    ("2d_noise", lambda: np.random.default_rng(7).standard_normal((90, 70)).astype(np.float32), 1e-2),
    ("1d_tiny", lambda: np.array([1.0, 1.0, 2.0, 2.0, 2.0, -1.0, 5.0], np.float32), 1e-3),
]


@pytest.mark.parametrize("name,make,eb", CASES, ids=[c[0] for c in CASES])
def test_forced_rle_vle_bytes(E, name, make, eb):
    check(E, make(), eb, "rle_vle", want_codec=O.ARC_RLE_VLE)


@pytest.mark.parametrize("hc", [64, 256, 4096])
def test_rle_vle_chunk_sizes(E, hc):
    x = synth.lognormal_3d((40, 48, 56), 8)
    check(E, x, 3e-2, "rle_vle", hc=hc, want_codec=O.ARC_RLE_VLE)


def test_auto_vle_picks_rle_vle_by_the_rule(E):
    """A field whose codes average <= 1.09 bits goes to the run-length branch
    with VLE on; one above it stays Huffman-coded."""
    x = synth.lognormal_3d((48, 64, 80), 3)
    check(E, x, 3e-2, "auto_vle", want_codec=O.ARC_RLE_VLE)
    check(E, x, 1e-3, "auto_vle", want_codec=O.ARC_HUFFMAN)


def test_rle_vle_many_runs_and_bins(E):
    """Noise at a tight bound: about one run per element (the value stream is
    nearly as long as the field) and 4096 bins."""
    x = np.random.default_rng(9).standard_normal(2_000_003).astype(np.float32)
    ref = check(E, x, 1e-3, "rle_vle", n_bins=4096, want_codec=O.ARC_RLE_VLE)
    assert O.archive_info(ref)["n_a"] > 1_900_000


@pytest.mark.parametrize("name,make,eb,nb", [
    ("3d_lognormal_16384", lambda: synth.lognormal_3d((48, 64, 80), 3), 3e-2, 16384),
    ("1d_noise_65536", lambda: np.random.default_rng(10).standard_normal(500_001).astype(np.float32),
     1e-5, 65536),
], ids=["3d_lognormal_16384", "1d_noise_65536"])
def test_rle_vle_wide_bins(E, name, make, eb, nb):
    """Above 4096 bins: the run-value histogram's LDS window and HBM counts,
    and the second (run-value) codebook built in HBM."""
    check(E, make(), eb, "rle_vle", n_bins=nb, want_codec=O.ARC_RLE_VLE)


def test_rle_vle_in_a_batch(E):
    """Fields of mixed rank through the batched entry point with VLE on: each
    archive equal to the oracle's (codec chosen per field)."""
    from paper_2105_12912_amd import batch

    xs = [synth.lognormal_3d((24, 40, 33), 11), synth.smooth_2d(120, 90, 12),
          synth.random_walk_1d(70_000, 13)]
    B = batch.BatchCompress([dev(x) for x in xs], 3e-2, codec="auto_vle")
    B.launch()
    torch.cuda.synchronize()
    for x, a in zip(xs, B.archives()):
        assert a.cpu().numpy().tobytes() == O.compress(x, 3e-2, codec="auto_vle")


def test_corrupt_rle_vle_rejected(E):
    x = synth.lognormal_3d((40, 48, 56), 8)
    raw = np.frombuffer(O.compress(x, 3e-2, codec="rle_vle"), np.uint8).copy()
    s = O.sections(raw.tobytes())
    R = s["info"]["n_a"]
    for mutate in ("sbits", "rlen"):
        b = raw.copy()
        if mutate == "sbits":
            o = s["layout"]["sbits"]
            v = int(b[o:o + 2].view(np.uint16)[0]) + 1
            b[o:o + 2] = np.frombuffer(np.uint16(v).tobytes(), np.uint8)
        else:
            o = s["off_rlen"]
            L = b[o:o + 4 * R].view(np.uint32).copy()
            L[0] += 1  # runs no longer cover the field exactly
            b[o:o + 4 * R] = L.view(np.uint8)
        assert O.decompress_status(b.tobytes()) == -9, mutate
        assert E.decompress_status(dev(b)) == E.EBC_ERR_ARCHIVE, mutate
