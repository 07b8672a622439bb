"""GPU parity on the remaining benchmark configurations and on the decision
threshold, at full size: archive bytes and reconstruction bits equal to the
oracle's.

* the 512^3 lognormal field at rel 1e-3 (its second bound);
* a 1D random walk of 280,953,867 values (the HACC length of the dataset
  table, the largest 1D member of the 64-field batch);
* a 1.2e8-value field that the 1.09-bit rule sends to run-length coding;
* two fields whose codebooks cost exactly 1.09 N and 1.09 N + 1 bits, on
  either side of the rule (Sec. III-B.2: RLE when <b> is at most 1.09)."""
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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def full_parity(E, x, eb, label, want_codec=None):
    print(f"[{label}] oracle", flush=True)
    ref = O.compress(x, eb)
    if want_codec is not None:
        assert O.archive_info(ref)["codec"] == want_codec
    print(f"[{label}] gpu", flush=True)
    xd = torch.from_numpy(x).cuda()
    a = E.compress(xd, eb)
    got = a.cpu().numpy().tobytes()
    assert len(got) == len(ref) and got == ref
    del xd
    y = E.decompress(a)
    print(f"[{label}] oracle decompress", flush=True)
    np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(O.decompress(ref)))


def test_nyx512_rel_1e3(E):
    import bench

    _, gen, eb = bench.WORKLOADS["nyx512_1e-3"]
    full_parity(E, gen(synth), eb, "512^3 1e-3")


def test_hacc_length_random_walk(E):
    x = synth.random_walk_1d(280_953_867, 4004)
    full_parity(E, x, 1e-4, "1D 280953867")


def test_large_field_auto_rle(E):
    x = synth.sparse_background_1d(120_000_000)
    full_parity(E, x, 1e-2, "1.2e8 sparse background", want_codec=O.ARC_RLE)


def threshold_field(n, extra, seed):
    """1D codes at abs eb 0.5 (x = d * step exactly, so prequantisation returns
    d): deltas 0 (n - m times), +1 and -1 (m = 0.09 n + extra together, split
    unevenly) in seeded order; the first delta of each 256-chunk is taken
    against zero, which the deltas themselves define.  Huffman gives the
    zero delta 1 bit and the other two 2 bits: n + m bits in all."""
    m = 9 * n // 100 + extra
    delta = np.zeros(n, np.int64)
    delta[:m // 3] = 1
    delta[m // 3:m] = -1
    np.random.default_rng(seed).shuffle(delta)
    c = np.cumsum(delta)
    starts = np.arange(0, n, 256)
    base = np.concatenate([[0], c[starts[1:] - 1]])
    d = c - np.repeat(base, np.diff(np.append(starts, n)))
    step = O.quant_step(float(max(np.abs(d).max(), 1)), 0.5)[0]
    x = (d * step).astype(np.float32)
    assert (x.astype(np.float64) == d * step).all()
    assert O.quant_step(float(np.abs(x).max()), 0.5)[0] == step
    return x


@pytest.mark.parametrize("extra,want", [(0, O.ARC_RLE), (1, O.ARC_HUFFMAN)])
def test_decision_threshold_on_the_gpu(E, extra, want):
    n = 1_000_000
    x = threshold_field(n, extra, 70 + extra)
    it = O.intermediates(x, 0.5, "abs")
    cost = int((it["hist"] * it["len"].astype(np.uint64)).sum())
    assert cost == 109 * n // 100 + extra
    ref = O.compress(x, 0.5, "abs")
    assert O.archive_info(ref)["codec"] == want
    a, st = E.compress(torch.from_numpy(x).cuda(), 0.5, "abs", stats=True)
    assert st.huff_bits == cost and st.codec == want
    assert a.cpu().numpy().tobytes() == ref
    np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))
