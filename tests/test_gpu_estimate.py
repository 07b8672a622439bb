"""GPU parity of the compressibility estimates (Sec. III-B): the histogram
bounds and the sampled binary madogram of the quant-codes.

Integer results (the count of the most likely code, the madogram's pair
counts per distance) must equal the oracle's exactly; the floating-point
ones (entropy, redundancy bounds) are sums of log2 terms whose order and
libm differ between the two sides, so they must agree within a relative
1e-12 (each term is exact to a few ulp, and at most 65536 terms are summed
in double)."""
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


CASES = [
    ("smooth256", lambda: synth.smooth_2d(256, 256, 1), 1e-4, 1024),
    ("lognormal3d", lambda: synth.lognormal_3d((48, 64, 80), 3), 3e-2, 1024),
    ("walk1d", lambda: synth.random_walk_1d(1_000_003, 5), 1e-3, 256),
    ("noise2d", lambda: np.random.default_rng(6).standard_normal((300, 200)).astype(np.float32), 1e-4, 4096),
]


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("name,make,eb,nb", CASES, ids=[c[0] for c in CASES])
def test_estimates_match_the_oracle(E, name, make, eb, nb):
    x = make()
    it = O.intermediates(x, eb, n_bins=nb)
    want = O.estimate_hist(it["hist"], x.size)
    samples, seed = 300_000, 0x1234ABCD
    s, c = O.madogram(it["q"], samples, seed)
    got = E.estimate(torch.from_numpy(x).cuda(), eb, n_bins=nb, samples=samples, seed=seed)
    assert got["hist_max"] == int(it["hist"].max())
    assert got["n_elems"] == x.size
    np.testing.assert_array_equal(got["mado_sum"], s)
    np.testing.assert_array_equal(got["mado_cnt"], c)
    for k in ("entropy", "p1", "r_lo", "r_hi", "bits_lo", "bits_hi"):
        assert close(got[k], want[k]), (k, got[k], want[k])
    assert got["codec_hint"] == want["predict"]
    # the bounds hold for the codebook the compressor builds
    a, st = E.compress(torch.from_numpy(x).cuda(), eb, n_bins=nb, stats=True)
    avg = st.huff_bits / x.size
    assert got["bits_lo"] - 1e-12 <= avg <= got["bits_hi"] + 1e-12
    assert close(st.entropy, want["entropy"]) and st.predict == want["predict"]


def test_madogram_of_a_constant_background(E):
    """Codes of a field that is one constant over its first half: every pair
    inside that half has equal codes; the roughness comes from the rest."""
    x = synth.lognormal_3d((32, 48, 64), 9)
    x[:16] = x.min()
    it = O.intermediates(x, 1e-3)
    s, c = O.madogram(it["q"], 200_000, 77)
    got = E.estimate(torch.from_numpy(x).cuda(), 1e-3, samples=200_000, seed=77)
    np.testing.assert_array_equal(got["mado_sum"], s)
    np.testing.assert_array_equal(got["mado_cnt"], c)
    assert 0.0 < got["roughness"] < 1.0
