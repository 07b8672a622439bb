"""Pins of the RLE+VLE workflow of the oracle (Sec. III-A, "RLE with optional
VLE"): run-length coding whose run values are Huffman-coded with a codebook
of their own, the run lengths left plain (the paper leaves that metadata
uncoded by default).

* round trip through the archive, and the decoded runs are the maximal runs
  of the codes (the plain RLE archive's runs);
* the value stream's code is an optimal prefix code for the run values'
  histogram (its cost equals the optimum from a separate heap construction);
* the value section is never larger than plain RLE's two bytes per value,
  up to the fixed overheads (length table, sub-chunk counts, word padding),
  and strictly smaller whenever the values average under 16 bits;
* the 1.09-bit rule decides the branch exactly as for plain RLE."""
import heapq

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import synth


def heap_optimum(h):
    w = [int(v) for v in h if v > 0]
    if len(w) == 1:
        return w[0]
    heapq.heapify(w)
    cost = 0
    while len(w) > 1:
        a, b = heapq.heappop(w), heapq.heappop(w)
        cost += a + b
        heapq.heappush(w, a + b)
    return cost


FIELDS = [
    ("lognormal3d", lambda: synth.lognormal_3d((32, 40, 48), 3), 3e-2),
    ("smooth2d", lambda: synth.smooth_2d(120, 100, 4), 1e-3),
    ("walk1d", lambda: synth.random_walk_1d(100_000, 5), 1e-3),
    ("noise", lambda: np.random.default_rng(6).standard_normal((60, 50)).astype(np.float32), 1e-2),
    ("sparse1d", lambda: synth.sparse_background_1d(2_000_000, 7, 0.02), 1e-2),
]


@pytest.mark.parametrize("name,make,eb", FIELDS, ids=[f[0] for f in FIELDS])
def test_rle_vle_roundtrip_and_runs(name, make, eb):
    x = make()
    a = O.compress(x, eb, codec="rle_vle")
    r = O.compress(x, eb, codec="rle")
    sa, sr = O.sections(a), O.sections(r)
    assert sa["info"]["codec"] == O.ARC_RLE_VLE
    # the same runs as plain run-length coding
    assert sa["info"]["n_a"] == sr["info"]["n_a"]
    np.testing.assert_array_equal(sa["rlen"], sr["rlen"])
    vals = O.huffman_decode(sa["sbits"], sa["words"], sa["info"]["n_a"], sa["len"], sa["info"]["hc"])
    np.testing.assert_array_equal(vals, sr["val"])
    # the maximal runs of the codes themselves
    q = O.intermediates(x, eb)["q"].ravel()
    np.testing.assert_array_equal(np.repeat(vals, sa["rlen"].astype(np.int64)), q)
    # whole round trip equal to plain RLE's reconstruction
    np.testing.assert_array_equal(O.decompress(a).view(np.uint32), O.decompress(r).view(np.uint32))


@pytest.mark.parametrize("name,make,eb", FIELDS, ids=[f[0] for f in FIELDS])
def test_rle_vle_value_code_is_optimal_and_small(name, make, eb):
    x = make()
    s = O.sections(O.compress(x, eb, codec="rle_vle"))
    R = s["info"]["n_a"]
    vals = O.huffman_decode(s["sbits"], s["words"], R, s["len"], s["info"]["hc"])
    h = np.bincount(vals, minlength=s["len"].size).astype(np.uint64)
    cost = int((h * s["len"].astype(np.uint64)).sum())
    assert cost == heap_optimum(h)
    assert cost == int(s["sbits"].astype(np.int64).sum())
    # value section vs plain RLE's 16 bits per value
    hc = s["info"]["hc"]
    nch = (R + hc - 1) // hc
    section = s["layout"]["end"] - s["layout"]["len"]
    overhead = s["len"].size + 2 * s["layout"]["n_sub"] + 4 * nch + 3 * 16
    assert section <= 2 * R + overhead
    if cost < 16 * R:
        assert 4 * s["info"]["n_words"] < 2 * R + 4 * nch


def test_auto_vle_follows_the_rule():
    x = synth.lognormal_3d((32, 40, 48), 3)
    for eb in (3e-2, 1e-4):
        it = O.intermediates(x, eb)
        a = O.archive_info(O.compress(x, eb, codec="auto_vle"))
        b = O.archive_info(O.compress(x, eb, codec="auto"))
        assert (a["codec"] == O.ARC_RLE_VLE) == it["rle"] == (b["codec"] == O.ARC_RLE)
