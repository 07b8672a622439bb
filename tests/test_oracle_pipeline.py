"""Pins of the oracle's RLE, quantisation and whole pipeline (CPU only).

Pins: the RLE worked example of Sec. III-B (golden fixture), the 2D predictor
of the Sec. II-A footnote (golden fixture), the prequantisation error bound of
Sec. IV-A.1 (|x - d*2eb| < eb) on every element after fp32 output rounding,
the uniform-error PSNR closed form 20 log10(sqrt(3)/eb_rel) (Sec. V-B quotes
PSNR above 85 dB at 1e-4), and the error paths.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rle_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "rle_example.json")))
    m = g["symbol_codes"]
    q = np.array([m[c] for c in g["symbols"]], dtype=np.uint16)
    val, ln = O.rle_encode(q)
    assert [(int(v), int(n)) for v, n in zip(val, ln)] == [(m[s], n) for s, n in g["runs"]]
    np.testing.assert_array_equal(O.rle_decode(val, ln, q.size), q)


def test_lorenzo_2d_golden():
    g = json.load(open(os.path.join(GOLDEN, "lorenzo_2d_footnote.json")))
    d = np.array(g["d"], dtype=np.int32)
    np.testing.assert_array_equal(O.lorenzo(d, 2), np.array(g["delta"]))


@pytest.mark.parametrize("seed", range(5))
def test_rle_roundtrip_and_run_count(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 20000))
    q = np.repeat(rng.integers(0, 5, size=n), rng.integers(1, 30, size=n))[:n].astype(np.uint16)
    val, ln = O.rle_encode(q)
    assert val.size == 1 + int((q[1:] != q[:-1]).sum())
    assert int(ln.astype(np.int64).sum()) == q.size
    assert np.all(val[1:] != val[:-1])
    np.testing.assert_array_equal(O.rle_decode(val, ln, q.size), q)


def test_quant_step_closed_form():
    # M = 1, eb = 2e-4 (rel 1e-4 on [-1, 1]): ilogb(1) = 0, ilogb(2e-4) = -13,
    # e = max(0 + 13 - 21, -22) = -8
    ebx2, inv, e = O.quant_step(1.0, 2e-4)
    assert e == -8
    assert ebx2 == (2e-4 * (1 - 2.0 ** -8)) * 2
    assert inv == 1.0 / ebx2
    # M = 0 takes the floor exponent
    assert O.quant_step(0.0, 1e-3)[2] == -22
    # too small a bound relative to the magnitude is rejected
    with pytest.raises(O.OracleError) as ei:
        O.quant_step(1.0, 2.0 ** -18)
    assert ei.value.status == -4


def test_prequant_bound_every_element():
    """|x - d*ebx2| <= eb_abs*(1-eps) + |x|*2^-52 for every element (Sec. IV-A.1)."""
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200000) * 10).astype(np.float32)
    M = float(np.abs(x).max())
    for eb in (1e-1, 1e-2, 1.3e-3):
        ebx2, inv, e = O.quant_step(M, eb)
        d = O.prequant(x, inv)
        err = np.abs(x.astype(np.float64) - d.astype(np.float64) * ebx2)
        assert np.all(err <= eb * (1 - 2.0 ** e) + np.abs(x) * 2.0 ** -52)


def test_prequant_recovers_integer_multiples():
    """x = k * ebx2 with small integers k comes back exactly (ABS mode)."""
    ebx2, inv, _ = O.quant_step(1000 * 2e-3, 1e-3)
    k = np.arange(-1000, 1001, dtype=np.int64)
    x = (k * ebx2).astype(np.float32)
    d = O.prequant(x, inv)
    np.testing.assert_array_equal(d, k)


def psnr(x, y):
    rng = float(x.max()) - float(x.min())
    mse = float(np.mean((x.astype(np.float64) - y.astype(np.float64)) ** 2))
    return 20 * math.log10(rng) - 10 * math.log10(mse)


CASES = [
    ("smooth2d", lambda: synth.smooth_2d(256, 256, 1), 1e-4, "rel"),
    ("smooth2d_1e-2", lambda: synth.smooth_2d(128, 96, 5), 1e-2, "rel"),
    ("walk1d", lambda: synth.random_walk_1d(50000, 3), 1e-4, "rel"),
    ("lognormal3d", lambda: synth.lognormal_3d((24, 40, 33), 9), 1e-3, "rel"),
    ("grf3d_abs", lambda: synth.grf_field((20, 17, 30), 8), 1e-3, "abs"),
    ("noise2d", lambda: np.random.default_rng(4).standard_normal((70, 90)).astype(np.float32),
     1e-4, "rel"),
]


@pytest.mark.parametrize("name,make,eb,mode", CASES, ids=[c[0] for c in CASES])
def test_pipeline_roundtrip_error_bound(name, make, eb, mode):
    x = make()
    a = O.compress(x, eb, mode)
    y = O.decompress(a)
    assert y.shape == x.shape
    rng = float(x.max()) - float(x.min())
    eb_abs = eb * rng if mode == "rel" else eb
    err = np.abs(x.astype(np.float64) - y.astype(np.float64))
    assert float(err.max()) <= eb_abs
    info = O.archive_info(a)
    assert info["rank"] == x.ndim


@pytest.mark.parametrize("name,make,eb,mode", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_pipeline_forced_codecs_agree(name, make, eb, mode):
    x = make()
    ya = O.decompress(O.compress(x, eb, mode, codec="huffman"))
    yb = O.decompress(O.compress(x, eb, mode, codec="rle"))
    np.testing.assert_array_equal(ya, yb)


def test_psnr_closed_form_at_1e_4():
    x = synth.smooth_2d(256, 256, 1)
    y = O.decompress(O.compress(x, 1e-4, "rel"))
    want = 20 * math.log10(math.sqrt(3) / 1e-4)  # 84.77 dB for uniform error
    assert abs(psnr(x, y) - want) < 0.5


def test_intermediates_consistent_with_archive():
    x = synth.smooth_2d(64, 80, 2)
    it = O.intermediates(x, 1e-4)
    a = O.compress(x, 1e-4)
    s = O.sections(a)
    assert s["info"]["n_outliers"] == it["oidx"].size == int(it["hist"][0])
    np.testing.assert_array_equal(s["oidx"], it["oidx"])
    np.testing.assert_array_equal(s["oval"], it["oval"])
    assert np.all(np.diff(s["oidx"].astype(np.int64)) > 0)
    r = 512
    assert np.all(np.abs(it["oval"].astype(np.int64)) >= r)
    inr = it["q"] != 0
    assert np.all(np.abs(it["delta"][inr].astype(np.int64)) < r)
    np.testing.assert_array_equal(it["q"][inr].astype(np.int64), it["delta"][inr] + r)
    if s["info"]["codec"] == O.ARC_HUFFMAN:
        np.testing.assert_array_equal(s["len"], it["len"])


def test_constant_field_rel_is_const_codec():
    x = np.full((33, 45), 3.25, dtype=np.float32)
    a = O.compress(x, 1e-4)
    assert len(a) == O.HDR_BYTES and O.archive_info(a)["codec"] == O.ARC_CONST
    np.testing.assert_array_equal(O.decompress(a), x)


def test_constant_field_abs_uses_single_run():
    x = np.full((1000,), 0.5, dtype=np.float32)
    a = O.compress(x, 1e-3, "abs")
    info = O.archive_info(a)
    assert info["codec"] == O.ARC_RLE
    assert np.max(np.abs(O.decompress(a) - x)) <= 1e-3


def test_single_element():
    x = np.array([1.5], dtype=np.float32)
    y = O.decompress(O.compress(x, 1e-3, "abs"))
    assert abs(float(y[0]) - 1.5) <= 1e-3


@pytest.mark.parametrize("n_bins", [4, 1024, 65536])
def test_bin_counts(n_bins):
    x = synth.smooth_2d(48, 40, 3)
    a = O.compress(x, 1e-4, n_bins=n_bins)
    y = O.decompress(a)
    assert np.max(np.abs(x.astype(np.float64) - y)) <= 1e-4 * (float(x.max()) - float(x.min()))
    it = O.intermediates(x, 1e-4, n_bins=n_bins)
    assert int(it["hist"].sum()) == x.size
    assert np.all(it["q"] < n_bins)


def test_huge_eb_all_zero_codes():
    x = synth.smooth_2d(32, 32, 4)
    a = O.compress(x, 10.0, "abs")
    y = O.decompress(a)
    assert np.max(np.abs(x.astype(np.float64) - y)) <= 10.0


def test_error_paths():
    x = np.ones((8, 8), np.float32)
    assert O.compress_status(x, 0.0) == -3
    assert O.compress_status(x, float("nan")) == -3
    assert O.compress_status(x, 1e-3, n_bins=3) == -5
    assert O.compress_status(x, 1e-3, n_bins=1025) == -5
    assert O.compress_status(x, 1e-3, rank=4) == -2
    assert O.compress_status(x, 1e-3, dims=(8, 0, 1)) == -2
    y = x.copy()
    y[3, 3] = np.nan
    assert O.compress_status(y, 1e-3) == -6
    y[3, 3] = np.inf
    assert O.compress_status(y, 1e-3) == -6
    z = np.linspace(-1, 1, 64, dtype=np.float32).reshape(8, 8)
    assert O.compress_status(z * 1e6, 1e-12, "abs") == -4


def test_corrupted_archive_rejected():
    x = synth.smooth_2d(32, 32, 4)
    a = bytearray(O.compress(x, 1e-4))
    bad = bytearray(a)
    bad[0] = ord("X")
    assert O.decompress_status(bytes(bad)) == -9
    assert O.decompress_status(bytes(a[:100])) == -9
    trunc = bytes(a[: len(a) - 16])
    assert O.decompress_status(trunc) == -9


def test_header_fields():
    x = synth.smooth_2d(40, 56, 6)
    a = O.compress(x, 1e-4)
    b = np.frombuffer(a, np.uint8)
    assert bytes(b[:4]) == b"EBC1"
    assert int(b[4:6].view(np.uint16)[0]) == 2  # format version
    assert int(b[8]) == 2  # rank
    assert int(b[11]) == 0  # fp32
    assert int(b[12:16].view(np.uint32)[0]) == 1024
    assert list(b[16:40].view(np.uint64)) == [56, 40, 1]
    assert list(b[40:52].view(np.uint32)) == [16, 16, 1]
    assert int(b[52:56].view(np.uint32)[0]) == 1024
    assert int(b[112:120].view(np.uint64)[0]) == len(a)
    assert int(b[120:124].view(np.uint32)[0]) == 256  # Huffman sub-chunk symbols
    assert len(a) % 16 == 0
