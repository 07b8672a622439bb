"""Pins of the compressibility estimates (Sec. III-B): the histogram-based
entropy and redundancy bounds, and the sampled binary madogram.

The bounds are theorems about optimal prefix codes (Gallager: R <= p1 + 0.086;
for p1 > 0.4, R >= 1 - H(p1, 1 - p1)), checked against the oracle's actual
Huffman code; the entropy against closed forms; the sampler's generator
against its published outputs; the madogram against fields whose roughness is
known exactly at every distance."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))
    got = [O.splitmix64(g["seed"], k) for k in range(len(g["outputs_hex"]))]
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_entropy_closed_forms():
    for k in range(0, 11):
        h = np.zeros(2048, np.uint64)
        h[:1 << k] = 7
        e = O.estimate_hist(h)
        assert abs(e["entropy"] - k) < 1e-12
    for p in (0.5, 0.25, 0.1, 0.9):
        n = 1 << 20
        a = int(round(p * n))
        h = np.array([a, n - a], np.uint64)
        q = a / n
        e = O.estimate_hist(h)
        assert abs(e["entropy"] - (-q * np.log2(q) - (1 - q) * np.log2(1 - q))) < 1e-12
        assert e["p1"] == max(a, n - a) / n


def test_single_symbol_histogram():
    h = np.zeros(64, np.uint64)
    h[9] = 1000
    e = O.estimate_hist(h)
    assert e["entropy"] == 0.0 and e["p1"] == 1.0
    # one bit per symbol: Huffman gives length 1, inside [H + R-, H + R+]
    assert e["bits_lo"] <= 1.0 <= e["bits_hi"] and e["predict"] == 1


def _hists():
    rng = np.random.default_rng(77)
    out = []
    for _ in range(60):
        m = int(rng.integers(2, 300))
        w = rng.pareto(rng.uniform(0.3, 3.0), m) + 1e-3
        if rng.random() < 0.5:
            w[0] = w.sum() * rng.uniform(0.5, 20.0)  # p1 above 0.4
        h = np.maximum(1, np.round(w / w.sum() * 100000)).astype(np.uint64)
        out.append(h)
    return out


@pytest.mark.parametrize("h", _hists(), ids=lambda h: f"m{h.size}")
def test_redundancy_bounds_hold_for_the_actual_code(h):
    ln = O.huffman_lengths(h)
    n = int(h.sum())
    avg = float((h * ln.astype(np.uint64)).sum()) / n
    e = O.estimate_hist(h)
    assert e["entropy"] <= avg + 1e-12
    assert avg <= e["bits_hi"] + 1e-12
    assert e["bits_lo"] <= avg + 1e-12
    if e["p1"] > 0.4:
        assert e["r_lo"] > 0.0
    # a confident prediction agrees with the exact 1.09-bit rule
    if e["predict"] == 1:
        assert O.choose_rle(h, ln, n)
    elif e["predict"] == 0:
        assert not O.choose_rle(h, ln, n)


def test_madogram_of_constant_and_alternating_codes():
    s, c = O.madogram(np.full(10000, 5, np.uint16), 200000, 3)
    assert s.sum() == 0 and c[0] == 0 and c[1:].min() > 0
    q = (np.arange(10000) % 2).astype(np.uint16)
    s, c = O.madogram(q, 200000, 4)
    d = np.arange(201)
    np.testing.assert_array_equal(s[1:], np.where(d[1:] % 2 == 1, c[1:], 0))


def test_madogram_sampling_counts():
    n = 5000
    s, c = O.madogram(np.zeros(n, np.uint16), 100000, 9)
    # pairs past the end are skipped: about d/n of them at distance d
    assert c[0] == 0
    assert abs(int(c.sum()) - 100000 * (1 - 100.5 / n)) < 1500
    assert c[1:].min() > 100000 / 200 * 0.8 and c[1:].max() < 100000 / 200 * 1.2


def test_madogram_of_iid_codes_is_flat():
    """Independent symbols with probabilities p: every distance has roughness
    1 - sum p^2 (two draws differ), within sampling error."""
    rng = np.random.default_rng(12)
    p = np.array([0.7, 0.2, 0.1])
    q = rng.choice(3, size=200000, p=p).astype(np.uint16)
    s, c = O.madogram(q, 400000, 13)
    v = s[1:].sum() / c[1:].sum()
    assert abs(v - (1 - (p ** 2).sum())) < 0.005
