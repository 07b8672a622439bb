"""Pins of the oracle's histogram / Huffman / decision steps (CPU only).

The optimal cost comes from an independent heap-based Huffman (sum of merged
weights, tie-independent); the tie rule is pinned by brute force over every
complete prefix code on tiny alphabets (the leaf-first two-queue rule yields
the minimum-variance optimal code); the redundancy bounds are the ones the
paper quotes in Sec. III-B.1 (upper p1 + 0.086; lower 1 - H(p1, 1 - p1) when
p1 > 0.4); the decision threshold 1.09 is Sec. I / Sec. III-B.2.
"""
import heapq
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O


def heap_optimal_cost(freqs):
    h = [int(f) for f in freqs if f > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def entropy(freqs):
    f = np.asarray([v for v in freqs if v > 0], dtype=np.float64)
    p = f / f.sum()
    return float(-(p * np.log2(p)).sum())


def random_hists():
    rng = np.random.default_rng(21)
    out = []
    for nb in (4, 16, 64, 1024):
        for _ in range(6):
            h = rng.integers(0, 1000, size=nb).astype(np.uint64)
            h[rng.random(nb) < 0.3] = 0
            if h.sum() == 0:
                h[0] = 1
            out.append(h)
    # skewed (smooth-field-like) histograms
    for p1 in (0.45, 0.6, 0.8, 0.95, 0.99, 0.999):
        h = np.zeros(1024, dtype=np.uint64)
        n = 100000
        h[512] = int(p1 * n)
        rest = n - int(h[512])
        tail = rng.geometric(0.3, size=rest)
        for t in tail:
            h[512 + (t if rng.random() < 0.5 else -t) % 400] += 1
        out.append(h)
    # geometric frequencies (deep trees)
    out.append(np.array([2 ** k for k in range(30)], dtype=np.uint64))
    out.append(np.array([1, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144], dtype=np.uint64))
    return out


HISTS = random_hists()


@pytest.mark.parametrize("h", HISTS, ids=lambda h: f"nb{h.size}")
def test_lengths_are_optimal_and_complete(h):
    ln = O.huffman_lengths(h).astype(np.int64)
    used = h > 0
    assert np.all((ln > 0) == used)
    m = int(used.sum())
    kraft = sum(2.0 ** -int(v) for v in ln[used])
    if m >= 2:
        assert kraft == 1.0
        assert int((h.astype(np.int64) * ln).sum()) == heap_optimal_cost(h)
    else:
        assert ln[used][0] == 1


@pytest.mark.parametrize("h", HISTS, ids=lambda h: f"nb{h.size}")
def test_canonical_codes_prefix_free_and_ordered(h):
    ln = O.huffman_lengths(h)
    code = O.canonical_codes(ln)
    syms = [s for s in range(h.size) if ln[s] > 0]
    strings = {s: format(int(code[s]), f"0{int(ln[s])}b") for s in syms}
    for s in syms:
        assert len(strings[s]) == ln[s]
    # prefix-free
    items = sorted(strings.values())
    for a, b in zip(items, items[1:]):
        assert not b.startswith(a)
    # canonical: ordered by (len, symbol), left-aligned values strictly increase,
    # and within one length consecutive symbols get consecutive codes
    order = sorted(syms, key=lambda s: (int(ln[s]), s))
    L = 64
    vals = [int(code[s]) << (L - int(ln[s])) for s in order]
    assert all(a < b for a, b in zip(vals, vals[1:]))
    assert int(code[order[0]]) == 0
    for a, b in zip(order, order[1:]):
        if ln[a] == ln[b]:
            assert code[b] == code[a] + 1


@pytest.mark.parametrize("w", (4, 8, 12))
@pytest.mark.parametrize("h", HISTS, ids=lambda h: f"nb{h.size}")
def test_long_codeword_prefixes_are_the_top_ones(h, w):
    """A decoder that looks up w bits at a time can index its second-level
    table from the bits alone when the w-bit prefixes that start a codeword
    longer than w are the top ones, numbered in prefix order. Canonical codes
    (longer codewords numerically larger) make it so: every w-bit prefix is
    covered by exactly one codeword of length <= w or starts a longer one,
    and the latter form the range [2^w - nlong, 2^w)."""
    ln = O.huffman_lengths(h)
    code = O.canonical_codes(ln)
    covered = np.zeros(1 << w, dtype=np.int64)
    long_pref = set()
    for s in range(h.size):
        L = int(ln[s])
        if L == 0:
            continue
        c = int(code[s])
        if L <= w:
            base = c << (w - L)
            covered[base:base + (1 << (w - L))] += 1
        else:
            long_pref.add(c >> (L - w))
    assert covered.max(initial=0) <= 1
    if int((ln > 0).sum()) < 2:
        assert not long_pref  # a lone symbol has a 1-bit code
        return
    nlong = (1 << w) - int(covered.sum())
    assert long_pref == set(range((1 << w) - nlong, 1 << w))
    assert not covered[(1 << w) - nlong:].any()


@pytest.mark.parametrize("h", HISTS, ids=lambda h: f"nb{h.size}")
def test_redundancy_bounds(h):
    """H <= <b> <= H + p1 + 0.086, and <b> >= H + 1 - H(p1, 1-p1) for p1 > 0.4."""
    ln = O.huffman_lengths(h).astype(np.float64)
    n = float(h.sum())
    if (h > 0).sum() < 2:
        return
    avg = float((h * ln).sum()) / n
    H = entropy(h)
    p1 = float(h.max()) / n
    assert avg >= H - 1e-12
    assert avg <= H + p1 + 0.086 + 1e-12
    if p1 > 0.4:
        hb = -(p1 * math.log2(p1) + (1 - p1) * math.log2(1 - p1))
        assert avg >= H + 1 - hb - 1e-12


def all_complete_codes(m, maxlen):
    for lens in itertools.product(range(1, maxlen + 1), repeat=m):
        if sum(2.0 ** -l for l in lens) == 1.0:
            yield lens


@pytest.mark.parametrize("seed", range(30))
def test_tie_rule_gives_minimum_variance_optimal_code(seed):
    """Brute force over every complete code: among all minimum-cost length
    vectors the oracle picks one of minimum sum f*len^2 and minimum max length."""
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(2, 7))
    f = rng.integers(1, 5, size=m).astype(np.uint64)  # small values: many ties
    ln = tuple(int(v) for v in O.huffman_lengths(f))
    cands = list(all_complete_codes(m, m - 1))
    cost = lambda L: sum(int(a) * b for a, b in zip(f, L))
    best = min(cost(L) for L in cands)
    opt = [L for L in cands if cost(L) == best]
    assert cost(ln) == best
    var = lambda L: sum(int(a) * b * b for a, b in zip(f, L))
    assert var(ln) == min(var(L) for L in opt)
    assert max(ln) == min(max(L) for L in opt)


def test_tie_rule_golden_example():
    # frequencies 1,1,2,2 have two optimal codes, (3,3,2,1) and (2,2,2,2);
    # the leaf-first rule takes the flat one
    assert list(O.huffman_lengths(np.array([1, 1, 2, 2], np.uint64))) == [2, 2, 2, 2]


def test_single_symbol_gets_length_one():
    h = np.zeros(1024, np.uint64)
    h[512] = 12345
    ln = O.huffman_lengths(h)
    assert ln[512] == 1 and ln.sum() == 1
    assert O.canonical_codes(ln)[512] == 0


def test_decision_threshold_is_exactly_1_09():
    # two symbols of length 1 and length-9 tail symbols; tune sum f*len around 1.09 N
    n = 10000
    for bits, want in ((10900, True), (10901, False), (10899, True)):
        h = np.zeros(8, np.uint64)
        ln = np.zeros(8, np.uint8)
        # construct directly: one symbol of length 1 with count a, one of length b
        # so that a + b*L == bits and a + b == n  (L = 2)
        b_cnt = bits - n
        h[0], ln[0] = n - b_cnt, 1
        h[1], ln[1] = b_cnt, 2
        assert int((h * ln).sum()) == bits
        assert O.choose_rle(h, ln, n) is want


def test_decision_single_symbol_is_rle():
    h = np.zeros(1024, np.uint64)
    h[512] = 777
    assert O.choose_rle(h, O.huffman_lengths(h), 777)


@pytest.mark.parametrize("h", HISTS[:8] + HISTS[-8:], ids=lambda h: f"nb{h.size}")
def test_huffman_encode_decode_roundtrip(h):
    rng = np.random.default_rng(31)
    p = h.astype(np.float64) / h.sum()
    for hc in (64, 1024, 4096):
        n = int(rng.integers(1, 9000))
        q = rng.choice(h.size, size=n, p=p).astype(np.uint16)
        ln = O.huffman_lengths(O.histogram(q, h.size))
        code = O.canonical_codes(ln)
        sb, words = O.huffman_encode(q, ln, code, hc)
        # one u16 entry per sub-chunk of min(hc, 256) symbols: the sum of its
        # code lengths; a chunk takes ceil(sum of its sub-chunks / 32) words
        hs = min(hc, 256)
        assert O.sub_chunk(hc) == hs and sb.size == (n + hs - 1) // hs
        for k in range(sb.size):
            assert int(sb[k]) == int(ln[q[k * hs:(k + 1) * hs]].astype(np.int64).sum())
        per = hc // hs
        chunk_bits = [int(sb[c * per:(c + 1) * per].astype(np.int64).sum())
                      for c in range((n + hc - 1) // hc)]
        for c, b in enumerate(chunk_bits):
            assert b == int(ln[q[c * hc:(c + 1) * hc]].astype(np.int64).sum())
        assert words.size == sum((b + 31) // 32 for b in chunk_bits)
        # payload never below one bit per symbol (CR <= 32 for fp32, Sec. II-B.1)
        assert sum(chunk_bits) >= n
        np.testing.assert_array_equal(O.huffman_decode(sb, words, n, ln, hc), q)
        # a sub-chunk count that is off by one is a corrupt archive
        if sb.size > 1:
            for k in (0, sb.size - 1):
                bad = sb.copy()
                bad[k] += 1
                with pytest.raises(O.OracleError):
                    O.huffman_decode(bad, words, n, ln, hc)


def test_huffman_sub_chunks_in_long_chunks():
    """Chunks longer than 256 symbols are cut into 256-symbol sub-chunks whose
    bits follow each other inside the chunk (no padding between them)."""
    rng = np.random.default_rng(32)
    q = rng.integers(0, 5, size=5000).astype(np.uint16)
    ln = O.huffman_lengths(O.histogram(q, 5))
    code = O.canonical_codes(ln)
    sb, words = O.huffman_encode(q, ln, code, 2048)
    assert sb.size == (5000 + 255) // 256
    for k in range(sb.size):
        assert sb[k] == int(ln[q[k * 256:(k + 1) * 256]].astype(np.int64).sum())
    # the stream of chunk 0 is the concatenation of its 8 sub-chunks
    bits = "".join(format(int(code[s]), f"0{int(ln[s])}b") for s in q[:2048])
    got = "".join(format(int(w), "032b") for w in words)[:len(bits)]
    assert got == bits
    np.testing.assert_array_equal(O.huffman_decode(sb, words, q.size, ln, 2048), q)


def test_huffman_bitstream_layout_msb_first():
    """Three symbols with codes 0, 10, 11: the stream 'a b c a' packs to 0 10 11 0."""
    h = np.array([2, 1, 1], np.uint64)
    ln = O.huffman_lengths(h)
    code = O.canonical_codes(ln)
    assert list(ln) == [1, 2, 2] and list(code) == [0, 2, 3]
    q = np.array([0, 1, 2, 0], np.uint16)
    bits, words = O.huffman_encode(q, ln, code, 64)
    assert list(bits) == [6]  # one sub-chunk of 6 bits
    assert list(words) == [0b010110 << 26]


def test_histogram_counts():
    rng = np.random.default_rng(5)
    q = rng.integers(0, 1024, size=100003).astype(np.uint16)
    h = O.histogram(q, 1024)
    assert h.sum() == q.size
    np.testing.assert_array_equal(h, np.bincount(q, minlength=1024))


def test_fibonacci_weights_give_the_deepest_tree():
    """Fibonacci weights F1..Fm make every merge take the previous subtree and
    the next leaf, so the lengths are 1, 2, ..., m-2, m-1, m-1 (closed form);
    m = 34 reaches 33-bit codewords, past one 32-bit word."""
    m = 34
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    h = np.zeros(1024, dtype=np.uint64)
    h[100:100 + m] = f
    L = O.huffman_lengths(h)
    got = sorted(int(v) for v in L[100:100 + m])
    assert got == list(range(1, m - 1)) + [m - 1, m - 1]
    assert int(L[100 + m - 1]) == 1 and int(L[100]) == m - 1 and int(L[101]) == m - 1
    assert (L[:100] == 0).all() and (L[100 + m:] == 0).all()
