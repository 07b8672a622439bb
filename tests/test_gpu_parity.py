"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything after prequantisation is integer, so the bar is bit-exact:
identical quant-codes, histogram, ordered outlier list, archive bytes and
reconstructed floats (compared as bit patterns).
"""
import math

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


def rng_field(shape, seed, kind="grf"):
    if kind == "noise":
        return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)
    if kind == "lognormal":
        return synth.lognormal_3d(shape, seed) if len(shape) == 3 else np.exp(
            1.5 * synth.grf(shape, -3.0, seed)).astype(np.float32)
    if kind == "walk":
        return synth.random_walk_1d(shape[0], seed)
    return synth.grf_field(shape, seed)


CASES = [
    # name, shape, kind, eb, mode, n_bins
    ("smooth256", (256, 256), "grf", 1e-4, "rel", 1024),
    ("2d_ragged", (37, 53), "grf", 1e-4, "rel", 1024),
    ("2d_narrow", (300, 6), "grf", 1e-3, "rel", 1024),
    ("2d_noise", (70, 90), "noise", 1e-4, "rel", 1024),
    ("1d_walk", (50000,), "walk", 1e-4, "rel", 1024),
    ("1d_ragged", (1000003,), "walk", 1e-3, "rel", 256),
    ("1d_tiny", (7,), "noise", 1e-2, "rel", 1024),
    ("3d_grf", (40, 48, 64), "grf", 1e-4, "rel", 1024),
    ("3d_ragged", (9, 10, 11), "grf", 1e-3, "rel", 1024),
    ("3d_lognormal", (24, 40, 33), "lognormal", 1e-3, "rel", 1024),
    ("3d_abs", (20, 17, 30), "grf", 1e-3, "abs", 1024),
    ("3d_wide", (16, 8, 600), "grf", 1e-4, "rel", 1024),
    ("bins4", (64, 64), "grf", 1e-3, "rel", 4),
    ("bins4096", (64, 80), "noise", 1e-4, "rel", 4096),
    ("bins64", (33, 65, 17), "noise", 1e-3, "rel", 64),
    # above 4096 bins (LDS histogram window + HBM counts, codebook and decoder
    # tables built in HBM): codes spread over more bins than the window, and
    # over 35k used symbols at 65536 bins
    ("bins8192_noise", (96, 120), "noise", 1e-5, "rel", 8192),
    ("bins65536_noise", (256, 300), "noise", 1e-5, "rel", 65536),
    ("bins65536_smooth", (256, 256), "grf", 2e-5, "rel", 65536),
    ("bins16384_3d", (24, 40, 33), "lognormal", 1e-5, "rel", 16384),
    ("bins32768_1d", (200003,), "walk", 1e-5, "rel", 32768),
]


@pytest.mark.parametrize("name,shape,kind,eb,mode,nb", CASES, ids=[c[0] for c in CASES])
def test_construct_intermediates(E, name, shape, kind, eb, mode, nb):
    x = rng_field(shape, 11, kind)
    it = O.intermediates(x, eb, mode, n_bins=nb)
    g = E.debug_construct(dev(x), eb, mode, n_bins=nb)
    assert g["ebx2"] == it["ebx2"]
    np.testing.assert_array_equal(g["q"].cpu().numpy().view(np.uint16), it["q"].ravel())
    np.testing.assert_array_equal(g["hist"].cpu().numpy().astype(np.uint64), it["hist"])
    np.testing.assert_array_equal(g["oidx"].cpu().numpy().view(np.uint32), it["oidx"])
    np.testing.assert_array_equal(g["oval"].cpu().numpy(), it["oval"])


@pytest.mark.parametrize("name,shape,kind,eb,mode,nb", CASES, ids=[c[0] for c in CASES])
def test_archive_bytes_and_roundtrip(E, name, shape, kind, eb, mode, nb):
    x = rng_field(shape, 12, kind)
    ref = O.compress(x, eb, mode, n_bins=nb)
    a = E.compress(dev(x), eb, mode, n_bins=nb)
    got = a.cpu().numpy().tobytes()
    assert len(got) == len(ref)
    assert got == ref
    y = E.decompress(a)
    yo = O.decompress(ref)
    np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(yo))
    rng = float(x.max()) - float(x.min())
    eb_abs = eb * rng if mode == "rel" else eb
    assert float(np.max(np.abs(y.cpu().numpy().astype(np.float64) - x))) <= eb_abs


@pytest.mark.parametrize("codec", ["huffman", "rle"])
@pytest.mark.parametrize("shape", [(256, 256), (9, 10, 11), (5000,)])
def test_forced_codecs(E, codec, shape):
    x = rng_field(shape, 13)
    ref = O.compress(x, 1e-3, codec=codec)
    a = E.compress(dev(x), 1e-3, codec=codec)
    assert a.cpu().numpy().tobytes() == ref
    np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))


@pytest.mark.parametrize("hc", [64, 128, 256, 512, 2048, 4096])
def test_huffman_chunk_sizes(E, hc):
    x = rng_field((70, 90), 14, "noise")
    ref = O.compress(x, 1e-4, codec="huffman", hc=hc)
    a = E.compress(dev(x), 1e-4, codec="huffman", huff_chunk=hc)
    assert a.cpu().numpy().tobytes() == ref
    np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))


def fibonacci_deltas_field(m, seed):
    """1D field whose quant-codes are m symbols with Fibonacci frequencies in a
    seeded random order at abs eb = 0.5: the integers d whose first
    differences within each 256-element chunk (the first element of a chunk
    taken against zero) are those symbols, times the quantisation step (each
    product is exact in fp32, so prequantisation returns d)."""
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    delta = np.repeat(np.arange(m, dtype=np.int64) - m // 2, f)
    np.random.default_rng(seed).shuffle(delta)
    c = np.cumsum(delta)
    starts = np.arange(0, delta.size, 256)
    base = np.concatenate([[0], c[starts[1:] - 1]])
    d = c - np.repeat(base, np.diff(np.append(starts, delta.size)))
    step = O.quant_step(float(np.abs(d).max()), 0.5)[0]
    x = (d * step).astype(np.float32)
    assert (x.astype(np.float64) == d * step).all()
    assert O.quant_step(float(np.abs(x).max()), 0.5)[0] == step
    return x, delta


def test_codewords_longer_than_32_bits(E):
    """A Fibonacci histogram over 34 symbols gives codewords of up to 33 bits:
    the encoder's and the decoder's paths for codewords that span two words,
    bit-exact against the oracle, from the smallest to the largest chunk size."""
    x, delta = fibonacci_deltas_field(34, 31)
    it = O.intermediates(x, 0.5, "abs")
    np.testing.assert_array_equal(it["q"].astype(np.int64), delta + it["hist"].size // 2)
    assert int(it["len"].max()) == 33
    xd = dev(x)
    for hc in (64, 512, 1024, 4096):
        print(f"[long codes] hc={hc}", flush=True)
        ref = O.compress(x, 0.5, "abs", codec="huffman", hc=hc)
        a = E.compress(xd, 0.5, "abs", codec="huffman", huff_chunk=hc)
        assert a.cpu().numpy().tobytes() == ref
        y = E.decompress(a).cpu().numpy()
        np.testing.assert_array_equal(y, x)
        np.testing.assert_array_equal(bits(y), bits(O.decompress(ref)))


def test_forced_rle_with_millions_of_runs(E):
    """Run-length coding forced on noise: one run per element or so (4.8M
    runs), so the run-start scan covers more tiles than the direct
    down-sweep takes and goes through the scanned tile sums."""
    x = np.random.default_rng(41).standard_normal(5_000_000).astype(np.float32)
    ref = O.compress(x, 1e-2, codec="rle")
    assert O.archive_info(ref)["n_a"] > 1024 * 4096
    a = E.compress(dev(x), 1e-2, codec="rle")
    assert a.cpu().numpy().tobytes() == ref
    np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))


def test_constant_field(E):
    x = np.full((33, 45), -2.5, np.float32)
    a = E.compress(dev(x), 1e-4)
    assert a.cpu().numpy().tobytes() == O.compress(x, 1e-4)
    np.testing.assert_array_equal(E.decompress(a).cpu().numpy(), x)


def test_constant_field_abs(E):
    x = np.full((3, 5, 7), 0.25, np.float32)
    a = E.compress(dev(x), 1e-3, "abs")
    assert a.cpu().numpy().tobytes() == O.compress(x, 1e-3, "abs")


def test_signed_zero_and_single(E):
    x = np.array([0.0, -0.0, 0.0], np.float32)
    assert E.compress(dev(x), 1e-3).cpu().numpy().tobytes() == O.compress(x, 1e-3)
    x1 = np.array([1.5], np.float32)
    assert E.compress(dev(x1), 1e-3, "abs").cpu().numpy().tobytes() == O.compress(x1, 1e-3, "abs")
    x3 = np.array([[[2.0]]], np.float32)
    assert E.compress(dev(x3), 1e-3, "abs").cpu().numpy().tobytes() == O.compress(x3, 1e-3, "abs")


def test_denormal_and_huge_eb(E):
    x = (np.random.default_rng(3).standard_normal((40, 40)) * 1e-39).astype(np.float32)
    assert E.compress(dev(x), 1e-2).cpu().numpy().tobytes() == O.compress(x, 1e-2)
    y = rng_field((32, 32), 4)
    assert E.compress(dev(y), 10.0, "abs").cpu().numpy().tobytes() == O.compress(y, 10.0, "abs")


def test_reconstruct_alone_matches_oracle(E):
    """Reconstruction from oracle-made codes and outliers (partial sum vs recurrence)."""
    for shape in [(257,), (37, 53), (17, 9, 20), (8, 8, 600)]:
        x = rng_field(shape, 15, "noise")
        it = O.intermediates(x, 1e-4, n_bins=64)
        qp = O.fuse(it["q"], 64, it["oidx"], it["oval"])
        want = O.dequant(O.reconstruct(qp, len(shape)), it["ebx2"])
        out = E.debug_reconstruct(dev(it["q"].view(np.int16).ravel()), dev(it["oidx"].view(np.int32)),
                                  dev(it["oval"]), len(shape), shape[::-1], 64, it["ebx2"])
        np.testing.assert_array_equal(bits(out.cpu().numpy()), bits(want.ravel()))


def test_error_paths(E):
    x = rng_field((16, 16), 5)
    y = x.copy()
    y[3, 4] = np.nan
    with pytest.raises(E.EbcError) as ei:
        E.compress(dev(y), 1e-3)
    assert ei.value.status == E.EBC_ERR_NONFINITE
    y[3, 4] = np.inf
    with pytest.raises(E.EbcError) as ei:
        E.compress(dev(y), 1e-3)
    assert ei.value.status == E.EBC_ERR_NONFINITE
    with pytest.raises(E.EbcError) as ei:
        E.compress(dev(x * 1e6), 1e-12, "abs")
    assert ei.value.status == E.EBC_ERR_EB_TOO_SMALL
    assert O.compress_status(x * 1e6, 1e-12, "abs") == E.EBC_ERR_EB_TOO_SMALL
    # output buffer too small: detected on the device, reported after the sync
    xt = dev(x)
    out = torch.empty(200, dtype=torch.uint8, device="cuda")
    p = E.make_params(1e-4)
    ws = E.default_workspace()
    wptr, wlen = ws.get(E.ebc_compress_workspace_size(2, (16, 16), p))
    st, size = E.ebc_compress(xt.data_ptr(), 2, (16, 16), p, out.data_ptr(), out.numel(), wptr,
                              wlen, E._stream_handle(None))
    assert st == E.EBC_ERR_OUT_TOO_SMALL and size == 0
    st, _ = E.ebc_compress(xt.data_ptr(), 2, (16, 16), p, out.data_ptr(), out.numel(), wptr, 16,
                           E._stream_handle(None))
    assert st == E.EBC_ERR_WS_TOO_SMALL


def test_corrupt_archives_rejected(E):
    x = rng_field((64, 64), 6, "noise")
    a = E.compress(dev(x), 1e-4)
    raw = a.cpu().numpy().copy()
    for mutate in ("magic", "truncate", "bits", "outlier"):
        b = raw.copy()
        if mutate == "magic":
            b[0] = ord("X")
        elif mutate == "truncate":
            b = b[:-16]
        elif mutate == "bits":
            # the first sub-chunk's bit count off by one
            ob = O.sections(raw.tobytes())["layout"]["sbits"]
            v = int(b[ob:ob + 2].view(np.uint16)[0]) + 1
            b[ob:ob + 2] = np.frombuffer(np.uint16(v).tobytes(), np.uint8)
        else:
            s = O.sections(raw.tobytes())
            if s["info"]["n_outliers"] == 0:
                continue
            # point the first outlier at a non-placeholder code
            oo = s["off_oidx"]
            it = O.intermediates(x, 1e-4)
            nz = int(np.flatnonzero(it["q"].ravel() != 0)[0])
            b[oo:oo + 4] = np.frombuffer(np.uint32(nz).tobytes(), np.uint8)
        st_o = O.decompress_status(b.tobytes())
        st_g = E.decompress_status(dev(b))
        assert st_o == -9, mutate
        assert st_g == E.EBC_ERR_ARCHIVE, mutate


def test_full_size_2d_bytes(E):
    """1800 x 3600 (CESM-ATM shape): whole archive equal at rel 1e-4 and 1e-3."""
    x = synth.climate_2d()
    xd = dev(x)
    for eb in (1e-4, 1e-3):
        ref = O.compress(x, eb)
        a = E.compress(xd, eb)
        assert a.cpu().numpy().tobytes() == ref
        y = E.decompress(a)
        np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(O.decompress(ref)))


def test_3d_dense_outliers(E):
    """Almost every delta out of range (4 bins): every 8x8x8 chunk, including
    the ragged ones on all three far faces, goes through the outlier fix-up."""
    for shape in [(19, 23, 41), (8, 8, 256)]:
        x = rng_field(shape, 21, "noise")
        ref = O.compress(x, 1e-3, n_bins=4)
        info = O.archive_info(ref)
        assert info["n_outliers"] > x.size // 2
        a = E.compress(dev(x), 1e-3, n_bins=4)
        assert a.cpu().numpy().tobytes() == ref
        y = E.decompress(a)
        np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(O.decompress(ref)))


def test_3d_corrupt_outlier_rejected(E):
    """A 3D outlier index moved onto a non-placeholder code is rejected."""
    x = rng_field((24, 40, 33), 25, "lognormal")
    raw = E.compress(dev(x), 1e-4).cpu().numpy().copy()
    s = O.sections(raw.tobytes())
    assert s["info"]["n_outliers"] > 0
    oo = s["off_oidx"]
    it = O.intermediates(x, 1e-4)
    nz = int(np.flatnonzero(it["q"].ravel() != 0)[0])
    b = raw.copy()
    b[oo:oo + 4] = np.frombuffer(np.uint32(nz).tobytes(), np.uint8)
    assert O.decompress_status(b.tobytes()) == -9
    assert E.decompress_status(dev(b)) == E.EBC_ERR_ARCHIVE


def test_stage_timing_options(E):
    """Every stage timed, or only the named one (one event pair)."""
    x = dev(rng_field((24, 40, 33), 25, "lognormal"))
    a, cs = E.compress(x, 1e-4, stats=True)
    y, ds = E.decompress(a, stats=True)
    assert {"construct", "encode_write"} <= set(cs.stages())
    assert {"huffman_decode", "reconstruct", "outlier_scatter", "outlier_fix"} <= set(ds.stages())
    y2, d1 = E.decompress(a, stats="reconstruct")
    st = d1.stages()
    assert list(st) == ["reconstruct"] and st["reconstruct"] > 0
    np.testing.assert_array_equal(bits(y2.cpu().numpy()), bits(y.cpu().numpy()))
    _, c1 = E.compress(x, 1e-4, stats="construct")
    assert list(c1.stages()) == ["construct"]


def test_full_size_3d_bench_workload(E):
    """The benchmark's 512^3 lognormal field at rel 1e-4, plain path with the
    default tiling (the configuration the benchmark times): whole archive and
    every reconstructed value equal to the oracle's."""
    import bench

    _, gen, eb = bench.WORKLOADS["nyx512"]
    x = gen(synth)
    print("[full-size 3d] oracle", flush=True)
    ref = O.compress(x, eb)
    want = O.decompress(ref)
    print("[full-size 3d] gpu", flush=True)
    xd = dev(x)
    a = E.compress(xd, eb)
    assert a.cpu().numpy().tobytes() == ref
    del xd
    y = E.decompress(a)
    np.testing.assert_array_equal(bits(y.cpu().numpy()), bits(want))


def test_corrupt_rle_archives_rejected(E):
    """Run lengths that are zero, longer than the field, or that wrap modulo
    2^32 while every one stays within the field and their sum modulo 2^32 is
    still N, are rejected on both sides: the runs must cover the field
    exactly, one non-empty run after the other."""
    n = 1 << 20
    x = np.random.default_rng(7).standard_normal(n).astype(np.float32)
    raw = np.frombuffer(O.compress(x, 1e-2, codec="rle"), np.uint8).copy()
    info = O.archive_info(raw.tobytes())
    R = info["n_a"]
    assert info["codec"] == O.ARC_RLE and R > 8192
    off_len = (128 + 2 * R + 15) & ~15
    lens = raw[off_len:off_len + 4 * R].view(np.uint32).copy()
    for mutate in ("zero", "long", "wrap"):
        L = lens.astype(np.uint64)
        if mutate == "zero":
            # a zero-length run, its length moved to the next run (sum unchanged)
            L[1] += L[0]
            L[0] = 0
        elif mutate == "long":
            L[0] = n + 1
        else:
            # 4096 runs of length n add 2^32 (zero modulo 2^32); the last run
            # takes what they displaced, so the sum modulo 2^32 is n again
            moved = int(L[:4096].sum())
            L[:4096] = n
            L[-1] += moved
            assert int(L.max()) <= n and int(L.sum()) % (1 << 32) == n
        b = raw.copy()
        b[off_len:off_len + 4 * R] = L.astype(np.uint32).view(np.uint8)
        assert O.decompress_status(b.tobytes()) == -9, mutate
        assert E.decompress_status(dev(b)) == E.EBC_ERR_ARCHIVE, mutate


@pytest.mark.parametrize("hc", [8192, 65536])
def test_huffman_chunks_longer_than_a_pass(E, hc):
    """Chunks longer than one encode pass (4096 symbols): the encoder carries
    the partial word between passes; the decoder starts every 256-symbol
    sub-chunk on its own.  Fields span several chunks and end on a short one."""
    for x in (rng_field((300, 500), 15, "grf"), rng_field((70, 90), 16, "noise")):
        ref = O.compress(x, 1e-4, codec="huffman", hc=hc)
        a = E.compress(dev(x), 1e-4, codec="huffman", huff_chunk=hc)
        assert a.cpu().numpy().tobytes() == ref
        np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))
    # codewords longer than 32 bits across passes
    xf, _ = fibonacci_deltas_field(34, 33)
    ref = O.compress(xf, 0.5, "abs", codec="huffman", hc=hc)
    a = E.compress(dev(xf), 0.5, "abs", codec="huffman", huff_chunk=hc)
    assert a.cpu().numpy().tobytes() == ref


@pytest.mark.parametrize("hc", [64, 8192])
def test_wide_bins_chunk_sizes(E, hc):
    """65536 bins with the shortest chunk and with chunks longer than an
    encode pass (the wide-table variants of both encode paths)."""
    x = rng_field((256, 300), 15, "noise")
    ref = O.compress(x, 1e-5, n_bins=65536, codec="huffman", hc=hc)
    a = E.compress(dev(x), 1e-5, n_bins=65536, codec="huffman", huff_chunk=hc)
    assert a.cpu().numpy().tobytes() == ref
    np.testing.assert_array_equal(bits(E.decompress(a).cpu().numpy()), bits(O.decompress(ref)))
