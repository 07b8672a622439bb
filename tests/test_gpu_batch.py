"""GPU: the batched path (many fields through one launch sequence), its HIP
graph replay, and tuning invariance, all checked against the CPU oracle.

The bar is the same as for single fields: archive bytes identical to the
oracle's, reconstructions bit-identical.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EB = 1e-4


@pytest.fixture(scope="module")
def E():
    from paper_2105_12912_amd import ebc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ebc.lib()
    return ebc


def make(shape, kind, seed):
    if kind == "walk":
        return synth.random_walk_1d(shape[0], seed)
    if kind == "noise":
        return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)
    if kind == "const":
        return np.full(shape, 0.25, dtype=np.float32)
    if kind == "lognormal":
        return synth.lognormal_3d(shape, seed)
    return synth.grf_field(shape, seed)


# mixed ranks and sizes: ragged tails, tiny, constant, several tiles
BATCH = [
    ((50000,), "walk", 21), ((37, 53), "grf", 22), ((9, 10, 11), "grf", 23),
    ((256, 256), "grf", 24), ((24, 40, 33), "lognormal", 25), ((1000003,), "walk", 26),
    ((16, 8, 600), "grf", 27), ((7,), "noise", 28), ((64, 64), "const", 29),
    ((100, 50, 50), "grf", 30), ((300, 6), "noise", 31), ((1,), "noise", 32),
]


@pytest.fixture(scope="module")
def fields():
    return [make(s, k, sd) for s, k, sd in BATCH]


@pytest.fixture(scope="module")
def oracle_arcs(fields):
    return [O.compress(x, EB, "rel") for x in fields]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_batch_compress_matches_oracle_and_single(E, fields, oracle_arcs):
    from paper_2105_12912_amd.batch import BatchCompress

    xs = [dev(x) for x in fields]
    B = BatchCompress(xs, EB)
    B.launch()
    arcs = B.archives()
    for i, (a, ref) in enumerate(zip(arcs, oracle_arcs)):
        got = a.cpu().numpy().tobytes()
        assert got == ref, f"field {i} {BATCH[i]}"
        single = E.compress(xs[i], EB, "rel").cpu().numpy().tobytes()
        assert single == ref, f"single field {i}"


def test_batch_decompress_matches_oracle(E, fields, oracle_arcs):
    from paper_2105_12912_amd.batch import BatchDecompress

    arcs = [torch.from_numpy(np.frombuffer(a, dtype=np.uint8).copy()).cuda() for a in oracle_arcs]
    D = BatchDecompress(arcs)
    D.launch()
    assert D.statuses() == [0] * len(arcs)
    for i, (y, a) in enumerate(zip(D.outs, oracle_arcs)):
        ref = O.decompress(a)
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32).ravel(),
                                      ref.view(np.uint32).ravel(), err_msg=f"field {i}")


def test_batch_graph_replays_match_eager(E, fields, oracle_arcs):
    """Capture once, replay several times with eager work in between; every
    replay must rewrite every byte identically."""
    from paper_2105_12912_amd.batch import BatchCompress, BatchDecompress

    xs = [dev(x) for x in fields]
    B = BatchCompress(xs, EB)
    B.capture()
    for rep in range(3):
        for o in B.outs:
            o.fill_(0xA5)
        B.res.zero_()
        torch.cuda.synchronize()
        B.replay()
        torch.cuda.synchronize()
        arcs = B.archives()
        for i, a in enumerate(arcs):
            assert a.cpu().numpy().tobytes() == oracle_arcs[i], f"replay {rep} field {i}"
    D = BatchDecompress(arcs)
    D.capture()
    refs = [O.decompress(a) for a in oracle_arcs]
    for rep in range(3):
        for o in D.outs:
            o.fill_(float("nan"))
        D.status.fill_(-99)
        torch.cuda.synchronize()
        D.replay()
        torch.cuda.synchronize()
        assert D.statuses() == [0] * len(arcs)
        for i, y in enumerate(D.outs):
            np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32).ravel(),
                                          refs[i].view(np.uint32).ravel(),
                                          err_msg=f"replay {rep} field {i}")


def test_batch_field_error_is_isolated(E, fields, oracle_arcs):
    from paper_2105_12912_amd.batch import BatchCompress

    bad = fields[3].copy()
    bad[5, 7] = np.nan
    xs = [dev(x) for x in fields[:3]] + [dev(bad)] + [dev(x) for x in fields[4:6]]
    B = BatchCompress(xs, EB)
    B.launch()
    res = B.results()
    assert res[3][1] == E.EBC_ERR_NONFINITE and res[3][0] == 0
    for i in (0, 1, 2, 4, 5):
        assert res[i][1] == 0
        assert B.outs[i][:res[i][0]].cpu().numpy().tobytes() == oracle_arcs[i]


@pytest.mark.parametrize("wx,grid,scan", [(1, 64, 1), (2, 1024, 0), (4, 4096, 1 << 20), (1, 16384, 2),
                                          (4, 64, 64)])
def test_tuning_never_changes_bytes(E, fields, oracle_arcs, wx, grid, scan):
    """Extreme tiles, grids and scan schedules (1: every scan of more than one
    tile scans its tile sums first; 2^20: never) give the same bytes."""
    entries = []
    for x in fields:
        rank = x.ndim
        nxc, nc = E.ebc_shape_class(rank, tuple(reversed(x.shape)))
        entries.append(dict(rank=rank, nx_class=nxc, n_class=nc, tile_wx=wx, grid=grid,
                            scan_direct=scan))
    assert E.ebc_set_tuning(entries) == 0
    try:
        ws = E.Workspace("cuda")
        for i, x in enumerate(fields):
            a = E.compress(dev(x), EB, "rel", workspace=ws)
            assert a.cpu().numpy().tobytes() == oracle_arcs[i], f"field {i} wx {wx} grid {grid}"
            y = E.decompress(a, workspace=ws)
            ref = O.decompress(oracle_arcs[i])
            np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32).ravel(),
                                          ref.view(np.uint32).ravel())
    finally:
        assert E.ebc_set_tuning([]) == 0


def test_batch_decompress_mixed_bin_counts(E):
    """One batched decompression over archives of different bin counts (64,
    1024, 8192, 65536; Huffman and RLE+VLE): narrow and wide decoder tables
    are built in the same call at the stride of the widest."""
    from paper_2105_12912_amd.batch import BatchDecompress

    rng = np.random.default_rng(21)
    cases = [
        (synth.smooth_2d(96, 130, 3), 1e-4, 64, "huffman"),
        (rng.standard_normal((200, 150)).astype(np.float32), 1e-5, 65536, "huffman"),
        (synth.lognormal_3d((24, 40, 33), 5), 1e-3, 1024, "auto"),
        (synth.random_walk_1d(300_001, 8), 1e-5, 8192, "huffman"),
        (synth.lognormal_3d((32, 48, 40), 6), 3e-2, 16384, "rle_vle"),
    ]
    refs = [O.compress(x, eb, n_bins=nb, codec=c) for x, eb, nb, c in cases]
    arcs = [torch.from_numpy(np.frombuffer(a, dtype=np.uint8).copy()).cuda() for a in refs]
    D = BatchDecompress(arcs)
    D.launch()
    assert D.statuses() == [0] * len(arcs)
    for i, (y, a) in enumerate(zip(D.outs, refs)):
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32).ravel(),
                                      O.decompress(a).view(np.uint32).ravel(), err_msg=f"field {i}")
