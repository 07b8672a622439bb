"""The C-ABI library loads on the CPU, exports every declared entry point, and
its host-only logic (validation, sizing, header parsing) behaves; no device
work is launched here."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import ebc, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ebc.LIB_PATH):
        pytest.fail("libebc.so is not built (python -m paper_2105_12912_amd.build)")
    return ebc.lib()


def test_every_declared_symbol_is_exported(L):
    names = ebc.header_symbols()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", ebc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)


def test_version_and_strings(L):
    assert ebc.ebc_version() == 1
    assert ebc.status_string(0) == "ok"
    assert "archive" in ebc.status_string(-9)
    assert ebc.status_string(12345) == "unknown status"


def test_param_validation(L):
    good = ebc.make_params(1e-4)
    assert ebc.ebc_compress_bound(2, (16, 16), good) > 0
    cases = [
        (ebc.make_params(0.0), -3), (ebc.make_params(float("inf")), -3),
        (ebc.make_params(1e-4, n_bins=3), -5), (ebc.make_params(1e-4, n_bins=70000), -5),
        (ebc.make_params(1e-4, n_bins=65538), -5), (ebc.make_params(1e-4, huff_chunk=100), -1),
        (ebc.make_params(1e-4, huff_chunk=131072), -1),
    ]
    for p, want in cases:
        with pytest.raises(ebc.EbcError) as ei:
            ebc.ebc_compress_workspace_size(2, (16, 16), p)
        assert ei.value.status == want
    # every power-of-two Huffman chunk from 64 to 65536 and every even bin
    # count from 4 to 65536 is implemented
    for hc in (64, 4096, 8192, 65536):
        assert ebc.ebc_compress_workspace_size(2, (16, 16), ebc.make_params(1e-4, huff_chunk=hc)) > 0
    for nb in (4, 4096, 4098, 8192, 65536):
        assert ebc.ebc_compress_workspace_size(2, (16, 16), ebc.make_params(1e-4, n_bins=nb)) > 0
    for rank, dims, want in [(4, (2, 2, 2), -2), (2, (16, 0), -2), (1, (5, 2), -2),
                             (3, (1 << 16, 1 << 16, 2), -2)]:
        with pytest.raises(ebc.EbcError) as ei:
            ebc.ebc_compress_workspace_size(rank, dims, good)
        assert ei.value.status == want


def test_host_side_rejections_need_no_device(L):
    p = ebc.make_params(1e-4)
    st, size = ebc.ebc_compress(None, 2, (8, 8), p, None, 0, None, 0, None)
    assert st == ebc.EBC_ERR_ARG and size == 0
    st, _ = ebc.ebc_compress(1 << 20, 2, (8, 8), p, 1 << 21, 1 << 20, 1 << 22, 16, None)
    assert st == ebc.EBC_ERR_WS_TOO_SMALL


def test_compress_bound_matches_oracle(L):
    for rank, dims, nb in [(1, (1000003,), 1024), (2, (3600, 1800), 1024), (3, (33, 17, 9), 64),
                           (2, (300, 256), 65536)]:
        assert ebc.ebc_compress_bound(rank, dims, ebc.make_params(1e-3, n_bins=nb)) == \
            O.compress_bound(rank, dims, nb)


def test_archive_info_parses_oracle_archives(L):
    x = synth.smooth_2d(40, 56, 1)
    for codec in ("huffman", "rle"):
        a = O.compress(x, 1e-3, codec=codec)
        info = ebc.ebc_archive_info(a[:128])
        assert info["rank"] == 2 and info["dims"] == (56, 40, 1)
        assert info["codec"] == (0 if codec == "huffman" else 1)
        assert info["total"] == len(a) and info["n_bins"] == 1024
        assert ebc.ebc_decompress_workspace_size(a[:128]) > 0
    with pytest.raises(ebc.EbcError) as ei:
        ebc.ebc_archive_info(b"XBC1" + bytes(124))
    assert ei.value.status == -9
    bad = bytearray(O.compress(x, 1e-3))
    bad[112] ^= 0x10  # total size field no longer matches the sections
    with pytest.raises(ebc.EbcError) as ei:
        ebc.ebc_archive_info(bytes(bad[:128]))
    assert ei.value.status == -9


def test_workspace_grows_with_field(L):
    p = ebc.make_params(1e-4)
    a = ebc.ebc_compress_workspace_size(3, (64, 64, 64), p)
    b = ebc.ebc_compress_workspace_size(3, (128, 128, 128), p)
    assert b > 6 * a
    assert a >= 6 * 64 ** 3


def test_tuning_table_validation_and_shape_class(L):
    bad = [dict(rank=4, nx_class=0, n_class=0, tile_wx=0, grid=0),
           dict(rank=2, nx_class=0, n_class=0, tile_wx=3, grid=0),
           dict(rank=2, nx_class=0, n_class=0, tile_wx=2, grid=10),
           dict(rank=3, nx_class=0, n_class=0, tile_wx=2, grid=20000)]
    for e in bad:
        assert ebc.ebc_set_tuning([e]) == ebc.EBC_ERR_ARG
    ok = dict(rank=3, nx_class=9, n_class=2, tile_wx=2, grid=1024)
    assert ebc.ebc_set_tuning([ok]) == 0
    assert ebc.ebc_set_tuning([]) == 0
    assert ebc.ebc_shape_class(3, (512, 512, 512)) == (9, 2)
    assert ebc.ebc_shape_class(2, (3600, 1800)) == (12, 1)
    assert ebc.ebc_shape_class(1, (1000,)) == (10, 0)
    assert ebc.ebc_shape_class(1, (1,)) == (0, 0)
    with pytest.raises(ebc.EbcError):
        ebc.ebc_shape_class(2, (5, 0))


def test_tuning_changes_workspace_plan_not_validity(L):
    """A tile choice changes the planned workspace (tile counts) but sizing is
    always self-consistent; tuning is host-side state only."""
    p = ebc.make_params(1e-4)
    base = ebc.ebc_compress_workspace_size(3, (100, 100, 100), p)
    nxc, nc = ebc.ebc_shape_class(3, (100, 100, 100))
    sizes = []
    for wx in (1, 2, 4):
        assert ebc.ebc_set_tuning([dict(rank=3, nx_class=nxc, n_class=nc, tile_wx=wx, grid=0)]) == 0
        sizes.append(ebc.ebc_compress_workspace_size(3, (100, 100, 100), p))
    assert ebc.ebc_set_tuning([]) == 0
    assert ebc.ebc_compress_workspace_size(3, (100, 100, 100), p) == base
    assert all(s > 0 for s in sizes)


def test_batch_unit_totals_beyond_32_bits_are_rejected(L):
    """Two 2D fields of 1 x 3e9 hold 3e9 outlier row segments each: the batch
    total passes 2^32, which the 32-bit unit indices of the kernels cannot
    address, so sizing (host only) refuses the batch instead of wrapping."""
    p = ebc.make_params(1e-4)
    one = ebc.ebc_field(d_field=None, rank=2, reserved=0, dims=(C.c_uint64 * 3)(1, 3_000_000_000, 1),
                        d_out=None, out_cap=0)
    assert ebc.ebc_batch_compress_workspace_size([one], p) > 0
    with pytest.raises(ebc.EbcError) as ei:
        ebc.ebc_batch_compress_workspace_size([one, one], p)
    assert ei.value.status == ebc.EBC_ERR_DIMS
