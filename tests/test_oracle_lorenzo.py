"""Pins of the oracle's prediction / reconstruction steps (CPU only).

Nothing here re-types the oracle's formulas.  The Lorenzo difference is pinned
against a different formulation (the separable backward-difference operator
Delta_z Delta_y Delta_x with zero boundaries), against closed forms, and its
inverse against numpy's cumulative sum per chunk and axis -- the N-D partial
sum of Sec. IV-B.2 computed with a textbook routine.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O


def chunk_views(shape, chunk):
    """Yield index slices of every chunk (x fastest in `chunk`, numpy order in shape)."""
    nd = len(shape)
    ch = list(chunk[:nd])[::-1]  # numpy axis order
    ranges = [range(0, s, c) for s, c in zip(shape, ch)]
    for starts in itertools.product(*ranges):
        yield tuple(slice(s, min(s + c, n)) for s, c, n in zip(starts, ch, shape))


def backward_diff_within_chunks(d, chunk):
    """Apply Delta along every axis: v[i] - v[i-1], with v[-1] := 0 at a chunk start."""
    out = d.astype(np.int64)
    for sl in chunk_views(d.shape, chunk):
        blk = out[sl]
        for ax in range(blk.ndim):
            blk = np.diff(blk, axis=ax, prepend=0)
        out[sl] = blk
    return out


def cumsum_within_chunks(q, chunk):
    out = q.astype(np.int64)
    for sl in chunk_views(q.shape, chunk):
        blk = out[sl]
        for ax in range(blk.ndim):
            blk = np.cumsum(blk, axis=ax)
        out[sl] = blk
    return out


SHAPES = [
    ((37,), (8, 1, 1)),
    ((600,), None),
    ((1,), None),
    ((13, 21), (4, 8, 1)),
    ((40, 35), None),
    ((1, 1), None),
    ((9, 11, 13), (4, 2, 8)),
    ((17, 9, 20), None),
    ((1, 1, 1), None),
]


@pytest.mark.parametrize("shape,chunk", SHAPES)
def test_lorenzo_equals_separable_differences(shape, chunk):
    rng = np.random.default_rng(11)
    rank = len(shape)
    d = rng.integers(-1000, 1000, size=shape, dtype=np.int32)
    ch = chunk or O.default_chunk(rank)
    got = O.lorenzo(d, rank, ch)
    want = backward_diff_within_chunks(d, ch)
    np.testing.assert_array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("shape,chunk", SHAPES)
def test_reconstruct_equals_chunked_cumsum(shape, chunk):
    """Sequential recurrence == N-D partial sum per chunk (Sec. IV-B.2)."""
    rng = np.random.default_rng(12)
    rank = len(shape)
    qp = rng.integers(-50, 50, size=shape, dtype=np.int32)
    ch = chunk or O.default_chunk(rank)
    got = O.reconstruct(qp, rank, ch)
    want = cumsum_within_chunks(qp, ch)
    np.testing.assert_array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("shape,chunk", SHAPES)
def test_partial_sum_inverts_lorenzo(shape, chunk):
    rng = np.random.default_rng(13)
    rank = len(shape)
    d = rng.integers(-(1 << 18), 1 << 18, size=shape, dtype=np.int32)
    ch = chunk or O.default_chunk(rank)
    np.testing.assert_array_equal(O.reconstruct(O.lorenzo(d, rank, ch), rank, ch), d)


def test_lorenzo_2d_linear_field_closed_form():
    """d = a + b x + c y: the 2D difference vanishes inside a chunk; on a chunk's
    first row it is the 1D x-difference (b, or d itself at the corner), and on its
    first column the 1D y-difference."""
    ny, nx = 35, 50
    y, x = np.mgrid[0:ny, 0:nx]
    a, b, c = 7, 3, -5
    d = (a + b * x + c * y).astype(np.int32)
    delta = O.lorenzo(d, 2)
    for yy in range(ny):
        for xx in range(nx):
            fy, fx = yy % 16 == 0, xx % 16 == 0
            if fy and fx:
                want = d[yy, xx]
            elif fy:
                want = b
            elif fx:
                want = c
            else:
                want = 0
            assert delta[yy, xx] == want, (yy, xx)


def test_lorenzo_3d_constant_field_closed_form():
    """A constant c gives delta = c at each 8x8x8 chunk origin and 0 elsewhere."""
    d = np.full((19, 10, 17), 42, dtype=np.int32)
    delta = O.lorenzo(d, 3)
    z, y, x = np.indices(d.shape)
    origin = (z % 8 == 0) & (y % 8 == 0) & (x % 8 == 0)
    np.testing.assert_array_equal(delta[origin], 42)
    np.testing.assert_array_equal(delta[~origin], 0)


def test_lorenzo_1d_is_first_difference():
    d = np.arange(1000, dtype=np.int32) ** 2 % 977
    delta = O.lorenzo(d, 1)
    for i in range(1000):
        want = d[i] if i % 256 == 0 else d[i] - d[i - 1]
        assert delta[i] == want


def test_lorenzo_axes_are_not_transposed():
    """An impulse at one point only affects the +x, +y, +z neighbours of its chunk."""
    d = np.zeros((8, 8, 8), dtype=np.int32)
    d[2, 3, 4] = 1
    delta = O.lorenzo(d, 3)
    nz = np.argwhere(delta != 0)
    got = {tuple(p): int(delta[tuple(p)]) for p in nz}
    want = {}
    for dz, dy, dx in itertools.product((0, 1), repeat=3):
        want[(2 + dz, 3 + dy, 4 + dx)] = (-1) ** (dz + dy + dx)
    assert got == want
