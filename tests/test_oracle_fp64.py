"""Pins of the fp64 path of the oracle (Sec. III: fp64 fields through the same
integer core, where a Huffman code of at least one bit per value caps the
ratio at 64).

The quantisation step for fp64 output keeps |x - xhat| <= eb on every
element after the final binary64 rounding: the guard eps = 2^max(k - 48, -49)
with k = ilogb(M) - ilogb(eb) covers the two roundings (product and output,
each 2^-53 relative), and k > 27 is refused because the codes would leave the
int32 range of the Lorenzo arithmetic."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_12912_amd import synth


def test_quant_step64_closed_form():
    for M, eb in [(1.0, 1e-6), (3.0, 1e-7), (1e7, 1.0), (0.0, 1e-3), (5e-300, 1e-305)]:
        ebx2, inv, e = O.quant_step(M, eb, fp64=True)
        k = (math.frexp(M)[1] - 1 if M else 0) - (math.frexp(eb)[1] - 1)
        want_e = max(k - 48, -49) if M else -49
        assert e == want_e
        assert ebx2 == (eb * (1.0 - 2.0 ** want_e)) * 2.0
        assert inv == 1.0 / ebx2
    # codes beyond the int32 Lorenzo range: the bound is too small for them
    with pytest.raises(O.OracleError) as ei:
        O.quant_step(1.0, 2.0 ** -29, fp64=True)
    assert ei.value.status == -4
    O.quant_step(1.0, 2.0 ** -27, fp64=True)


def test_fp64_error_bound_every_element():
    rng = np.random.default_rng(3)
    for shape, eb, mode in [((200, 300), 1e-7, "rel"), ((40, 30, 50), 1e-5, "rel"),
                            ((100003,), 3e-8, "abs"), ((64, 64), 1e-3, "rel")]:
        x = rng.standard_normal(shape) * 10.0 ** rng.uniform(-3, 3)
        x = np.cumsum(x, axis=-1)  # smooth along x
        if mode == "abs":
            eb = eb * float(np.abs(x).max())  # near the finest bound the codes allow
        a = O.compress(x, eb, mode)
        assert O.archive_info(a)["dtype"] == O.DT_F64
        y = O.decompress(a)
        assert y.dtype == np.float64 and y.shape == x.shape
        eb_abs = eb * (float(x.max()) - float(x.min())) if mode == "rel" else eb
        assert float(np.abs(y - x).max()) <= eb_abs


def test_fp64_integer_multiples_are_exact():
    """x = k * step with small integers k: prequantisation returns k exactly
    and the output is x itself."""
    ebx2 = O.quant_step(100.0, 0.5, fp64=True)[0]
    k = np.random.default_rng(4).integers(-100, 101, size=(30, 40))
    x = k * ebx2
    assert O.quant_step(float(np.abs(x).max()), 0.5, fp64=True)[0] == ebx2
    np.testing.assert_array_equal(O.prequant(x, 1.0 / ebx2), k)
    np.testing.assert_array_equal(O.decompress(O.compress(x, 0.5, "abs")), x)


def test_fp64_huffman_ratio_ceiling_is_64():
    """At least one bit per value: the Huffman payload of an fp64 field is at
    least N bits, so its ratio before metadata is at most 64 (32 for fp32)."""
    x = np.zeros((256, 256))
    x[0, 0] = 1.0  # range 1, almost every code the same
    a = O.compress(x, 1e-2, codec="huffman")
    s = O.sections(a)
    payload_bits = int(s["sbits"].astype(np.int64).sum())
    assert payload_bits >= x.size
    assert x.nbytes * 8 / payload_bits <= 64.0
    y = O.compress(x.astype(np.float32), 1e-2, codec="huffman")
    sy = O.sections(y)
    assert x.size * 32 / int(sy["sbits"].astype(np.int64).sum()) <= 32.0


def test_fp64_and_fp32_share_the_integer_core():
    """An fp32 field given as fp64 quantises to the same codes when the bound
    is loose enough that neither guard moves a code (both sides are exact
    there), so every section after the header matches."""
    x = synth.smooth_2d(64, 96, 8)
    a32 = O.compress(x, 1e-2)
    a64 = O.compress(x.astype(np.float64), 1e-2)
    s32, s64 = O.sections(a32), O.sections(a64)
    it32 = O.intermediates(x, 1e-2)
    it64 = O.intermediates(x.astype(np.float64), 1e-2)
    same = np.array_equal(it32["q"], it64["q"])
    if same:
        np.testing.assert_array_equal(s32["sbits"], s64["sbits"])
        np.testing.assert_array_equal(s32["words"], s64["words"])
    assert np.abs(O.decompress(a64) - x).max() <= 1e-2 * (float(x.max()) - float(x.min()))


def test_fp64_constant_and_errors():
    c = np.full((10, 10), math.pi)
    a = O.compress(c, 1e-3)
    assert O.archive_info(a)["codec"] == O.ARC_CONST
    y = O.decompress(a)
    assert y.dtype == np.float64 and (y == math.pi).all()
    z = np.linspace(-1, 1, 100)
    z[5] = np.nan
    assert O.compress_status(z, 1e-3) == -6
    assert O.compress_status(np.linspace(-1, 1, 100), 2.0 ** -40, "abs") == -4
