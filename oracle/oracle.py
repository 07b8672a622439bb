"""ctypes wrapper around the plain CPU oracle (``libebc_oracle.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product library never does.
Every function returns numpy arrays and raises ``OracleError`` on a non-zero
status.  Arrays are field-shaped ``(nz, ny, nx)`` for rank 3, ``(ny, nx)`` for
rank 2 and ``(nx,)`` for rank 1; ``dims`` is always ``(nx, ny, nz)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ebc_oracle.c")
LIB = os.path.join(HERE, "libebc_oracle.so")

OK = 0
ERR = {
    -1: "ARG", -2: "DIMS", -3: "EB", -4: "EB_TOO_SMALL", -5: "BINS", -6: "NONFINITE",
    -7: "OUT_TOO_SMALL", -8: "WS_TOO_SMALL", -9: "ARCHIVE", -10: "HIP", -11: "UNSUPPORTED",
    -12: "NOMEM",
}
ARC_HUFFMAN, ARC_RLE, ARC_CONST, ARC_RLE_VLE = 0, 1, 2, 3
REQ_AUTO, REQ_HUFFMAN, REQ_RLE, REQ_RLE_VLE, REQ_AUTO_VLE = 0, 1, 2, 3, 4
CODEC_REQ = {"auto": REQ_AUTO, "huffman": REQ_HUFFMAN, "rle": REQ_RLE, "rle_vle": REQ_RLE_VLE,
             "auto_vle": REQ_AUTO_VLE}
EB_ABS, EB_REL = 0, 1
DT_F32, DT_F64 = 0, 1
HDR_BYTES = 128


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__(f"oracle {what}: status {status} ({ERR.get(status, '?')})")
        self.status = status


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (binary64 SSE2, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        u64, u32, i32, f64 = C.c_uint64, C.c_uint32, C.c_int, C.c_double
        sig = {
            "ora_value_range": (i32, [P, u64, P, P]),
            "ora_value_range64": (i32, [P, u64, P, P]),
            "ora_quant_step": (i32, [f64, f64, P, P, P]),
            "ora_quant_step64": (i32, [f64, f64, P, P, P]),
            "ora_prequant": (None, [P, u64, f64, P]),
            "ora_prequant64": (None, [P, u64, f64, P]),
            "ora_sub_chunk": (u32, [u32]),
            "ora_lorenzo": (None, [P, i32, P, P, P]),
            "ora_postquant": (u64, [P, u64, u32, P, P, P]),
            "ora_histogram": (None, [P, u64, u32, P]),
            "ora_huffman_lengths": (i32, [P, u32, P]),
            "ora_canonical_codes": (i32, [P, u32, P]),
            "ora_choose_rle": (i32, [P, P, u32, u64]),
            "ora_huffman_encode": (u64, [P, u64, P, P, u32, P, P]),
            "ora_huffman_decode": (i32, [P, P, u64, u64, u32, P, u32, P]),
            "ora_rle_encode": (u64, [P, u64, P, P]),
            "ora_rle_decode": (i32, [P, P, u64, u64, P]),
            "ora_fuse": (i32, [P, u64, u32, P, P, u64, P]),
            "ora_reconstruct": (None, [P, i32, P, P, P]),
            "ora_dequant": (None, [P, u64, f64, P]),
            "ora_dequant64": (None, [P, u64, f64, P]),
            "ora_estimate_hist": (None, [P, u32, u64, P, P, P, P, P]),
            "ora_splitmix64": (u64, [u64, u64]),
            "ora_madogram": (None, [P, u64, u64, u64, u32, P, P]),
            "ora_compress_bound": (u64, [i32, P, u32, u32]),
            "ora_compress": (i32, [P, i32, i32, P, i32, f64, u32, i32, u32, P, P, u64, P]),
            "ora_decompress": (i32, [P, u64, P, u64]),
            "ora_archive_info": (i32, [P, u64, P, P, P, P, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dims(dims) -> np.ndarray:
    d = np.ones(3, dtype=np.uint64)
    d[: len(dims)] = dims
    return d


def default_chunk(rank: int):
    return {1: (256, 1, 1), 2: (16, 16, 1), 3: (8, 8, 8)}[rank]


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


# ----------------------------------------------------------------- steps

def _is64(x) -> bool:
    return np.asarray(x).dtype == np.float64


def value_range(x: np.ndarray):
    if _is64(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        mn, mx = C.c_double(), C.c_double()
        _check(lib().ora_value_range64(_p(x), x.size, C.byref(mn), C.byref(mx)), "value_range")
        return np.float64(mn.value), np.float64(mx.value)
    x = np.ascontiguousarray(x, dtype=np.float32)
    mn, mx = C.c_float(), C.c_float()
    _check(lib().ora_value_range(_p(x), x.size, C.byref(mn), C.byref(mx)), "value_range")
    return np.float32(mn.value), np.float32(mx.value)


def quant_step(M: float, eb_abs: float, fp64: bool = False):
    ebx2, inv, e = C.c_double(), C.c_double(), C.c_int()
    fn = lib().ora_quant_step64 if fp64 else lib().ora_quant_step
    _check(fn(float(M), float(eb_abs), C.byref(ebx2), C.byref(inv), C.byref(e)), "quant_step")
    return ebx2.value, inv.value, e.value


def prequant(x: np.ndarray, inv: float) -> np.ndarray:
    if _is64(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        d = np.empty(x.shape, dtype=np.int32)
        lib().ora_prequant64(_p(x), x.size, float(inv), _p(d))
        return d
    x = np.ascontiguousarray(x, dtype=np.float32)
    d = np.empty(x.shape, dtype=np.int32)
    lib().ora_prequant(_p(x), x.size, float(inv), _p(d))
    return d


def lorenzo(d: np.ndarray, rank: int, chunk=None) -> np.ndarray:
    """delta = d - Lorenzo prediction, zero outside each chunk."""
    d = np.ascontiguousarray(d, dtype=np.int32)
    dims = _dims(d.shape[::-1])
    ch = np.array(chunk or default_chunk(rank), dtype=np.uint32)
    out = np.empty_like(d)
    lib().ora_lorenzo(_p(d), rank, _p(dims), _p(ch), _p(out))
    return out


def postquant(delta: np.ndarray, n_bins: int):
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    q = np.empty(delta.shape, dtype=np.uint16)
    n = lib().ora_postquant(_p(delta), delta.size, n_bins, _p(q), None, None)
    idx = np.empty(max(n, 1), dtype=np.uint32)
    val = np.empty(max(n, 1), dtype=np.int32)
    lib().ora_postquant(_p(delta), delta.size, n_bins, _p(q), _p(idx), _p(val))
    return q, idx[:n], val[:n]


def histogram(q: np.ndarray, n_bins: int) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.uint16)
    h = np.empty(n_bins, dtype=np.uint64)
    lib().ora_histogram(_p(q), q.size, n_bins, _p(h))
    return h


def huffman_lengths(hist: np.ndarray) -> np.ndarray:
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    ln = np.empty(hist.size, dtype=np.uint8)
    _check(lib().ora_huffman_lengths(_p(hist), hist.size, _p(ln)), "huffman_lengths")
    return ln


def canonical_codes(length: np.ndarray) -> np.ndarray:
    length = np.ascontiguousarray(length, dtype=np.uint8)
    code = np.empty(length.size, dtype=np.uint64)
    _check(lib().ora_canonical_codes(_p(length), length.size, _p(code)), "canonical_codes")
    return code


def choose_rle(hist: np.ndarray, length: np.ndarray, n: int) -> bool:
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    length = np.ascontiguousarray(length, dtype=np.uint8)
    return bool(lib().ora_choose_rle(_p(hist), _p(length), hist.size, int(n)))


def sub_chunk(hc: int) -> int:
    """Symbols per Huffman sub-chunk (the unit of the stored bit counts)."""
    return int(lib().ora_sub_chunk(hc))


def huffman_encode(q: np.ndarray, length: np.ndarray, code: np.ndarray, hc: int = 1024):
    """Returns (sbits, words): u16 bit count per sub-chunk, u32 words."""
    q = np.ascontiguousarray(q, dtype=np.uint16).ravel()
    hs = sub_chunk(hc)
    nsub = (q.size + hs - 1) // hs
    bits = np.empty(max(nsub, 1), dtype=np.uint16)
    nw = lib().ora_huffman_encode(_p(q), q.size, _p(length), _p(code), hc, _p(bits), None)
    words = np.empty(max(nw, 1), dtype=np.uint32)
    lib().ora_huffman_encode(_p(q), q.size, _p(length), _p(code), hc, _p(bits), _p(words))
    return bits[:nsub], words[:nw]


def huffman_decode(bits, words, n: int, length, hc: int = 1024) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint16)
    words = np.ascontiguousarray(words, dtype=np.uint32)
    length = np.ascontiguousarray(length, dtype=np.uint8)
    q = np.empty(n, dtype=np.uint16)
    w = words if words.size else np.zeros(1, dtype=np.uint32)
    _check(lib().ora_huffman_decode(_p(bits), _p(w), words.size, n, hc, _p(length), length.size,
                                    _p(q)), "huffman_decode")
    return q


def rle_encode(q: np.ndarray):
    q = np.ascontiguousarray(q, dtype=np.uint16).ravel()
    r = lib().ora_rle_encode(_p(q), q.size, None, None)
    val = np.empty(max(r, 1), dtype=np.uint16)
    ln = np.empty(max(r, 1), dtype=np.uint32)
    lib().ora_rle_encode(_p(q), q.size, _p(val), _p(ln))
    return val[:r], ln[:r]


def rle_decode(val, ln, n: int) -> np.ndarray:
    val = np.ascontiguousarray(val, dtype=np.uint16)
    ln = np.ascontiguousarray(ln, dtype=np.uint32)
    q = np.empty(n, dtype=np.uint16)
    _check(lib().ora_rle_decode(_p(val), _p(ln), val.size, n, _p(q)), "rle_decode")
    return q


def fuse(q: np.ndarray, n_bins: int, idx, val) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.uint16)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    val = np.ascontiguousarray(val, dtype=np.int32)
    qp = np.empty(q.shape, dtype=np.int32)
    i = idx if idx.size else np.zeros(1, np.uint32)
    v = val if val.size else np.zeros(1, np.int32)
    _check(lib().ora_fuse(_p(q), q.size, n_bins, _p(i), _p(v), idx.size, _p(qp)), "fuse")
    return qp


def reconstruct(qp: np.ndarray, rank: int, chunk=None) -> np.ndarray:
    qp = np.ascontiguousarray(qp, dtype=np.int32)
    dims = _dims(qp.shape[::-1])
    ch = np.array(chunk or default_chunk(rank), dtype=np.uint32)
    d = np.empty_like(qp)
    lib().ora_reconstruct(_p(qp), rank, _p(dims), _p(ch), _p(d))
    return d


def dequant(d: np.ndarray, ebx2: float, fp64: bool = False) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.int32)
    out = np.empty(d.shape, dtype=np.float64 if fp64 else np.float32)
    (lib().ora_dequant64 if fp64 else lib().ora_dequant)(_p(d), d.size, float(ebx2), _p(out))
    return out


def estimate_hist(hist: np.ndarray, n: int | None = None) -> dict:
    """Entropy, p1, the redundancy bounds and the predicted workflow
    (1 run-length, 0 Huffman, 2 undecided) from a histogram."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    n = int(hist.sum()) if n is None else int(n)
    H, p1, lo, hi, pr = C.c_double(), C.c_double(), C.c_double(), C.c_double(), C.c_int()
    lib().ora_estimate_hist(_p(hist), hist.size, n, C.byref(H), C.byref(p1), C.byref(lo),
                            C.byref(hi), C.byref(pr))
    return dict(entropy=H.value, p1=p1.value, r_lo=lo.value, r_hi=hi.value, predict=pr.value,
                bits_lo=H.value + lo.value, bits_hi=H.value + hi.value)


def splitmix64(seed: int, k: int) -> int:
    return int(lib().ora_splitmix64(seed, k))


def madogram(q: np.ndarray, samples: int, seed: int, dmax: int = 200):
    """(sum, cnt) per distance 0..dmax of the sampled binary madogram."""
    q = np.ascontiguousarray(q, dtype=np.uint16).ravel()
    s = np.zeros(dmax + 1, dtype=np.uint64)
    c = np.zeros(dmax + 1, dtype=np.uint64)
    lib().ora_madogram(_p(q), q.size, int(samples), int(seed), dmax, _p(s), _p(c))
    return s, c


# -------------------------------------------------------------- pipeline

def compress_bound(rank: int, dims, n_bins: int = 1024, hc: int = 1024) -> int:
    return int(lib().ora_compress_bound(rank, _p(_dims(dims)), n_bins, hc))


def compress(x: np.ndarray, eb: float, mode: str = "rel", n_bins: int = 1024,
             codec: str = "auto", hc: int = 1024, chunk=None, rank: int | None = None) -> bytes:
    """Whole compression pipeline; returns the archive bytes.  x is fp32, or
    fp64 (an fp64 archive)."""
    fp64 = _is64(x)
    x = np.ascontiguousarray(x, dtype=np.float64 if fp64 else np.float32)
    rank = rank or x.ndim
    dims = _dims(x.shape[::-1])
    cap = max(compress_bound(rank, dims[:rank], n_bins, hc), HDR_BYTES)
    out = np.empty(cap, dtype=np.uint8)
    size = C.c_uint64()
    ch = None if chunk is None else _p(np.array(chunk, dtype=np.uint32))
    st = lib().ora_compress(_p(x), DT_F64 if fp64 else DT_F32, rank, _p(dims),
                            EB_REL if mode == "rel" else EB_ABS, float(eb), n_bins,
                            CODEC_REQ[codec], hc, ch, _p(out), cap, C.byref(size))
    _check(st, "compress")
    return out[: size.value].tobytes()


def compress_status(x: np.ndarray, eb: float, mode: str = "rel", n_bins: int = 1024,
                    rank: int | None = None, dims=None, codec: str = "auto", hc: int = 1024) -> int:
    """Status of a compression attempt (for error-path tests)."""
    fp64 = _is64(x)
    x = np.ascontiguousarray(x, dtype=np.float64 if fp64 else np.float32)
    rank = rank if rank is not None else x.ndim
    d = _dims(dims if dims is not None else x.shape[::-1])
    out = np.empty(max(24 * x.size + 4096, 256), dtype=np.uint8)
    size = C.c_uint64()
    return lib().ora_compress(_p(x), DT_F64 if fp64 else DT_F32, rank, _p(d),
                              EB_REL if mode == "rel" else EB_ABS, float(eb), n_bins,
                              CODEC_REQ[codec], hc, None, _p(out), out.size, C.byref(size))


def archive_info(a: bytes) -> dict:
    buf = np.frombuffer(a, dtype=np.uint8)
    rank, codec, nb, dt, hc = C.c_int(), C.c_int(), C.c_uint32(), C.c_int(), C.c_uint32()
    dims = np.zeros(3, dtype=np.uint64)
    no, na, nw, ebx2 = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_double()
    _check(lib().ora_archive_info(_p(buf), buf.size, C.byref(rank), _p(dims), C.byref(codec),
                                  C.byref(nb), C.byref(no), C.byref(na), C.byref(nw),
                                  C.byref(ebx2), C.byref(dt), C.byref(hc)), "archive_info")
    return dict(rank=rank.value, dims=tuple(int(v) for v in dims), codec=codec.value,
                n_bins=nb.value, n_outliers=no.value, n_a=na.value, n_words=nw.value,
                ebx2=ebx2.value, dtype=dt.value, hc=hc.value)


def decompress(a: bytes) -> np.ndarray:
    info = archive_info(a)
    nx, ny, nz = info["dims"]
    shape = {1: (nx,), 2: (ny, nx), 3: (nz, ny, nx)}[info["rank"]]
    out = np.empty(shape, dtype=np.float64 if info["dtype"] == DT_F64 else np.float32)
    buf = np.frombuffer(a, dtype=np.uint8)
    _check(lib().ora_decompress(_p(buf), buf.size, _p(out), out.size), "decompress")
    return out


def decompress_status(a: bytes) -> int:
    buf = np.frombuffer(bytes(a), dtype=np.uint8)
    try:
        info = archive_info(bytes(a))
        n = int(np.prod(info["dims"]))
    except OracleError as e:
        return e.status
    out = np.empty(max(n, 1), dtype=np.float64)
    return lib().ora_decompress(_p(buf), buf.size, _p(out), out.size)


def _a16(v):
    return (v + 15) & ~15


def huffman_layout(m: int, n_bins: int, hc: int, n_words: int, base: int = HDR_BYTES) -> dict:
    """Section offsets of a Huffman stream of m symbols (format v2)."""
    hs = sub_chunk(hc)
    nsub = (m + hs - 1) // hs
    ol = base
    ob = _a16(ol + n_bins)
    ow = _a16(ob + 2 * nsub)
    return dict(len=ol, sbits=ob, words=ow, end=_a16(ow + 4 * n_words), n_sub=nsub)


def sections(a: bytes) -> dict:
    """Split an archive into its named arrays (format v2 layout)."""
    info = archive_info(a)
    buf = np.frombuffer(a, dtype=np.uint8)
    nb, no = info["n_bins"], info["n_outliers"]
    nx, ny, nz = info["dims"]
    out = dict(info=info)
    if info["codec"] in (ARC_HUFFMAN, ARC_RLE_VLE):
        m = nx * ny * nz if info["codec"] == ARC_HUFFMAN else info["n_a"]
        L = huffman_layout(m, nb, info["hc"], info["n_words"])
        out["layout"] = L
        out["len"] = buf[L["len"]:L["len"] + nb].copy()
        out["sbits"] = buf[L["sbits"]:L["sbits"] + 2 * L["n_sub"]].view(np.uint16).copy()
        out["words"] = buf[L["words"]:L["words"] + 4 * info["n_words"]].view(np.uint32).copy()
        oo = L["end"]
        if info["codec"] == ARC_RLE_VLE:
            r = info["n_a"]
            out["off_rlen"] = oo
            out["rlen"] = buf[oo:oo + 4 * r].view(np.uint32).copy()
            oo = _a16(oo + 4 * r)
    elif info["codec"] == ARC_RLE:
        r = info["n_a"]
        ol = _a16(HDR_BYTES + 2 * r)
        oo = _a16(ol + 4 * r)
        out["off_rlen"] = ol
        out["val"] = buf[HDR_BYTES:HDR_BYTES + 2 * r].view(np.uint16).copy()
        out["rlen"] = buf[ol:ol + 4 * r].view(np.uint32).copy()
    else:
        return out
    out["off_oidx"] = oo
    out["oidx"] = buf[oo:oo + 4 * no].view(np.uint32).copy()
    ov = _a16(oo + 4 * no)
    out["oval"] = buf[ov:ov + 4 * no].view(np.int32).copy()
    return out


def intermediates(x: np.ndarray, eb: float, mode: str = "rel", n_bins: int = 1024, chunk=None,
                  rank: int | None = None) -> dict:
    """Every intermediate of the compression pipeline, step by step."""
    fp64 = _is64(x)
    x = np.ascontiguousarray(x, dtype=np.float64 if fp64 else np.float32)
    rank = rank or x.ndim
    mn, mx = value_range(x)
    rng = float(mx) - float(mn)
    M = max(abs(float(mn)), abs(float(mx)))
    eb_abs = eb * rng if mode == "rel" else eb
    ebx2, inv, e = quant_step(M, eb_abs, fp64)
    d = prequant(x, inv)
    delta = lorenzo(d, rank, chunk)
    q, idx, val = postquant(delta, n_bins)
    hist = histogram(q, n_bins)
    ln = huffman_lengths(hist)
    code = canonical_codes(ln)
    return dict(mn=mn, mx=mx, eb_abs=eb_abs, ebx2=ebx2, inv=inv, e=e, d=d, delta=delta, q=q,
                oidx=idx, oval=val, hist=hist, len=ln, code=code,
                rle=choose_rle(hist, ln, x.size))
