"""ctypes binding of the HIP C-ABI library ``libebc.so``.

Two layers:

* the raw entry points, with the same names and arguments as ``include/ebc.h``
  (``ebc_compress``, ``ebc_decompress``, ... ; pointers and streams are plain
  integers), and
* thin conveniences over torch tensors (``compress``, ``decompress``,
  ``debug_construct``, ...).  torch only provides device memory and streams;
  every step of the pipeline runs in the library's HIP kernels.

There is no fallback: if ``libebc.so`` is missing or cannot be loaded, every
call raises.  Build it with ``python -m paper_2105_12912_amd.build``.
"""
from __future__ import annotations

import ctypes as C
import threading
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebc.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "ebc.h")

EBC_OK = 0
EBC_ERR_ARG, EBC_ERR_DIMS, EBC_ERR_EB, EBC_ERR_EB_TOO_SMALL = -1, -2, -3, -4
EBC_ERR_BINS, EBC_ERR_NONFINITE, EBC_ERR_OUT_TOO_SMALL, EBC_ERR_WS_TOO_SMALL = -5, -6, -7, -8
EBC_ERR_ARCHIVE, EBC_ERR_HIP, EBC_ERR_UNSUPPORTED = -9, -10, -11
EBC_EB_ABS, EBC_EB_REL = 0, 1
EBC_CODEC_AUTO, EBC_CODEC_HUFFMAN, EBC_CODEC_RLE, EBC_CODEC_RLE_VLE, EBC_CODEC_AUTO_VLE = 0, 1, 2, 3, 4
EBC_ARC_HUFFMAN, EBC_ARC_RLE, EBC_ARC_CONST, EBC_ARC_RLE_VLE = 0, 1, 2, 3
CODECS = {"auto": EBC_CODEC_AUTO, "huffman": EBC_CODEC_HUFFMAN, "rle": EBC_CODEC_RLE,
          "rle_vle": EBC_CODEC_RLE_VLE, "auto_vle": EBC_CODEC_AUTO_VLE}
EBC_STATS_TIMING = 1
EBC_MAX_STAGES = 16
HDR_BYTES = 128
EBC_NOALLOC_SCRATCH_BYTES = 64 << 20  # fixed device scratch of ebc_compress_async_noalloc


EBC_F32, EBC_F64 = 0, 1


class ebc_params(C.Structure):
    _fields_ = [("eb_mode", C.c_int32), ("codec", C.c_int32), ("eb", C.c_double),
                ("n_bins", C.c_uint32), ("huff_chunk", C.c_uint32), ("dtype", C.c_int32),
                ("reserved", C.c_int32)]


class ebc_stats(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("codec", C.c_int32), ("n_elems", C.c_uint64),
                ("n_outliers", C.c_uint64), ("n_runs", C.c_uint64), ("n_words", C.c_uint64),
                ("huff_bits", C.c_uint64), ("out_bytes", C.c_uint64), ("eb_abs", C.c_double),
                ("ebx2", C.c_double), ("value_min", C.c_float), ("value_max", C.c_float),
                ("n_stages", C.c_uint32), ("stage_ms", C.c_float * EBC_MAX_STAGES),
                ("stage_name", C.c_char_p * EBC_MAX_STAGES), ("time_only", C.c_char_p),
                ("entropy", C.c_double), ("p1", C.c_double), ("r_lo", C.c_double),
                ("r_hi", C.c_double), ("predict", C.c_int32), ("pad", C.c_int32)]

    def stages(self) -> dict:
        return {self.stage_name[k].decode(): float(self.stage_ms[k]) for k in range(self.n_stages)}


EBC_MADO_DMAX = 200


class ebc_estimates(C.Structure):
    _fields_ = [("codec_hint", C.c_int32), ("pad", C.c_int32), ("entropy", C.c_double),
                ("p1", C.c_double), ("r_lo", C.c_double), ("r_hi", C.c_double),
                ("bits_lo", C.c_double), ("bits_hi", C.c_double), ("hist_max", C.c_uint64),
                ("n_elems", C.c_uint64), ("samples", C.c_uint64), ("roughness", C.c_double),
                ("mado_sum", C.c_uint64 * (EBC_MADO_DMAX + 1)),
                ("mado_cnt", C.c_uint64 * (EBC_MADO_DMAX + 1))]


class ebc_field(C.Structure):
    _fields_ = [("d_field", C.c_void_p), ("rank", C.c_int32), ("reserved", C.c_uint32),
                ("dims", C.c_uint64 * 3), ("d_out", C.c_void_p), ("out_cap", C.c_uint64)]


class ebc_result(C.Structure):
    _fields_ = [("out_size", C.c_uint64), ("status", C.c_int32), ("codec", C.c_int32)]


class ebc_archive_ref(C.Structure):
    _fields_ = [("d_archive", C.c_void_p), ("size", C.c_uint64), ("h_header", C.c_void_p),
                ("d_out", C.c_void_p), ("out_elems", C.c_uint64)]


class ebc_tuning_entry(C.Structure):
    _fields_ = [("rank", C.c_int32), ("nx_class", C.c_uint32), ("n_class", C.c_uint32),
                ("tile_wx", C.c_uint32), ("grid", C.c_uint32), ("scan_direct", C.c_uint32)]


class EbcError(RuntimeError):
    def __init__(self, status: int, call: str):
        detail = ""
        try:
            detail = lib().ebc_last_error().decode()
        except Exception:  # pragma: no cover
            pass
        super().__init__(f"{call}: status {status} ({status_string(status)}) {detail}")
        self.status = status


_P, _U64, _I32, _U32, _F64 = C.c_void_p, C.c_uint64, C.c_int, C.c_uint32, C.c_double
_SIGS = {
    "ebc_version": (_I32, []),
    "ebc_status_string": (C.c_char_p, [_I32]),
    "ebc_last_error": (C.c_char_p, []),
    "ebc_compress_bound": (_I32, [_I32, _P, _P, _P]),
    "ebc_compress_workspace_size": (_I32, [_I32, _P, _P, _P]),
    "ebc_compress": (_I32, [_P, _I32, _P, _P, _P, _U64, _P, _P, _U64, _P, _P]),
    "ebc_compress_async": (_I32, [_P, _I32, _P, _P, _P, _U64, _P, _P, _U64, _P]),
    "ebc_compress_async_noalloc": (_I32, [_P, _I32, _P, _P, _P, _U64, _P, _P]),
    "ebc_archive_info": (_I32, [_P, _U64, _P, _P, _P, _P, _P]),
    "ebc_decompress_workspace_size": (_I32, [_P, _U64, _P]),
    "ebc_decompress": (_I32, [_P, _U64, _P, _U64, _P, _U64, _P, _P]),
    "ebc_decompress_async": (_I32, [_P, _P, _U64, _P, _U64, _P, _U64, _P, _P]),
    "ebc_batch_compress_workspace_size": (_I32, [_I32, _P, _P, _P]),
    "ebc_batch_compress": (_I32, [_I32, _P, _P, _P, _P, _U64, _P]),
    "ebc_batch_decompress_workspace_size": (_I32, [_I32, _P, _P]),
    "ebc_batch_decompress": (_I32, [_I32, _P, _P, _P, _U64, _P]),
    "ebc_batch_compress_async": (_I32, [_I32, _P, _P, _P, _P, _U64, _P]),
    "ebc_set_tuning": (_I32, [_P, _I32]),
    "ebc_shape_class": (_I32, [_I32, _P, _P, _P]),
    "ebc_batch_decompress_async": (_I32, [_I32, _P, _P, _P, _U64, _P]),
    "ebc_debug_construct": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _U64, _P]),
    "ebc_estimate": (_I32, [_P, _I32, _P, _P, _U64, _U64, _P, _P, _U64, _P]),
    "ebc_debug_reconstruct": (_I32, [_P, _P, _P, _U64, _I32, _P, _U32, _F64, _P, _P, _U64, _P]),
}

_lib = None


def lib():
    """Load libebc.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run python -m paper_2105_12912_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols(path: str = HEADER_PATH) -> list[str]:
    """Names of every function declared in include/ebc.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebc_\w+)\s*\(", text)))


def status_string(status: int) -> str:
    return lib().ebc_status_string(int(status)).decode()


def _dims3(dims) -> C.Array:
    d = [1, 1, 1]
    for i, v in enumerate(dims):
        d[i] = int(v)
    return (C.c_uint64 * 3)(*d)


# --------------------------------------------------------------- raw entry points
# Same names and argument order as the C ABI; pointers are ints (or None).

def ebc_version() -> int:
    return lib().ebc_version()


def ebc_status_string(status: int) -> str:
    return status_string(status)


def ebc_last_error() -> str:
    return lib().ebc_last_error().decode()


def ebc_compress_bound(rank, dims, params) -> int:
    out = C.c_uint64()
    st = lib().ebc_compress_bound(rank, _dims3(dims), C.byref(params), C.byref(out))
    _check(st, "ebc_compress_bound")
    return out.value


def ebc_compress_workspace_size(rank, dims, params) -> int:
    out = C.c_uint64()
    st = lib().ebc_compress_workspace_size(rank, _dims3(dims), C.byref(params), C.byref(out))
    _check(st, "ebc_compress_workspace_size")
    return out.value


def ebc_compress(d_field, rank, dims, params, d_out, out_cap, d_ws, ws_bytes, stream,
                 stats: ebc_stats | None = None) -> tuple[int, int]:
    """Returns (status, out_size)."""
    size = C.c_uint64()
    st = lib().ebc_compress(d_field, rank, _dims3(dims), C.byref(params), d_out, out_cap,
                            C.byref(size), d_ws, ws_bytes, stream,
                            C.byref(stats) if stats is not None else None)
    return st, size.value


def ebc_compress_async(d_field, rank, dims, params, d_out, out_cap, d_result, d_ws, ws_bytes,
                       stream) -> int:
    return lib().ebc_compress_async(d_field, rank, _dims3(dims), C.byref(params), d_out, out_cap,
                                    d_result, d_ws, ws_bytes, stream)


def ebc_compress_async_noalloc(d_field, rank, dims, params, d_out, out_cap, d_result,
                               stream) -> int:
    return lib().ebc_compress_async_noalloc(d_field, rank, _dims3(dims), C.byref(params), d_out,
                                            out_cap, d_result, stream)


def ebc_archive_info(header: bytes) -> dict:
    rank, codec = C.c_int(), C.c_int()
    dims = (C.c_uint64 * 3)()
    p = ebc_params()
    total = C.c_uint64()
    buf = C.create_string_buffer(bytes(header), len(header))
    st = lib().ebc_archive_info(buf, len(header), C.byref(rank), dims, C.byref(p), C.byref(codec),
                                C.byref(total))
    _check(st, "ebc_archive_info")
    return dict(rank=rank.value, dims=tuple(dims), codec=codec.value, n_bins=p.n_bins,
                huff_chunk=p.huff_chunk, eb=p.eb, eb_mode=p.eb_mode, total=total.value,
                dtype=p.dtype)


def ebc_decompress_workspace_size(header: bytes) -> int:
    out = C.c_uint64()
    buf = C.create_string_buffer(bytes(header), len(header))
    _check(lib().ebc_decompress_workspace_size(buf, len(header), C.byref(out)),
           "ebc_decompress_workspace_size")
    return out.value


def ebc_decompress(d_archive, size, d_out, out_elems, d_ws, ws_bytes, stream,
                   stats: ebc_stats | None = None) -> int:
    return lib().ebc_decompress(d_archive, size, d_out, out_elems, d_ws, ws_bytes, stream,
                                C.byref(stats) if stats is not None else None)


def ebc_decompress_async(header: bytes, d_archive, size, d_out, out_elems, d_ws, ws_bytes,
                         d_status, stream) -> int:
    buf = C.create_string_buffer(bytes(header), len(header))
    return lib().ebc_decompress_async(buf, d_archive, size, d_out, out_elems, d_ws, ws_bytes,
                                      d_status, stream)


def ebc_batch_compress_workspace_size(fields, params) -> int:
    arr = (ebc_field * len(fields))(*fields)
    out = C.c_uint64()
    _check(lib().ebc_batch_compress_workspace_size(len(fields), arr, C.byref(params),
                                                   C.byref(out)), "ebc_batch_compress_workspace_size")
    return out.value


def ebc_batch_compress(fields, params, d_ws, ws_bytes, stream):
    """Returns (status, [ebc_result])."""
    arr = (ebc_field * len(fields))(*fields)
    res = (ebc_result * len(fields))()
    st = lib().ebc_batch_compress(len(fields), arr, C.byref(params), res, d_ws, ws_bytes, stream)
    return st, list(res)


def ebc_batch_decompress_workspace_size(refs) -> int:
    arr = (ebc_archive_ref * len(refs))(*refs)
    out = C.c_uint64()
    _check(lib().ebc_batch_decompress_workspace_size(len(refs), arr, C.byref(out)),
           "ebc_batch_decompress_workspace_size")
    return out.value


def ebc_batch_decompress(refs, d_ws, ws_bytes, stream):
    arr = (ebc_archive_ref * len(refs))(*refs)
    sts = (C.c_int32 * len(refs))()
    st = lib().ebc_batch_decompress(len(refs), arr, sts, d_ws, ws_bytes, stream)
    return st, list(sts)


def ebc_batch_compress_async(fields, params, d_results, d_ws, ws_bytes, stream) -> int:
    arr = (ebc_field * len(fields))(*fields)
    return lib().ebc_batch_compress_async(len(fields), arr, C.byref(params), d_results, d_ws,
                                          ws_bytes, stream)


def ebc_batch_decompress_async(refs, d_statuses, d_ws, ws_bytes, stream) -> int:
    arr = (ebc_archive_ref * len(refs))(*refs)
    return lib().ebc_batch_decompress_async(len(refs), arr, d_statuses, d_ws, ws_bytes, stream)


def ebc_set_tuning(entries) -> int:
    """entries: iterable of dicts with rank, nx_class, n_class, tile_wx, grid
    and optionally scan_direct."""
    entries = list(entries)
    arr = (ebc_tuning_entry * max(len(entries), 1))(
        *[ebc_tuning_entry(**{k: int(e.get(k, 0)) for k in ("rank", "nx_class", "n_class",
                                                             "tile_wx", "grid", "scan_direct")})
          for e in entries])
    return lib().ebc_set_tuning(arr if entries else None, len(entries))


def ebc_shape_class(rank, dims):
    """(nx_class, n_class) of a field."""
    a, b = C.c_uint32(), C.c_uint32()
    _check(lib().ebc_shape_class(rank, _dims3(dims), C.byref(a), C.byref(b)), "ebc_shape_class")
    return a.value, b.value


def ebc_estimate(d_field, rank, dims, params, samples, seed, d_ws, ws_bytes, stream):
    """Returns (status, ebc_estimates)."""
    out = ebc_estimates()
    st = lib().ebc_estimate(d_field, rank, _dims3(dims), C.byref(params), int(samples), int(seed),
                            C.byref(out), d_ws, ws_bytes, stream)
    return st, out


def ebc_debug_construct(d_field, rank, dims, params, d_q, d_hist, d_oidx, d_oval, d_ws, ws_bytes,
                        stream):
    """Returns (status, n_outliers, ebx2)."""
    n = C.c_uint64()
    ebx2 = C.c_double()
    st = lib().ebc_debug_construct(d_field, rank, _dims3(dims), C.byref(params), d_q, d_hist,
                                   d_oidx, d_oval, C.byref(n), C.byref(ebx2), d_ws, ws_bytes,
                                   stream)
    return st, n.value, ebx2.value


def ebc_debug_reconstruct(d_q, d_oidx, d_oval, n_outliers, rank, dims, n_bins, ebx2, d_out, d_ws,
                          ws_bytes, stream) -> int:
    return lib().ebc_debug_reconstruct(d_q, d_oidx, d_oval, n_outliers, rank, _dims3(dims), n_bins,
                                       float(ebx2), d_out, d_ws, ws_bytes, stream)


def _check(st: int, call: str):
    if st != EBC_OK:
        raise EbcError(st, call)


# --------------------------------------------------------------- torch conveniences

def make_params(eb: float, mode: str = "rel", n_bins: int = 1024, codec: str = "auto",
                huff_chunk: int = 1024, dtype: int = EBC_F32) -> ebc_params:
    return ebc_params(eb_mode=EBC_EB_REL if mode == "rel" else EBC_EB_ABS,
                      codec=CODECS[codec],
                      eb=float(eb), n_bins=int(n_bins), huff_chunk=int(huff_chunk),
                      dtype=int(dtype), reserved=0)


def _dtype_code(x) -> int:
    torch = _torch()
    if x.dtype == torch.float32:
        return EBC_F32
    if x.dtype == torch.float64:
        return EBC_F64
    raise ValueError("fields are float32 or float64 tensors")


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Workspace:
    """Grow-only device scratch buffer (allocated by torch, never by the library)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf.data_ptr(), self.buf.numel()


_default_ws = {}


def default_workspace(device="cuda") -> Workspace:
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def field_rank_dims(x, rank: int | None = None):
    rank = rank or x.dim()
    dims = tuple(int(s) for s in reversed(x.shape))
    if len(dims) > 3:
        raise ValueError("rank > 3")
    return rank, dims


def compress(x, eb: float, mode: str = "rel", n_bins: int = 1024, codec: str = "auto",
             huff_chunk: int = 1024, stream=None, stats: bool | str = False, workspace=None,
             out=None):
    """Compress a contiguous fp32 CUDA tensor; returns a uint8 CUDA tensor (and stats)."""
    torch = _torch()
    if x.dtype not in (torch.float32, torch.float64) or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 or float64 CUDA tensor")
    rank, dims = field_rank_dims(x)
    p = make_params(eb, mode, n_bins, codec, huff_chunk, _dtype_code(x))
    bound = ebc_compress_bound(rank, dims, p)
    wsz = ebc_compress_workspace_size(rank, dims, p)
    ws = workspace or default_workspace(x.device)
    wptr, wlen = ws.get(wsz)
    if out is None or out.numel() < bound:
        out = torch.empty(bound, dtype=torch.uint8, device=x.device)
    st_obj = _stats_obj(stats)
    st, size = ebc_compress(x.data_ptr(), rank, dims, p, out.data_ptr(), out.numel(), wptr, wlen,
                            _stream_handle(stream), st_obj)
    _check(st, "ebc_compress")
    a = out[:size]
    return (a, st_obj) if stats else a


def _stats_obj(stats):
    """stats: False (none), True (time every stage) or a stage name (time only it)."""
    if not stats:
        return None
    st = ebc_stats(flags=EBC_STATS_TIMING)
    if isinstance(stats, str):
        st._only = stats.encode()  # keeps the string alive for the call
        st.time_only = st._only
    return st


_hdr_stage = threading.local()


def archive_header(a) -> bytes:
    """The archive's 128-byte header, read through a page-locked buffer (a
    direct copy on the current stream) when the archive is on the GPU."""
    torch = _torch()
    if not a.is_cuda:
        return bytes(a[:HDR_BYTES].numpy().tobytes())
    bufs = _hdr_stage.__dict__.setdefault("bufs", {})
    buf = bufs.get(a.device)
    if buf is None:
        buf = bufs[a.device] = torch.empty(HDR_BYTES, dtype=torch.uint8, pin_memory=True)
    n = min(HDR_BYTES, a.numel())
    buf[:n].copy_(a[:n], non_blocking=True)
    torch.cuda.current_stream(a.device).synchronize()
    return bytes(buf[:n].numpy().tobytes())


def decompress(a, out=None, stream=None, stats: bool | str = False, workspace=None):
    """Decompress a uint8 CUDA archive tensor into a float32 CUDA tensor."""
    torch = _torch()
    hdr = archive_header(a)
    info = ebc_archive_info(hdr)
    nx, ny, nz = info["dims"]
    shape = {1: (nx,), 2: (ny, nx), 3: (nz, ny, nx)}[info["rank"]]
    dt = torch.float64 if info["dtype"] == EBC_F64 else torch.float32
    if out is None:
        out = torch.empty(shape, dtype=dt, device=a.device)
    elif out.dtype != dt:
        raise ValueError(f"output must be {dt} for this archive")
    wsz = ebc_decompress_workspace_size(hdr)
    ws = workspace or default_workspace(a.device)
    wptr, wlen = ws.get(wsz)
    st_obj = _stats_obj(stats)
    st = ebc_decompress(a.data_ptr(), a.numel(), out.data_ptr(), out.numel(), wptr, wlen,
                        _stream_handle(stream), st_obj)
    _check(st, "ebc_decompress")
    return (out, st_obj) if stats else out


def decompress_status(a, workspace=None) -> int:
    """Status code of a decompression attempt (for error-path tests)."""
    torch = _torch()
    n = a.numel()
    hdr = archive_header(a) if n >= HDR_BYTES else bytes(n)
    try:
        info = ebc_archive_info(hdr)
        cnt = info["dims"][0] * info["dims"][1] * info["dims"][2]
        wsz = ebc_decompress_workspace_size(hdr)
    except EbcError as e:
        return e.status
    out = torch.empty(max(cnt, 1), dtype=torch.float64, device=a.device)  # room for either type
    ws = workspace or default_workspace(a.device)
    wptr, wlen = ws.get(wsz)
    return ebc_decompress(a.data_ptr(), n, out.data_ptr(), out.numel(), wptr, wlen,
                          _stream_handle(None), None)


def debug_construct(x, eb: float, mode: str = "rel", n_bins: int = 1024, workspace=None):
    """Quant-codes, histogram and ordered outliers from the construct stage."""
    torch = _torch()
    rank, dims = field_rank_dims(x)
    p = make_params(eb, mode, n_bins, dtype=_dtype_code(x))
    n = x.numel()
    q = torch.empty(n, dtype=torch.int16, device=x.device)
    hist = torch.empty(n_bins, dtype=torch.int32, device=x.device)
    oidx = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    oval = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    wsz = ebc_compress_workspace_size(rank, dims, p)
    ws = workspace or default_workspace(x.device)
    wptr, wlen = ws.get(wsz)
    st, no, ebx2 = ebc_debug_construct(x.data_ptr(), rank, dims, p, q.data_ptr(), hist.data_ptr(),
                                       oidx.data_ptr(), oval.data_ptr(), wptr, wlen,
                                       _stream_handle(None))
    _check(st, "ebc_debug_construct")
    return dict(q=q, hist=hist, oidx=oidx[:no], oval=oval[:no], ebx2=ebx2)


def estimate(x, eb: float, mode: str = "rel", n_bins: int = 1024, samples: int = 1 << 20,
             seed: int = 0, workspace=None) -> dict:
    """Compressibility estimates of a field (histogram bounds and madogram)."""
    rank, dims = field_rank_dims(x)
    p = make_params(eb, mode, n_bins, dtype=_dtype_code(x))
    wsz = ebc_compress_workspace_size(rank, dims, p)
    ws = workspace or default_workspace(x.device)
    wptr, wlen = ws.get(wsz)
    st, e = ebc_estimate(x.data_ptr(), rank, dims, p, samples, seed, wptr, wlen,
                         _stream_handle(None))
    _check(st, "ebc_estimate")
    out = {k: getattr(e, k) for k, _ in ebc_estimates._fields_ if k not in ("pad", "mado_sum",
                                                                            "mado_cnt")}
    import numpy as np
    out["mado_sum"] = np.array(e.mado_sum[:], dtype=np.uint64)
    out["mado_cnt"] = np.array(e.mado_cnt[:], dtype=np.uint64)
    return out


def debug_reconstruct(q, oidx, oval, rank: int, dims, n_bins: int, ebx2: float, workspace=None):
    torch = _torch()
    n = q.numel()
    out = torch.empty(n, dtype=torch.float32, device=q.device)
    hdr = bytearray(HDR_BYTES)
    ws = workspace or default_workspace(q.device)
    # generous scratch: codes, delta scratch, per-tile counts
    wptr, wlen = ws.get(8 * n + (1 << 22))
    no = oidx.numel()
    st = ebc_debug_reconstruct(q.data_ptr(), oidx.data_ptr() if no else None,
                               oval.data_ptr() if no else None, no, rank, dims, n_bins, ebx2,
                               out.data_ptr(), wptr, wlen, _stream_handle(None))
    _check(st, "ebc_debug_reconstruct")
    return out
