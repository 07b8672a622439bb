"""Batched compression and decompression of many fields through the C ABI.

A batch of fields of mixed rank and size goes through one sequence of kernel
launches: every kernel's grid covers the work units of all fields, found by a
binary search over per-field bases, so small fields fill the GPU together and
per-field launch and synchronisation costs disappear.  The async entry points
(``ebc_batch_compress_async`` / ``ebc_batch_decompress_async``) enqueue kernel
launches only, so a whole batch can be captured once into a HIP graph
(``torch.cuda.CUDAGraph``) and replayed.

torch supplies the device buffers and the stream; all work runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C

from . import ebc


def _torch():
    import torch
    return torch


class BatchCompress:
    """Compress a fixed list of contiguous CUDA tensors (all fp32, or all fp64)
    with one parameter set.

    Output buffers (one per field, sized by the compress bound), the result
    records and the workspace are allocated once, here; ``launch`` enqueues
    the whole batch asynchronously, ``capture`` records it into a graph.
    """

    def __init__(self, fields, eb: float, mode: str = "rel", n_bins: int = 1024,
                 codec: str = "auto", huff_chunk: int = 1024):
        torch = _torch()
        if not fields:
            raise ValueError("empty batch")
        self.fields = list(fields)
        self.device = self.fields[0].device
        dt = self.fields[0].dtype
        self.params = ebc.make_params(eb, mode, n_bins, codec, huff_chunk, ebc._dtype_code(self.fields[0]))
        self.outs = []
        descs = []
        for x in self.fields:
            if x.dtype != dt or not x.is_cuda or not x.is_contiguous():
                raise ValueError("fields must be contiguous CUDA tensors of one float type")
            rank, dims = ebc.field_rank_dims(x)
            bound = ebc.ebc_compress_bound(rank, dims, self.params)
            out = torch.empty(bound, dtype=torch.uint8, device=self.device)
            self.outs.append(out)
            d3 = (C.c_uint64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
            descs.append(ebc.ebc_field(d_field=x.data_ptr(), rank=rank, reserved=0, dims=d3,
                                       d_out=out.data_ptr(), out_cap=bound))
        self.descs = descs
        self.ws_bytes = ebc.ebc_batch_compress_workspace_size(descs, self.params)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        # 16-byte records {out_size u64, status i32, codec i32}
        self.res = torch.zeros((len(descs), 2), dtype=torch.int64, device=self.device)
        self.graph = None

    @property
    def input_bytes(self) -> int:
        return sum(x.numel() * x.element_size() for x in self.fields)

    def launch(self, stream=None):
        st = ebc.ebc_batch_compress_async(self.descs, self.params, self.res.data_ptr(),
                                          self.ws.data_ptr(), self.ws.numel(),
                                          ebc._stream_handle(stream))
        ebc._check(st, "ebc_batch_compress_async")

    def capture(self):
        """Record the batch into a graph (after one eager warm-up launch)."""
        torch = _torch()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.launch(side)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.launch(side)
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self):
        """[(out_size, status, codec)] in field order (synchronises)."""
        r = self.res.cpu().tolist()
        out = []
        for size, word in r:
            word &= (1 << 64) - 1
            status = word & 0xFFFFFFFF
            status = status - (1 << 32) if status >= 1 << 31 else status
            out.append((int(size), int(status), int(word >> 32)))
        return out

    def archives(self):
        """Archive tensors (views of the output buffers); raises on any field error."""
        arcs = []
        for i, (size, status, _codec) in enumerate(self.results()):
            if status != ebc.EBC_OK:
                raise ebc.EbcError(status, f"batch field {i}")
            arcs.append(self.outs[i][:size])
        return arcs


class BatchDecompress:
    """Decompress a fixed list of archives (uint8 CUDA tensors) into tensors of
    each archive's element type (fp32 or fp64)."""

    def __init__(self, archives, outs=None):
        torch = _torch()
        if not archives:
            raise ValueError("empty batch")
        self.archives = list(archives)
        self.device = self.archives[0].device
        self.headers = [ebc.archive_header(a) for a in self.archives]
        self._hbufs = [C.create_string_buffer(h, len(h)) for h in self.headers]
        self.outs = []
        refs = []
        for i, a in enumerate(self.archives):
            info = ebc.ebc_archive_info(self.headers[i])
            nx, ny, nz = info["dims"]
            shape = {1: (nx,), 2: (ny, nx), 3: (nz, ny, nx)}[info["rank"]]
            dt = torch.float64 if info["dtype"] == ebc.EBC_F64 else torch.float32
            out = outs[i] if outs is not None else torch.empty(shape, dtype=dt, device=self.device)
            self.outs.append(out)
            refs.append(ebc.ebc_archive_ref(d_archive=a.data_ptr(), size=a.numel(),
                                            h_header=C.cast(self._hbufs[i], C.c_void_p),
                                            d_out=out.data_ptr(), out_elems=out.numel()))
        self.refs = refs
        self.ws_bytes = ebc.ebc_batch_decompress_workspace_size(refs)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.status = torch.zeros(len(refs), dtype=torch.int32, device=self.device)
        self.graph = None

    @property
    def output_bytes(self) -> int:
        return sum(o.numel() * o.element_size() for o in self.outs)

    def launch(self, stream=None):
        st = ebc.ebc_batch_decompress_async(self.refs, self.status.data_ptr(), self.ws.data_ptr(),
                                            self.ws.numel(), ebc._stream_handle(stream))
        ebc._check(st, "ebc_batch_decompress_async")

    def capture(self):
        torch = _torch()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.launch(side)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.launch(side)
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def statuses(self):
        return [int(s) for s in self.status.cpu().tolist()]
