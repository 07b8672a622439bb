"""Continuous-batching request loop for compress / decompress jobs on one GPU.

Requests arrive at any time.  A fixed number of execution slots, each with
its own HIP stream and workspace, run batches concurrently on the device.
Whenever a slot is free, the scheduler forms a batch from the pending
requests, oldest first: requests of the same kind (compress with the same
bound, or decompress) whose device memory (output buffer plus their share of
the slot's workspace) fits in what the HBM budget has left.  A request that
does not fit waits until running batches complete and release memory (the
budget counts each running batch's output buffers and every workspace a slot
holds, running or idle; idle slots give their workspaces back when the
oldest request would not fit otherwise); it is never overtaken by a later
request of its own kind, and a request larger than the whole budget is
rejected.  Batches go through the library's async
batched entry points, so each batch is one sequence of kernel launches on
its slot's stream and batches on different slots overlap on the device.

Stream order: a request's work starts only after everything the submitting
stream had enqueued when it was submitted (so an input written
asynchronously just before submit() is complete), and its input and output
tensors are marked as used by the slot stream and the submitting stream, so
the caching allocator never hands their memory out early.  A result is valid
once the request is returned by poll() (its batch's completion event has
been observed).

Latency is measured from a request's arrival time to the moment the loop
observes its batch's completion event.  The result of each request is the
same as when it runs alone: batching changes launch geometry, never bytes.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

from . import ebc


def _torch():
    import torch
    return torch


@dataclass(eq=False)
class Request:
    op: str                      # "compress" | "decompress"
    t_arrival: float             # seconds, server clock
    x: object = None             # compress: contiguous fp32 CUDA tensor
    eb: float = 1e-4             # compress: relative bound
    archive: object = None       # decompress: uint8 CUDA tensor
    header: bytes = b""          # decompress: first 128 bytes (host)
    rid: int = 0
    # filled by the server
    out: object = None           # compress: archive view; decompress: fp32 tensor
    status: int = 0
    codec: int = -1
    t_done: float = 0.0
    batch_size: int = 0
    footprint: int = 0           # output buffer + workspace when run alone
    out_bytes: int = 0           # output buffer
    nbytes: int = 0              # fp32 bytes of the field (input or output)
    stream: object = None        # submitting stream (consumer of the output)
    ready: object = None         # event on `stream` at submission

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass(eq=False)
class _Slot:
    stream: object
    ws: object = None            # uint8 tensor, grow-only
    busy: bool = False
    event: object = None
    reqs: list = field(default_factory=list)
    res: object = None           # device results (compress) / statuses (decompress)
    descs: object = None         # keeps ctypes arrays alive until completion
    reserved: int = 0            # output bytes of the running batch


class Server:
    """Continuous-batching compressor service on one device."""

    def __init__(self, device="cuda", hbm_budget: int = 64 << 30, slots: int = 4,
                 max_batch: int = 32, n_bins: int = 1024, huff_chunk: int = 1024):
        torch = _torch()
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.n_bins, self.huff_chunk = n_bins, huff_chunk
        self.slots = [_Slot(stream=torch.cuda.Stream(device=self.device)) for _ in range(slots)]
        self.pending: list[Request] = []
        self.in_use = 0               # outputs of running batches + every slot's workspace
        self.peak_in_use = 0
        self.batches = 0
        self.mem_waits = 0            # scheduling rounds in which the oldest request had to wait
        self.ws_released = 0          # idle workspaces given back to the budget
        self._next_id = 0
        self.t0 = time.perf_counter()

    # ------------------------------------------------------------ clock
    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ intake
    def submit(self, req: Request) -> Request:
        req.rid = self._next_id
        self._next_id += 1
        if req.op == "compress":
            x = req.x
            if not (x.is_cuda and x.is_contiguous()):
                raise ValueError("compress input must be a contiguous CUDA tensor")
            rank, dims = ebc.field_rank_dims(x)
            p = self._params(req.eb)
            req.out_bytes = ebc.ebc_compress_bound(rank, dims, p)
            req.footprint = req.out_bytes + ebc.ebc_compress_workspace_size(rank, dims, p)
            req.nbytes = 4 * x.numel()
        elif req.op == "decompress":
            if len(req.header) < ebc.HDR_BYTES:
                req.header = ebc.archive_header(req.archive)
            info = ebc.ebc_archive_info(req.header)
            nx, ny, nz = info["dims"]
            req.out_bytes = 4 * nx * ny * nz
            req.footprint = req.out_bytes + ebc.ebc_decompress_workspace_size(req.header)
            req.nbytes = 4 * nx * ny * nz
        else:
            raise ValueError(req.op)
        if req.footprint > self.budget:
            req.status = ebc.EBC_ERR_OUT_TOO_SMALL
            req.t_done = self.now()
            return req
        torch = _torch()
        req.stream = torch.cuda.current_stream(self.device)
        req.ready = torch.cuda.Event()
        req.ready.record(req.stream)
        self.pending.append(req)
        return req

    def _params(self, eb):
        return ebc.make_params(eb, "rel", self.n_bins, "auto", self.huff_chunk)

    # ------------------------------------------------------------ scheduling
    def _ws_bytes(self, reqs) -> int:
        """Exact workspace of a batch (host-side sizing, no device work)."""
        if reqs[0].op == "compress":
            descs = []
            for r in reqs:
                rank, dims = ebc.field_rank_dims(r.x)
                d3 = (C.c_uint64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
                descs.append(ebc.ebc_field(d_field=None, rank=rank, reserved=0, dims=d3,
                                           d_out=None, out_cap=0))
            return ebc.ebc_batch_compress_workspace_size(descs, self._params(reqs[0].eb))
        hbufs, refs = [], []
        for r in reqs:
            hb = C.create_string_buffer(bytes(r.header[:ebc.HDR_BYTES]), ebc.HDR_BYTES)
            hbufs.append(hb)
            refs.append(ebc.ebc_archive_ref(d_archive=None, size=0, h_header=C.cast(hb, C.c_void_p),
                                            d_out=None, out_elems=0))
        return ebc.ebc_batch_decompress_workspace_size(refs)

    def _need(self, slot, reqs) -> int:
        """Budget a batch needs on `slot`: its outputs plus the growth of the
        slot's workspace (a workspace already held is counted already)."""
        held = slot.ws.numel() if slot.ws is not None else 0
        return sum(r.out_bytes for r in reqs) + max(0, self._ws_bytes(reqs) - held)

    def _pick(self, slot):
        """Oldest-first batch of one kind that fits the remaining budget."""
        if not self.pending:
            return []
        head = self.pending[0]
        key = (head.op, head.eb if head.op == "compress" else None)
        held = slot.ws.numel() if slot.ws is not None else 0
        free = self.budget - self.in_use
        picked, est = [], 0
        for r in self.pending:
            if (r.op, r.eb if r.op == "compress" else None) != key:
                continue
            # solo footprints bound the batch's needs from above (roughly)
            if picked and est + r.footprint - held > free:
                break  # never overtake an older request of this kind
            picked.append(r)
            est += r.footprint
            if len(picked) == self.max_batch:
                break
        while picked and self._need(slot, picked) > free:
            picked.pop()
        if not picked:
            # the oldest request does not fit: idle slots return their cached
            # workspaces to the budget, and the request waits if still too big
            for s in self.slots:
                if not s.busy and s.ws is not None and s is not slot:
                    self.in_use -= s.ws.numel()
                    s.ws = None
                    self.ws_released += 1
            if self._need(slot, [head]) <= self.budget - self.in_use:
                picked = [head]
            else:
                self.mem_waits += 1
        return picked

    def _launch(self, slot, reqs):
        torch = _torch()
        n = len(reqs)
        for r in reqs:
            # the submitting stream's work up to submit() comes first, and the
            # input's memory stays reserved until the slot stream is done with it
            slot.stream.wait_event(r.ready)
            (r.x if r.op == "compress" else r.archive).record_stream(slot.stream)
        with torch.cuda.stream(slot.stream):
            if reqs[0].op == "compress":
                p = self._params(reqs[0].eb)
                descs, outs = [], []
                for r in reqs:
                    rank, dims = ebc.field_rank_dims(r.x)
                    bound = ebc.ebc_compress_bound(rank, dims, p)
                    o = torch.empty(bound, dtype=torch.uint8, device=self.device)
                    outs.append(o)
                    d3 = (C.c_uint64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
                    descs.append(ebc.ebc_field(d_field=r.x.data_ptr(), rank=rank, reserved=0,
                                               dims=d3, d_out=o.data_ptr(), out_cap=bound))
                wsz = ebc.ebc_batch_compress_workspace_size(descs, p)
                self._grow_ws(slot, wsz)
                slot.res = torch.empty((n, 2), dtype=torch.int64, device=self.device)
                st = ebc.ebc_batch_compress_async(descs, p, slot.res.data_ptr(), slot.ws.data_ptr(),
                                                  slot.ws.numel(), int(slot.stream.cuda_stream))
                for r, o in zip(reqs, outs):
                    r.out = o
                reserved = sum(o.numel() for o in outs)
            else:
                hbufs, refs, outs = [], [], []
                for r in reqs:
                    info = ebc.ebc_archive_info(r.header)
                    nx, ny, nz = info["dims"]
                    shape = {1: (nx,), 2: (ny, nx), 3: (nz, ny, nx)}[info["rank"]]
                    o = torch.empty(shape, dtype=torch.float32, device=self.device)
                    outs.append(o)
                    hb = C.create_string_buffer(bytes(r.header[:ebc.HDR_BYTES]), ebc.HDR_BYTES)
                    hbufs.append(hb)
                    refs.append(ebc.ebc_archive_ref(d_archive=r.archive.data_ptr(),
                                                    size=r.archive.numel(),
                                                    h_header=C.cast(hb, C.c_void_p),
                                                    d_out=o.data_ptr(), out_elems=o.numel()))
                wsz = ebc.ebc_batch_decompress_workspace_size(refs)
                self._grow_ws(slot, wsz)
                slot.res = torch.empty(n, dtype=torch.int32, device=self.device)
                st = ebc.ebc_batch_decompress_async(refs, slot.res.data_ptr(), slot.ws.data_ptr(),
                                                    slot.ws.numel(), int(slot.stream.cuda_stream))
                descs = (hbufs, refs)
                for r, o in zip(reqs, outs):
                    r.out = o
                reserved = sum(4 * o.numel() for o in outs)
            ebc._check(st, "batched " + reqs[0].op)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.busy, slot.event, slot.reqs, slot.descs = True, ev, reqs, descs
        slot.reserved = reserved
        self.in_use += reserved
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.batches += 1
        for r in reqs:
            r.batch_size = n

    def _grow_ws(self, slot, nbytes):
        """Grow the slot's workspace (allocated on the slot stream); the
        budget counts a workspace for as long as the slot holds it."""
        torch = _torch()
        if slot.ws is None or slot.ws.numel() < nbytes:
            if slot.ws is not None:
                self.in_use -= slot.ws.numel()
            slot.ws = None
            slot.ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            self.in_use += slot.ws.numel()

    def _finish(self, slot):
        reqs = slot.reqs
        t = self.now()
        res = slot.res.cpu()  # the event has completed: no wait
        if reqs[0].op == "compress":
            for i, r in enumerate(reqs):
                size = int(res[i, 0])
                word = int(res[i, 1]) & ((1 << 64) - 1)
                st = word & 0xFFFFFFFF
                r.status = st - (1 << 32) if st >= 1 << 31 else st
                r.codec = word >> 32
                r.out = r.out[:size] if r.status == ebc.EBC_OK else None
                if r.out is not None and r.stream is not None:
                    r.out.record_stream(r.stream)
                r.t_done = t
        else:
            for i, r in enumerate(reqs):
                r.status = int(res[i])
                if r.status != ebc.EBC_OK:
                    r.out = None
                elif r.stream is not None:
                    r.out.record_stream(r.stream)
                r.t_done = t
        self.in_use -= slot.reserved
        slot.busy, slot.event, slot.reqs, slot.descs, slot.reserved = False, None, [], None, 0
        return reqs

    def poll(self):
        """Retire finished batches, then fill free slots.  Returns finished requests."""
        finished = []
        for s in self.slots:
            if s.busy and s.event.query():
                finished.extend(self._finish(s))
        for s in self.slots:
            if s.busy or not self.pending:
                continue
            reqs = self._pick(s)
            if not reqs:
                break
            for r in reqs:
                self.pending.remove(r)
            self._launch(s, reqs)
        return finished

    def busy(self) -> bool:
        return bool(self.pending) or any(s.busy for s in self.slots)

    def drain(self, timeout: float = 600.0):
        end = time.perf_counter() + timeout
        while self.busy():
            self.poll()
            if time.perf_counter() > end:
                raise TimeoutError("requests still pending")
            time.sleep(0.0002)


def percentile(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]


def run_stream(server: Server, stream, make_input, archive_pool: int = 32, warmup: float = 0.0,
               on_result=None, keep_results: bool = False):
    """Replay a request stream in real time.

    stream: dicts with t (arrival, s), op, rank, kind, n, eb (see
    synth.request_stream).  make_input(spec) -> contiguous fp32 CUDA tensor
    for a compress request.  Decompress requests take an archive produced
    earlier in the run (a bounded pool of recent ones, copied to exact-size
    buffers); with none yet they become compress requests.  Results are
    dropped after `on_result` unless keep_results.  Returns a summary dict.
    """
    import torch

    import random

    rng = random.Random(12345)
    pool = []
    reqs = []
    i = 0
    server.t0 = time.perf_counter()
    while i < len(stream) or server.busy():
        now = server.now()
        while i < len(stream) and stream[i]["t"] <= now:
            spec = stream[i]
            if spec["op"] == "decompress" and pool:
                a, hdr = pool[rng.randrange(len(pool))]
                r = Request("decompress", spec["t"], archive=a, header=hdr)
            else:
                r = Request("compress", spec["t"], x=make_input(spec), eb=spec["eb"])
            reqs.append(server.submit(r))
            i += 1
        for r in server.poll():
            if r.op == "compress" and r.status == ebc.EBC_OK:
                a = r.out.clone()
                hdr = bytes(a[:ebc.HDR_BYTES].cpu().numpy().tobytes())  # also orders the copy
                pool.append((a, hdr))
                if len(pool) > archive_pool:
                    pool.pop(0)
            if on_result is not None:
                on_result(r)
            if not keep_results:
                r.out = r.x = r.archive = None
        time.sleep(0.0001)
    ok = [r for r in reqs if r.status == ebc.EBC_OK and r.t_arrival >= warmup]
    lat = [1e3 * r.latency for r in ok]
    # measured window: first measured arrival to last measured completion
    span = max(r.t_done for r in ok) - min(r.t_arrival for r in ok) if ok else 0.0
    nbytes = sum(r.nbytes for r in ok)
    # requests the library refused, by status (e.g. a short slice of a smooth
    # field whose relative bound falls below fp32 resolution)
    errors = {}
    for r in reqs:
        if r.status != ebc.EBC_OK:
            key = f"{r.status} {ebc.status_string(r.status)}"
            errors[key] = errors.get(key, 0) + 1
    return {
        "requests": len(reqs), "ok": sum(r.status == ebc.EBC_OK for r in reqs),
        "errors": errors,
        "measured": len(ok),
        "compress": sum(r.op == "compress" for r in ok),
        "decompress": sum(r.op == "decompress" for r in ok),
        "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
        "mean_ms": round(sum(lat) / len(lat), 3) if lat else None,
        "throughput_GBps": round(nbytes / 1e9 / span, 3) if span > 0 else None,
        "batches": server.batches, "memory_waits": server.mem_waits,
        "workspaces_released": server.ws_released,
        "mean_batch": round(sum(r.batch_size for r in reqs) / max(len(reqs), 1), 2),
        "peak_hbm_in_use_GB": round(server.peak_in_use / 1e9, 3),
        "torch_peak_allocated_GB": round(torch.cuda.max_memory_allocated() / 1e9, 3),
        "hbm_budget_GB": round(server.budget / 1e9, 3), "slots": len(server.slots),
    }
