"""Autotuner for the launch geometry: tiles, construction grid, scan schedule.

For each shape class (rank, ceil(log2 nx), size class) present in a set of
fields, every candidate (workgroup tile width in waves along x, persistent
construction grid) is installed in the library's tuning table, the class's
largest field is compressed and decompressed with per-stage event timing, and
the candidate with the smallest construct + reconstruct time wins.  Then the
scan schedule (tile count up to which a prefix sum adds the preceding tile
sums directly instead of scanning them first) is chosen the same way from
the stages made of scans.  Every candidate's archive must be byte-identical
to the first one's and its reconstruction bit-identical: tuning is only
allowed to change speed.

The chosen table is installed with ``ebc_set_tuning`` and can be saved to /
loaded from a JSON cache.
"""
from __future__ import annotations

import json
import os

from . import ebc

GRIDS = (1024, 2048, 4096)
CANDIDATES = {
    1: [(0, g) for g in GRIDS],
    2: [(wx, g) for wx in (1, 2, 4) for g in GRIDS],
    3: [(wx, g) for wx in (1, 2, 4) for g in GRIDS],
}


SCANS = (64, 1024, 16384)
SCAN_STAGES = ("scan_outliers", "encode_scan", "decode_prep")


class TuningChangedBytes(AssertionError):
    pass


def shape_key(x):
    rank = x.dim()
    dims = tuple(int(s) for s in reversed(x.shape))
    nxc, nc = ebc.ebc_shape_class(rank, dims)
    return rank, nxc, nc


def _entry(key, wx, grid, scan=0):
    return dict(rank=key[0], nx_class=key[1], n_class=key[2], tile_wx=wx, grid=grid,
                scan_direct=scan)


def _time_candidate(x, eb, reps, ws, stages=("construct", "reconstruct")):
    import torch

    best = None
    a = y = None
    for _ in range(reps):
        a, cs = ebc.compress(x, eb, "rel", stats=True, workspace=ws)
        y, ds = ebc.decompress(a, stats=True, workspace=ws)
        st = dict(cs.stages())
        for k, v in ds.stages().items():
            st[k] = st.get(k, 0.0) + v
        t = sum(st.get(k, 0.0) for k in stages)
        best = t if best is None else min(best, t)
    torch.cuda.synchronize()
    return best, a, y


def tune(fields, eb: float = 1e-4, reps: int = 2, install: bool = True):
    """Tune every shape class present in `fields` (CUDA fp32 tensors).

    Returns (table, report): table = list of tuning entries, report = per
    class the candidate times in ms.
    """
    import torch

    classes = {}
    for x in fields:
        k = shape_key(x)
        if k not in classes or x.numel() > classes[k].numel():
            classes[k] = x
    table, report = [], {}
    ws = ebc.Workspace(fields[0].device)
    try:
        for key in sorted(classes):
            x = classes[key]
            ref_a = ref_y = None
            times = {}
            for wx, grid in CANDIDATES[key[0]]:
                st = ebc.ebc_set_tuning(table + [_entry(key, wx, grid)])
                if st != ebc.EBC_OK:
                    raise ebc.EbcError(st, "ebc_set_tuning")
                t, a, y = _time_candidate(x, eb, reps, ws)
                if ref_a is None:
                    ref_a, ref_y = a.clone(), y.clone()
                elif not (a.numel() == ref_a.numel() and torch.equal(a, ref_a)
                          and torch.equal(y.view(torch.int32), ref_y.view(torch.int32))):
                    raise TuningChangedBytes(f"class {key}: tile {wx} grid {grid} changed the output")
                times[(wx, grid)] = t
            wx, grid = min(times, key=times.get)
            rep = {f"{w}x{g}": round(v, 4) for (w, g), v in times.items()}
            stimes = {}
            for scan in SCANS:
                st = ebc.ebc_set_tuning(table + [_entry(key, wx, grid, scan)])
                if st != ebc.EBC_OK:
                    raise ebc.EbcError(st, "ebc_set_tuning")
                t, a, y = _time_candidate(x, eb, reps, ws, SCAN_STAGES)
                if not (a.numel() == ref_a.numel() and torch.equal(a, ref_a)
                        and torch.equal(y.view(torch.int32), ref_y.view(torch.int32))):
                    raise TuningChangedBytes(f"class {key}: scan schedule {scan} changed the output")
                stimes[scan] = t
            scan = min(stimes, key=stimes.get)
            rep.update({f"scan{k}": round(v, 4) for k, v in stimes.items()})
            table.append(_entry(key, wx, grid, scan))
            report[str(key)] = rep
    finally:
        ebc.ebc_set_tuning(table if install else [])
    return table, report


def save(table, path: str, meta: dict | None = None):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"version": 1, "meta": meta or {}, "entries": table}, f, indent=1)


def load(path: str, install: bool = True):
    with open(path) as f:
        data = json.load(f)
    if data.get("version") != 1:
        raise ValueError("unknown tuning cache version")
    table = data["entries"]
    if install:
        st = ebc.ebc_set_tuning(table)
        if st != ebc.EBC_OK:
            raise ebc.EbcError(st, "ebc_set_tuning")
    return table
