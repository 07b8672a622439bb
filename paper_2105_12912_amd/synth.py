"""Seeded synthetic scientific fields (shared input generators).

This module only draws random numbers and shapes them into fields; it holds
none of the compressor's arithmetic, so both the HIP path and the CPU oracle
can be fed from it.  Every field is generated in float64 with
``numpy.random.default_rng(seed)`` and cast to float32 once, at the end.

The recipes stand in for the paper's evaluation datasets (Sec. V-A.3, the
dataset table: HACC 1D, CESM-ATM 2D 1800x3600, Hurricane 100x500x500,
Nyx 512^3, ...), which are not available here: same shapes, similar
smoothness (power-law Gaussian random fields with spectral slope -3) and
sparsity (a lognormal density with a constant background).

Arrays are C-ordered with x fastest: ``(nx,)``, ``(ny, nx)``, ``(nz, ny, nx)``.
"""
from __future__ import annotations

import math

import numpy as np

try:  # multi-threaded FFT when available (deterministic per transform)
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def grf(shape, beta: float = -3.0, seed: int = 0) -> np.ndarray:
    """Gaussian random field with power spectrum ~ k^beta, mean 0, sd 1 (float64).

    White N(0,1) noise is filtered in Fourier space by the amplitude k^(beta/2)
    with integer wavenumbers k = |fftfreq * n| (k = 0 removed).
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = _rfftn(white)
    del white
    k2 = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            f = np.fft.rfftfreq(n) * n
        else:
            f = np.fft.fftfreq(n) * n
        sh = [1] * len(shape)
        sh[ax] = f.size
        term = (f.astype(np.float64) ** 2).reshape(sh)
        k2 = term if k2 is None else k2 + term
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (beta / 4.0), 0.0)  # (k^2)^(beta/4) = k^(beta/2)
    del k2
    spec *= amp
    del amp
    field = _irfftn(spec, shape)
    del spec
    field -= field.mean()
    sd = field.std()
    if sd > 0:
        field /= sd
    return field


def scale_to(a: np.ndarray, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    amin, amax = float(a.min()), float(a.max())
    if amax == amin:
        return np.full_like(a, lo)
    return lo + (a - amin) * ((hi - lo) / (amax - amin))


def smooth_2d(ny: int = 256, nx: int = 256, seed: int = 1) -> np.ndarray:
    """GRF (slope -3) scaled to [-1, 1]; the 256x256 small case."""
    return scale_to(grf((ny, nx), -3.0, seed)).astype(np.float32)


def climate_2d(ny: int = 1800, nx: int = 3600, seed: int = 2, noise_seed: int = 102,
               noise_rel: float = 1e-5) -> np.ndarray:
    """CESM-ATM-shaped field: GRF scaled to [-1, 1] plus white noise of 1e-5 of the range."""
    f = scale_to(grf((ny, nx), -3.0, seed))
    rng = np.random.default_rng(noise_seed)
    f += rng.standard_normal(f.shape) * (noise_rel * 2.0)
    return f.astype(np.float32)


def lognormal_3d(shape=(512, 512, 512), seed: int = 3, sigma: float = 1.5,
                 background_frac: float = 0.40) -> np.ndarray:
    """Nyx-like density: exp(sigma * g) with the lowest 40% of g set to one constant."""
    g = grf(shape, -3.0, seed)
    flat = g.reshape(-1)
    kth = int(math.floor(background_frac * (flat.size - 1)))
    thr = float(np.partition(flat, kth)[kth])
    out = np.exp(sigma * g)
    out[g <= thr] = math.exp(sigma * thr)
    del g
    return out.astype(np.float32)


def random_walk_1d(n: int, seed: int = 4) -> np.ndarray:
    """Smooth 1D field: cumulative sum of N(0,1) steps scaled to [-1, 1]."""
    rng = np.random.default_rng(seed)
    w = np.cumsum(rng.standard_normal(int(n)))
    return scale_to(w).astype(np.float32)


def sparse_background_1d(n: int, seed: int = 15, active: float = 0.004,
                         block: int = 4096) -> np.ndarray:
    """1D field that is constant almost everywhere: blocks of `block` values,
    each a random-walk segment with probability `active` and otherwise the
    constant level the walk last reached (a mostly empty domain, the
    background-dominated case where the run-length workflow wins)."""
    rng = np.random.default_rng(seed)
    nb = (n + block - 1) // block
    on = rng.random(nb) < active
    steps = np.zeros(nb * block, np.float64)
    k = int(on.sum())
    steps.reshape(nb, block)[on] = rng.standard_normal((k, block))
    x = np.cumsum(steps)[:n]
    return scale_to(x).astype(np.float32)


def grf_field(shape, seed: int, kind: str = "grf") -> np.ndarray:
    if kind == "grf":
        return scale_to(grf(shape, -3.0, seed)).astype(np.float32)
    if kind == "lognormal":
        return lognormal_3d(shape, seed)
    raise ValueError(kind)


# ----------------------------------------------------------------- manifests

def batch_manifest(seed: int = 4, n_fields: int = 64, max_1d: int = 280_953_867):
    """The 64-field mixed-rank batch: list of dicts (rank, shape, kind, seed).

    Ranks cycle 1/2/3.  Fixed members: 1D 1e6 and 280,953,867 (HACC length),
    2D 1800x3600, 3D 64^3, 384^3 and 100x500x500 (Hurricane shape).  Others:
    1D log-uniform in [1e6, 2.8e8] (random walk), 2D ny log-uniform in
    [256, 1800] with nx = 2 ny (GRF), 3D cube side log-uniform in [64, 384]
    alternating GRF and lognormal.
    """
    rng = np.random.default_rng(seed)
    fixed = {
        1: [(1_000_000,), (max_1d,)],
        2: [(1800, 3600)],
        3: [(64, 64, 64), (384, 384, 384), (100, 500, 500)],
    }
    out = []
    alt = 0
    for i in range(n_fields):
        rank = 1 + i % 3
        if fixed[rank]:
            shape = fixed[rank].pop(0)
        elif rank == 1:
            shape = (int(math.exp(rng.uniform(math.log(1e6), math.log(2.8e8)))),)
        elif rank == 2:
            ny = int(math.exp(rng.uniform(math.log(256), math.log(1800))))
            shape = (ny, 2 * ny)
        else:
            s = int(math.exp(rng.uniform(math.log(64), math.log(384))))
            shape = (s, s, s)
        if rank == 1:
            kind = "walk"
        elif rank == 2:
            kind = "grf"
        else:
            kind = "grf" if alt % 2 == 0 else "lognormal"
            alt += 1
        out.append(dict(rank=rank, shape=tuple(int(v) for v in shape), kind=kind,
                        seed=int(1000 * seed + i)))
    return out


def make_manifest_field(entry) -> np.ndarray:
    if entry["kind"] == "walk":
        return random_walk_1d(entry["shape"][0], entry["seed"])
    return grf_field(entry["shape"], entry["seed"], entry["kind"])


def request_stream(seed: int = 5, rate: float = 200.0, duration: float = 60.0,
                   min_bytes: float = 1e6, max_bytes: float = 2e9):
    """Poisson request stream for the serving loop.

    Each request: arrival time (s), op ('compress'|'decompress'), rank, kind
    ('grf'|'lognormal'), element count (log-uniform bytes / 4), rel eb drawn
    from {1e-2, 1e-3, 1e-4}.
    """
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        nbytes = math.exp(rng.uniform(math.log(min_bytes), math.log(max_bytes)))
        out.append(dict(t=t, op="compress" if rng.random() < 0.5 else "decompress",
                        rank=int(rng.integers(1, 4)),
                        kind="grf" if rng.random() < 0.5 else "lognormal",
                        n=max(1, int(nbytes // 4)),
                        eb=float(rng.choice([1e-2, 1e-3, 1e-4]))))
    return out


# ------------------------------------------------------- device-side variants
# The same recipes drawn with torch's generator on the GPU, for the large
# benchmark batches (seconds instead of minutes to generate).  Same
# definitions, a different random stream: these fields are not bit-identical
# to the numpy ones above.

def _t():
    import torch
    return torch


def grf_torch(shape, beta: float = -3.0, seed: int = 0, device="cuda"):
    """Device GRF: white N(0,1) filtered by k^(beta/2), standardised (float64)."""
    torch = _t()
    shape = tuple(int(s) for s in shape)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    white = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    spec = torch.fft.rfftn(white)
    del white
    k2 = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            f = torch.fft.rfftfreq(n, device=device, dtype=torch.float64) * n
        else:
            f = torch.fft.fftfreq(n, device=device, dtype=torch.float64) * n
        sh = [1] * len(shape)
        sh[ax] = f.numel()
        term = (f * f).reshape(sh)
        k2 = term if k2 is None else k2 + term
    amp = torch.where(k2 > 0, k2.clamp(min=1e-300) ** (beta / 4.0), torch.zeros_like(k2))
    out = torch.fft.irfftn(spec * amp, s=shape)
    del spec
    sd = out.std()
    return (out - out.mean()) / (sd if float(sd) > 0 else 1.0)


def _scale_t(a, lo=-1.0, hi=1.0):
    amin, amax = float(a.min()), float(a.max())
    if amax == amin:
        return a.new_full(a.shape, lo)
    return lo + (a - amin) * ((hi - lo) / (amax - amin))


def manifest_field_torch(entry, device="cuda"):
    """A batch-manifest field generated on the device (float32, contiguous)."""
    torch = _t()
    shape, seed, kind = entry["shape"], entry["seed"], entry["kind"]
    if kind == "walk":
        g = torch.Generator(device=device)
        g.manual_seed(int(seed))
        w = torch.randn(int(shape[0]), generator=g, device=device, dtype=torch.float64).cumsum_(0)
        return _scale_t(w).float().contiguous()
    gr = grf_torch(shape, -3.0, seed, device)
    if kind == "grf":
        return _scale_t(gr).float().contiguous()
    return lognormal_from_torch(gr).float().contiguous()


def lognormal_from_torch(g, sigma: float = 1.5, background_frac: float = 0.40):
    """exp(sigma g) with the lowest `background_frac` of g set to one constant."""
    torch = _t()
    flat = g.reshape(-1)
    kth = int(math.floor(background_frac * (flat.numel() - 1)))
    thr = float(torch.kthvalue(flat.cpu() if flat.numel() < (1 << 24) else flat, kth + 1).values)
    out = torch.exp(sigma * g)
    out[g <= thr] = math.exp(sigma * thr)
    return out


def serving_base_torch(rank: int, kind: str, n: int, seed: int, device="cuda"):
    """A device-resident base field of about n elements for the serving stream:
    1D (n,), 2D (n / 16384, 16384), 3D (n / 512^2, 512, 512); requests take
    prefixes of whole rows / planes."""
    torch = _t()
    if rank == 1:
        shape = (int(n),)
    elif rank == 2:
        shape = (max(1, int(n) // 16384), 16384)
    else:
        shape = (max(1, int(n) // (512 * 512)), 512, 512)
    if rank == 1 and kind == "grf":
        return manifest_field_torch(dict(shape=shape, seed=seed, kind="walk"), device)
    g = grf_torch(shape, -3.0, seed, device)
    if kind == "grf":
        return _scale_t(g).float().contiguous()
    return lognormal_from_torch(g).float().contiguous()
