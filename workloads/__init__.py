"""Seeded synthetic inputs shaped like the paper's benchmark workloads.

This module only draws random numbers and lays out input arrays. It holds none
of the imaging method's arithmetic (no measurement operator, no wavelet, no
proximal step), so both the FP64 CPU oracle and the GPU library can be fed
from it without sharing any code of the method.

Workload shapes follow the paper's benchmark description (Section "Benchmark
Timings" and "Application to Big-Data"): a random Gaussian density of
baselines spanning +-pi on each axis, a Kaiser-Bessel kernel with J = 4, and a
sky made of compact and extended sources. The sizes are the five workload
workload configurations listed in ``CONFIGS``.

Conventions shared with every consumer:
  * image ``x`` is real, shape (n, n), row index = v axis, column = u axis;
  * ``uv`` has shape (M, 2), column 0 = u, column 1 = v, in radians per pixel,
    each value in [-pi, pi);
  * visibility arrays are complex, shape (M,).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def rng_for(config_index: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator seeded with 1000 + config index (plus a sub-stream)."""
    return np.random.Generator(np.random.PCG64([1000 + int(config_index), int(stream)]))


# --------------------------------------------------------------------------
# sky
# --------------------------------------------------------------------------
def gaussian_sky(n: int, n_sources: int, rng: np.random.Generator,
                 width_range=(0.5, 3.0)) -> np.ndarray:
    """Real n x n image made of ``n_sources`` circular Gaussian sources.

    Centres are uniform over the pixels, widths (sigma, in pixels) uniform in
    ``width_range`` and peak amplitudes uniform in [0, 1). Each source is
    rendered on a window of +-5 sigma (periodic wrap is not used: sources
    near the edge are simply clipped).
    """
    x = np.zeros((n, n), dtype=np.float64)
    cy = rng.uniform(0, n, n_sources)
    cx = rng.uniform(0, n, n_sources)
    sig = rng.uniform(width_range[0], width_range[1], n_sources)
    amp = rng.uniform(0.0, 1.0, n_sources)
    for k in range(n_sources):
        r = int(math.ceil(5 * sig[k]))
        y0, y1 = max(0, int(cy[k]) - r), min(n, int(cy[k]) + r + 1)
        x0, x1 = max(0, int(cx[k]) - r), min(n, int(cx[k]) + r + 1)
        yy = np.arange(y0, y1)[:, None] + 0.5
        xx = np.arange(x0, x1)[None, :] + 0.5
        x[y0:y1, x0:x1] += amp[k] * np.exp(-((yy - cy[k]) ** 2 + (xx - cx[k]) ** 2)
                                           / (2.0 * sig[k] ** 2))
    return x


def n_sources_for(n: int) -> int:
    """20 sources per 256^2 of image area, at least 20."""
    return max(20, int(round(20 * (n / 256.0) ** 2)))


# --------------------------------------------------------------------------
# baselines
# --------------------------------------------------------------------------
def _in_square(a: np.ndarray) -> np.ndarray:
    return (a >= -math.pi) & (a < math.pi)


def uv_gaussian(M: int, rng: np.random.Generator, sigma: float = math.pi / 3,
                dtype=np.float32, chunk: int = 1 << 24) -> np.ndarray:
    """(M, 2) baselines with u, v iid N(0, sigma^2) truncated to [-pi, pi).

    Out-of-range draws are re-drawn (a truncated normal), so no sample sits on
    the clipping edge. Values are rounded to ``dtype`` and re-checked so the
    rounded value is still inside [-pi, pi).
    """
    out = np.empty((M, 2), dtype=dtype)
    flat = out.reshape(-1)
    filled = 0
    total = 2 * M
    while filled < total:
        want = min(chunk, total - filled)
        d = rng.normal(0.0, sigma, int(want * 1.01) + 16).astype(dtype)
        d = d[_in_square(d.astype(np.float64))][:want]
        flat[filled:filled + d.size] = d
        filled += d.size
    return out


def uv_ring_core(M: int, rng: np.random.Generator, dtype=np.float32,
                 chunk: int = 1 << 24) -> np.ndarray:
    """(M, 2) baselines from a radially decaying ring-plus-core mixture.

    Radius: with probability 0.6 |N(0, (pi/6)^2)| (core), else
    N(0.55 pi, (0.08 pi)^2) (ring); angle uniform in [0, 2 pi). Points outside
    the square [-pi, pi)^2 are re-drawn.
    """
    out = np.empty((M, 2), dtype=dtype)
    filled = 0
    while filled < M:
        want = min(chunk, M - filled)
        m = int(want * 1.05) + 16
        core = rng.uniform(0.0, 1.0, m) < 0.6
        r = np.where(core, np.abs(rng.normal(0.0, math.pi / 6, m)),
                     rng.normal(0.55 * math.pi, 0.08 * math.pi, m))
        th = rng.uniform(0.0, TWO_PI, m)
        u = (r * np.cos(th)).astype(dtype)
        v = (r * np.sin(th)).astype(dtype)
        ok = _in_square(u.astype(np.float64)) & _in_square(v.astype(np.float64))
        u, v = u[ok][:want], v[ok][:want]
        out[filled:filled + u.size, 0] = u
        out[filled:filled + u.size, 1] = v
        filled += u.size
    return out


def unit_complex_noise(M: int, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian draws with E|n|^2 = 1 (independent real/imag parts)."""
    return (rng.standard_normal(M) + 1j * rng.standard_normal(M)) / math.sqrt(2.0)


def add_noise(y0: np.ndarray, draws: np.ndarray, snr_db: float = 30.0):
    """Add noise at an input SNR and return (y, sigma, epsilon).

    SNR = 20 log10(||y0||_2 / (sqrt(M) sigma)); epsilon = sigma sqrt(M + 2 sqrt(M)),
    i.e. the mean of ||n||^2 plus two standard deviations, so the true sky lies
    inside the l2 ball with high probability.
    """
    M = y0.size
    sigma = float(np.linalg.norm(y0)) / math.sqrt(M) * 10.0 ** (-snr_db / 20.0)
    y = y0 + sigma * draws
    eps = sigma * math.sqrt(M + 2.0 * math.sqrt(M))
    return y, sigma, eps


# --------------------------------------------------------------------------
# the workload configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    index: int
    n: int                 # image side
    oversample: int        # grid side K = oversample * n
    M: int                 # visibilities
    J: int                 # kernel support
    D: int                 # table samples per grid cell
    levels: int            # wavelet levels
    iters: int             # ADMM iterations
    uv_law: str = "gaussian"
    snr_db: float = 30.0
    extra: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return self.oversample * self.n


CONFIGS = {
    # plain FP64 ADMM, seconds on a CPU
    "admm64": Workload("admm-64sq-M8192-J4-fp64", 0, 64, 2, 8192, 4, 2000, 3, 50),
    # single-operator throughput, J in {4, 6}
    "op256": Workload("op-256sq-M1e6-J4", 1, 256, 2, 1_000_000, 4, 2000, 4, 1),
    "op256j6": Workload("op-256sq-M1e6-J6", 1, 256, 2, 1_000_000, 6, 2000, 4, 1),
    # mid-size solver parity: several wavelet levels run per level (not in the
    # small-image tail), work items span many staged chunks
    "mid128": Workload("mid-128sq-M4e4-J4", 5, 128, 2, 40_000, 4, 2000, 3, 20),
    # one GPU's share of the large distributed run
    "share2048": Workload("share-2048sq-M5e8-J4-ringcore", 2, 2048, 2, 500_000_000, 4, 2000, 4, 20,
                   uv_law="ringcore"),
}


def make_sky(w: Workload, rng: np.random.Generator) -> np.ndarray:
    return gaussian_sky(w.n, n_sources_for(w.n), rng)


def make_uv(w: Workload, rng: np.random.Generator, M: int | None = None,
            dtype=np.float32) -> np.ndarray:
    M = w.M if M is None else M
    if w.uv_law == "ringcore":
        return uv_ring_core(M, rng, dtype=dtype)
    return uv_gaussian(M, rng, dtype=dtype)


def batch_channels(n_channels: int, rng: np.random.Generator,
                   sizes=(128, 256, 512, 1024), m_lo=1e4, m_hi=5e6):
    """Per-channel (n, M) for the batched multi-channel workload.

    n is drawn uniformly from ``sizes`` and M log-uniformly in [m_lo, m_hi].
    """
    ns = rng.choice(np.asarray(sizes), n_channels)
    ms = np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), n_channels)).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(ns, ms)]


# --------------------------------------------------------------------------
# device-side generators for the 5e8-visibility workload (torch RNG, seeded)
# --------------------------------------------------------------------------
def torch_generator(config_index: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(1000 + int(config_index))
    return g


def uv_ring_core_torch(M: int, gen, device, chunk: int = 1 << 26):
    """Ring-plus-core baselines drawn on the device (same law as uv_ring_core)."""
    import torch
    out = torch.empty((M, 2), dtype=torch.float32, device=device)
    filled = 0
    while filled < M:
        want = min(chunk, M - filled)
        m = int(want * 1.05) + 16
        core = torch.rand(m, generator=gen, device=device) < 0.6
        r = torch.where(core, torch.randn(m, generator=gen, device=device).abs() * (math.pi / 6),
                        0.55 * math.pi + 0.08 * math.pi * torch.randn(m, generator=gen, device=device))
        th = torch.rand(m, generator=gen, device=device) * TWO_PI
        u = (r * torch.cos(th)).float()
        v = (r * torch.sin(th)).float()
        ok = (u >= -math.pi) & (u < math.pi) & (v >= -math.pi) & (v < math.pi)
        u, v = u[ok][:want], v[ok][:want]
        out[filled:filled + u.numel(), 0] = u
        out[filled:filled + u.numel(), 1] = v
        filled += u.numel()
    return out


def unit_complex_noise_torch(M: int, gen, device, dtype=None):
    import torch
    dtype = torch.complex64 if dtype is None else dtype
    re = torch.randn(M, generator=gen, device=device)
    im = torch.randn(M, generator=gen, device=device)
    return torch.complex(re, im).to(dtype) / math.sqrt(2.0)


def add_noise_torch(y0, draws, snr_db: float = 30.0):
    """Device version of add_noise: returns (y, sigma, epsilon)."""
    import torch
    M = y0.numel()
    nrm = float(torch.linalg.vector_norm(y0.to(torch.complex128) if y0.numel() < (1 << 27) else y0).item())
    sigma = nrm / math.sqrt(M) * 10.0 ** (-snr_db / 20.0)
    y = y0 + sigma * draws
    eps = sigma * math.sqrt(M + 2.0 * math.sqrt(M))
    return y, sigma, eps
