"""Seeded synthetic input fields.

This module only draws inputs; it holds none of the compressor's arithmetic, and
it is the one module that both the oracle-side tests and the GPU-side tests and
benchmark import.  Every field is generated in float64 with NumPy's PCG64
``default_rng`` and FFTs from ``scipy.fft`` (deterministic for any thread
count), then cast to the requested dtype.

The paper's datasets (turbulence, seismic, weather, combustion; Tab. "apps") are
not available; these fields stand in for them with matching shapes and value
structure:

* ``blobs_64``        smooth 64^3 field: 8 Gaussian blobs, a sine product and
                      weak white noise.
* ``grf``             Gaussian random field with a power-law spectrum (the
                      512^3 turbulence-like field uses P(k) ~ k^-5/3).
* ``climate_2d``      1800 x 3600 latitude-longitude field: zonal bands plus
                      k^-3 spectral noise, optionally 30 % masked with a
                      constant fill just below the data.
* ``lognormal``       log-normal density exp(1.5 * GRF(k^-2)), heavy tailed.
* ``random_field`` / ``poly_field`` small test inputs.
"""

from __future__ import annotations

import numpy as np

try:
    import scipy.fft as _fft
    _WORKERS = {"workers": -1}
except ImportError:  # pragma: no cover
    import numpy.fft as _fft
    _WORKERS = {}


def value_range(x: np.ndarray) -> float:
    """max - min over all values, in float64 (the relative-bound reference)."""
    x64 = np.asarray(x, dtype=np.float64)
    return float(np.max(x64) - np.min(x64))


def _kmag(shape):
    ks = [np.fft.fftfreq(n) * n for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    k2 = None
    for j, kj in enumerate(ks):
        sh = [1] * len(shape)
        sh[j] = kj.size
        term = (kj.reshape(sh)) ** 2
        k2 = term if k2 is None else k2 + term
    return np.sqrt(k2)


def grf(shape, amp_exponent: float, seed: int, dtype=np.float32) -> np.ndarray:
    """Unit-variance Gaussian random field; spectral amplitude ~ |k|^amp_exponent.

    amp_exponent = -5/6 gives a 3-D power spectrum P(k) ~ k^-5/3.
    Wavenumbers are integers (fftfreq * n); the k = 0 mode is removed.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = _fft.rfftn(white, **_WORKERS)
    del white
    k = _kmag(shape)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** amp_exponent, 0.0)
    spec *= amp
    del amp, k
    f = _fft.irfftn(spec, s=shape, **_WORKERS)
    del spec
    f -= f.mean()
    f /= f.std()
    return f.astype(dtype)


def blobs_64(seed: int = 0, n: int = 64, dtype=np.float32) -> np.ndarray:
    """Sum of 8 Gaussian blobs + sine product + N(0, 1e-3) noise on n^3."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, n, size=(8, 3))
    widths = rng.uniform(4, 16, size=8)
    amps = rng.uniform(0.5, 1.5, size=8)
    i = np.arange(n, dtype=np.float64)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    f = np.zeros((n, n, n), dtype=np.float64)
    for b in range(8):
        r2 = (I - centres[b, 0]) ** 2 + (J - centres[b, 1]) ** 2 + (K - centres[b, 2]) ** 2
        f += amps[b] * np.exp(-r2 / (2.0 * widths[b] ** 2))
    f += 0.5 * np.sin(2 * np.pi * I / n) * np.sin(4 * np.pi * J / n) * np.sin(6 * np.pi * K / n)
    f += rng.normal(0.0, 1e-3, size=f.shape)
    return f.astype(dtype)


def climate_2d(field_index: int, shape=(1800, 3600), masked=None, dtype=np.float32):
    """Latitude-longitude field: zonal bands + k^-3 noise, unit std.

    Odd field indices (or ``masked=True``) set the 30 % of points where a smooth
    k^-2 random field exceeds its 70th percentile to the fill value -5.0.
    """
    seed = 1000 + field_index
    rng = np.random.default_rng(seed)
    ny, nx = shape
    phi = (np.arange(ny) + 0.5) * np.pi / ny - np.pi / 2
    a = rng.uniform(0.2, 1.0, size=4) / np.arange(1, 5)
    th = rng.uniform(0, 2 * np.pi, size=4)
    bands = np.zeros(ny)
    for m in range(4):
        bands += a[m] * np.cos(2 * (m + 1) * phi + th[m])
    bands2 = np.repeat(bands[:, None], nx, axis=1)
    white = rng.standard_normal(shape)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(ky ** 2 + kx ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** -1.5, 0.0)
    noise = _fft.irfft2(_fft.rfft2(white, **_WORKERS) * amp, s=shape, **_WORKERS)
    noise = (noise - noise.mean()) / noise.std() * (0.3 * bands2.std())
    f = bands2 + noise
    f = (f - f.mean()) / f.std()
    if masked is None:
        masked = field_index % 2 == 1
    if masked:
        w2 = rng.standard_normal(shape)
        with np.errstate(divide="ignore"):
            amp2 = np.where(k > 0, k ** -2.0, 0.0)
        sm = _fft.irfft2(_fft.rfft2(w2, **_WORKERS) * amp2, s=shape, **_WORKERS)
        thr = np.percentile(sm, 70.0)
        f = np.where(sm > thr, -5.0, f)
    return f.astype(dtype)


def lognormal(shape=(256, 384, 384), seed: int = 0, dtype=np.float64) -> np.ndarray:
    """exp(1.5 * unit GRF with amplitude k^-1), i.e. P(k) ~ k^-2, heavy tailed."""
    g = grf(shape, -1.0, seed, dtype=np.float64)
    return np.exp(1.5 * g).astype(dtype)


def random_field(shape, seed: int = 0, dtype=np.float32, scale: float = 1.0,
                 smooth: bool = True) -> np.ndarray:
    """Small test field: smooth trend plus noise (or pure noise)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(shape) * scale
    if smooth:
        grids = np.meshgrid(*[np.linspace(0, 1, n) for n in shape], indexing="ij")
        trend = np.zeros(shape)
        for j, g in enumerate(grids):
            trend += np.sin(2.0 * np.pi * (j + 1) * g + 0.3 * j)
        f = trend * 10.0 * scale + 0.05 * f
    return f.astype(dtype)


def poly_field(shape, degrees, seed: int = 0, dtype=np.float64, max_abs: int = 1 << 19):
    """Integer-valued tensor-product polynomial on the integer grid.

    ``degrees[j]`` is the degree in coordinate j; each factor is a product of
    (t - r) with integer roots drawn near the middle of the axis.  Raises if a
    value would exceed ``max_abs`` (callers pick small shapes and degrees).
    """
    rng = np.random.default_rng(seed)
    facs = []
    for n, deg in zip(shape, degrees):
        t = np.arange(n, dtype=np.float64)
        roots = rng.integers(n // 4, max(n // 4 + 1, (3 * n) // 4 + 1), size=deg)
        p = np.ones(n)
        for r in roots:
            p = p * (t - r)
        facs.append(p)
    f = facs[0]
    for p in facs[1:]:
        f = np.multiply.outer(f, p)
    if np.max(np.abs(f)) > max_abs:
        raise ValueError("polynomial too large for the grid; pick smaller degrees or shape")
    return f.astype(dtype)


def grf_torch(shape, amp_exponent: float, seed: int, device="cuda:0"):
    """Same recipe as :func:`grf`, computed on the GPU in float32 with torch.

    Used where a large field has to be drawn quickly on the device (the
    512^3 benchmark field); the values differ from :func:`grf` in rounding and
    random stream, not in distribution.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    white = torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(white)
    del white
    k2 = None
    for j, n in enumerate(shape):
        if j == len(shape) - 1:
            kj = torch.fft.rfftfreq(n, device=device) * n
        else:
            kj = torch.fft.fftfreq(n, device=device) * n
        sh = [1] * len(shape)
        sh[j] = kj.numel()
        term = (kj.reshape(sh)) ** 2
        k2 = term if k2 is None else k2 + term
    k = torch.sqrt(k2)
    amp = torch.where(k > 0, k.clamp_min(1e-30) ** amp_exponent, torch.zeros_like(k))
    spec *= amp
    del amp, k, k2
    f = torch.fft.irfftn(spec, s=tuple(shape))
    del spec
    f -= f.mean()
    f /= f.std()
    return f.contiguous()


def lognormal_torch(shape=(256, 384, 384), seed: int = 0, device="cuda:0"):
    """:func:`lognormal` drawn on the GPU (float64 result) from :func:`grf_torch`."""
    import torch
    g = grf_torch(shape, -1.0, seed, device=device).to(torch.float64)
    return torch.exp(1.5 * g)
