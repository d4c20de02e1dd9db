"""Seeded synthetic inputs for the hybrid-dealiased real convolution.

This module only draws numbers: it holds none of the convolution method's
arithmetic, so both the GPU path's tests/benchmarks and the CPU oracle can be
fed from it without sharing any of the method's code.

Every draw uses ``numpy.random.default_rng(SeedSequence([SEED, cfg, pair, role]))``
with role 0 = f, 1 = g, 2 = upstream gradient, 3 = auxiliary (phases, sizes).
Values are drawn in float64 and rounded once to the run dtype; consumers that
need a float64 reference upcast the rounded values.

Workload shapes (the paper's benchmark setting, Sec. 6: padding ratio 2 per
axis, power-of-two sizes, equal-length real inputs):

* cfg 1: 1D, L=1024, U[-1,1], one pair (correctness/latency case);
* cfg 2: 1D, L=2^20, N(0,1), batch of 64 pairs;
* cfg 3: 2D, 2048x2048, U[-1,1], batch of 4;
* cfg 4: 3D, 256^3, N(0,1) white noise shaped by a |k|^(-5/3) spectral
  envelope with seeded random phases, then standardised; upstream gradient
  N(0,1);
* cfg 5: an uneven batch -- 512 1D pairs with L = round(2^U(8,16)), 64 2D
  pairs with each side from {128,256,384,512}, 8 3D cubes with side from
  {32,64,96}; all U[-1,1].
"""
from __future__ import annotations

import numpy as np

SEED = 260814497

ROLE_F, ROLE_G, ROLE_U, ROLE_AUX = 0, 1, 2, 3


def rng(cfg: int, pair: int, role: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED, int(cfg), int(pair), int(role)]))


def _cast(x: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(x.astype(dtype))


def uniform(shape, cfg: int, pair: int, role: int, dtype=np.float64) -> np.ndarray:
    return _cast(rng(cfg, pair, role).uniform(-1.0, 1.0, size=shape), dtype)


def normal(shape, cfg: int, pair: int, role: int, dtype=np.float64) -> np.ndarray:
    return _cast(rng(cfg, pair, role).standard_normal(size=shape), dtype)


def small_ints(shape, cfg: int, pair: int, role: int, lo: int = -3, hi: int = 3,
               dtype=np.float64) -> np.ndarray:
    """Integers in [lo, hi]: products and sums stay exact in float64."""
    return _cast(rng(cfg, pair, role).integers(lo, hi + 1, size=shape), dtype)


def spectral_field(shape, cfg: int, pair: int, role: int, slope: float = -5.0 / 3.0,
                   dtype=np.float64) -> np.ndarray:
    """Real field with a |k|^slope amplitude envelope and random phases.

    White N(0,1) noise is transformed with a real FFT; its amplitude is
    replaced by |k|^slope (k = 0 removed) using integer wavenumbers, its phase
    by a seeded U[0, 2 pi) draw from the same stream; the inverse real FFT is standardised to mean 0
    and standard deviation 1.  (A shaped field is not i.i.d.; this is the
    reading used for the 3D workload.)
    """
    g = rng(cfg, pair, role)
    white = g.standard_normal(size=shape)
    spec = np.fft.rfftn(white)
    ks = [np.fft.fftfreq(n) * n for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    grids = np.meshgrid(*ks, indexing="ij")
    kmag = np.sqrt(sum(k * k for k in grids))
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = kmag[nz] ** slope
    phase = g.uniform(0.0, 2.0 * np.pi, size=spec.shape)
    field = np.fft.irfftn(amp * np.exp(1j * phase), s=shape, axes=list(range(len(shape))))
    field = (field - field.mean()) / field.std()
    return _cast(field, dtype)


def cfg5_items(cfg: int = 5):
    """Shapes of the uneven batch: list of tuples (extents per axis)."""
    a = rng(cfg, 0, ROLE_AUX)
    items = []
    for _ in range(512):
        items.append((int(round(2.0 ** a.uniform(8.0, 16.0))),))
    for _ in range(64):
        items.append((int(a.choice([128, 256, 384, 512])), int(a.choice([128, 256, 384, 512]))))
    for _ in range(8):
        s = int(a.choice([32, 64, 96]))
        items.append((s, s, s))
    return items


def pair_for(cfg: int, pair: int, shape, dtype=np.float32, dist: str = "uniform"):
    """(f, g) for one pair of a workload."""
    if dist == "uniform":
        return uniform(shape, cfg, pair, ROLE_F, dtype), uniform(shape, cfg, pair, ROLE_G, dtype)
    if dist == "normal":
        return normal(shape, cfg, pair, ROLE_F, dtype), normal(shape, cfg, pair, ROLE_G, dtype)
    if dist == "spectral":
        return (spectral_field(shape, cfg, pair, ROLE_F, dtype=dtype),
                spectral_field(shape, cfg, pair, ROLE_G, dtype=dtype))
    if dist == "ints":
        return small_ints(shape, cfg, pair, ROLE_F, dtype=dtype), small_ints(shape, cfg, pair, ROLE_G, dtype=dtype)
    raise ValueError(dist)
