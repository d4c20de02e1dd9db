"""Plain definitions of the truncated real linear convolution and its adjoint.

Test infrastructure only (see the package docstring).

The paper computes a "dealiased binary convolution" f * g of two real arrays
of equal length L (Sec. 1, Sec. 6).  The truncated linear convolution it
reaches, for j = 0..L-1 (componentwise in d dimensions), is

    h_j = sum_{0 <= k <= j} f_k g_{j-k}.

Hybrid dealiasing produces exactly this (up to rounding) for any valid
(m, p, q): the implicitly padded DFT of Sec. 2 eq. (forwardr) is the DFT of
the input zero padded to length qm >= 2L - 1, so the circular convolution of
length qm has no wrapped terms at indices j < L.
"""
from __future__ import annotations

from fractions import Fraction
import itertools

import numpy as np


def _as64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def direct_conv(f, g) -> np.ndarray:
    """h_j = sum_{0<=k<=j} f_k g_{j-k}, j < L, in float64 (any dimension).

    Each output entry is one float64 dot product of the index box [0, j] of f
    with the flipped box of g.  O(L^(2d)) in total: use on small/mid sizes.
    """
    f = _as64(f)
    g = _as64(zero_extend(g, f.shape))
    h = np.empty_like(f)
    for j in itertools.product(*[range(n) for n in f.shape]):
        box = tuple(slice(0, jj + 1) for jj in j)
        flip = tuple(slice(jj, None, -1) if jj > 0 else slice(0, 1) for jj in j)
        h[j] = np.sum(f[box] * g[flip])
    return h


def direct_conv_at(f, g, indices) -> np.ndarray:
    """Selected entries h_j of direct_conv (for large arrays, sampled parity)."""
    f = _as64(f)
    g = _as64(zero_extend(g, f.shape))
    out = np.empty(len(indices), dtype=np.float64)
    for n, j in enumerate(indices):
        j = tuple(int(v) for v in np.atleast_1d(j))
        box = tuple(slice(0, jj + 1) for jj in j)
        flip = tuple(slice(jj, None, -1) if jj > 0 else slice(0, 1) for jj in j)
        out[n] = np.sum(f[box] * g[flip])
    return out


def zero_extend(g, shape) -> np.ndarray:
    """A kernel g of extents Lg <= L (per axis) written as an array of the
    extents L of f, zero beyond Lg.

    The conclusion section (Sec. 7, unequal lengths) proposes convolving f of
    length L_f with a shorter kernel g of length L_g by padding both
    implicitly; the result it reaches is the truncated convolution with g
    extended by zeros, h_j = sum_{k<=j, j-k<L_g} f_k g_{j-k}, j < L_f.  Every
    function of this module that takes (f, g) accepts such a g through this
    definition.
    """
    g = np.asarray(g)
    if g.ndim != len(shape) or any(a > b for a, b in zip(g.shape, shape)):
        raise ValueError("the kernel must have the dimension of f and extents <= f's")
    if tuple(g.shape) == tuple(shape):
        return g
    out = np.zeros(shape, dtype=g.dtype)
    out[tuple(slice(0, n) for n in g.shape)] = g
    return out


def brute_conv_exact(f, g):
    """The same sum with Python Fractions: exact for integer or dyadic inputs.

    Returns a nested list of Fractions with the shape of f (tiny sizes only).
    """
    fa = np.asarray(f)
    ga = zero_extend(g, fa.shape)
    shape = fa.shape
    F = {j: Fraction(float(fa[j])) for j in itertools.product(*[range(n) for n in shape])}
    G = {j: Fraction(float(ga[j])) for j in itertools.product(*[range(n) for n in shape])}
    H = np.empty(shape, dtype=object)
    for j in itertools.product(*[range(n) for n in shape]):
        acc = Fraction(0)
        for k in itertools.product(*[range(jj + 1) for jj in j]):
            acc += F[k] * G[tuple(a - b for a, b in zip(j, k))]
        H[j] = acc
    return H


def fft_conv(f, g, M=None, workers=1) -> np.ndarray:
    """Explicitly zero padded FFT convolution in float64, truncated to L.

    The standard dealiasing of Sec. 1: pad each axis to M_i >= L_i + Lg_i - 1
    (2 L_i - 1 for equal extents; default L_i + Lg_i), real FFTs, pointwise
    product, inverse, truncate.  A library FFT is one step; nothing is fused.
    """
    import scipy.fft as sfft

    f = _as64(f)
    Lg = np.asarray(g).shape
    g = _as64(zero_extend(g, f.shape))
    L = f.shape
    if M is None:
        M = tuple(n + k for n, k in zip(L, Lg))
    M = tuple(int(v) for v in np.atleast_1d(M))
    if any(m_ < n + k - 1 for m_, n, k in zip(M, L, Lg)):
        raise ValueError("padding M must satisfy M >= L + Lg - 1 on every axis")
    axes = tuple(range(f.ndim))
    Fh = sfft.rfftn(f, s=M, axes=axes, workers=workers)
    Gh = sfft.rfftn(g, s=M, axes=axes, workers=workers)
    h = sfft.irfftn(Fh * Gh, s=M, axes=axes, workers=workers)
    return np.ascontiguousarray(h[tuple(slice(0, n) for n in L)])


def grad_direct(f, g, u):
    """Adjoint of h = conv(f, g) for an upstream gradient u = dLoss/dh.

    Since h_j = sum_{k<=j} f_k g_{j-k} (j < L),
        df_k = sum_{0<=i<L-k} g_i u_{k+i},   dg_k = sum_{0<=i<L-k} f_i u_{k+i}
    (componentwise boxes in d dimensions).  Direct float64 sums.
    """
    f = _as64(f)
    g = _as64(g)
    u = _as64(u)
    L = f.shape
    df = np.empty_like(f)
    dg = np.empty_like(f)
    for k in itertools.product(*[range(n) for n in L]):
        ubox = tuple(slice(kk, None) for kk in k)
        box = tuple(slice(0, n - kk) for n, kk in zip(L, k))
        df[k] = np.sum(g[box] * u[ubox])
        dg[k] = np.sum(f[box] * u[ubox])
    return df, dg


def grad_direct_at(f, g, u, indices):
    """Selected entries of grad_direct (sampled parity at large sizes)."""
    f = _as64(f)
    g = _as64(g)
    u = _as64(u)
    L = f.shape
    df = np.empty(len(indices))
    dg = np.empty(len(indices))
    for n, k in enumerate(indices):
        k = tuple(int(v) for v in np.atleast_1d(k))
        ubox = tuple(slice(kk, None) for kk in k)
        box = tuple(slice(0, nn - kk) for nn, kk in zip(L, k))
        df[n] = np.sum(g[box] * u[ubox])
        dg[n] = np.sum(f[box] * u[ubox])
    return df, dg


def fft_grad(f, g, u, workers=1):
    """Full-size adjoint via explicitly padded FFT correlations (float64).

    df_k = sum_i g_i u_{k+i}: a cross-correlation, computed as the
    convolution of g with the reversal of u, read back reversed.
    """
    f = _as64(f)
    g = _as64(g)
    u = _as64(u)
    rev = tuple(slice(None, None, -1) for _ in range(u.ndim))
    ur = np.ascontiguousarray(u[rev])
    df = fft_conv(g, ur, workers=workers)[rev]
    dg = fft_conv(f, ur, workers=workers)[rev]
    return np.ascontiguousarray(df), np.ascontiguousarray(dg)


def relerr(h, ref) -> float:
    """Normwise relative error ||h - ref||_2 / ||ref||_2 in float64."""
    h = _as64(h)
    ref = _as64(ref)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((h - ref).ravel())
    if den == 0.0:
        return float(num)
    return float(num / den)
