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


def brute_conv_nary_exact(arrays):
    """The truncated convolution of n >= 2 arrays (Sec. 4.1: convolutions of more than
    two real arrays), written out literally with Python Fractions:

        h_j = sum over k^1 + ... + k^n = j of f^1_{k^1} f^2_{k^2} ... f^n_{k^n},  j < L

    (componentwise in d dimensions; every k^i is a multi-index with 0 <= k^i <= j).
    Exact for integer or dyadic inputs; tiny sizes only.  Returns an object array.
    """
    arrs = [np.asarray(a) for a in arrays]
    shape = arrs[0].shape
    if len(arrs) < 2 or any(a.shape != shape for a in arrs):
        raise ValueError("need n >= 2 arrays of one shape")
    vals = [{j: Fraction(float(a[j])) for j in itertools.product(*[range(n) for n in shape])} for a in arrs]
    H = np.empty(shape, dtype=object)
    for j in itertools.product(*[range(n) for n in shape]):
        acc = Fraction(0)
        # all (k^1, ..., k^{n-1}) with partial sums <= j; k^n is the remainder
        boxes = [itertools.product(*[range(jj + 1) for jj in j]) for _ in range(len(arrs) - 1)]
        for ks in itertools.product(*[list(b) for b in boxes]):
            rest = list(j)
            ok = True
            for k in ks:
                rest = [r - kk for r, kk in zip(rest, k)]
                if min(rest) < 0:
                    ok = False
                    break
            if not ok:
                continue
            term = vals[-1][tuple(rest)]
            for i, k in enumerate(ks):
                term *= vals[i][k]
            acc += term
        H[j] = acc
    return H


def direct_conv_nary(arrays) -> np.ndarray:
    """The same n-fold truncated convolution in float64 (any dimension), by direct sums.

    Every index of a term that reaches h_j with j < L is itself < L, so the
    n-fold sum equals nested binary truncated convolutions,
    h = trunc(f^1 * trunc(f^2 * ... trunc(f^{n-1} * f^n))), each evaluated with
    direct_conv.  O(n L^(2d)): small and mid sizes.
    """
    arrs = [_as64(a) for a in arrays]
    if len(arrs) < 2 or any(a.shape != arrs[0].shape for a in arrs):
        raise ValueError("need n >= 2 arrays of one shape")
    h = arrs[-1]
    for a in reversed(arrs[:-1]):
        h = direct_conv(a, h)
    return h


def fft_conv_nary(arrays, M=None, workers=1) -> np.ndarray:
    """The n-fold truncated convolution by explicit zero padding: every array padded to
    M_i >= n (L_i - 1) + 1 per axis (the length of the n-fold linear convolution, so no
    wrapped term reaches j < L; default M_i = n L_i), real FFTs, the product of all n
    spectra, inverse, truncate to L.  A library FFT is one step; nothing is fused.
    """
    import scipy.fft as sfft

    arrs = [_as64(a) for a in arrays]
    n = len(arrs)
    if n < 2 or any(a.shape != arrs[0].shape for a in arrs):
        raise ValueError("need n >= 2 arrays of one shape")
    L = arrs[0].shape
    if M is None:
        M = tuple(n * v for v in L)
    M = tuple(int(v) for v in np.atleast_1d(M))
    if any(m_ < n * (v - 1) + 1 for m_, v in zip(M, L)):
        raise ValueError("padding M must satisfy M >= n (L - 1) + 1 on every axis")
    axes = tuple(range(arrs[0].ndim))
    P = sfft.rfftn(arrs[0], s=M, axes=axes, workers=workers)
    for a in arrs[1:]:
        P = P * sfft.rfftn(a, s=M, axes=axes, workers=workers)
    h = sfft.irfftn(P, s=M, axes=axes, workers=workers)
    return np.ascontiguousarray(h[tuple(slice(0, v) for v in L)])


def relerr(h, ref) -> float:
    """Normwise relative error ||h - ref||_2 / ||ref||_2 in float64."""
    h = _as64(h)
    ref = _as64(ref)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((h - ref).ravel())
    if den == 0.0:
        return float(num)
    return float(num / den)
