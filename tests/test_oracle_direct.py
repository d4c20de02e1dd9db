"""Pins of the plain-definition oracle (no GPU).

The truncated convolution h_j = sum_{k<=j} f_k g_{j-k} (j < L) is checked
against exact rational brute force, a library routine for the 1D special
case (numpy.convolve), impulses, commutativity and bilinearity; the padded
FFT reference and the adjoint are checked against those.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import (brute_conv_exact, brute_conv_nary_exact, direct_conv, direct_conv_at, direct_conv_nary, fft_conv,
                    fft_conv_nary, fft_grad,
                    grad_direct, grad_direct_at, relerr)
from paper_2608_14497_amd import synth


def _ints(shape, seed):
    return np.random.default_rng(seed).integers(-3, 4, size=shape).astype(np.float64)


@pytest.mark.parametrize("shape", [(1,), (2,), (7,), (12,), (3, 4), (5, 5), (2, 3, 4), (3, 3, 3)])
def test_direct_equals_exact_brute_force(shape):
    f = _ints(shape, 1)
    g = _ints(shape, 2)
    H = brute_conv_exact(f, g)
    h = direct_conv(f, g)
    for idx in np.ndindex(*shape):
        assert Fraction(h[idx]) == H[idx]


def test_direct_dyadic_exact():
    # dyadic rationals with short mantissas: float64 sums are exact
    rng = np.random.default_rng(3)
    f = rng.integers(-64, 65, size=9) / 16.0
    g = rng.integers(-64, 65, size=9) / 32.0
    H = brute_conv_exact(f, g)
    h = direct_conv(f, g)
    assert all(Fraction(h[i]) == H[i] for i in range(9))


def test_direct_1d_matches_numpy_convolve():
    f, g = synth.pair_for(1, 0, (1024,), np.float64)
    h = direct_conv(f, g)
    ref = np.convolve(f, g)[:1024]
    assert relerr(h, ref) < 1e-14


@pytest.mark.parametrize("shape", [(9,), (4, 6), (3, 4, 5)])
def test_impulses(shape):
    f = synth.uniform(shape, 99, 0, 0)
    d0 = np.zeros(shape)
    d0[(0,) * len(shape)] = 1.0
    assert np.array_equal(direct_conv(f, d0), f)
    # shifted impulse: h_j = f_{j - s} for j >= s componentwise, else 0
    s = tuple(min(2, n - 1) for n in shape)
    ds = np.zeros(shape)
    ds[s] = 1.0
    h = direct_conv(f, ds)
    ref = np.zeros(shape)
    dst = tuple(slice(ss, None) for ss in s)
    src = tuple(slice(0, n - ss) for n, ss in zip(shape, s))
    ref[dst] = f[src]
    assert np.array_equal(h, ref)


def test_commutative_and_bilinear_exact():
    f = _ints((11, 6), 4)
    g = _ints((11, 6), 5)
    a = _ints((11, 6), 6)
    assert np.array_equal(direct_conv(f, g), direct_conv(g, f))
    assert np.array_equal(direct_conv(f + 2 * a, g), direct_conv(f, g) + 2 * direct_conv(a, g))


@pytest.mark.parametrize("shape,M", [((300,), None), ((301,), (601,)), ((20, 17), None),
                                     ((13, 9), (25, 20)), ((6, 5, 7), None)])
def test_fft_conv_matches_direct(shape, M):
    f, g = synth.pair_for(7, 0, shape, np.float64, "normal")
    assert relerr(fft_conv(f, g, M=M), direct_conv(f, g)) < 1e-13


def test_fft_conv_rejects_aliasing_padding():
    with pytest.raises(ValueError):
        fft_conv(np.ones(8), np.ones(8), M=(14,))


def test_direct_conv_at_matches_full():
    f, g = synth.pair_for(8, 0, (9, 10), np.float64)
    h = direct_conv(f, g)
    idx = [(0, 0), (8, 9), (3, 7), (8, 0)]
    np.testing.assert_array_equal(direct_conv_at(f, g, idx), np.array([h[i] for i in idx]))


@pytest.mark.parametrize("shape", [(10,), (5, 4), (3, 4, 2)])
def test_gradient_is_exact_adjoint(shape):
    """<u, conv(a, g)> = <df, a> and <u, conv(f, b)> = <dg, b>, exactly on integers."""
    f = _ints(shape, 10)
    g = _ints(shape, 11)
    u = _ints(shape, 12)
    df, dg = grad_direct(f, g, u)
    for seed in range(3):
        a = _ints(shape, 20 + seed)
        assert np.sum(u * direct_conv(a, g)) == np.sum(df * a)
        assert np.sum(u * direct_conv(f, a)) == np.sum(dg * a)


def test_gradient_finite_difference():
    """h is bilinear, so a finite difference is exact up to rounding."""
    f, g = synth.pair_for(11, 0, (17,), np.float64)
    u = synth.uniform((17,), 11, 0, 2)
    df, dg = grad_direct(f, g, u)
    eps = 1e-3
    for k in (0, 5, 16):
        e = np.zeros(17)
        e[k] = eps
        fd = (np.sum(u * direct_conv(f + e, g)) - np.sum(u * direct_conv(f - e, g))) / (2 * eps)
        assert abs(fd - df[k]) < 1e-12
        fd = (np.sum(u * direct_conv(f, g + e)) - np.sum(u * direct_conv(f, g - e))) / (2 * eps)
        assert abs(fd - dg[k]) < 1e-12


@pytest.mark.parametrize("shape", [(64,), (9, 7), (4, 5, 6)])
def test_fft_grad_matches_direct(shape):
    f, g = synth.pair_for(12, 0, shape, np.float64, "normal")
    u = synth.normal(shape, 12, 0, 2)
    df, dg = grad_direct(f, g, u)
    df2, dg2 = fft_grad(f, g, u)
    assert relerr(df2, df) < 1e-13 and relerr(dg2, dg) < 1e-13
    idx = [tuple(0 for _ in shape), tuple(n - 1 for n in shape)]
    a, b = grad_direct_at(f, g, u, idx)
    np.testing.assert_allclose(a, [df[i] for i in idx], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b, [dg[i] for i in idx], rtol=0, atol=1e-12)


def test_relerr():
    assert relerr(np.array([1.0, 0.0]), np.array([1.0, 0.0])) == 0.0
    assert abs(relerr(np.array([3.0, 5.0]), np.array([0.0, 5.0])) - 0.6) < 1e-15


GOLDEN = ["int_1d_L37", "int_1d_L64", "int_2d_9x12", "int_3d_5x4x6"]


@pytest.mark.parametrize("name", GOLDEN)
def test_golden_exact(name):
    """Stored exact integers (tests/golden, written from exact brute force) = direct sums."""
    from tests.golden.make_golden import load

    f, g, h = load(name)
    assert np.array_equal(direct_conv(f, g), h)


# ---- a kernel shorter than f (the unequal-length convolution of Sec. 7)
@pytest.mark.parametrize("L,Lg", [(1024, 1), (1024, 37), (1000, 999), (7, 3)])
def test_short_kernel_1d_matches_numpy_convolve(L, Lg):
    f = synth.normal((L,), 21, 0, synth.ROLE_F, np.float64)
    g = synth.normal((Lg,), 21, 0, synth.ROLE_G, np.float64)
    ref = np.convolve(f, g)[:L]  # library routine: the full linear convolution, truncated to L
    assert relerr(direct_conv(f, g), ref) < 1e-14
    assert relerr(fft_conv(f, g), ref) < 1e-13  # default M = L + Lg
    assert relerr(fft_conv(f, g, M=(L + Lg - 1,)), ref) < 1e-13
    idx = [0, Lg - 1, L - 1, L // 2]
    assert relerr(direct_conv_at(f, g, idx), ref[idx]) < 1e-14


@pytest.mark.parametrize("shape,kshape", [((12, 9), (3, 4)), ((8, 8), (8, 1)), ((5, 6, 7), (2, 3, 1))])
def test_short_kernel_nd_matches_scipy_and_brute_force(shape, kshape):
    import scipy.signal

    f = _ints(shape, 22)
    g = _ints(kshape, 23)
    ref = scipy.signal.convolve(f, g, method="direct")[tuple(slice(0, n) for n in shape)]
    h = direct_conv(f, g)
    assert np.array_equal(h, ref)  # small integers: both sums are exact
    H = brute_conv_exact(f, g)
    assert all(Fraction(h[i]) == H[i] for i in np.ndindex(*shape))
    assert relerr(fft_conv(f, g), ref) < 1e-13


def test_short_kernel_padding_bound():
    # M >= L + Lg - 1 is needed; at M = L + Lg - 2 the product f_{L-1} g_{Lg-1} wraps onto h_0
    with pytest.raises(ValueError):
        fft_conv(np.ones(10), np.ones(4), M=(12,))
    with pytest.raises(ValueError):
        direct_conv(np.ones(4), np.ones(5))  # a kernel longer than f


# ------------------------------------------------------------------ n >= 2 arrays (Sec. 4.1)
@pytest.mark.parametrize("shape,n", [((1,), 3), ((6,), 3), ((9,), 4), ((3, 4), 3), ((3, 3), 4), ((2, 3, 3), 3)])
def test_nary_direct_equals_exact_brute_force(shape, n):
    """The nested binary form equals the literal n-fold sum exactly on small integers."""
    arrs = [_ints(shape, 30 + i) for i in range(n)]
    H = brute_conv_nary_exact(arrs)
    h = direct_conv_nary(arrs)
    for idx in np.ndindex(*shape):
        assert Fraction(h[idx]) == H[idx], idx


@pytest.mark.parametrize("n", [2, 3, 5])
def test_nary_1d_matches_numpy_convolve(n):
    L = 57
    arrs = [synth.normal((L,), 31, i, synth.ROLE_F, np.float64) for i in range(n)]
    ref = arrs[0]
    for a in arrs[1:]:
        ref = np.convolve(ref, a)  # the full linear convolutions, chained by the library routine
    ref = ref[:L]
    assert relerr(direct_conv_nary(arrs), ref) < 1e-13
    assert relerr(fft_conv_nary(arrs), ref) < 1e-12
    if n == 2:
        assert np.array_equal(direct_conv_nary(arrs), direct_conv(arrs[0], arrs[1]))


@pytest.mark.parametrize("shape", [(9, 7), (4, 5, 6)])
def test_nary_nd_matches_scipy(shape):
    import scipy.signal

    arrs = [_ints(shape, 40 + i) for i in range(3)]
    ref = scipy.signal.convolve(scipy.signal.convolve(arrs[0], arrs[1], method="direct"), arrs[2], method="direct")
    ref = ref[tuple(slice(0, v) for v in shape)]
    assert np.array_equal(direct_conv_nary(arrs), ref)  # small integers: exact
    assert relerr(fft_conv_nary(arrs), ref) < 1e-13


def test_nary_padding_bound():
    """M >= n (L - 1) + 1: at M = n (L - 1) the product of the last entries wraps onto h_0."""
    L, n = 6, 3
    arrs = [np.ones(L) for _ in range(n)]
    with pytest.raises(ValueError):
        fft_conv_nary(arrs, M=(n * (L - 1),))
    import scipy.fft as sfft

    P = np.ones(n * (L - 1) // 2 + 1, dtype=complex)
    for a in arrs:
        P = P * sfft.rfft(a, n * (L - 1))
    wrapped = sfft.irfft(P, n * (L - 1))
    assert abs(wrapped[0] - 1.0) > 0.5  # h_0 = 1 exactly, the wrapped term adds f_5 g_5 k_5 = 1
    assert abs(fft_conv_nary(arrs, M=(n * (L - 1) + 1,))[0] - 1.0) < 1e-12
