"""Accuracy of the roots of unity the kernels use (host only: hdc_twiddle_values).

Every twiddle zeta_N^k = exp(2 pi i k / N) (Sec. 2; the residue twiddles of eqs.
(forwardr) and (accumulator), the FFT stage roots, the RCM factor) comes from
tables whose entries are computed in extended precision and rounded once.  Up
to 4096 points a lookup returns an entry; above, it multiplies two entries in
the working precision.  The error is measured per component in units of
u = 2^-24 (FP32) / 2^-53 (FP64), the spacing of the numbers in [0.5, 1):

* exhaustively against numpy's long double cos/sin (64-bit significand, so the
  reference error is below 2^-11 u in FP64), and
* on a sample of k against mpmath at 40 digits, which shares no code with the
  C library's cosl/sinl.

Bounds asserted: single-level entries are correctly rounded (<= 0.5 u; an
entry whose exact value lies in a lower binade is rounded more finely); the
two-level product stays within 2.5 u (each factor <= 0.5 u, plus the rounding
of the product and of the fused sum).
"""
import math

import numpy as np
import pytest

import paper_2608_14497_amd as hd

UNIT = {"float32": 2.0 ** -24, "float64": 2.0 ** -53}

# powers of two up to 2^22 (the RCM factor of a 2^20-point problem runs at 2 q m = 2^22) and lengths q m with
# q not a power of two, as the planner makes them
LENGTHS = [2 ** e for e in range(0, 23)] + [3 * 512, 5 * 1024, 13 * 16, 7 * 2048, 3 * 2 ** 13, 6 * 2 ** 16,
                                            3 * 2 ** 20, 10 * 2 ** 12]
SINGLE_MAX = 4096


def _exact_ld(N):
    k = np.arange(N, dtype=np.longdouble)
    # the argument's own rounding (relative 2^-64) is far below the FP64 unit
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    a = two_pi * k / np.longdouble(N)
    return np.cos(a), np.sin(a)


def _err_units(w, N, dtype):
    c, s = _exact_ld(N)
    er = np.abs(np.asarray(w.real, dtype=np.longdouble) - c)
    ei = np.abs(np.asarray(w.imag, dtype=np.longdouble) - s)
    return float(np.max(np.maximum(er, ei)) / np.longdouble(UNIT[dtype]))


@pytest.fixture(scope="module")
def lib():
    return hd.load()


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("N", LENGTHS)
def test_twiddle_error_exhaustive(lib, N, dtype):
    w = hd.twiddle_values(N, dtype)
    assert w.shape == (N,)
    err = _err_units(w, N, dtype)
    # the long double reference is exact to 2^-11 u in FP64
    bound = (0.5 + (1e-3 if dtype == "float64" else 0.0)) if N <= SINGLE_MAX else 2.5
    print(f"N={N} {dtype}: max error {err:.3f} u (bound {bound} u)")
    assert err <= bound, f"N={N} {dtype}: {err:.3f} u"
    # exact values at multiples of N/4 (the octant reduction is exact)
    if N % 4 == 0:
        q = N // 4
        assert w[0] == 1 and w[q] == 1j and w[2 * q] == -1 and w[3 * q] == -1j


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("N", [4096, 8192, 3 * 2 ** 13, 2 ** 20, 2 ** 22])
def test_twiddle_error_mpmath_sample(lib, N, dtype):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    rng = np.random.default_rng(N)
    ks = np.unique(np.concatenate([rng.integers(0, N, 300), [1, N // 8 + 1, N - 1, N // 3]]))
    w = hd.twiddle_values(N, dtype)
    worst = 0.0
    for k in ks:
        a = 2 * mpmath.pi * int(k) / N
        c, s = mpmath.cos(a), mpmath.sin(a)
        worst = max(worst, float(abs(mpmath.mpf(float(w[k].real)) - c)), float(abs(mpmath.mpf(float(w[k].imag)) - s)))
    worst /= UNIT[dtype]
    bound = 0.5 + 1e-9 if N <= SINGLE_MAX else 2.5
    print(f"N={N} {dtype}: sampled max error {worst:.3f} u against mpmath")
    assert worst <= bound


def test_twiddle_values_errors(lib):
    with pytest.raises(hd.HdcError):
        hd.twiddle_values(0)
    with pytest.raises(hd.HdcError):
        hd.twiddle_values(16, k0=10, count=7)
    with pytest.raises(KeyError):
        hd.twiddle_values(16, dtype="float16")
    assert math.isclose(hd.twiddle_values(16, "float64", 4, 1)[0].imag, 1.0)
