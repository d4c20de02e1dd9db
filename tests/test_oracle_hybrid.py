"""Pins of the step-by-step oracle of the paper's algorithms (no GPU).

Each algorithm is pinned to the plain definition (direct summation, itself
pinned to exact brute force) and each intermediate to a closed form or an
invariant the paper states:
* residue transforms = subsequences of the explicitly padded DFT (Sec. 2);
* conjugate symmetries of residues (Sec. 3 eqs. (hrHerm), (realq2symmetry));
* eq. (RCM) = eq. (RCM-U) and the A, B, C symmetries of Appendix B;
* unpacking/packing identities (Sec. 4 eqs. (fourierUnpack), (fourierPack)).
"""
import numpy as np
import pytest

from oracle import direct_conv, relerr
from oracle import hybrid as hy
from paper_2608_14497_amd import synth


def padded_dft(x, N):
    """Closed form: DFT (paper sign) of x explicitly zero padded to N."""
    xp = np.zeros(N, dtype=np.complex128)
    xp[: len(x)] = x
    return N * np.fft.ifft(xp)


def rand_c(n, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(n) + 1j * r.standard_normal(n)


# ---------------------------------------------------------------- Sec. 2
@pytest.mark.parametrize("L,m,q", [(10, 4, 5), (16, 8, 2), (7, 7, 3), (33, 6, 12), (5, 16, 1)])
def test_residue_forward_is_padded_dft_subsequence(L, m, q):
    x = rand_c(L, L)
    F = padded_dft(x, q * m)
    for r in range(q):
        np.testing.assert_allclose(hy.residue_forward(x, m, q, r), F[r::q], atol=1e-12)
    np.testing.assert_allclose(hy.hybrid_forward(x, m, q), F, atol=1e-12)


@pytest.mark.parametrize("L,m,q", [(10, 4, 5), (33, 6, 12), (12, 12, 2)])
def test_hybrid_round_trip(L, m, q):
    x = rand_c(L, 100 + L)
    np.testing.assert_allclose(hy.hybrid_backward(hy.hybrid_forward(x, m, q), m, q, L), x, atol=1e-12)


def test_hybrid_axis_transform_matches_numpy_2d():
    x = rand_c(35, 5).reshape(5, 7)
    X = hy.hybrid_forward(x, m=4, q=3, axis=0)           # 5 -> 12 along axis 0
    xp = np.zeros((12, 7), dtype=np.complex128)
    xp[:5] = x
    np.testing.assert_allclose(X, 12 * np.fft.ifft(xp, axis=0), atol=1e-12)


def test_residue_backward_matches_eq_backwardr():
    # the accumulated inverse equals the plain inverse DFT of the full spectrum
    m, q, L = 6, 4, 11
    X = rand_c(q * m, 9)
    p = -(-L // m)
    acc = sum(hy.residue_backward(X[r::q], m, q, r, p) for r in range(q)) / (q * m)
    ref = np.fft.fft(X)[: p * m] / (q * m)   # sum_k zeta^{-jk} X_k / N (paper sign)
    np.testing.assert_allclose(acc, ref, atol=1e-12)


@pytest.mark.parametrize("m,q", [(8, 4), (6, 5)])
def test_real_residue_conjugate_symmetry(m, q):
    """eq. (hrHerm): conj h_r = h_{q-r} for real data."""
    f = np.random.default_rng(1).standard_normal(2 * m - 3)
    F = padded_dft(f, q * m)
    p = -(-len(f) // m)
    h = [hy.residue_backward(F[r::q], m, q, r, p) for r in range(q)]
    for r in range(1, q):
        np.testing.assert_allclose(np.conj(h[r]), h[q - r], atol=1e-11)


def test_q2_residue_closure_and_even_fold():
    """eq. (realq2symmetry) and eq. (forwardq2) against the padded DFT."""
    m, q, L = 8, 6, 20
    f = np.random.default_rng(2).standard_normal(L)
    F = padded_dft(f, q * m)
    Fq2 = F[q // 2::q]
    for l in range(m):
        assert abs(np.conj(Fq2[l]) - Fq2[m - 1 - l]) < 1e-11
    p = -(-L // m)
    fp = np.zeros(p * m)
    fp[:L] = f
    np.testing.assert_allclose(hy.cs_q2_forward(fp, m, p), Fq2[0::2], atol=1e-11)
    # eqs. (wb),(accumulateq2): h_{q/2} from the even half equals the full residue contribution
    full = hy.residue_backward(Fq2, m, q, q // 2, p)
    np.testing.assert_allclose(hy.cs_q2_backward(Fq2[0::2], m, p), full.real, atol=1e-10)
    assert np.max(np.abs(full.imag)) < 1e-10


# ---------------------------------------------------------------- Sec. 4
@pytest.mark.parametrize("L", [8, 9, 1, 2])
def test_complex_pack_roundtrip(L):
    f = np.arange(L, dtype=np.float64) + 1
    ft = hy.complex_pack(f)
    assert ft.shape == ((L + 1) // 2,)
    assert ft[0] == 1 + 2j or L == 1
    np.testing.assert_array_equal(hy.complex_unpack(ft, L), f)


@pytest.mark.parametrize("N", [8, 7, 16])
def test_fourier_unpack_gives_real_dft(N):
    f = np.random.default_rng(N).standard_normal(2 * N)
    Ft = hy.dft(hy.complex_pack(f))
    F = hy.fourier_unpack(Ft)
    Fref = hy.dft(f.astype(np.complex128))[: N + 1]
    np.testing.assert_allclose(F, Fref, atol=1e-11)
    np.testing.assert_allclose(hy.fourier_pack(F), Ft, atol=1e-11)


def test_fourier_unpack_2d():
    f = np.random.default_rng(4).standard_normal((6, 10))
    Ft = np.fft.ifft2(hy.complex_pack(f)) * 30
    F = hy.fourier_unpack(Ft)
    Fref = (np.fft.ifft2(f) * 60)[:, :6]
    np.testing.assert_allclose(F, Fref, atol=1e-11)
    np.testing.assert_allclose(hy.fourier_pack(F), Ft, atol=1e-11)


@pytest.mark.parametrize("shape", [(8,), (9,), (6, 8), (4, 6, 5)])
def test_rcm_equals_unpack_multiply_pack(shape):
    """eq. (RCM) = eq. (RCM-U) (derived in Appendix B) on random complex arrays."""
    r = np.random.default_rng(sum(shape))
    Ft = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    Gt = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    np.testing.assert_allclose(hy.rcm(Ft, Gt), hy.rcm_via_unpack(Ft, Gt), atol=1e-11)


def test_appendix_b_symmetries():
    N = 10
    Ft = rand_c(N, 1)
    Gt = rand_c(N, 2)
    k = np.arange(N)
    Fc = np.conj(Ft[(N - k) % N])
    Gc = np.conj(Gt[(N - k) % N])
    A = Ft * Gt + Fc * Gt + Ft * Gc + Fc * Gc
    B = Ft * Gt - Fc * Gc
    C = Ft * Gt - Fc * Gt - Ft * Gc + Fc * Gc
    rev = (N - k) % N
    np.testing.assert_allclose(A, np.conj(A[rev]), atol=1e-12)
    np.testing.assert_allclose(B, -np.conj(B[rev]), atol=1e-12)
    np.testing.assert_allclose(C, np.conj(C[rev]), atol=1e-12)


@pytest.mark.parametrize("m,q", [(4, 4), (5, 3), (8, 2), (3, 6)])
def test_rcm_residue_pairs(m, q):
    Ft = rand_c(q * m, 11)
    Gt = rand_c(q * m, 12)
    H = hy.rcm(Ft, Gt)
    Hp = hy.rcm_residue_pairs(Ft.reshape(m, q).T.copy(), Gt.reshape(m, q).T.copy())
    np.testing.assert_allclose(Hp.T.reshape(-1), H, atol=1e-12)
    # conj W_{l,r} = W_{m-l-1, q-r} for r not in {0, q/2}
    Fr = Ft.reshape(m, q).T
    Gr = Gt.reshape(m, q).T

    def W(l, r):
        r2 = (q - r) % q
        l2 = (m - l - (1 if r else 0)) % m
        return 0.25 * (Fr[r, l] - np.conj(Fr[r2, l2])) * (Gr[r, l] - np.conj(Gr[r2, l2])) \
            * (1 + hy.zeta(q * m, q * l + r))
    for r in range(1, q):
        if 2 * r == q:
            continue
        for l in range(m):
            assert abs(np.conj(W(l, r)) - W(m - l - 1, q - r)) < 1e-12


def test_rcm_nary_is_packed_triple_convolution():
    N = 8
    fs = [np.random.default_rng(s).standard_normal(2 * N) for s in range(3)]
    Fts = [hy.dft(hy.complex_pack(f)) for f in fs]
    R = hy.rcm_nary(Fts)
    Fr = [hy.dft(f.astype(np.complex128)) for f in fs]
    circ = np.fft.fft(Fr[0] * Fr[1] * Fr[2]).real / (2 * N)       # circular triple conv, length 2N
    np.testing.assert_allclose(R, hy.dft(hy.complex_pack(circ)), atol=1e-9)


# ------------------------------------------------- whole algorithms vs definition
CASES_1D_PACKED = [  # (L, m~, q~) on the packed axis; 2 q m >= 2L - 1
    (1024, 256, 4), (1024, 512, 2), (1024, 64, 16), (37, 4, 10), (33, 3, 11), (40, 8, 5),
    (64, 32, 2), (50, 5, 10), (1, 1, 1), (2, 1, 2), (3, 2, 2), (17, 17, 1), (100, 7, 15),
]


@pytest.mark.parametrize("L,m,q", CASES_1D_PACKED)
def test_hybrid_rcm_1d(L, m, q):
    f, g = synth.pair_for(20, L, (L,), np.float64)
    ref = direct_conv(f, g)
    assert relerr(hy.hybrid_rcm_conv(f, g, (m,), (q,)), ref) < 1e-13
    assert relerr(hy.hybrid_rcm_conv_1d_residues(f, g, m, q), ref) < 1e-13


def test_hybrid_rcm_1d_exact_integers():
    f, g = synth.pair_for(21, 0, (301,), np.float64, "ints")
    h = hy.hybrid_rcm_conv(f, g, (64,), (5,))
    assert np.array_equal(np.rint(h), direct_conv(f, g))
    assert np.max(np.abs(h - np.rint(h))) < 1e-9


@pytest.mark.parametrize("shape,m,q", [
    ((8, 8), (8, 4), (2, 2)), ((9, 7), (6, 2), (3, 4)), ((5, 12), (3, 6), (4, 2)),
    ((16, 10), (16, 5), (2, 2)), ((4, 5, 6), (4, 5, 3), (2, 2, 2)), ((3, 4, 7), (2, 3, 2), (3, 3, 4)),
])
def test_hybrid_rcm_nd(shape, m, q):
    f, g = synth.pair_for(22, 0, shape, np.float64)
    assert relerr(hy.hybrid_rcm_conv(f, g, m, q), direct_conv(f, g)) < 1e-13


def test_hybrid_rcm_rejects_aliasing():
    with pytest.raises(ValueError):
        hy.hybrid_rcm_conv(np.ones(8), np.ones(8), (3,), (2,))


@pytest.mark.parametrize("L,M", [(16, 32), (15, 32), (9, 20), (10, 24)])
def test_explicit_rcm_1d(L, M):
    f, g = synth.pair_for(23, L, (L,), np.float64)
    assert relerr(hy.explicit_rcm_conv_1d(f, g, M), direct_conv(f, g)) < 1e-13


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (7, 6)])
def test_explicit_rcm_2d(shape):
    f, g = synth.pair_for(24, 0, shape, np.float64)
    M = tuple(2 * n for n in shape)
    assert relerr(hy.explicit_rcm_conv_2d(f, g, M), direct_conv(f, g)) < 1e-13


CASES_CS = [(1024, 512, 4), (37, 8, 10), (40, 16, 5), (33, 6, 12), (64, 64, 2), (50, 10, 11),
            (1, 1, 1), (1, 2, 2), (9, 4, 6), (31, 32, 2), (20, 20, 2)]


@pytest.mark.parametrize("L,m,q", CASES_CS)
def test_hybrid_cs_1d(L, m, q):
    f, g = synth.pair_for(25, L, (L,), np.float64)
    assert relerr(hy.hybrid_cs_conv_1d(f, g, m, q), direct_conv(f, g)) < 1e-13


def test_hybrid_cs_rejects_odd_m_with_even_q():
    with pytest.raises(ValueError):
        hy.hybrid_cs_conv_1d(np.ones(8), np.ones(8), 5, 4)


@pytest.mark.parametrize("L,m,n", [(64, 8, 2), (60, 8, 2), (64, 4, 3), (100, 10, 4), (30, 6, 2),
                                   (96, 8, 5), (40, 8, 2), (21, 4, 6)])
def test_hybrid_cs_1d_inner_loop(L, m, n):
    f, g = synth.pair_for(26, L, (L,), np.float64)
    assert relerr(hy.hybrid_cs_conv_1d_inner(f, g, m, n), direct_conv(f, g)) < 1e-13


@pytest.mark.parametrize("shape,m,q", [
    ((8, 8), (8, 8), (2, 2)), ((9, 7), (4, 7), (5, 2)), ((6, 10), (6, 4), (2, 5)),
    ((4, 5, 6), (4, 5, 6), (2, 2, 2)), ((5, 3, 4), (2, 3, 4), (6, 2, 2)),
])
def test_hybrid_cs_nd(shape, m, q):
    f, g = synth.pair_for(27, 0, shape, np.float64)
    assert relerr(hy.hybrid_cs_conv(f, g, m, q), direct_conv(f, g)) < 1e-13


@pytest.mark.parametrize("shape,m,q", [((7,), (4,), (4,)), ((5, 6), (3, 4), (4, 3)), ((3, 4, 2), (2, 4, 2), (3, 2, 2))])
def test_complex_hybrid_conv(shape, m, q):
    r = np.random.default_rng(3)
    a = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    ref = direct_conv(a.real, b.real) - direct_conv(a.imag, b.imag) + \
        1j * (direct_conv(a.real, b.imag) + direct_conv(a.imag, b.real))
    h = hy.complex_hybrid_conv(a, b, m, q)
    assert np.linalg.norm(h - ref) / np.linalg.norm(ref) < 1e-13


# ------------------------------------------------------------------ CS residues with packed 0 and q/2
def _cyclic(a, b):
    m = len(a)
    return np.array([sum(a[k] * b[(s - k) % m] for k in range(m)) for s in range(m)])


def _negacyclic(a, b):
    m = len(a)
    return np.array([sum(a[k] * b[s - k] if k <= s else -a[k] * b[m + s - k] for k in range(m)) for s in range(m)])


@pytest.mark.parametrize("m", [2, 4, 8, 12, 16])
def test_packed_product_is_the_packed_cyclic_and_negacyclic_convolution(m):
    """Brute-force cyclic / negacyclic convolutions of real sequences, packed and transformed, equal the packed
    product of the packed transforms (twist 0: eq. (RCM) at length m/2; twist 1: its half-shifted form)."""
    rng = np.random.default_rng(m)
    a, b = rng.standard_normal(m), rng.standard_normal(m)
    for twist, conv in ((False, _cyclic), (True, _negacyclic)):
        want = hy.packed_forward(conv(a, b), twist)
        got = hy.packed_product(hy.packed_forward(a, twist), hy.packed_forward(b, twist), twist)
        assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("m", [2, 6, 16])
def test_packed_transform_round_trip_and_odd_frequencies(m):
    rng = np.random.default_rng(100 + m)
    a = rng.standard_normal(m)
    for twist in (False, True):
        assert np.allclose(hy.packed_backward(hy.packed_forward(a, twist), twist), (m // 2) * a, atol=1e-12)
    # the odd-frequency transform of residue q/2 from the packed twisted transform (even and odd samples)
    P = hy.packed_forward(a, True)
    e = m // 2
    l = np.arange(e)
    Pc = np.conj(P[e - 1 - l])
    E, O = (P + Pc) / 2, (P - Pc) / 2j
    A = np.array([sum(a[s] * np.exp(2j * np.pi * s * (2 * k + 1) / (2 * m)) for s in range(m)) for k in range(m)])
    z = np.exp(2j * np.pi * (2 * l + 1) / (2 * m))
    assert np.allclose(A[:e], E + z * O, atol=1e-12) and np.allclose(A[e:], E - z * O, atol=1e-12)


@pytest.mark.parametrize("L,m,q", [(1024, 512, 4), (37, 8, 10), (40, 16, 5), (33, 6, 12), (64, 64, 2), (50, 10, 11),
                                   (100, 20, 10), (16, 2, 16), (999, 256, 8), (1, 2, 2)])
def test_hybrid_mix_matches_direct(L, m, q):
    f, g = synth.pair_for(60, L, (L,), np.float64, "normal")
    assert relerr(hy.hybrid_mix_conv_1d(f, g, m, q), direct_conv(f, g)) < 1e-13


def test_hybrid_mix_exact_integers():
    f, g = synth.pair_for(61, 0, (64,), np.float64, "ints")
    h = hy.hybrid_mix_conv_1d(f, g, 16, 8)
    assert np.array_equal(np.rint(h), direct_conv(f, g))


@pytest.mark.parametrize("shape,m,q", [
    ((20, 30), (8, 16), (5, 4)),       # odd q0: residue 0 packed, 1 and 2 conjugate-symmetric
    ((16, 12), (4, 8), (8, 3)),        # even q0 = 8: 0 and 4 packed, 1..3 conjugate-symmetric
    ((9, 10), (4, 4), (5, 5)),
    ((9, 10), (16, 32), (2, 1)),       # q0 = 2: packed residues only
    ((9, 10), (32, 32), (1, 1)),       # q0 = 1: residue 0 only
    ((6, 5, 7), (2, 4, 4), (6, 3, 4)),  # 3D
    ((5, 4, 6), (4, 8, 4), (3, 1, 3)),
])
def test_hybrid_mix_nd_matches_direct(shape, m, q):
    f, g = synth.pair_for(62, 0, shape, np.float64, "normal")
    assert relerr(hy.hybrid_mix_conv_nd(f, g, m, q), direct_conv(f, g)) < 1e-13


def test_hybrid_mix_nd_exact_integers():
    f, g = synth.pair_for(63, 0, (12, 10), np.float64, "ints")
    assert np.array_equal(np.rint(hy.hybrid_mix_conv_nd(f, g, (4, 8), (6, 3))), direct_conv(f, g))


@pytest.mark.parametrize("q", [2, 4, 6, 10])
def test_packed_residues_are_the_q2_residues(q):
    """Residues 0 and q/2 of an axis are residues 0 and 1 of the same axis with q = 2 (zeta_q^{(q/2) t} =
    (-1)^t, zeta_{qm}^{(q/2) s} = zeta_{2m}^s), forward (eq. (forwardr)) and backward (eq. (accumulator)); with
    the inverse's 1/(q m) against 1/(2 m), their contribution is 2/q times that of the q = 2 problem (the
    sub-plan of the mixed variant in 2D/3D).  p <= 2 so that both q are defined."""
    m = 8
    x = synth.normal((2 * m - 3, 5), 64, q, synth.ROLE_F, np.float64)
    for r, r2 in ((0, 0), (q // 2, 1)):
        Fq = hy.residue_forward(x, m, q, r)
        assert np.allclose(Fq, hy.residue_forward(x, m, 2, r2), rtol=0, atol=1e-12)
        assert np.allclose(hy.residue_backward(Fq, m, q, r, 2), hy.residue_backward(Fq, m, 2, r2, 2), rtol=0, atol=1e-12)
    # a middle residue is not one of them
    if q > 2:
        assert not np.allclose(hy.residue_forward(x, m, q, 1), hy.residue_forward(x, m, 2, 1))
