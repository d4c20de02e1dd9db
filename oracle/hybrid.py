"""The paper's hybrid-dealiasing algorithms, step by step, in float64.

Test infrastructure only (see the package docstring).  Each function follows
the cited section/equation of Murasko & Bowman, "Hybrid Dealiasing and
Implicit Packing for Real Convolutions", in the paper's notation:

* zeta_N = exp(+2 pi i / N); the forward DFT is F_k = sum_j zeta_N^{kj} f_j and
  the inverse carries zeta^{-} and 1/N (Sec. 2);
* j = t m + s (t < p, s < m), k = q l + r (l < m, r < q), p = ceil(L/m),
  q = ceil(M/m) (Sec. 2);
* e = floor(m/2) (Sec. 3.1.3); r = u n + v with q = n p (Appendix A);
* complex packing f~_j = f_{2j} + i f_{2j+1} (Sec. 4, eq. (complexPacking)).

A library FFT serves as the length-m (or length-p) DFT step; the pre- and
post-processing sums, twiddles, residue loops and multiplication operators
are written out as the paper states them.  None of this is optimised.
"""
from __future__ import annotations

from math import ceil

import numpy as np


# ---------------------------------------------------------------------------
# notation helpers (Sec. 2)
# ---------------------------------------------------------------------------

def zeta(N: int, k) -> np.ndarray:
    """zeta_N^k = exp(2 pi i k / N), with k reduced mod N in exact integers."""
    k = np.mod(np.asarray(k, dtype=np.int64), int(N))
    return np.exp(2j * np.pi * k.astype(np.float64) / float(N))


def dft(x: np.ndarray, axis: int = 0) -> np.ndarray:
    """X_l = sum_s zeta_n^{l s} x_s along ``axis`` (the paper's + sign)."""
    n = x.shape[axis]
    return n * np.fft.ifft(x, axis=axis)


def idft_unnormalized(X: np.ndarray, axis: int = 0) -> np.ndarray:
    """x_s = sum_l zeta_n^{-s l} X_l along ``axis`` (no 1/n)."""
    return np.fft.fft(X, axis=axis)


def _bshape(vec: np.ndarray, ndim: int, axis: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = vec.shape[0]
    return vec.reshape(shape)


# ---------------------------------------------------------------------------
# complex hybrid dealiasing one residue at a time (Sec. 2, 2.1)
# ---------------------------------------------------------------------------

def residue_forward(x: np.ndarray, m: int, q: int, r: int, axis: int = 0) -> np.ndarray:
    """Residue contribution F_r = {F_{q l + r}}_{l<m}, eq. (forwardr).

    x is zero padded explicitly to length p m along ``axis`` (p = ceil(L/m));
    the padding from p m to q m is implicit: pre-process
    y_s = zeta_{qm}^{r s} sum_{t<p} zeta_q^{r t} x_{t m + s}, then a length-m DFT.
    """
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, 0)
    L = x.shape[0]
    p = ceil(L / m)
    if p > q:
        raise ValueError("need p <= q")
    xp = np.zeros((p * m,) + x.shape[1:], dtype=np.complex128)
    xp[:L] = x
    xr = xp.reshape((p, m) + x.shape[1:])
    t = np.arange(p)
    s = np.arange(m)
    y = np.tensordot(zeta(q, r * t), xr, axes=(0, 0))
    y = y * _bshape(zeta(q * m, r * s), y.ndim, 0)
    F = dft(y, axis=0)
    return np.moveaxis(F, 0, axis)


def residue_backward(Fr: np.ndarray, m: int, q: int, r: int, p: int, axis: int = 0) -> np.ndarray:
    """h_r = {h_{r, t m + s}}, eq. (accumulator), length p m along ``axis``.

    h_{r, t m + s} = zeta_q^{-t r} zeta_{qm}^{-s r} sum_l zeta_m^{-s l} F_{q l + r}.
    """
    Fr = np.moveaxis(np.asarray(Fr, dtype=np.complex128), axis, 0)
    s = np.arange(m)
    w = idft_unnormalized(Fr, axis=0) * _bshape(zeta(q * m, -r * s), Fr.ndim, 0)
    h = np.concatenate([zeta(q, -t * r) * w for t in range(p)], axis=0)
    return np.moveaxis(h, 0, axis)


def hybrid_forward(x: np.ndarray, m: int, q: int, axis: int = 0) -> np.ndarray:
    """Implicitly padded DFT of length q m along ``axis``, natural order k = q l + r.

    Assembled residue by residue from residue_forward (Sec. 2.1).
    """
    x = np.asarray(x, dtype=np.complex128)
    shape = list(x.shape)
    shape[axis] = q * m
    out = np.empty(shape, dtype=np.complex128)
    for r in range(q):
        sl = [slice(None)] * x.ndim
        sl[axis] = slice(r, q * m, q)
        out[tuple(sl)] = residue_forward(x, m, q, r, axis=axis)
    return out


def hybrid_backward(X: np.ndarray, m: int, q: int, L: int, axis: int = 0) -> np.ndarray:
    """Inverse of hybrid_forward truncated to L, eqs. (accumulator), (accumulation).

    f = (1/(qm)) sum_r h_r, keeping j < L.
    """
    X = np.asarray(X, dtype=np.complex128)
    p = ceil(L / m)
    acc = None
    for r in range(q):
        sl = [slice(None)] * X.ndim
        sl[axis] = slice(r, q * m, q)
        hr = residue_backward(X[tuple(sl)], m, q, r, p, axis=axis)
        acc = hr if acc is None else acc + hr
    acc = acc / float(q * m)
    sl = [slice(None)] * X.ndim
    sl[axis] = slice(0, L)
    return acc[tuple(sl)]


def complex_hybrid_conv(a: np.ndarray, b: np.ndarray, m, q) -> np.ndarray:
    """Complex hybrid-dealiased linear convolution (Sec. 2) over every axis.

    Implicitly padded transforms per axis, elementwise product, inverse with
    accumulation over residues, truncated to the input extents.
    """
    A = np.asarray(a, dtype=np.complex128)
    B = np.asarray(b, dtype=np.complex128)
    L = A.shape
    for ax in range(A.ndim):
        if q[ax] * m[ax] < 2 * L[ax] - 1:
            raise ValueError("q m must be >= 2L-1 on every axis")
        A = hybrid_forward(A, m[ax], q[ax], axis=ax)
        B = hybrid_forward(B, m[ax], q[ax], axis=ax)
    H = A * B
    for ax in reversed(range(A.ndim)):
        H = hybrid_backward(H, m[ax], q[ax], L[ax], axis=ax)
    return H


# ---------------------------------------------------------------------------
# complex packing and the RCM operator (Sec. 4, Appendix B)
# ---------------------------------------------------------------------------

def complex_pack(f: np.ndarray) -> np.ndarray:
    """eq. (complexPacking) along the last axis; an odd length gets an implicit zero partner."""
    f = np.asarray(f, dtype=np.float64)
    L = f.shape[-1]
    Lt = (L + 1) // 2
    out = np.zeros(f.shape[:-1] + (Lt,), dtype=np.complex128)
    out.real = f[..., 0::2]
    out.imag[..., : L // 2] = f[..., 1::2]
    return out


def complex_unpack(ht: np.ndarray, L: int) -> np.ndarray:
    """Inverse of complex_pack, keeping the first L reals of the last axis."""
    h = np.empty(ht.shape[:-1] + (L,), dtype=np.float64)
    h[..., 0::2] = ht.real[..., : (L + 1) // 2]
    h[..., 1::2] = ht.imag[..., : L // 2]
    return h


def conj_reflect(A: np.ndarray) -> np.ndarray:
    """conj(A_{k*}) with k*_i = (N_i - k_i) mod N_i on every axis (Sec. 5)."""
    B = A
    for ax in range(A.ndim):
        B = np.roll(np.flip(B, axis=ax), 1, axis=ax)
    return np.conj(B)


def fourier_unpack(Ft: np.ndarray) -> np.ndarray:
    """eq. (fourierUnpack): F_k for k = 0..N~ from the packed DFT (last axis), F~_{N~} := F~_0.

    In several dimensions the partner index is the conjugate multi-index k*
    (the packed axis is the last one).
    """
    N = Ft.shape[-1]
    ext = np.concatenate([Ft, Ft[..., :1]], axis=-1)          # F~_0 .. F~_N
    cr = conj_reflect(Ft)
    cr_ext = np.concatenate([cr, cr[..., :1]], axis=-1)       # conj F~_{(N-k)*}
    k = np.arange(N + 1)
    tw = zeta(2 * N, k)
    return 0.5 * (ext + cr_ext) - 0.5j * (ext - cr_ext) * tw


def fourier_pack(F: np.ndarray) -> np.ndarray:
    """eq. (fourierPack): F~_k (k < N~) from F_k, k = 0..N~ (last axis)."""
    N = F.shape[-1] - 1
    Fk = F[..., :N]
    # conj F_{N~-k} with the other axes reflected as well (multi-index conjugate)
    Fr = F[..., N - np.arange(N)]
    for ax in range(F.ndim - 1):
        Fr = np.roll(np.flip(Fr, axis=ax), 1, axis=ax)
    Fc = np.conj(Fr)
    k = np.arange(N)
    return 0.5 * (Fk + Fc) + 0.5j * (Fk - Fc) * zeta(2 * N, -k)


def rcm(Ft: np.ndarray, Gt: np.ndarray) -> np.ndarray:
    """The RCM operator, eq. (RCM) in 1D and eq. (RCM-ndim) in n dimensions.

    (F~ [.] G~)_k = F~_k G~_k - 1/4 (F~_k - conj F~_{k*})(G~_k - conj G~_{k*})(1 + zeta_{N~}^{k_n}).
    """
    N = Ft.shape[-1]
    Fc = conj_reflect(Ft)
    Gc = conj_reflect(Gt)
    z = 1.0 + zeta(N, np.arange(N))
    return Ft * Gt - 0.25 * (Ft - Fc) * (Gt - Gc) * z


def rcm_via_unpack(Ft: np.ndarray, Gt: np.ndarray) -> np.ndarray:
    """eq. (RCM-U): U^{-1}(U(F~) . U(G~)) with explicit unpacking and packing."""
    return fourier_pack(fourier_unpack(Ft) * fourier_unpack(Gt))


def rcm_residue_pairs(Fres: np.ndarray, Gres: np.ndarray) -> np.ndarray:
    """eqs. (Hr), (Hr-conj): RCM over residues, one unordered pair at a time.

    Fres[r, l] = F~_{q l + r}.  For residue r the partner of (l, r) is
    (m - l - 1, q - r) when r != 0 and ((m - l) mod m, 0) when r = 0, i.e. the
    index N~ - k reduced mod N~.  W (the paper's script-A) is formed once per
    pair and enters the two outputs as W and conj W.
    """
    q, m = Fres.shape
    H = np.empty_like(Fres)
    done = np.zeros((q, m), dtype=bool)
    for r in range(q):
        r2 = (q - r) % q
        for l in range(m):
            if done[r, l]:
                continue
            l2 = (m - l - (1 if r != 0 else 0)) % m
            W = 0.25 * (Fres[r, l] - np.conj(Fres[r2, l2])) * (Gres[r, l] - np.conj(Gres[r2, l2])) \
                * (1.0 + zeta(q * m, q * l + r))
            H[r, l] = Fres[r, l] * Gres[r, l] - W
            done[r, l] = True
            if not done[r2, l2]:
                H[r2, l2] = Fres[r2, l2] * Gres[r2, l2] - np.conj(W)
                done[r2, l2] = True
    return H


def rcm_nary(Fts) -> np.ndarray:
    """eqs. (Akn), (Rnk), (RnMk): R^j = R^{j-1} [.] F~^j for n >= 2 packed spectra (1D)."""
    R = Fts[0]
    N = R.shape[-1]
    k = np.arange(N)
    z = 1.0 + zeta(N, k)
    for Fj in Fts[1:]:
        Rc = np.conj(R[(N - k) % N])
        Fc = np.conj(Fj[(N - k) % N])
        A = 0.25 * (R - Rc) * (Fj - Fc) * z
        R = R * Fj - A
    return R


def hybrid_rcm_conv(f: np.ndarray, g: np.ndarray, m, q) -> np.ndarray:
    """hybridRCM (Sec. 4 with Sec. 5): implicit packing plus hybrid dealiasing.

    m, q are per axis; on the last axis they describe the complex-packed axis
    (length ceil(L_n/2), transform length N~ = q m with 2 N~ >= 2 L_n - 1).
    Steps: pack along the last axis, implicitly padded residue transforms on
    every axis, RCM-ndim product with the conjugate multi-index, inverse with
    accumulation over residues, unpack.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    d = f.ndim
    L = f.shape
    m = tuple(int(v) for v in m)
    q = tuple(int(v) for v in q)
    for ax in range(d - 1):
        if q[ax] * m[ax] < 2 * L[ax] - 1:
            raise ValueError("outer axis: q m must be >= 2L-1")
    if 2 * q[-1] * m[-1] < 2 * L[-1] - 1:
        raise ValueError("packed axis: 2 q m must be >= 2L-1")
    F = complex_pack(f)
    G = complex_pack(g)
    Lp = F.shape
    for ax in range(d):
        F = hybrid_forward(F, m[ax], q[ax], axis=ax)
        G = hybrid_forward(G, m[ax], q[ax], axis=ax)
    H = rcm(F, G)
    for ax in reversed(range(d)):
        H = hybrid_backward(H, m[ax], q[ax], Lp[ax], axis=ax)
    return complex_unpack(H, L[-1])


def hybrid_rcm_conv_1d_residues(f: np.ndarray, g: np.ndarray, m: int, q: int) -> np.ndarray:
    """1D hybridRCM computed literally one residue pair at a time (Sec. 4, eqs. (Hr), (Hr-conj)).

    Residue pairs {r, q-r} (0 and q/2 self-paired) are formed, multiplied and
    accumulated into h~ with eq. (accumulation); then unpacked.
    """
    ft = complex_pack(f)
    gt = complex_pack(g)
    Lt = ft.shape[0]
    L = np.asarray(f).shape[0]
    if 2 * q * m < 2 * L - 1:
        raise ValueError("2 q m must be >= 2L-1")
    p = ceil(Lt / m)
    acc = np.zeros(p * m, dtype=np.complex128)
    for r in range(q // 2 + 1):
        r2 = (q - r) % q
        rs = [r] if r2 == r else [r, r2]
        Fr = {x: residue_forward(ft, m, q, x) for x in rs}
        Gr = {x: residue_forward(gt, m, q, x) for x in rs}
        Hr = {}
        for x in rs:
            x2 = (q - x) % q
            l = np.arange(m)
            l2 = (m - l - (1 if x != 0 else 0)) % m
            W = 0.25 * (Fr[x] - np.conj(Fr[x2][l2])) * (Gr[x] - np.conj(Gr[x2][l2])) \
                * (1.0 + zeta(q * m, q * l + x))
            Hr[x] = Fr[x] * Gr[x] - W
        for x in rs:
            acc += residue_backward(Hr[x], m, q, x, p)
    ht = acc[:Lt] / float(q * m)
    return complex_unpack(ht, L)


# ---------------------------------------------------------------------------
# explicit padding with implicit packing (Sec. 5 algorithms)
# ---------------------------------------------------------------------------

def mult_rcm(A, B, C, D, first: bool) -> None:
    """In-place implicit-packing multiply on length-M arrays (M even), output in A and C.

    Z_k = (1 + zeta_M^k)/4.  The pair (k, M-k) shares one product term alpha,
    entering A_k and C_{M-k} as alpha and conj(alpha); k = 0 is handled when
    ``first`` (Z_0 = 1/2) and k = M/2 needs no correction (Z_{M/2} = 0).
    """
    M = A.shape[0]
    same = (A is C) or (B is D)
    if first:
        alpha = 0.5 * (A[0] - np.conj(C[0])) * (B[0] - np.conj(D[0]))
        c0 = C[0] * D[0] - np.conj(alpha)
        A[0] = A[0] * B[0] - alpha
        if not same:
            C[0] = c0
    for k in range(1, M // 2):
        Z = (1.0 + zeta(M, k)) / 4.0
        alpha = (A[k] - np.conj(C[M - k])) * (B[k] - np.conj(D[M - k])) * Z
        A[k] = A[k] * B[k] - alpha
        C[M - k] = C[M - k] * D[M - k] - np.conj(alpha)
    A[M // 2] = A[M // 2] * B[M // 2]


def explicit_rcm_conv_1d(f: np.ndarray, g: np.ndarray, M: int | None = None) -> np.ndarray:
    """explicitRCM in 1D: zero pad to M, pack, FFT, in-place RCM multiply, inverse, unpack."""
    f = np.asarray(f, dtype=np.float64)
    L = f.shape[0]
    M = 2 * L if M is None else int(M)
    if M % 4 or M < 2 * L - 1:
        # the in-place multiply assumes an even packed length M/2
        raise ValueError("M must be a multiple of 4 and >= 2L-1")
    fp = np.zeros(M)
    gp = np.zeros(M)
    fp[:L] = f
    gp[:L] = g
    F = dft(complex_pack(fp))
    G = dft(complex_pack(gp))
    mult_rcm(F, G, F, G, True)
    ht = idft_unnormalized(F) / (M // 2)
    return complex_unpack(ht, M)[:L]


def explicit_rcm_conv_2d(f: np.ndarray, g: np.ndarray, M=None) -> np.ndarray:
    """explicitRCM in 2D: FFT along x, then conjugate slice pairs (k1, k1*) along y."""
    f = np.asarray(f, dtype=np.float64)
    L1, L2 = f.shape
    M1, M2r = (2 * L1, 2 * L2) if M is None else (int(M[0]), int(M[1]))
    if M1 % 2 or M2r % 4:
        raise ValueError("padded sizes must be even (packed last axis even)")
    fp = np.zeros((M1, M2r))
    gp = np.zeros((M1, M2r))
    fp[:L1, :L2] = f
    gp[:L1, :L2] = g
    F = dft(complex_pack(fp), axis=0)
    G = dft(complex_pack(gp), axis=0)
    for k1 in range(M1 // 2):
        k1s = M1 // 2 if k1 == 0 else M1 - k1
        Fa = dft(F[k1].copy())
        Ga = dft(G[k1].copy())
        Fc = dft(F[k1s].copy())
        Gc = dft(G[k1s].copy())
        if k1 == 0:
            mult_rcm(Fa, Ga, Fa, Ga, True)
            mult_rcm(Fc, Gc, Fc, Gc, True)
        else:
            mult_rcm(Fa, Ga, Fc, Gc, True)
            mult_rcm(Fc, Gc, Fa, Ga, False)
        F[k1] = idft_unnormalized(Fa)
        F[k1s] = idft_unnormalized(Fc)
    ht = idft_unnormalized(F, axis=0) / float(M1 * (M2r // 2))
    return complex_unpack(ht, M2r)[:L1, :L2]


# ---------------------------------------------------------------------------
# real hybrid dealiasing via conjugate symmetries (Sec. 3, Appendix A)
# ---------------------------------------------------------------------------

def _hermitian_extend(half: np.ndarray, m: int, axis: int = 0) -> np.ndarray:
    """Full length-m spectrum from entries l = 0..floor(m/2), using X_{m-l} = conj X_l."""
    half = np.moveaxis(half, axis, 0)
    full = np.empty((m,) + half.shape[1:], dtype=np.complex128)
    nh = m // 2 + 1
    full[:nh] = half[:nh]
    for l in range(nh, m):
        full[l] = np.conj(half[m - l])
    return np.moveaxis(full, 0, axis)


def cs_q2_forward(xp: np.ndarray, m: int, p: int) -> np.ndarray:
    """Even-index residue q/2 values F_{2cq+q/2}, c < e, eq. (forwardq2) (first axis).

    F_{2cq+q/2} = sum_{b<e} zeta_e^{cb} zeta_{2m}^b sum_t (-1)^t (x_{tm+b} + i x_{tm+e+b}).
    """
    e = m // 2
    xr = xp.reshape((p, m) + xp.shape[1:])
    sgn = np.array([(-1.0) ** t for t in range(p)])
    z = np.tensordot(sgn, xr[:, :e] + 1j * xr[:, e:2 * e], axes=(0, 0))
    z = z * _bshape(zeta(2 * m, np.arange(e)), z.ndim, 0)
    return dft(z, axis=0)


def cs_q2_backward(Hq2: np.ndarray, m: int, p: int) -> np.ndarray:
    """h_{q/2} from its even-index values, eqs. (wb), (accumulateq2) (first axis).

    w_b = zeta_{2m}^{-b} sum_c zeta_e^{-bc} H_{2cq+q/2};
    h_{q/2, tm+b} = (-1)^t 2 Re w_b and h_{q/2, tm+e+b} = (-1)^t 2 Im w_b.
    """
    e = m // 2
    w = idft_unnormalized(Hq2, axis=0) * _bshape(zeta(2 * m, -np.arange(e)), Hq2.ndim, 0)
    out = np.zeros((p * m,) + Hq2.shape[1:], dtype=np.float64)
    for t in range(p):
        sg = (-1.0) ** t
        out[t * m: t * m + e] = sg * 2.0 * w.real
        out[t * m + e: t * m + 2 * e] = sg * 2.0 * w.imag
    return out


def _cs_check(L: int, M_eff: int, m: int, q: int):
    if q * m < 2 * L - 1:
        raise ValueError("q m must be >= 2L-1")
    if q % 2 == 0 and m % 2:
        raise ValueError("q even requires m even (Sec. 3.1.3)")


def hybrid_cs_conv_1d(f: np.ndarray, g: np.ndarray, m: int, q: int) -> np.ndarray:
    """hybridCS in 1D (Sec. 3), general p = ceil(L/m) without the inner loop.

    eq. (real-accumulation): f = (1/qm)(h_0 + 2 sum_{r=1}^{ceil(q/2)-1} Re h_r + h_{q/2}),
    with r = 0 through a real transform of sum_t f_{tm+s} (Sec. 3.1.1), the
    middle residues through complex transforms, and r = q/2 through the
    even-index fold (Sec. 3.1.3).  Products are elementwise per residue.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    L = f.shape[0]
    _cs_check(L, q * m, m, q)
    p = ceil(L / m)
    fp = np.zeros(p * m)
    gp = np.zeros(p * m)
    fp[:L] = f
    gp[:L] = g
    acc = np.zeros(p * m)
    # r = 0: real-to-complex of sum_t f_{tm+s}, half spectrum, complex-to-real
    a = fp.reshape(p, m).sum(axis=0)
    b = gp.reshape(p, m).sum(axis=0)
    nh = m // 2 + 1
    P0 = dft(a)[:nh] * dft(b)[:nh]
    h0 = idft_unnormalized(_hermitian_extend(P0, m)).real
    acc += np.tile(h0, p)
    # 1 <= r <= ceil(q/2) - 1: complex residues, 2 Re h_r
    for r in range(1, (q + 1) // 2):
        Hr = residue_forward(fp, m, q, r) * residue_forward(gp, m, q, r)
        acc += 2.0 * residue_backward(Hr, m, q, r, p).real
    # r = q/2 (q even): length-e transforms of the folded data
    if q % 2 == 0:
        Hq2 = cs_q2_forward(fp, m, p) * cs_q2_forward(gp, m, p)
        acc += cs_q2_backward(Hq2, m, p)
    return acc[:L] / float(q * m)


# ---------------------------------------------------------------------------
# conjugate-symmetry residues with implicit packing for r = 0 and r = q/2
# (the combination the discussion of Sec. 6 proposes)
# ---------------------------------------------------------------------------

def packed_forward(a: np.ndarray, twist: bool) -> np.ndarray:
    """Packed transform of a real sequence a of even length m along axis 0 (eq. (complexPacking)):
    a~_j = a_{2j} + i a_{2j+1}, j < m/2, and P_l = sum_j zeta_m^{j (2 l + twist)} a~_j, l < m/2.

    twist = 0: the DFT of length m/2 of the packed data (residue 0, whose contribution is a cyclic
    convolution of length m); twist = 1: the packed transform that carries the odd frequencies
    A_l = sum_s zeta_{2m}^{s (2l+1)} a_s of residue q/2 (eq. (forwardq2): a negacyclic convolution).
    """
    a = np.asarray(a, dtype=np.float64)
    m = a.shape[0]
    at = a[0::2] + 1j * a[1::2]
    if twist:
        at = at * _bshape(zeta(m, np.arange(m // 2)), at.ndim, 0)
    return dft(at, axis=0)


def packed_backward(P: np.ndarray, twist: bool) -> np.ndarray:
    """Inverse of packed_forward without normalisation, unpacked: x~_j = zeta_m^{-j twist}
    sum_l zeta_{m/2}^{-j l} P_l, x_{2j} = Re x~_j, x_{2j+1} = Im x~_j (real length m)."""
    xt = idft_unnormalized(P, axis=0)
    if twist:
        xt = xt * _bshape(zeta(2 * P.shape[0], -np.arange(P.shape[0])), xt.ndim, 0)
    out = np.empty((2 * P.shape[0],) + P.shape[1:], dtype=np.float64)
    out[0::2] = xt.real
    out[1::2] = xt.imag
    return out


def packed_product(P: np.ndarray, Q: np.ndarray, twist: bool) -> np.ndarray:
    """The RCM operator on packed transforms of length e = m/2 (axis 0):

    twist = 0: eq. (RCM) with N~ = e: R_l = P_l Q_l - 1/4 (P_l - conj P_{e-l})(Q_l - conj Q_{e-l})(1 + zeta_e^l);
    twist = 1: the same with the frequency l shifted by 1/2: partner l' = e - 1 - l and factor
    (1 + zeta_m^{2l+1}).  (With E_l, O_l the transforms of the even and odd samples, P_l = E_l + i O_l
    and conj P_{l'} = E_l - i O_l; the product A_l B_l and A_{l+e} B_{l+e} of the odd-frequency
    transforms A_l = E_l + zeta_{2m}^{2l+1} O_l, packed again, reduce to this form as eq. (RCM) does.)
    R is the packed transform of the cyclic (twist 0) or negacyclic (twist 1) convolution.
    """
    e = P.shape[0]
    l = np.arange(e)
    part = (e - l) % e if not twist else e - 1 - l
    Pc = np.conj(P[part])
    Qc = np.conj(Q[part])
    z = 1.0 + (zeta(e, l) if not twist else zeta(2 * e, 2 * l + 1))
    z = _bshape(z, P.ndim, 0)
    return P * Q - 0.25 * (P - Pc) * (Q - Qc) * z


def hybrid_mix_conv_1d(f: np.ndarray, g: np.ndarray, m: int, q: int) -> np.ndarray:
    """hybridCS (Sec. 3) with implicit packing for the self-conjugate residues 0 and q/2.

    eq. (real-accumulation), f = (1/qm)(h_0 + 2 sum_{r=1}^{ceil(q/2)-1} Re h_r + h_{q/2}), where
    the middle residues are the complex residue transforms of Sec. 2 with elementwise products, and
    h_0, h_{q/2} come from the real sums y_s = sum_t f_{tm+s} and y'_s = sum_t (-1)^t f_{tm+s}
    (Secs. 3.1.1, 3.1.3) packed into m/2 complex values and multiplied by packed_product: every
    residue is computed on its own, and the two self-conjugate ones at half length.  m must be even.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    L = f.shape[0]
    _cs_check(L, q * m, m, q)
    if m % 2:
        raise ValueError("the packed residues need an even m")
    p = ceil(L / m)
    fp = np.zeros(p * m)
    gp = np.zeros(p * m)
    fp[:L] = f
    gp[:L] = g
    fr, gr = fp.reshape(p, m), gp.reshape(p, m)
    acc = np.zeros(p * m)
    # r = 0: h_0 = m (y^f cyclically convolved with y^g) = 2 x the unnormalised packed inverse
    R0 = packed_product(packed_forward(fr.sum(axis=0), False), packed_forward(gr.sum(axis=0), False), False)
    acc += np.tile(2.0 * packed_backward(R0, False), p)
    for r in range(1, (q + 1) // 2):
        Hr = residue_forward(fp, m, q, r) * residue_forward(gp, m, q, r)
        acc += 2.0 * residue_backward(Hr, m, q, r, p).real
    if q % 2 == 0:
        sg = np.array([(-1.0) ** t for t in range(p)])
        Rq = packed_product(packed_forward(sg @ fr, True), packed_forward(sg @ gr, True), True)
        hq = 2.0 * packed_backward(Rq, True)
        for t in range(p):
            acc[t * m:(t + 1) * m] += sg[t] * hq
    return acc[:L] / float(q * m)


def hybrid_mix_conv_nd(f: np.ndarray, g: np.ndarray, m, q) -> np.ndarray:
    """The mixed variant in 2D/3D: conjugate symmetry on the first axis (Secs. 3 and 5), implicit packing
    (Sec. 4) for that axis's self-conjugate residues 0 and q0/2.

    m, q per axis describe the first axis (real data, q0 m0 >= 2 L0 - 1) and the complex transforms of the
    other axes.  Residues r = 1 .. ceil(q0/2) - 1: residue transforms of f and g along the first axis
    (eq. (forwardr)), implicitly padded transforms along the others, elementwise product, inverse, and
    2 Re h_r in eq. (real-accumulation).  Residues 0 and q0/2: f and g packed along the last axis
    (eq. (complexPacking)), their residue-0 and residue-q0/2 transforms along the first axis placed at
    k0 = q0 l + r of the natural order (the other residues zero), implicitly padded transforms along the
    middle axes and the packed last axis (m_p = max(m_n / 2, 1), 2 q_p m_p >= 2 L_n - 1), eq. (RCM-ndim)
    (its conjugate multi-index maps residue 0 and residue q0/2 onto themselves, so the zero residues stay
    zero), inverse with eq. (accumulation), unpacked.  h = both parts (each carries 1/(q0 m0)).
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    d = f.ndim
    L = f.shape
    m = tuple(int(v) for v in m)
    q = tuple(int(v) for v in q)
    m0, q0 = m[0], q[0]
    _cs_check(L[0], q0 * m0, m0, q0)
    for ax in range(1, d):
        if q[ax] * m[ax] < 2 * L[ax] - 1:
            raise ValueError("q m must be >= 2L-1 on every axis")
    p0 = ceil(L[0] / m0)
    # residues 1 .. ceil(q0/2) - 1
    mid = np.zeros(L)
    for r in range(1, (q0 + 1) // 2):
        Fr = residue_forward(f, m0, q0, r, axis=0)
        Gr = residue_forward(g, m0, q0, r, axis=0)
        for ax in range(1, d):
            Fr = hybrid_forward(Fr, m[ax], q[ax], axis=ax)
            Gr = hybrid_forward(Gr, m[ax], q[ax], axis=ax)
        Hr = Fr * Gr
        for ax in reversed(range(1, d)):
            Hr = hybrid_backward(Hr, m[ax], q[ax], L[ax], axis=ax)
        mid += 2.0 * residue_backward(Hr, m0, q0, r, p0, axis=0)[:L[0]].real
    # residues 0 and q0/2 with implicit packing along the last axis
    mp = max(m[-1] // 2, 1)
    qp = ceil((2 * L[-1] - 1) / (2 * mp))
    Ft, Gt = complex_pack(f), complex_pack(g)
    Lp = Ft.shape
    packed_res = [0] + ([q0 // 2] if q0 % 2 == 0 else [])
    spec = []
    for X in (Ft, Gt):
        S = np.zeros((q0 * m0,) + X.shape[1:], dtype=np.complex128)
        for r in packed_res:
            S[r::q0] = residue_forward(X, m0, q0, r, axis=0)
        for ax in range(1, d):
            mm, qq = (mp, qp) if ax == d - 1 else (m[ax], q[ax])
            S = hybrid_forward(S, mm, qq, axis=ax)
        spec.append(S)
    H = rcm(spec[0], spec[1])
    for ax in reversed(range(d)):
        mm, qq = (mp, qp) if ax == d - 1 else (m[ax], q[ax])
        H = hybrid_backward(H, mm, qq, Lp[ax], axis=ax)
    return complex_unpack(H, L[-1]) + mid / float(q0 * m0)


def hybrid_cs_conv_1d_inner(f: np.ndarray, g: np.ndarray, m: int, n: int) -> np.ndarray:
    """hybridCS with the real inner loop (Appendix A): q = n p, r = u n + v.

    eq. (real-accumulationInner): f = (1/qm)(h_0 + 2 sum_{v=1}^{ceil(n/2)-1} Re h_v + h_{n/2}).
    * v = 0: length-p real DFT over t, then the Sec. 3 case split over u
      (u = 0 real, 1 <= u < p/2 complex, u = p/2 folded), eq. (Fv0);
    * 1 <= v < n/2: complex inner loop, length-p FFTs of zeta_q^{vt} f_{tm+s};
    * v = n/2 (n even): p even -> the folded length-p/2 transforms of
      eq. (Fn2gamma) and w_{s,beta}; p odd -> a full complex length-p
      transform (no saving, same result).
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    L = f.shape[0]
    p = ceil(L / m)
    q = n * p
    _cs_check(L, q * m, m, q)
    N = q * m
    fp = np.zeros(p * m)
    gp = np.zeros(p * m)
    fp[:L] = f
    gp[:L] = g
    X = fp.reshape(p, m)
    Y = gp.reshape(p, m)
    s = np.arange(m)
    acc = np.zeros((p, m))

    # ---- v = 0 ------------------------------------------------------------
    # length-p DFT over t (real data): Xu[u, s] = sum_t zeta_p^{ut} f_{tm+s}
    Xu = dft(X.astype(np.complex128), axis=0)
    Yu = dft(Y.astype(np.complex128), axis=0)
    # per u: residue r = u n with twiddle zeta_{qm}^{u n s}; only u <= p/2 are needed
    h0u = {}
    for u in range(p // 2 + 1):
        if 2 * u == p:
            continue
        tw = zeta(N, u * n * s)
        if u == 0:
            nh = m // 2 + 1
            P = dft(Xu[0].real)[:nh] * dft(Yu[0].real)[:nh]
            h0u[u] = idft_unnormalized(_hermitian_extend(P, m))            # zeta_{qm}^0 = 1
        else:
            P = dft(Xu[u] * tw) * dft(Yu[u] * tw)
            h0u[u] = idft_unnormalized(P) * np.conj(tw)
    # u = p/2 (p even): data sum_t (-1)^t f_{tm+s} is real, twiddle zeta_{2m}^s -> fold to length m/2
    if p % 2 == 0:
        e = m // 2
        a = Xu[p // 2].real
        b = Yu[p // 2].real
        Fa = dft((a[:e] + 1j * a[e:2 * e]) * zeta(2 * m, np.arange(e)))
        Fb = dft((b[:e] + 1j * b[e:2 * e]) * zeta(2 * m, np.arange(e)))
        w = idft_unnormalized(Fa * Fb) * zeta(2 * m, -np.arange(e))
        hp2 = np.concatenate([2.0 * w.real, 2.0 * w.imag])                # real, length m
    # inverse length-p real DFT over u: h_{0,tm+s} = sum_u zeta_p^{-tu} (post-twiddled) contribution
    for t in range(p):
        row = h0u[0].real.copy()
        for u in range(1, (p + 1) // 2):
            row += 2.0 * (zeta(p, -t * u) * h0u[u]).real
        if p % 2 == 0:
            row += ((-1.0) ** t) * hp2
        acc[t] += row

    # ---- 1 <= v < n/2: complex inner loop -----------------------------------
    def complex_v(v):
        tv = zeta(q, v * np.arange(p))[:, None]
        Fx = dft(X * tv, axis=0)                        # Y[u, s], length-p FFT over t
        Fy = dft(Y * tv, axis=0)
        hv = np.zeros((p, m), dtype=np.complex128)
        W = np.empty((p, m), dtype=np.complex128)
        for u in range(p):
            tw = zeta(N, (u * n + v) * s)
            P = dft(Fx[u] * tw) * dft(Fy[u] * tw)
            W[u] = idft_unnormalized(P) * np.conj(tw)
        Z = idft_unnormalized(W, axis=0)                # sum_u zeta_p^{-tu}
        hv = Z * np.conj(tv)                            # zeta_q^{-tv}
        return hv

    for v in range(1, (n + 1) // 2):
        acc += 2.0 * complex_v(v).real

    # ---- v = n/2 (n even) ---------------------------------------------------
    if n % 2 == 0:
        v = n // 2
        if p % 2 == 0:
            P2 = p // 2
            beta = np.arange(P2)
            tb = zeta(2 * p, beta)[:, None]
            zx = (X[:P2] + 1j * X[P2:2 * P2]) * tb       # zeta_{2p}^beta [f_{beta m+s} + i f_{(P+beta)m+s}]
            zy = (Y[:P2] + 1j * Y[P2:2 * P2]) * tb
            Gx = dft(zx, axis=0)                         # sum_beta zeta_P^{gamma beta}
            Gy = dft(zy, axis=0)
            Wg = np.empty((P2, m), dtype=np.complex128)
            for gam in range(P2):
                tw = zeta(N, (2 * gam * n + v) * s)
                P = dft(Gx[gam] * tw) * dft(Gy[gam] * tw)
                Wg[gam] = idft_unnormalized(P) * np.conj(tw)
            w = idft_unnormalized(Wg, axis=0) * np.conj(tb)   # w_{s,beta}
            acc[:P2] += 2.0 * w.real
            acc[P2:2 * P2] += 2.0 * w.imag
        else:
            acc += complex_v(v).real

    return acc.reshape(-1)[:L] / float(N)


def hybrid_cs_conv(f: np.ndarray, g: np.ndarray, m, q) -> np.ndarray:
    """hybridCS in d dimensions (Sec. 5): real first-axis residues, complex inner sub-convolutions.

    The first axis gets the real residue treatment of Sec. 3 (r = 0 real,
    1 <= r < q/2 complex with 2 Re, r = q/2 folded); for every retained
    first-axis mode the remaining axes are convolved with the complex hybrid
    algorithm of Sec. 2 (elementwise products).  m, q per axis, real units.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if f.ndim == 1:
        return hybrid_cs_conv_1d(f, g, int(m[0]), int(q[0]))
    L = f.shape
    m1, q1 = int(m[0]), int(q[0])
    mi, qi = tuple(m[1:]), tuple(q[1:])
    _cs_check(L[0], q1 * m1, m1, q1)
    p1 = ceil(L[0] / m1)
    rest = L[1:]
    fp = np.zeros((p1 * m1,) + rest)
    gp = np.zeros((p1 * m1,) + rest)
    fp[:L[0]] = f
    gp[:L[0]] = g
    acc = np.zeros((p1 * m1,) + rest)

    def inner(A, B):
        return np.stack([complex_hybrid_conv(A[i], B[i], mi, qi) for i in range(A.shape[0])])

    # r1 = 0: real sums over t, half spectrum along the first axis
    a = fp.reshape((p1, m1) + rest).sum(axis=0)
    b = gp.reshape((p1, m1) + rest).sum(axis=0)
    nh = m1 // 2 + 1
    P0 = inner(dft(a, axis=0)[:nh], dft(b, axis=0)[:nh])
    h0 = idft_unnormalized(_hermitian_extend(P0, m1), axis=0).real
    acc += np.concatenate([h0] * p1, axis=0)
    for r in range(1, (q1 + 1) // 2):
        Hr = inner(residue_forward(fp, m1, q1, r), residue_forward(gp, m1, q1, r))
        acc += 2.0 * residue_backward(Hr, m1, q1, r, p1).real
    if q1 % 2 == 0:
        Hq2 = inner(cs_q2_forward(fp, m1, p1), cs_q2_forward(gp, m1, p1))
        acc += cs_q2_backward(Hq2, m1, p1)
    return acc[:L[0]] / float(q1 * m1)
