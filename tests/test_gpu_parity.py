"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (stated per result): normwise relative error <= 1e-12 in float64
and <= 1e-5 in float32 (inputs rounded to float32 first; the oracle sees the
rounded values upcast to float64).
"""
import numpy as np
import pytest

from oracle import direct_conv, direct_conv_at, fft_conv, grad_direct, fft_grad, relerr, zero_extend
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}


def _run(hd, f, g, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm"):
    import torch

    tf = torch.from_numpy(f).cuda()
    tg = torch.from_numpy(g).cuda()
    h = hd.conv_forward(tf, tg, ndim=ndim, M=M, m=m, q=q, variant=variant)
    torch.cuda.synchronize()
    return h.cpu().numpy()


def _check(h, ref, dtype, what):
    err = relerr(h, ref)
    print(f"{what}: relerr {err:.3e} (tol {TOL[dtype]:.0e})", flush=True)
    assert np.all(np.isfinite(h)), what
    assert err <= TOL[dtype], f"{what}: relerr {err:.3e}"


# ------------------------------------------------------------------ 1D
CASES_1D = [
    # (L, M, m, q) in real-sample units; None = planner default
    (1024, 2048, 512, 4),      # the 1024-point plain FP64 workload: packed m~=256, q=4, p=2
    (1024, None, None, None),
    (1, None, None, None), (2, None, None, None), (3, None, None, None), (37, None, None, None),
    (37, 80, 8, 10), (33, 66, 8, 17), (100, 199, 16, 13), (257, None, 64, None), (1000, None, None, None),
    (4096, None, None, None), (8192, None, None, None), (999, 2048, 256, 8),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,M,m,q", CASES_1D)
def test_1d_hybrid_rcm(hd, L, M, m, q, dtype):
    f, g = synth.pair_for(101, L, (L,), dtype)
    h = _run(hd, f, g, M=None if M is None else (M,), m=None if m is None else (m,), q=None if q is None else (q,))
    ref = direct_conv(f, g) if L <= 2048 else fft_conv(f, g)
    _check(h, ref, dtype, f"1D L={L} M={M} m={m} q={q} {dtype}")


CASES_1D_MULTI = [
    (1 << 14, None, None, None),        # rows of 2048, column FFTs of 4, n = 2
    (12345, None, None, None),          # ragged: p rounded up to a power of two
    (1 << 16, None, 1024, None),        # rows of 512
    (20000, 40000, 2048, 48),           # q given: 48 = n p with p = 16, n = 3
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,M,m,q", CASES_1D_MULTI)
def test_1d_multipass(hd, L, M, m, q, dtype):
    f, g = synth.pair_for(102, L, (L,), dtype, "normal")
    try:
        h = _run(hd, f, g, M=None if M is None else (M,), m=None if m is None else (m,),
                 q=None if q is None else (q,))
    except hd.HdcError as e:
        if e.status == -2:
            pytest.skip(f"unsupported parameters: {e}")
        raise
    ref = fft_conv(f, g, M=None if M is None else (M,))
    _check(h, ref, dtype, f"1D-multi L={L} M={M} m={m} q={q} {dtype}")


def test_1d_batch(hd):
    import torch

    B, L = 5, 300
    f = np.stack([synth.pair_for(103, b, (L,), np.float32)[0] for b in range(B)])
    g = np.stack([synth.pair_for(103, b, (L,), np.float32)[1] for b in range(B)])
    h = _run(hd, f, g, ndim=1)
    for b in range(B):
        _check(h[b], direct_conv(f[b], g[b]), "float32", f"1D batch item {b}")


@pytest.mark.parametrize("name", ["int_1d_L37", "int_1d_L64", "int_2d_9x12", "int_3d_5x4x6"])
def test_golden_exact_integers(hd, name):
    from tests.golden.make_golden import load

    f, g, h = load(name)
    out = _run(hd, f, g)
    assert np.array_equal(np.rint(out), h)
    assert np.max(np.abs(out - h)) < 1e-9


def test_impulse_and_shift(hd):
    L = 500
    f = synth.uniform((L,), 104, 0, 0)
    d = np.zeros(L)
    d[0] = 1.0
    assert relerr(_run(hd, f, d), f) < 1e-14
    d = np.zeros(L)
    d[7] = 1.0
    ref = np.concatenate([np.zeros(7), f[:-7]])
    assert relerr(_run(hd, f, d), ref) < 1e-14


# ------------------------------------------------------------------ 2D / 3D
CASES_ND = [
    ((9, 12), None, None, None),
    ((64, 48), None, None, None),
    ((100, 75), None, None, None),
    ((33, 17), (70, 40), (16, 8), (5, 6)),
    ((1, 1), None, None, None),
    ((2, 3), None, None, None),
    ((128, 256), None, None, None),
    ((24, 1500), None, None, None),       # last axis: a complex line of 1024 in both precisions
    ((1500, 12), None, None, None),       # outer axis m = 1024, two blocks, q = 3 (compensated inverse)
    ((3500, 8), None, None, None),        # outer axis m = 1024, four blocks, q = 7
    ((1500, 12), None, (512, 0), None),   # outer axis m = 512 (odd log2 m), three blocks, q = 6
    ((5, 4, 6), None, None, None),
    ((16, 12, 10), None, None, None),
    ((7, 9, 11), None, None, None),
    ((20, 8, 30), (40, 20, 60), (8, 4, 16), (5, 5, 4)),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,M,m,q", CASES_ND)
def test_nd_hybrid_rcm(hd, shape, M, m, q, dtype):
    f, g = synth.pair_for(105, 0, shape, dtype)
    h = _run(hd, f, g, M=M, m=m, q=q)
    ref = direct_conv(f, g) if np.prod(shape) <= 1500 else fft_conv(f, g, M=M)
    _check(h, ref, dtype, f"{len(shape)}D {shape} M={M} m={m} q={q} {dtype}")


def test_planner_defaults(hd):
    """Default FFT lengths that were chosen by measurement: FP64 1D hybridCS at 2^20 keeps rows of
    1024 and takes q = 2048 residues on column pairs; the FP64 2D last axis runs complex lines of 1024;
    1D problems in one workgroup run complex lines of at most 1024 (FP32) or 512 (FP64) and, in FP32, two
    blocks from 64 packed points; the conjugate-symmetry 1D form takes the smallest m with at most four blocks."""
    p = hd.get_plan((1 << 20,), variant="hybrid_cs", dtype="float64")
    assert p.resolved() == ((1024,), (1024,), (2048,)), p.resolved()
    assert p.describe().startswith("cs_col_fwd"), p.describe()
    p = hd.get_plan((2048, 2048), dtype="float64")
    assert p.resolved()[0][1] == 1024, p.resolved()
    p = hd.get_plan((24, 1500), dtype="float64")
    assert p.resolved()[0][1] == 1024, p.resolved()
    # 1D in one workgroup: complex lines of at most 1024 (FP32) / 512 (FP64), up to four blocks
    for L, dt, mc, blocks in ((3000, "float32", 1024, 2), (5000, "float32", 1024, 3), (8000, "float32", 1024, 4),
                              (1500, "float64", 512, 2), (3000, "float64", 512, 3)):
        p = hd.get_plan((L,), dtype=dt)
        assert p.describe() == "line_1d;" and p.resolved()[:2] == ((mc,), (blocks,)), (L, dt, p.describe(), p.resolved())
    p = hd.get_plan((700,), dtype="float32")
    assert p.resolved()[:2] == ((256,), (2,)), p.resolved()  # FP32 from 64 packed points: two blocks
    # conjugate symmetry in one workgroup: the smallest m with at most four blocks; multi-pass beyond
    for L, dt, m, blocks in ((1500, "float32", 512, 3), (3000, "float32", 1024, 3), (3000, "float64", 1024, 3)):
        p = hd.get_plan((L,), variant="hybrid_cs", dtype=dt)
        assert p.describe() == "line_cs;" and p.resolved()[:2] == ((m,), (blocks,)), (L, dt, p.describe(), p.resolved())
    p = hd.get_plan((8000,), variant="hybrid_cs", dtype="float32")
    assert p.describe().startswith("cs_col_fwd"), p.describe()


# ------------------------------------------------------------------ explicit comparators
@pytest.mark.parametrize("variant", ["explicit_rcm", "explicit"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(1024,), (37,), (1 << 14,), (9, 12), (64, 48), (5, 4, 6), (16, 12, 10)])
def test_explicit_variants(hd, shape, variant, dtype):
    f, g = synth.pair_for(106, 0, shape, dtype)
    try:
        h = _run(hd, f, g, variant=variant)
    except hd.HdcError as e:
        if e.status == -2:
            pytest.skip(f"unsupported: {e}")
        raise
    ref = direct_conv(f, g) if np.prod(shape) <= 1500 else fft_conv(f, g)
    _check(h, ref, dtype, f"{variant} {shape} {dtype}")


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(37,), (1024,), (1 << 14,), (9, 12), (5, 4, 6)])
def test_backward(hd, shape, dtype):
    import torch

    f, g = synth.pair_for(107, 0, shape, dtype)
    u = synth.uniform(shape, 107, 0, 2, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    df, dg = hd.conv_backward(tf, tg, tu)
    torch.cuda.synchronize()
    if np.prod(shape) <= 2000:
        rdf, rdg = grad_direct(f, g, u)
    else:
        rdf, rdg = fft_grad(f, g, u)
    _check(df.cpu().numpy(), rdf, dtype, f"df {shape} {dtype}")
    _check(dg.cpu().numpy(), rdg, dtype, f"dg {shape} {dtype}")


@pytest.mark.parametrize("variant", ["explicit_rcm", "explicit"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(37,), (1 << 14,), (9, 12), (5, 4, 6)])
def test_backward_explicit(hd, shape, dtype, variant):
    """The comparators' adjoint: reversed reads and writes through the padding copies."""
    import torch

    f, g = synth.pair_for(114, 0, shape, dtype)
    u = synth.uniform(shape, 114, 0, 2, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    df, dg = hd.conv_backward(tf, tg, tu, variant=variant)
    torch.cuda.synchronize()
    rdf, rdg = grad_direct(f, g, u) if np.prod(shape) <= 2000 else fft_grad(f, g, u)
    _check(df.cpu().numpy(), rdf, dtype, f"{variant} df {shape} {dtype}")
    _check(dg.cpu().numpy(), rdg, dtype, f"{variant} dg {shape} {dtype}")


@pytest.mark.parametrize("variant,shape", [
    ("hybrid_rcm", (1000,)), ("hybrid_rcm", (12345,)), ("hybrid_rcm", (64, 48)), ("hybrid_rcm", (16, 12, 10)),
    ("hybrid_cs", (1000,)), ("hybrid_cs", (12345,)), ("hybrid_cs", (64, 48)), ("explicit_rcm", (9, 12)),
    ("explicit", (1 << 14,)),
])
def test_in_place_output(hd, variant, shape):
    """h may be f or g itself (the header's exact-alias rule): same bits as out of place."""
    import torch

    f, g = synth.pair_for(115, 0, shape, "float32")
    tf, tg = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    want = hd.conv_forward(tf, tg, variant=variant).cpu()
    for target in ("f", "g"):
        a, b = tf.clone(), tg.clone()
        out = a if target == "f" else b
        h = hd.conv_forward(a, b, variant=variant, out=out)
        torch.cuda.synchronize()
        assert h.data_ptr() == out.data_ptr()
        assert torch.equal(out.cpu(), want), f"{variant} {shape}: h aliasing {target}"


def test_unsupported_and_invalid_are_reported(hd):
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), m=(12,))            # packed FFT length 6 is not a power of two
    assert e.value.status == -2
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), M=(150,))           # M < 2L - 1
    assert e.value.status == -1
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), m=(15,))            # odd m on the packed axis
    assert e.value.status == -1


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(1 << 14,), (12345,), (300,), (64, 48), (16, 12, 10)])
def test_deterministic(hd, shape, dtype):
    """Fixed plan -> bitwise identical results run to run (each unordered pair has one owner, no atomics)."""
    import torch

    f, g = synth.pair_for(108, 0, shape, dtype)
    tf = torch.from_numpy(f).cuda()
    tg = torch.from_numpy(g).cuda()
    outs = []
    for _ in range(4):
        outs.append(hd.conv_forward(tf, tg).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    u = torch.from_numpy(synth.uniform(shape, 108, 0, 2, dtype)).cuda()
    d0 = [x.cpu().numpy() for x in hd.conv_backward(tf, tg, u)]
    d1 = [x.cpu().numpy() for x in hd.conv_backward(tf, tg, u)]
    assert np.array_equal(d0[0], d1[0]) and np.array_equal(d0[1], d1[1])


# ------------------------------------------------------------------ conjugate-symmetry variant
CASES_CS_1D = [
    (1024, 2048, 512, 4),      # p = 2, residues 0, 1, q/2 = 2 (folded)
    (1024, None, None, None), (1, None, None, None), (2, None, None, None), (3, None, None, None),
    (37, 80, 8, 10), (33, 66, 8, 9), (100, 199, 16, 13), (257, None, 64, None), (999, 2048, 256, 8),
    (4096, None, None, None), (50, 100, 2, 50),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,M,m,q", CASES_CS_1D)
def test_1d_hybrid_cs(hd, L, M, m, q, dtype):
    f, g = synth.pair_for(111, L, (L,), dtype)
    h = _run(hd, f, g, M=None if M is None else (M,), m=None if m is None else (m,),
             q=None if q is None else (q,), variant="hybrid_cs")
    _check(h, direct_conv(f, g), dtype, f"CS 1D L={L} M={M} m={m} q={q} {dtype}")


CASES_CS_ND = [
    ((9, 12), None, None, None), ((64, 48), None, None, None), ((100, 75), None, None, None),
    ((33, 17), (70, 40), (16, 8), (5, 5)), ((1, 1), None, None, None), ((2, 3), None, None, None),
    ((128, 256), None, None, None), ((5, 4, 6), None, None, None), ((16, 12, 10), None, None, None),
    ((7, 9, 11), None, None, None), ((20, 8, 30), (40, 20, 60), (8, 4, 16), (5, 5, 4)),
    ((12, 10), (24, 20), (4, 8), (6, 3)),
    ((3500, 8), None, None, None),        # first axis m = 1024, four blocks, q = 7
    ((1500, 12), None, (512, 0), None),   # first axis m = 512 (odd log2 m), three blocks, q = 6
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,M,m,q", CASES_CS_ND)
def test_nd_hybrid_cs(hd, shape, M, m, q, dtype):
    f, g = synth.pair_for(112, 0, shape, dtype)
    h = _run(hd, f, g, M=M, m=m, q=q, variant="hybrid_cs")
    ref = direct_conv(f, g) if np.prod(shape) <= 1500 else fft_conv(f, g, M=M)
    _check(h, ref, dtype, f"CS {len(shape)}D {shape} M={M} m={m} q={q} {dtype}")


@pytest.mark.parametrize("name", ["int_1d_L37", "int_1d_L64", "int_2d_9x12", "int_3d_5x4x6"])
def test_golden_exact_integers_cs(hd, name):
    from tests.golden.make_golden import load

    f, g, h = load(name)
    out = _run(hd, f, g, variant="hybrid_cs")
    assert np.array_equal(np.rint(out), h)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(37,), (1024,), (9, 12), (5, 4, 6)])
def test_backward_cs(hd, shape, dtype):
    import torch

    f, g = synth.pair_for(113, 0, shape, dtype)
    u = synth.uniform(shape, 113, 0, 2, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    df, dg = hd.conv_backward(tf, tg, tu, variant="hybrid_cs")
    torch.cuda.synchronize()
    rdf, rdg = grad_direct(f, g, u)
    _check(df.cpu().numpy(), rdf, dtype, f"CS df {shape} {dtype}")
    _check(dg.cpu().numpy(), rdg, dtype, f"CS dg {shape} {dtype}")


CASES_CS_1D_MULTI = [
    # (L, M, m, q): the multi-pass form (rows of m, real length-q transform over the rows)
    (1 << 14, None, None, None),        # rows of 4096 (FP32) / 2048 (FP64)
    (12345, None, None, None),          # ragged last row
    (20000, 40000, 1024, 64),           # q given (power of two), q m > M
    (1 << 16, None, 512, None),         # short rows: 128 rows, q = 256
    (20000, None, 64, 2048),            # q = 2048: the longest column-pair transform
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,M,m,q", CASES_CS_1D_MULTI)
def test_1d_hybrid_cs_multipass(hd, L, M, m, q, dtype):
    f, g = synth.pair_for(112, L, (L,), dtype, "normal")
    plan = hd.get_plan((L,), None if M is None else (M,), None if m is None else (m,), None if q is None else (q,),
                       "hybrid_cs", dtype, 1)
    assert plan.describe().startswith("cs_col_fwd"), plan.describe()
    h = _run(hd, f, g, M=None if M is None else (M,), m=None if m is None else (m,),
             q=None if q is None else (q,), variant="hybrid_cs")
    _check(h, fft_conv(f, g, M=None if M is None else (M,)), dtype, f"CS 1D multi L={L} M={M} m={m} q={q} {dtype}")


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L", [12345, 1 << 14])
def test_1d_hybrid_cs_multipass_backward_and_batch(hd, dtype, L):
    """Odd L: batch elements 1, 3, ... start misaligned for packed column pairs
    (scalar loads); even L: packed loads and stores on every element."""
    import torch

    B = 3
    f = np.stack([synth.pair_for(113, b, (L,), dtype, "normal")[0] for b in range(B)])
    g = np.stack([synth.pair_for(113, b, (L,), dtype, "normal")[1] for b in range(B)])
    dh = np.stack([synth.normal((L,), 113, b, synth.ROLE_U, dtype) for b in range(B)])
    tf, tg, tdh = (torch.from_numpy(x).cuda() for x in (f, g, dh))
    h = hd.conv_forward(tf, tg, ndim=1, variant="hybrid_cs").cpu().numpy()
    df, dg = hd.conv_backward(tf, tg, tdh, ndim=1, variant="hybrid_cs")
    df, dg = df.cpu().numpy(), dg.cpu().numpy()
    for b in range(B):
        _check(h[b], fft_conv(f[b], g[b]), dtype, f"CS 1D multi batch {b}")
        rdf, rdg = fft_grad(f[b], g[b], dh[b])
        _check(df[b], rdf, dtype, f"CS 1D multi df {b}")
        _check(dg[b], rdg, dtype, f"CS 1D multi dg {b}")


def test_cs_rejects_odd_m_with_even_q(hd):
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((8,), m=(1,), q=(16,), variant="hybrid_cs")
    assert e.value.status == -1


# ------------------------------------------------------------------ shorter kernel g (Sec. 7)
CASES_SHORT_KERNEL = [
    # (shape of f and h, shape of g, variant)
    ((1000,), (37,), "hybrid_rcm"),          # one workgroup, odd kernel
    ((1000,), (1,), "hybrid_rcm"),
    ((1000,), (999,), "hybrid_rcm"),
    ((12345,), (100,), "hybrid_rcm"),        # ragged last block
    ((1 << 16,), (4096,), "hybrid_rcm"),     # multi-pass rows
    ((1 << 16,), (33,), "hybrid_rcm"),
    ((300, 200), (31, 17), "hybrid_rcm"),    # 2D, odd kernel width (general raw loads)
    ((64, 48), (40, 6), "hybrid_rcm"),       # 2D, fewer kernel rows (packed loads with a row limit)
    ((256, 256), (9, 9), "hybrid_rcm"),
    ((1000,), (37,), "explicit_rcm"),
    ((300, 200), (31, 17), "explicit"),
    ((20, 18, 16), (5, 4, 3), "explicit_rcm"),
    ((20, 18, 16), (5, 4, 3), "hybrid_rcm"),     # 3D: odd kernel last axis (general loads)
    ((16, 12, 10), (8, 6, 10), "hybrid_rcm"),    # 3D: same last axis, fewer rows and middle planes (packed loads)
    ((16, 12, 10), (8, 6, 4), "hybrid_rcm"),     # 3D: shorter even last axis (column indices split by f's layout)
    # conjugate symmetry and the mixed variant: the kernel read at its own extents
    ((1000,), (37,), "hybrid_cs"),               # one workgroup
    ((1000,), (1000,), "hybrid_cs"),
    ((1 << 16,), (4096,), "hybrid_cs"),          # multi-pass (pair transform of the rows)
    ((1 << 16,), (33,), "hybrid_cs"),
    ((12345,), (101,), "hybrid_cs"),
    ((300, 200), (31, 17), "hybrid_cs"),         # 2D: first-axis columns index f's layout
    ((64, 48), (40, 48), "hybrid_cs"),
    ((20, 18, 16), (5, 4, 3), "hybrid_cs"),      # 3D
    ((16, 12, 10), (8, 12, 10), "hybrid_cs"),
    ((1000,), (37,), "hybrid_mix"),
    ((3000,), (999,), "hybrid_mix"),
    ((2048,), (1,), "hybrid_mix"),
    ((4000,), (2000,), "hybrid_mix"),            # the kernel spans several blocks
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,kshape,variant", CASES_SHORT_KERNEL)
def test_short_kernel(hd, shape, kshape, variant, dtype):
    f = synth.normal(shape, 116, 0, synth.ROLE_F, dtype)
    g = synth.normal(kshape, 116, 0, synth.ROLE_G, dtype)
    h = _run(hd, f, g, variant=variant)
    assert h.shape == f.shape
    ref = direct_conv(f, g) if f.size * g.size <= 4e6 else fft_conv(f, g)
    _check(h, ref, dtype, f"short kernel {shape} * {kshape} {variant} {dtype}")


def test_short_kernel_batch_and_plan(hd):
    """A batch of two pairs with one plan; the resolved residues shrink with the kernel (M = L + Lg)."""
    import torch

    L, Lg, B = 20000, 300, 2
    f = np.stack([synth.normal((L,), 117, b, synth.ROLE_F, "float32") for b in range(B)])
    g = np.stack([synth.normal((Lg,), 117, b, synth.ROLE_G, "float32") for b in range(B)])
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), ndim=1).cpu().numpy()
    for b in range(B):
        _check(h[b], fft_conv(f[b], g[b]), "float32", f"short kernel batch {b}")
    full = hd.Plan((L,), dtype="float32")
    short = hd.Plan((L,), dtype="float32", kernel_shape=(Lg,))
    mf, pf, qf = full.resolved()
    ms, ps, qs = short.resolved()
    assert qs[0] * ms[0] <= qf[0] * mf[0], (full.resolved(), short.resolved())


def test_short_kernel_unsupported(hd):
    import torch

    with pytest.raises(hd.HdcError) as e:  # n arrays: equal extents only
        hd.Plan((100,), kernel_shape=(10,), nin=3)
    assert e.value.status == -2
    plan = hd.Plan((100,), kernel_shape=(10,))
    assert plan.bwd_ws_bytes >= plan.ws_bytes + 100 * 4  # scratch of f's extents for dg
    f = torch.zeros(100, device="cuda")
    g = torch.zeros(10, device="cuda")
    dh = torch.zeros(100, device="cuda")
    df = torch.empty(100, device="cuda")
    ws = torch.empty(max(plan.ws_bytes, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(hd.HdcError) as e:  # the forward workspace is too small for the adjoint
        plan.backward_ptr(f.data_ptr(), g.data_ptr(), dh.data_ptr(), df.data_ptr(), None, ws.data_ptr(),
                          plan.ws_bytes, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == -3
    with pytest.raises(ValueError, match="extents"):  # a kernel longer than f: the binding rejects it
        hd.conv_forward(g, f)
    with pytest.raises(hd.HdcError) as e:  # and so does the library
        hd.Plan((10,), kernel_shape=(100,))
    assert e.value.status == -1


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,kshape,variant", [
    ((1000,), (37,), "hybrid_rcm"), ((12345,), (100,), "hybrid_rcm"), ((1 << 16,), (4096,), "hybrid_rcm"),
    ((300, 200), (31, 17), "hybrid_rcm"), ((64, 48), (40, 6), "hybrid_rcm"),
    ((1000,), (37,), "explicit_rcm"), ((300, 200), (31, 17), "explicit"), ((20, 18, 16), (5, 4, 3), "explicit_rcm"),
    ((20, 18, 16), (5, 4, 3), "hybrid_rcm"), ((16, 12, 10), (8, 6, 4), "hybrid_rcm"),
    ((1000,), (37,), "hybrid_cs"), ((1 << 16,), (4096,), "hybrid_cs"), ((300, 200), (31, 17), "hybrid_cs"),
    ((20, 18, 16), (5, 4, 3), "hybrid_cs"), ((1000,), (37,), "hybrid_mix"), ((4000,), (2000,), "hybrid_mix"),
])
def test_short_kernel_adjoint(hd, shape, kshape, variant, dtype):
    """df has f's extents; dg has g's: the gradient of the zero-extended kernel restricted to g's box."""
    import torch

    f = synth.normal(shape, 118, 0, synth.ROLE_F, dtype)
    g = synth.normal(kshape, 118, 0, synth.ROLE_G, dtype)
    u = synth.normal(shape, 118, 0, synth.ROLE_U, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    df, dg = hd.conv_backward(tf, tg, tu, variant=variant)
    df, dg = df.cpu().numpy(), dg.cpu().numpy()
    assert df.shape == f.shape and dg.shape == g.shape
    gz = zero_extend(g, f.shape)
    if f.size <= 70000:
        rdf, rdg = grad_direct(f, gz, u)
    else:
        rdf, rdg = fft_grad(f, gz, u)
    rdg = rdg[tuple(slice(0, n) for n in kshape)]
    _check(df, rdf, dtype, f"short kernel adjoint df {shape} * {kshape} {variant} {dtype}")
    _check(dg, rdg, dtype, f"short kernel adjoint dg {shape} * {kshape} {variant} {dtype}")


def test_short_kernel_autograd(hd):
    import torch

    f = torch.from_numpy(synth.normal((2, 500), 119, 0, synth.ROLE_F, "float64")).cuda().requires_grad_()
    g = torch.from_numpy(synth.normal((2, 31), 119, 0, synth.ROLE_G, "float64")).cuda().requires_grad_()
    h = hd.conv(f, g, ndim=1)
    assert h.shape == f.shape
    w = torch.from_numpy(synth.normal((2, 500), 119, 0, synth.ROLE_U, "float64")).cuda()
    (h * w).sum().backward()
    for b in range(2):
        fb, gb, wb = f[b].detach().cpu().numpy(), g[b].detach().cpu().numpy(), w[b].cpu().numpy()
        rdf, rdg = grad_direct(fb, zero_extend(gb, fb.shape), wb)
        _check(f.grad[b].cpu().numpy(), rdf, "float64", f"autograd short kernel df {b}")
        _check(g.grad[b].cpu().numpy(), rdg[:31], "float64", f"autograd short kernel dg {b}")


# ------------------------------------------------------------------ cached kernel spectra (Sec. 7)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,Lg,B", [(1 << 16, None, 1), (1 << 16, 4096, 2), (12345, 333, 1)])
def test_cached_kernel(hd, L, Lg, B, dtype):
    """Transform g once, convolve several f: bit for bit the plain forward, and the oracle's result."""
    import torch

    kshape = (L if Lg is None else Lg,)
    g = np.stack([synth.normal(kshape, 120, b, synth.ROLE_G, dtype) for b in range(B)])
    tg = torch.from_numpy(g).cuda()
    ck = hd.CachedKernel(tg, (L,))
    assert ck.plan.describe().startswith("col_fwd;line_rows"), ck.plan.describe()
    for k in range(3):
        f = np.stack([synth.normal((L,), 120 + k, b, synth.ROLE_F, dtype) for b in range(B)])
        tf = torch.from_numpy(f).cuda()
        h = ck(tf)
        assert torch.equal(h, hd.conv_forward(tf, tg, ndim=1)), f"call {k}: cached forward differs from the plain one"
        if k == 0:
            for b in range(B):
                _check(h[b].cpu().numpy(), fft_conv(f[b], g[b]), dtype, f"cached kernel L={L} Lg={Lg} item {b}")


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,kshape,B", [((1000,), None, 2), ((3001,), (37,), 1), ((64, 48), None, 2),
                                            ((300, 200), (31, 17), 1), ((16, 12, 10), None, 2),
                                            ((20, 18, 16), (5, 4, 3), 1)])
def test_cached_kernel_lines(hd, shape, kshape, B, dtype):
    """Cached spectra of one-workgroup 1D, 2D and 3D plans: bit for bit the plain forward, and the oracle."""
    import torch

    ks = shape if kshape is None else kshape
    g = np.stack([synth.normal(ks, 121, b, synth.ROLE_G, dtype) for b in range(B)])
    tg = torch.from_numpy(g).cuda()
    ck = hd.CachedKernel(tg, shape)
    for k in range(2):
        f = np.stack([synth.normal(shape, 121 + k, b, synth.ROLE_F, dtype) for b in range(B)])
        tf = torch.from_numpy(f).cuda()
        h = ck(tf)
        assert torch.equal(h, hd.conv_forward(tf, tg, ndim=len(shape))), f"{shape}: cached forward differs"
        if k == 0:
            for b in range(B):
                _check(h[b].cpu().numpy(), fft_conv(f[b], g[b]), dtype, f"cached {shape} * {ks} item {b}")


def test_cached_kernel_unsupported(hd):
    import torch

    with pytest.raises(hd.HdcError) as e:  # the conjugate-symmetry variant has no cached form
        p = hd.Plan((1000,), variant="hybrid_cs")
        p.spectrum_bytes()
    assert e.value.status == -2
    ck = hd.CachedKernel(torch.zeros(1 << 14, device="cuda"), (1 << 14,))
    with pytest.raises(ValueError):
        ck(torch.zeros(1 << 13, device="cuda"))


def test_usage_examples(hd):
    """The calls a user starts from, at small sizes: a differentiable batched convolution, the conjugate-symmetry
    variant, a shorter kernel given as a strided view, cached kernel spectra, an uneven batch and the autotuner."""
    import torch

    L, B = 1 << 15, 3
    f = torch.from_numpy(np.stack([synth.normal((L,), 130, b, synth.ROLE_F, "float32") for b in range(B)])).cuda()
    g = torch.from_numpy(np.stack([synth.normal((L,), 130, b, synth.ROLE_G, "float32") for b in range(B)])).cuda()
    fn, gn = f.cpu().numpy(), g.cpu().numpy()
    h = hd.conv(f, g, ndim=1)
    _check(h[1].cpu().numpy(), fft_conv(fn[1], gn[1]), "float32", "conv")
    h = hd.conv(f, g, ndim=1, variant="hybrid_cs")
    _check(h[2].cpu().numpy(), fft_conv(fn[2], gn[2]), "float32", "conv hybrid_cs")
    h = hd.conv(f, g[..., :300], ndim=1)
    _check(h[0].cpu().numpy(), fft_conv(fn[0], np.ascontiguousarray(gn[0, :300])), "float32", "conv shorter kernel view")
    k = hd.CachedKernel(g, (L,))
    assert torch.equal(k(f), hd.conv_forward(f, g, ndim=1))
    a = [torch.from_numpy(synth.normal(s, 131, i, synth.ROLE_F, "float32")).cuda()
         for i, s in enumerate([(1000,), (40, 30), (8, 9, 10)])]
    c = [torch.from_numpy(synth.normal(s, 131, i, synth.ROLE_G, "float32")).cuda()
         for i, s in enumerate([(1000,), (40, 30), (8, 9, 10)])]
    hs = hd.conv_batch(a, c)
    for x, y, z in zip(a, c, hs):
        _check(z.cpu().numpy(), fft_conv(x.cpu().numpy(), y.cpu().numpy()), "float32", f"conv_batch {tuple(x.shape)}")
    m = hd.autotune((64, 48), batch=2)
    assert len(m) == 2 and all(v > 0 for v in m), m
