"""GPU parity for plans the default cases do not reach, and memory-safety checks.

* The one-workgroup 1D line kernel at every FFT length the planner or the
  autotuner can choose for it (packed complex lengths 2048 and 4096 in FP32,
  1024 and 2048 in FP64), with three or four residues so that the compensated
  accumulation runs, forward and adjoint; and an uneven batch of such items.
* Planner defaults chosen by measurement, run once each against the oracle.
* Guard bands: every output (h, df, dg) is written into the middle of a larger
  buffer whose margins hold a sentinel; after the call the margins must be
  unchanged (odd extents, reversed adjoint stores, every variant).
* Strided axes padded beyond 4096 points (their single-level residue tables), every variant.
* Misaligned pointers are rejected; a NaN input is not silently dropped.

Bars as everywhere: normwise relative error <= 1e-12 (FP64), <= 1e-5 (FP32)
against the oracle's direct sums or its explicitly padded FFT convolution.
"""
import numpy as np
import pytest

from oracle import direct_conv, fft_conv, fft_grad, grad_direct, relerr, zero_extend
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}


def _check(h, ref, dtype, what):
    err = relerr(h, ref)
    print(f"{what}: relerr {err:.3e} (tol {TOL[dtype]:.0e})", flush=True)
    assert np.all(np.isfinite(h)), what
    assert err <= TOL[dtype], f"{what}: relerr {err:.3e}"


# ------------------------------------------------------------------ long lines (the autotuner's candidates)
# (L, M, m in real units, dtype, expected passes, expected packed FFT length, expected residues).  One
# workgroup holds a line of complex 2048 (FP32) or 1024 (FP64) only as a single block; longer lines per lane
# would spill, so those m take the multi-pass form with rows of m/2.
ONE_WG_LONG = [
    (5000, None, 4096, "float32", "col_fwd;line_rows;col_inv;", 2048, None),
    (8192, None, 4096, "float32", "col_fwd;line_rows;col_inv;", 2048, None),
    (3000, 8000, 4096, "float32", "line_1d;", 2048, 2),      # one block of 2048
    (6000, None, 8192, "float32", "col_fwd;line_rows;col_inv;", 4096, None),
    (8192, None, 8192, "float32", "col_fwd;line_rows;col_inv;", 4096, None),
    (1500, 5000, 2048, "float64", "line_1d;", 1024, 3),      # FP64 complex 1024 with three residues
    (2000, None, 2048, "float64", "line_1d;", 1024, 2),
    (4000, None, 4096, "float64", "col_fwd;line_rows;col_inv;", 2048, None),
    (3001, None, 4096, "float64", "col_fwd;line_rows;col_inv;", 2048, None),  # odd length
]


@pytest.mark.parametrize("L,M,m,dtype,passes,mc,q", ONE_WG_LONG)
def test_one_workgroup_long_lines(hd, L, M, m, dtype, passes, mc, q):
    import torch

    plan = hd.get_plan((L,), None if M is None else (M,), (m,), None, "hybrid_rcm", dtype, 1)
    assert plan.describe() == passes, plan.describe()
    assert plan.resolved()[0] == (mc,), plan.resolved()
    if q is not None:
        assert plan.resolved()[2] == (q,), plan.resolved()
    f, g = synth.pair_for(140, L, (L,), dtype, "normal")
    u = synth.normal((L,), 140, L, synth.ROLE_U, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    kw = dict(M=None if M is None else (M,), m=(m,))
    h = hd.conv_forward(tf, tg, **kw).cpu().numpy()
    _check(h, fft_conv(f, g, M=kw["M"]), dtype, f"one workgroup L={L} m={m} {dtype}")
    df, dg = hd.conv_backward(tf, tg, tu, **kw)
    rdf, rdg = fft_grad(f, g, u)
    _check(df.cpu().numpy(), rdf, dtype, f"one workgroup adjoint df L={L} m={m} {dtype}")
    _check(dg.cpu().numpy(), rdg, dtype, f"one workgroup adjoint dg L={L} m={m} {dtype}")


def test_uneven_batch_with_long_lines(hd):
    """Uneven-batch items forced onto the long one-workgroup lines, as the autotuner may choose them:
    grouped launches equal the single calls bit for bit and the oracle within tolerance."""
    import torch

    items = [((5000,), (4096,)), ((8192,), (4096,)), ((6000,), (8192,)), ((3001,), (4096,)), ((8192,), (8192,)),
             ((700,), (4096,)), ((4100,), (8192,)), ((300,), None), ((1 << 14,), None), ((64, 48), None)]
    shapes = [s for s, _ in items]
    ms = [m for _, m in items]
    fs, gs = [], []
    for i, s in enumerate(shapes):
        f, g = synth.pair_for(141, i, s, "float32", "uniform")
        fs.append(torch.from_numpy(f).cuda())
        gs.append(torch.from_numpy(g).cuda())
    plan = hd.BatchPlan([{"shape": s, "m": m} for s, m in zip(shapes, ms)], "float32")
    for rep in range(2):
        hs = hd.conv_batch(fs, gs, plan)
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            h1 = hd.conv_forward(fs[i], gs[i], m=ms[i]).cpu()
            assert torch.equal(hs[i].cpu(), h1), f"rep {rep} item {i} {s} m={ms[i]}"
    for i, s in enumerate(shapes):
        _check(hs[i].cpu().numpy(), fft_conv(fs[i].cpu().numpy(), gs[i].cpu().numpy()), "float32",
               f"batch item {i} {s} m={ms[i]}")


# ------------------------------------------------------------------ planner defaults
@pytest.mark.parametrize("shape,variant,dtype", [
    ((3000,), "hybrid_cs", "float32"),     # one workgroup, m = 1024, three blocks, q = 6
    ((3000,), "hybrid_cs", "float64"),
    ((40, 400), "hybrid_rcm", "float32"),  # one residue on a packed last axis of 512 points
    ((16, 512), "hybrid_rcm", "float32"),
    ((4, 4, 300), "hybrid_rcm", "float64"),  # one residue on the FP64 3D last axis
    ((64, 64, 64), "hybrid_rcm", "float32"),
    ((384, 512), "hybrid_rcm", "float32"),
])
def test_planner_default_parity(hd, shape, variant, dtype):
    import torch

    f, g = synth.pair_for(142, 0, shape, dtype)
    plan = hd.get_plan(shape, None, None, None, variant, dtype, 1)
    print(f"{shape} {variant} {dtype}: {plan.describe()} {plan.resolved()}", flush=True)
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), variant=variant).cpu().numpy()
    ref = direct_conv(f, g) if np.prod(shape) <= 5000 else fft_conv(f, g)
    _check(h, ref, dtype, f"planner default {shape} {variant} {dtype}")


# ------------------------------------------------------------------ long strided axes
# The residue tables of the strided axes are single-level: above 4096 points their entries are still read with
# one load (no two-level product).  Strided axes whose padded length q m exceeds 4096: axis 0 of a 2D problem,
# axis 1 of a 3D one, axis 0 of a 3D one; every variant that runs column passes, both precisions.
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,variant", [
    ((3000, 6), "hybrid_rcm"), ((3000, 6), "hybrid_cs"), ((3000, 6), "explicit_rcm"), ((3000, 6), "hybrid_mix"),
    ((2, 2500, 4), "hybrid_rcm"), ((2500, 3, 4), "hybrid_rcm"), ((2500, 3, 4), "hybrid_cs"),
])
def test_long_strided_axes(hd, shape, variant, dtype):
    import torch

    f, g = synth.pair_for(143, 0, shape, dtype)
    plan = hd.get_plan(shape, None, None, None, variant, dtype, 1)
    print(f"{shape} {variant} {dtype}: {plan.describe()} {plan.resolved()}", flush=True)
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), variant=variant).cpu().numpy()
    _check(h, fft_conv(f, g), dtype, f"long strided axis {shape} {variant} {dtype}")


# ------------------------------------------------------------------ guard bands
SENT = 12345.5  # exactly representable in both precisions


def _guarded(torch, n, dtype, pad=64):
    buf = torch.full((pad + n + pad,), SENT, dtype=dtype, device="cuda")
    return buf, buf[pad:pad + n]


def _margins_ok(buf, n, pad=64):
    b = buf.cpu().numpy()
    return bool(np.all(b[:pad] == SENT) and np.all(b[pad + n:] == SENT))


GUARD_CASES = [
    ((37,), None, "hybrid_rcm"), ((1001,), None, "hybrid_rcm"), ((12345,), None, "hybrid_rcm"),
    ((33, 17), None, "hybrid_rcm"), ((7, 9, 11), None, "hybrid_rcm"),
    ((37,), None, "hybrid_cs"), ((12345,), None, "hybrid_cs"), ((33, 17), None, "hybrid_cs"),
    ((7, 9, 11), None, "hybrid_cs"),
    ((37,), None, "explicit_rcm"), ((33, 17), None, "explicit"), ((7, 9, 11), None, "explicit_rcm"),
    ((1001,), (37,), "hybrid_rcm"), ((33, 17), (5, 3), "hybrid_rcm"), ((7, 9, 11), (3, 4, 5), "hybrid_rcm"),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,kshape,variant", GUARD_CASES)
def test_guard_bands(hd, shape, kshape, variant, dtype):
    import torch

    tdt = torch.float64 if dtype == "float64" else torch.float32
    ks = shape if kshape is None else kshape
    n, ng = int(np.prod(shape)), int(np.prod(ks))
    f = synth.normal(shape, 143, 0, synth.ROLE_F, dtype)
    g = synth.normal(ks, 143, 0, synth.ROLE_G, dtype)
    u = synth.normal(shape, 143, 0, synth.ROLE_U, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    plan = hd.Plan(shape, variant=variant, dtype=dtype, kernel_shape=kshape)
    st = torch.cuda.current_stream().cuda_stream
    ws = torch.empty(max(plan.bwd_ws_bytes, 1), dtype=torch.uint8, device="cuda")
    hb, h = _guarded(torch, n, tdt)
    plan.forward_ptr(tf.data_ptr(), tg.data_ptr(), h.data_ptr(), ws.data_ptr(), plan.ws_bytes, st)
    dfb, df = _guarded(torch, n, tdt)
    dgb, dg = _guarded(torch, ng, tdt)
    plan.backward_ptr(tf.data_ptr(), tg.data_ptr(), tu.data_ptr(), df.data_ptr(), dg.data_ptr(), ws.data_ptr(),
                      plan.bwd_ws_bytes, st)
    torch.cuda.synchronize()
    assert _margins_ok(hb, n), f"h margins overwritten: {shape} {variant}"
    assert _margins_ok(dfb, n), f"df margins overwritten: {shape} {variant}"
    assert _margins_ok(dgb, ng), f"dg margins overwritten: {shape} {variant}"
    gz = zero_extend(g, f.shape)
    _check(h.cpu().numpy().reshape(shape), direct_conv(f, gz), dtype, f"guarded h {shape} {variant}")
    rdf, rdg = grad_direct(f, gz, u)
    _check(df.cpu().numpy().reshape(shape), rdf, dtype, f"guarded df {shape} {variant}")
    _check(dg.cpu().numpy().reshape(ks), rdg[tuple(slice(0, k) for k in ks)], dtype, f"guarded dg {shape} {variant}")


# ------------------------------------------------------------------ alignment and NaN
def test_misaligned_pointers_rejected(hd):
    import torch

    plan = hd.Plan((100,), dtype="float32")
    f = torch.zeros(1024, device="cuda")
    ws = torch.empty(max(plan.ws_bytes, 1), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(hd.HdcError) as e:  # 4-byte offset: not 8-byte aligned
        plan.forward_ptr(f.data_ptr() + 4, f.data_ptr(), f.data_ptr() + 4, ws.data_ptr(), plan.ws_bytes, st)
    assert e.value.status == -1
    plan64 = hd.Plan((100,), dtype="float64")
    d = torch.zeros(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(hd.HdcError) as e:  # 8-byte offset: not 16-byte aligned
        plan64.forward_ptr(d.data_ptr(), d.data_ptr() + 8, d.data_ptr() + 16 * 8, ws.data_ptr(), plan64.ws_bytes, st)
    assert e.value.status == -1


@pytest.mark.parametrize("shape", [(1000,), (1 << 14,), (64, 48)])
def test_nan_input_propagates(hd, shape):
    import torch

    f, g = synth.pair_for(144, 0, shape, "float32")
    f.reshape(-1)[5] = np.nan
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()).cpu().numpy()
    assert np.isnan(h).any(), f"{shape}: NaN input produced an all-finite output"


# ------------------------------------------------------------------ batched adjoint without a plan
def test_batch_backward_short_kernel_without_plan(hd):
    """The default batch plan carries every item's kernel extents, so a shorter kernel's gradient has g's
    extents and matches the per-item adjoint (it is not read or written as f-sized)."""
    import torch

    fs = [torch.from_numpy(synth.normal((1000,), 145, 0, synth.ROLE_F, "float32")).cuda(),
          torch.from_numpy(synth.normal((64, 48), 145, 1, synth.ROLE_F, "float32")).cuda()]
    gs = [torch.from_numpy(synth.normal((37,), 145, 0, synth.ROLE_G, "float32")).cuda(),
          torch.from_numpy(synth.normal((64, 48), 145, 1, synth.ROLE_G, "float32")).cuda()]
    dhs = [torch.from_numpy(synth.normal(tuple(f.shape), 145, i, synth.ROLE_U, "float32")).cuda()
           for i, f in enumerate(fs)]
    dfs, dgs = hd.conv_batch_backward(fs, gs, dhs)
    for i in range(2):
        df1, dg1 = hd.conv_backward(fs[i], gs[i], dhs[i])
        assert dgs[i].shape == gs[i].shape
        assert torch.equal(dfs[i], df1) and torch.equal(dgs[i], dg1), f"item {i}"
