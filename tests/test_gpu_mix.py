"""GPU parity: conjugate-symmetry residues with implicit packing for residues 0 and q/2.

In 2D/3D the first axis's residues 0 and q/2 run as an implicit-packing problem with q = 2 on that
axis (q = 1 for an odd q) scaled by 2/q, and the other residues add to its result through conjugate
symmetry.

HDC_HYBRID_MIX runs the residues 1 .. ceil(q/2) - 1 as the conjugate-symmetry
variant does (complex transforms, elementwise products) and the self-conjugate
residues 0 and q/2 through implicit packing at length m/2 (residue q/2 after a
twist, with the half-shifted RCM operator).  Checked against the oracle's direct
sums within 1e-12 (FP64) / 1e-5 (FP32), on exact integers, for the adjoint and
batches; the oracle's step-by-step form (oracle.hybrid.hybrid_mix_conv_1d) is
pinned to the same definition on the CPU.
"""
import numpy as np
import pytest

from oracle import direct_conv, fft_conv, grad_direct, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}

CASES = [
    # (L, M, m, q) in real units; None = planner default
    (1024, 2048, 512, 4),      # p = 2: residues 0, 1, 2 = q/2
    (1024, None, None, None), (1, None, None, None), (2, None, None, None), (3, None, None, None),
    (37, 80, 8, 10), (33, 66, 8, 9), (100, 199, 16, 13), (257, None, 64, None), (999, 2048, 256, 8),
    (2048, None, None, None), (50, 100, 2, 50), (3000, None, None, None), (64, 128, 64, 2), (40, 80, 16, 5),
]


def _run(hd, f, g, M, m, q):
    import torch

    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), M=None if M is None else (M,),
                        m=None if m is None else (m,), q=None if q is None else (q,), variant="hybrid_mix")
    return h.cpu().numpy()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L,M,m,q", CASES)
def test_1d_hybrid_mix(hd, L, M, m, q, dtype):
    f, g = synth.pair_for(180, L, (L,), dtype)
    plan = hd.get_plan((L,), None if M is None else (M,), None if m is None else (m,), None if q is None else (q,),
                       "hybrid_mix", dtype, 1)
    assert plan.describe() == "line_mix;", plan.describe()
    h = _run(hd, f, g, M, m, q)
    err = relerr(h, direct_conv(f, g))
    print(f"mix L={L} M={M} m={m} q={q} {dtype} {plan.resolved()}: relerr {err:.3e}", flush=True)
    assert np.all(np.isfinite(h)) and err <= TOL[dtype]


@pytest.mark.parametrize("name", ["int_1d_L37", "int_1d_L64"])
def test_hybrid_mix_golden_integers(hd, name):
    from tests.golden.make_golden import load

    f, g, h = load(name)
    out = _run(hd, f, g, None, None, None)
    assert np.array_equal(np.rint(out), h)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("L", [37, 1024, 3000])
def test_hybrid_mix_adjoint_and_batch(hd, L, dtype):
    import torch

    B = 3
    f = np.stack([synth.pair_for(181, b, (L,), dtype)[0] for b in range(B)])
    g = np.stack([synth.pair_for(181, b, (L,), dtype)[1] for b in range(B)])
    u = np.stack([synth.uniform((L,), 181, b, synth.ROLE_U, dtype) for b in range(B)])
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    h = hd.conv_forward(tf, tg, ndim=1, variant="hybrid_mix").cpu().numpy()
    df, dg = hd.conv_backward(tf, tg, tu, ndim=1, variant="hybrid_mix")
    for b in range(B):
        assert relerr(h[b], direct_conv(f[b], g[b])) <= TOL[dtype]
        rdf, rdg = grad_direct(f[b], g[b], u[b])
        assert relerr(df[b].cpu().numpy(), rdf) <= TOL[dtype]
        assert relerr(dg[b].cpu().numpy(), rdg) <= TOL[dtype]


# 2D / 3D: residues 0 and q/2 of the first axis through an implicit-packing plan with q = 2 on that axis
# (q = 1 for an odd q), the others through conjugate symmetry; (shape, M, m) with q on the first axis noted
CASES_ND = [
    ((64, 48), None, (16, 0)),         # q = 8: residues 1..3 conjugate-symmetric, 0 and 4 packed
    ((20, 30), None, (8, 0)),          # q = 5 (odd): residue 0 packed alone, 1 and 2 conjugate-symmetric
    ((9, 12), None, None),
    ((300, 200), None, None),          # q = 2: only the packed residues
    ((300, 200), None, (64, 0)),       # q = 10, p = 5
    ((33, 17), (100, 50), (16, 8)),
    ((128, 96), None, (32, 0)),
    ((16, 12, 10), None, (4, 0, 0)),   # 3D, q = 8
    ((20, 18, 33), None, (8, 0, 0)),   # 3D, q = 5
    ((5, 4, 6), None, None),
    ((32, 32, 32), None, (8, 0, 0)),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,M,m", CASES_ND)
def test_nd_hybrid_mix(hd, shape, M, m, dtype):
    import torch

    f, g = synth.pair_for(182, 0, shape, dtype, "normal")
    plan = hd.get_plan(shape, M, m, None, "hybrid_mix", dtype, 1)
    print(f"mix {shape} M={M} m={m} {dtype}: {plan.describe()} {plan.resolved()}", flush=True)
    assert plan.describe().startswith("col_fwd;")  # the packed residues' sub-plan runs first
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), M=M, m=m,
                        variant="hybrid_mix").cpu().numpy()
    ref = direct_conv(f, g) if f.size <= 20000 else fft_conv(f, g)
    err = relerr(h, ref)
    print(f"  relerr {err:.3e}", flush=True)
    assert np.all(np.isfinite(h)) and err <= TOL[dtype]
    # the same result as the conjugate-symmetry variant with the same first-axis m and q
    hc = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), M=M, m=m,
                         variant="hybrid_cs").cpu().numpy()
    assert relerr(h, hc) <= 4 * TOL[dtype]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,kshape,m", [((64, 48), (64, 48), (16, 0)), ((20, 30), (20, 30), (8, 0)),
                                            ((64, 48), (10, 7), (16, 0)), ((16, 12, 10), (16, 12, 10), (4, 0, 0)),
                                            ((20, 18, 33), (5, 4, 3), (8, 0, 0))])
def test_nd_hybrid_mix_adjoint_batch_short(hd, shape, kshape, m, dtype):
    """Batch of two, the adjoint, a shorter kernel: against the oracle's gradient of the zero-extended kernel."""
    import torch

    from oracle import zero_extend

    B = 2
    f = np.stack([synth.normal(shape, 183, b, synth.ROLE_F, dtype) for b in range(B)])
    g = np.stack([synth.normal(kshape, 183, b, synth.ROLE_G, dtype) for b in range(B)])
    u = np.stack([synth.normal(shape, 183, b, synth.ROLE_U, dtype) for b in range(B)])
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    nd = len(shape)
    h = hd.conv_forward(tf, tg, ndim=nd, m=m, variant="hybrid_mix").cpu().numpy()
    df, dg = hd.conv_backward(tf, tg, tu, ndim=nd, m=m, variant="hybrid_mix")
    for b in range(B):
        gz = zero_extend(g[b], shape)
        assert relerr(h[b], direct_conv(f[b], gz)) <= TOL[dtype], f"h {b}"
        rdf, rdg = grad_direct(f[b], gz, u[b])
        assert relerr(df[b].cpu().numpy(), rdf) <= TOL[dtype], f"df {b}"
        assert relerr(dg[b].cpu().numpy(), rdg[tuple(slice(0, k) for k in kshape)]) <= TOL[dtype], f"dg {b}"


def test_hybrid_mix_unsupported(hd):
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), m=(7,), variant="hybrid_mix")
    assert e.value.status == -1
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((1 << 20,), variant="hybrid_mix")  # the multi-pass form
    assert e.value.status == -2
