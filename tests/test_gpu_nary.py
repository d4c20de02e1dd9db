"""GPU parity: implicitly packed convolution of n > 2 real arrays (Sec. 4.1).

hdc_forward_n with nin = 3..8 arrays combines the packed spectra pairwise by the
recursion R^j = R^{j-1} [.] F^j (eqs. (Akn), (Rnk), (RnMk)) inside the line
kernels.  Checked against the oracle's n-fold truncated convolution (direct
sums, or its explicitly padded FFT form at larger sizes) within 1e-12 (FP64) /
1e-5 (FP32), on exact small integers, with n = 2 equal to hdc_forward, and the
error paths.
"""
import numpy as np
import pytest

from oracle import direct_conv_nary, fft_conv_nary, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}

CASES = [
    # (shape, n, M or None, m or None)
    ((37,), 3, None, None), ((1000,), 3, None, None), ((1000,), 4, None, None), ((999,), 5, None, None),
    ((3000,), 3, None, None), ((1,), 3, None, None), ((2,), 8, None, None),
    ((1 << 14,), 3, None, None), ((12345,), 3, None, None), ((1 << 14,), 4, None, None), ((20000,), 6, None, None),
    ((1 << 14,), 3, None, (2048,)),                    # multi-pass rows of 1024 given
    ((9, 12), 3, None, None), ((64, 48), 3, None, None), ((100, 75), 4, None, None), ((300, 200), 3, None, None),
    ((33, 17), 3, (100, 50), (16, 8)),
    ((5, 4, 6), 3, None, None), ((16, 12, 10), 3, None, None), ((20, 18, 33), 4, None, None),
]


def _inputs(shape, n, dtype, cfg=170):
    return [synth.uniform(shape, cfg, i, synth.ROLE_F, dtype) for i in range(n)]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape,n,M,m", CASES)
def test_nary(hd, shape, n, M, m, dtype):
    import torch

    xs = _inputs(shape, n, dtype)
    plan = hd.get_plan(shape, M, m, None, "hybrid_rcm", dtype, 1, None, 0, n)
    print(f"{shape} n={n} {dtype}: {plan.describe()} {plan.resolved()}", flush=True)
    h = hd.conv_nary([torch.from_numpy(x).cuda() for x in xs], M=M, m=m).cpu().numpy()
    ref = direct_conv_nary(xs) if np.prod(shape) <= 2000 else fft_conv_nary(xs)
    err = relerr(h, ref)
    print(f"  relerr {err:.3e}", flush=True)
    assert np.all(np.isfinite(h)) and err <= TOL[dtype], f"{shape} n={n} {dtype}: {err:.3e}"


@pytest.mark.parametrize("shape,n", [((40,), 3), ((64,), 4), ((9, 10), 3), ((4, 5, 6), 3)])
def test_nary_exact_integers(hd, shape, n):
    import torch

    xs = [synth.small_ints(shape, 171, i, synth.ROLE_F, dtype=np.float64) for i in range(n)]
    h = hd.conv_nary([torch.from_numpy(x).cuda() for x in xs]).cpu().numpy()
    ref = direct_conv_nary(xs)  # small integers: every sum is exact in float64
    assert np.array_equal(np.rint(h), ref) and np.max(np.abs(h - ref)) < 1e-8


def test_nary_batch_and_binary(hd):
    import torch

    B, shape = 3, (2000,)
    xs = [np.stack([synth.normal(shape, 172, b * 8 + i, synth.ROLE_F, "float32") for b in range(B)])
          for i in range(3)]
    h = hd.conv_nary([torch.from_numpy(x).cuda() for x in xs], ndim=1).cpu().numpy()
    for b in range(B):
        err = relerr(h[b], direct_conv_nary([x[b] for x in xs]))
        assert err <= TOL["float32"], f"batch item {b}: {err:.3e}"
    # n = 2 is the binary convolution
    t0, t1 = torch.from_numpy(xs[0]).cuda(), torch.from_numpy(xs[1]).cuda()
    assert torch.equal(hd.conv_nary([t0, t1], ndim=1), hd.conv_forward(t0, t1, ndim=1))


def test_nary_errors(hd):
    import torch

    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), nin=9)
    assert e.value.status == -1
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), nin=3, variant="hybrid_cs")
    assert e.value.status == -2
    with pytest.raises(hd.HdcError) as e:
        hd.Plan((100,), nin=3, M=(297,))  # M < n (L - 1) + 1 = 298
    assert e.value.status == -1
    plan = hd.Plan((100,), nin=3)
    x = torch.zeros(100, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(hd.HdcError) as e:  # the binary entry point on a 3-array plan
        plan.forward_ptr(x.data_ptr(), x.data_ptr(), x.data_ptr(), None, 0, st)
    assert e.value.status == -1
    with pytest.raises(hd.HdcError) as e:
        plan.backward_ptr(x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), None, 0, st)
    assert e.value.status == -2
