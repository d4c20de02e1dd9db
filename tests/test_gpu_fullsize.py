"""GPU parity at the benchmark's full sizes, with the plans and batch sizes the
benchmark times (default FFT lengths, one plan for the whole batch).

  1D  L = 2^20, batch 64: FP32 hybridRCM (the headline), hybridCS and
      explicitRCM; FP64 hybridRCM and hybridCS.  Two whole pairs against oracle.fft_conv
      (normwise), and sampled outputs of every pair against the direct sum
      oracle.direct_conv_at: tile boundaries of the row length, the first and
      last index, and seeded random indices.
  2D  2048^2, batch 4, FP32 hybridRCM and hybridCS: one whole pair against
      fft_conv, samples of every pair against the direct sum.
  3D  256^3, batch 1, FP32 hybridRCM (spectral-field inputs): samples against the direct sum.

Inputs follow the benchmark's recipe (synth.pair_for with its configuration
numbers and value distributions).  Bars: normwise relative error <= 1e-5 in
FP32 and <= 1e-12 in FP64, for whole arrays and for each sample vector.
"""
import numpy as np
import pytest

from oracle import direct_conv_at, fft_conv, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}


def _inputs(cfg, shape, batch, dtype, dist):
    f = np.empty((batch,) + shape, dtype=dtype)
    g = np.empty_like(f)
    for b in range(batch):
        f[b], g[b] = synth.pair_for(cfg, b, shape, dtype, dist)
    return f, g


def _run(hd, f, g, variant, dtype):
    import torch

    shape = f.shape[1:]
    plan = hd.Plan(shape, variant=variant, dtype=dtype, batch=f.shape[0])
    tf, tg = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    th = torch.empty_like(tf)
    ws = torch.empty(max(plan.ws_bytes, 1), dtype=torch.uint8, device="cuda")
    plan.forward_ptr(tf.data_ptr(), tg.data_ptr(), th.data_ptr(), ws.data_ptr(), plan.ws_bytes,
                     torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return th.cpu().numpy(), plan


def _samples_1d(L, row, n, seed):
    a = np.random.default_rng(seed)
    idx = {0, 1, L - 1, L - 2, row - 1, row, 2 * row - 1, L // 2}
    idx |= set(int(x) for x in a.integers(0, L, n))
    return sorted(i for i in idx if 0 <= i < L)


@pytest.mark.parametrize("variant,dtype", [("hybrid_rcm", "float32"), ("hybrid_cs", "float32"),
                                           ("explicit_rcm", "float32"), ("hybrid_rcm", "float64"),
                                           ("hybrid_cs", "float64")])
def test_1d_full_size(hd, variant, dtype):
    L, B = 1 << 20, 64
    f, g = _inputs(2, (L,), B, dtype, "normal")
    h, plan = _run(hd, f, g, variant, dtype)
    print(f"1D {variant} {dtype}: plan {plan.describe()} {plan.resolved()}", flush=True)
    # real row length of the multi-pass form: twice the complex row length m
    row = 2 * plan.resolved()[0][0]
    for b in (0, B - 1):
        err = relerr(h[b], fft_conv(f[b], g[b]))
        print(f"  pair {b}: whole-array relerr {err:.3e}", flush=True)
        assert err <= TOL[dtype], f"pair {b}: {err:.3e}"
    worst = 0.0
    for b in range(B):
        idx = _samples_1d(L, row, 8, 1000 + b)
        err = relerr(h[b][idx], direct_conv_at(f[b], g[b], idx))
        worst = max(worst, err)
        assert err <= TOL[dtype], f"pair {b}: sampled relerr {err:.3e} at {idx}"
    print(f"  sampled outputs of all {B} pairs: max relerr {worst:.3e}", flush=True)


@pytest.mark.parametrize("variant", ["hybrid_rcm", "hybrid_cs"])
def test_2d_full_size(hd, variant):
    n, B, dtype = 2048, 4, "float32"
    f, g = _inputs(3, (n, n), B, dtype, "uniform")
    h, plan = _run(hd, f, g, variant, dtype)
    print(f"2D {variant}: plan {plan.describe()} {plan.resolved()}", flush=True)
    err = relerr(h[0], fft_conv(f[0], g[0]))
    print(f"  pair 0: whole-array relerr {err:.3e}", flush=True)
    assert err <= TOL[dtype]
    a = np.random.default_rng(2000)
    for b in range(B):
        idx = [(0, 0), (n - 1, n - 1), (n - 1, 0), (0, n - 1), (1023, 1024), (1024, 1023)]
        idx += [tuple(int(v) for v in a.integers(0, n, 2)) for _ in range(10)]
        ref = direct_conv_at(f[b], g[b], idx)
        got = np.array([h[b][i] for i in idx])
        err = relerr(got, ref)
        assert err <= TOL[dtype], f"pair {b}: sampled relerr {err:.3e}"


def test_3d_full_size(hd):
    n, dtype = 256, "float32"
    f, g = _inputs(4, (n, n, n), 1, dtype, "spectral")
    h, plan = _run(hd, f, g, "hybrid_rcm", dtype)
    print(f"3D: plan {plan.describe()} {plan.resolved()}", flush=True)
    a = np.random.default_rng(3000)
    idx = [(0, 0, 0), (n - 1, n - 1, n - 1), (n - 1, 0, 127), (0, n - 1, 128), (127, 128, n - 1)]
    idx += [tuple(int(v) for v in a.integers(0, n, 3)) for _ in range(24)]
    ref = direct_conv_at(f[0], g[0], idx)
    got = np.array([h[0][i] for i in idx])
    err = relerr(got, ref)
    print(f"  {len(idx)} sampled outputs: relerr {err:.3e}", flush=True)
    assert err <= TOL[dtype]
