"""GPU: the shared-transform adjoint and the saved forward spectra.

For implicit-packing hybrid plans with equal extents, hdc_backward transforms
R(dh) once and multiplies its spectra with g's (df) and f's (dg) in one line
kernel launch; with HDC_SAVE_SPECTRA the forward leaves f's and g's outer-axis
transforms in the workspace and the backward takes them from there.

Checked: df and dg against the oracle's gradient (direct sums, or explicitly
padded FFT correlations at larger sizes) within 1e-12 (FP64) / 1e-5 (FP32);
agreement with the single-output adjoint (one correlation per call, which
transforms R(dh) again); bit-for-bit equality with and without saved spectra;
saved spectra are only used for the forward they came from.
"""
import numpy as np
import pytest

from oracle import fft_grad, grad_direct, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}

SHAPES = [(37,), (1000,), (5000,), (1 << 14,), (12345,), (9, 12), (64, 48), (300, 200), (5, 4, 6), (16, 12, 10),
          (20, 18, 33)]


def _check(x, ref, dtype, what):
    err = relerr(x, ref)
    print(f"{what}: relerr {err:.3e} (tol {TOL[dtype]:.0e})", flush=True)
    assert np.all(np.isfinite(x)), what
    assert err <= TOL[dtype], f"{what}: relerr {err:.3e}"


def _ref(f, g, u):
    return grad_direct(f, g, u) if f.size <= 3000 else fft_grad(f, g, u)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_shared_transform_adjoint(hd, shape, dtype):
    import torch

    f, g = synth.pair_for(150, 0, shape, dtype, "normal")
    u = synth.normal(shape, 150, 0, synth.ROLE_U, dtype)
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    df, dg = hd.conv_backward(tf, tg, tu)
    rdf, rdg = _ref(f, g, u)
    _check(df.cpu().numpy(), rdf, dtype, f"df {shape} {dtype}")
    _check(dg.cpu().numpy(), rdg, dtype, f"dg {shape} {dtype}")
    # one correlation per call (transforms R(dh) again): the same arithmetic, up to how the compiler
    # contracts the raw loads' kernel instantiations
    df1, _ = hd.conv_backward(tf, tg, tu, need_g=False)
    _, dg1 = hd.conv_backward(tf, tg, tu, need_f=False)
    close = {"float64": 1e-15, "float32": 1e-7}[dtype]
    assert relerr(df.cpu().numpy(), df1.cpu().numpy()) <= close, f"{shape} {dtype}: df vs single-output adjoint"
    assert relerr(dg.cpu().numpy(), dg1.cpu().numpy()) <= close, f"{shape} {dtype}: dg vs single-output adjoint"


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shape", [(1000,), (1 << 14,), (12345,), (64, 48), (300, 200), (16, 12, 10), (20, 18, 33)])
def test_saved_spectra_autograd(hd, shape, dtype):
    """conv(..., save_spectra=True): gradients bit for bit those of save_spectra=False, and the oracle's;
    a second backward through the same graph (retain_graph) reuses the spectra again."""
    import torch

    f, g = synth.pair_for(151, 0, shape, dtype, "normal")
    u = synth.normal(shape, 151, 0, synth.ROLE_U, dtype)
    tu = torch.from_numpy(u).cuda()
    grads = {}
    for save in (False, True):
        tf = torch.from_numpy(f).cuda().requires_grad_(True)
        tg = torch.from_numpy(g).cuda().requires_grad_(True)
        h = hd.conv(tf, tg, save_spectra=save)
        h.backward(tu, retain_graph=True)
        grads[save] = (tf.grad.clone(), tg.grad.clone())
        if save:
            tf.grad = None
            tg.grad = None
            h.backward(tu)
            assert torch.equal(tf.grad, grads[True][0]) and torch.equal(tg.grad, grads[True][1]), "second backward"
    assert torch.equal(grads[True][0], grads[False][0]), f"{shape} {dtype}: df with saved spectra differs"
    assert torch.equal(grads[True][1], grads[False][1]), f"{shape} {dtype}: dg with saved spectra differs"
    rdf, rdg = _ref(f, g, u)
    _check(grads[True][0].cpu().numpy(), rdf, dtype, f"saved df {shape} {dtype}")
    _check(grads[True][1].cpu().numpy(), rdg, dtype, f"saved dg {shape} {dtype}")


def test_saved_spectra_belong_to_their_forward(hd):
    """Two forwards on one plan with separate workspaces, then the backwards in reverse order: each
    backward gets its own forward's f and g (the older one transforms them again)."""
    import torch

    shape, dtype = (1 << 14,), "float32"
    us = [synth.normal(shape, 152, k, synth.ROLE_U, dtype) for k in range(2)]
    pairs = [synth.pair_for(152, k, shape, dtype, "normal") for k in range(2)]
    leaves, outs = [], []
    for (f, g) in pairs:
        tf = torch.from_numpy(f).cuda().requires_grad_(True)
        tg = torch.from_numpy(g).cuda().requires_grad_(True)
        leaves.append((tf, tg))
        outs.append(hd.conv(tf, tg))
    for k in (1, 0):
        outs[k].backward(torch.from_numpy(us[k]).cuda())
        rdf, rdg = fft_grad(pairs[k][0], pairs[k][1], us[k])
        _check(leaves[k][0].grad.cpu().numpy(), rdf, dtype, f"forward {k}: df")
        _check(leaves[k][1].grad.cpu().numpy(), rdg, dtype, f"forward {k}: dg")


def test_saved_spectra_flag_through_the_abi(hd):
    """The C ABI directly: a plan with HDC_SAVE_SPECTRA, hdc_forward then hdc_backward on the same pointers,
    equal to a plan without the flag; the forward's h is unchanged by the flag."""
    import torch

    shape, B, dtype = (256, 96), 3, "float64"
    f = np.stack([synth.normal(shape, 153, b, synth.ROLE_F, dtype) for b in range(B)])
    g = np.stack([synth.normal(shape, 153, b, synth.ROLE_G, dtype) for b in range(B)])
    u = np.stack([synth.normal(shape, 153, b, synth.ROLE_U, dtype) for b in range(B)])
    tf, tg, tu = (torch.from_numpy(x).cuda() for x in (f, g, u))
    st = torch.cuda.current_stream().cuda_stream
    res = {}
    for flags in (0, hd.HDC_SAVE_SPECTRA):
        plan = hd.Plan(shape, dtype=dtype, batch=B, flags=flags)
        nb = max(plan.ws_bytes, plan.bwd_ws_bytes)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        h, df, dg = torch.empty_like(tf), torch.empty_like(tf), torch.empty_like(tf)
        plan.forward_ptr(tf.data_ptr(), tg.data_ptr(), h.data_ptr(), ws.data_ptr(), nb, st)
        plan.backward_ptr(tf.data_ptr(), tg.data_ptr(), tu.data_ptr(), df.data_ptr(), dg.data_ptr(), ws.data_ptr(),
                          nb, st)
        torch.cuda.synchronize()
        res[flags] = (h.cpu(), df.cpu(), dg.cpu())
        if flags:
            assert plan.ws_bytes > hd.Plan(shape, dtype=dtype, batch=B).ws_bytes  # the product region
    for a, b_ in zip(res[0], res[hd.HDC_SAVE_SPECTRA]):
        assert torch.equal(a, b_)
    for b in range(B):
        rdf, rdg = fft_grad(f[b], g[b], u[b])
        _check(res[0][1][b].numpy(), rdf, dtype, f"abi df {b}")
        _check(res[0][2][b].numpy(), rdg, dtype, f"abi dg {b}")
