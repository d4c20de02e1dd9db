"""GPU: HDC_USE_GRAPH (the plan's launch sequence replayed from a captured hipGraph) and HDC_DETERMINISTIC.

A plan with HDC_USE_GRAPH gives bitwise the results of the same plan without it, forward and adjoint, on
replays with the same pointers (with other eager work queued between them), after a pointer change (captured
again) and with saved spectra; every variant's pass sequence is captured (one-workgroup 1D, multi-pass 1D, 2D,
3D, conjugate symmetry, the mixed variant's two pass sequences, explicit padding).  HDC_DETERMINISTIC makes
hdc_autotune return the planner's defaults without timing.
"""
import numpy as np
import pytest

from oracle import direct_conv, fft_conv, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

CASES = [((2000,), None, "hybrid_rcm"), ((1 << 16,), None, "hybrid_rcm"), ((300, 200), None, "hybrid_rcm"),
         ((16, 12, 10), None, "hybrid_rcm"), ((300, 200), None, "hybrid_cs"), ((1 << 16,), None, "hybrid_cs"),
         ((64, 48), (16, 0), "hybrid_mix"), ((1000,), None, "explicit_rcm"), ((40, 30), None, "explicit")]


def _run(torch, plan, f, g, h, ws):
    st = torch.cuda.current_stream().cuda_stream
    plan.forward_ptr(f.data_ptr(), g.data_ptr(), h.data_ptr(), ws.data_ptr(), plan.ws_bytes, st)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("shape,m,variant", CASES)
def test_graph_replay_forward_and_adjoint(hd, shape, m, variant, dtype):
    import torch

    B = 2
    f = torch.from_numpy(np.stack([synth.normal(shape, 190, b, synth.ROLE_F, dtype) for b in range(B)])).cuda()
    g = torch.from_numpy(np.stack([synth.normal(shape, 190, b, synth.ROLE_G, dtype) for b in range(B)])).cuda()
    u = torch.from_numpy(np.stack([synth.normal(shape, 190, b, synth.ROLE_U, dtype) for b in range(B)])).cuda()
    base = hd.Plan(shape, m=m, variant=variant, dtype=dtype, batch=B)
    gp = hd.Plan(shape, m=m, variant=variant, dtype=dtype, batch=B, flags=hd.HDC_USE_GRAPH)
    nb = max(base.ws_bytes, base.bwd_ws_bytes, gp.ws_bytes, gp.bwd_ws_bytes, 1)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    ref = torch.empty_like(f)
    _run(torch, base, f, g, ref, ws)
    rdf, rdg = torch.empty_like(f), torch.empty_like(f)
    base.backward_ptr(f.data_ptr(), g.data_ptr(), u.data_ptr(), rdf.data_ptr(), rdg.data_ptr(), ws.data_ptr(), nb, st)
    torch.cuda.synchronize()
    h = torch.empty_like(f)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        h.fill_(float("nan"))
        _run(torch, gp, f, g, h, ws)
        junk.add_(1.0)  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(h, ref), f"replay {rep}"
    h2 = torch.empty_like(f)  # another output pointer: captured again
    _run(torch, gp, f, g, h2, ws)
    torch.cuda.synchronize()
    assert torch.equal(h2, ref)
    for rep in range(2):
        df, dg = torch.full_like(f, float("nan")), torch.full_like(f, float("nan"))
        gp.backward_ptr(f.data_ptr(), g.data_ptr(), u.data_ptr(), df.data_ptr(), dg.data_ptr(), ws.data_ptr(), nb, st)
        torch.cuda.synchronize()
        assert torch.equal(df, rdf) and torch.equal(dg, rdg), f"adjoint replay {rep}"
    f0, g0 = f[0].double().cpu().numpy(), g[0].double().cpu().numpy()
    tol = 1e-5 if dtype == "float32" else 1e-12
    assert relerr(h[0].double().cpu().numpy(), direct_conv(f0, g0) if f0.size <= 20000 else fft_conv(f0, g0)) <= tol


@pytest.mark.parametrize("shape", [(1 << 14,), (256, 96), (20, 18, 16)])
def test_graph_with_saved_spectra(hd, shape):
    import torch

    dtype = "float32"
    f = torch.from_numpy(synth.normal(shape, 191, 0, synth.ROLE_F, dtype)).cuda()
    g = torch.from_numpy(synth.normal(shape, 191, 0, synth.ROLE_G, dtype)).cuda()
    u = torch.from_numpy(synth.normal(shape, 191, 0, synth.ROLE_U, dtype)).cuda()
    st = torch.cuda.current_stream().cuda_stream
    out = {}
    for flags in (hd.HDC_SAVE_SPECTRA, hd.HDC_SAVE_SPECTRA | hd.HDC_USE_GRAPH):
        plan = hd.Plan(shape, dtype=dtype, flags=flags)
        nb = max(plan.ws_bytes, plan.bwd_ws_bytes, 1)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        res = []
        for rep in range(2):
            h, df, dg = torch.empty_like(f), torch.empty_like(f), torch.empty_like(f)
            plan.forward_ptr(f.data_ptr(), g.data_ptr(), h.data_ptr(), ws.data_ptr(), nb, st)
            plan.backward_ptr(f.data_ptr(), g.data_ptr(), u.data_ptr(), df.data_ptr(), dg.data_ptr(), ws.data_ptr(),
                              nb, st)
            torch.cuda.synchronize()
            res.append((h.clone(), df.clone(), dg.clone()))
        out[flags] = res
    for a, b in zip(out[hd.HDC_SAVE_SPECTRA], out[hd.HDC_SAVE_SPECTRA | hd.HDC_USE_GRAPH]):
        for x, y in zip(a, b):
            assert torch.equal(x, y)


@pytest.mark.parametrize("shape,variant", [((1000,), "hybrid_rcm"), ((1 << 20,), "hybrid_rcm"), ((2048, 2048), "hybrid_rcm"),
                                           ((256, 256, 256), "hybrid_rcm"), ((2048, 2048), "hybrid_cs"),
                                           ((3000,), "hybrid_cs"), ((300, 200), "hybrid_mix"), ((64, 48, 40), "explicit_rcm")])
def test_deterministic_autotune_returns_defaults(hd, shape, variant):
    import time

    t0 = time.perf_counter()
    m1 = hd.autotune(shape, variant=variant, deterministic=True)
    m2 = hd.autotune(shape, variant=variant, deterministic=True)
    dt = time.perf_counter() - t0
    assert m1 == m2
    assert hd.Plan(shape, m=m1, variant=variant).resolved() == hd.Plan(shape, variant=variant).resolved(), (m1,)
    assert dt < 2.0, dt  # nothing timed
