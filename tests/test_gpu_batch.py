"""GPU: uneven batches (grouped launches, hipGraph replay) and the autotuner.

A batch item runs the same kernels on the same data as a single-problem call,
so batch results must equal the per-item hdc_forward / hdc_backward results
bit for bit; a sample of items is also checked against the oracle with the
usual tolerances (normwise relative error <= 1e-12 float64, <= 1e-5 float32).
"""
import numpy as np
import pytest

from oracle import direct_conv, fft_conv, grad_direct, relerr
from paper_2608_14497_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5}

# mixed shapes: one-workgroup 1D, multi-pass 1D (two row lengths, ragged), 2D, 3D
MIXED = [(37,), (1024,), (300,), (4096,), (1 << 14,), (12345,), (1 << 16,), (9, 12), (64, 48), (128, 128),
         (5, 4, 6), (16, 12, 10), (1,), (2,), (7, 3)]


def _pairs(shapes, dtype, cfg=501):
    import torch

    fs, gs = [], []
    for i, s in enumerate(shapes):
        f, g = synth.pair_for(cfg, i, s, dtype)
        fs.append(torch.from_numpy(f).cuda())
        gs.append(torch.from_numpy(g).cuda())
    return fs, gs


def _ref(f, g):
    return direct_conv(f, g) if f.size <= 4096 else fft_conv(f, g)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batch_equals_single_calls(hd, dtype):
    import torch

    fs, gs = _pairs(MIXED, dtype)
    plan = hd.BatchPlan([{"shape": s} for s in MIXED], dtype)
    hs = hd.conv_batch(fs, gs, plan)
    torch.cuda.synchronize()
    for i, s in enumerate(MIXED):
        h1 = hd.conv_forward(fs[i], gs[i]).cpu().numpy()
        hb = hs[i].cpu().numpy()
        assert np.array_equal(hb, h1), f"item {i} shape {s}: batch differs from the single call"
        f, g = fs[i].cpu().numpy(), gs[i].cpu().numpy()
        err = relerr(hb, _ref(f, g))
        print(f"item {i} {s} {dtype}: relerr {err:.3e}", flush=True)
        assert err <= TOL[dtype], f"item {i} {s}: relerr {err:.3e}"


@pytest.mark.parametrize("graph", [True, False])
def test_batch_replays_and_pointer_changes(hd, graph, monkeypatch):
    """Replays with eager work in between, then new buffers (tables rewritten)."""
    import torch

    if not graph:
        monkeypatch.setenv("HDC_BATCH_NO_GRAPH", "1")
    shapes = MIXED[:11]
    dtype = "float32"
    plan = hd.BatchPlan([{"shape": s} for s in shapes], dtype)
    fs, gs = _pairs(shapes, dtype)
    want = [hd.conv_forward(f, g).cpu() for f, g in zip(fs, gs)]
    hs = [torch.empty_like(f) for f in fs]
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for h in hs:
            h.fill_(float("nan"))
        hd.conv_batch(fs, gs, plan, out=hs)
        # unrelated eager work and a synchronisation between replays
        scratch.mul_(1.0001).add_(0.5)
        _ = hd.conv_forward(fs[1], gs[1])
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(hs[i].cpu(), want[i]), f"replay {rep}, item {i} {shapes[i]}"
    # new input and output buffers: the parameter tables must follow them
    fs2, gs2 = _pairs(shapes, dtype, cfg=502)
    want2 = [hd.conv_forward(f, g).cpu() for f, g in zip(fs2, gs2)]
    for rep in range(2):
        hs2 = hd.conv_batch(fs2, gs2, plan)
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(hs2[i].cpu(), want2[i]), f"new buffers, replay {rep}, item {i}"
    # and back to the first set
    hd.conv_batch(fs, gs, plan, out=hs)
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        assert torch.equal(hs[i].cpu(), want[i]), f"first buffers again, item {i}"


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batch_backward_equals_single_calls(hd, dtype):
    import torch

    shapes = [(37,), (1024,), (1 << 14,), (9, 12), (5, 4, 6), (300,)]
    fs, gs = _pairs(shapes, dtype, cfg=503)
    dhs, _ = _pairs(shapes, dtype, cfg=504)
    plan = hd.BatchPlan([{"shape": s} for s in shapes], dtype)
    for rep in range(2):
        dfs, dgs = hd.conv_batch_backward(fs, gs, dhs, plan)
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            df1, dg1 = hd.conv_backward(fs[i], gs[i], dhs[i])
            assert torch.equal(dfs[i].cpu(), df1.cpu()), f"rep {rep} item {i} {s}: df"
            assert torch.equal(dgs[i].cpu(), dg1.cpu()), f"rep {rep} item {i} {s}: dg"
            if rep == 0 and np.prod(s) <= 1100:
                f, g, dh = fs[i].cpu().numpy(), gs[i].cpu().numpy(), dhs[i].cpu().numpy()
                rdf, rdg = grad_direct(f, g, dh)
                e1, e2 = relerr(dfs[i].cpu().numpy(), rdf), relerr(dgs[i].cpu().numpy(), rdg)
                print(f"item {i} {s} {dtype}: df {e1:.3e} dg {e2:.3e}", flush=True)
                assert e1 <= TOL[dtype] and e2 <= TOL[dtype]


@pytest.mark.parametrize("graph", [True, False])
def test_batch_dominant_component_split_across_lanes(hd, graph, monkeypatch):
    """A batch whose items mostly share their launch groups: the component they form costs more than an even
    share of the four stream lanes, so it is dealt to the lanes by launch-sequence class (the ten equal 1D items
    form one class larger than a share: dealt item by item) and its groups split by lane.  Forward and adjoint
    must still equal the per-item calls bit for bit, on replays too."""
    import torch

    if not graph:
        monkeypatch.setenv("HDC_BATCH_NO_GRAPH", "1")
    shapes = [(1 << 14,)] * 10 + [(12345,)] * 3 + [(1 << 16,)] * 2 + [(64, 48), (5, 4, 6), (300,)]
    dtype = "float32"
    fs, gs = _pairs(shapes, dtype, cfg=506)
    dhs, _ = _pairs(shapes, dtype, cfg=507)
    plan = hd.BatchPlan([{"shape": s} for s in shapes], dtype)
    want = [hd.conv_forward(f, g).cpu() for f, g in zip(fs, gs)]
    wantb = [tuple(x.cpu() for x in hd.conv_backward(f, g, dh)) for f, g, dh in zip(fs, gs, dhs)]
    for rep in range(3):
        hs = hd.conv_batch(fs, gs, plan)
        dfs, dgs = hd.conv_batch_backward(fs, gs, dhs, plan)
        torch.cuda.synchronize()
        for i, sh in enumerate(shapes):
            assert torch.equal(hs[i].cpu(), want[i]), f"rep {rep} item {i} {sh}: h"
            assert torch.equal(dfs[i].cpu(), wantb[i][0]), f"rep {rep} item {i} {sh}: df"
            assert torch.equal(dgs[i].cpu(), wantb[i][1]), f"rep {rep} item {i} {sh}: dg"
    for i in (0, 10, 13, 15, 16):
        f, g = fs[i].cpu().numpy(), gs[i].cpu().numpy()
        err = relerr(hs[i].cpu().numpy(), _ref(f, g))
        print(f"item {i} {shapes[i]}: relerr {err:.3e}", flush=True)
        assert err <= TOL[dtype]


@pytest.mark.parametrize("variant", ["hybrid_cs", "explicit_rcm", "explicit"])
def test_batch_per_item_variants(hd, variant):
    """Variants with per-item launches (padding copies, conjugate-symmetry passes) run ungraphed."""
    import torch

    shapes = [(37,), (1024,), (9, 12), (5, 4, 6), (64, 48)]
    fs, gs = _pairs(shapes, "float64", cfg=505)
    plan = hd.BatchPlan([{"shape": s, "variant": variant} for s in shapes], "float64")
    for rep in range(2):
        hs = hd.conv_batch(fs, gs, plan)
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            h1 = hd.conv_forward(fs[i], gs[i], variant=variant).cpu()
            assert torch.equal(hs[i].cpu(), h1), f"{variant} rep {rep} item {i} {s}"
            err = relerr(hs[i].cpu().numpy(), _ref(fs[i].cpu().numpy(), gs[i].cpu().numpy()))
            assert err <= TOL["float64"], f"{variant} item {i}: {err:.3e}"


def test_batch_uneven_workload_sample(hd):
    """A scaled-down uneven batch of the benchmark's mix (log-uniform 1D, 2D, 3D)."""
    import torch

    a = np.random.default_rng(7)
    shapes = [(int(round(2.0 ** a.uniform(4.0, 15.0))),) for _ in range(40)]
    shapes += [(int(a.choice([16, 48, 128])), int(a.choice([16, 48, 128]))) for _ in range(6)]
    shapes += [(8, 8, 8), (12, 12, 12)]
    fs, gs = _pairs(shapes, "float32", cfg=506)
    plan = hd.BatchPlan([{"shape": s} for s in shapes], "float32")
    hs = hd.conv_batch(fs, gs, plan)
    torch.cuda.synchronize()
    for i, s in enumerate(shapes):
        h1 = hd.conv_forward(fs[i], gs[i]).cpu()
        assert torch.equal(hs[i].cpu(), h1), f"item {i} {s}"
    for i in range(0, len(shapes), 7):
        err = relerr(hs[i].cpu().numpy(), _ref(fs[i].cpu().numpy(), gs[i].cpu().numpy()))
        assert err <= TOL["float32"], f"item {i} {shapes[i]}: {err:.3e}"


def test_batch_errors(hd):
    import torch

    shapes = [(1 << 14,), (64, 48)]
    plan = hd.BatchPlan([{"shape": s} for s in shapes], "float32")
    assert plan.ws_bytes > 0
    fs, gs = _pairs(shapes, "float32")
    hs = [torch.empty_like(f) for f in fs]
    with pytest.raises(hd.HdcError) as e:
        plan.forward_ptr([f.data_ptr() for f in fs], [g.data_ptr() for g in gs], [h.data_ptr() for h in hs],
                         None, 0, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == -3
    with pytest.raises(hd.HdcError) as e:
        hd.BatchPlan([{"shape": (37,)}, {"shape": (16, 12), "m": (5, 0)}], "float32")
    assert "item 1" in str(e.value)


def test_autotune(hd, tmp_path):
    import torch

    cache = tmp_path / "tune.txt"
    shape = (1 << 16,)
    m = hd.autotune(shape, dtype="float32", batch=4, cache_path=cache)
    assert len(m) == 1 and m[0] > 0 and (m[0] & (m[0] - 1)) == 0
    text = cache.read_text()
    assert text.count("|") == 1 and text.strip().endswith(f"{m[0]} 0 0")
    # a second call reads the cache
    assert hd.autotune(shape, dtype="float32", batch=4, cache_path=cache) == m
    assert cache.read_text() == text
    f, g = synth.pair_for(507, 0, shape, "float32")
    tf, tg = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    h = hd.conv_forward(tf, tg, m=m).cpu().numpy()
    assert relerr(h, fft_conv(f, g)) <= TOL["float32"]
    # a 2D case tunes both axes
    m2 = hd.autotune((96, 80), dtype="float64")
    assert len(m2) == 2 and all(x > 0 for x in m2)
    f, g = synth.pair_for(507, 1, (96, 80), "float64")
    h = hd.conv_forward(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), m=m2).cpu().numpy()
    assert relerr(h, direct_conv(f, g)) <= TOL["float64"]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batch_short_kernels(hd, dtype):
    """Items with shorter kernels (Sec. 7) in grouped launches: equal to the per-item calls, and to the oracle."""
    import torch

    from oracle import zero_extend

    items = [((1000,), (37,)), ((12345,), (100,)), ((1 << 14,), (1 << 14,)), ((1 << 14,), (512,)),
             ((300, 200), (31, 17)), ((64, 48), (40, 6)), ((64, 48), (64, 48)), ((16, 12, 10), (8, 6, 4)),
             ((20, 18, 16), (5, 4, 3))]
    fs, gs = [], []
    for i, (s, k) in enumerate(items):
        fs.append(torch.from_numpy(synth.normal(s, 508, i, synth.ROLE_F, dtype)).cuda())
        gs.append(torch.from_numpy(synth.normal(k, 508, i, synth.ROLE_G, dtype)).cuda())
    plan = hd.BatchPlan([{"shape": s, "kernel_shape": k} for s, k in items], dtype)
    for rep in range(2):
        hs = hd.conv_batch(fs, gs, plan)
        torch.cuda.synchronize()
        for i, (s, k) in enumerate(items):
            h1 = hd.conv_forward(fs[i], gs[i]).cpu()
            assert torch.equal(hs[i].cpu(), h1), f"rep {rep} item {i} {s} * {k}"
            if rep == 0:
                f, g = fs[i].cpu().numpy(), gs[i].cpu().numpy()
                err = relerr(hs[i].cpu().numpy(), fft_conv(f, zero_extend(g, f.shape)))
                assert err <= TOL[dtype], f"item {i} {s} * {k}: {err:.3e}"
    # the batched adjoint: df has f's extents, dg g's; equal to the per-item hdc_backward bit for bit
    dhs = [torch.from_numpy(synth.normal(s, 509, i, synth.ROLE_U, dtype)).cuda() for i, (s, k) in enumerate(items)]
    for rep in range(2):
        dfs, dgs = hd.conv_batch_backward(fs, gs, dhs, plan)
        torch.cuda.synchronize()
        for i, (s, k) in enumerate(items):
            df1, dg1 = hd.conv_backward(fs[i], gs[i], dhs[i])
            assert dfs[i].shape == fs[i].shape and dgs[i].shape == gs[i].shape
            assert torch.equal(dfs[i].cpu(), df1.cpu()), f"rep {rep} item {i} {s} * {k}: df"
            assert torch.equal(dgs[i].cpu(), dg1.cpu()), f"rep {rep} item {i} {s} * {k}: dg"
    from oracle import fft_grad

    for i, (s, k) in enumerate(items):
        f, g, u = fs[i].cpu().numpy(), gs[i].cpu().numpy(), dhs[i].cpu().numpy()
        rdf, rdg = fft_grad(f, zero_extend(g, f.shape), u)
        assert relerr(dfs[i].cpu().numpy(), rdf) <= TOL[dtype], f"item {i}: df"
        assert relerr(dgs[i].cpu().numpy(), rdg[tuple(slice(0, v) for v in k)]) <= TOL[dtype], f"item {i}: dg"


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batch_short_kernels_cs_and_mixed(hd, dtype):
    """Conjugate-symmetry and mixed items with shorter kernels: equal to the per-item calls bit for bit, forward
    and adjoint, and to the oracle."""
    import torch

    from oracle import fft_grad, zero_extend

    items = [((1000,), (37,), "hybrid_cs"), ((1 << 16,), (4096,), "hybrid_cs"), ((300, 200), (31, 17), "hybrid_cs"),
             ((20, 18, 16), (5, 4, 3), "hybrid_cs"), ((1000,), (37,), "hybrid_mix"), ((4000,), (2000,), "hybrid_mix"),
             ((64, 48), (10, 7), "hybrid_mix", (16, 0)), ((300, 200), (300, 200), "hybrid_mix", (64, 0)),
             ((16, 12, 10), (8, 6, 4), "hybrid_mix", (4, 0, 0)), ((1000,), (37,), "hybrid_rcm")]
    items = [it if len(it) == 4 else it + (None,) for it in items]
    fs, gs, dhs = [], [], []
    for i, (s, k, _, _) in enumerate(items):
        fs.append(torch.from_numpy(synth.normal(s, 510, i, synth.ROLE_F, dtype)).cuda())
        gs.append(torch.from_numpy(synth.normal(k, 510, i, synth.ROLE_G, dtype)).cuda())
        dhs.append(torch.from_numpy(synth.normal(s, 510, i, synth.ROLE_U, dtype)).cuda())
    plan = hd.BatchPlan([{"shape": s, "kernel_shape": k, "variant": v, "m": m} for s, k, v, m in items], dtype)
    hs = hd.conv_batch(fs, gs, plan)
    dfs, dgs = hd.conv_batch_backward(fs, gs, dhs, plan)
    torch.cuda.synchronize()
    for i, (s, k, v, m) in enumerate(items):
        assert torch.equal(hs[i].cpu(), hd.conv_forward(fs[i], gs[i], m=m, variant=v).cpu()), f"item {i} {s} * {k} {v}"
        df1, dg1 = hd.conv_backward(fs[i], gs[i], dhs[i], m=m, variant=v)
        assert torch.equal(dfs[i].cpu(), df1.cpu()) and torch.equal(dgs[i].cpu(), dg1.cpu()), f"item {i}: adjoint"
        f, g, u = fs[i].cpu().numpy(), gs[i].cpu().numpy(), dhs[i].cpu().numpy()
        gz = zero_extend(g, f.shape)
        assert relerr(hs[i].cpu().numpy(), fft_conv(f, gz)) <= TOL[dtype], f"item {i} {s} * {k} {v}"
        rdf, rdg = fft_grad(f, gz, u)
        assert relerr(dfs[i].cpu().numpy(), rdf) <= TOL[dtype], f"item {i} {v}: df"
        assert relerr(dgs[i].cpu().numpy(), rdg[tuple(slice(0, n) for n in k)]) <= TOL[dtype], f"item {i} {v}: dg"
