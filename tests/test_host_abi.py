"""CPU-only checks of the C ABI and host logic (no kernel launches).

The library must load without a GPU and export every function the header
declares; descriptor validation runs on the host and reports invalid or
unsupported parameters before any device call.  Also checks the binding's
struct layout against the header and the algorithmic byte model.
"""
import ctypes
import os
import re

import pytest

import paper_2608_14497_amd as hd
from paper_2608_14497_amd import model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdconv.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdc_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hd.LIB_PATH):
        from paper_2608_14497_amd import build

        build.build(verbose=False)
    return hd.load()


def test_header_declares_the_binding_names():
    assert _declared() == sorted(hd.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version(lib):
    assert lib.hdc_version().decode().startswith("hdconv")
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.hdc_status_string(st)
    buf = ctypes.create_string_buffer(8)
    assert lib.hdc_last_error(buf, 8) >= 0


def test_desc_layout_matches_header():
    # int32 ndim; int64 L[3], M[3]; int32 m[3], q[3], variant, dtype; int64 batch; uint32 flags; int64 Lg[3];
    # int32 nin
    assert hd.Desc.L.offset == 8 and hd.Desc.M.offset == 32 and hd.Desc.m.offset == 56
    assert hd.Desc.q.offset == 68 and hd.Desc.variant.offset == 80 and hd.Desc.batch.offset == 88
    assert hd.Desc.Lg.offset == 104 and hd.Desc.nin.offset == 128 and ctypes.sizeof(hd.Desc) == 136
    text = open(HEADER).read()
    body = text[text.index("typedef struct"):text.index("} hdc_desc;")]
    fields = re.findall(r"\b(int32_t|int64_t|uint32_t)\s+(\w+)(\[3\])?;", body)
    want = [("int32_t", "ndim"), ("int64_t", "L"), ("int64_t", "M"), ("int32_t", "m"), ("int32_t", "q"),
            ("int32_t", "variant"), ("int32_t", "dtype"), ("int64_t", "batch"), ("uint32_t", "flags"),
            ("int64_t", "Lg"), ("int32_t", "nin")]
    assert [(t, n) for t, n, _ in fields] == want


def _create(lib, shape, **kw):
    kernel = kw.pop("kernel", None)
    d = hd.make_desc(shape, kernel_shape=kernel, **kw)
    h = ctypes.c_void_p()
    st = lib.hdc_plan_create(ctypes.byref(d), ctypes.byref(h))
    buf = ctypes.create_string_buffer(512)
    lib.hdc_last_error(buf, 512)
    return st, buf.value.decode()


@pytest.mark.parametrize("shape,kw,status,words", [
    ((1024,), {"M": (2000,)}, -1, "2L-1"),                 # wrapped terms would reach j < L
    ((1024,), {"m": (5,)}, -1, "even"),                    # packed last axis needs an even m
    ((64, 64), {"m": (48, 0)}, -2, "power of two"),        # outer FFT length
    ((64, 64), {"m": (8, 0), "q": (4, 0)}, -1, "q m"),     # q m < M
    ((37,), {"variant": "explicit", "M": (73,)}, -1, "even M"),
    ((0,), {}, -1, "L[0]"),
    # a shorter kernel g (Lg <= L; M >= L + Lg - 1; two arrays)
    ((100,), {"kernel": (101,)}, -1, "Lg[0]"),
    ((100,), {"kernel": (10,), "M": (108,)}, -1, "L+Lg-1"),
    ((100,), {"kernel": (10,), "variant": "hybrid_cs", "M": (108,)}, -1, "L+Lg-1"),
    ((100,), {"kernel": (10,), "nin": 3}, -2, "equal extents"),
    ((100,), {"flags": 0x1}, -1, "unknown flag"),
    ((100,), {"flags": 0x10}, -1, "unknown flag"),
    # strided axes keep single-level residue tables, at most 2^22 points
    ((1000, 2), {"M": (1 << 23, 4)}, -2, "exceeds 2^22"),
    ((4, 1000, 2), {"M": (8, 1 << 23, 4)}, -2, "exceeds 2^22"),
])
def test_descriptor_validation_on_host(lib, shape, kw, status, words):
    st, msg = _create(lib, shape, **kw)
    assert st == status, msg
    assert words in msg


def test_bad_descriptor_fields(lib):
    for field, val in (("ndim", 4), ("batch", 0), ("variant", 9), ("dtype", 7)):
        d = hd.make_desc((16,))
        setattr(d, field, val)
        h = ctypes.c_void_p()
        assert lib.hdc_plan_create(ctypes.byref(d), ctypes.byref(h)) == -1, field
        assert not h.value
    h = ctypes.c_void_p()
    assert lib.hdc_plan_create(None, ctypes.byref(h)) == -1
    assert lib.hdc_forward(None, None, None, None, None, 0, None) == -1
    assert lib.hdc_batch_plan_create(None, 0, ctypes.byref(h)) == -1
    assert lib.hdc_autotune(None, None) == -1


def test_byte_model_closed_forms():
    """15 N w per pair in 1D and 2D, 39 N w in 3D (M = 2L per axis, hybrid)."""
    for shape, k in (((1 << 20,), 15), ((2048, 2048), 15), ((256, 256, 256), 39)):
        nd = len(shape)
        n = 1
        for s in shape:
            n *= s
        if nd == 1:
            names = ["col_fwd", "line_rows", "col_inv"]
            res = ((2048,), (256,), (512,))   # packed rows of 2048, q m = 2^20 = M/2
        elif nd == 2:
            names = ["col_fwd", "line_2d", "col_inv"]
            res = ((1024, 1024), (2, 1), (4, 2))
        else:
            names = ["col_fwd", "col_fwd", "line_3d", "col_inv", "col_inv"]
            res = ((256, 256, 128), (1, 1, 1), (2, 2, 2))
        for w, dt in ((4, "float32"), (8, "float64")):
            tot = model.total_bytes(names, shape, res, dt, 3)
            assert tot == 3 * k * n * w, (shape, dt, tot)


def test_binding_fails_loudly_without_library(tmp_path):
    """No fallback: loading a missing library raises."""
    saved = hd._lib
    hd._lib = None
    try:
        with pytest.raises(RuntimeError):
            hd.load(str(tmp_path / "missing.so"))
    finally:
        hd._lib = saved


def test_adjoint_and_nary_byte_model_closed_forms():
    """The shared-transform adjoint with saved spectra: 19 N w (1D, 2D) and 47 N w (3D); without them the
    forward passes of f and g add 6 N w (1D, 2D) and 18 N w (3D).  Three arrays at M = 3L in 1D: 28 N w."""
    cases = [((1 << 20,), ((2048,), (256,), (512,)), 19, 25), ((2048, 2048), ((1024, 1024), (2, 1), (4, 2)), 19, 25),
             ((256, 256, 256), ((256, 256, 128), (1, 1, 1), (2, 2, 2)), 47, 65)]
    for shape, res, k_saved, k_full in cases:
        n = 1
        for s in shape:
            n *= s
        assert model.adjoint_bytes(shape, res, "float32", 2, True) == 2 * k_saved * n * 4
        assert model.adjoint_bytes(shape, res, "float64", 1, False) == k_full * n * 8
    L = 1 << 20
    names = ["col_fwd", "col_fwd", "line_rows", "col_inv"]
    assert model.total_bytes(names, (L,), ((1024,), (512,), (1536,)), "float32", 1, nin=3) == 28 * L * 4


def test_mixed_nd_byte_model():
    """The mixed variant in 2D at M = 2L with q = 4 on the first axis: the implicit-packing passes of
    residues 0 and 2 (q = 2 on that axis: 9 N w) and the conjugate-symmetry passes of residue 1 (m lines,
    the inverse reading and writing h: 10 N w)."""
    shape = (2048, 2048)
    n = shape[0] * shape[1]
    names = ["col_fwd", "line_2d", "col_inv", "cs_col_fwd", "line_plain", "cs_col_inv"]
    res = ((1024, 1024), (2, 2), (4, 4))
    passes = model.pass_bytes(names, shape, res, "float32", 1)
    assert [p for p, _ in passes] == names
    assert sum(b for _, b in passes[:3]) == 9 * n * 4
    assert sum(b for _, b in passes[3:]) == 10 * n * 4
    # q = 2 (m = L on the first axis): only the packed residues, the implicit-packing plan's 15 N w
    assert model.total_bytes(names[:3], shape, ((2048, 1024), (1, 2), (2, 4)), "float32", 1) == 15 * n * 4
