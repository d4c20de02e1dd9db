"""hdconv: hybrid-dealiased real convolution on MI355X -- Python binding.

Thin ctypes marshalling over the C ABI in ``include/hdconv.h`` (library
``libhdconv.so`` next to this file, built by ``paper_2608_14497_amd.build``).
Every arithmetic step runs in the HIP kernels; PyTorch only provides device
memory and the current stream.  Importing this package does not load the
library or torch; ``load()`` (called by every entry point) raises if the
library is missing -- there is no fallback path.

Python names follow the C names: ``Plan`` wraps ``hdc_plan_create`` /
``hdc_forward`` / ``hdc_backward``; ``conv`` is the convenience entry point
and ``HybridConvFn`` the autograd function whose backward is the hand-written
adjoint (``hdc_backward``).
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdconv.so")

HDC_OK = 0
HDC_SAVE_SPECTRA = 0x2
HDC_USE_GRAPH = 0x4
HDC_DETERMINISTIC = 0x8
VARIANTS = {"hybrid_rcm": 0, "hybrid_cs": 1, "explicit_rcm": 2, "explicit": 3, "hybrid_mix": 4}
DTYPES = {"float32": 0, "float64": 1}

EXPORTED = [
    "hdc_plan_create", "hdc_plan_workspace_size", "hdc_plan_backward_workspace_size", "hdc_plan_resolved",
    "hdc_plan_describe", "hdc_forward", "hdc_backward", "hdc_plan_destroy", "hdc_batch_plan_create",
    "hdc_batch_workspace_size", "hdc_batch_forward", "hdc_batch_backward", "hdc_batch_plan_destroy",
    "hdc_autotune", "hdc_status_string", "hdc_last_error", "hdc_version", "hdc_profile_enable",
    "hdc_profile_read", "hdc_plan_spectrum_size", "hdc_transform_kernel", "hdc_forward_cached",
    "hdc_forward_n", "hdc_forward_noalloc", "hdc_twiddle_values",
]


class Desc(ctypes.Structure):
    """hdc_desc."""
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("L", ctypes.c_int64 * 3),
        ("M", ctypes.c_int64 * 3),
        ("m", ctypes.c_int32 * 3),
        ("q", ctypes.c_int32 * 3),
        ("variant", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("Lg", ctypes.c_int64 * 3),
        ("nin", ctypes.c_int32),
    ]


_lib = None
_lock = threading.Lock()


def load(path: str | None = None):
    """Load libhdconv.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"hdconv: {p} is not built (run python -m paper_2608_14497_amd.build)")
        # torch's HIP runtime first: the library then binds to the runtime torch's tensors and streams
        # belong to (loading it first would bring in a second runtime beside torch's)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(p)
        vp = ctypes.c_void_p
        lib.hdc_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
        lib.hdc_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        lib.hdc_plan_backward_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        i3 = ctypes.c_int32 * 3
        lib.hdc_plan_resolved.argtypes = [vp, i3, i3, i3]
        lib.hdc_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        lib.hdc_forward.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.hdc_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.hdc_plan_destroy.argtypes = [vp]
        lib.hdc_plan_spectrum_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        lib.hdc_transform_kernel.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.hdc_forward_cached.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.hdc_forward_n.argtypes = [vp, ctypes.POINTER(vp), vp, vp, ctypes.c_size_t, vp]
        lib.hdc_forward_noalloc.argtypes = [vp, vp, vp, vp, vp]
        dp = ctypes.POINTER(ctypes.c_double)
        lib.hdc_twiddle_values.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, dp, dp]
        lib.hdc_batch_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.c_int64, ctypes.POINTER(vp)]
        lib.hdc_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        lib.hdc_batch_forward.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                          ctypes.c_size_t, vp]
        lib.hdc_batch_backward.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
        lib.hdc_batch_plan_destroy.argtypes = [vp]
        lib.hdc_autotune.argtypes = [ctypes.POINTER(Desc), ctypes.c_char_p]
        lib.hdc_status_string.argtypes = [ctypes.c_int]
        lib.hdc_status_string.restype = ctypes.c_char_p
        lib.hdc_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.hdc_last_error.restype = ctypes.c_size_t
        lib.hdc_version.restype = ctypes.c_char_p
        lib.hdc_profile_enable.argtypes = [vp, ctypes.c_int]
        lib.hdc_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        for name in EXPORTED:
            fn = getattr(lib, name)
            if fn.restype is None and name not in ("hdc_status_string", "hdc_last_error", "hdc_version"):
                fn.restype = ctypes.c_int
        _lib = lib
        return lib


class HdcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(st: int):
    if st != HDC_OK:
        lib = load()
        buf = ctypes.create_string_buffer(1024)
        lib.hdc_last_error(buf, 1024)
        raise HdcError(st, f"{lib.hdc_status_string(st).decode()}: {buf.value.decode()}")


def make_desc(shape, M=None, m=None, q=None, variant="hybrid_rcm", dtype="float32", batch=1,
              kernel_shape=None, flags=0, nin=2) -> Desc:
    """kernel_shape: extents of g when shorter than f (None: the same as shape); flags: HDC_* bits;
    nin: number of input arrays (2 for the binary convolution)."""
    nd = len(shape)
    if kernel_shape is not None and len(kernel_shape) != nd:
        raise ValueError("hdconv: kernel_shape needs one extent per axis")
    d = Desc()
    d.ndim = nd
    for a in range(3):
        d.L[a] = int(shape[a]) if a < nd else 1
        d.Lg[a] = int(kernel_shape[a]) if (kernel_shape is not None and a < nd) else 0
        d.M[a] = int(M[a]) if (M is not None and a < nd and M[a]) else 0
        d.m[a] = int(m[a]) if (m is not None and a < nd and m[a]) else 0
        d.q[a] = int(q[a]) if (q is not None and a < nd and q[a]) else 0
    d.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    d.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    d.batch = int(batch)
    d.flags = int(flags)
    d.nin = int(nin)
    return d


class Plan:
    """An hdc_plan: fixed shape, padding, hybrid parameters, variant, dtype, batch."""

    def __init__(self, shape, M=None, m=None, q=None, variant="hybrid_rcm", dtype="float32", batch=1,
                 kernel_shape=None, flags=0, nin=2):
        lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.kernel_shape = self.shape if kernel_shape is None else tuple(int(s) for s in kernel_shape)
        self.batch = int(batch)
        self.dtype = dtype
        self.variant = variant
        self.flags = int(flags)
        self.nin = int(nin)
        self.desc = make_desc(shape, M, m, q, variant, dtype, batch, kernel_shape, flags, nin)
        h = ctypes.c_void_p()
        _check(lib.hdc_plan_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        _check(lib.hdc_plan_workspace_size(h, ctypes.byref(n)))
        self.ws_bytes = n.value
        _check(lib.hdc_plan_backward_workspace_size(h, ctypes.byref(n)))
        self.bwd_ws_bytes = n.value

    def resolved(self):
        i3 = ctypes.c_int32 * 3
        m, p, q = i3(), i3(), i3()
        _check(load().hdc_plan_resolved(self._h, m, p, q))
        nd = len(self.shape)
        return tuple(m[:nd]), tuple(p[:nd]), tuple(q[:nd])

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(load().hdc_plan_describe(self._h, buf, 512))
        return buf.value.decode()

    def forward_ptr(self, f, g, h, ws, ws_bytes, stream):
        _check(load().hdc_forward(self._h, f, g, h, ws, ws_bytes, stream))

    def backward_ptr(self, f, g, dh, df, dg, ws, ws_bytes, stream):
        _check(load().hdc_backward(self._h, f, g, dh, df, dg, ws, ws_bytes, stream))

    def forward_noalloc_ptr(self, f, g, h, stream):
        """hdc_forward with the library's static device workspace (allocates nothing)."""
        _check(load().hdc_forward_noalloc(self._h, f, g, h, stream))

    def forward_n_ptr(self, xs, h, ws, ws_bytes, stream):
        arr = (ctypes.c_void_p * len(xs))(*xs)
        _check(load().hdc_forward_n(self._h, arr, h, ws, ws_bytes, stream))

    def spectrum_bytes(self) -> int:
        """Bytes of a cached kernel spectrum for this plan (raises HdcError if the plan has none)."""
        n = ctypes.c_size_t()
        _check(load().hdc_plan_spectrum_size(self._h, ctypes.byref(n)))
        return n.value

    def transform_kernel_ptr(self, g, spec, ws, ws_bytes, stream):
        _check(load().hdc_transform_kernel(self._h, g, spec, ws, ws_bytes, stream))

    def forward_cached_ptr(self, f, spec, h, ws, ws_bytes, stream):
        _check(load().hdc_forward_cached(self._h, f, spec, h, ws, ws_bytes, stream))

    def profile(self, on: bool = True):
        _check(load().hdc_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(names, average ms per launch position, number of calls) since the last read."""
        buf = (ctypes.c_double * 64)()
        nl, nc = ctypes.c_int32(), ctypes.c_int32()
        _check(load().hdc_profile_read(self._h, buf, 64, ctypes.byref(nl), ctypes.byref(nc)))
        names = [x for x in self.describe().split(";") if x]
        return names, list(buf[: nl.value]), nc.value

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.hdc_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


class BatchPlan:
    """An hdc_batch_plan: a list of problems of differing shapes run as grouped launches."""

    def __init__(self, items, dtype="float32"):
        """items: list of dicts with keys shape and optionally M, m, q, variant."""
        lib = load()
        self.items = [dict(it) for it in items]
        self.dtype = dtype
        arr = (Desc * len(items))()
        for i, it in enumerate(items):
            arr[i] = make_desc(it["shape"], it.get("M"), it.get("m"), it.get("q"),
                               it.get("variant", "hybrid_rcm"), dtype, 1, it.get("kernel_shape"))
        self._descs = arr
        h = ctypes.c_void_p()
        _check(lib.hdc_batch_plan_create(arr, len(items), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        _check(lib.hdc_batch_workspace_size(h, ctypes.byref(n)))
        self.ws_bytes = n.value

    def __len__(self):
        return len(self.items)

    @staticmethod
    def _ptrs(xs):
        arr = (ctypes.c_void_p * len(xs))()
        for i, x in enumerate(xs):
            arr[i] = x
        return arr

    def forward_ptr(self, f, g, h, ws, ws_bytes, stream):
        _check(load().hdc_batch_forward(self._h, self._ptrs(f), self._ptrs(g), self._ptrs(h), ws, ws_bytes, stream))

    def backward_ptr(self, f, g, dh, df, dg, ws, ws_bytes, stream):
        _check(load().hdc_batch_backward(self._h, self._ptrs(f), self._ptrs(g), self._ptrs(dh), self._ptrs(df),
                                         self._ptrs(dg), ws, ws_bytes, stream))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.hdc_batch_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def twiddle_values(N: int, dtype="float32", k0: int = 0, count=None):
    """zeta_N^k for k = k0 .. k0+count-1 as the kernels use them (hdc_twiddle_values): complex128 numpy array."""
    import numpy as np

    lib = load()
    count = N - k0 if count is None else int(count)
    re = np.empty(count, dtype=np.float64)
    im = np.empty(count, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.hdc_twiddle_values(int(N), DTYPES[dtype], int(k0), count, re.ctypes.data_as(dp),
                                  im.ctypes.data_as(dp)))
    return re + 1j * im


def autotune(shape, M=None, variant="hybrid_rcm", dtype="float32", batch=1, cache_path=None, deterministic=False):
    """Time the candidate FFT lengths on the current device; returns m per axis (real-sample units).

    deterministic: HDC_DETERMINISTIC, the planner's defaults without timing (the same on every run)."""
    lib = load()
    d = make_desc(shape, M, None, None, variant, dtype, batch, flags=HDC_DETERMINISTIC if deterministic else 0)
    _check(lib.hdc_autotune(ctypes.byref(d), None if cache_path is None else str(cache_path).encode()))
    return tuple(int(d.m[a]) for a in range(len(shape)))


# ---------------------------------------------------------------- torch layer
_plans: dict = {}


def _torch():
    import torch

    return torch


def get_plan(shape, M=None, m=None, q=None, variant="hybrid_rcm", dtype="float32", batch=1,
             kernel_shape=None, flags=0, nin=2) -> Plan:
    kshape = None if kernel_shape is None or tuple(kernel_shape) == tuple(shape) else tuple(kernel_shape)
    key = (tuple(shape), None if M is None else tuple(M), None if m is None else tuple(m),
           None if q is None else tuple(q), variant, dtype, batch, kshape, int(flags), int(nin))
    p = _plans.get(key)
    if p is None:
        p = Plan(shape, M, m, q, variant, dtype, batch, kshape, flags, nin)
        _plans[key] = p
    return p


def _split(x, ndim):
    shape = tuple(x.shape)
    if ndim is None:
        ndim = len(shape)
    batch = 1
    for s in shape[: len(shape) - ndim]:
        batch *= int(s)
    return shape[len(shape) - ndim:], batch


def _split_pair(f, g, ndim):
    """(extents of f, batch, extents of g) over the last ``ndim`` axes; f and g share the batch axes and
    g's extents are at most f's (a shorter kernel)."""
    shape, batch = _split(f, ndim)
    nd = len(shape)
    if g.dim() != f.dim() or tuple(g.shape[: g.dim() - nd]) != tuple(f.shape[: f.dim() - nd]):
        raise ValueError("hdconv: f and g must have the same batch axes and number of dimensions")
    kshape = tuple(int(v) for v in g.shape[g.dim() - nd:])
    if any(k > n or k < 1 for k, n in zip(kshape, shape)):
        raise ValueError(f"hdconv: g's extents {kshape} must be between 1 and f's {tuple(shape)}")
    return tuple(int(v) for v in shape), batch, kshape


def _prep(x, dt):
    torch = _torch()
    if not x.is_cuda:
        raise ValueError("hdconv: tensors must be on the GPU")
    if x.dtype != dt:
        raise ValueError(f"hdconv: expected {dt}, got {x.dtype}")
    return x.contiguous()


def _workspace(nbytes, device):
    torch = _torch()
    if nbytes == 0:
        return None, 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return ws, ws.data_ptr()


def conv_nary(xs, ndim=None, M=None, m=None, q=None, out=None):
    """h = x_0 * x_1 * ... * x_{n-1} truncated to the extents of the inputs (n = len(xs), 2..8).

    All inputs have one shape and dtype; the last ``ndim`` axes are convolved and the
    leading ones form a batch.  M defaults to n L per axis (M >= n (L - 1) + 1).
    """
    torch = _torch()
    n = len(xs)
    if n < 2:
        raise ValueError("hdconv: need at least two arrays")
    dt = xs[0].dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("hdconv: float32 or float64 tensors only")
    for i, x in enumerate(xs):
        _check_shape(x, xs[0].shape, f"xs[{i}]")
    shape, batch = _split(xs[0], ndim)
    xs = [_prep(x, dt) for x in xs]
    if n == 2:
        return conv_forward(xs[0], xs[1], ndim, M, m, q, out=out)
    plan = get_plan(tuple(int(v) for v in shape), M, m, q, "hybrid_rcm",
                    "float64" if dt == torch.float64 else "float32", batch, None, 0, n)
    if out is not None:
        _check_out(out, xs[0])
    h = torch.empty_like(xs[0]) if out is None else out
    ws, wsp = _workspace(plan.ws_bytes, xs[0].device)
    stream = torch.cuda.current_stream(xs[0].device).cuda_stream
    plan.forward_n_ptr([x.data_ptr() for x in xs], h.data_ptr(), wsp, plan.ws_bytes, stream)
    return h


def _check_shape(x, shape, what):
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"hdconv: {what} must have shape {tuple(shape)}, got {tuple(x.shape)}")


def _check_out(out, like, what="out"):
    """A caller-supplied output: the kernels write prod(like.shape) elements through its pointer."""
    if tuple(out.shape) != tuple(like.shape):
        raise ValueError(f"hdconv: {what} must have shape {tuple(like.shape)}, got {tuple(out.shape)}")
    if out.dtype != like.dtype:
        raise ValueError(f"hdconv: {what} must be {like.dtype}, got {out.dtype}")
    if out.device != like.device:
        raise ValueError(f"hdconv: {what} must be on {like.device}")
    if not out.is_contiguous():
        raise ValueError(f"hdconv: {what} must be contiguous")


def conv_forward(f, g, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm", out=None):
    """h = conv(f, g) over the last ``ndim`` axes (leading axes are the batch).

    g may be a shorter kernel (each of its last ``ndim`` extents <= f's, the same
    batch axes); h has f's shape.
    """
    return _forward(f, g, ndim, M, m, q, variant, out)[0]


def _forward(f, g, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm", out=None, save=False):
    """(h, plan, workspace).  save: the plan carries HDC_SAVE_SPECTRA and the workspace is sized for the
    adjoint, so that _backward with the same f, g and workspace reuses f's and g's spectra."""
    torch = _torch()
    dt = f.dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("hdconv: float32 or float64 tensors only")
    shape, batch, kshape = _split_pair(f, g, ndim)
    f = _prep(f, dt)
    g = _prep(g, dt)
    plan = get_plan(shape, M, m, q, variant, "float64" if dt == torch.float64 else "float32", batch,
                    None if kshape == shape else kshape, HDC_SAVE_SPECTRA if save else 0)
    if out is not None:
        _check_out(out, f)
    h = torch.empty_like(f) if out is None else out
    nbytes = max(plan.ws_bytes, plan.bwd_ws_bytes) if save else plan.ws_bytes
    ws, wsp = _workspace(nbytes, f.device)
    stream = torch.cuda.current_stream(f.device).cuda_stream
    plan.forward_ptr(f.data_ptr(), g.data_ptr(), h.data_ptr(), wsp, nbytes, stream)
    return h, plan, ws


class CachedKernel:
    """A kernel g transformed once and convolved with many f ("transform once, multiply many").

    ``shape`` is the extent of f (and h) over the last len(shape) axes; g has
    the same batch axes and extents <= shape.  Available for the implicit-packing
    hybrid variant in 1D, 2D and 3D; results equal conv_forward(f, g) bit for bit.
    """

    def __init__(self, g, shape, M=None, m=None, q=None):
        torch = _torch()
        dt = g.dtype
        g = _prep(g, dt)
        shape = tuple(int(s) for s in shape)
        kshape, batch = _split(g, len(shape))
        self.dtype = dt
        self.shape, self.batch_shape = shape, tuple(g.shape[: g.dim() - len(shape)])
        self.plan = get_plan(shape, M, m, q, "hybrid_rcm", "float64" if dt == torch.float64 else "float32", batch,
                             None if kshape == shape else kshape)
        self.spec = torch.empty(self.plan.spectrum_bytes(), dtype=torch.uint8, device=g.device)
        ws, wsp = _workspace(self.plan.ws_bytes, g.device)
        stream = torch.cuda.current_stream(g.device).cuda_stream
        self.plan.transform_kernel_ptr(g.data_ptr(), self.spec.data_ptr(), wsp, self.plan.ws_bytes, stream)

    def __call__(self, f, out=None):
        torch = _torch()
        _check_shape(f, self.batch_shape + self.shape, "f")
        f = _prep(f, self.dtype)
        if out is not None:
            _check_out(out, f)
        h = torch.empty_like(f) if out is None else out
        ws, wsp = _workspace(self.plan.ws_bytes, f.device)
        stream = torch.cuda.current_stream(f.device).cuda_stream
        self.plan.forward_cached_ptr(f.data_ptr(), self.spec.data_ptr(), h.data_ptr(), wsp, self.plan.ws_bytes, stream)
        return h


def conv_backward(f, g, dh, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm", need_f=True, need_g=True):
    """(df, dg) for an upstream gradient dh (the adjoint of conv_forward; None where not needed)."""
    return _backward(f, g, dh, ndim, M, m, q, variant, need_f, need_g)


def _backward(f, g, dh, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm", need_f=True, need_g=True,
              plan=None, ws=None):
    """plan, ws: those of a _forward(..., save=True) of the same f and g (its spectra are reused)."""
    torch = _torch()
    dt = f.dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("hdconv: float32 or float64 tensors only")
    shape, batch, kshape = _split_pair(f, g, ndim)
    _check_shape(dh, f.shape, "dh")
    f = _prep(f, dt)
    g = _prep(g, dt)
    dh = _prep(dh, dt)
    if plan is None:
        plan = get_plan(shape, M, m, q, variant, "float64" if dt == torch.float64 else "float32", batch,
                        None if kshape == shape else kshape)
    df = torch.empty_like(f) if need_f else None
    dg = torch.empty_like(g) if need_g else None
    if ws is None or ws.numel() < plan.bwd_ws_bytes:
        ws, wsp = _workspace(plan.bwd_ws_bytes, f.device)
    else:
        wsp = ws.data_ptr()
    stream = torch.cuda.current_stream(f.device).cuda_stream
    plan.backward_ptr(f.data_ptr(), g.data_ptr(), dh.data_ptr(), df.data_ptr() if need_f else None,
                      dg.data_ptr() if need_g else None, wsp, plan.bwd_ws_bytes, stream)
    return df, dg


def _check_batch_items(plan, fs, gs):
    """The tensors of a call must match the items the batch plan was made for."""
    if len(plan.items) != len(fs):
        raise ValueError(f"hdconv: the batch plan has {len(plan.items)} items, got {len(fs)}")
    for i, (it, f, g) in enumerate(zip(plan.items, fs, gs)):
        shape = tuple(int(v) for v in it["shape"])
        ks = it.get("kernel_shape")
        ks = shape if ks is None else tuple(int(v) for v in ks)
        _check_shape(f, shape, f"f[{i}]")
        _check_shape(g, ks, f"g[{i}]")


def conv_batch(fs, gs, plan: "BatchPlan" = None, variant="hybrid_rcm", out=None):
    """h_i = conv(f_i, g_i) for lists of tensors of differing shapes, one grouped launch sequence.

    Every tensor of item i has the full shape of that problem (no batch axis);
    g_i may be a shorter kernel (same number of axes, extents <= f_i's).
    Pass a BatchPlan to reuse it across calls (its graph and parameter tables).
    """
    torch = _torch()
    if len(fs) != len(gs) or not fs:
        raise ValueError("hdconv: need equal, non-empty lists")
    dt = fs[0].dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("hdconv: float32 or float64 tensors only")
    for f, g in zip(fs, gs):
        _split_pair(f, g, None)
    if plan is not None:
        _check_batch_items(plan, fs, gs)
    if out is not None and len(out) != len(fs):
        raise ValueError("hdconv: out needs one tensor per item")
    fs = [_prep(f, dt) for f in fs]
    gs = [_prep(g, dt) for g in gs]
    if plan is None:
        plan = BatchPlan([{"shape": tuple(f.shape), "variant": variant,
                           "kernel_shape": None if g.shape == f.shape else tuple(g.shape)} for f, g in zip(fs, gs)],
                         "float64" if dt == torch.float64 else "float32")
    if out is not None:
        for i, (o, f) in enumerate(zip(out, fs)):
            _check_out(o, f, f"out[{i}]")
    hs = [torch.empty_like(f) for f in fs] if out is None else out
    ws, wsp = _workspace(plan.ws_bytes, fs[0].device)
    stream = torch.cuda.current_stream(fs[0].device).cuda_stream
    plan.forward_ptr([f.data_ptr() for f in fs], [g.data_ptr() for g in gs], [h.data_ptr() for h in hs], wsp,
                     plan.ws_bytes, stream)
    return hs


def conv_batch_backward(fs, gs, dhs, plan: "BatchPlan" = None, variant="hybrid_rcm"):
    """(df_i, dg_i) for lists of problems of differing shapes (adjoint of conv_batch)."""
    torch = _torch()
    if not fs or len(fs) != len(gs) or len(fs) != len(dhs):
        raise ValueError("hdconv: need equal, non-empty lists of f, g and dh")
    dt = fs[0].dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("hdconv: float32 or float64 tensors only")
    for i, (f, g, d) in enumerate(zip(fs, gs, dhs)):
        _split_pair(f, g, None)
        _check_shape(d, f.shape, f"dh[{i}]")
    if plan is not None:
        _check_batch_items(plan, fs, gs)
    fs = [_prep(f, dt) for f in fs]
    gs = [_prep(g, dt) for g in gs]
    dhs = [_prep(d, dt) for d in dhs]
    if plan is None:
        # every item's kernel extents go into its descriptor, so the library sees a shorter kernel
        # (and reports the batched adjoint of one as unsupported) instead of reading g as f-sized
        plan = BatchPlan([{"shape": tuple(f.shape), "variant": variant,
                           "kernel_shape": None if g.shape == f.shape else tuple(g.shape)} for f, g in zip(fs, gs)],
                         "float64" if dt == torch.float64 else "float32")
    dfs = [torch.empty_like(f) for f in fs]
    dgs = [torch.empty_like(g) for g in gs]
    ws, wsp = _workspace(plan.ws_bytes, fs[0].device)
    stream = torch.cuda.current_stream(fs[0].device).cuda_stream
    plan.backward_ptr([f.data_ptr() for f in fs], [g.data_ptr() for g in gs], [d.data_ptr() for d in dhs],
                      [x.data_ptr() for x in dfs], [x.data_ptr() for x in dgs], wsp, plan.ws_bytes, stream)
    return dfs, dgs


def _make_fn():
    torch = _torch()

    class HybridConvFn(torch.autograd.Function):
        """h = conv(f, g); backward: df = R(conv(g, R(dh))), dg = R(conv(f, R(dh))) via hdc_backward.

        With save_spectra the forward's plan carries HDC_SAVE_SPECTRA and its workspace is kept until the
        backward, which then transforms only R(dh) (f and g are not transformed a second time)."""

        @staticmethod
        def forward(ctx, f, g, ndim, M, m, q, variant, save_spectra):
            f = f.contiguous()
            g = g.contiguous()
            ctx.save_for_backward(f, g)
            ctx.cfg = (ndim, M, m, q, variant)
            save = bool(save_spectra) and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
            h, plan, ws = _forward(f, g, ndim, M, m, q, variant, save=save)
            ctx.plan, ctx.ws = (plan, ws) if save else (None, None)
            return h

        @staticmethod
        def backward(ctx, dh):
            f, g = ctx.saved_tensors
            ndim, M, m, q, variant = ctx.cfg
            df, dg = _backward(f, g, dh.contiguous(), ndim, M, m, q, variant,
                               ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.plan, ctx.ws)
            return df, dg, None, None, None, None, None, None

    return HybridConvFn


_fn_cls = None


def conv(f, g, ndim=None, M=None, m=None, q=None, variant="hybrid_rcm", save_spectra=True):
    """Differentiable hybrid-dealiased convolution of real tensors.

    ndim: number of trailing axes convolved (default: all); leading axes are a
    uniform batch.  g may be a shorter kernel (trailing extents <= f's); h has
    f's shape.  M, m, q: per-axis padding length and hybrid parameters in
    real-sample units (None = defaults: M = L + Lg, planner's m and q).
    save_spectra: when a gradient is needed, keep f's and g's transforms from
    the forward for the backward (HDC_SAVE_SPECTRA; the workspace stays
    allocated until the backward).
    """
    global _fn_cls
    if _fn_cls is None:
        _fn_cls = _make_fn()
    return _fn_cls.apply(f, g, ndim, M, m, q, variant, save_spectra)


def __getattr__(name):
    if name == "HybridConvFn":
        global _fn_cls
        if _fn_cls is None:
            _fn_cls = _make_fn()
        return _fn_cls
    raise AttributeError(name)
