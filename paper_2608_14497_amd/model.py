"""Algorithmic HBM bytes of each pass (the roofline's numerator).

Counts only what the pass structure must move: every input element read once,
every output element written once; the hybrid variants never read or write
zero padding, the explicit comparators read and write their materialised
padded arrays.  Units: bytes per launch (whole batch).

w = bytes per real.  With implicit packing the last axis holds Lh = ceil(L/2)
complex values per row (2w bytes each); N_a = q_a m_a is the transform length
on axis a (packed units on the last axis).  Per pair with M = 2L on every
axis this gives 15 N w in 1D and 2D and 39 N w in 3D (N = prod L).
"""
from __future__ import annotations

from math import prod


def pass_bytes(names, shape, resolved, dtype: str, batch: int, explicit_M=None, kernel_shape=None, nin=2):
    """[(pass name, bytes)] for one hdc_forward call, in launch order.

    names: the plan's launch sequence (Plan.describe().split(';'));
    resolved: (m, p, q) per axis as reported by the plan;
    explicit_M: padded extents for the explicit comparators (None for hybrid);
    kernel_shape: extents of a shorter kernel g (None: g has f's extents);
    nin: input arrays (hdc_forward_n; the forward passes take two arrays per launch).
    """
    names = [n for n in names if n]
    if nin > 2:
        return [(name, b * batch) for name, b in _nary_bytes(names, shape, resolved, dtype, nin)]
    w = 8 if dtype == "float64" else 4
    c = 2 * w
    m, p, q = resolved
    nd = len(shape)
    Le = tuple(explicit_M) if explicit_M else tuple(shape)
    n_user = prod(shape)
    n_exec = prod(Le)
    ng_user = prod(kernel_shape) if kernel_shape else n_user
    ng_exec = n_exec if explicit_M else ng_user  # reals of g the first pass reads
    Lh = (Le[-1] + 1) // 2
    out = []
    if names and names[0] in ("line_cs", "line_mix", "cs_col_fwd"):
        return [(name, b * batch) for name, b in _cs_bytes(names, shape, resolved, w)]
    if nd > 1 and "cs_col_fwd" in names:
        # mixed variant in 2D/3D: the implicit-packing passes of residues 0 and q/2 (q = 2, or 1 for an odd q,
        # on the first axis), then the conjugate-symmetry passes of the other residues, adding to h
        k = names.index("cs_col_fwd")
        qs = 2 if q[0] % 2 == 0 else 1
        sub = pass_bytes(names[:k], shape, (m, p, (qs,) + tuple(q[1:])), dtype, batch, None, kernel_shape)
        return sub + [(name, b * batch) for name, b in _cs_bytes(names[k:], shape, resolved, w, mid_only=True)]
    for k in range(names.count("pad")):  # one launch per padded input (f, then g)
        out.append(("pad", (n_user if k == 0 else ng_user) * w + n_exec * w))
    if nd == 1:
        N = q[0] * m[0]
        if "line_1d" in names:
            out.append(("line_1d", (2 * n_exec + ng_exec) * w))
        else:
            out.append(("col_fwd", (n_exec + ng_exec) * w + 2 * N * c))
            out.append(("line_rows", 2 * N * c + N * c))
            out.append(("col_inv", N * c + n_exec * w))
    elif nd == 2:
        N0 = q[0] * m[0]
        out.append(("col_fwd", (n_exec + ng_exec) * w + 2 * N0 * Lh * c))
        out.append(("line_2d", 3 * N0 * Lh * c))
        out.append(("col_inv", N0 * Lh * c + n_exec * w))
    else:
        N0, N1 = q[0] * m[0], q[1] * m[1]
        out.append(("col_fwd", (n_exec + ng_exec) * w + 2 * N0 * Le[1] * Lh * c))
        out.append(("col_fwd", 2 * N0 * Le[1] * Lh * c + 2 * N0 * N1 * Lh * c))
        out.append(("line_3d", 3 * N0 * N1 * Lh * c))
        out.append(("col_inv", N0 * N1 * Lh * c + N0 * Le[1] * Lh * c))
        out.append(("col_inv", N0 * Le[1] * Lh * c + n_exec * w))
    if "truncate" in names:
        out.append(("truncate", n_exec * w + n_user * w))
    return [(name, b * batch) for name, b in out]


def total_bytes(names, shape, resolved, dtype, batch, explicit_M=None, nin=2):
    return sum(b for _, b in pass_bytes(names, shape, resolved, dtype, batch, explicit_M, None, nin))


def _nary_bytes(names, shape, resolved, dtype, nin):
    """Implicitly packed convolution of nin arrays: each forward pass launch reads and transforms two
    arrays (the last launch one when nin is odd), the line kernel reads nin spectra and writes one."""
    w = 8 if dtype == "float64" else 4
    c = 2 * w
    m, p, q = resolved
    nd = len(shape)
    n = prod(shape)
    Lh = (shape[-1] + 1) // 2
    per = [min(2, nin - a) for a in range(0, nin, 2)]  # arrays per forward launch
    out = []
    if nd == 1:
        N = q[0] * m[0]
        if "line_1d" in names:
            return [("line_1d", (nin + 1) * n * w)]
        out += [("col_fwd", k * (n * w + N * c)) for k in per]
        out += [("line_rows", (nin + 1) * N * c), ("col_inv", N * c + n * w)]
    elif nd == 2:
        N0 = q[0] * m[0]
        out += [("col_fwd", k * (n * w + N0 * Lh * c)) for k in per]
        out += [("line_2d", (nin + 1) * N0 * Lh * c), ("col_inv", N0 * Lh * c + n * w)]
    else:
        N0, N1 = q[0] * m[0], q[1] * m[1]
        a = N0 * shape[1] * Lh * c
        bfull = N0 * N1 * Lh * c
        out += [("col_fwd", k * (n * w + a)) for k in per]
        out += [("col_fwd", k * (a + bfull)) for k in per]
        out += [("line_3d", (nin + 1) * bfull), ("col_inv", bfull + a), ("col_inv", a + n * w)]
    return out


def _cs_bytes(names, shape, resolved, w, mid_only=False):
    """Conjugate-symmetry variant: unpacked real data, retained first-axis lines.

    mid_only: the mixed variant's residues 1 .. ceil(q/2) - 1 on the first axis (m lines each); the inverse
    reads h (the packed residues' result) and writes it back."""
    c = 2 * w
    m, p, q = resolved
    n = prod(shape)
    if len(shape) == 1:
        if names and names[0] == "cs_col_fwd":
            # multi-pass: q/2 + 1 retained residue rows of m complex values per array
            rows = (q[0] // 2 + 1) * m[0]
            return [("cs_col_fwd", 2 * n * w + 2 * rows * c), ("line_rows", 3 * rows * c),
                    ("cs_col_inv", rows * c + n * w)]
        return [(names[0], 3 * n * w)]
    m0, q0 = m[0], q[0]
    if mid_only:
        nret = ((q0 + 1) // 2 - 1) * m0
    else:
        nret = m0 // 2 + 1 + ((q0 + 1) // 2 - 1) * m0 + (m0 // 2 if q0 % 2 == 0 else 0)
    hout = (2 if mid_only else 1) * n * w  # h written (mixed: read and written)
    Ld = shape[-1]
    if len(shape) == 2:
        lines = nret * Ld
        return [("cs_col_fwd", 2 * n * w + 2 * lines * c), ("line_plain", 3 * lines * c),
                ("cs_col_inv", lines * c + hout)]
    N1 = q[1] * m[1]
    a = nret * shape[1] * Ld
    bfull = nret * N1 * Ld
    return [("cs_col_fwd", 2 * n * w + 2 * a * c), ("col_fwd", 2 * a * c + 2 * bfull * c),
            ("line_plain", 3 * bfull * c), ("col_inv", bfull * c + a * c), ("cs_col_inv", a * c + hout)]


def adjoint_bytes(shape, resolved, dtype: str, batch: int, saved: bool, one_workgroup: bool = False):
    """Algorithmic bytes of one hdc_backward of the implicit-packing hybrid variant (equal extents), which
    transforms R(dh) once and multiplies its spectra with g's and with f's in one line-kernel launch.

    saved: f's and g's outer-axis spectra come from the preceding forward (HDC_SAVE_SPECTRA); otherwise
    their forward passes run here too.  Per pair at M = 2L and with saved spectra: 19 N w in 1D and 2D,
    47 N w in 3D; a one-workgroup 1D problem reads f, g, dh and writes df, dg (5 N w).
    """
    w = 8 if dtype == "float64" else 4
    c = 2 * w
    m, p, q = resolved
    nd = len(shape)
    n = prod(shape)
    Lh = (shape[-1] + 1) // 2
    if nd == 1 and one_workgroup:
        return 5 * n * w * batch
    if nd == 1:
        A = q[0] * m[0] * c           # one array's residue rows
        fwd = n * w + A               # the column pass of one array
        line = 3 * A + 2 * A
        inv = 2 * (A + n * w)
        tot = fwd + (0 if saved else 2 * fwd) + line + inv
    elif nd == 2:
        A = q[0] * m[0] * Lh * c
        fwd = n * w + A
        tot = fwd + (0 if saved else 2 * fwd) + 5 * A + 2 * (A + n * w)
    else:
        N0, N1 = q[0] * m[0], q[1] * m[1]
        A = N0 * shape[1] * Lh * c
        Bf = N0 * N1 * Lh * c
        fwd = (n * w + A) + (A + Bf)
        tot = fwd + (0 if saved else 2 * fwd) + 5 * Bf + 2 * (Bf + A) + 2 * (A + n * w)
    return tot * batch
