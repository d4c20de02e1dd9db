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


def pass_bytes(names, shape, resolved, dtype: str, batch: int, explicit_M=None, kernel_shape=None):
    """[(pass name, bytes)] for one hdc_forward call, in launch order.

    names: the plan's launch sequence (Plan.describe().split(';'));
    resolved: (m, p, q) per axis as reported by the plan;
    explicit_M: padded extents for the explicit comparators (None for hybrid);
    kernel_shape: extents of a shorter kernel g (None: g has f's extents).
    """
    names = [n for n in names if n]
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
    if names and names[0] in ("line_cs", "cs_col_fwd"):
        return [(name, b * batch) for name, b in _cs_bytes(names, shape, resolved, w)]
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


def total_bytes(names, shape, resolved, dtype, batch, explicit_M=None):
    return sum(b for _, b in pass_bytes(names, shape, resolved, dtype, batch, explicit_M))


def _cs_bytes(names, shape, resolved, w):
    """Conjugate-symmetry variant: unpacked real data, retained first-axis lines."""
    c = 2 * w
    m, p, q = resolved
    n = prod(shape)
    if len(shape) == 1:
        if names and names[0] == "cs_col_fwd":
            # multi-pass: q/2 + 1 retained residue rows of m complex values per array
            rows = (q[0] // 2 + 1) * m[0]
            return [("cs_col_fwd", 2 * n * w + 2 * rows * c), ("line_rows", 3 * rows * c),
                    ("cs_col_inv", rows * c + n * w)]
        return [("line_cs", 3 * n * w)]
    m0, q0 = m[0], q[0]
    nret = m0 // 2 + 1 + ((q0 + 1) // 2 - 1) * m0 + (m0 // 2 if q0 % 2 == 0 else 0)
    Ld = shape[-1]
    if len(shape) == 2:
        lines = nret * Ld
        return [("cs_col_fwd", 2 * n * w + 2 * lines * c), ("line_plain", 3 * lines * c),
                ("cs_col_inv", lines * c + n * w)]
    N1 = q[1] * m[1]
    a = nret * shape[1] * Ld
    bfull = nret * N1 * Ld
    return [("cs_col_fwd", 2 * n * w + 2 * a * c), ("col_fwd", 2 * a * c + 2 * bfull * c),
            ("line_plain", 3 * bfull * c), ("col_inv", bfull * c + a * c), ("cs_col_inv", a * c + n * w)]
