"""Write the exact-integer golden fixtures in this folder.

Calls only the oracle (exact rational brute force of
h_j = sum_{0<=k<=j} f_k g_{j-k}, j < L) on small integer inputs drawn from the
seeded generator.  Each file holds the shape, f, g and the exact h as
integers, one array per line.  Re-run with ``python tests/golden/make_golden.py``.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import brute_conv_exact  # noqa: E402
from paper_2608_14497_amd import synth  # noqa: E402

CASES = {
    "int_1d_L37": (37,),
    "int_1d_L64": (64,),
    "int_2d_9x12": (9, 12),
    "int_3d_5x4x6": (5, 4, 6),
}


def main():
    for i, (name, shape) in enumerate(CASES.items()):
        f, g = synth.pair_for(900, i, shape, np.float64, "ints")
        H = brute_conv_exact(f, g)
        h = np.array([int(H[idx]) for idx in np.ndindex(*shape)], dtype=np.int64)
        with open(os.path.join(HERE, name + ".txt"), "w") as fh:
            fh.write("# exact truncated linear convolution h_j = sum_{k<=j} f_k g_{j-k}, j < L\n")
            fh.write("# written by tests/golden/make_golden.py (oracle brute force, Fractions)\n")
            fh.write("shape " + " ".join(str(v) for v in shape) + "\n")
            fh.write("f " + " ".join(str(int(v)) for v in f.ravel()) + "\n")
            fh.write("g " + " ".join(str(int(v)) for v in g.ravel()) + "\n")
            fh.write("h " + " ".join(str(int(v)) for v in h) + "\n")


def load(name):
    """(f, g, h) as float64 arrays of the stored shape."""
    rows = {}
    with open(os.path.join(HERE, name + ".txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            rows[key] = [int(v) for v in vals]
    shape = tuple(rows["shape"])
    return tuple(np.array(rows[k], dtype=np.float64).reshape(shape) for k in ("f", "g", "h"))


if __name__ == "__main__":
    main()
