"""CPU oracle for the hybrid-dealiased real convolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU product path never calls it and
shares no code with it.

Contents
--------
``direct``  the plain definitions, in float64 or exact arithmetic:
            * the truncated linear convolution h_j = sum_{0<=k<=j} f_k g_{j-k},
              j < L (componentwise in d dimensions) -- the result hybrid
              dealiasing reaches exactly in exact arithmetic (Sec. 2, eqs.
              (forwardr), (backwardr), (accumulation));
            * its gradient (adjoint) with respect to f and g;
            * an explicitly zero-padded FFT convolution (the "explicit"
              dealiasing of Sec. 1) used as a fast full-size reference;
            * the normwise relative error;
            * a shorter kernel g written out as f's extents with zeros (the
              unequal-length convolution of the conclusion, Sec. 7);
            * the truncated convolution of n >= 2 arrays (Sec. 4.1), literally
              in exact arithmetic, by direct float64 sums, and explicitly padded.
``hybrid``  the paper's algorithms written out step by step in its notation
            (residue transforms of Sec. 2, conjugate-symmetry residues of
            Sec. 3 and Appendix A, complex packing and the RCM operator of
            Sec. 4, the multidimensional decomposition of Sec. 5, the
            explicitly padded implicit-packing algorithms of Sec. 5).  These
            restate what the GPU kernels compute so that intermediate results
            can be checked; they are pinned to the plain definition by the
            ``-m "not gpu"`` tests.

Every function is pinned by a test against something other than itself
(brute force in exact arithmetic, closed forms, invariants the paper states,
library routines for special cases).  No function here is "parity unpinned".
"""
from .direct import (  # noqa: F401
    brute_conv_exact,
    brute_conv_nary_exact,
    direct_conv,
    direct_conv_at,
    direct_conv_nary,
    fft_conv,
    fft_conv_nary,
    grad_direct,
    grad_direct_at,
    fft_grad,
    relerr,
    zero_extend,
)
from . import hybrid  # noqa: F401
