"""Oracle: plain, slow, obviously correct FP64 CPU reference (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library (``paper_2105_02995_amd``)
never imports, links or calls anything here, and nothing here imports the
product library: the two share no code.

It computes what the method approximates, from the paper's definitions:

* the grids X and Omega and the discrete FIO matrix K (section 1, eq3/eq6);
* the normalised DFT F and its inverse (section 1), dense or row by row;
* u = K fhat by dense products (small N) or by direct summation in C (any N);
* the exact solve fhat = K^{-1} u by dense LU, cross-checked by Cholesky on
  the normal equations K^*K fhat = K^* u (section 5, eq:pseudoinv);
* conjugate gradients on K^*K x = K^* b (section 6, eq_NR_1), used to pin the
  discretisation against the unpreconditioned iteration counts the paper prints.
"""
from .fio_oracle import *  # noqa: F401,F403
