"""CPU oracle for the extra-component method (Terekhov, arXiv 2004.11610).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
constant generator with the HIP library; it is written from the paper, in
plain NumPy/SciPy float64, slow and obvious on purpose.

Modules
-------
params      Kaiser window (sec. 2.1), zeta(eps1) by Newton and the extra-component
            count s(zeta, eps2) (sec. 2.2), block partition (sec. 3, Table 1).
nodes       Quadrature nodes and Christoffel weights of every family.
entries     Matrix entries A[j, k] by three-term recurrences (DLMF 18.9).
direct      The plain definition y = A x (dense, float64).
compressed  Algorithm 1 (two-sided extras) and the block Algorithm 3 (one-sided
            extras), computation stage exactly in the paper's order: extend,
            divide by the window, F*, sparse product, sum of blocks.
transposed  Algorithm 2 / block Algorithm 4 (product with the transpose): sparse
            product with the column-compressed matrix, F*, divide by the window,
            discard the extras.
appendix_a  Appendix A: compressed rows of the trigonometric generators from the
            closed-form row spectra convolved with 2q+1 window coefficients.
two_d       The two-dimensional compression of sec. 4.2 (eq. comp_2d) as a
            density measure, beside the row and column compressions.

Pins (what ties this oracle to something other than itself) live in
``tests/test_oracle_*.py``.  Parity unpinned: the compression ratios of the
Laguerre and Hermite function families at their Gauss nodes (the paper gives
them only for an equispaced grid, and only as figures).
"""

from . import params, nodes, entries, direct, compressed, transposed, appendix_a, two_d  # noqa: F401
