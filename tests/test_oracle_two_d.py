"""The two-dimensional compression of sec. 4.2 (eq. comp_2d) against the
paper's statements, and on the Laguerre-function workload's matrix (why the
library builds the row compression only):

* on the paper's grid (Laguerre functions l_m(eta t_i) at t_i = 12 i / (N-1),
  eta = 100, 500, 1000; accuracy 1e-10) the two-dimensional compression keeps
  a few percent of the entries (the paper: up to 3-4%), while the row and
  column compressions keep most of them (the paper: they do not decrease the
  number of nonzero elements);
* at the Gauss-Laguerre nodes of the Laguerre-function workload the row
  compression keeps about 55% and the two-dimensional one about a third: no
  order-of-magnitude gain, and a second transform per right-hand side plus
  extra components in the node direction, which Gauss nodes do not define.
"""

import numpy as np
import pytest

from oracle import entries, nodes, two_d


@pytest.mark.slow
@pytest.mark.parametrize("eta", [100.0, 500.0, 1000.0])
def test_two_d_on_the_papers_grid(eta):
    N = 2048
    t = 12.0 * np.arange(1, N + 1) / (N - 1)
    row, col, both = two_d.densities(entries.laguerre_fn(eta * t, 0, N), 1e-10)
    assert both <= 0.05
    assert row >= 0.3 and col >= 0.9
    assert both * 6 <= row


@pytest.mark.slow
def test_two_d_at_gauss_laguerre_nodes():
    N = 1024
    row, col, both = two_d.densities(entries.laguerre_fn(nodes.gauss_laguerre(N), 0, N), 1e-7)
    assert 0.45 <= row <= 0.65 and 0.25 <= both <= 0.4
    assert row / both < 2.0
