"""Device memory of a context stays bounded over repeated observable calls:
buffers kept for the next call are only those of the last two calls, so
alternating query shapes plateau instead of accumulating."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite

pytestmark = pytest.mark.gpu


def test_observable_buffers_plateau():
    from paper_2301_05844_amd import bbp
    A = peps_finite(8, 8, 2, seed=2)
    g = bbp.BlockBP(Lx=8, Ly=8, bx=2, by=2, D=2, chi=4)
    g.set_tensors(A)
    held = []
    for rep in range(6):
        # three query shapes: a block (site), a horizontal and a vertical
        # union of two blocks (bonds crossing blocks); a sweep between calls
        # invalidates the region results, so every call recomputes
        for q in range(3):
            g.sweep(1)
            if q == 0:
                g.expect_site(rep % 8, 3, op_sz())
            elif q == 1:
                g.expect_bond(1, rep % 8, 2, rep % 8, op_heis())
            else:
                g.expect_bond(rep % 8, 1, rep % 8, 2, op_heis())
            held.append(g.memory()[0])
    print("device bytes held after each call:", held, flush=True)
    assert max(held[6:]) <= max(held[:6])
    assert np.isfinite(g.log_norm()[0])
