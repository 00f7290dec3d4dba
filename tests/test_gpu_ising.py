"""Classical Ising on the infinite lattice through the PEPS whose norm is
its partition function: the GPU's magnetisation equals the oracle's after the
same sweeps and lies within the block-BP error of Onsager's closed form."""

import numpy as np
import pytest

from bbp_inputs import ising_peps, op_sz

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("beta,b,chi,tol_onsager", [(0.8, 4, 8, 1e-6), (0.6, 2, 4, 1e-3)])
def test_ising_magnetisation(beta, b, chi, tol_onsager):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle.blockbp import BlockBP as OracleBP
    from paper_2301_05844_amd import bbp
    A = ising_peps(beta, 1e-6)
    ref = OracleBP(A, D=2, chi=chi, bx=b, by=b, infinite=True, ucx=1, ucy=1)
    g = bbp.BlockBP(infinite=True, ucx=1, ucy=1, bx=b, by=b, D=2, chi=chi)
    g.set_tensors(A)
    n = 0
    for n in range(1, 121):
        r_ref = ref.sweep()
        r = g.sweep(1)
        if r_ref < 1e-12:
            break
    m = g.expect_site(0, 0, op_sz())
    m_ref = ref.expect_site(0, 0, op_sz())
    onsager = (1 - np.sinh(2 * beta) ** -4) ** 0.125
    print(f"beta {beta} block {b} chi {chi}: {n} sweeps, m {m:.10f}, oracle {m_ref:.10f}, "
          f"Onsager {onsager:.10f}")
    assert abs(m - m_ref) < 1e-10
    assert abs(m - onsager) < tol_onsager
