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


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_05844_amd import bbp
    return bbp


@pytest.mark.parametrize("beta,b,chi,tol_onsager", [(0.8, 4, 4, 1e-6), (0.6, 2, 2, 1e-3),
                                                    (0.6, 4, 8, 1e-4)])
def test_single_layer_ising_magnetisation(beta, b, chi, tol_onsager):
    """The single-layer network of the classical Ising model (bond dimension
    2; the "single_layer" option): the GPU's centre magnetisation equals the
    oracle's after the same sweeps and lies within the block-BP error of
    Onsager's closed form (Sec. V).  (At beta 0.6 with 4x4 blocks a message
    bond of 4 truncates at a nearly degenerate point: the oracle's own fixed
    point moves by 1.6e-9 under a 1e-14 change of the tensors, so parity is
    taken at bond 8, where it moves by 5e-14.)"""
    from bbp_inputs import ising_single_layer
    from oracle.blockbp import BlockBP as OracleBP
    bbp = _gpu()
    A = ising_single_layer(beta, 1e-6)
    ref = OracleBP(A, D=2, chi=chi, bx=b, by=b, infinite=True, ucx=1, ucy=1, single_layer=True)
    g = bbp.BlockBP(infinite=True, ucx=1, ucy=1, bx=b, by=b, D=2, chi=chi, single_layer=1)
    g.set_tensors(A)
    n = 0
    for n in range(1, 201):
        r_ref = ref.sweep()
        r = g.sweep(1)
        if r_ref < 1e-13:
            break
    m, m_ref = g.expect_site(0, 0, op_sz()), ref.expect_site(0, 0, op_sz())
    onsager = (1 - np.sinh(2 * beta) ** -4) ** 0.125
    print(f"single layer beta {beta} block {b} chi {chi}: {n} sweeps (residual {r:.1e}), "
          f"m {m:.12f}, oracle {m_ref:.12f}, Onsager {onsager:.12f}", flush=True)
    assert abs(m - m_ref) < 1e-10
    assert abs(m - onsager) < tol_onsager


def test_single_layer_finite_lattice_matches_oracle():
    """An open 8x8 single-layer Ising network in a field (4x4 blocks, message
    bonds truncated to 4): every site's magnetisation and log Z after six
    sweeps against the oracle."""
    from bbp_inputs import ising_single_layer
    from oracle.blockbp import BlockBP as OracleBP
    bbp = _gpu()
    A = ising_single_layer(0.45, 0.1, 8, 8)
    ref = OracleBP(A, D=2, chi=4, bx=4, by=4, Lx=8, Ly=8, chi_env=8, single_layer=True)
    g = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=2, chi=4, chi_env=8, single_layer=1)
    g.set_tensors(A)
    res = [g.sweep(1) for _ in range(6)]
    rref = [ref.sweep() for _ in range(6)]
    for a, r_ in zip(res, rref):
        assert abs(a - r_) <= 1e-6 * r_ + 1e-14
    xs = [x for y in range(8) for x in range(8)]
    ys = [y for y in range(8) for x in range(8)]
    m = g.expect_sites(xs, ys, op_sz())
    err = max(abs(m[i] - ref.expect_site(xs[i], ys[i], op_sz())) for i in range(64))
    lz, ref_lz = g.log_norm()[0], ref.log_norm()[0]
    print(f"single layer 8x8: max |d m| {err:.2e}, log Z {lz:.12f} vs {ref_lz:.12f}", flush=True)
    assert err < 1e-10 and abs(lz - ref_lz) < 1e-10 * abs(ref_lz)
