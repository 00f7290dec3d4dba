"""Degenerate and extreme cases of the block-BP path against the oracle:
D = 1 (product states: every message a scalar, block BP exact), single-site
blocks (plain BP), one-row lattices, bond cap 1, the largest bond caps the
ABI accepts (chi = chi_env = 128), empty queries and an infinite lattice
whose block is the unit cell."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite, peps_infinite
from oracle import blockbp as ob
from oracle import brute

pytestmark = pytest.mark.gpu


def _all_terms(Lx, Ly):
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    return xs, ys, bonds


def _compare(kw, sweeps, seed=2, tol=1e-10, exact=False):
    from paper_2301_05844_amd import bbp
    Lx, Ly, D = kw["Lx"], kw["Ly"], kw["D"]
    A = peps_finite(Lx, Ly, D, seed=seed)
    g = bbp.BlockBP(**kw)
    g.set_tensors(A)
    okw = {k: v for k, v in kw.items() if k != "chi_env"}
    ref = ob.BlockBP(A, **okw, chi_env=kw.get("chi_env"))
    r_gpu = g.sweep(sweeps)
    r_ref = ref.sweep(sweeps)
    xs, ys, bonds = _all_terms(Lx, Ly)
    sz = g.expect_sites(xs, ys, op_sz())
    ss = g.expect_bonds(bonds, op_heis()) if bonds else []
    e_sz = max(abs(sz[i] - ref.expect_site(int(xs[i]), int(ys[i]), op_sz()))
               for i in range(len(xs)))
    e_ss = max([abs(ss[i] - ref.expect_bond(*b, op_heis())) for i, b in enumerate(bonds)]
               or [0.0])
    lz, _ = g.log_norm()
    e_lz = abs(lz - ref.log_norm()[0])
    print(f"{kw}: residual {r_gpu:.2e} (oracle {r_ref:.2e}), max |d sz| {e_sz:.1e}, "
          f"max |d SS| {e_ss:.1e}, |d log-norm| {e_lz:.1e}", flush=True)
    assert e_sz < tol and e_ss < tol and e_lz < tol * max(1.0, abs(lz))
    if exact:  # the block graph is a tree or the state a product: exact contraction
        psi = brute.state_vector(A, Lx, Ly)
        for i in range(len(xs)):
            exact_sz = brute.expect_site(psi, int(ys[i]) * Lx + int(xs[i]), op_sz())
            assert abs(sz[i] - exact_sz) < 1e-10


def test_product_state_D1_is_exact():
    _compare(dict(Lx=4, Ly=4, bx=2, by=2, D=1, chi=1), 2, exact=True)


def test_single_site_blocks_plain_bp():
    _compare(dict(Lx=4, Ly=3, bx=1, by=1, D=2, chi=4), 12)


def test_one_row_lattice():
    _compare(dict(Lx=8, Ly=1, bx=4, by=1, D=3, chi=9), 3)


def test_one_column_lattice():
    _compare(dict(Lx=1, Ly=8, bx=1, by=4, D=3, chi=9), 3)


def test_bond_cap_one():
    _compare(dict(Lx=6, Ly=6, bx=3, by=3, D=2, chi=1, chi_env=4), 4)


def test_largest_bond_caps():
    # chi = chi_env = 128 (the ABI's limit): the tiled D = 4 visit at K = 128,
    # every true bond far below the cap
    _compare(dict(Lx=4, Ly=4, bx=2, by=2, D=4, chi=128, chi_env=128), 3)


def test_empty_queries():
    from paper_2301_05844_amd import bbp
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    g.set_tensors(peps_finite(4, 4, 2, seed=1))
    g.sweep(2)
    assert len(g.expect_sites(np.zeros(0, np.int32), np.zeros(0, np.int32), op_sz())) == 0
    assert len(g.expect_bonds([], op_heis())) == 0
    assert len(g.rdm_sites(np.zeros(0, np.int32), np.zeros(0, np.int32))) == 0


def test_infinite_block_equal_to_cell():
    from paper_2301_05844_amd import bbp
    A = peps_infinite(2, 2, 2, seed=3)
    kw = dict(D=2, chi=8, bx=2, by=2, infinite=True, ucx=2, ucy=2)
    g = bbp.BlockBP(**kw)
    g.set_tensors(A)
    ref = ob.BlockBP(A, **kw)
    for _ in range(5):
        r_gpu, r_ref = g.sweep(1), ref.sweep()
        assert abs(r_gpu - r_ref) <= 1e-6 * r_ref + 1e-14
    for (x, y) in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        assert abs(g.expect_site(x, y, op_sz()) - ref.expect_site(x, y, op_sz())) < 1e-10
