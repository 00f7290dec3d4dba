"""Pins of the oracle's shifted partitions, reduced density matrices and
trace distance (Sec. II: observables at the centre of a block, several
partitions of the lattice that differ by a shift; App. C: trace distances
between reduced density matrices).  CPU only."""

import math

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sx, op_sz, peps_finite
from oracle import blockbp as ob
from oracle import brute

TOL = 1e-12


def _exact_rdm_bond(A, Lx, Ly, i, j, d=2):
    """rho[(s0,s1),(s0',s1')] of sites i, j by exact strip contraction."""
    Z = brute.strip_value(A, Lx, Ly)
    rho = np.zeros((d * d, d * d))
    for s0 in range(d):
        for s1 in range(d):
            for s0p in range(d):
                for s1p in range(d):
                    u0 = np.zeros((d, d))
                    u1 = np.zeros((d, d))
                    u0[s0p, s0] = 1.0
                    u1[s1p, s1] = 1.0
                    rho[s0 * d + s1, s0p * d + s1p] = \
                        brute.strip_value(A, Lx, Ly, {i: u0, j: u1}) / Z
    return rho


# --- trace distance (App. C) ---------------------------------------------------
def test_trace_distance_closed_forms():
    rng = np.random.default_rng(0)
    # commuting (diagonal) states: half the l1 distance of the spectra
    p, q = rng.random(4), rng.random(4)
    p, q = p / p.sum(), q / q.sum()
    assert abs(ob.trace_distance(np.diag(p), np.diag(q))
               - 0.5 * np.abs(p - q).sum()) < 1e-15
    # pure states: sqrt(1 - |<psi|phi>|^2)
    a, b = rng.standard_normal(4), rng.standard_normal(4)
    a, b = a / np.linalg.norm(a), b / np.linalg.norm(b)
    ref = math.sqrt(1.0 - np.dot(a, b) ** 2)
    assert abs(ob.trace_distance(np.outer(a, a), np.outer(b, b)) - ref) < 1e-14
    # unitary invariance, zero on equal arguments, symmetric
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    r, s = np.outer(a, a), np.diag(q)
    assert abs(ob.trace_distance(Q @ r @ Q.T, Q @ s @ Q.T)
               - ob.trace_distance(r, s)) < 1e-14
    assert ob.trace_distance(r, r) == 0.0
    assert ob.trace_distance(r, s) == ob.trace_distance(s, r)


# --- reduced density matrices ---------------------------------------------------
def test_rdms_reproduce_expectation_values():
    A = peps_finite(4, 4, 2, seed=3)
    bp = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4, chi_env=18)
    bp.sweep(10)
    for (x, y) in [(1, 1), (2, 3)]:
        rho = bp.rdm_site(x, y)
        assert abs(np.trace(rho) - 1.0) < TOL
        assert np.abs(rho - rho.T).max() < TOL
        for op in (op_sz(), op_sx()):
            assert abs(np.trace(rho @ op) - bp.expect_site(x, y, op)) < TOL
    for b in [(1, 1, 2, 1), (2, 1, 2, 2), (0, 0, 1, 0)]:
        rho = bp.rdm_bond(*b)
        assert abs(np.trace(rho) - 1.0) < TOL
        assert abs(np.trace(rho @ op_heis()) - bp.expect_bond(*b, op_heis())) < TOL


def test_bond_rdm_equals_brute_force_when_exact():
    # one 4x4 block covering the lattice: exact
    A = peps_finite(4, 4, 2, seed=8)
    bp = ob.BlockBP(A, D=2, chi=4, bx=4, by=4, Lx=4, Ly=4, chi_env=64)
    psi = brute.state_vector(A, 4, 4)
    for (x, y) in [(0, 0), (2, 1)]:
        i, j = y * 4 + x, y * 4 + x + 1
        rho = _exact_rdm_bond(A, 4, 4, i, j)
        assert ob.trace_distance(bp.rdm_bond(x, y, x + 1, y), rho) < TOL
        # the same matrix from the state vector: <S.S> as a check of the layout
        assert abs(np.trace(rho @ op_heis())
                   - brute.expect_bond(psi, i, j, op_heis())) < TOL


# --- shifted partitions (Sec. II) -----------------------------------------------
def test_zero_shift_is_the_default_partition():
    A = peps_finite(6, 6, 2, seed=2)
    a = ob.BlockBP(A, D=2, chi=4, bx=3, by=3, Lx=6, Ly=6)
    b = ob.BlockBP(A, D=2, chi=4, bx=3, by=3, Lx=6, Ly=6, shift=(0, 0))
    assert a.sweep(4) == b.sweep(4)
    assert a.expect_bond(2, 2, 3, 2, op_heis()) == b.expect_bond(2, 2, 3, 2, op_heis())


@pytest.mark.parametrize("Lx,Ly,b,shift", [
    (4, 4, 4, (2, 0)),   # two blocks side by side (a tree)
    (4, 4, 4, (0, 3)),   # two blocks stacked
    (3, 3, 4, (1, 1)),   # one block holds the whole shifted lattice
    (4, 2, 2, (1, 0)),   # three blocks in a row
])
def test_shifted_partitions_exact_on_trees(Lx, Ly, b, shift):
    """A shifted partition whose block graph is a tree is exact at its fixed
    point (Sec. II), with chi and chi_env above the exact ranks; the shift
    pads trivial sites on the left and top, which leave the network's value
    unchanged."""
    A = peps_finite(Lx, Ly, 2, seed=4)
    bp = ob.BlockBP(A, D=2, chi=16, bx=b, by=b, Lx=Lx, Ly=Ly, chi_env=64, shift=shift)
    bp.sweep(4)
    psi = brute.state_vector(A, Lx, Ly)
    for y in range(Ly):
        for x in range(Lx):
            assert abs(bp.expect_site(x, y, op_sz())
                       - brute.expect_site(psi, y * Lx + x, op_sz())) < TOL
    for y in range(Ly):
        for x in range(Lx - 1):
            assert abs(bp.expect_bond(x, y, x + 1, y, op_heis())
                       - brute.expect_bond(psi, y * Lx + x, y * Lx + x + 1,
                                           op_heis())) < TOL
    assert abs(bp.log_norm()[0] - math.log(brute.norm2(psi))) < TOL


def test_shift_must_lie_inside_a_block():
    A = peps_finite(4, 4, 2, seed=0)
    with pytest.raises(ValueError):
        ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4, shift=(2, 0))


def test_centre_depth_and_best_shift():
    # block of 4: coordinates 1 and 2 are the centre (depth 1)
    assert [ob.centre_depth(4, 0, x, x) for x in range(4)] == [0, 1, 1, 0]
    assert ob.centre_depth(4, 0, 1, 2) == 1        # bond at the centre
    assert ob.centre_depth(4, 0, 3, 4) == -1       # bond across two blocks
    assert ob.centre_depth(4, 2, 3, 4) == 1        # shifted by 2: positions 5, 6 -> 1, 2
    assert ob.centre_depth(4, 1, 2, 3) == -1       # shifted by 1: 3, 4 in two blocks
    shifts = [(sx, sy) for sy in range(4) for sx in range(4)]
    for x in range(8):
        (sx, sy), dep = ob.best_shift(4, 4, shifts, x, 5, x + 1, 5)
        assert dep == 1 and (x + sx) % 4 == 1 and (5 + sy) % 4 in (1, 2)


def test_block_rdms_far_closer_than_plain_bp():
    """App. C: bond reduced density matrices of block BP (3x3 blocks) lie far
    closer to the exact ones than those of plain BP (blocks of one site, the
    simple-update environment).  A 6x6 lattice with a more strongly
    correlated state (noise 0.4)."""
    A = peps_finite(6, 6, 2, seed=7, noise=0.4)
    res = {}
    for b, chi_env in ((3, 18), (1, 8)):
        bp = ob.BlockBP(A, D=2, chi=4, bx=b, by=b, Lx=6, Ly=6, chi_env=chi_env)
        for _ in range(60):
            if bp.sweep() < 1e-14:
                break
        res[b] = bp
    tds = {1: [], 3: []}
    for y in (1, 4):
        for x in range(5):
            ex = _exact_rdm_bond(A, 6, 6, y * 6 + x, y * 6 + x + 1)
            for b in (1, 3):
                tds[b].append(ob.trace_distance(res[b].rdm_bond(x, y, x + 1, y), ex))
    assert max(tds[3]) < min(tds[1]) / 4
    assert max(tds[3]) < 1e-2 and min(tds[1]) > 1e-2
