"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU and never touches the GPU library.

P1a  one block covering the whole lattice, chi_env above the exact rank:
     equals the brute-force state vector (App. B procedure exact when nothing
     is truncated).
P1b  tree block graphs: block BP is exact at its fixed point (Sec. II,
     paragraph after Eq. (1)), checked against brute force for all four
     message directions.
P1c  one loop (4x4 lattice, 2x2 blocks): a small, nonzero block-BP error.
P2   D=1 product states: closed forms.
P3   blocks of one site reduce to plain BP (Sec. II).
P4   the fit's loss identity (App. A) and exactness when chi >= rank.
P5   rescaling invariance and log-norm shift; gauge invariance, a quarter
     turn and a mirror image of the lattice (untruncated cases).
P6   ket<->bra symmetry of messages (real tensors, untruncated).
P7   the fixed-point iteration converges: per-sweep observable changes
     bounded by the residual, and below 1e-10 at the rounding floor.
P8   the infinite lattice is the limit of finite tilings of its unit cell
     (Sec. II iPEPS paragraph; App. E), which pins the self-message routing.
Mutations planted in the oracle must make the pins fail.
"""

import math

import numpy as np
import pytest

from bbp_inputs import (op_heis, op_sx, op_sz, op_szsz, peps_finite,
                        peps_infinite)
from oracle import blockbp as ob
from oracle import brute
from oracle.plain_bp import PlainBP

TOL = 1e-12


def _psi_checks(A, Lx, Ly, bp, sites=None, bonds=None):
    psi = brute.state_vector(A, Lx, Ly)
    sites = sites or [(x, y) for y in range(Ly) for x in range(Lx)]
    err = 0.0
    for (x, y) in sites:
        err = max(err, abs(bp.expect_site(x, y, op_sz())
                           - brute.expect_site(psi, y * Lx + x, op_sz())))
    if bonds is None:
        bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
        bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    for (x0, y0, x1, y1) in bonds:
        err = max(err, abs(bp.expect_bond(x0, y0, x1, y1, op_heis())
                           - brute.expect_bond(psi, y0 * Lx + x0,
                                               y1 * Lx + x1, op_heis())))
    lz, sign = bp.log_norm()
    return err, abs(lz - math.log(brute.norm2(psi))), sign


# --- generator and brute force ------------------------------------------------
def test_splitmix_published_value():
    # First output of SplitMix64 from state 0 (reference implementation).
    assert int(ob._splitmix(np.uint64(0))) == 0xE220A8397B1DCDAF
    u = ob.counter_uniform(7, 11, 3, 1000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert np.all(np.round(u * 2.0 ** 52) == u * 2.0 ** 52)
    assert abs(u.mean()) < 0.1


def test_operators():
    # S.S has the singlet at -3/4 and the triplet at +1/4.
    ev = np.sort(np.linalg.eigvalsh(op_heis()))
    assert np.allclose(ev, [-0.75, 0.25, 0.25, 0.25], atol=1e-15)
    assert np.allclose(np.linalg.eigvalsh(op_szsz()), [-1, -1, 1, 1])


def test_two_brute_force_methods_agree():
    A = peps_finite(3, 3, 2, seed=4)
    psi = brute.state_vector(A, 3, 3)
    assert abs(brute.norm2(psi) - brute.strip_value(A, 3, 3)) < 1e-12
    assert abs(brute.expect_site(psi, 4, op_sz())
               - brute.strip_expect_site(A, 3, 3, 4, op_sz())) < 1e-13
    assert abs(brute.expect_bond(psi, 4, 5, op_heis())
               - brute.strip_expect_bond(A, 3, 3, 4, 5, op_heis())) < 1e-13


def test_state_vector_product_state():
    A = peps_finite(3, 2, 1, seed=5)
    psi = brute.state_vector(A, 3, 2)
    a = A[:, :, 0, 0, 0, 0]
    dense = a[0]
    for t in a[1:]:
        dense = np.multiply.outer(dense, t)
    assert np.allclose(psi, dense, atol=1e-15)


# --- P1 -----------------------------------------------------------------------
def test_p1a_single_block_is_exact():
    A = peps_finite(4, 4, 2, seed=0)
    bp = ob.BlockBP(A, D=2, chi=4, bx=4, by=4, Lx=4, Ly=4, chi_env=64)
    assert bp.order == []
    err, lerr, sign = _psi_checks(A, 4, 4, bp)
    assert err < TOL and lerr < TOL and sign == 1.0


@pytest.mark.parametrize("Lx,Ly,bx,by,chi,chi_env,sweeps", [
    (4, 2, 2, 2, 4, 18, 3),    # 2 blocks side by side: L and R messages
    (2, 6, 2, 2, 4, 18, 4),    # 3 blocks stacked: U and D messages
    (6, 2, 2, 2, 4, 18, 4),
    (4, 3, 2, 3, 9, 36, 3),    # non-square blocks
])
def test_p1b_tree_block_graph_is_exact(Lx, Ly, bx, by, chi, chi_env, sweeps):
    A = peps_finite(Lx, Ly, 2, seed=1)
    bp = ob.BlockBP(A, D=2, chi=chi, bx=bx, by=by, Lx=Lx, Ly=Ly,
                    chi_env=chi_env)
    res = bp.sweep(sweeps)
    assert res < 1e-13
    err, lerr, sign = _psi_checks(A, Lx, Ly, bp)
    assert err < TOL and lerr < TOL and sign == 1.0


@pytest.mark.parametrize("Lx,Ly,bx,by,chi,chi_env,sweeps", [
    (6, 2, 2, 2, 4, 18, 5),
    (4, 3, 2, 3, 9, 36, 4),
])
def test_random_initial_messages_reach_the_exact_fixed_point(Lx, Ly, bx, by, chi,
                                                            chi_env, sweeps):
    """The random product MPDO start (init 1, App. A): every initial site is
    positive semidefinite with unit norm, the start differs from the
    identity one, and on a tree block graph the sweeps still reach the
    exact contraction (BP's fixed point on a tree does not depend on the
    start)."""
    A = peps_finite(Lx, Ly, 2, seed=1)
    bp = ob.BlockBP(A, D=2, chi=chi, bx=bx, by=by, Lx=Lx, Ly=Ly,
                    chi_env=chi_env, init=1, seed=7)
    ident = ob.identity_mps(by, 2)
    for key, m in bp.msgs.items():
        for t in m:
            M = t.reshape(2, 2)
            assert abs(np.linalg.norm(M) - 1.0) < 1e-14
            assert np.allclose(M, M.T) and np.linalg.eigvalsh(M).min() > -1e-14
        if key[2] in ("L", "R"):
            assert not np.allclose(m[0], ident[0])
    res = bp.sweep(sweeps)
    assert res < 1e-13
    err, lerr, sign = _psi_checks(A, Lx, Ly, bp)
    assert err < TOL and lerr < TOL and sign == 1.0


def test_p1b_large_blocks_strip():
    A = peps_finite(8, 4, 2, seed=2)
    bp = ob.BlockBP(A, D=2, chi=16, bx=4, by=4, Lx=8, Ly=4, chi_env=64)
    bp.sweep(3)
    for (x, y) in [(1, 1), (4, 2), (7, 0)]:
        ref = brute.strip_expect_site(A, 8, 4, y * 8 + x, op_sz())
        assert abs(bp.expect_site(x, y, op_sz()) - ref) < TOL
    for (x0, y0, x1, y1) in [(3, 1, 4, 1), (5, 2, 5, 3)]:
        ref = brute.strip_expect_bond(A, 8, 4, y0 * 8 + x0, y1 * 8 + x1,
                                      op_heis())
        assert abs(bp.expect_bond(x0, y0, x1, y1, op_heis()) - ref) < TOL
    assert abs(bp.log_norm()[0] - math.log(brute.strip_value(A, 8, 4))) < TOL


def test_p1c_one_loop_error_is_small_and_nonzero():
    A = peps_finite(4, 4, 2, seed=0)
    bp = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4, chi_env=18)
    res = bp.sweep(30)
    assert res < 1e-14
    err, lerr, _ = _psi_checks(A, 4, 4, bp, sites=[(0, 0), (1, 2), (3, 1)],
                               bonds=[(1, 1, 2, 1), (2, 1, 2, 2)])
    assert 1e-9 < err < 1e-2
    assert lerr < 1e-2


# --- P2 -----------------------------------------------------------------------
def _product_values(A):
    a0, a1 = A[:, 0, 0, 0, 0, 0], A[:, 1, 0, 0, 0, 0]
    n = a0 ** 2 + a1 ** 2
    return (a0 ** 2 - a1 ** 2) / n, 2 * a0 * a1 / n, n


def test_p2_product_state_finite():
    A = peps_finite(5, 4, 1, seed=2)
    bp = ob.BlockBP(A, D=1, chi=2, bx=2, by=2, Lx=5, Ly=4)
    assert bp.sweep(2) == 0.0
    sz, sx, n = _product_values(A)
    for i in range(20):
        x, y = i % 5, i // 5
        assert abs(bp.expect_site(x, y, op_sz()) - sz[i]) < 1e-14
        assert abs(bp.expect_site(x, y, op_sx()) - sx[i]) < 1e-14
    for (i, j) in [(6, 7), (6, 11), (8, 9), (13, 18)]:
        x0, y0, x1, y1 = i % 5, i // 5, j % 5, j // 5
        ref = 0.25 * (sz[i] * sz[j] + sx[i] * sx[j])
        assert abs(bp.expect_bond(x0, y0, x1, y1, op_heis()) - ref) < 1e-14
    assert abs(bp.log_norm()[0] - np.sum(np.log(n))) < 1e-13


def test_p2_product_state_infinite():
    A = peps_infinite(2, 2, 1, seed=3)
    bp = ob.BlockBP(A, D=1, chi=2, bx=4, by=4, infinite=True, ucx=2, ucy=2)
    assert bp.sweep(2) == 0.0
    sz, sx, n = _product_values(A)
    for c in range(4):
        x, y = c % 2, c // 2
        assert abs(bp.expect_site(x, y, op_sz()) - sz[c]) < 1e-14
        assert abs(bp.expect_site(x, y, op_sx()) - sx[c]) < 1e-14
        xr = (x + 1) % 2
        assert abs(bp.expect_bond(x, y, x + 1, y, op_szsz())
                   - sz[c] * sz[y * 2 + xr]) < 1e-14
    # one 4x4 block holds four copies of the cell
    assert abs(bp.log_norm()[0] - 4 * np.sum(np.log(n))) < 1e-13


# --- P3 -----------------------------------------------------------------------
def test_p3_single_site_blocks_are_plain_bp():
    A = peps_finite(3, 3, 2, seed=1)
    bp = ob.BlockBP(A, D=2, chi=4, bx=1, by=1, Lx=3, Ly=3, chi_env=8)
    pb = PlainBP(A, 3, 3)
    for _ in range(6):
        bp.sweep()
        pb.sweep()
    for (bi, bj, dr), m in bp.msgs.items():
        v = m[0].reshape(-1)
        w = pb.m[(bi, bj, dr)]
        assert min(np.abs(v - w).max(), np.abs(v + w).max()) < TOL
    for y in range(3):
        for x in range(3):
            assert abs(bp.expect_site(x, y, op_sz())
                       - pb.expect_site(x, y, op_sz())) < TOL


def test_p3_chain_is_exact():
    A = peps_finite(6, 1, 2, seed=6)
    bp = ob.BlockBP(A, D=2, chi=4, bx=1, by=1, Lx=6, Ly=1, chi_env=8)
    bp.sweep(6)
    err, lerr, _ = _psi_checks(A, 6, 1, bp)
    assert err < TOL and lerr < TOL


# --- P4 -----------------------------------------------------------------------
def _random_mpo_mps(rng, N, p, w, bx):
    O = [rng.standard_normal(((w if j else 1), p, p, (w if j < N - 1 else 1)))
         for j in range(N)]
    X = [rng.standard_normal(((bx if j else 1), p, (bx if j < N - 1 else 1)))
         for j in range(N)]
    return O, X


def _dense_ox(O, X):
    v = np.ones((1, 1, 1))  # [out..., w, x]
    for o, x in zip(O, X):
        v = np.einsum("...wx,wpqv,xqz->...pvz", v, o, x)
    return v.reshape(-1)


def test_p4_fit_exact_when_untruncated():
    rng = np.random.default_rng(0)
    O, X = _random_mpo_mps(rng, 5, 2, 2, 2)
    Y, nu = ob.fit(O, X, chi=64, n_fit=1, seed=1, slot=2)
    Y[0] = Y[0]  # centre carries the norm
    ref = _dense_ox(O, X)
    assert np.abs(ob.mps_dense(Y) - ref).max() < 1e-12 * np.abs(ref).max()
    assert abs(nu - np.linalg.norm(ref)) < 1e-12 * nu


def test_p4_fit_loss_identity():
    rng = np.random.default_rng(1)
    O, X = _random_mpo_mps(rng, 6, 3, 2, 3)
    ref = _dense_ox(O, X)
    for n_fit in (1, 2, 4):
        Y, nu = ob.fit(O, X, chi=4, n_fit=n_fit, seed=3, slot=4)
        y = ob.mps_dense(Y)
        # ||Y - OX||^2 = ||OX||^2 - ||Yt||^2 when Y holds the optimal centre
        lhs = np.sum((y - ref) ** 2)
        rhs = np.sum(ref ** 2) - nu ** 2
        assert abs(lhs - rhs) < 1e-10 * np.sum(ref ** 2)
    # more sweeps never increase the loss
    losses = []
    for n_fit in (1, 2, 3, 6):
        Y, nu = ob.fit(O, X, chi=4, n_fit=n_fit, seed=3, slot=4)
        losses.append(np.sum(ref ** 2) - nu ** 2)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(losses, losses[1:]))


# --- P5, P6 ---------------------------------------------------------------------
def test_p5_rescaling_and_gauge():
    A = peps_finite(4, 4, 2, seed=0)
    base = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4, chi_env=18)
    base.sweep(8)
    B = A.copy()
    B[5] *= 3.7
    sc = ob.BlockBP(B, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4, chi_env=18)
    sc.sweep(8)
    for (x, y) in [(1, 1), (2, 3)]:
        assert abs(base.expect_site(x, y, op_sz())
                   - sc.expect_site(x, y, op_sz())) < TOL
    assert abs(sc.log_norm()[0] - base.log_norm()[0]
               - 2 * math.log(3.7)) < TOL
    # gauge G, G^-1 on the bond between sites 1 and 2 (inside block (0,0)
    # and block (1,0)); untruncated tree case 4x2 with 2x2 blocks
    A = peps_finite(4, 2, 2, seed=1)
    G = np.eye(2) + 0.3 * np.random.default_rng(9).standard_normal((2, 2))
    Gi = np.linalg.inv(G)
    C = A.copy()
    C[1] = np.einsum("suldr,re->sulde", A[1], G)
    C[2] = np.einsum("el,suldr->suedr", Gi, A[2])
    r1 = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=2, chi_env=18)
    r2 = ob.BlockBP(C, D=2, chi=4, bx=2, by=2, Lx=4, Ly=2, chi_env=18)
    r1.sweep(3)
    r2.sweep(3)
    for (x, y) in [(1, 0), (2, 1)]:
        assert abs(r1.expect_site(x, y, op_sz())
                   - r2.expect_site(x, y, op_sz())) < TOL


def test_p6_messages_symmetric_under_ket_bra_swap():
    A = peps_finite(4, 4, 2, seed=0)
    bp = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=4, Ly=4)
    bp.sweep(5)
    D = 2
    for m in bp.msgs.values():
        sw = [t.reshape(t.shape[0], D, D, t.shape[2]).transpose(0, 2, 1, 3)
              .reshape(t.shape) for t in m]
        assert abs(abs(ob.mps_overlap(m, sw)) - 1.0) < TOL


# --- planted mistakes -------------------------------------------------------
def _tree_error(Lx, Ly):
    A = peps_finite(Lx, Ly, 2, seed=1)
    bp = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=Lx, Ly=Ly, chi_env=18)
    bp.sweep(4)
    return _psi_checks(A, Lx, Ly, bp)[0]


@pytest.mark.parametrize("mutation", ["perm_U", "perm_R", "reverse_D",
                                      "mpo_legs", "caps"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "perm_U":
        monkeypatch.setitem(ob.ROT_PERM, "U", (0, 4, 3, 2, 1))
        err = _tree_error(2, 6)
    elif mutation == "perm_R":
        monkeypatch.setitem(ob.ROT_PERM, "R", (0, 3, 2, 1, 4))
        err = _tree_error(6, 2)
    elif mutation == "reverse_D":
        monkeypatch.setitem(ob.OUT_REVERSED, "D", True)
        err = _tree_error(2, 6)
    elif mutation == "mpo_legs":
        orig = ob.column_mpo

        def bad(Egrid, MT, MB, c):
            O = orig(Egrid, MT, MB, c)
            return [O[0]] + [o.transpose(0, 2, 1, 3) for o in O[1:-1]] + [O[-1]]
        monkeypatch.setattr(ob, "column_mpo", bad)
        err = _tree_error(4, 2)
    else:
        orig = ob.bond_caps

        def bad(O, X, chi):
            p, b = orig(O, X, chi)
            return p, [max(1, v - 1) for v in b]
        monkeypatch.setattr(ob, "bond_caps", bad)
        err = _tree_error(4, 2)
    assert err > 1e-6


# ---- classical Ising through the PEPS whose norm is its partition function ----

def _ising_brute(beta, h, Lx, Ly):
    """Classical sums over all 2^(Lx*Ly) configurations: <s> per site."""
    import itertools
    n = Lx * Ly
    Z = 0.0
    m = np.zeros(n)
    for conf in itertools.product((1, -1), repeat=n):
        s = np.array(conf).reshape(Ly, Lx)
        e = beta * ((s[:, :-1] * s[:, 1:]).sum() + (s[:-1, :] * s[1:, :]).sum()) + h * s.sum()
        w = np.exp(e)
        Z += w
        m += w * s.ravel()
    return m / Z


def test_ising_peps_norm_is_the_classical_partition_function():
    """One block covering a 3x3 open lattice (exact): <sigma_z> of the Ising
    PEPS equals the classical magnetisation summed over all configurations."""
    from bbp_inputs import ising_peps
    from oracle.blockbp import BlockBP
    beta, h = 0.7, 0.3
    A = ising_peps(beta, h, 3, 3)
    g = BlockBP(A, D=2, chi=4, bx=3, by=3, Lx=3, Ly=3)
    m = _ising_brute(beta, h, 3, 3)
    for y in range(3):
        for x in range(3):
            assert abs(g.expect_site(x, y, op_sz()) - m[y * 3 + x]) < 1e-12


def _ising_infinite_m(beta, b, chi, h=1e-6):
    from bbp_inputs import ising_peps
    from oracle.blockbp import BlockBP
    g = BlockBP(ising_peps(beta, h), D=2, chi=chi, bx=b, by=b, infinite=True, ucx=1, ucy=1)
    for _ in range(120):
        if g.sweep() < 1e-12:
            break
    return g.expect_site(0, 0, op_sz())


def test_ising_magnetisation_approaches_onsager():
    """Infinite lattice below T_c (beta_c = 0.4407): block BP's magnetisation
    approaches Onsager and Yang's closed form (1 - sinh(2 beta)^-4)^(1/8) and
    improves with the block size."""
    onsager = lambda beta: (1 - np.sinh(2 * beta) ** -4) ** 0.125
    assert abs(_ising_infinite_m(0.8, 4, 8) - onsager(0.8)) < 1e-6
    e2 = abs(_ising_infinite_m(0.6, 2, 4) - onsager(0.6))
    e4 = abs(_ising_infinite_m(0.6, 4, 8) - onsager(0.6))
    assert e4 < 1e-4 and e4 < 0.5 * e2


# --- P5: lattice symmetries (untruncated loopy case) ---------------------------
def _c1_observables(A, Lx, Ly):
    bp = ob.BlockBP(A, D=2, chi=4, bx=2, by=2, Lx=Lx, Ly=Ly, chi_env=18)
    bp.sweep(30)
    sz = {(x, y): bp.expect_site(x, y, op_sz())
          for y in range(Ly) for x in range(Lx)}
    ss = {}
    for y in range(Ly):
        for x in range(Lx):
            if x + 1 < Lx:
                ss[frozenset({(x, y), (x + 1, y)})] = bp.expect_bond(
                    x, y, x + 1, y, op_heis())
            if y + 1 < Ly:
                ss[frozenset({(x, y), (x, y + 1)})] = bp.expect_bond(
                    x, y, x, y + 1, op_heis())
    return sz, ss, bp.log_norm()[0]


@pytest.mark.parametrize("how", ["rotate", "transpose"])
def test_p5_rotation_and_transpose_invariance(how):
    """The 4x4 lattice with 2x2 blocks is a loop of four blocks with chi and
    chi_env above every exact rank: its block-BP fixed point is a property of
    the network, so turning or mirroring the lattice permutes the observables
    and keeps the log-norm (to rounding), although every message now runs
    through other orientation code."""
    from bbp_inputs import peps_rotate, peps_transpose
    A = peps_finite(4, 4, 2, seed=7)
    if how == "rotate":
        B, Lx2, Ly2 = peps_rotate(A, 4, 4)
        where = lambda x, y: (4 - 1 - y, x)
    else:
        B, Lx2, Ly2 = peps_transpose(A, 4, 4)
        where = lambda x, y: (y, x)
    sz, ss, lz = _c1_observables(A, 4, 4)
    sz2, ss2, lz2 = _c1_observables(B, Lx2, Ly2)
    for (x, y), v in sz.items():
        assert abs(v - sz2[where(x, y)]) < TOL
    for key, v in ss.items():
        assert abs(v - ss2[frozenset(where(*p) for p in key)]) < TOL
    assert abs(lz - lz2) < TOL


def test_p5_infinite_rotation_invariance():
    """An infinite lattice of an anisotropic 2x2 cell, one cell per block and
    chi above the exact ranks: turning the cell a quarter turn permutes the
    cell's observables."""
    from bbp_inputs import peps_rotate
    cell = peps_infinite(2, 2, 2, seed=11)
    rot, _, _ = peps_rotate(cell, 2, 2)

    def run(c):
        bp = ob.BlockBP(c, D=2, chi=16, bx=2, by=2, infinite=True, ucx=2, ucy=2)
        bp.sweep(12)
        return bp
    a, b = run(cell), run(rot)
    for y in range(2):
        for x in range(2):
            xr, yr = 1 - y, x
            assert abs(a.expect_site(x, y, op_sz()) - b.expect_site(xr, yr, op_sz())) < TOL
            assert abs(a.expect_site(x, y, op_sx()) - b.expect_site(xr, yr, op_sx())) < TOL
            # horizontal bond (x,y)-(x+1,y) becomes the vertical bond between
            # (1-y, x) and (1-y, x+1)
            assert abs(a.expect_bond(x, y, x + 1, y, op_szsz())
                       - b.expect_bond(xr, yr, xr, yr + 1, op_szsz())) < TOL


# --- P7: convergence of the fixed-point iteration -------------------------------
@pytest.mark.parametrize("case", ["finite", "infinite"])
def test_p7_extra_sweeps_converge(case):
    """Truncated loopy cases: once the residual (a squared message distance)
    is below 1e-10, the observables move by at most a small multiple of its
    square root per sweep, and once it reaches the rounding floor one more
    sweep moves every observable by less than 1e-10."""
    if case == "finite":
        A = peps_finite(8, 8, 2, seed=3)
        bp = ob.BlockBP(A, D=2, chi=6, bx=4, by=4, Lx=8, Ly=8, chi_env=18)
        sites = [(1, 1), (4, 3), (6, 6), (3, 5)]
        bonds = [(3, 3, 4, 3), (5, 3, 5, 4), (1, 2, 2, 2)]
    else:
        A = peps_infinite(2, 2, 2, seed=11)
        bp = ob.BlockBP(A, D=2, chi=6, bx=4, by=4, infinite=True, ucx=2, ucy=2)
        sites = [(0, 0), (1, 0), (0, 1), (1, 1)]
        bonds = [(0, 0, 1, 0), (1, 1, 1, 2), (0, 1, 1, 1)]

    def obs():
        bp._cache = {}
        return np.array([bp.expect_site(x, y, op_sz()) for (x, y) in sites]
                        + [bp.expect_bond(*b, op_heis()) for b in bonds])
    r = bp.sweep()
    n = 1
    while r >= 1e-10:
        r = bp.sweep()
        n += 1
        assert n < 30
    o1 = obs()
    bp.sweep()
    o2 = obs()
    assert np.abs(o2 - o1).max() < 10 * math.sqrt(r)
    while r > 1e-15 and n < 40:
        r = bp.sweep()
        n += 1
    o1 = obs()
    bp.sweep()
    assert np.abs(obs() - o1).max() < 1e-10


# --- P8: the infinite lattice as the limit of finite tilings --------------------
def _p8_gap(D, b, chi, sizes, seed=11):
    """Largest difference, over the unit cell's <sigma_z>, <sigma_x> and
    horizontal <sigma_z sigma_z>, between the infinite-lattice oracle and the
    centre block of finite L x L tilings of the same anisotropic 2x2 cell."""
    from bbp_inputs import peps_tiled
    cell = peps_infinite(2, 2, D, seed=seed)
    inf = ob.BlockBP(cell, D=D, chi=chi, bx=b, by=b, infinite=True, ucx=2, ucy=2)
    for _ in range(40):
        if inf.sweep() < 1e-15:
            break
    ox = (b - 2) // 2
    gaps = []
    for L in sizes:
        fin = ob.BlockBP(peps_tiled(cell, 2, 2, L, L), D=D, chi=chi, bx=b, by=b,
                         Lx=L, Ly=L)
        for _ in range(40):
            if fin.sweep() < 1e-15:
                break
        g = L // b
        pos = lambda x: (g // 2) * b + ox + (x - ox) % 2  # cell coordinate x
        gap = 0.0
        for y in range(2):
            for x in range(2):
                for op in (op_sz(), op_sx()):
                    gap = max(gap, abs(inf.expect_site(x, y, op)
                                       - fin.expect_site(pos(x), pos(y), op)))
                gap = max(gap, abs(inf.expect_bond(x, y, x + 1, y, op_szsz())
                                   - fin.expect_bond(pos(x), pos(y), pos(x) + 1,
                                                     pos(y), op_szsz())))
        gaps.append(gap)
    return gaps


def test_p8_finite_tilings_approach_the_infinite_lattice():
    """Sec. II (iPEPS: one block exchanging messages with its own copies) and
    App. E: the centre block of growing finite tilings of an anisotropic 2x2
    cell (no reflection symmetry, so the four self-messages all differ)
    converges geometrically to the infinite-lattice values.  One cell per
    block; chi above the exact ranks."""
    gaps = _p8_gap(2, 2, 16, [6, 10, 14])
    assert gaps[0] > gaps[1] * 20 > gaps[2] * 400
    assert gaps[2] < 1e-7


def test_p8_block_of_four_cells():
    """The same limit for a 4x4 block holding four copies of the cell (the
    block shape of the infinite workload), chi = 16 truncated nowhere."""
    gaps = _p8_gap(2, 4, 16, [12])
    assert gaps[0] < 1e-6


def test_p8_catches_same_direction_routing(monkeypatch):
    """Planted mistake: on the infinite lattice a block receives its own
    message in the same direction instead of its neighbour's opposite one."""
    orig = ob.BlockBP.incoming

    def bad(self, bi, bj, side, msgs=None):
        if not self.infinite:
            return orig(self, bi, bj, side, msgs)
        msgs = self.msgs if msgs is None else msgs
        return msgs[(bi, bj, side)]
    monkeypatch.setattr(ob.BlockBP, "incoming", bad)
    assert _p8_gap(2, 2, 16, [14])[0] > 1e-4
    assert _p8_gap(2, 4, 16, [12])[0] > 1e-5


# ---- single-layer networks (Sec. V classical Ising, bond dimension 2) -------------

def test_single_layer_ising_is_exact_on_one_block():
    """One block covering a 3x3 open lattice: the single-layer network of the
    Ising Gibbs weights gives the classical magnetisation of every site and
    log Z, summed over all configurations."""
    from bbp_inputs import ising_single_layer
    beta, h = 0.7, 0.3
    A = ising_single_layer(beta, h, 3, 3)
    g = ob.BlockBP(A, D=2, chi=4, bx=3, by=3, Lx=3, Ly=3, chi_env=16, single_layer=True)
    m = _ising_brute(beta, h, 3, 3)
    for y in range(3):
        for x in range(3):
            assert abs(g.expect_site(x, y, op_sz()) - m[y * 3 + x]) < 1e-12
    import itertools
    Z = 0.0
    for conf in itertools.product((1, -1), repeat=9):
        s = np.array(conf).reshape(3, 3)
        Z += np.exp(beta * ((s[:, :-1] * s[:, 1:]).sum() + (s[:-1, :] * s[1:, :]).sum())
                    + h * s.sum())
    assert abs(g.log_norm()[0] - math.log(Z)) < 1e-12


def test_single_layer_ising_approaches_onsager():
    """Infinite single-layer Ising network below T_c: block BP's magnetisation
    at the block centre approaches Onsager and Yang's closed form and
    improves with the block size (Sec. V)."""
    from bbp_inputs import ising_single_layer
    onsager = lambda beta: (1 - np.sinh(2 * beta) ** -4) ** 0.125

    def m(beta, b, chi):
        g = ob.BlockBP(ising_single_layer(beta, 1e-6), D=2, chi=chi, bx=b, by=b,
                       infinite=True, ucx=1, ucy=1, single_layer=True)
        for _ in range(200):
            if g.sweep() < 1e-13:
                break
        return g.expect_site(0, 0, op_sz())
    assert abs(m(0.8, 4, 4) - onsager(0.8)) < 1e-6
    e2 = abs(m(0.6, 2, 2) - onsager(0.6))
    e4 = abs(m(0.6, 4, 4) - onsager(0.6))
    assert e4 < 1e-4 and e4 < 0.2 * e2


@pytest.mark.parametrize("mutation", ["double_layer", "bra_index_1"])
def test_single_layer_bra_planted_mistakes(mutation):
    """The bra layer taken as the tensor itself (the double layer of the split
    tensors) or fixed at the wrong index breaks the exactness pin."""
    from bbp_inputs import ising_single_layer
    beta, h = 0.7, 0.3
    A = ising_single_layer(beta, h, 3, 3)
    g = ob.BlockBP(A, D=2, chi=4, bx=3, by=3, Lx=3, Ly=3, chi_env=16, single_layer=True)
    if mutation == "double_layer":
        g.bra = None
    else:
        def bra(t):
            B = np.zeros_like(t)
            B[:, 0, 0, 0, 0] = 1.0
            B[1, 0, 0, 0, 0] = 0.0
            B[1, 1, 1, 1, 1] = 1.0
            return B
        g.bra = bra
    m = _ising_brute(beta, h, 3, 3)
    err = max(abs(g.expect_site(x, y, op_sz()) - m[y * 3 + x])
              for y in range(3) for x in range(3))
    assert err > 1e-6
