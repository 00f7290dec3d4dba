"""Pins of the oracle's blockBP update (App. B, Eq. (Ut)): a product gate
is represented exactly (the fitted state equals the gated state), the fit of
a pair in a trivial environment is the best rank-D approximation
(Eckart-Young), and imaginary time evolution of a 3x3 transverse-field Ising
PEPS lowers the energy towards the exact ground state.  CPU only."""

import numpy as np
import pytest
from scipy.linalg import expm

from bbp_inputs import op_sx, op_sz, peps_finite
from oracle import brute
from oracle import ite


def _apply_site_ops(psi, ops):
    for i, op in ops.items():
        psi = np.moveaxis(np.tensordot(op, psi, axes=([1], [i])), 0, i)
    return psi


def test_product_gate_is_exact():
    """G = g (x) g on every bond: each site's tensor can absorb its g's, so
    the fitted PEPS equals the gated state (one block, exact environment)."""
    A = peps_finite(3, 3, 2, seed=1, noise=0.3)
    g = expm(-0.1 * op_sx())
    psi = brute.state_vector(A, 3, 3)
    A2, _ = ite.ite_step(A, 3, 3, 2, 4, 3, 3, np.kron(g, g), n_als=3, chi_env=64, sweeps=1)
    count = {}
    for a, b in ite.bond_order(3, 3):
        for s in (a, b):
            count[s] = count.get(s, 0) + 1
    ref = _apply_site_ops(psi, {y * 3 + x: np.linalg.matrix_power(g, n)
                                for (x, y), n in count.items()})
    psi2 = brute.state_vector(A2, 3, 3)
    ov = abs(np.vdot(psi2, ref)) / (np.linalg.norm(psi2) * np.linalg.norm(ref))
    assert 1.0 - ov < 1e-12


def test_fit_in_a_trivial_environment_is_the_truncated_svd():
    rng = np.random.default_rng(3)
    k, d, kb, D = 4, 2, 4, 2
    Theta = rng.standard_normal((k, d, d, kb))
    G = np.eye(d * d)
    R, L = ite.fit_pair(np.eye(k * kb), Theta, G, D, n_als=6)
    fit = np.einsum("asr,rub->asub", R, L).reshape(k * d, d * kb)
    S = np.linalg.svd(Theta.reshape(k * d, d * kb), compute_uv=False)
    loss = np.sum((fit - Theta.reshape(k * d, d * kb)) ** 2)
    assert abs(loss - np.sum(S[D:] ** 2)) < 1e-10 * np.sum(S ** 2)


def _ti_hamiltonian(B):
    sx, sz = op_sx(), op_sz()
    return -np.kron(sz, sz) - B / 4 * (np.kron(sx, np.eye(2)) + np.kron(np.eye(2), sx))


def _energy(A, Lx, Ly, h):
    psi = brute.state_vector(A, Lx, Ly)
    return sum(brute.expect_bond(psi, a[1] * Lx + a[0], b[1] * Lx + b[0], h)
               for a, b in ite.bond_order(Lx, Ly))


def _exact_ground_energy(Lx, Ly, B):
    n = Lx * Ly
    H = np.zeros((2 ** n, 2 ** n))

    def at(ops):
        m = np.array([[1.0]])
        for i in range(n):
            m = np.kron(m, ops.get(i, np.eye(2)))
        return m
    for a, b in ite.bond_order(Lx, Ly):
        i, j = a[1] * Lx + a[0], b[1] * Lx + b[0]
        H -= at({i: op_sz(), j: op_sz()})
        H -= B / 4 * (at({i: op_sx()}) + at({j: op_sx()}))
    return np.linalg.eigvalsh(H)[0]


def test_imaginary_time_evolution_lowers_the_energy():
    """3x3 transverse-field Ising model (B = 3, bond terms -sz sz - B/4 (sx 1
    + 1 sx)), D = 2, one block over the lattice: every Trotter step (dtau =
    0.1) lowers the energy, which closes in on the exact ground energy."""
    h = _ti_hamiltonian(3.0)
    G = expm(-0.1 * h)
    A = peps_finite(3, 3, 2, seed=2)
    E0 = _exact_ground_energy(3, 3, 3.0)
    es = [_energy(A, 3, 3, h)]
    for _ in range(6):
        A, _ = ite.ite_step(A, 3, 3, 2, 4, 3, 3, G, n_als=3, chi_env=64, sweeps=1)
        es.append(_energy(A, 3, 3, h))
    print("energies", es, "exact", E0)
    assert all(b < a for a, b in zip(es, es[1:]))
    assert es[-1] - E0 < 0.25 * (es[0] - E0)
    assert es[-1] > E0 - 1e-9


def test_planted_gate_order_mistake():
    """A gate applied with its two sites swapped breaks product-gate
    exactness when g0 and g1 differ."""
    A = peps_finite(3, 2, 2, seed=4, noise=0.3)
    g0, g1 = expm(-0.2 * op_sx()), expm(-0.3 * op_sz())
    psi = brute.state_vector(A, 3, 2)
    bad = ite.ite_step(A, 3, 2, 2, 4, 3, 2, np.kron(g1, g0), n_als=3, chi_env=64, sweeps=1)[0]
    good = ite.ite_step(A, 3, 2, 2, 4, 3, 2, np.kron(g0, g1), n_als=3, chi_env=64, sweeps=1)[0]
    ops = {}
    for a, b in ite.bond_order(3, 2):
        ia, ib = a[1] * 3 + a[0], b[1] * 3 + b[0]
        ops[ia] = g0 @ ops.get(ia, np.eye(2))
        ops[ib] = g1 @ ops.get(ib, np.eye(2))
    ref = _apply_site_ops(psi, ops)
    for A2, want in ((good, True), (bad, False)):
        p2 = brute.state_vector(A2, 3, 2)
        ov = abs(np.vdot(p2, ref)) / (np.linalg.norm(p2) * np.linalg.norm(ref))
        assert (1.0 - ov < 1e-12) == want


def test_edge_padding_stays_zero_and_state_moves_with_blocks():
    """4x4 lattice in 2x2 blocks (block-BP messages as the environments):
    the new tensors keep zero entries on every open-edge leg index above 0
    (the isometries span the true leg extents only), and the step lowers
    the transverse-field Ising energy as the exact (one-block) update does."""
    h = _ti_hamiltonian(3.0)
    G = expm(-0.1 * h)
    A = peps_finite(4, 3, 2, seed=6)
    A2, _ = ite.ite_step(A, 4, 3, 2, 8, 2, 2, G, n_als=3, chi_env=16, sweeps=6, tol=0.0)
    for y in range(3):
        for x in range(4):
            t = A2[y * 4 + x]
            for leg, edge in ((1, y == 0), (2, x == 0), (3, y == 2), (4, x == 3)):
                if edge:
                    assert np.all(np.take(t, [1], axis=leg) == 0.0)
    assert _energy(A2, 4, 3, h) < _energy(A, 4, 3, h)


def _exact_trotter(psi, Lx, Ly, G, steps):
    """The state vector after `steps` Trotter steps: G applied to every bond
    in the update's order (first site of a bond the major index of G)."""
    n = Lx * Ly
    for _ in range(steps):
        for a, b in ite.bond_order(Lx, Ly):
            i, j = a[1] * Lx + a[0], b[1] * Lx + b[0]
            t = np.moveaxis(psi.reshape([2] * n), [i, j], [0, 1]).reshape(4, -1)
            t = (G @ t).reshape([2, 2] + [2] * (n - 2))
            psi = np.moveaxis(t, [0, 1], [i, j]).reshape(-1)
    return psi


@pytest.mark.parametrize("lat", [(3, 1, 2), (1, 3, 2)])
def test_chain_evolution_is_exact(lat):
    """Open chains of 3 sites at D = 2, horizontal and vertical (every
    cut's Schmidt rank fits the bond): the update reproduces exact Trotterised
    evolution of the state vector, for a generic real two-site gate (no
    symmetry under transposition or under exchange of its sites), one
    block, three steps; the gate transposed or with its sites exchanged
    does not."""
    Lx, Ly, D = lat
    rng = np.random.default_rng(8)
    G = np.eye(4) + 0.3 * rng.standard_normal((4, 4))
    A = peps_finite(Lx, Ly, D, seed=3)
    ref = _exact_trotter(brute.state_vector(A, Lx, Ly), Lx, Ly, G, 3)
    for _ in range(3):
        A, _ = ite.ite_step(A, Lx, Ly, D, 16, Lx, Ly, G, n_als=2, chi_env=16, sweeps=1)
    psi = brute.state_vector(A, Lx, Ly)
    ov = abs(np.vdot(psi, ref)) / (np.linalg.norm(psi) * np.linalg.norm(ref))
    assert 1.0 - ov < 1e-12
    # planted: the gate transposed, or its two sites exchanged
    swap = G.reshape(2, 2, 2, 2).transpose(1, 0, 3, 2).reshape(4, 4)
    for bad in (G.T, swap):
        B = peps_finite(Lx, Ly, D, seed=3)
        for _ in range(3):
            B, _ = ite.ite_step(B, Lx, Ly, D, 16, Lx, Ly, bad, n_als=2, chi_env=16, sweeps=1)
        pb = brute.state_vector(B, Lx, Ly)
        ovb = abs(np.vdot(pb, ref)) / (np.linalg.norm(pb) * np.linalg.norm(ref))
        assert 1.0 - ovb > 1e-6
