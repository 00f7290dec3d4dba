"""Pins of the truncated-SVD oracle (the compression step of App. A's
standard MPO x MPS alternative) against what the mathematics fixes.

Every test here runs on the CPU and never touches the GPU library.

S1  2 x 2 closed form: S^2 = (T +- sqrt(T^2 - 4 det^2)) / 2, T = |A|_F^2.
S2  signed permutation of a diagonal: S = sorted |d|, U columns the unit
    vectors (positive by the sign convention), V the signed ones.
S3  rank one u v^T: S = (|u| |v|, 0, ...), U[:, 0] = u / |u| signed, the
    other U columns zero.
S4  S^2 are the eigenvalues of A^T A (a symmetric eigensolver, not an SVD).
S5  Eckart-Young: the discarded weight is |A - U_k S_k V_k^T|_F^2, and at
    k = n the factors reconstruct A with orthonormal U and V.
S6  invariances: S(c A) = |c| S(A); S(Q A) = S(A) for orthogonal Q.
S7  the sign convention: the largest-magnitude entry of each U column is
    positive.
Planted mistakes in the oracle (a shifted discard sum, no sign fix, a
transposed V) must each fail a pin.
"""

import numpy as np
import pytest

from bbp_inputs import dense_matrices
from oracle import svd as osvd

EPS = np.finfo(np.float64).eps


def _tol(A):
    """Backward-stable SVD: errors of order m eps |A|; a factor 32 of room."""
    m = A.shape[0]
    return 32 * m * EPS * max(np.linalg.norm(A, 2), 1e-300)


def pin_closed_form_2x2(f):
    rng = np.random.default_rng(3)
    for _ in range(20):
        A = rng.standard_normal((2, 2))
        T = np.sum(A * A)
        det = np.linalg.det(A)
        r = np.sqrt(max(T * T - 4 * det * det, 0.0))
        want = np.sqrt(np.array([(T + r) / 2, max((T - r) / 2, 0.0)]))
        _, S, _, _ = f(A)
        assert np.allclose(S, want, atol=1e-13 * want[0]), (S, want)


def pin_signed_permutation(f):
    rng = np.random.default_rng(4)
    m, n = 7, 5
    d = np.array([3.0, -0.5, 2.0, -7.0, 1.0])
    rows = rng.permutation(m)[:n]
    cols = rng.permutation(n)
    sgn = rng.choice([-1.0, 1.0], size=n)
    A = np.zeros((m, n))
    for t in range(n):
        A[rows[t], cols[t]] = sgn[t] * d[t]
    U, S, V, e2 = f(A)
    order = np.argsort(-np.abs(d), kind="stable")
    assert np.allclose(S, np.abs(d)[order], atol=0, rtol=1e-15)
    for j, t in enumerate(order):
        u = np.zeros(m)
        u[rows[t]] = 1.0
        v = np.zeros(n)
        v[cols[t]] = np.sign(sgn[t] * d[t])
        assert np.allclose(U[:, j], u, atol=1e-15)
        assert np.allclose(V[:, j], v, atol=1e-15)
    assert e2 == 0.0


def pin_rank_one(f):
    rng = np.random.default_rng(5)
    u = rng.standard_normal(9)
    v = rng.standard_normal(4)
    A = np.outer(u, v)
    U, S, V, _ = f(A)
    nu, nv = np.linalg.norm(u), np.linalg.norm(v)
    assert abs(S[0] - nu * nv) <= 1e-14 * nu * nv
    assert np.all(S[1:] <= 1e-14 * nu * nv)
    want = u / nu * (1.0 if u[np.argmax(np.abs(u))] > 0 else -1.0)
    assert np.allclose(U[:, 0], want, atol=1e-14)
    assert np.allclose(np.outer(U[:, 0], V[:, 0]) * S[0], A, atol=1e-13 * nu * nv)


def pin_eigenvalues(f):
    for seed, (m, n) in enumerate([(12, 5), (40, 16), (6, 6)]):
        A = dense_matrices(1, m, n, seed=seed)[0]
        _, S, _, _ = f(A)
        ev = np.sort(np.linalg.eigvalsh(A.T @ A))[::-1]
        assert np.allclose(S ** 2, np.maximum(ev, 0), atol=_tol(A) * S[0])


def pin_eckart_young(f):
    for seed, (m, n, k) in enumerate([(30, 10, 4), (16, 16, 15), (9, 3, 1)]):
        A = dense_matrices(1, m, n, seed=10 + seed)[0]
        U, S, V, e2 = f(A, k)
        R = A - (U * S) @ V.T
        assert abs(np.sum(R * R) - e2) <= 8 * _tol(A) * S[0]
        Uf, Sf, Vf, e0 = f(A)
        assert e0 == 0.0
        assert np.abs((Uf * Sf) @ Vf.T - A).max() <= _tol(A)
        assert np.abs(Uf.T @ Uf - np.eye(n)).max() <= _tol(A) / S[0] + 1e-14
        assert np.abs(Vf.T @ Vf - np.eye(n)).max() <= _tol(A) / S[0] + 1e-14


def pin_invariances(f):
    A = dense_matrices(1, 20, 8, seed=21)[0]
    _, S, _, _ = f(A)
    _, S2, _, _ = f(-2.5 * A)
    assert np.allclose(S2, 2.5 * S, atol=2.5 * _tol(A))
    Q, _ = np.linalg.qr(np.random.default_rng(22).standard_normal((20, 20)))
    _, S3, _, _ = f(Q @ A)
    assert np.allclose(S3, S, atol=4 * _tol(A))


def pin_sign_convention(f):
    A = dense_matrices(1, 25, 9, seed=30)[0]
    U, _, _, _ = f(A)
    for j in range(U.shape[1]):
        assert U[np.argmax(np.abs(U[:, j])), j] > 0


PINS = [pin_closed_form_2x2, pin_signed_permutation, pin_rank_one, pin_eigenvalues,
        pin_eckart_young, pin_invariances, pin_sign_convention]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(osvd.truncated_svd)


def _mut_discard(A, k=None):
    U, S, V, _ = osvd.truncated_svd(A, k)
    Sf = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    kk = A.shape[1] if k is None else k
    return U, S, V, float(np.sum(Sf[kk + 1:] ** 2))


def _mut_no_sign(A, k=None):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    kk = n if k is None else k
    Uf, S, Vt = np.linalg.svd(A, full_matrices=False)
    return Uf[:, :kk], S[:kk], Vt.T[:, :kk], float(np.sum(S[kk:] ** 2))


def _mut_transposed_v(A, k=None):
    U, S, V, e2 = osvd.truncated_svd(A, k)
    n = V.shape[0]
    if V.shape[1] == n:
        V = V.T.copy()
    return U, S, V, e2


@pytest.mark.parametrize("mutant", [_mut_discard, _mut_no_sign, _mut_transposed_v],
                         ids=lambda f: f.__name__)
def test_planted_mistakes_fail_a_pin(mutant):
    failed = []
    for pin in PINS:
        try:
            pin(mutant)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"{mutant.__name__} passed every pin"
