"""bbp_svd_jacobi (batched one-sided Jacobi truncated SVD, the compression
step of App. A's standard MPO x MPS alternative) against the oracle's
definition (LAPACK SVD, the same sign convention and discarded weight).

Tolerances: both sides are backward stable, so a singular value differs by
at most a few m eps |A|_2 (32 m eps sigma_max here), the discarded weight by
that times sigma_max, and a singular vector by that over the gap to its
nearest other singular value (Wedin).  Equal or zero singular values have no
unique vectors: there the test checks what is unique (the values, the
reconstruction, orthonormality)."""

import numpy as np
import pytest

from bbp_inputs import dense_matrices

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _bbp():
    import torch
    from paper_2301_05844_amd import bbp
    if not torch.cuda.is_available():
        pytest.fail("no GPU")
    return bbp, torch


def _run(A, k=None):
    bbp, torch = _bbp()
    t = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, e2, sw = bbp.svd_jacobi(t, k)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (U, S, V, e2, sw)]


def _oracle(A, k):
    from oracle.svd import truncated_svd
    return truncated_svd(A, k)


CASES = [
    # name, batch, m, n, k, kind, extra
    ("message panel 512x32", 4, 512, 32, None, "gauss", {}),
    ("96x24 cut to 12", 3, 96, 24, 12, "gauss", {}),
    ("odd n 40x7 cut to 3", 5, 40, 7, 3, "gauss", {}),
    ("square 64x64", 2, 64, 64, None, "gauss", {}),
    ("largest at n=64: 248x64", 1, 248, 64, 32, "gauss", {}),
    ("largest at n=32: 592x32", 1, 592, 32, None, "gauss", {}),
    ("one column 33x1", 3, 33, 1, None, "gauss", {}),
    ("1x1", 2, 1, 1, None, "gauss", {}),
    ("graded 200x20 (cond 1e10) cut to 8", 3, 200, 20, 8, "graded", {"cond": 1e10}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_matches_the_oracle(case):
    name, batch, m, n, k, kind, extra = case
    A = dense_matrices(batch, m, n, seed=len(name), kind=kind, **extra)
    print(f"svd parity: {name}", flush=True)
    U, S, V, e2, sw = _run(A, k)
    kk = n if k is None else k
    assert U.shape == (batch, m, kk) and S.shape == (batch, kk) and V.shape == (batch, n, kk)
    for b in range(batch):
        Uo, So, Vo, eo = _oracle(A[b], kk)
        smax = So[0]
        tol = 32 * m * EPS * smax
        assert sw[b] > 0, f"item {b}: no clean sweep within the limit ({sw[b]})"
        assert np.abs(S[b] - So).max() <= tol, (b, np.abs(S[b] - So).max(), tol)
        assert abs(e2[b] - eo) <= 2 * tol * smax
        Sall = np.linalg.svd(A[b], compute_uv=False)
        for j in range(kk):
            others = np.delete(Sall, j)
            gap = np.min(np.abs(others - Sall[j])) if others.size else smax
            vt = tol / gap
            if vt > 1e-4:  # too close to a neighbour for a unique vector
                continue
            assert np.abs(U[b][:, j] - Uo[:, j]).max() <= vt, (b, j)
            assert np.abs(V[b][:, j] - Vo[:, j]).max() <= vt, (b, j)


def test_full_rank_factors_reconstruct():
    A = dense_matrices(3, 300, 40, seed=7)
    U, S, V, e2, sw = _run(A)
    for b in range(3):
        tol = 32 * 300 * EPS * S[b][0]
        assert np.abs((U[b] * S[b]) @ V[b].T - A[b]).max() <= tol
        assert np.abs(U[b].T @ U[b] - np.eye(40)).max() <= 32 * 300 * EPS
        assert np.abs(V[b].T @ V[b] - np.eye(40)).max() <= 32 * 300 * EPS
        assert e2[b] == 0.0
        assert np.all(np.diff(S[b]) <= 0)
        for j in range(40):  # the sign convention
            assert U[b][np.argmax(np.abs(U[b][:, j])), j] > 0


def test_low_rank_zero_and_equal_singular_values():
    # rank 5 of 512 x 32: five values match, the rest are at the rounding floor
    A = dense_matrices(2, 512, 32, seed=3, kind="lowrank", rank=5)
    U, S, V, e2, sw = _run(A, 5)
    for b in range(2):
        Uo, So, Vo, eo = _oracle(A[b], 5)
        tol = 32 * 512 * EPS * So[0]
        assert sw[b] > 0
        assert np.abs(S[b] - So).max() <= tol
        assert e2[b] <= (32 * tol) ** 2 + 32 * tol * So[0]  # only rounding discarded
        assert np.abs((U[b] * S[b]) @ V[b].T - A[b]).max() <= 4 * tol
    # all zeros: zero values, zero U, V the identity columns (ties keep order)
    Z = np.zeros((2, 10, 4))
    U, S, V, e2, sw = _run(Z, 3)
    assert np.all(S == 0) and np.all(U == 0) and np.all(e2 == 0) and np.all(sw == 1)
    assert np.array_equal(V[0], np.eye(4)[:, :3])
    # orthonormal columns: every singular value 1, factors reconstruct
    Q = dense_matrices(1, 48, 16, seed=9, kind="equal")
    U, S, V, e2, sw = _run(Q)
    assert np.abs(S[0] - 1).max() <= 32 * 48 * EPS
    assert np.abs((U[0] * S[0]) @ V[0].T - Q[0]).max() <= 32 * 48 * EPS


def test_items_are_independent_of_the_batch_bitwise():
    A = dense_matrices(6, 128, 24, seed=11)
    Ub, Sb, Vb, eb, swb = _run(A, 10)
    for b in (0, 3, 5):
        U1, S1, V1, e1, sw1 = _run(A[b:b + 1], 10)
        assert np.array_equal(U1[0], Ub[b]) and np.array_equal(S1[0], Sb[b])
        assert np.array_equal(V1[0], Vb[b]) and e1[0] == eb[b] and sw1[0] == swb[b]
    Ur, Sr, Vr, er, swr = _run(A, 10)  # and the same bits when repeated
    assert np.array_equal(Ur, Ub) and np.array_equal(Sr, Sb) and np.array_equal(Vr, Vb)


def test_sweep_limit_is_reported():
    A = dense_matrices(2, 64, 16, seed=13)
    bbp, torch = _bbp()
    t = torch.from_numpy(A).cuda()
    _, _, _, _, sw = bbp.svd_jacobi(t, max_sweeps=1)
    assert np.all(sw.cpu().numpy() == -1)


def test_non_finite_input_stays_in_its_item():
    """A matrix holding NaN or Inf gives non-finite or zero output without an
    error, and the other items of its batch keep their bits."""
    A = dense_matrices(4, 40, 8, seed=17)
    ref = _run(A[1:2], 4)
    bad = A.copy()
    bad[0, 3, 2] = np.nan
    bad[2, 0, 0] = np.inf
    U, S, V, e2, sw = _run(bad, 4)
    assert np.array_equal(U[1], ref[0][0]) and np.array_equal(S[1], ref[1][0])
    assert np.array_equal(V[1], ref[2][0])
    # the NaN column's value sorts last, so it shows in the discarded weight;
    # the infinite column's value comes first
    assert np.isnan(e2[0]) and S[2][0] == np.inf
