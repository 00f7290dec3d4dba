"""FP64 oracle for the truncated SVD of the compression step (test
infrastructure).

App. A names the standard way to absorb a line of block tensors into a
boundary MPS: multiply the MPO into the MPS, then compress the product bond
by bond, keeping the largest singular values.  The primitive of that
compression is the truncated singular value decomposition of a tall matrix,
``A = U diag(S) V^T`` cut to the k largest singular triplets, which this
module writes out by its definition with LAPACK's SVD (``numpy.linalg.svd``)
as the one library step:

* ``S`` descending, ``U`` (m x k) and ``V`` (n x k) with orthonormal columns;
* each U column and its V column signed so that the largest-magnitude entry
  of the U column (the first of equal ones) is positive, the U column of a
  zero singular value set to zero;
* the discarded weight ``sum_{i >= k} S_i^2`` (the squared Frobenius error of
  the rank-k approximation, Eckart-Young).

Only the tests use it; it shares no code with the GPU library.
"""

import numpy as np


def sign_fix(U, V):
    """U, V with each column pair signed so that the largest-magnitude entry
    of the U column (the first of equal magnitude) is positive."""
    U = U.copy()
    V = V.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))  # first index of the maximum
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
            V[:, j] = -V[:, j]
    return U, V


def truncated_svd(A, k=None):
    """(U, S, V, err2) of the m x n matrix A (m >= n) cut to its k largest
    singular triplets (k defaults to n)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("a tall matrix: m >= n")
    k = n if k is None else int(k)
    Uf, S, Vt = np.linalg.svd(A, full_matrices=False)
    U, V = sign_fix(Uf, Vt.T)
    U[:, S == 0.0] = 0.0
    err2 = float(np.sum(S[k:] ** 2))
    return U[:, :k], S[:k].copy(), V[:, :k], err2
