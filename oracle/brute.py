"""Brute-force references that pin the block-BP oracle (test infrastructure).

* ``state_vector``: the full single-layer PEPS contracted into a state vector
  (2^n amplitudes, n <= 16), from which norms and expectation values follow
  by textbook linear algebra.
* ``strip_value``: exact contraction of the double-layer network of a finite
  open lattice by a column transfer vector over the fused bonds of one
  column (no truncation), with one-site operators inserted; used for strips
  too large for a state vector (e.g. 4 x 8 at D=2).

Neither uses messages, fits or anything from ``blockbp``.
"""

import numpy as np


def state_vector(A, Lx, Ly):
    """Amplitudes ``psi[s_0, ..., s_{n-1}]`` (site 0 most significant, sites
    row-major) of the open-boundary PEPS with site tensors ``A[s,u,l,d,r]``.
    Legs pointing off the lattice are taken at index 0."""
    d = A.shape[1]
    psi = None
    for y in range(Ly):
        t = A[y * Lx][:, :, 0, :, :]  # [s, u, d, r]
        for x in range(1, Lx):
            a = A[y * Lx + x]  # [s, u, l, d, r]
            t = np.einsum("SUDr,surde->SsUuDde", t, a)
            S, s, U, u, Dd, dd, e = t.shape
            t = t.reshape(S * s, U * u, Dd * dd, e)
        t = t[..., 0]  # [S, U, Dn]
        if psi is None:
            psi = t[:, 0, :]  # top edge: every up leg at index 0
        else:
            psi = np.einsum("pu,sud->psd", psi, t)
            psi = psi.reshape(-1, t.shape[2])
    return psi[:, 0].reshape((d,) * (Lx * Ly))


def expect_site(psi, i, op):
    """``<psi|op_i|psi> / <psi|psi>`` for a real state."""
    v = np.moveaxis(np.tensordot(op, psi, axes=([1], [i])), 0, i)
    return float(np.vdot(psi, v) / np.vdot(psi, psi))


def expect_bond(psi, i, j, op2):
    """Two-site ``op2[(s_i', s_j'), (s_i, s_j)]`` on sites i and j."""
    d = psi.shape[0]
    o = op2.reshape(d, d, d, d)
    v = np.tensordot(o, psi, axes=([2, 3], [i, j]))
    v = np.moveaxis(v, [0, 1], [i, j])
    return float(np.vdot(psi, v) / np.vdot(psi, psi))


def norm2(psi):
    return float(np.vdot(psi, psi))


def _double(A, Aket):
    D = A.shape[1]
    E = np.einsum("suldr,sULDR->uUlLdDrR", Aket, A)
    return E.reshape(D * D, D * D, D * D, D * D)


def strip_value(A, Lx, Ly, ops=None):
    """Exact value of the double-layer network of an open Lx x Ly lattice,
    ``sum <psi| prod_i op_i |psi>``, by a transfer vector over the fused left
    legs of one column.  ``ops`` maps a site index to a one-site operator
    ``op[s', s]`` (applied on the ket)."""
    ops = ops or {}
    D = A.shape[2]
    q = D * D
    e0 = np.zeros(q)
    e0[0] = 1.0
    v = e0
    for _ in range(Ly - 1):
        v = np.multiply.outer(v, e0)
    v = v.reshape((q,) * Ly)
    for x in range(Lx):
        w = np.multiply.outer(v, e0)  # last axis: bond from the site above
        for y in range(Ly):
            i = y * Lx + x
            a = A[i]
            ak = np.einsum("ts,suldr->tuldr", ops[i], a) if i in ops else a
            E = _double(a, ak)  # [u, l, d, r]
            w = np.tensordot(w, E, axes=([y, Ly], [1, 0]))  # ..., d, r
            w = np.moveaxis(w, -1, y)  # new right leg into row slot y
        v = w[..., 0]  # bottom edge
    return float(v[(0,) * Ly])


def strip_expect_site(A, Lx, Ly, i, op):
    return strip_value(A, Lx, Ly, {i: op}) / strip_value(A, Lx, Ly)


def strip_expect_bond(A, Lx, Ly, i, j, op2):
    """Two-site operator expanded in matrix units on site i."""
    d = A.shape[1]
    o = op2.reshape(d, d, d, d)
    num = 0.0
    for sp in range(d):
        for s in range(d):
            unit = np.zeros((d, d))
            unit[sp, s] = 1.0
            num += strip_value(A, Lx, Ly, {i: unit, j: o[sp, :, s, :]})
    return num / strip_value(A, Lx, Ly)
