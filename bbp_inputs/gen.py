"""Seeded tensor generators and operator matrices (no block-BP arithmetic here)."""

import numpy as np


def _draw_site(rng, d, dims, D, noise=0.1):
    """One site: ``noise * N(0,1)`` over the true leg dimensions, plus 1 at
    the all-zero entry, zero-padded to ``D`` on every virtual leg."""
    du, dl, dd, dr = dims
    t = noise * rng.standard_normal((d, du, dl, dd, dr))
    t[0, 0, 0, 0, 0] += 1.0
    out = np.zeros((d, D, D, D, D))
    out[:, :du, :dl, :dd, :dr] = t
    return out


def peps_finite(Lx, Ly, D, d=2, seed=0, noise=0.1):
    """Finite open-boundary PEPS on an ``Lx`` x ``Ly`` square lattice.

    Returns an array of shape ``(Ly*Lx, d, D, D, D, D)``; sites in row-major
    order; legs pointing off the lattice have true dimension 1 (zero-padded).
    ``noise`` scales the Gaussian part (0.1 for every named workload; larger
    values give a more strongly correlated state).
    """
    rng = np.random.default_rng(seed)
    A = np.zeros((Ly * Lx, d, D, D, D, D))
    for y in range(Ly):
        for x in range(Lx):
            dims = (1 if y == 0 else D,
                    1 if x == 0 else D,
                    1 if y == Ly - 1 else D,
                    1 if x == Lx - 1 else D)
            A[y * Lx + x] = _draw_site(rng, d, dims, D, noise)
    return A


def peps_infinite(ucx, ucy, D, d=2, seed=0):
    """Unit cell of a translation-invariant PEPS: ``ucx*ucy`` tensors, all legs D."""
    rng = np.random.default_rng(seed)
    A = np.zeros((ucy * ucx, d, D, D, D, D))
    for i in range(ucx * ucy):
        A[i] = _draw_site(rng, d, (D, D, D, D), D)
    return A


def ising_peps(beta, h=0.0, Lx=0, Ly=0):
    """PEPS whose norm is the classical Ising partition function
    ``Z = sum_sigma exp(beta * sum_<ij> s_i s_j + h * sum_i s_i)``: the state
    ``psi(sigma) = prod_<ij> exp(beta s_i s_j / 2) prod_i exp(h s_i / 2)``
    squares to the Boltzmann weight, so ``<psi|psi> = Z`` and ``<sigma_z>`` of
    psi is the classical magnetisation.  Each bond factor is split as
    ``exp(beta s s' / 2) = sum_k Q[s, k] Q[s', k]`` (both eigenvalues of the
    2x2 factor are positive for beta > 0) and every site carries one ``Q`` per
    leg: D = 2.  ``Lx = Ly = 0``: one tensor, the 1x1 unit cell of the
    infinite lattice; otherwise the open ``Lx x Ly`` lattice, legs off the edge
    of true dimension 1 (zero-padded)."""
    w = np.array([[np.exp(beta / 2), np.exp(-beta / 2)],
                  [np.exp(-beta / 2), np.exp(beta / 2)]])
    lam, V = np.linalg.eigh(w)
    Q = V * np.sqrt(lam)                      # w = Q Q^T
    one = np.array([1.0, 0.0])
    infinite = Lx == 0
    nx, ny = (1, 1) if infinite else (Lx, Ly)
    A = np.zeros((nx * ny, 2, 2, 2, 2, 2))
    for y in range(ny):
        for x in range(nx):
            for s in range(2):
                sg = 1.0 if s == 0 else -1.0
                leg = lambda edge: one if (edge and not infinite) else Q[s]
                A[y * nx + x, s] = np.exp(h * sg / 2) * np.einsum(
                    "u,l,d,r->uldr", leg(y == 0), leg(x == 0), leg(y == ny - 1), leg(x == nx - 1))
    return A


def ising_single_layer(beta, h=0.0, Lx=0, Ly=0):
    """Single-layer tensor network of the classical Ising partition function
    ``Z = sum_sigma exp(beta * sum_<ij> s_i s_j + h * sum_i s_i)`` (bond
    dimension 2), split by the spin value: site tensor ``A[s, u, l, d, r] =
    exp(h s) W[s, u] W[s, l] W[s, d] W[s, r]`` with ``exp(beta s s') =
    sum_k W[s, k] W[s', k]``, so the network tensor is ``sum_s A[s]`` and
    ``sum_s s A[s]`` is the impurity of the magnetisation.  ``Lx = Ly = 0``:
    the 1x1 unit cell of the infinite lattice; otherwise the open ``Lx x Ly``
    lattice, legs off the edge of true dimension 1 (zero-padded)."""
    w = np.array([[np.exp(beta), np.exp(-beta)],
                  [np.exp(-beta), np.exp(beta)]])
    lam, V = np.linalg.eigh(w)
    W = V * np.sqrt(lam)                      # w = W W^T
    one = np.array([1.0, 0.0])
    infinite = Lx == 0
    nx, ny = (1, 1) if infinite else (Lx, Ly)
    A = np.zeros((nx * ny, 2, 2, 2, 2, 2))
    for y in range(ny):
        for x in range(nx):
            for s in range(2):
                sg = 1.0 if s == 0 else -1.0
                leg = lambda edge: one if (edge and not infinite) else W[s]
                A[y * nx + x, s] = np.exp(h * sg) * np.einsum(
                    "u,l,d,r->uldr", leg(y == 0), leg(x == 0), leg(y == ny - 1), leg(x == nx - 1))
    return A


def pauli():
    """Pauli matrices in the basis s=0 <-> sigma_z=+1; sigma_y returned as the
    real matrix i*sigma_y (so that sigma_y (x) sigma_y = -(i sy)(x)(i sy))."""
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    isy = np.array([[0.0, 1.0], [-1.0, 0.0]])
    sz = np.array([[1.0, 0.0], [0.0, -1.0]])
    return sx, isy, sz


def op_sz():
    return pauli()[2].copy()


def op_sx():
    return pauli()[0].copy()


def op_sy_real():
    """``i*sigma_y`` (real); the expectation of sigma_y of a real state is 0."""
    return pauli()[1].copy()


def op_szsz():
    sz = op_sz()
    return np.kron(sz, sz)


def op_heis():
    """S.S = (sx sx + sy sy + sz sz)/4 as a real 4x4 matrix, row-major
    ``op[(s0', s1'), (s0, s1)]`` with the first site as the major index."""
    sx, isy, sz = pauli()
    return (np.kron(sx, sx) - np.kron(isy, isy) + np.kron(sz, sz)) / 4.0


# Workloads named by what they are.  Each: lattice, block, D, chi, sweeps.
CONFIGS = {
    # 4x4 open lattice, D=2, 2x2 blocks, chi=4, 30 sweeps
    "obc4x4_D2_b2_chi4": dict(infinite=False, Lx=4, Ly=4, bx=2, by=2, D=2, chi=4,
                              sweeps=30),
    # 16x16 open lattice, D=4, 4x4 blocks, chi=32, until residual < 1e-10
    "obc16x16_D4_b4_chi32": dict(infinite=False, Lx=16, Ly=16, bx=4, by=4, D=4,
                                 chi=32, tol=1e-10),
    # infinite lattice, 2x2 unit cell, D=4, 4x4 block, chi=32
    "inf2x2_D4_b4_chi32": dict(infinite=True, ucx=2, ucy=2, bx=4, by=4, D=4,
                               chi=32, tol=1e-10),
    # 8x8 open lattice, D=4, 4x4 blocks, chi=56, chi_env=64, 2 sweeps (bond caps
    # 49..64 in the fits)
    "obc8x8_D4_b4_chi56": dict(infinite=False, Lx=8, Ly=8, bx=4, by=4, D=4, chi=56,
                               chi_env=64, sweeps=2),
    # 4x4 open lattice as one D=4 block, chi_env=80: the observables' fits at a
    # bond cap above 64
    "obc4x4_D4_b4_env80": dict(infinite=False, Lx=4, Ly=4, bx=4, by=4, D=4, chi=16,
                               chi_env=80, sweeps=1),
    # 6x6 open lattice, D=6, 3x3 blocks, chi=6, chi_env=16, 2 sweeps (D=6 parity)
    "obc6x6_D6_b3_chi6": dict(infinite=False, Lx=6, Ly=6, bx=3, by=3, D=6, chi=6,
                              chi_env=16, sweeps=2),
    # 8x8 open lattice, D=6, 4x4 blocks, chi=64, chi_env=82, 2 sweeps: the
    # D=6 workload's bond caps (message fits at 64, observables at 82)
    "obc8x8_D6_b4_chi64": dict(infinite=False, Lx=8, Ly=8, bx=4, by=4, D=6, chi=64,
                               chi_env=82, sweeps=2),
    # 16x16 open lattice, D=6, 4x4 blocks, chi=64 (mixed-precision workload)
    "obc16x16_D6_b4_chi64": dict(infinite=False, Lx=16, Ly=16, bx=4, by=4, D=6,
                                 chi=64, tol=1e-10),
}


def peps_tiled(cell, ucx, ucy, Lx, Ly):
    """Open ``Lx x Ly`` lattice tiled with the unit-cell tensors ``cell``
    (``ucy*ucx`` tensors, row-major): site (x, y) takes cell tensor
    ``(y % ucy, x % ucx)`` with every leg that points off the lattice
    restricted to index 0 (the other entries set to zero)."""
    cell = np.asarray(cell, dtype=np.float64)
    A = np.zeros((Ly * Lx,) + cell.shape[1:])
    for y in range(Ly):
        for x in range(Lx):
            t = cell[(y % ucy) * ucx + (x % ucx)].copy()
            if y == 0:
                t[:, 1:, :, :, :] = 0.0
            if x == 0:
                t[:, :, 1:, :, :] = 0.0
            if y == Ly - 1:
                t[:, :, :, 1:, :] = 0.0
            if x == Lx - 1:
                t[:, :, :, :, 1:] = 0.0
            A[y * Lx + x] = t
    return A


def peps_rotate(A, Lx, Ly):
    """The same network turned a quarter turn clockwise: an ``Ly x Lx``
    lattice whose site (Ly-1-y, x) holds old site (x, y) with legs
    (u, l, d, r) <- old (l, d, r, u).  Returns ``(B, Lx', Ly')``."""
    A = np.asarray(A)
    B = np.zeros_like(A)
    for y in range(Ly):
        for x in range(Lx):
            B[x * Ly + (Ly - 1 - y)] = A[y * Lx + x].transpose(0, 2, 3, 4, 1)
    return B, Ly, Lx


def peps_transpose(A, Lx, Ly):
    """Mirror image in the main diagonal: site (y, x) of an ``Ly x Lx``
    lattice holds old site (x, y) with legs (u, l, d, r) <- old (l, u, r, d)."""
    A = np.asarray(A)
    B = np.zeros_like(A)
    for y in range(Ly):
        for x in range(Lx):
            B[x * Ly + y] = A[y * Lx + x].transpose(0, 2, 1, 4, 3)
    return B, Ly, Lx


def dense_matrices(batch, m, n, seed=0, kind="gauss", rank=None, cond=1e3):
    """A seeded batch of real m x n matrices, shape (batch, m, n).

    ``gauss``: i.i.d. N(0, 1) entries.  ``graded``: Q1 diag(s) Q2^T with
    random orthogonal factors (QR of Gaussian matrices) and s falling
    geometrically from 1 to 1/cond, so the singular values are known and
    well separated.  ``lowrank``: a product of m x rank and rank x n Gaussian
    matrices.  ``equal``: the first n orthonormal columns of a random
    orthogonal matrix (every singular value 1).  ``zero``: all zeros."""
    rng = np.random.default_rng(seed)
    out = np.zeros((batch, m, n))
    for b in range(batch):
        if kind == "gauss":
            out[b] = rng.standard_normal((m, n))
        elif kind == "graded":
            q1, _ = np.linalg.qr(rng.standard_normal((m, n)))
            q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
            s = cond ** (-np.arange(n) / max(n - 1, 1))
            out[b] = (q1 * s) @ q2.T
        elif kind == "lowrank":
            r = rank if rank is not None else max(1, n // 3)
            out[b] = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
        elif kind == "equal":
            q, _ = np.linalg.qr(rng.standard_normal((m, n)))
            out[b] = q
        elif kind != "zero":
            raise ValueError(kind)
    return out
