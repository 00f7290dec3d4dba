"""Seeded tensor generators and operator matrices (no block-BP arithmetic here)."""

import numpy as np


def _draw_site(rng, d, dims, D):
    """One site: ``0.1 * N(0,1)`` over the true leg dimensions, plus 1 at the
    all-zero entry, zero-padded to ``D`` on every virtual leg."""
    du, dl, dd, dr = dims
    t = 0.1 * rng.standard_normal((d, du, dl, dd, dr))
    t[0, 0, 0, 0, 0] += 1.0
    out = np.zeros((d, D, D, D, D))
    out[:, :du, :dl, :dd, :dr] = t
    return out


def peps_finite(Lx, Ly, D, d=2, seed=0):
    """Finite open-boundary PEPS on an ``Lx`` x ``Ly`` square lattice.

    Returns an array of shape ``(Ly*Lx, d, D, D, D, D)``; sites in row-major
    order; legs pointing off the lattice have true dimension 1 (zero-padded).
    """
    rng = np.random.default_rng(seed)
    A = np.zeros((Ly * Lx, d, D, D, D, D))
    for y in range(Ly):
        for x in range(Lx):
            dims = (1 if y == 0 else D,
                    1 if x == 0 else D,
                    1 if y == Ly - 1 else D,
                    1 if x == Lx - 1 else D)
            A[y * Lx + x] = _draw_site(rng, d, dims, D)
    return A


def peps_infinite(ucx, ucy, D, d=2, seed=0):
    """Unit cell of a translation-invariant PEPS: ``ucx*ucy`` tensors, all legs D."""
    rng = np.random.default_rng(seed)
    A = np.zeros((ucy * ucx, d, D, D, D, D))
    for i in range(ucx * ucy):
        A[i] = _draw_site(rng, d, (D, D, D, D), D)
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
    # 16x16 open lattice, D=6, 4x4 blocks, chi=64 (mixed-precision workload)
    "obc16x16_D6_b4_chi64": dict(infinite=False, Lx=16, Ly=16, bx=4, by=4, D=6,
                                 chi=64, tol=1e-10),
}
