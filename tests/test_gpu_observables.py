"""GPU observables against the FP64 oracle (and brute force where exact).

Every <sigma_z>, bond <S.S> (and the infinite-lattice sigma_x, sigma_z
sigma_z) and the log-norm of the HIP library must match the oracle within
1e-10 absolute after the same number of sweeps.
"""

import math

import numpy as np
import pytest

from bbp_inputs import (op_heis, op_sx, op_sz, op_szsz, peps_finite,
                        peps_infinite)
from oracle import blockbp as ob
from oracle import brute

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _lib():
    from paper_2301_05844_amd import bbp
    return bbp


def _all_bonds(Lx, Ly):
    b = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    b += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    return b


def _run_pair(A, sweeps, **kw):
    bbp = _lib()
    ref = ob.BlockBP(A, **kw)
    g = bbp.BlockBP(**kw)
    g.set_tensors(A)
    for _ in range(sweeps):
        ref.sweep()
        g.sweep()
    return ref, g


FINITE = [
    ("loop_4x4_b2_chi4", dict(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4), 30),
    ("tree_2x6_b2", dict(Lx=2, Ly=6, bx=2, by=2, D=2, chi=4), 4),
    ("trunc_8x8_b4_chi8", dict(Lx=8, Ly=8, bx=4, by=4, D=2, chi=8), 5),
    ("ragged_7x5_b3x2", dict(Lx=7, Ly=5, bx=3, by=2, D=2, chi=6), 4),
    ("D3_6x6_b3_chi9", dict(Lx=6, Ly=6, bx=3, by=3, D=3, chi=9), 4),
]


@pytest.mark.parametrize("name,kw,sweeps", FINITE, ids=[f[0] for f in FINITE])
def test_finite_observables_match_oracle(name, kw, sweeps):
    A = peps_finite(kw["Lx"], kw["Ly"], kw["D"], seed=7)
    ref, g = _run_pair(A, sweeps, **kw)
    Lx, Ly = kw["Lx"], kw["Ly"]
    xs = [x for y in range(Ly) for x in range(Lx)]
    ys = [y for y in range(Ly) for x in range(Lx)]
    sz = g.expect_sites(xs, ys, op_sz())
    err = max(abs(sz[i] - ref.expect_site(xs[i], ys[i], op_sz()))
              for i in range(len(xs)))
    bonds = _all_bonds(Lx, Ly)
    ss = g.expect_bonds(bonds, op_heis())
    berr = max(abs(ss[i] - ref.expect_bond(*b, op_heis()))
               for i, b in enumerate(bonds))
    lz, sign = g.log_norm()
    lz_ref, sign_ref = ref.log_norm()
    print(f"{name}: sz {err:.2e} SS {berr:.2e} lognorm {abs(lz - lz_ref):.2e}",
          flush=True)
    assert err < TOL and berr < TOL
    assert abs(lz - lz_ref) < TOL * max(1.0, abs(lz_ref)) and sign == sign_ref


def test_single_block_equals_brute_force():
    A = peps_finite(4, 4, 2, seed=0)
    bbp = _lib()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=4, by=4, D=2, chi=4, chi_env=64)
    g.set_tensors(A)
    psi = brute.state_vector(A, 4, 4)
    xs = list(range(4)) * 4
    ys = [y for y in range(4) for _ in range(4)]
    sz = g.expect_sites(xs, ys, op_sz())
    for i in range(16):
        assert abs(sz[i] - brute.expect_site(psi, ys[i] * 4 + xs[i],
                                             op_sz())) < 1e-12
    bonds = _all_bonds(4, 4)
    ss = g.expect_bonds(bonds, op_heis())
    for i, (x0, y0, x1, y1) in enumerate(bonds):
        ref = brute.expect_bond(psi, y0 * 4 + x0, y1 * 4 + x1, op_heis())
        assert abs(ss[i] - ref) < 1e-12
    assert abs(g.log_norm()[0] - math.log(brute.norm2(psi))) < 1e-12


def test_infinite_observables_match_oracle():
    A = peps_infinite(2, 2, 2, seed=5)
    kw = dict(D=2, chi=8, bx=4, by=4, infinite=True, ucx=2, ucy=2)
    ref, g = _run_pair(A, 5, **kw)
    for (x, y) in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        for op in (op_sz(), op_sx()):
            assert abs(g.expect_site(x, y, op) - ref.expect_site(x, y, op)) < TOL
        for (x1, y1) in [(x + 1, y), (x, y + 1)]:
            assert abs(g.expect_bond(x, y, x1, y1, op_szsz())
                       - ref.expect_bond(x, y, x1, y1, op_szsz())) < TOL
    lz, _ = g.log_norm()
    assert abs(lz - ref.log_norm()[0]) < TOL * max(1.0, abs(lz))


def test_expect_rejects_bad_bond():
    A = peps_finite(4, 4, 2, seed=0)
    bbp = _lib()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    g.set_tensors(A)
    with pytest.raises(bbp.BBPError):
        g.expect_bond(0, 0, 1, 1, op_heis())
    with pytest.raises(bbp.BBPError):
        g.expect_site(4, 0, op_sz())
