"""Shifted partitions ("shift_x", "shift_y"), reduced density matrices
(bbp_rdm_sites / bbp_rdm_bonds) and the trace distance (bbp_trace_distance)
against the FP64 oracle: the same shifted partition, the same sweeps, every
site and bond within 1e-10 (Sec. II centre observables; App. C)."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Lx,Ly,b,D,chi,shift", [
    (8, 8, 4, 2, 4, (1, 2)),
    (8, 8, 4, 2, 4, (3, 0)),
    (7, 6, 3, 3, 9, (2, 1)),
])
def test_shifted_partition_matches_oracle(Lx, Ly, b, D, chi, shift):
    from oracle.blockbp import BlockBP as OracleBP
    from paper_2301_05844_amd import bbp
    A = peps_finite(Lx, Ly, D, seed=9, noise=0.3)
    ctx = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=b, by=b, D=D, chi=chi,
                      shift_x=shift[0], shift_y=shift[1])
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(3)]
    ref = OracleBP(A, D=D, chi=chi, bx=b, by=b, Lx=Lx, Ly=Ly, shift=shift)
    rref = [ref.sweep() for _ in range(3)]
    for a, r in zip(res, rref):
        assert abs(a - r) <= 1e-6 * r + 1e-14
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    sz = ctx.expect_sites(xs, ys, op_sz())
    rs = ctx.rdm_sites(xs, ys)
    err = 0.0
    for i, (x, y) in enumerate(zip(xs.tolist(), ys.tolist())):
        err = max(err, abs(sz[i] - ref.expect_site(x, y, op_sz())))
        err = max(err, np.abs(rs[i] - ref.rdm_site(x, y)).max())
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    sel = bonds[::3]
    ss = ctx.expect_bonds(sel, op_heis())
    rb = ctx.rdm_bonds(sel)
    for i, bd in enumerate(sel):
        err = max(err, abs(ss[i] - ref.expect_bond(*bd, op_heis())))
        err = max(err, np.abs(rb[i] - ref.rdm_bond(*bd)).max())
    lz, _ = ctx.log_norm()
    print(f"shift {shift}: max |d| {err:.2e}, log-norm {lz:.12f} vs {ref.log_norm()[0]:.12f}",
          flush=True)
    assert err < 1e-10
    assert abs(lz - ref.log_norm()[0]) < 1e-10 * abs(ref.log_norm()[0])


def test_trace_distance_matches_the_oracle():
    from oracle.blockbp import trace_distance
    from paper_2301_05844_amd import bbp
    rng = np.random.default_rng(1)
    for m in (2, 4, 16):
        a = rng.standard_normal((m, m))
        b = rng.standard_normal((m, m))
        r, s = a @ a.T, b @ b.T
        r, s = r / np.trace(r), s / np.trace(s)
        assert abs(bbp.trace_distance(r, s) - trace_distance(r, s)) < 1e-13
        assert bbp.trace_distance(r, r) == 0.0
    with pytest.raises(bbp.BBPError):
        bbp.trace_distance(np.zeros((65, 65)), np.zeros((65, 65)))


def test_shift_option_validation():
    from paper_2301_05844_amd import bbp
    with pytest.raises(bbp.BBPError):
        bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=2, chi=4, shift_x=4)
    with pytest.raises(bbp.BBPError):
        bbp.BlockBP(infinite=True, ucx=2, ucy=2, bx=4, by=4, D=2, chi=4, shift_x=1)
    ctx = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=2, chi=4)
    ctx.set_tensors(peps_finite(8, 8, 2, seed=0))
    with pytest.raises(bbp.BBPError):   # after the tensors
        ctx.set_option("shift_y", 1)
