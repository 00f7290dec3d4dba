"""Lanes (the "lanes" option): message batches (one per shape) and
boundary-stack batches (every shape split) on several streams give bitwise
the results of one stream, since every item is computed from its own inputs
only."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite

pytestmark = pytest.mark.gpu


def _run(lanes, A, Lx, Ly, bx, by, D, chi, sweeps):
    from paper_2301_05844_amd import bbp
    ctx = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=bx, by=by, D=D, chi=chi, lanes=lanes)
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(sweeps)]
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    sz = ctx.expect_sites(xs, ys, op_sz())
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    ss = ctx.expect_bonds(bonds, op_heis())
    lz = ctx.log_norm()
    msgs = ctx.get_messages_flat()
    return np.array(res), sz, ss, np.array(lz), msgs


@pytest.mark.parametrize("lanes", [2, 3, 4])
@pytest.mark.parametrize("lat", [(8, 8, 2, 2), (8, 6, 2, 3)])
def test_lanes_bitwise_equal(lanes, lat):
    # 8x8 lattice, 2x2 blocks: 48 messages of one shape in one batch, the
    # region stacks split over the lanes; 8x6 lattice, 2x3 blocks: two message
    # shapes, one batch on each lane
    Lx, Ly, bx, by = lat
    A = peps_finite(Lx, Ly, 3, seed=5)
    one = _run(1, A, Lx, Ly, bx, by, 3, 9, 3)
    many = _run(lanes, A, Lx, Ly, bx, by, 3, 9, 3)
    print(f"lanes {lanes}, lattice {lat}: residuals {many[0]}", flush=True)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_lanes_option_validation():
    from paper_2301_05844_amd import bbp
    for bad in (0, 5, 1.5):
        with pytest.raises(bbp.BBPError):
            bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4, lanes=bad)


@pytest.mark.parametrize("split", [0, 2, 3])
def test_message_split_bitwise_equal(split):
    # 8x8 lattice with 2x2 blocks, D=3: the 48 messages of one shape split
    # into `split` batches on their own lanes (0: one batch per message)
    from paper_2301_05844_amd import bbp
    A = peps_finite(8, 8, 3, seed=6)
    one = _run(3, A, 8, 8, 2, 2, 3, 9, 3)
    ctx_kw = dict(message_split=split)
    ctx = bbp.BlockBP(Lx=8, Ly=8, bx=2, by=2, D=3, chi=9, lanes=3, **ctx_kw)
    ctx.set_tensors(A)
    res = np.array([ctx.sweep(1) for _ in range(3)])
    assert np.array_equal(res, one[0])
    assert np.array_equal(ctx.get_messages_flat(), one[4])


@pytest.mark.parametrize("lanes", [1, 2, 3])
def test_expect_terms_bitwise_equal(lanes):
    # 8x8 lattice, 2x2 blocks, D=3: the sites' block regions and the bonds'
    # two-block unions contracted in one call (their stacks side by side on
    # the lanes) give bitwise the values of the two separate calls
    from paper_2301_05844_amd import bbp
    Lx = Ly = 8
    A = peps_finite(Lx, Ly, 3, seed=7)
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    sep = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9, lanes=1)
    sep.set_tensors(A)
    sep.sweep(3)
    sz = sep.expect_sites(xs, ys, op_sz())
    ss = sep.expect_bonds(bonds, op_heis())
    tog = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9, lanes=lanes)
    tog.set_tensors(A)
    tog.sweep(3)
    for rep in range(2):   # the second call: cached batches and buffers
        if rep:
            tog.set_tensors(A)
            tog.sweep(3)
        sz2, ss2 = tog.expect_terms(xs, ys, op_sz(), bonds, op_heis())
        print(f"lanes {lanes} call {rep}: max |sz| {np.abs(sz2).max():.3f}", flush=True)
        assert np.array_equal(sz, sz2)
        assert np.array_equal(ss, ss2)
    assert np.array_equal(np.array(sep.log_norm()), np.array(tog.log_norm()))
    # one kind only, and nothing at all
    s3, b3 = tog.expect_terms(xs[:5], ys[:5], op_sz(), [], op_heis())
    assert np.array_equal(s3, sz[:5]) and b3.size == 0
    s4, b4 = tog.expect_terms([], [], op_sz(), bonds[:7], op_heis())
    assert s4.size == 0 and np.array_equal(b4, ss[:7])
