"""Skipping the zero padding (the "skip_padding" option): the pair-per-wave
visit and the environment update stop at every item's true bond dimensions.
Everything they skip adds exact zeros, so every residual, message,
observable and the log-norm must be bitwise those of the padded kernels, in
FP64 and in FP32, with and without HIP graphs; and the true-shape operation
count must fall below the padded one."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sx, op_sz, op_szsz, peps_finite, peps_infinite

pytestmark = pytest.mark.gpu


def _solve(skip, A, sweeps, precision=64, graphs=1, **kw):
    from paper_2301_05844_amd import bbp
    ctx = bbp.BlockBP(skip_padding=skip, graphs=graphs, **kw)
    ctx.set_option("precision", precision)
    ctx.set_tensors(A)
    res, msgs = [], []
    for _ in range(sweeps):
        res.append(ctx.sweep(1))
        msgs.append(ctx.get_messages_flat())
    if kw.get("infinite"):
        sites = [(0, 0), (1, 0), (0, 1), (1, 1)]
        obs = [ctx.expect_site(x, y, op) for (x, y) in sites for op in (op_sz(), op_sx())]
        obs += [ctx.expect_bond(x, y, x + 1, y, op_szsz()) for (x, y) in sites]
        obs += [ctx.expect_bond(x, y, x, y + 1, op_szsz()) for (x, y) in sites]
        out = np.array(obs)
    else:
        Lx, Ly = kw["Lx"], kw["Ly"]
        xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
        ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
        bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
        bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
        out = np.concatenate([ctx.expect_sites(xs, ys, op_sz()),
                              ctx.expect_bonds(bonds, op_heis())])
    lz = np.array(ctx.log_norm())
    ctx.close()
    return np.array(res), msgs, out, lz


CASES = [
    # 8x8, 4x4 blocks, D=4: bond caps 16 (NE 2), 40 (NE 3), 56 (NE 4)
    dict(Lx=8, Ly=8, bx=4, by=4, D=4, chi=16, chi_env=24),
    dict(Lx=8, Ly=8, bx=4, by=4, D=4, chi=40, chi_env=42),
    dict(Lx=8, Ly=8, bx=4, by=4, D=4, chi=56, chi_env=60),
    # 12x8 with 4x4 blocks: interior blocks with non-trivial top and bottom
    dict(Lx=8, Ly=12, bx=4, by=4, D=4, chi=32, chi_env=42),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_skip_padding_bitwise_equal(case):
    kw = CASES[case]
    A = peps_finite(kw["Lx"], kw["Ly"], kw["D"], seed=11 + case)
    print(f"case {kw}", flush=True)
    a = _solve(0, A, 3, **kw)
    b = _solve(1, A, 3, **kw)
    assert np.array_equal(a[0], b[0])
    for ma, mb in zip(a[1], b[1]):
        assert np.array_equal(ma, mb)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3])


@pytest.mark.parametrize("precision,graphs", [(32, 1), (64, 0)])
def test_skip_padding_bitwise_fp32_and_eager(precision, graphs):
    kw = dict(Lx=8, Ly=12, bx=4, by=4, D=4, chi=32, chi_env=42)
    A = peps_finite(8, 12, 4, seed=21)
    a = _solve(0, A, 3, precision=precision, graphs=graphs, **kw)
    b = _solve(1, A, 3, precision=precision, graphs=graphs, **kw)
    assert np.array_equal(a[0], b[0])
    for ma, mb in zip(a[1], b[1]):
        assert np.array_equal(ma, mb)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_skip_padding_bitwise_infinite():
    kw = dict(infinite=True, ucx=2, ucy=2, bx=4, by=4, D=4, chi=32)
    A = peps_infinite(2, 2, 4, seed=3)
    a = _solve(0, A, 4, **kw)
    b = _solve(1, A, 4, **kw)
    assert np.array_equal(a[0], b[0])
    for ma, mb in zip(a[1], b[1]):
        assert np.array_equal(ma, mb)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_true_shape_counts_below_padded():
    from paper_2301_05844_amd import bbp
    ctx = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=4, chi=32)
    ctx.set_tensors(peps_finite(8, 8, 4, seed=2))
    ctx.sweep(2)
    ctx.set_option("timing", 1)
    ctx.sweep(1)
    ks = {k["name"]: k for k in ctx.kernel_stats()}
    v = ks["fit_visit"]
    print(v, flush=True)
    assert v["launches"] > 0
    assert 0 < v["flops"] < v["padded_flops"]
    assert 0 < v["bytes"] < v["padded_bytes"]
    # the sweep's own count (bbp_stats) is the same true-shape schedule
    _, sweep_flops = ctx.stats()
    total = sum(ks[n]["flops"] for n in ("fit_visit", "fit_env", "fit_end", "fit_T1",
                                          "fit_ket", "fit_bra", "fit_local"))
    assert abs(total - sweep_flops) <= 1e-9 * sweep_flops
    ctx.set_option("timing", 0)
