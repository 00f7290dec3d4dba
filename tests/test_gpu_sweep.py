"""GPU sweep parity: messages of the HIP library against the FP64 oracle.

Messages are compared as states (gauge free): as dense vectors with the free
sign fixed, every entry must agree within 1e-12; bond dimensions must agree
exactly, and the residual trajectories must agree.
"""

import numpy as np
import pytest

from bbp_inputs import peps_finite, peps_infinite
from oracle import blockbp as ob

pytestmark = pytest.mark.gpu

CASES = [
    # (name, kwargs, sweeps)
    ("tree_LR_4x2_b2", dict(Lx=4, Ly=2, bx=2, by=2, D=2, chi=4), 3),
    ("tree_UD_2x6_b2", dict(Lx=2, Ly=6, bx=2, by=2, D=2, chi=4), 4),
    ("loop_4x4_b2", dict(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4), 6),
    ("trunc_8x8_b4_chi8", dict(Lx=8, Ly=8, bx=4, by=4, D=2, chi=8), 4),
    ("ragged_7x5_b3x2", dict(Lx=7, Ly=5, bx=3, by=2, D=2, chi=6), 3),
    ("D3_6x6_b3_chi9", dict(Lx=6, Ly=6, bx=3, by=3, D=3, chi=9), 3),
]


def _lib():
    from paper_2301_05844_amd import bbp
    return bbp


def _compare(gpu_msgs, oracle_msgs):
    """Largest entry of the difference of the two messages as dense vectors,
    after fixing the free sign; both have unit norm."""
    worst = 0.0
    for mg, mo in zip(gpu_msgs, oracle_msgs):
        assert [t.shape for t in mg] == [t.shape for t in mo]
        a, b = ob.mps_dense(mg), ob.mps_dense(mo)
        s = 1.0 if np.dot(a, b) >= 0 else -1.0
        worst = max(worst, np.abs(a - s * b).max(), abs(np.linalg.norm(a) - 1))
    return worst


@pytest.mark.parametrize("name,kw,sweeps", CASES, ids=[c[0] for c in CASES])
def test_sweep_matches_oracle(name, kw, sweeps):
    bbp = _lib()
    A = peps_finite(kw["Lx"], kw["Ly"], kw["D"], seed=3)
    ref = ob.BlockBP(A, D=kw["D"], chi=kw["chi"], bx=kw["bx"], by=kw["by"],
                     Lx=kw["Lx"], Ly=kw["Ly"])
    g = bbp.BlockBP(**kw)
    g.set_tensors(A)
    for s in range(sweeps):
        r_ref = ref.sweep()
        r_gpu = g.sweep()
        print(f"{name} sweep {s}: residual gpu {r_gpu:.6e} oracle {r_ref:.6e}",
              flush=True)
        if r_ref > 1e-13:
            assert abs(r_gpu - r_ref) <= 1e-6 * r_ref + 1e-14
        else:
            assert r_gpu < 1e-12
    worst = _compare(g.get_messages(), [ref.msgs[k] for k in ref.order])
    print(f"{name}: worst dense difference {worst:.3e}", flush=True)
    assert worst < 1e-12


def test_sweep_infinite_matches_oracle():
    bbp = _lib()
    A = peps_infinite(2, 2, 2, seed=5)
    ref = ob.BlockBP(A, D=2, chi=8, bx=4, by=4, infinite=True, ucx=2, ucy=2)
    g = bbp.BlockBP(D=2, chi=8, bx=4, by=4, infinite=True, ucx=2, ucy=2)
    g.set_tensors(A)
    for s in range(4):
        r_ref, r_gpu = ref.sweep(), g.sweep()
        print(f"inf sweep {s}: {r_gpu:.6e} {r_ref:.6e}", flush=True)
        assert abs(r_gpu - r_ref) <= 1e-6 * r_ref + 1e-14
    worst = _compare(g.get_messages(), [ref.msgs[k] for k in ref.order])
    assert worst < 1e-12


def test_set_messages_round_trip():
    bbp = _lib()
    A = peps_finite(4, 4, 2, seed=1)
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    g.set_tensors(A)
    g.sweep(2)
    m = g.get_messages()
    g.set_messages(m)
    m2 = g.get_messages()
    for a, b in zip(m, m2):
        for ta, tb in zip(a, b):
            assert np.array_equal(ta, tb)


@pytest.mark.parametrize("lat", [(6, 6, 2, 2, 2, 4), (8, 8, 4, 4, 2, 8), (6, 6, 3, 3, 3, 9)])
def test_random_initial_messages_match_oracle(lat):
    """init 1 (App. A's random product MPDO start): the initial messages
    equal the oracle's entry by entry, and the sweeps from them follow the
    oracle's residuals and messages on loopy and truncated lattices."""
    bbp = _lib()
    Lx, Ly, bx, by, D, chi = lat
    A = peps_finite(Lx, Ly, D, seed=4)
    ref = ob.BlockBP(A, D=D, chi=chi, bx=bx, by=by, Lx=Lx, Ly=Ly, init=1, seed=7)
    g = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=bx, by=by, D=D, chi=chi, init=1, seed=7)
    g.set_tensors(A)
    init_err = max(np.abs(tg - to).max() for mg, mo in
                   zip(g.get_messages(), [ref.msgs[k] for k in ref.order])
                   for tg, to in zip(mg, mo))
    print(f"{lat}: initial messages max |d| {init_err:.2e}", flush=True)
    assert init_err < 1e-15
    for s in range(3):
        r_ref, r_gpu = ref.sweep(), g.sweep()
        print(f"  sweep {s}: gpu {r_gpu:.6e} oracle {r_ref:.6e}", flush=True)
        assert abs(r_gpu - r_ref) <= 1e-6 * r_ref + 1e-14
    worst = _compare(g.get_messages(), [ref.msgs[k] for k in ref.order])
    assert worst < 1e-12


def test_hbm_budget_limits_device_memory():
    """hbm_budget: a context held to 64 KiB cannot set its tensors (BBP_ENOMEM
    after freeing its kept buffers once); with the limit lifted the same
    context works, and a budget above its need changes nothing."""
    bbp = _lib()
    A = peps_finite(8, 8, 2, seed=2)
    g = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=2, chi=8, hbm_budget=1 << 16)
    with pytest.raises(bbp.BBPError) as ei:
        g.set_tensors(A)
        g.sweep(2)
    assert ei.value.status == 2
    g.set_option("hbm_budget", 0)
    g.set_tensors(A)
    r = g.sweep(3)
    ref = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=2, chi=8, hbm_budget=1 << 34)
    ref.set_tensors(A)
    assert r == ref.sweep(3)
    now, peak = ref.memory()
    print(f"budget test: peak {peak} bytes", flush=True)
    assert peak <= 1 << 34


def test_sweep_log_lines(tmp_path, monkeypatch):
    """BBP_SWEEP_LOG: one JSON line per sweep with the residual bbp_sweep
    returned, counted from the last set_tensors."""
    import json
    bbp = _lib()
    path = tmp_path / "sweeps.jsonl"
    monkeypatch.setenv("BBP_SWEEP_LOG", str(path))
    A = peps_finite(6, 6, 2, seed=2)
    g = bbp.BlockBP(Lx=6, Ly=6, bx=2, by=2, D=2, chi=4)
    g.set_tensors(A)
    res = [g.sweep(1) for _ in range(3)]
    monkeypatch.delenv("BBP_SWEEP_LOG")
    g.sweep(1)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [ln["sweep"] for ln in lines] == [1, 2, 3]
    assert [ln["residual"] for ln in lines] == res
    assert all(ln["messages"] == 24 and ln["fit_flops"] > 0 and ln["ms"] > 0 for ln in lines)
