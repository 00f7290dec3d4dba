"""The request server on the GPU: every result equals the same request run
alone (bitwise: requests share no state), equals a plain context run for the
same sweeps, matches the oracle on the small lattice, respects the memory
budget, and honours sweep caps and cancellation."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite

pytestmark = pytest.mark.gpu

REQS = [
    dict(Lx=6, Ly=6, bx=2, by=2, D=2, chi=8),
    dict(Lx=8, Ly=6, bx=3, by=2, D=2, chi=8),     # padded to 9 columns
    dict(Lx=6, Ly=6, bx=3, by=3, D=3, chi=18),
    dict(Lx=8, Ly=8, bx=4, by=4, D=4, chi=32),
    dict(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4),
    dict(Lx=10, Ly=6, bx=2, by=3, D=2, chi=8),
]


def _bbp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_05844_amd import bbp
    return bbp


def _tensors(r, seed):
    return peps_finite(r["Lx"], r["Ly"], r["D"], seed=seed)


def _run(bbp, reqs, budget=64 << 30, slots=4, together=True, tol=1e-10, max_sweeps=30):
    s = bbp.Server(budget_bytes=budget, max_slots=slots)
    out = []
    if together:
        ts = [s.submit(_tensors(r, i), tol=tol, max_sweeps=max_sweeps, **r)
              for i, r in enumerate(reqs)]
        out = [s.wait(t, timeout=300) for t in ts]
    else:
        for i, r in enumerate(reqs):
            t = s.submit(_tensors(r, i), tol=tol, max_sweeps=max_sweeps, **r)
            out.append(s.wait(t, timeout=300))
    stats = s.stats()
    errs = [s.error(t) for t in range(1, len(reqs) + 1)]
    s.close()
    return out, stats, errs


def _same(a, b):
    assert a["sweeps"] == b["sweeps"] and a["residual"] == b["residual"]
    assert a["log_norm"] == b["log_norm"] and a["sign"] == b["sign"]
    assert np.array_equal(a["sz"], b["sz"]) and np.array_equal(a["ss"], b["ss"])


def test_alone_equals_mix_and_requests_overlap():
    bbp = _bbp()
    alone, st1, _ = _run(bbp, REQS, slots=1, together=False)
    mix, st2, errs = _run(bbp, REQS, slots=4, together=True)
    for (sa, ra, _), (sm, rm, _), e in zip(alone, mix, errs):
        assert sa == "done" and sm == "done", e
        assert ra["converged"]
        _same(ra, rm)
    assert st1["max_running"] == 1
    assert st2["max_running"] >= 2   # resident together on the device
    # continuous batching: the sweeps of resident requests ran as shared
    # sweeps, several requests per launch set
    print(st1, st2, flush=True)
    assert st1["shared_sweeps"] == st1["request_sweeps"]
    assert st2["max_together"] >= 2
    assert st2["shared_sweeps"] < st2["request_sweeps"]
    assert st2["request_sweeps"] == sum(r["sweeps"] for _, r, _ in mix)


def test_transverse_ising_terms_match_the_oracle():
    """A request with operators: <sigma_x> of every site and <sigma_z
    sigma_z> of every bond (the transverse-field Ising energy terms), against
    the oracle after the same sweeps (chi_env = max(chi, 2 D^2 + 10))."""
    bbp = _bbp()
    from bbp_inputs import op_sx, op_szsz
    from oracle.blockbp import BlockBP as OracleBP
    r = dict(Lx=6, Ly=6, bx=3, by=3, D=2, chi=8)
    A = _tensors(r, 11)
    s = bbp.Server(budget_bytes=64 << 30, max_slots=2)
    t = s.submit(A, site_ops=[op_sx()], bond_ops=[op_szsz()], tol=1e-12, max_sweeps=30, **r)
    t2 = s.submit(_tensors(REQS[3], 3), **REQS[3])   # another request beside it
    state, res, _ = s.wait(t, timeout=300)
    assert s.wait(t2, timeout=300)[0] == "done"
    s.close()
    assert state == "done"
    ref = OracleBP(A, Lx=6, Ly=6, bx=3, by=3, D=2, chi=8, chi_env=max(8, 18))
    ref.sweep(res["sweeps"])
    sx = res["site_op_values"][0]
    err = max(abs(sx[y, x] - ref.expect_site(x, y, op_sx())) for y in range(6) for x in range(6))
    bonds = [(x, y, x + 1, y) for y in range(6) for x in range(5)]
    bonds += [(x, y, x, y + 1) for y in range(5) for x in range(6)]
    zz = res["bond_op_values"][0]
    err = max([err] + [abs(zz[i] - ref.expect_bond(*b, op_szsz())) for i, b in enumerate(bonds)])
    print(f"transverse-Ising terms: max |d| {err:.2e} after {res['sweeps']} sweeps", flush=True)
    assert err < 1e-10


def test_server_equals_a_plain_context_and_the_oracle():
    bbp = _bbp()
    from oracle.blockbp import BlockBP as OracleBP
    (state, res, times), = _run(bbp, [REQS[4]], slots=1)[0]
    assert state == "done" and times[0] <= times[1] <= times[2]
    r = REQS[4]
    A = _tensors(r, 0)
    g = bbp.BlockBP(Lx=r["Lx"], Ly=r["Ly"], bx=r["bx"], by=r["by"], D=r["D"], chi=r["chi"])
    g.set_tensors(A)
    g.sweep(res["sweeps"])
    xs = [x for y in range(4) for x in range(4)]
    ys = [y for y in range(4) for x in range(4)]
    assert np.array_equal(g.expect_sites(xs, ys, op_sz()), res["sz"].ravel())
    ref = OracleBP(A, Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    ref.sweep(res["sweeps"])
    err = max(abs(res["sz"][y, x] - ref.expect_site(x, y, op_sz()))
              for y in range(4) for x in range(4))
    bonds = [(x, y, x + 1, y) for y in range(4) for x in range(3)]
    bonds += [(x, y, x, y + 1) for y in range(3) for x in range(4)]
    err_ss = max(abs(res["ss"][i] - ref.expect_bond(*b, op_heis())) for i, b in enumerate(bonds))
    err_ln = abs(res["log_norm"] - ref.log_norm()[0])
    assert err < 1e-10 and err_ss < 1e-10 and err_ln < 1e-10


def test_budget_admits_one_at_a_time_and_estimate_bounds_the_peak():
    bbp = _bbp()
    same = [REQS[0]] * 4
    est0 = bbp.estimate_bytes(**REQS[0])
    alone, _, _ = _run(bbp, same, slots=1, together=False)
    tight, st, errs = _run(bbp, same, budget=est0 * 3 // 2, slots=4, together=True)
    assert st["max_running"] == 1   # a second one never fits beside the first
    for (sa, ra, _), (sb, rb, _), e in zip(alone, tight, errs):
        assert sb == "done", e
        _same(ra, rb)
    mix, _, errs = _run(bbp, REQS, slots=4, together=True)
    for (sm, rm, _), r, e in zip(mix, REQS, errs):
        assert sm == "done", e
        assert 0 < rm["peak_bytes"] <= bbp.estimate_bytes(**r)


def test_sweep_cap_and_cancellation():
    bbp = _bbp()
    s = bbp.Server(budget_bytes=64 << 30, max_slots=1)
    r = REQS[3]
    t1 = s.submit(_tensors(r, 3), tol=0.0, max_sweeps=2, **r)
    t2 = s.submit(_tensors(r, 3), tol=0.0, max_sweeps=1000, **r)   # never converges
    t3 = s.submit(_tensors(r, 3), **r)
    s.cancel(t3)                                                    # still queued
    state, res, _ = s.wait(t1, timeout=120)
    assert state == "done" and not res["converged"] and res["sweeps"] == 2
    assert s.poll(t3)[0] == "cancelled"
    import time
    t0 = time.perf_counter()
    while s.poll(t2)[0] != "running" and time.perf_counter() - t0 < 60:
        time.sleep(0.01)
    s.cancel(t2)
    assert s.wait(t2, timeout=120)[0] == "cancelled"
    s.close()
