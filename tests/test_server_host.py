"""Host-side checks of the request server (no GPU needed): request
validation, admission limits and the memory estimate."""

import pytest

from bbp_inputs import peps_finite


def _bbp():
    from paper_2301_05844_amd import bbp
    return bbp


def test_estimate_grows_with_the_problem():
    bbp = _bbp()
    base = dict(Lx=8, Ly=8, bx=2, by=2, D=2, chi=8)
    e0 = bbp.estimate_bytes(**base)
    assert e0 > 0
    assert bbp.estimate_bytes(**dict(base, Lx=12, Ly=12)) > e0
    assert bbp.estimate_bytes(**dict(base, D=3, chi=18)) > e0
    assert bbp.estimate_bytes(**dict(base, chi=16)) > e0
    with pytest.raises(bbp.BBPError):
        bbp.estimate_bytes(**dict(base, chi=0))


def test_submit_validates_requests():
    bbp = _bbp()
    s = bbp.Server(budget_bytes=64 << 30, max_slots=1)
    A = peps_finite(4, 4, 2, seed=0)
    ok = dict(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    for bad in [dict(ok, tol=-1.0), dict(ok, max_sweeps=0), dict(ok, chi=200),
                dict(ok, outputs=8), dict(ok, bx=0)]:
        with pytest.raises(bbp.BBPError) as e:
            s.submit(A, **bad)
        assert e.value.status == 1
    with pytest.raises(bbp.BBPError) as e:
        s.submit(A[:-1], **ok)   # tensor count does not match the lattice
    assert e.value.status == 1
    with pytest.raises(bbp.BBPError):
        s.poll(12345)
    s.close()


def test_request_above_the_budget_is_refused():
    bbp = _bbp()
    req = dict(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    est = bbp.estimate_bytes(**req)
    s = bbp.Server(budget_bytes=est - 1, max_slots=2)
    with pytest.raises(bbp.BBPError) as e:
        s.submit(peps_finite(4, 4, 2, seed=0), **req)
    assert e.value.status == 2   # BBP_ENOMEM: could never be admitted
    s.close()


def test_server_arguments():
    bbp = _bbp()
    for budget, slots in [(0, 1), (1 << 30, 0), (1 << 30, 65)]:
        with pytest.raises(bbp.BBPError):
            bbp.Server(budget_bytes=budget, max_slots=slots)


def test_without_gpu_requests_fail_with_the_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    bbp = _bbp()
    s = bbp.Server(budget_bytes=64 << 30, max_slots=2)
    t = s.submit(peps_finite(4, 4, 2, seed=0), Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    state, res, times = s.wait(t, timeout=60)
    assert state == "failed" and res is None
    assert "no HIP device" in s.error(t)
    assert times[0] <= times[1] <= times[2]
    s.close()
