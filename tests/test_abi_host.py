"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/bbp.h declares, and
reject bad arguments before touching a device.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from bbp_inputs import peps_finite

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbp.h")


def _bbp():
    try:
        from paper_2301_05844_amd import bbp
    except ImportError as e:
        pytest.fail(f"libbbp.so missing: {e}")
    return bbp


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbp_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    bbp = _bbp()
    assert set(_declared()) == set(bbp.EXPORTS)


def test_every_declared_symbol_is_exported():
    bbp = _bbp()
    lib = ctypes.CDLL(bbp.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_create_validates_arguments():
    bbp = _bbp()
    lib = bbp.lib()
    ctx = ctypes.c_void_p()
    bad = [
        (0, 4, 4, 0, 0, 0, 2, 2, 4),      # bx = 0
        (0, 4, 4, 0, 0, 2, 2, 0, 4),      # D = 0
        (0, 0, 4, 0, 0, 2, 2, 2, 4),      # Lx = 0
        (1, 0, 0, 2, 2, 3, 4, 2, 4),      # block not a multiple of the cell
        (0, 4, 4, 0, 0, 2, 2, 2, 200),    # chi above the supported cap
        (0, 80, 80, 0, 0, 40, 40, 2, 4),  # block longer than the boundary cap
    ]
    for args in bad:
        assert lib.bbp_create(ctypes.byref(ctx), *args) == 1, args
    assert lib.bbp_create(None, 0, 4, 4, 0, 0, 2, 2, 2, 4) == 1
    assert lib.bbp_create(ctypes.byref(ctx), 0, 4, 4, 0, 0, 2, 2, 2, 4) == 0
    lib.bbp_destroy(ctx)


def test_options_and_state_checks():
    bbp = _bbp()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    with pytest.raises(bbp.BBPError) as e:
        g.set_option("no_such_option", 1)
    assert e.value.status == 1
    for key, val in [("n_fit", 0), ("n_fit", 2.5), ("chi_env", 0),
                     ("chi_env", 500), ("d", 0), ("seed", -1), ("precision", 8),
                     ("lanes", 0), ("lanes", 5), ("graphs", 2), ("graphs", 0.5)]:
        with pytest.raises(bbp.BBPError):
            g.set_option(key, val)
    g.set_option("n_fit", 3)
    g.set_option("chi_env", 20)
    g.set_option("precision", 32)
    g.set_option("precision", 16)
    g.set_option("precision", 64)
    g.set_option("lanes", 1)
    g.set_option("graphs", 0)
    g.set_option("graphs", 1)
    with pytest.raises(bbp.BBPError) as e:
        g.sweep(1)
    assert e.value.status == 4  # BBP_ESTATE before the tensors
    with pytest.raises(bbp.BBPError) as e:
        g.expect_site(0, 0, np.eye(2))
    assert e.value.status == 4
    with pytest.raises(bbp.BBPError) as e:
        g.expect_terms([0], [0], np.eye(2), [(0, 0, 1, 0)], np.eye(4))
    assert e.value.status == 4


def test_allocator_validation():
    bbp = _bbp()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    lib = bbp.lib()
    # one function without the other
    assert lib.bbp_set_allocator(g._ctx, bbp.ALLOC_FN(lambda n, u: None), bbp.FREE_FN(),
                                 None) == 1
    assert lib.bbp_set_allocator(None, bbp.ALLOC_FN(), bbp.FREE_FN(), None) == 1
    calls = []
    g.set_allocator(lambda n: calls.append(n) or 0, lambda p: None)
    g.set_allocator(None, None)   # back to hipMalloc / hipFree
    assert calls == []             # nothing allocates before the tensors


def test_set_tensors_validates_before_device():
    bbp = _bbp()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    A = peps_finite(4, 4, 2, seed=0)
    with pytest.raises(bbp.BBPError) as e:
        g.set_tensors(A[:-1])
    assert e.value.status == 1
    B = A.copy()
    B[0, 0, 1, 0, 0, 0] = 0.5   # up leg of a top-edge site, index 1
    with pytest.raises(bbp.BBPError) as e:
        g.set_tensors(B)
    assert e.value.status == 1 and "open-edge" in str(e.value)
    B = A.copy()
    B[7, 1, 0, 1, 0, 1] = np.inf
    with pytest.raises(bbp.BBPError) as e:
        g.set_tensors(B)
    assert e.value.status == 1


def test_gpu_absence_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    bbp = _bbp()
    g = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    with pytest.raises(bbp.BBPError) as e:
        g.set_tensors(peps_finite(4, 4, 2, seed=0))
    assert e.value.status == 3  # BBP_EDEVICE, no silent CPU path


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_bench_lattice_terms():
    # the sites and nearest-neighbour bonds a bench solve evaluates: every
    # site and bond of a finite lattice; the unit cell and its right/down
    # bonds on the infinite lattice
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from bbp_inputs import CONFIGS
    sites, bonds = bench.lattice_terms(CONFIGS["obc16x16_D4_b4_chi32"])
    assert len(sites) == 256 and len(bonds) == 2 * 16 * 15
    assert len(set(map(tuple, sites.tolist()))) == 256
    assert all(abs(x1 - x0) + abs(y1 - y0) == 1 for x0, y0, x1, y1 in bonds)
    sites, bonds = bench.lattice_terms(CONFIGS["obc4x4_D2_b2_chi4"])
    assert len(sites) == 16 and len(bonds) == 24
    sites, bonds = bench.lattice_terms(CONFIGS["inf2x2_D4_b4_chi32"])
    assert sorted(map(tuple, sites.tolist())) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert len(bonds) == 8 and len(set(bonds)) == 8


def test_trace_distance_on_the_host():
    # bbp_trace_distance is host arithmetic: no device needed
    import numpy as np
    from oracle.blockbp import trace_distance
    from paper_2301_05844_amd import bbp
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((4, 4)), rng.standard_normal((4, 4))
    r, s = a @ a.T / np.trace(a @ a.T), b @ b.T / np.trace(b @ b.T)
    assert abs(bbp.trace_distance(r, s) - trace_distance(r, s)) < 1e-13
    p, q = np.diag([0.5, 0.3, 0.2, 0.0]), np.diag([0.25, 0.25, 0.25, 0.25])
    assert abs(bbp.trace_distance(p, q) - 0.5 * (0.25 + 0.05 + 0.05 + 0.25)) < 1e-15


def _ite_case(seed, k, kb, d=2, D=2, rank=None):
    from scipy.linalg import expm
    rng = np.random.default_rng(seed)
    n = k * kb
    B = rng.standard_normal((n, rank or n))
    N = B @ B.T
    N /= np.trace(N)
    theta = rng.standard_normal((k, d, d, kb))
    sz = np.diag([0.5, -0.5])
    sx = np.array([[0.0, 0.5], [0.5, 0.0]])
    h = -np.kron(sz, sz) * 4 - 0.5 * (np.kron(sx, np.eye(2)) + np.kron(np.eye(2), sx)) * 2
    return N, theta, expm(-0.1 * h)


@pytest.mark.parametrize("case", [(0, 4, 4, None), (1, 8, 8, None), (2, 6, 6, 20),
                                  (3, 4, 8, None)])
def test_ite_fit_on_the_host_matches_oracle(case):
    """bbp_ite_fit (host least squares of App. B) against the oracle's
    fit_pair on the same environment: the fitted pair R L (invariant under
    the bond gauge, which the SVD start's signs fix differently) and the
    fit error agree; a rank-deficient environment (k kb = 36, rank 20)
    included."""
    from oracle import ite
    bbp = _bbp()
    seed, k, kb, rank = case
    N, theta, gate = _ite_case(seed, k, kb, rank=rank)
    D = 2 if k == 4 and kb == 4 else 3
    R, L, loss = bbp.ite_fit(N, theta, gate, D, n_als=4)
    Ro, Lo = ite.fit_pair(N, theta, gate, D, 4)
    # the SVD start is signed by one convention on both sides: R, L agree
    assert np.abs(R - Ro).max() < 1e-9 * np.abs(Ro).max()
    assert np.abs(L - Lo).max() < 1e-9 * np.abs(Lo).max()
    pair = np.einsum("asr,rtb->astb", R, L)
    pair_o = np.einsum("asr,rtb->astb", Ro, Lo)
    err = np.abs(pair - pair_o).max() / np.abs(pair_o).max()
    T = np.einsum("tusv,asvb->atub", gate.reshape(2, 2, 2, 2), theta)
    diff = (pair_o - T).transpose(1, 2, 0, 3).reshape(4, -1)
    Tm = T.transpose(1, 2, 0, 3).reshape(4, -1)
    N4 = N.reshape(k * kb, k * kb)
    loss_o = np.trace(diff @ N4 @ diff.T) / np.trace(Tm @ N4 @ Tm.T)
    print(f"k {k} kb {kb} D {D}: max rel |d(RL)| {err:.2e}, loss {loss:.3e} vs {loss_o:.3e}")
    assert err < 1e-9
    assert abs(loss - loss_o) < 1e-9 * max(loss_o, 1e-3)


def test_ite_fit_rejects_bad_arguments():
    bbp = _bbp()
    N, theta, gate = _ite_case(0, 4, 4)
    with pytest.raises(bbp.BBPError):
        bbp.ite_fit(N, theta, gate, 2, n_als=0)
    bad = N.copy()
    bad[0, 0] = np.nan
    with pytest.raises(bbp.BBPError):
        bbp.ite_fit(bad, theta, gate, 2)


def test_init_and_hbm_budget_option_validation():
    bbp = _bbp()
    c = bbp.BlockBP(Lx=4, Ly=4, bx=2, by=2, D=2, chi=4)
    for key, bad in (("init", 2), ("init", 0.5), ("hbm_budget", -1), ("hbm_budget", 1.5)):
        with pytest.raises(bbp.BBPError):
            c.set_option(key, bad)
    c.set_option("init", 1)
    c.set_option("hbm_budget", 1 << 30)


def test_svd_jacobi_rejects_bad_arguments_before_the_device():
    """bbp_svd_jacobi checks its sizes and pointers before any HIP call."""
    bbp = _bbp()
    lib = bbp.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every case fails first
    bad = [
        (-1, 8, 4, 4, 60, 0.0),            # batch < 0
        (1, 8, 0, 1, 60, 0.0),             # n = 0
        (1, 80, 65, 65, 60, 0.0),          # n above 64
        (1, 3, 4, 4, 60, 0.0),             # m < n
        (1, 8, 4, 0, 60, 0.0),             # k = 0
        (1, 8, 4, 5, 60, 0.0),             # k > n
        (1, 8, 4, 4, 0, 0.0),              # max_sweeps = 0
        (1, 8, 4, 4, 101, 0.0),            # max_sweeps above 100
        (1, 8, 4, 4, 60, 1.0),             # tol >= 1
        (1, 8, 4, 4, 60, -1e-3),           # tol < 0
        (1, 8, 4, 4, 60, float("nan")),    # tol NaN
        (1, 400, 60, 60, 60, 0.0),         # m n + n n above BBP_SVD_MAX_WORDS
    ]
    for b, m, n, k, sw, tol in bad:
        st = lib.bbp_svd_jacobi(b, m, n, k, fake, fake, fake, fake, None, None, sw, tol, None)
        assert st == 1, (b, m, n, k, sw, tol)
    # null operands with work to do
    assert lib.bbp_svd_jacobi(1, 8, 4, 4, None, fake, fake, fake, None, None, 60, 0.0,
                              None) == 1
    assert lib.bbp_svd_jacobi(1, 8, 4, 4, fake, fake, None, fake, None, None, 60, 0.0,
                              None) == 1
    # an empty batch is a no-op that needs no pointers
    assert lib.bbp_svd_jacobi(0, 8, 4, 4, None, None, None, None, None, None, 60, 0.0,
                              None) == 0
    assert bbp.SVD_MAX_WORDS == 19968
