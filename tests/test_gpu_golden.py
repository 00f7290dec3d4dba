"""Full-size parity against stored oracle values (tests/golden/*.json,
written by tests/golden/make_golden.py from the FP64 oracle only).

16x16 open lattice, D=4, 4x4 blocks, chi=32 and the infinite lattice with a
2x2 unit cell, D=4, 4x4 block, chi=32: the same number of sweeps as the
oracle needed to bring the residual below 1e-10, then every observable
within 1e-10 absolute and the log-norm within 1e-10 relative.

6x6 open lattice, D=6, 3x3 blocks, chi=6, chi_env=16 (seed 3): a fixed two
sweeps, far from converged, so the comparison checks the D=6 kernels step by
step rather than a fixed point both sides fall into; same tolerances.

8x8 open lattice, D=4, 4x4 blocks, chi=56, chi_env=64 (seed 4): two sweeps,
the fits at bond caps 49..64 (the visit's widest pair-per-wave variant).

4x4 open lattice as one D=4 block, chi_env=80 (seed 5): the observables'
boundary fits at a bond cap above 64 (the tiled D=4 visit).

8x8 open lattice, D=6, 4x4 blocks, chi=64, chi_env=82 (seed 0): two sweeps
at the bond caps of the 16x16 D=6 workload (fused D=6 visit at 64, unfused
chain at 82, global-memory QR on both).
"""

import json
import os

import numpy as np
import pytest

from bbp_inputs import (CONFIGS, op_heis, op_sx, op_sz, op_szsz, peps_finite,
                        peps_infinite)

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10


def _golden(name, seed=0):
    path = os.path.join(HERE, "golden", f"{name}_seed{seed}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _check_residuals(gpu, ref, cfg):
    """Residual trajectories: 1e-6 relative, plus an absolute term for the
    rounding floor of 2 - 2|<m_new, m_old>|.  The overlap of two unit
    messages of n entries is a sum of n products: its rounding error is of
    order sqrt(n) eps for independent roundings (n eps at worst), so the
    absolute term is 2 sqrt(n) eps with n the entries of the longest message
    (sites x chi^2 x D^2)."""
    n = max(cfg["bx"], cfg["by"]) * cfg["chi"] ** 2 * cfg["D"] ** 2
    floor = 2.0 * np.sqrt(n) * np.finfo(np.float64).eps
    for k, (a, b) in enumerate(zip(gpu, ref)):
        print(f"sweep {k + 1}: gpu {a:.6e} oracle {b:.6e}", flush=True)
        assert abs(a - b) <= 1e-6 * b + floor, (k, a, b, floor)


def test_obc16x16_D4_chi32_matches_oracle():
    from paper_2301_05844_amd import bbp
    g = _golden("obc16x16_D4_b4_chi32")
    cfg = CONFIGS["obc16x16_D4_b4_chi32"]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"])
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(g["sweeps"])]
    _check_residuals(res, g["residuals"], cfg)
    assert res[-1] < 1e-10
    sites = np.array(g["sites"], dtype=np.int32)
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    err_sz = np.abs(sz - np.array(g["sz"])).max()
    ss = ctx.expect_bonds(g["bonds"], op_heis())
    err_ss = np.abs(ss - np.array(g["ss"])).max()
    lz, sign = ctx.log_norm()
    print(f"max |d sz| {err_sz:.2e}  max |d SS| {err_ss:.2e}  "
          f"log-norm {lz:.12f} vs {g['log_norm']:.12f}", flush=True)
    assert err_sz < TOL and err_ss < TOL
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])
    assert sign == g["log_norm_sign"]


def test_inf2x2_D4_chi32_matches_oracle():
    from paper_2301_05844_amd import bbp
    g = _golden("inf2x2_D4_b4_chi32")
    cfg = CONFIGS["inf2x2_D4_b4_chi32"]
    A = peps_infinite(cfg["ucx"], cfg["ucy"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(D=cfg["D"], chi=cfg["chi"], bx=cfg["bx"], by=cfg["by"],
                      infinite=True, ucx=cfg["ucx"], ucy=cfg["ucy"])
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(g["sweeps"])]
    _check_residuals(res, g["residuals"], cfg)
    assert res[-1] < 1e-10
    for i, (x, y) in enumerate(g["sites"]):
        assert abs(ctx.expect_site(x, y, op_sz()) - g["sz"][i]) < TOL
        assert abs(ctx.expect_site(x, y, op_sx()) - g["sx"][i]) < TOL
    for i, b in enumerate(g["bonds"]):
        assert abs(ctx.expect_bond(*b, op_szsz()) - g["szsz"][i]) < TOL
    lz, _ = ctx.log_norm()
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])


def test_obc6x6_D6_chi6_matches_oracle():
    from paper_2301_05844_amd import bbp
    g = _golden("obc6x6_D6_b3_chi6", seed=3)
    cfg = CONFIGS["obc6x6_D6_b3_chi6"]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"], chi_env=g["chi_env"])
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(g["sweeps"])]
    _check_residuals(res, g["residuals"], cfg)
    sites = np.array(g["sites"], dtype=np.int32)
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    err_sz = np.abs(sz - np.array(g["sz"])).max()
    ss = ctx.expect_bonds(g["bonds"], op_heis())
    err_ss = np.abs(ss - np.array(g["ss"])).max()
    lz, sign = ctx.log_norm()
    print(f"max |d sz| {err_sz:.2e}  max |d SS| {err_ss:.2e}  "
          f"log-norm {lz:.12f} vs {g['log_norm']:.12f}", flush=True)
    assert err_sz < TOL and err_ss < TOL
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])
    assert sign == g["log_norm_sign"]


def test_obc8x8_D4_chi56_matches_oracle():
    from paper_2301_05844_amd import bbp
    g = _golden("obc8x8_D4_b4_chi56", seed=4)
    cfg = CONFIGS["obc8x8_D4_b4_chi56"]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"], chi_env=g["chi_env"])
    ctx.set_tensors(A)
    res = [ctx.sweep(1) for _ in range(g["sweeps"])]
    _check_residuals(res, g["residuals"], cfg)
    sites = np.array(g["sites"], dtype=np.int32)
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    err_sz = np.abs(sz - np.array(g["sz"])).max()
    ss = ctx.expect_bonds(g["bonds"], op_heis())
    err_ss = np.abs(ss - np.array(g["ss"])).max()
    lz, sign = ctx.log_norm()
    print(f"max |d sz| {err_sz:.2e}  max |d SS| {err_ss:.2e}  "
          f"log-norm {lz:.12f} vs {g['log_norm']:.12f}", flush=True)
    assert err_sz < TOL and err_ss < TOL
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])
    assert sign == g["log_norm_sign"]


def test_obc4x4_D4_env80_matches_oracle():
    from paper_2301_05844_amd import bbp
    g = _golden("obc4x4_D4_b4_env80", seed=5)
    cfg = CONFIGS["obc4x4_D4_b4_env80"]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"], chi_env=g["chi_env"])
    ctx.set_tensors(A)
    ctx.sweep(g["sweeps"])
    sites = np.array(g["sites"], dtype=np.int32)
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    err_sz = np.abs(sz - np.array(g["sz"])).max()
    ss = ctx.expect_bonds(g["bonds"], op_heis())
    err_ss = np.abs(ss - np.array(g["ss"])).max()
    lz, sign = ctx.log_norm()
    print(f"max |d sz| {err_sz:.2e}  max |d SS| {err_ss:.2e}  "
          f"log-norm {lz:.12f} vs {g['log_norm']:.12f}", flush=True)
    assert err_sz < TOL and err_ss < TOL
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])
    assert sign == g["log_norm_sign"]


def test_obc8x8_D6_chi64_env82_matches_oracle():
    """8x8 open lattice, D=6, 4x4 blocks, chi=64, chi_env=82 (seed 0), two
    sweeps: the D=6 workload's bond caps.  The message fits run the fused
    D=6 visit at K=64 with the global-memory QR on its 2304 x 64 panels; the
    observables' boundary fits at K=82 run the unfused contraction chain
    (T1, ket, bra, local) with 2952 x 82 QR panels."""
    from paper_2301_05844_amd import bbp
    g = _golden("obc8x8_D6_b4_chi64", seed=0)
    cfg = CONFIGS["obc8x8_D6_b4_chi64"]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=g["seed"])
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"], chi_env=g["chi_env"])
    ctx.set_tensors(A)
    ctx.set_option("timing", 1)
    res = [ctx.sweep(1) for _ in range(g["sweeps"])]
    _check_residuals(res, g["residuals"], cfg)
    sweeps = {k["name"]: k["launches"] for k in ctx.kernel_stats()}
    ctx.kernel_stats_reset()
    sites = np.array(g["sites"], dtype=np.int32)
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    err_sz = np.abs(sz - np.array(g["sz"])).max()
    ss = ctx.expect_bonds(g["bonds"], op_heis())
    err_ss = np.abs(ss - np.array(g["ss"])).max()
    lz, sign = ctx.log_norm()
    obs = {k["name"]: k["launches"] for k in ctx.kernel_stats()}
    ctx.set_option("timing", 0)
    print(f"max |d sz| {err_sz:.2e}  max |d SS| {err_ss:.2e}  "
          f"log-norm {lz:.12f} vs {g['log_norm']:.12f}; launches: sweeps {sweeps}, "
          f"observables {obs}", flush=True)
    assert sweeps["fit_visit"] > 0 and sweeps["fit_T1"] == 0   # fused D=6 visit at K=64
    assert obs["fit_T1"] > 0 and obs["fit_bra"] > 0            # unfused chain at K=82
    assert err_sz < TOL and err_ss < TOL
    assert abs(lz - g["log_norm"]) < TOL * abs(g["log_norm"])
    assert sign == g["log_norm_sign"]
