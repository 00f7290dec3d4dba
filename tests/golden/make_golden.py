"""Write the oracle's expected values for the full-size workloads.

Calls only the FP64 oracle (``oracle/``) and the seeded input generator
(``bbp_inputs``).  Each output JSON holds the workload, the sweep count used
(the first sweep whose residual is below the tolerance), the residual
trajectory, every <sigma_z> and bond <S.S> (or the infinite-lattice terms),
and the log-norm.

    python tests/golden/make_golden.py obc16x16_D4_b4_chi32
    python tests/golden/make_golden.py inf2x2_D4_b4_chi32
    python tests/golden/make_golden.py obc6x6_D6_b3_chi6 3
    python tests/golden/make_golden.py obc8x8_D4_b4_chi56 4
    python tests/golden/make_golden.py obc4x4_D4_b4_env80 5
    python tests/golden/make_golden.py obc8x8_D6_b4_chi64 0
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from bbp_inputs import (CONFIGS, op_heis, op_sx, op_sz, op_szsz,  # noqa: E402
                        peps_finite, peps_infinite)
from oracle.blockbp import BlockBP  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
MAX_SWEEPS = 40


def run(name, seed=0):
    cfg = CONFIGS[name]
    t0 = time.time()
    if cfg["infinite"]:
        A = peps_infinite(cfg["ucx"], cfg["ucy"], cfg["D"], seed=seed)
        bp = BlockBP(A, D=cfg["D"], chi=cfg["chi"], bx=cfg["bx"], by=cfg["by"],
                     infinite=True, ucx=cfg["ucx"], ucy=cfg["ucy"])
    else:
        A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=seed)
        bp = BlockBP(A, D=cfg["D"], chi=cfg["chi"], bx=cfg["bx"], by=cfg["by"],
                     Lx=cfg["Lx"], Ly=cfg["Ly"], chi_env=cfg.get("chi_env"))
    tol = cfg.get("tol")
    res = []
    while True:
        res.append(bp.sweep())
        print(f"{name} sweep {len(res)}: {res[-1]:.3e} ({time.time() - t0:.0f}s)",
              flush=True)
        if tol is None and len(res) == cfg["sweeps"]:
            break
        if tol is not None and (res[-1] < tol or len(res) == MAX_SWEEPS):
            break
    t_sweeps = time.time() - t0
    out = dict(workload=name, config=cfg, seed=seed, sweeps=len(res),
               residuals=res, chi_env=bp.chi_env, n_fit=bp.n_fit)
    if cfg["infinite"]:
        cells = [(x, y) for y in range(cfg["ucy"]) for x in range(cfg["ucx"])]
        out["sites"] = cells
        out["sz"] = [bp.expect_site(x, y, op_sz()) for (x, y) in cells]
        out["sx"] = [bp.expect_site(x, y, op_sx()) for (x, y) in cells]
        bonds = [(x, y, x + 1, y) for (x, y) in cells]
        bonds += [(x, y, x, y + 1) for (x, y) in cells]
        out["bonds"] = bonds
        out["szsz"] = [bp.expect_bond(*b, op_szsz()) for b in bonds]
    else:
        Lx, Ly = cfg["Lx"], cfg["Ly"]
        sites = [(x, y) for y in range(Ly) for x in range(Lx)]
        out["sites"] = sites
        out["sz"] = [bp.expect_site(x, y, op_sz()) for (x, y) in sites]
        bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
        bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
        out["bonds"] = bonds
        out["ss"] = [bp.expect_bond(*b, op_heis()) for b in bonds]
    out["log_norm"], out["log_norm_sign"] = bp.log_norm()
    out["oracle_seconds"] = dict(sweeps=t_sweeps, total=time.time() - t0)
    path = os.path.join(HERE, f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[2].isdigit():
        run(sys.argv[1], seed=int(sys.argv[2]))
        sys.exit(0)
    for n in sys.argv[1:]:
        run(n)
