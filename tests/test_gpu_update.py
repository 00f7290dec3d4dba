"""One directed message update outside a context (bbp_update_message):
the block in its canonical frame (receiver on the left) with its three other
incoming messages, against the FP64 oracle's column absorptions of the same
block (App. A: the same counter-based fit starts, the same n_fit), and
against a context's first sweep.  Messages are compared as states (their
overlap), the removed log-scale absolutely."""

import numpy as np
import pytest

from bbp_inputs import peps_finite

pytestmark = pytest.mark.gpu


def _slots(sites, chi, P):
    """Message site tensors (b, P, b') padded into chi x P x chi slots."""
    out = np.zeros((len(sites), chi, P, chi))
    for i, t in enumerate(sites):
        out[i, :t.shape[0], :, :t.shape[2]] = t
    return out


def _bonds(sites):
    return [sites[0].shape[0]] + [t.shape[2] for t in sites]


def _unslot(flat, bonds, chi, P):
    f = flat.reshape(-1, chi, P, chi)
    return [f[i, :bonds[i], :, :bonds[i + 1]].copy() for i in range(len(bonds) - 1)]


def _dense(m):
    v = m[0]
    for t in m[1:]:
        v = np.tensordot(v, t, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


def _case(Lx, Ly, b, D, chi, key, sweeps_before, seed):
    """Oracle state after `sweeps_before` sweeps, the canonical inputs of
    message `key`, and the oracle's update of it."""
    from oracle import blockbp as ob
    A = peps_finite(Lx, Ly, D, seed=seed)
    bp = ob.BlockBP(A, D=D, chi=chi, bx=b, by=b, Lx=Lx, Ly=Ly)
    bp.sweep(sweeps_before)
    e = bp.order.index(key)
    bi, bj, dr = key
    grid, MT, MR, MB = ob.canonical(bp.block_region(bi, bj), dr)
    Y, ls, _, _ = ob.absorb(grid, MT, MR, MB, chi, bp.n_fit, bp.seed,
                            lambda c: ob.slot_message(e, c))
    ref = ob.extract_message(Y)
    return A, bp, e, grid, MT, MR, MB, ref, ls


def _gpu_update(grid, MT, MR, MB, D, chi, e, trivial=()):
    import torch
    from paper_2301_05844_amd import bbp
    P = D * D
    H, W = len(grid), len(grid[0])
    Ahost = np.stack([t for row in grid for t in row])
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    sides = []
    for name, m in (("T", MT), ("R", MR), ("B", MB)):
        if name in trivial:
            sides.append(None)
        else:
            sides.append((dev(_slots(m, chi, P)), _bonds(m)))
    out, bonds, ls = bbp.update_message(dev(Ahost), *sides, H=H, W=W, D=D, chi=chi,
                                        slot=(1 << 40) | (e << 8))
    torch.cuda.synchronize()
    return _unslot(out.cpu().numpy(), bonds, chi, P), bonds, ls


@pytest.mark.parametrize("Lx,Ly,b,D,chi,key,before", [
    (8, 8, 4, 4, 32, (1, 1, "L"), 2),    # interior-like: all three sides non-trivial
    (8, 8, 4, 4, 32, (0, 0, "D"), 1),    # a corner block sending down
    (12, 8, 4, 3, 20, (1, 0, "R"), 2),   # D=3, rightwards
    (6, 6, 3, 2, 8, (1, 1, "U"), 3),     # 3x3 blocks, upwards
])
def test_update_matches_oracle(Lx, Ly, b, D, chi, key, before):
    A, bp, e, grid, MT, MR, MB, ref, ls = _case(Lx, Ly, b, D, chi, key, before, seed=3)
    got, bonds, gls = _gpu_update(grid, MT, MR, MB, D, chi, e)
    assert list(bonds) == _bonds(ref)
    a, r = _dense(got), _dense(ref)
    ov = abs(np.dot(a, r)) / (np.linalg.norm(a) * np.linalg.norm(r))
    print(f"{key}: overlap 1 - {1 - ov:.2e}, log-scale {gls:.12f} vs {ls:.12f}", flush=True)
    assert abs(np.linalg.norm(a) - 1.0) < 1e-12
    assert 1.0 - ov < 1e-12
    assert abs(gls - ls) < 1e-10 * max(1.0, abs(ls))


def test_update_with_trivial_sides_equals_the_first_sweep():
    # a corner block in the first sweep: the messages are the identity
    # product state, edges trivial; the context's sweep computes the same
    # update from the same inputs
    from paper_2301_05844_amd import bbp
    A, bp, e, grid, MT, MR, MB, ref, ls = _case(8, 8, 4, 4, 16, (0, 0, "R"), 0, seed=4)
    # block (0,0) sending right: in the canonical frame (rotated by a half
    # turn) its top side is the lattice's bottom edge... its trivial sides are
    # the lattice edges, passed as null messages
    from oracle import blockbp as ob
    triv = []
    for name, m in (("T", MT), ("R", MR), ("B", MB)):
        if all(t.shape == (1, 16, 1) and t[0, 0, 0] == 1.0 and np.count_nonzero(t) == 1
               for t in m):
            triv.append(name)
    assert triv  # a corner block has lattice edges among its sides
    got, bonds, gls = _gpu_update(grid, MT, MR, MB, 4, 16, e, trivial=triv)
    ctx = bbp.BlockBP(Lx=8, Ly=8, bx=4, by=4, D=4, chi=16)
    ctx.set_tensors(A)
    ctx.sweep(1)
    msgs = ctx.get_messages()
    m = msgs[e]
    m = m if not ob.OUT_REVERSED["R"] else ob.mps_reverse(m)
    a, r = _dense(got), _dense(m)
    assert abs(abs(np.dot(a, r)) - 1.0) < 1e-12
    assert 1.0 - abs(np.dot(a, _dense(ref))) < 1e-12


def test_update_rejects_bad_arguments():
    import torch
    from paper_2301_05844_amd import bbp
    A = torch.zeros(2 * 2 * 2 * 16, dtype=torch.float64, device="cuda")
    with pytest.raises(bbp.BBPError):
        bbp.update_message(A, H=2, W=2, D=2, chi=0)
    m = torch.zeros(2 * 4 * 4 * 4, dtype=torch.float64, device="cuda")
    with pytest.raises(bbp.BBPError):   # bond above chi
        bbp.update_message(A, None, (m, [1, 5, 1]), None, H=2, W=2, D=2, chi=4)
    with pytest.raises(bbp.BBPError):   # end bond not 1
        bbp.update_message(A, None, (m, [2, 2, 1]), None, H=2, W=2, D=2, chi=4)
    assert bbp.update_workspace(4, 4, 4, 32) > 0
