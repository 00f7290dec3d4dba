"""bbp_update_message_noalloc, the update for callers that cannot allocate
device memory (its workspace is a static device array): through the C ABI,
two calls in a row, the second with a smaller input, each bitwise equal to
bbp_update_message on the same inputs; a shape beyond the static workspace
is rejected."""

import numpy as np
import pytest

from bbp_inputs import peps_finite

pytestmark = pytest.mark.gpu


def _inputs(Lx, Ly, b, D, chi, key, before, seed):
    import torch
    from oracle import blockbp as ob
    A = peps_finite(Lx, Ly, D, seed=seed)
    bp = ob.BlockBP(A, D=D, chi=chi, bx=b, by=b, Lx=Lx, Ly=Ly)
    bp.sweep(before)
    e = bp.order.index(key)
    grid, MT, MR, MB = ob.canonical(bp.block_region(*key[:2]), key[2])
    P = D * D
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    def slots(m):
        out = np.zeros((len(m), chi, P, chi))
        for i, t in enumerate(m):
            out[i, :t.shape[0], :, :t.shape[2]] = t
        return dev(out), [m[0].shape[0]] + [t.shape[2] for t in m]
    Ad = dev(np.stack([t for row in grid for t in row]))
    return Ad, [slots(MT), slots(MR), slots(MB)], dict(H=len(grid), W=len(grid[0]), D=D,
                                                       chi=chi, slot=(1 << 40) | (e << 8))


def _both(Ad, sides, kw):
    import torch
    from paper_2301_05844_amd import bbp
    a = bbp.update_message(Ad, *sides, **kw)
    b = bbp.update_message(Ad, *sides, noalloc=True, **kw)
    torch.cuda.synchronize()
    return a, b


def test_noalloc_equals_allocating_update_twice():
    from paper_2301_05844_amd import bbp
    cases = [
        (8, 8, 4, 4, 32, (1, 1, "L"), 2, 3),   # 4x4 block, D=4, chi=32
        (6, 6, 3, 2, 8, (1, 1, "U"), 3, 5),    # then a smaller one: 3x3 block, D=2, chi=8
    ]
    for case in cases:
        Ad, sides, kw = _inputs(*case)
        assert bbp.update_workspace(kw["H"], kw["W"], kw["D"], kw["chi"]) <= bbp.NOALLOC_BYTES
        (oa, ba, la), (ob_, bb, lb) = _both(Ad, sides, kw)
        print(f"{case}: log-scale {la:.15f} / {lb:.15f}", flush=True)
        assert np.array_equal(ba, bb)
        assert la == lb
        assert np.array_equal(oa.cpu().numpy(), ob_.cpu().numpy())


def test_noalloc_rejects_a_shape_beyond_its_workspace():
    import torch
    from paper_2301_05844_amd import bbp
    # 4x4 block, D=6, chi=64: about 150 MB of workspace
    assert bbp.update_workspace(4, 4, 6, 64) > bbp.NOALLOC_BYTES
    A = torch.zeros(16 * 2 * 6 ** 4, dtype=torch.float64, device="cuda")
    with pytest.raises(bbp.BBPError, match="workspace"):
        bbp.update_message(A, H=4, W=4, D=6, chi=64, noalloc=True)
