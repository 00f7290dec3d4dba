"""bbp_set_allocator with PyTorch's caching allocator: the context's device
memory comes from torch (torch.cuda.memory_allocated counts it while the
context lives and drops back when it is destroyed), and every result equals
the hipMalloc context's bitwise."""

import numpy as np
import pytest

from bbp_inputs import op_heis, op_sz, peps_finite

pytestmark = pytest.mark.gpu


def _solve(ctx, A, Lx, Ly):
    ctx.set_tensors(A)
    res = ctx.sweep(3)
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    sz = ctx.expect_sites(xs, ys, op_sz())
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    ss = ctx.expect_bonds(bonds, op_heis())
    return res, sz, ss, ctx.log_norm()[0], ctx.get_messages_flat()


def test_torch_allocator_matches_hipmalloc():
    import torch
    from paper_2301_05844_amd import bbp
    Lx = Ly = 6
    A = peps_finite(Lx, Ly, 3, seed=11)
    plain = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9)
    ref = _solve(plain, A, Lx, Ly)
    plain.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ctx = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9,
                      allocator=bbp.torch_allocator())
    got = _solve(ctx, A, Lx, Ly)
    held = torch.cuda.memory_allocated() - before
    _, peak = ctx.memory()
    print(f"torch-allocated while the context lives: {held} bytes; context peak {peak}",
          flush=True)
    assert held > 0
    for a, b in zip(ref, got):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
