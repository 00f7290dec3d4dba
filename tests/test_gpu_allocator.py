"""bbp_set_allocator with PyTorch's caching allocator: the context's device
memory comes from torch (torch.cuda.memory_allocated counts it while the
context lives and drops back when it is destroyed), and every result equals
the hipMalloc context's bitwise.  An allocator that fails on purpose drives
the out-of-memory path: the kept buffers are freed and the allocation tried
once more; a second failure is reported as BBP_ENOMEM."""

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


class _FailingAllocator:
    """torch's allocator, except that allocations of at least `min_bytes`
    fail while `fail_left` > 0 (each failure counts one down)."""

    def __init__(self, min_bytes):
        from paper_2301_05844_amd import bbp
        self.alloc_t, self.free_t = bbp.torch_allocator()
        self.min_bytes = min_bytes
        self.fail_left = 0
        self.failed = 0

    def alloc(self, nbytes):
        if self.fail_left > 0 and nbytes >= self.min_bytes:
            self.fail_left -= 1
            self.failed += 1
            return 0
        return self.alloc_t(nbytes)

    def free(self, ptr):
        self.free_t(ptr)


def test_failed_allocation_frees_kept_buffers_and_retries():
    # one failed allocation inside an observables call: the context frees
    # the buffers it keeps for reuse, tries once more, and every result
    # equals the undisturbed context's bitwise
    import torch
    from paper_2301_05844_amd import bbp
    Lx = Ly = 6
    A = peps_finite(Lx, Ly, 3, seed=11)
    plain = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9)
    ref = _solve(plain, A, Lx, Ly)
    plain.close()
    fa = _FailingAllocator(min_bytes=1 << 16)
    ctx = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9, allocator=(fa.alloc, fa.free))
    ctx.set_tensors(A)
    res = ctx.sweep(3)
    xs = np.array([x for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    ys = np.array([y for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    sz = ctx.expect_sites(xs, ys, op_sz())       # fills the reuse caches
    fa.fail_left = 1
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    ss = ctx.expect_bonds(bonds, op_heis())      # new shapes: allocates
    print(f"failed allocations: {fa.failed}", flush=True)
    assert fa.failed == 1
    got = (res, sz, ss, ctx.log_norm()[0], ctx.get_messages_flat())
    for a, b in zip(ref, got):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    ctx.close()
    # an allocation that fails again after the retry is reported as
    # BBP_ENOMEM, and the context works once memory is available again
    fa.fail_left = 2
    ctx2 = bbp.BlockBP(Lx=Lx, Ly=Ly, bx=2, by=2, D=3, chi=9, allocator=(fa.alloc, fa.free))
    with pytest.raises(bbp.BBPError) as ei:
        ctx2.set_tensors(A)
    print(f"second context: {ei.value}", flush=True)
    assert "ENOMEM" in str(ei.value) and fa.fail_left == 0
    ctx2.set_tensors(A)
    assert np.array_equal(np.asarray(ctx2.sweep(3)), np.asarray(ref[0]))
    assert np.array_equal(ctx2.get_messages_flat(), ref[4])
    ctx2.close()
    torch.cuda.synchronize()
