"""cr_set_allocator with torch's caching allocator as the hook: every device
block of the batch workspaces and of a cr_mlp handle comes from the hook and
returns through it, and the results equal those of the library's own
hipMalloc workspaces bit for bit."""
import numpy as np
import pytest

from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

pytestmark = pytest.mark.gpu


def items(name, js):
    fam = C.family(3, 5)
    out = []
    for j in js:
        out.append(workload.first_accepted(name, j, lambda p, c: C.cr_check_smooth(fam, p, c)))
    return out


def test_torch_caching_allocator_hook():
    import torch
    live = {}
    log = {"alloc": 0, "free": 0}

    def alloc(n):
        ptr = torch.cuda.caching_allocator_alloc(n, device=0)
        live[ptr] = n
        log["alloc"] += 1
        return ptr

    def free(ptr):
        assert ptr in live, "free of a block the hook did not allocate"
        del live[ptr]
        log["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    batch = items("quintic_curves_mixed", range(40))
    fam = C.family(3, 5)
    C.cr_release()
    want = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
    x = np.random.default_rng(0).standard_normal((10, C.CR_MLP_INPUTS)).astype(np.float32)
    ref = C.Mlp(seed=3)
    y_ref = ref.forward(x)
    ref.close()
    try:
        C.cr_set_allocator(alloc, free)
        got = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
        assert log["alloc"] >= 2 and live
        assert np.array_equal(got["scaled"], want["scaled"]) and np.array_equal(got["frob"], want["frob"])
        assert got["lpoly"] == want["lpoly"]
        # a larger batch grows the workspaces through the hook
        more = items("quintic_curves_mixed", range(40, 120))
        big = C.cr_frobenius_batch(fam, [p for p, _ in batch + more], [c for _, c in batch + more])
        assert np.array_equal(big["scaled"][:40], want["scaled"]) and big["lpoly"][:40] == want["lpoly"]
        # a network handle allocates through the hook too
        a0 = log["alloc"]
        m = C.Mlp(seed=3)
        y = m.forward(x)
        assert log["alloc"] > a0 and np.array_equal(y, y_ref)
        f0 = log["free"]
        m.close()
        assert log["free"] - f0 == log["alloc"] - a0
        C.cr_release()
        assert not live, "blocks not returned through the hook: %r" % live
    finally:
        C.cr_set_allocator()
    again = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
    assert np.array_equal(again["scaled"], want["scaled"])
