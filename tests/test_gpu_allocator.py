"""cr_set_allocator: every device block of the batch workspaces and of a
cr_mlp handle comes from the caller's hook and returns through it, and the
results equal those of the library's own hipMalloc workspaces bit for bit.

Two hooks: a small caching pool over hipMalloc / hipFree of the HIP runtime
the library runs on (in this process), and torch's caching allocator (in a
child process that imports torch before the library, so that both share
torch's HIP runtime)."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def items(name, js):
    fam = C.family(3, 5)
    return [workload.first_accepted(name, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in js]


class Pool:
    """Blocks by size, kept after free and handed out again (a caching allocator)."""

    def __init__(self):
        C.lib()
        self.hip = ctypes.CDLL("libamdhip64.so.7")  # by its soname: the runtime the library already loaded
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.live, self.cache, self.log = {}, {}, {"alloc": 0, "free": 0, "reused": 0}

    def alloc(self, n):
        self.log["alloc"] += 1
        if self.cache.get(n):
            ptr = self.cache[n].pop()
            self.log["reused"] += 1
        else:
            p = ctypes.c_void_p()
            assert self.hip.hipMalloc(ctypes.byref(p), n) == 0
            ptr = p.value
        self.live[ptr] = n
        return ptr

    def free(self, ptr):
        n = self.live.pop(ptr)  # KeyError: a block this hook did not allocate
        self.log["free"] += 1
        self.cache.setdefault(n, []).append(ptr)

    def drain(self):
        for blocks in self.cache.values():
            for ptr in blocks:
                self.hip.hipFree(ptr)
        self.cache.clear()


def run_with_hooks(alloc, free, live):
    batch = items("quintic_curves_mixed", range(40))
    more = items("quintic_curves_mixed", range(40, 120))
    fam = C.family(3, 5)
    C.cr_release()
    want = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
    x = np.random.default_rng(0).standard_normal((10, C.CR_MLP_INPUTS)).astype(np.float32)
    ref = C.Mlp(seed=3)
    y_ref = ref.forward(x)
    ref.close()
    del C._hook_errors[:]
    try:
        C.cr_set_allocator(alloc, free)
        got = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
        assert live(), "no block came from the hook"
        assert np.array_equal(got["scaled"], want["scaled"]) and np.array_equal(got["frob"], want["frob"])
        assert got["lpoly"] == want["lpoly"]
        # a larger batch grows the workspaces through the hook
        big = C.cr_frobenius_batch(fam, [p for p, _ in batch + more], [c for _, c in batch + more])
        assert np.array_equal(big["scaled"][:40], want["scaled"]) and big["lpoly"][:40] == want["lpoly"]
        # a network handle allocates through the hook too, and returns every block on close
        n0 = len(live())
        m = C.Mlp(seed=3)
        y = m.forward(x)
        assert len(live()) > n0 and np.array_equal(y, y_ref)
        m.close()
        assert len(live()) == n0
        # a second pass reuses the hook's cached blocks: the library must not see stale contents
        C.cr_release()
        again = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
        assert np.array_equal(again["scaled"], want["scaled"]) and again["lpoly"] == want["lpoly"]
        C.cr_release()
        assert not live(), "blocks not returned through the hook"
        assert not C._hook_errors, C._hook_errors
    finally:
        C.cr_set_allocator()
    after = C.cr_frobenius_batch(fam, [p for p, _ in batch], [c for _, c in batch])
    assert np.array_equal(after["scaled"], want["scaled"])


def test_caching_pool_hook():
    pool = Pool()
    try:
        run_with_hooks(pool.alloc, pool.free, lambda: pool.live)
        assert pool.log["alloc"] == pool.log["free"] and pool.log["reused"] > 0
    finally:
        pool.drain()


CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import torch
torch.zeros(1, device="cuda")
sys.path.insert(0, {tests!r})
import test_gpu_allocator as T
live = {{}}
def alloc(n):
    ptr = torch.cuda.caching_allocator_alloc(n, device=0)
    live[ptr] = n
    return ptr
def free(ptr):
    del live[ptr]
    torch.cuda.caching_allocator_delete(ptr)
T.run_with_hooks(alloc, free, lambda: live)
print("hooks ok")
"""


def test_torch_caching_allocator_hook():
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "hooks ok" in r.stdout, r.stdout[-2000:] + r.stderr[-3000:]
