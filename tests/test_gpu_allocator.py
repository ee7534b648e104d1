"""The handle allocator hook (hipbmg_set_allocator), through the C ABI: handle
memory taken from a caller's allocator (here PyTorch's caching allocator,
wrapped to count) gives bitwise the same solves as memory from hipMalloc,
every block goes back to the allocator that made it when its handle is
destroyed, and a failing allocator makes setup fail cleanly."""
import os
import subprocess
import sys

import pytest
import torch

from paper_1803_02481_amd import hipbmg as HB
from paper_1803_02481_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def g(a):
    return torch.from_numpy(a).to(DEV)


class Pool:
    """Counting wrapper around torch's caching allocator; optionally fails the
    k-th request or returns misaligned blocks."""

    def __init__(self, fail_at=None, misalign=False):
        self.live, self.n_alloc, self.n_free = {}, 0, 0
        self.fail_at, self.misalign = fail_at, misalign

    def alloc(self, nbytes):
        self.n_alloc += 1
        if self.fail_at is not None and self.n_alloc == self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes + (8 if self.misalign else 0), device=0)
        q = p + 8 if self.misalign else p
        self.live[q] = p
        return q

    def free(self, q):
        p = self.live.pop(q)   # KeyError: a block this pool never made
        self.n_free += 1
        torch.cuda.caching_allocator_delete(p)


def problems():
    c2 = HB.fv5_from_cells(g(inputs.cells_log10_blocks(65, 65, block=8, seed=21)))
    b2 = g(inputs.load_uniform(65, 65, seed=22))
    c3 = HB.fv7_from_cells(g(inputs.cells3_log10_blocks(17, 17, 17, block=4, seed=23)))
    b3 = g(inputs.load3_uniform(17, 17, 17, seed=24))
    cb = [HB.fv5_from_cells(g(inputs.cells_lognormal(n, n, sigma=1.0, seed=31 + k)))
          for k, n in enumerate((33, 65, 129))]
    bb = [g(inputs.load_uniform(n, n, seed=41 + k)) for k, n in enumerate((33, 65, 129))]
    return c2, b2, c3, b3, cb, bb


def run_all(p):
    c2, b2, c3, b3, cb, bb = p
    out = []
    for prec in (0, 1):
        h = HB.Hierarchy(c2, precision=prec)
        out.append(h.solve(b2, tol=1e-10))
        h.close()
    h3 = HB.Hierarchy3(c3)
    out.append(h3.solve(b3, tol=1e-10))
    h3.close()
    hb = HB.BatchHierarchy(cb)
    us, infos = hb.solve(bb, tol=1e-10)
    hb.close()
    out += list(zip(us, infos))
    torch.cuda.synchronize()
    return out


@pytest.fixture(autouse=True, scope="module")
def calibrated():
    # warm-up: the first hierarchies of each kind in the process are built
    # before any test allocator is registered, so the counts below see only
    # the tests' own handles
    c2, b2, c3, b3, _, _ = problems()
    HB.Hierarchy(c2).close()
    HB.Hierarchy3(c3).close()
    torch.cuda.synchronize()
    yield


def same(a, b):
    for (ua, ia), (ub, ib) in zip(a, b):
        assert ia.cycles == ib.cycles
        assert torch.equal(ua, ub)


def test_solves_from_a_registered_allocator_match_hipmalloc():
    p = problems()
    HB.set_allocator()
    try:
        ref = run_all(p)   # hipMalloc
    finally:
        HB.use_torch_allocator()
    pool = Pool()
    HB.set_allocator(pool.alloc, pool.free)
    try:
        got = run_all(p)
    finally:
        HB.use_torch_allocator()
    same(ref, got)
    assert pool.n_alloc > 0
    assert pool.n_free == pool.n_alloc and not pool.live
    # back on the binding's default (torch's caching allocator): the pool sees nothing more
    again = run_all(p)
    same(ref, again)
    assert pool.n_alloc == pool.n_free


def test_blocks_return_to_their_own_allocator_after_a_switch():
    c2, b2, c3, b3, _, _ = problems()
    pool = Pool()
    HB.set_allocator(pool.alloc, pool.free)
    try:
        h = HB.Hierarchy(c2)
        h3 = HB.Hierarchy3(c3)
    finally:
        HB.use_torch_allocator()
    n = pool.n_alloc
    assert n > 0 and len(pool.live) == n
    # a handle built on the default allocator in between, and solves on the pooled ones
    h_plain = HB.Hierarchy(c2)
    u1, _ = h.solve(b2, tol=1e-10)
    u2, _ = h_plain.solve(b2, tol=1e-10)
    assert torch.equal(u1, u2)
    h3.solve(b3, tol=1e-10)
    h.close()
    h3.close()
    h_plain.close()
    assert pool.n_alloc == n and not pool.live


@pytest.mark.parametrize("which", ["first", "middle", "last"])
def test_a_failing_allocator_fails_setup_without_leaks(which):
    # the setup's first, middle or last request fails (the number of requests
    # is counted on a setup that succeeds: small arrays share zeroed chunks)
    c2, _, c3, _, _, _ = problems()
    for make in (lambda: HB.Hierarchy(c2), lambda: HB.Hierarchy3(c3)):
        make().close()   # the process's one-time model calibration, if not done yet
        count = Pool()
        HB.set_allocator(count.alloc, count.free)
        try:
            make().close()
        finally:
            HB.use_torch_allocator()
        n = count.n_alloc
        assert n >= 1 and not count.live
        fail_at = {"first": 1, "middle": (n + 1) // 2, "last": n}[which]
        pool = Pool(fail_at=fail_at)
        HB.set_allocator(pool.alloc, pool.free)
        try:
            with pytest.raises(HB.HipBMGError) as e:
                make()
        finally:
            HB.use_torch_allocator()
        assert e.value.status == HB.ENOMEM
        assert not pool.live, "blocks left behind after a failed setup"


def test_misaligned_blocks_are_refused():
    c2, _, _, _, _, _ = problems()
    pool = Pool(misalign=True)
    HB.set_allocator(pool.alloc, pool.free)
    try:
        with pytest.raises(HB.HipBMGError) as e:
            HB.Hierarchy(c2)
    finally:
        HB.use_torch_allocator()
    assert e.value.status == HB.ENOMEM
    assert pool.n_alloc >= 1 and not pool.live


def test_handles_left_open_at_exit_are_closed_cleanly():
    # a program that takes handle memory from torch's allocator and leaves its
    # handles open: they are closed at exit, while the callbacks still work
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import torch\n"
        "from paper_1803_02481_amd import hipbmg as HB, inputs\n"
        "HB.lib()\n"
        "c = HB.fv5_from_cells(torch.from_numpy(inputs.cells_log10_blocks(33, 33, block=8, seed=1)).to('cuda:0'))\n"
        "h = HB.Hierarchy(c)\n"
        "d = torch.from_numpy(inputs.cells3_log10_blocks(9, 9, 9, block=4, seed=2)).to('cuda:0')\n"
        "h3 = HB.Hierarchy3(HB.fv7_from_cells(d))\n"
        "print('built', len(HB._open_handles), flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "built 2" in r.stdout


def test_many_handles_share_the_pinned_pool():
    # every handle takes three 512-byte pinned slots (scalars, flags, the
    # host-mapped test slots) from slabs of 256 slots kept for the process:
    # 300 open handles need several slabs, and the slots of destroyed handles
    # serve the next ones; every solve still reads its own convergence test
    c2, b2, _, _, _, _ = problems()
    hs = [HB.Hierarchy(c2) for _ in range(300)]
    ref, info_ref = hs[0].solve(b2, tol=1e-10)
    for k in (1, 150, 299):
        u, info = hs[k].solve(b2, tol=1e-10)
        assert torch.equal(u, ref) and info.cycles == info_ref.cycles and info.history() == info_ref.history()
    for h in hs[::2]:
        h.close()
    more = [HB.Hierarchy(c2) for _ in range(150)]
    for h in (more[0], more[-1], hs[1]):
        u, info = h.solve(b2, tol=1e-10)
        assert torch.equal(u, ref) and info.cycles == info_ref.cycles
    for h in hs[1::2] + more:
        h.close()
