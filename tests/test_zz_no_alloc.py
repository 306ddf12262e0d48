"""The allocation-free entry point (dm_enumerate_noalloc) against the
allocating one (dm_enumerate), through the C ABI on the GPU.

The context is given a counting device allocator, so a call that took any
device memory through the library would show up in its count; torch's own
allocator statistics must not move either.  Two calls in a row, the second
with a smaller pattern and table, must each equal dm_enumerate's table (and
the oracle's); a capped call, the count+hash mode, a count-only call and a
destination that is too small are checked as well."""
import sys

import numpy as np
import pytest

import oracle
import paper_2508_21287_amd as dm
from paper_2508_21287_amd import workloads as W

pytestmark = pytest.mark.gpu

BUDGET = -6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingAllocator:
    def __init__(self, torch):
        self.torch = torch
        self.calls = 0
        self.live = {}

    def alloc(self, nbytes, stream):
        self.calls += 1
        p = self.torch.cuda.caching_allocator_alloc(nbytes, 0, stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, stream):
        del self.live[ptr]
        self.torch.cuda.caching_allocator_delete(ptr)


def plain_rows(dg, p, cap=-1):
    with dg.enumerate(p.n, p.edges, cap) as r:
        return r.to_numpy(), r.total


def test_noalloc_matches_enumerate():
    import torch
    torch.cuda.set_device(0)
    al = CountingAllocator(torch)
    ctx = dm.Context(0, allocator=(al.alloc, al.free))
    g, pats = W.config2(12)
    dg = ctx.datagraph(g.n, g.edges)
    want = {p.name: plain_rows(dg, p) for p in pats}
    order = sorted(pats, key=lambda p: (len(want[p.name][0]), p.n), reverse=True)
    big, small = order[0], order[-3]
    assert len(want[small.name][0]) < len(want[big.name][0]) and small.n <= big.n
    cap_rows = len(want[big.name][0]) + 5
    out = torch.full((cap_rows, big.n), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    for p in (big, small):
        say(f"noalloc: {p.name} ({p.n} vertices) into a {cap_rows} x {big.n} buffer")
        rows_w, total_w = want[p.name]
        o = torch.full((cap_rows, p.n), -7, dtype=torch.int32, device="cuda") if p is small else out
        torch.cuda.synchronize()
        c0, m0 = al.calls, torch.cuda.memory_allocated()
        rows, total, _ = dg.enumerate_noalloc(p.n, p.edges, o.data_ptr(), cap_rows)
        torch.cuda.synchronize()
        assert al.calls == c0 and torch.cuda.memory_allocated() == m0, "the call allocated device memory"
        got = o[:rows].cpu().numpy()
        assert rows == total == total_w and np.array_equal(got, rows_w), p.name
        assert (o[rows:].cpu().numpy() == -7).all(), "rows past the result were written"
        oracle_rows, _ = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
        assert np.array_equal(got, oracle_rows), p.name

    say("noalloc: capped, count+hash, count-only")
    cap = 17
    rows, total, _ = dg.enumerate_noalloc(big.n, big.edges, out.data_ptr(), cap_rows, cap)
    assert rows == min(cap, total_w := want[big.name][1]) and total == total_w
    assert np.array_equal(out[:rows].cpu().numpy(), want[big.name][0][:cap])
    rows, total, hh = dg.enumerate_noalloc(big.n, big.edges, 0, 0, mode=dm.OUT_COUNT_HASH)
    assert rows == 0 and (total,) + hh == oracle.count_hash(g.n, g.edges, big.n, big.edges)
    rows, total, _ = dg.enumerate_noalloc(small.n, small.edges, 0, 0)
    assert rows == 0 and total == want[small.name][1]

    say("noalloc: a destination one row short")
    n_small = len(want[small.name][0])
    if n_small > 1:
        short = torch.zeros((n_small - 1, small.n), dtype=torch.int32, device="cuda")
        with pytest.raises(dm.DMError) as ei:
            dg.enumerate_noalloc(small.n, small.edges, short.data_ptr(), n_small - 1)
        assert ei.value.code == BUDGET
    say("noalloc: HH(90,90) P16 (tables beyond the scratch), then HH(28,28) P16 (fits)")
    p16 = W.path(16)
    g90 = W.heavy_hex(90, 90)
    dg90 = ctx.datagraph(g90.n, g90.edges)
    c0 = al.calls
    with pytest.raises(dm.DMError) as ei:
        dg90.enumerate_noalloc(p16.n, p16.edges, 0, 0)
    assert ei.value.code == BUDGET and al.calls == c0
    dg90.free()
    g28 = W.heavy_hex(28, 28)
    dg28 = ctx.datagraph(g28.n, g28.edges)
    rows_w, total_w = plain_rows(dg28, p16)
    buf = torch.empty((total_w, p16.n), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    c0 = al.calls
    rows, total, _ = dg28.enumerate_noalloc(p16.n, p16.edges, buf.data_ptr(), total_w)
    assert al.calls == c0 and rows == total == total_w
    assert np.array_equal(buf.cpu().numpy(), rows_w)
    dg28.free()
    # every entry point still works after the allocation-free calls
    for p in (big, small):
        assert np.array_equal(plain_rows(dg, p)[0], want[p.name][0])
    dg.free()
    ctx.close()
    torch.cuda.synchronize()
    assert not al.live
