"""Control paths of the C ABI on the GPU: the context's cancel word, the
bound on device-side waits, the caller's device allocator with injected
failures, and the data graph held by a server.

Every case ends with a normal call whose result is compared with the oracle,
so a path that leaves the device or the context in a bad state fails here.
No case makes a kernel fault or hang: cancelling and the wait bound are set
from the host, and every kernel still leaves its loops normally."""
import sys

import numpy as np
import pytest

import oracle
import paper_2508_21287_amd as dm
from paper_2508_21287_amd import workloads as W

pytestmark = pytest.mark.gpu

CANCELLED, DEVICE, OOM, BUSY = -8, -7, -5, -9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_batch(dg, g, pats):
    res = dg.enumerate_batch([(p.n, p.edges) for p in pats])
    for p, r in zip(pats, res):
        want, total = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
        assert r.total == total and np.array_equal(r.to_numpy(), want), p.name
        r.free()


@pytest.fixture(scope="module")
def ctx():
    c = dm.Context(0)
    yield c
    c.close()


def test_cancel_word(ctx):
    g, pats = W.config2(16)
    dg = ctx.datagraph(g.n, g.edges)
    specs = [(p.n, p.edges) for p in pats]
    ctx.cancel(True)
    try:
        say("cancel: batched call with the cancel word set (the persistent kernel leaves at its start)")
        with pytest.raises(dm.DMError) as ei:
            dg.enumerate_batch(specs)
        assert ei.value.code == CANCELLED, ei.value
        say("cancel: plain call with the cancel word set")
        with pytest.raises(dm.DMError) as ei:
            dg.enumerate(pats[0].n, pats[0].edges)
        assert ei.value.code == CANCELLED
    finally:
        ctx.cancel(False)
    say("cancel: cleared, batch against the oracle")
    check_batch(dg, g, pats)
    dg.free()


def test_wait_limit_gives_up(ctx):
    # A 1 us bound on a batch of one 16-vertex path: each of its 15 steps has
    # a single tile, so while one workgroup runs it every other one polls
    # for work with no tile finishing for microseconds; they give up, record
    # the wait and leave, and the call fails with DM_ERR_DEVICE naming it.
    g, pats = W.config2(64)
    dg = ctx.datagraph(g.n, g.edges)
    specs = [(p.n, p.edges) for p in pats]
    p16 = W.path(16)
    say("wait limit: batched call with a 1 us bound")
    with pytest.raises(dm.DMError) as ei:
        dg.enumerate_batch([(p16.n, p16.edges)], wait_limit_us=1, motif_mask=dm.MOTIF_M2_ONLY)
    assert ei.value.code == DEVICE, ei.value
    msg = str(ei.value)
    assert "persistent scheduler" in msg or "look-back" in msg, msg
    say(f"wait limit: gave up as expected: {msg}")
    say("wait limit: default bound, batch against the oracle")
    check_batch(dg, g, pats)
    dg.free()


class CountingAllocator:
    """Device memory from torch's caching allocator; the k-th call from
    `fail_at` on returns NULL once."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_at = -1
        self.failed = 0

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.calls == self.fail_at:
            self.failed += 1
            return 0
        p = self.torch.cuda.caching_allocator_alloc(nbytes, 0, stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, stream):
        assert ptr in self.live, "free of a pointer the allocator did not hand out"
        del self.live[ptr]
        self.torch.cuda.caching_allocator_delete(ptr)


def test_allocator_failure_injection():
    import torch
    torch.cuda.set_device(0)
    al = CountingAllocator()
    c = dm.Context(0, allocator=(al.alloc, al.free))
    g, pats = W.config2(8)
    dg = c.datagraph(g.n, g.edges)
    assert al.calls > 0 and len(al.live) > 0, "the data graph did not come from the allocator"
    specs = [(p.n, p.edges) for p in pats]
    check_batch(dg, g, pats)
    # fail the k-th allocation of a batched call, for every k it makes
    base = al.calls
    check_batch(dg, g, pats)
    per_call = al.calls - base
    say(f"allocator: a batched call takes {per_call} allocations")
    failures = 0
    for k in range(1, per_call + 2):
        al.fail_at = al.calls + k
        try:
            res = dg.enumerate_batch(specs)
            dm.free_results(res)
        except dm.DMError as e:
            assert e.code == OOM, e
            failures += 1
        al.fail_at = -1
        check_batch(dg, g, pats)  # the context is still usable
    assert failures >= 1
    # a failure inside the build of a data graph leaves nothing behind
    before = set(al.live)
    al.fail_at = al.calls + 3
    with pytest.raises(dm.DMError) as ei:
        c.datagraph(g.n, g.edges)
    assert ei.value.code == OOM
    al.fail_at = -1
    torch.cuda.synchronize()
    assert set(al.live) == before, "a failed build kept device memory"
    # served queries whose allocations fail report it through wait
    srv = dm.Server(dg, n_streams=2, max_batch=4)
    al.fail_at = al.calls + 1
    t = srv.submit(pats[0].n, pats[0].edges)
    try:
        srv.wait(t, 60000).free()
    except dm.DMError as e:
        assert e.code == OOM, e
    al.fail_at = -1
    t = srv.submit(pats[1].n, pats[1].edges)
    r = srv.wait(t, 60000)
    want, _ = oracle.enumerate_embeddings(g.n, g.edges, pats[1].n, pats[1].edges)
    assert np.array_equal(r.to_numpy(), want)
    r.free()
    srv.stop()
    dg.free()
    c.close()
    torch.cuda.synchronize()
    assert not al.live, f"{len(al.live)} device allocations outlived the context"


def test_served_result_outlives_server(ctx):
    g, pats = W.config2(6)
    dg = ctx.datagraph(g.n, g.edges)
    srv = dm.Server(dg, n_streams=2, max_batch=3)
    tickets = [srv.submit(p.n, p.edges) for p in pats]
    results = [srv.wait(t, 60000) for t in tickets]
    srv.stop()  # destroys the worker streams; the results stay readable
    for p, r in zip(pats, results):
        want, _ = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
        assert np.array_equal(r.to_numpy(), want), p.name
        r.free()
    dg.free()


def test_datagraph_busy_while_served(ctx):
    g, pats = W.config2(2)
    dg = ctx.datagraph(g.n, g.edges)
    srv = dm.Server(dg)
    with pytest.raises(dm.DMError) as ei:
        dg.free()
    assert ei.value.code == BUSY
    with pytest.raises(dm.DMError) as ei:
        dg.set_costs(np.zeros(g.n, np.uint32))
    assert ei.value.code == BUSY
    # the owning thread may still enumerate on it beside the server
    t = srv.submit(pats[0].n, pats[0].edges)
    with dg.enumerate(pats[1].n, pats[1].edges) as r:
        want, _ = oracle.enumerate_embeddings(g.n, g.edges, pats[1].n, pats[1].edges)
        assert np.array_equal(r.to_numpy(), want)
    srv.wait(t, 60000).free()
    srv.stop()
    dg.free()


def test_server_wait_any(ctx):
    # completions collected in completion order with one blocking call each;
    # a ticket taken by wait() first is passed over by wait_any()
    g, pats = W.config2(10)
    dg = ctx.datagraph(g.n, g.edges)
    srv = dm.Server(dg, n_streams=2, max_batch=4)
    tickets = {srv.submit(p.n, p.edges): p for p in pats}
    first = next(iter(tickets))
    r0 = srv.wait(first, 60000)
    want, _ = oracle.enumerate_embeddings(g.n, g.edges, tickets[first].n, tickets[first].edges)
    assert np.array_equal(r0.to_numpy(), want)
    r0.free()
    seen = {first}
    while len(seen) < len(tickets):
        t, r, code = srv.wait_any(60000)
        assert code == 0 and t in tickets and t not in seen, (t, code)
        seen.add(t)
        p = tickets[t]
        want, total = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
        assert r.total == total and np.array_equal(r.to_numpy(), want), p.name
        r.free()
    with pytest.raises(dm.DMError) as ei:
        srv.wait_any(0)
    assert ei.value.code == -10  # DM_ERR_TIMEOUT: nothing left
    srv.stop()
    dg.free()
