"""A host model of the persistent join kernel's protocol, run on the CPU.

The batched form runs every (pattern, step, tile) of a batch in one launch:
workgroups poll per-pattern stage words, claim tiles with an atomic ticket per
step, publish a tile aggregate and wait on their predecessors (decoupled
look-back), and the workgroup that finishes a step's last tile publishes the
next step or retires the pattern; everyone leaves once every pattern has
retired.  This model replays that protocol with one atomic action per
scheduler tick under random interleavings of many workgroups, so that
termination and the accounting can be checked exhaustively on the host:

* every schedule of every random batch ends with all patterns retired, each
  tile claimed and finished exactly once, each look-back ending with the
  exact exclusive prefix of its tile;
* a planted protocol mistake (a step published with no tiles, or a tile that
  never publishes its look-back word) is caught by the bounded waits of the
  kernel: the model's workgroups give up after a fixed number of polls
  without progress, record the stuck (pattern, step) and leave, instead of
  polling forever.

The model follows the kernel's rules, not its code: a stage becomes
claimable only after its tile count is set; claims beyond the count are
wasted; a look-back waits only on tiles claimed earlier, which running
workgroups hold.  The per-workgroup loop of the sort tiers has no
inter-workgroup wait (barriers only, on block-uniform conditions), so it has
no counterpart here."""
import random

import pytest


class Batch:
    def __init__(self, rng, n_patterns, plant=None):
        self.n = n_patterns
        self.nsteps = [rng.randint(1, 6) for _ in range(n_patterns)]
        # rows of every step's output (>= 1 so that the next step has input;
        # a pattern whose step produces nothing retires early)
        self.rows = [[rng.choice([0] + [rng.randint(1, 40)] * 6) for _ in range(s)] for s in self.nsteps]
        self.block = 8
        self.stage = [0] * n_patterns
        self.ntiles = [[0] * (s + 1) for s in self.nsteps]
        self.claim = [[0] * (s + 1) for s in self.nsteps]
        self.done = [[0] * (s + 1) for s in self.nsteps]
        self.status = {}  # (p, s, tile) -> (flag, value)
        self.agg = {}     # (p, s, tile) -> the tile's own count (random)
        self.finished = 0
        self.tiles_done = 0
        self.abort = None
        self.plant = plant
        self.rng = rng
        for p in range(n_patterns):
            self.ntiles[p][0] = rng.randint(1, 5)

    def tile_count(self, p, s):
        return self.agg.setdefault((p, s, None), None)


def workgroup(b, wid, limit, log):
    """One workgroup as a generator: each `yield` is one atomic action."""
    rot = wid % b.n
    while True:
        # ---- find a claimable tile
        got = None
        polls, last_prog = 0, None
        while got is None:
            if b.abort is not None:
                return
            for i in range(b.n):
                q = (rot + i) % b.n
                st = b.stage[q]
                yield
                if st >= b.nsteps[q]:
                    continue
                nt = b.ntiles[q][st]
                yield
                if b.claim[q][st] >= nt:
                    continue
                t = b.claim[q][st]
                b.claim[q][st] += 1  # one atomic add
                yield
                if t < nt:
                    got = (q, st, t, nt)
                    break
            if got is not None:
                break
            if b.finished >= b.n:
                return
            yield
            # bounded idle wait: progress = some tile finishing anywhere
            if last_prog != b.tiles_done:
                last_prog, polls = b.tiles_done, 0
            else:
                polls += 1
                if polls > limit:
                    stuck = next(q for q in range(b.n) if b.stage[q] < b.nsteps[q])
                    b.abort = ("idle", stuck, b.stage[stuck])
                    return
        p, s, tile, nt = got
        rot = (p + 1) % b.n
        # ---- the tile: aggregate, then look-back over predecessors
        my = b.rng.randint(0, 9)
        b.agg[(p, s, tile)] = my
        if not (b.plant == "silent tile" and (p, s, tile) == (0, 0, 1)):
            b.status[(p, s, tile)] = (1, my)
        yield
        excl, j, spins = 0, tile - 1, 0
        while j >= 0:
            w = b.status.get((p, s, j))
            yield
            if w is None:
                spins += 1
                if b.abort is not None:
                    return
                if spins > limit:
                    b.abort = ("look-back", p, s, tile)
                    return
                continue
            flag, val = w
            excl += val
            if flag == 2:
                break
            j -= 1
        if not (b.plant == "silent tile" and (p, s, tile) == (0, 0, 1)):
            b.status[(p, s, tile)] = (2, excl + my)
        log.append((p, s, tile, excl))
        yield
        # ---- completion: the last tile of a step publishes the next one
        b.done[p][s] += 1
        b.tiles_done += 1
        d = b.done[p][s]
        yield
        if d == nt:
            out = sum(b.agg[(p, s, t)] for t in range(nt)) if b.rows[p][s] else 0
            if s + 1 < b.nsteps[p] and out > 0:
                ntl = (out + b.block - 1) // b.block
                if b.plant == "empty stage" and p == 0:
                    ntl = 0
                b.ntiles[p][s + 1] = ntl
                yield
                b.stage[p] = s + 1
            else:
                b.stage[p] = b.nsteps[p]
                b.finished += 1
            yield


def run(seed, n_patterns, n_wg, plant=None, limit=400, max_ticks=2_000_000):
    rng = random.Random(seed)
    b = Batch(rng, n_patterns, plant)
    log = []
    wgs = {w: workgroup(b, w, limit, log) for w in range(n_wg)}
    ticks = 0
    while wgs:
        w = rng.choice(list(wgs))
        try:
            next(wgs[w])
        except StopIteration:
            del wgs[w]
        ticks += 1
        assert ticks < max_ticks, "the model did not terminate"
    return b, log


@pytest.mark.parametrize("seed", range(40))
def test_protocol_terminates_and_accounts(seed):
    n_patterns = 1 + seed % 9
    n_wg = 1 + (seed * 7) % 13
    b, log = run(seed, n_patterns, n_wg)
    assert b.abort is None, b.abort
    assert b.finished == b.n
    assert all(b.stage[p] == b.nsteps[p] for p in range(b.n))
    for p in range(b.n):
        for s in range(b.nsteps[p]):
            if b.ntiles[p][s]:
                # every tile claimed (extra claims are wasted) and finished once
                assert b.claim[p][s] >= b.ntiles[p][s]
                assert b.done[p][s] == b.ntiles[p][s]
    seen = set()
    for p, s, tile, excl in log:
        assert (p, s, tile) not in seen
        seen.add((p, s, tile))
        assert excl == sum(b.agg[(p, s, t)] for t in range(tile)), (p, s, tile)


@pytest.mark.parametrize("plant", ["empty stage", "silent tile"])
def test_bounded_waits_catch_a_stuck_step(plant):
    for seed in range(10):
        rng = random.Random(seed)
        b, _ = run(seed, 3, 6, plant=plant)
        if plant == "empty stage" and b.stage[0] == b.nsteps[0] and b.abort is None:
            continue  # pattern 0 retired before its second step: the plant never fired
        if plant == "silent tile" and b.ntiles[0][0] < 2:
            assert b.abort is None
            continue
        assert b.abort is not None, (plant, seed)
        if plant == "empty stage":
            assert b.abort[0] == "idle" and b.abort[1] == 0, b.abort
        else:
            assert b.abort[:3] in (("look-back", 0, 0), ("idle", 0, 0)), b.abort
