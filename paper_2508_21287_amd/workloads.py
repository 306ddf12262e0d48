"""Seeded synthetic workloads: data graphs, pattern graphs, circuit interaction
graphs and query traces.

This module only *describes inputs*. It holds none of the enumeration method's
arithmetic (no joins, no filters, no embedding logic), so that both the HIP
path and the CPU oracle can be fed from it without sharing any code with each
other. Every random draw uses numpy's PCG64 (`numpy.random.default_rng(seed)`).

Graphs are returned as ``(n_vertices, edges)`` with ``edges`` an ``int32``
array of shape ``[m, 2]`` of undirected pairs; vertex ids are ``0..n-1``.

Lattice families follow the paper's benchmark topologies (Sec. VI-A: heavy-hex
lattices with 1990/4485 vertices and square grids of 1600/3600 vertices):

* ``heavy_hex(R, C)``: ``R`` horizontal chains of ``C`` vertices; chain vertex
  ``(r, c)`` has id ``r*C + c``.  Between chains ``g`` and ``g+1`` there is a
  bridge vertex at every column ``c = 0, 4, 8, ...`` when ``g`` is even and
  ``c = 2, 6, 10, ...`` when ``g`` is odd; bridge ids are appended after the
  chain vertices in ``(g, c)`` order.  ``heavy_hex(n, n)`` has
  ``n**2 + (n-1)*n/4`` vertices for ``n`` divisible by 4: 1990 at ``n=40``
  and 4485 at ``n=60``, the two heavy-hex sizes of the paper's Table I.
* ``grid(a, b)``: the ``a x b`` square grid, id ``i*b + j``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "Pattern", "heavy_hex", "heavy_hex_cells", "grid", "path", "cycle",
    "star", "prufer_tree", "random_gnp", "lattice_subgraph_pattern",
    "circuit_pattern", "config1", "config2", "config3", "config4", "config5",
    "adjacency_lists", "max_degree",
]


@dataclass
class Graph:
    n: int
    edges: np.ndarray  # int32 [m, 2]
    name: str = ""

    def __post_init__(self):
        self.edges = np.ascontiguousarray(np.asarray(self.edges, dtype=np.int32).reshape(-1, 2))


@dataclass
class Pattern(Graph):
    planted: np.ndarray | None = None  # int32 [n]: a known embedding (lattice-grown patterns)
    seed: int | None = None
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------

def heavy_hex(R: int, C: int) -> Graph:
    """Heavy-hex lattice of ``R`` chains x ``C`` columns (see module doc)."""
    edges = []
    for r in range(R):
        for c in range(C - 1):
            edges.append((r * C + c, r * C + c + 1))
    nid = R * C
    for g in range(R - 1):
        start = 0 if g % 2 == 0 else 2
        for c in range(start, C, 4):
            edges.append((g * C + c, nid))
            edges.append((nid, (g + 1) * C + c))
            nid += 1
    return Graph(nid, np.array(edges, dtype=np.int32).reshape(-1, 2), f"HH({R},{C})")


def heavy_hex_cells(R: int, C: int) -> int:
    """Number of 12-vertex faces of ``heavy_hex(R, C)``: bridges - 1 per gap."""
    cells = 0
    for g in range(R - 1):
        start = 0 if g % 2 == 0 else 2
        nb = len(range(start, C, 4))
        cells += max(nb - 1, 0)
    return cells


def grid(a: int, b: int) -> Graph:
    edges = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                edges.append((v, v + 1))
            if i + 1 < a:
                edges.append((v, v + b))
    return Graph(a * b, np.array(edges, dtype=np.int32).reshape(-1, 2), f"GRID({a},{b})")


# ----------------------------------------------------------------------------
# fixed pattern shapes
# ----------------------------------------------------------------------------

def path(k: int) -> Pattern:
    e = [(i, i + 1) for i in range(k - 1)]
    return Pattern(k, np.array(e, dtype=np.int32).reshape(-1, 2), f"P{k}")


def cycle(k: int) -> Pattern:
    e = [(i, (i + 1) % k) for i in range(k)]
    return Pattern(k, np.array(e, dtype=np.int32).reshape(-1, 2), f"C{k}")


def star(r: int) -> Pattern:
    e = [(0, i) for i in range(1, r + 1)]
    return Pattern(r + 1, np.array(e, dtype=np.int32).reshape(-1, 2), f"K1,{r}")


def prufer_tree(k: int, seed: int) -> Pattern:
    """Tree on ``k`` labelled vertices from a seeded Pruefer code.

    The code is ``k-2`` draws from ``U{0..k-1}``; it is decoded with the
    smallest-leaf rule (repeatedly join the smallest current leaf to the next
    code symbol, then join the last two leaves)."""
    rng = np.random.default_rng(seed)
    if k == 1:
        return Pattern(1, np.zeros((0, 2), np.int32), f"T{k}s{seed}", seed=seed)
    if k == 2:
        return Pattern(2, np.array([[0, 1]], np.int32), f"T{k}s{seed}", seed=seed)
    code = rng.integers(0, k, size=k - 2).tolist()
    deg = [1] * k
    for x in code:
        deg[x] += 1
    edges = []
    for x in code:
        leaf = min(j for j in range(k) if deg[j] == 1)
        edges.append((leaf, x))
        deg[leaf] -= 1
        deg[x] -= 1
    last = [j for j in range(k) if deg[j] == 1]
    edges.append((last[0], last[1]))
    return Pattern(k, np.array(edges, dtype=np.int32), f"T{k}s{seed}", seed=seed)


def random_gnp(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) (used by the tiny brute-force cross-checks)."""
    rng = np.random.default_rng(seed)
    e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return Graph(n, np.array(e, dtype=np.int32).reshape(-1, 2), f"G({n},{p})s{seed}")


# ----------------------------------------------------------------------------
# helpers (input description only)
# ----------------------------------------------------------------------------

def adjacency_lists(g: Graph) -> list[list[int]]:
    adj: list[set[int]] = [set() for _ in range(g.n)]
    for u, v in g.edges.tolist():
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    return [sorted(s) for s in adj]


def max_degree(g: Graph) -> int:
    return max((len(a) for a in adjacency_lists(g)), default=0)


def _connected(k: int, edge_set: set) -> bool:
    if k <= 1:
        return True
    adj = [[] for _ in range(k)]
    for u, v in edge_set:
        adj[u].append(v)
        adj[v].append(u)
    seen = {0}
    st = [0]
    while st:
        u = st.pop()
        for w in adj[u]:
            if w not in seen:
                seen.add(w)
                st.append(w)
    return len(seen) == k


def _random_bfs(adj: list[list[int]], root: int, k: int, rng) -> list[int]:
    """Random BFS: the frontier is shuffled before every pop, each popped
    vertex's neighbours are visited in shuffled order; stops at ``k`` vertices."""
    order = [root]
    seen = {root}
    frontier = [root]
    while frontier and len(order) < k:
        rng.shuffle(frontier)
        u = frontier.pop()
        nb = list(adj[u])
        rng.shuffle(nb)
        for w in nb:
            if w not in seen and len(order) < k:
                seen.add(w)
                order.append(w)
                frontier.append(w)
    return order


def _relabel(order: list[int], edges: list[tuple[int, int]]):
    lab = {v: i for i, v in enumerate(order)}
    e = sorted((min(lab[u], lab[v]), max(lab[u], lab[v])) for u, v in edges)
    return np.array(e, dtype=np.int32).reshape(-1, 2), np.array(order, dtype=np.int32)


def lattice_subgraph_pattern(g: Graph, k: int, rng, thin: bool = True, adj=None) -> Pattern:
    """A connected subgraph of ``g`` with ``k`` vertices.

    Random BFS from a uniform root, induced subgraph on the visited vertices,
    then (``thin``) every edge is visited in random order and deleted with
    probability 1/2 unless it is a cut edge at that moment.  Vertices are
    relabelled ``0..k-1`` in BFS order; ``planted[i]`` is vertex ``i``'s
    lattice id, so the identity map is a known embedding."""
    adj = adj if adj is not None else adjacency_lists(g)
    root = int(rng.integers(0, g.n))
    order = _random_bfs(adj, root, k, rng)
    if len(order) < k:
        raise ValueError("lattice component smaller than the requested pattern")
    lab = {v: i for i, v in enumerate(order)}
    es = set()
    for v in order:
        for w in adj[v]:
            if w in lab and lab[v] < lab[w]:
                es.add((lab[v], lab[w]))
    if thin:
        elist = sorted(es)
        perm = rng.permutation(len(elist))
        for idx in perm.tolist():
            e = elist[idx]
            if rng.random() < 0.5:
                es.discard(e)
                if not _connected(k, es):
                    es.add(e)  # cut edge: keep it
    edges = np.array(sorted(es), dtype=np.int32).reshape(-1, 2)
    return Pattern(k, edges, f"sub{k}", planted=np.array(order, dtype=np.int32))


def lattice_tree_pattern(g: Graph, k: int, seed: int, adj=None) -> Pattern:
    """A random ``k``-vertex subtree of ``g``: random BFS from a uniform root
    (seeded), each visited vertex joined to the vertex it was discovered
    from.  Relabelled ``0..k-1`` in BFS order (``planted`` as for
    ``lattice_subgraph_pattern``)."""
    adj = adj if adj is not None else adjacency_lists(g)
    rng = np.random.default_rng(seed)
    root = int(rng.integers(0, g.n))
    order, parent = [root], {root: -1}
    frontier = [root]
    while frontier and len(order) < k:
        rng.shuffle(frontier)
        u = frontier.pop()
        nb = list(adj[u])
        rng.shuffle(nb)
        for w in nb:
            if w not in parent and len(order) < k:
                parent[w] = u
                order.append(w)
                frontier.append(w)
    if len(order) < k:
        raise ValueError("lattice component smaller than the requested tree")
    edges, planted = _relabel(order, [(parent[v], v) for v in order[1:]])
    return Pattern(k, edges, f"L{k}s{seed}", seed=seed, planted=planted)


def circuit_pattern(g: Graph, seed: int, k_lo: int = 4, k_hi: int = 40, adj=None) -> Pattern:
    """Interaction graph of a random two-qubit-gate circuit on a lattice
    subgraph: ``k = round(exp(U[ln k_lo, ln k_hi]))`` qubits, ``H`` a random-BFS
    connected induced subgraph on ``k`` lattice vertices, ``g ~ U{2..200}``
    gates raised to at least ``k-1``; the first ``k-1`` gates follow a random
    spanning tree of ``H`` (Kruskal over shuffled edges) so the circuit touches
    all ``k`` qubits, the rest are uniform over ``H``'s edges.  The pattern is
    the set of distinct gate pairs (connected, exactly ``k`` vertices)."""
    rng = np.random.default_rng(seed)
    adj = adj if adj is not None else adjacency_lists(g)
    k = int(round(math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))))
    k = max(k_lo, min(k_hi, k))
    root = int(rng.integers(0, g.n))
    order = _random_bfs(adj, root, k, rng)
    lab = {v: i for i, v in enumerate(order)}
    h_edges = sorted({(min(lab[v], lab[w]), max(lab[v], lab[w]))
                      for v in order for w in adj[v] if w in lab})
    n_gates = max(int(rng.integers(2, 201)), k - 1)
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    tree = []
    for idx in rng.permutation(len(h_edges)).tolist():
        u, v = h_edges[idx]
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[ru] = rv
            tree.append((u, v))
    gates = list(tree)
    for _ in range(n_gates - len(tree)):
        gates.append(h_edges[int(rng.integers(0, len(h_edges)))])
    es = sorted(set(gates))
    return Pattern(k, np.array(es, dtype=np.int32).reshape(-1, 2), f"circ{k}s{seed}",
                   planted=np.array(order, dtype=np.int32), seed=seed,
                   meta={"gates": n_gates})


# ----------------------------------------------------------------------------
# the five benchmark configurations
# ----------------------------------------------------------------------------

def config1():
    """Tiny: HH(3,9) (32 vertices, 34 edges); P6, C12 and a 6-vertex Pruefer tree."""
    g = heavy_hex(3, 9)
    pats = [path(6), cycle(12), prufer_tree(6, 0)]
    return g, pats


def config2(n_patterns: int = 64, k_lo: int = 8, k_hi: int = 30):
    """Device-scale: HH(7,19) (163 vertices, 186 edges) and 64 seeded
    connected thinned lattice subgraphs of 8..30 vertices (seeds 0..63)."""
    g = heavy_hex(7, 19)
    adj = adjacency_lists(g)
    pats = []
    for s in range(n_patterns):
        rng = np.random.default_rng(s)
        k = int(rng.integers(k_lo, k_hi + 1))
        p = lattice_subgraph_pattern(g, k, rng, thin=True, adj=adj)
        p.seed = s
        p.name = f"sub{k}s{s}"
        pats.append(p)
    return g, pats


def config3_lattices():
    return {
        "HH28": heavy_hex(28, 28), "HH56": heavy_hex(56, 56),
        "HH90": heavy_hex(90, 90), "GRID100": grid(100, 100),
    }


def config3(lattice: str, n_trees: int = 4):
    """Scaling: one of HH(28,28), HH(56,56), HH(90,90), GRID(100,100), with
    P8, P12, P16, C12, ``n_trees`` random 16-vertex trees and the 2x3 / 3x3
    grids.  On the grid the trees are uniformly random labelled trees
    (Pruefer codes; the first seeds whose maximum degree is at most 4).  A
    random labelled tree almost never fits a heavy-hex lattice (its degree-3
    vertices sit too close), so there the trees are random subtrees of the
    lattice (``lattice_tree_pattern``, seeds 0..n_trees-1)."""
    g = config3_lattices()[lattice]
    dmax = max_degree(g)
    pats = [path(8), path(12), path(16), cycle(12)]
    s = 0
    trees = []
    if lattice.startswith("HH"):
        adj = adjacency_lists(g)
        trees = [lattice_tree_pattern(g, 16, t, adj=adj) for t in range(n_trees)]
    while len(trees) < n_trees:
        t = prufer_tree(16, s)
        if max_degree(t) <= dmax:
            trees.append(t)
        s += 1
    g23 = grid(2, 3)
    g33 = grid(3, 3)
    pats += trees
    pats.append(Pattern(g23.n, g23.edges, "grid2x3"))
    pats.append(Pattern(g33.n, g33.edges, "grid3x3"))
    return g, pats


def config4(n_patterns: int = 256):
    """Batched: HH(28,28) (973 vertices) and 256 circuit interaction graphs of
    4..40 qubits (log-uniform), seeds 0..255."""
    g = heavy_hex(28, 28)
    adj = adjacency_lists(g)
    return g, [circuit_pattern(g, s, 4, 40, adj=adj) for s in range(n_patterns)]


def config5(rate: float, n_queries: int = 2000):
    """Served: HH(56,56) (3906 vertices); an open-loop Poisson trace of
    ``n_queries`` pattern queries at ``rate``/s (trace seed = rate).  Each
    query is a circuit pattern of 4..60 qubits and carries a cap drawn
    uniformly from {1, 1000, all(-1)}.  Returns ``(graph, arrivals_s,
    patterns, caps)``."""
    g = heavy_hex(56, 56)
    adj = adjacency_lists(g)
    rng = np.random.default_rng(int(rate))
    gaps = rng.exponential(1.0 / rate, size=n_queries)
    arrivals = np.cumsum(gaps)
    seeds = rng.integers(0, 2**31 - 1, size=n_queries)
    caps = rng.choice(np.array([1, 1000, -1], dtype=np.int64), size=n_queries)
    pats = [circuit_pattern(g, int(s), 4, 60, adj=adj) for s in seeds.tolist()]
    return g, arrivals, pats, caps
