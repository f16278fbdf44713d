"""Pins of the oracle's Algorithm 2 driver (Section 3: every rank colors its
local graph, ranks exchange boundary colors, detect conflicts with the key
rule of Algorithm 4, sum them over ranks, and recolor until none is left),
the ranks emulated one after another on the host."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle


def _locals(g, owner, parts, layers=1):
    zeros = np.zeros(g.n, np.int32)
    return [gg.ghost_local_graph(g, owner, p, layers, zeros) for p in range(parts)]


def _assemble(g, locs, r):
    C = np.zeros(g.n, np.int32)
    for p, lg in enumerate(locs):
        C[lg.gid[:lg.n_owned]] = r.colors[p]
    return C


def _rounds_sets(W, adj, colors_of, keys):
    """Synchronous rounds over the vertex set W: every vertex takes the
    smallest color absent from colors_of(u) of its neighbours; it loses when
    a neighbour in W drew the same color and has the greater key."""
    colors = {}
    while W:
        T = {}
        for v in W:
            used = {colors_of(u, colors) for u in adj[v]}
            t = 1
            while t in used:
                t += 1
            T[v] = t
        L = {v for v in W if any(u in W and T[u] == T[v] and keys[u] > keys[v] for u in adj[v])}
        for v in W - L:
            colors[v] = T[v]
        W = L
    return colors


def _alg2_twin(n, adj, owner, keys):
    """Algorithm 2 written with Python sets straight from Section 3 (an
    independent formulation for tiny graphs).  Returns the colors, the
    per-detection conflict sums and the per-exchange counts of ghost copies
    sent."""
    P = max(owner) + 1
    owned = [{v for v in range(n) if owner[v] == p} for p in range(P)]
    ghosts = [{u for v in owned[p] for u in adj[v] if owner[u] != p} for p in range(P)]
    C = [0] * n
    for p in range(P):   # ghost-blind initial coloring of each rank's owned vertices
        got = _rounds_sets(set(owned[p]), [[u for u in adj[v] if owner[u] == owner[v]] for v in range(n)],
                           lambda u, cur: cur.get(u, 0), keys)
        for v, c in got.items():
            C[v] = c
    sent = [sum(len(gs) for gs in ghosts)]
    gc = list(C)          # the colors the ranks hold for ghost copies
    trace = []
    while True:
        total = 0
        newC = list(C)
        for p in range(P):
            losers = set()
            for v in owned[p]:
                for u in adj[v]:
                    if owner[u] != p and gc[u] == C[v]:
                        total += 1
                        if keys[u] > keys[v]:
                            losers.add(v)
            mine = {v: (0 if v in losers else C[v]) for v in owned[p]}
            got = _rounds_sets(losers, adj,
                               lambda u, cur, p=p, mine=mine: cur.get(u, mine[u]) if owner[u] == p else gc[u], keys)
            for v in owned[p]:
                newC[v] = got.get(v, mine[v])
        trace.append(total)
        C = newC
        if total == 0:
            break
        sent.append(sum(1 for p in range(P) for u in ghosts[p] if C[u] != gc[u]))
        gc = list(C)
    return C, trace, sent


def test_twin_agrees_on_small_graphs_and_partitions():
    """Random graphs of up to 12 vertices, 2 to 4 ranks, random priorities:
    colors, conflict sums per detection and ghost copies sent per exchange."""
    rng = np.random.default_rng(21)
    multi = 0
    for case in range(400):
        n = int(rng.integers(2, 13))
        g = gg.random_small_graph(n, float(rng.uniform(0.15, 0.8)), rng)
        P = int(rng.integers(2, 5))
        owner = rng.integers(0, P, n).astype(np.int32)
        owner[:P] = np.arange(P)[:min(P, n)] if n >= P else owner[:P]
        P = int(owner.max()) + 1
        seed = int(rng.integers(1, 1000))
        locs = _locals(g, owner, P)
        r = oracle.color_d1_distributed(locs, seed=seed)
        keys = [oracle.priority(v, seed) for v in range(n)]
        adj = [list(g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(n)]
        C, trace, sent = _alg2_twin(n, adj, owner.tolist(), keys)
        assert _assemble(g, locs, r).tolist() == C, case
        assert r.conflicts == trace and r.exchanged == sent, case
        multi += len(trace) > 2
    assert multi > 10   # many cases needed more than one recoloring


def test_one_rank_is_the_plain_method():
    g = gg.rmat(12, 8, 4)
    locs = _locals(g, np.zeros(g.n, np.int32), 1)
    r = oracle.color_d1_distributed(locs, seed=3)
    assert np.array_equal(_assemble(g, locs, r), oracle.color_d1(g, seed=3).colors)
    assert r.conflicts == [0] and r.iterations == 0


@pytest.mark.parametrize("make,parts", [(lambda: gg.rmat(14, 16, 2), 8), (lambda: gg.erdos_renyi(6000, 20, 3), 5),
                                        (lambda: gg.stencil((24, 24, 24), 27), 4)])
@pytest.mark.parametrize("degrees", [False, True])
def test_final_coloring_is_proper_and_first_detect_counts_cut_edges(make, parts, degrees):
    g = make()
    owner = gg.hash_partition(g.n, parts, 5)
    locs = _locals(g, owner, parts)
    deg = g.degrees()
    gdeg = [deg[lg.gid[lg.n_owned:]].astype(np.int32) for lg in locs]
    r = oracle.color_d1_distributed(locs, seed=7, recolor_degrees=degrees, ghost_degrees=gdeg)
    C = _assemble(g, locs, r)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert np.all(C >= 1) and np.all(C[src] != C[g.col])
    assert r.conflicts[-1] == 0 and all(c > 0 for c in r.conflicts[:-1])
    # the first detection sees the ranks' ghost-blind colorings: every cut
    # edge whose ends got the same color, counted once from each side
    C0 = np.zeros(g.n, np.int32)
    for p, lg in enumerate(locs):
        no = lg.n_owned
        s = np.repeat(np.arange(no), np.diff(lg.row_ptr))
        keep = lg.col < no
        sub = gg.csr_from_pairs(no, s[keep], lg.col[keep], True)
        pr = np.array([oracle.priority(int(x), 7) for x in lg.gid[:no]], dtype=np.uint32)
        if degrees:   # the degree key, as ranks: (degree, priority)
            d = deg[lg.gid[:no]].astype(np.int64)
            pr = np.lexsort((pr.astype(np.int64), d)).argsort().astype(np.uint32)
        C0[lg.gid[:no]] = oracle.color_d1(sub, prio=pr).colors
    cut = owner[src] != owner[g.col]
    assert r.conflicts[0] == int(np.count_nonzero(cut & (C0[src] == C0[g.col])))
    assert r.exchanged[0] == sum(lg.n_ghost for lg in locs)
