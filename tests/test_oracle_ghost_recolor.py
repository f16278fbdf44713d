"""Pins of the oracle's tentative ghost recoloring (Section 3.2: a rank may
temporarily recolor ghosts in its recoloring step and restores their colors
afterwards; Section 3.4: with a second ghost layer the ghosts' recoloring
sees their whole neighbourhood)."""
import numpy as np
import pytest

import graphgen as gg
import oracle


def _sync_rounds(W, nbrs, color, keys):
    """Synchronous rounds over W: color(u) gives the committed color of a
    neighbour (0 = none); a vertex loses when a neighbour in W drew the same
    color with a greater key."""
    got = {}
    while W:
        T = {}
        for v in W:
            used = {got.get(u, color(u)) for u in nbrs(v)}
            t = 1
            while t in used:
                t += 1
            T[v] = t
        L = {v for v in W if any(u in W and T[u] == T[v] and keys[u] > keys[v] for u in nbrs(v))}
        for v in W - L:
            got[v] = T[v]
        W = L
    return got


def _step_twin(lg, keys):
    """One rank's step with tentative ghost recoloring, written with sets
    from the reading: ghost-blind phase 1; phase 2 uncolors the losing end of
    every equal-colored owned-ghost pair; phase 3 recolors owned losers and
    losing ghosts together on the local graph (a ghost's row: its row with
    two layers, its owned neighbours with one); ghosts are then restored."""
    no, m = lg.n_owned, lg.n_owned + lg.n_ghost
    rows = {v: set(lg.col[lg.row_ptr[v]:lg.row_ptr[v + 1]].tolist()) for v in range(len(lg.row_ptr) - 1)}
    if lg.layers == 1:
        for v in range(no):
            for u in rows[v]:
                if u >= no:
                    rows.setdefault(u, set()).add(v)
    nbrs = lambda v: rows.get(v, set())  # noqa: E731
    c1 = _sync_rounds(set(range(no)), lambda v: {u for u in nbrs(v) if u < no}, lambda u: 0, keys)
    C = [c1[v] for v in range(no)]
    gc = [int(x) for x in lg.ghost_colors]
    lose, glose = set(), set()
    for v in range(no):
        for u in nbrs(v):
            if u >= no and C[v] == gc[u - no]:
                (lose if keys[u] > keys[v] else glose).add(v if keys[u] > keys[v] else u)
    local = {v: (0 if v in lose else C[v]) for v in range(no)}
    local.update({u: (0 if u in glose else gc[u - no]) for u in range(no, m)})
    got = _sync_rounds(lose | glose, nbrs, lambda u: local[u], keys)
    return [got.get(v, local[v]) for v in range(no)], sorted(u - no for u in glose)


def _case(rng, layers):
    n = int(rng.integers(6, 22))
    g = gg.random_small_graph(n, float(rng.uniform(0.15, 0.6)), rng)
    parts = int(rng.integers(2, 4))
    owner = rng.integers(0, parts, n).astype(np.int32)
    owner[0] = 0
    gcol = rng.integers(1, 4, n).astype(np.int32)   # few colors: many conflicts
    return g, gg.ghost_local_graph(g, owner, 0, layers, gcol)


@pytest.mark.parametrize("layers", [1, 2])
def test_step_twin_agrees(layers):
    rng = np.random.default_rng(40 + layers)
    differ_fixed = recolored = 0
    for case in range(500):
        g, lg = _case(rng, layers)
        seed = int(rng.integers(1, 999))
        keys = {i: oracle.priority(int(x), seed) for i, x in enumerate(lg.gid)}
        r = oracle.color_d1_ghost(lg, seed=seed, ghost_recolor=True)
        C, glose = _step_twin(lg, keys)
        assert r.colors.tolist() == C, case
        assert np.nonzero(r.remote_loser)[0].tolist() == glose, case
        fixed = oracle.color_d1_ghost(lg, seed=seed)
        assert np.array_equal(fixed.remote_loser, r.remote_loser)
        if not glose:
            assert np.array_equal(fixed.colors, r.colors), case   # nothing to recolor tentatively
        else:
            recolored += 1
            differ_fixed += not np.array_equal(fixed.colors, r.colors)
    assert recolored > 100 and differ_fixed > 10


def test_second_layer_changes_the_result():
    """With ghosts recolored tentatively, their second-layer neighbours'
    colors matter, so two layers and one layer differ on some inputs (with
    fixed ghosts they never do)."""
    rng = np.random.default_rng(9)
    differ = 0
    for _ in range(300):
        n = int(rng.integers(8, 24))
        g = gg.random_small_graph(n, float(rng.uniform(0.15, 0.5)), rng)
        owner = rng.integers(0, 3, n).astype(np.int32)
        owner[0] = 0
        gcol = rng.integers(1, 4, n).astype(np.int32)
        l1 = gg.ghost_local_graph(g, owner, 0, 1, gcol)
        l2 = gg.ghost_local_graph(g, owner, 0, 2, gcol)
        a = oracle.color_d1_ghost(l1, seed=3, ghost_recolor=True)
        b = oracle.color_d1_ghost(l2, seed=3, ghost_recolor=True)
        assert np.array_equal(oracle.color_d1_ghost(l1, seed=3).colors, oracle.color_d1_ghost(l2, seed=3).colors)
        differ += not np.array_equal(a.colors, b.colors)
    assert differ > 5


@pytest.mark.parametrize("layers", [1, 2])
def test_invariants_on_larger_graphs(layers):
    g = gg.rmat(13, 8, 2)
    owner = gg.hash_partition(g.n, 4, 3)
    gcol = np.random.default_rng(1).integers(1, 6, g.n).astype(np.int32)
    lg = gg.ghost_local_graph(g, owner, 0, layers, gcol)
    r = oracle.color_d1_ghost(lg, seed=5, ghost_recolor=True)
    no = lg.n_owned
    C = r.colors
    assert np.all(C >= 1) and r.remote_losers > 0
    for v in range(no):
        nb = lg.col[lg.row_ptr[v]:lg.row_ptr[v + 1]]
        own, gh = nb[nb < no], nb[nb >= no] - no
        assert C[v] not in set(C[own].tolist())
        kept = gh[r.remote_loser[gh] == 0]            # ghosts whose owners keep their color
        assert C[v] not in set(lg.ghost_colors[kept].tolist())


def test_distributed_with_ghost_recoloring_is_proper():
    g = gg.rmat(14, 16, 4)
    owner = gg.hash_partition(g.n, 6, 2)
    zeros = np.zeros(g.n, np.int32)
    for layers in (1, 2):
        locs = [gg.ghost_local_graph(g, owner, p, layers, zeros) for p in range(6)]
        r = oracle.color_d1_distributed(locs, seed=4, ghost_recolor=True)
        C = np.zeros(g.n, np.int32)
        for lg, c in zip(locs, r.colors):
            C[lg.gid[:lg.n_owned]] = c
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        assert np.all(C[src] != C[g.col]) and r.conflicts[-1] == 0
