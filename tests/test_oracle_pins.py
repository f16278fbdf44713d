"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests re-types the oracle's own round loop: they check closed
forms, the hand-worked fixture in tests/golden, published hash vectors,
reductions to independently built graphs (scipy sparse products), properness
and first-fit (Grundy) certificates, brute-force chromatic numbers and
textbook graphs with known chromatic number.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _adj_sets(g):
    return [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]


def _square(g):
    """G^2 built with a sparse matrix product (independent of the oracle's walk)."""
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    a2 = (a + a @ a).tocoo()
    keep = a2.row != a2.col
    return gg.csr_from_pairs(g.n, a2.row[keep], a2.col[keep], True)


def _column_intersection(b):
    a = sp.csr_matrix((np.ones(b.nnz), b.col_idx, b.row_ptr), shape=(b.n_rows, b.n_cols))
    c = (a.T @ a).tocoo()
    keep = c.row != c.col
    return gg.csr_from_pairs(b.n_cols, c.row[keep], c.col[keep], True)


def _ranks_desc(keys):
    """rank[v] = 1 + number of vertices with a greater key."""
    keys = np.asarray(keys, dtype=np.int64)
    return np.array([1 + int(np.sum(keys > k)) for k in keys])


# --------------------------------------------------------------------------
# hash
# --------------------------------------------------------------------------

def test_fmix32_published_vectors():
    with open(os.path.join(GOLDEN, "murmur3_fmix32.json")) as f:
        vec = json.load(f)["vectors"]
    for x, h in vec:
        assert oracle.fmix32(x) == h


def _unfmix32(h):
    """Inverse of the MurmurHash3 finalizer: undo each xor-shift and multiply
    (multiplicative inverses computed here, mod 2^32)."""
    m = 0xFFFFFFFF
    def unxorshift(x, s):
        y = x
        for _ in range(32 // s + 1):
            y = x ^ (y >> s)
        return y & m
    h = unxorshift(h, 16)
    h = (h * pow(0xC2B2AE35, -1, 1 << 32)) & m
    h = unxorshift(h, 13)
    h = (h * pow(0x85EBCA6B, -1, 1 << 32)) & m
    return unxorshift(h, 16)


def test_fmix32_is_inverted_by_independent_inverse():
    rng = np.random.default_rng(5)
    for x in rng.integers(0, 1 << 32, size=200, dtype=np.uint64).tolist() + [0, 1, 0xFFFFFFFF]:
        assert _unfmix32(oracle.fmix32(x)) == x


def test_priority_is_a_bijection_per_seed():
    for seed in (0, 1, 12345):
        s = oracle.fmix32(seed ^ 0x9E3779B9)
        ids = list(range(2000))
        p = [oracle.priority(i, seed) for i in ids]
        assert len(set(p)) == len(p)
        # the priority is fmix32 of (gid xor a per-seed constant): inverting
        # fmix32 must give back gid xor the same constant for every gid
        assert {(_unfmix32(pi) ^ i) for i, pi in zip(ids, p)} == {s}


# --------------------------------------------------------------------------
# closed forms (D1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_complete_graph_ranks(n):
    g = gg.complete(n)
    rng = np.random.default_rng(n)
    prio = rng.permutation(n).astype(np.uint32) + 10
    r = oracle.color_d1(g, prio=prio)
    assert np.array_equal(r.colors, _ranks_desc(prio))
    assert r.rounds == n and r.num_colors == n
    # with the hash priority the same holds for the hashed keys
    r2 = oracle.color_d1(g, seed=7)
    keys = [oracle.priority(v, 7) for v in range(n)]
    assert np.array_equal(r2.colors, _ranks_desc(keys))


def test_complete_graph_equal_priorities_break_ties_by_id():
    g = gg.complete(5)
    r = oracle.color_d1(g, prio=np.full(5, 3, np.uint32))
    # equal p: the higher id has the higher key, so id 4 keeps color 1
    assert r.colors.tolist() == [5, 4, 3, 2, 1]


def test_matching():
    g = gg.matching(50)
    rng = np.random.default_rng(1)
    prio = rng.permutation(100).astype(np.uint32)
    r = oracle.color_d1(g, prio=prio)
    for i in range(50):
        a, b = 2 * i, 2 * i + 1
        hi, lo = (a, b) if prio[a] > prio[b] else (b, a)
        assert r.colors[hi] == 1 and r.colors[lo] == 2
    assert r.rounds == 2


@pytest.mark.parametrize("n", [2, 3, 4, 9, 10])
def test_monotone_path(n):
    g = gg.path(n)
    prio = np.arange(n, 0, -1).astype(np.uint32)
    r = oracle.color_d1(g, prio=prio)
    assert r.colors.tolist() == [1 + (i % 2) for i in range(n)]
    assert r.rounds == 1 + (n - 1 + 1) // 2
    # forced order: equals serial greedy in descending key order (Algorithm 1)
    assert np.array_equal(r.colors, oracle.serial_greedy(g, np.argsort(-prio.astype(np.int64))))


@pytest.mark.parametrize("center_high", [True, False])
def test_star(center_high):
    m = 9
    g = gg.star(m)
    prio = np.arange(1, m + 2, dtype=np.uint32)
    if center_high:
        prio[0] = 100
    else:
        prio[0] = 0
    r = oracle.color_d1(g, prio=prio)
    if center_high:
        assert r.colors[0] == 1 and np.all(r.colors[1:] == 2)
    else:
        assert r.colors[0] == 2 and np.all(r.colors[1:] == 1)
    assert r.rounds == 2
    assert np.array_equal(r.colors, oracle.serial_greedy(g, np.argsort(-prio.astype(np.int64))))


def test_edgeless():
    g = gg.csr_from_pairs(12, np.array([], np.int64), np.array([], np.int64))
    r = oracle.color_d1(g, seed=3)
    assert np.all(r.colors == 1) and r.rounds == 1


def test_empty_graph():
    g = gg.csr_from_pairs(0, np.array([], np.int64), np.array([], np.int64))
    r = oracle.color_d1(g, seed=3)
    assert r.colors.size == 0 and r.rounds == 0 and r.num_colors == 0


def test_golden_path_sync_differs_from_serial():
    with open(os.path.join(GOLDEN, "path6_sync_vs_serial.json")) as f:
        fx = json.load(f)
    g = gg.from_edge_list(fx["n"], fx["edges"])
    r = oracle.color_d1(g, prio=np.array(fx["prio"], np.uint32))
    assert r.colors.tolist() == fx["sync_colors"]
    assert r.rounds == fx["sync_rounds"]
    assert r.worklist == fx["sync_worklist"]
    assert oracle.serial_greedy(g, fx["serial_order"]).tolist() == fx["serial_colors"]


# --------------------------------------------------------------------------
# certificates on random graphs: proper, first-fit complete, bounds
# --------------------------------------------------------------------------

def _check_d1_certificate(g, r, prio=None, seed=1):
    adj = _adj_sets(g)
    c = r.colors
    assert np.all(c >= 1)
    for v in range(g.n):
        nb_colors = {int(c[u]) for u in adj[v]}
        assert int(c[v]) not in nb_colors                       # proper
        assert set(range(1, int(c[v]))) <= nb_colors            # Grundy / first-fit
        assert c[v] <= len(adj[v]) + 1                          # deg + 1 bound
    assert r.num_colors == int(c.max(initial=0))
    assert r.rounds >= r.num_colors                            # a round-r commit has color <= r
    # key-local maxima get color 1 in round 1
    keys = prio if prio is not None else np.array([oracle.priority(v, seed) for v in range(g.n)])
    for v in range(g.n):
        if all(keys[u] < keys[v] for u in adj[v]):
            assert c[v] == 1


@pytest.mark.parametrize("seed", range(6))
def test_random_graph_certificates(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 120))
    g = gg.random_small_graph(n, float(rng.uniform(0.02, 0.5)), rng)
    r = oracle.color_d1(g, seed=seed)
    _check_d1_certificate(g, r, seed=seed)
    assert r.vertex_visits == sum(r.worklist)
    assert r.worklist[0] == n


def test_er_config_certificate():
    g = gg.erdos_renyi(10000, 16, 1)
    r = oracle.color_d1(g, seed=1)
    _check_d1_certificate(g, r, seed=1)


def _dense_twin_d1(a, keys):
    """Synchronous rounds written with dense boolean matrices (an independent
    formulation, used only as a cross-check of the C loop on small graphs)."""
    n = a.shape[0]
    C = np.zeros(n, dtype=np.int64)
    W = np.ones(n, dtype=bool)
    rounds = 0
    big = np.iinfo(np.int64).max
    while W.any():
        rounds += 1
        nbc = np.where(a, C[None, :], 0)
        T = np.zeros(n, dtype=np.int64)
        for v in np.nonzero(W)[0]:
            used = set(nbc[v][a[v]].tolist())
            t = 1
            while t in used:
                t += 1
            T[v] = t
        Tm = np.where(W, T, -big)
        clash = a & (Tm[:, None] == Tm[None, :]) & W[None, :] & (keys[None, :] > keys[:, None])
        lose = W & clash.any(axis=1)
        C = np.where(W & ~lose, T, C)
        W = lose
    return C, rounds


@pytest.mark.parametrize("seed", range(8))
def test_dense_twin_agrees(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    g = gg.random_small_graph(n, float(rng.uniform(0.05, 0.7)), rng)
    prio = rng.permutation(n).astype(np.uint32)
    r = oracle.color_d1(g, prio=prio)
    C, rounds = _dense_twin_d1(gg.to_dense(g), prio.astype(np.int64))
    assert np.array_equal(r.colors, C) and r.rounds == rounds


def _sets_twin_d1(n, adj, keys):
    """The synchronous rounds written with Python sets, straight from the
    definition (a second, independent formulation for tiny graphs): every
    worklist vertex takes the smallest color absent from its neighbours'
    committed colors; it loses when a worklist neighbour drew the same color
    and has the greater key; winners commit."""
    C = [0] * n
    W = set(range(n))
    rounds = 0
    while W:
        rounds += 1
        T = {}
        for v in W:
            used = {C[u] for u in adj[v]}
            t = 1
            while t in used:
                t += 1
            T[v] = t
        L = {v for v in W if any(u in W and T[u] == T[v] and keys[u] > keys[v] for u in adj[v])}
        for v in W - L:
            C[v] = T[v]
        W = L
    return C, rounds


def test_all_graphs_up_to_five_vertices_all_orders():
    """Every labelled graph on 1..5 vertices under every priority order
    (1 + 2*2 + 8*6 + 64*24 + 1024*120 = 124,469 cases): the oracle equals the
    set-based twin; the result is a first-fit (Grundy) coloring; it equals
    serial greedy (Algorithm 1) in descending key order exactly where the
    order is forced, which differs in 240 of the cases."""
    cases = differ = 0
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            edges = [p for k, p in enumerate(pairs) if mask >> k & 1]
            g = gg.from_edge_list(n, edges)
            adj = [set() for _ in range(n)]
            for a, b in edges:
                adj[a].add(b)
                adj[b].add(a)
            for perm in itertools.permutations(range(n)):
                prio = np.array(perm, np.uint32)
                r = oracle.color_d1(g, prio=prio)
                C, rounds = _sets_twin_d1(n, adj, perm)
                assert r.colors.tolist() == C and r.rounds == rounds, (n, edges, perm)
                for v in range(n):
                    nb = {C[u] for u in adj[v]}
                    assert all(c in nb for c in range(1, C[v])), (n, edges, perm, v)
                order = np.argsort(-prio.astype(np.int64), kind="stable").astype(np.int32)
                differ += not np.array_equal(oracle.serial_greedy(g, order), r.colors)
                cases += 1
    assert cases == 124469
    assert differ == 240


# --------------------------------------------------------------------------
# lower bounds: brute-force chromatic number, Mycielski graphs
# --------------------------------------------------------------------------

def _chromatic_number(g):
    adj = _adj_sets(g)
    n = g.n
    for k in range(1, n + 1):
        col = [0] * n
        def bt(v):
            if v == n:
                return True
            for c in range(1, k + 1):
                if all(col[u] != c for u in adj[v] if u < v):
                    col[v] = c
                    if bt(v + 1):
                        return True
            col[v] = 0
            return False
        if bt(0):
            return k
    return 0


@pytest.mark.parametrize("seed", range(10))
def test_colors_at_least_chromatic_number(seed):
    rng = np.random.default_rng(seed + 50)
    g = gg.random_small_graph(int(rng.integers(3, 10)), float(rng.uniform(0.2, 0.8)), rng)
    r = oracle.color_d1(g, seed=seed)
    assert r.num_colors >= _chromatic_number(g)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
def test_mycielski_lower_bound(k):
    g = gg.mycielski(k)
    # triangle-free (the construction's defining property)
    a = gg.to_dense(g).astype(np.int64)
    assert np.trace(a @ a @ a) == 0
    if k <= 4:
        assert _chromatic_number(g) == k
    for seed in range(3):
        r = oracle.color_d1(g, seed=seed)
        assert r.num_colors >= k
        _check_d1_certificate(g, r, seed=seed)


def test_stencil_27pt_contains_k8():
    g = gg.stencil((6, 6, 6), 27)
    r = oracle.color_d1(g, seed=1)
    assert r.num_colors >= 8


# --------------------------------------------------------------------------
# distance-2 and partial distance-2: reductions to D1 on built graphs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_d2_equals_d1_of_square(seed):
    rng = np.random.default_rng(seed + 200)
    g = gg.random_small_graph(int(rng.integers(3, 80)), float(rng.uniform(0.02, 0.2)), rng)
    prio = rng.permutation(g.n).astype(np.uint32)
    r2 = oracle.color_d2(g, prio=prio)
    r1 = oracle.color_d1(_square(g), prio=prio)
    assert np.array_equal(r2.colors, r1.colors) and r2.rounds == r1.rounds
    # same with the hash priority
    assert np.array_equal(oracle.color_d2(g, seed=seed).colors,
                          oracle.color_d1(_square(g), seed=seed).colors)


def test_d2_stencil_reduction_and_bound():
    g = gg.stencil((7, 6, 5), 7)
    r = oracle.color_d2(g, seed=4)
    assert np.array_equal(r.colors, oracle.color_d1(_square(g), seed=4).colors)
    # closed neighbourhood of an interior vertex is a 7-clique of G^2
    assert r.num_colors >= 7


@pytest.mark.parametrize("m", [1, 3, 8])
def test_d2_star_ranks(m):
    g = gg.star(m)
    prio = np.random.default_rng(m).permutation(m + 1).astype(np.uint32)
    r = oracle.color_d2(g, prio=prio)
    assert np.array_equal(r.colors, _ranks_desc(prio))


def test_d2_proper_at_distance_two():
    rng = np.random.default_rng(9)
    g = gg.random_small_graph(60, 0.06, rng)
    r = oracle.color_d2(g, seed=2)
    a = gg.to_dense(g).astype(np.int64)
    reach = ((a + a @ a) > 0)
    np.fill_diagonal(reach, False)
    c = r.colors
    assert not np.any(reach & (c[:, None] == c[None, :]))


@pytest.mark.parametrize("seed", range(6))
def test_pd2_equals_d1_of_column_intersection(seed):
    rng = np.random.default_rng(seed + 300)
    nr, nc = int(rng.integers(1, 60)), int(rng.integers(1, 50))
    b = gg.bipartite_from_dense(rng.random((nr, nc)) < rng.uniform(0.02, 0.2))
    prio = rng.permutation(nc).astype(np.uint32)
    rp = oracle.color_pd2(b, prio=prio)
    r1 = oracle.color_d1(_column_intersection(b), prio=prio)
    assert np.array_equal(rp.colors, r1.colors) and rp.rounds == r1.rounds


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_pd2_single_row_ranks(k):
    a = np.ones((1, k), dtype=bool)
    b = gg.bipartite_from_dense(a)
    prio = np.random.default_rng(k).permutation(k).astype(np.uint32)
    r = oracle.color_pd2(b, prio=prio)
    assert np.array_equal(r.colors, _ranks_desc(prio))


def test_pd2_powerlaw_small_proper():
    b = gg.bipartite_powerlaw(2000, 500, 4, 2.1, seed=3)
    r = oracle.color_pd2(b, seed=1)
    c = r.colors
    for row in range(b.n_rows):
        cols = b.col_idx[b.row_ptr[row]:b.row_ptr[row + 1]]
        assert len(set(c[cols].tolist())) == cols.size
    assert np.array_equal(c, oracle.color_d1(_column_intersection(b), seed=1).colors)


# --------------------------------------------------------------------------
# work counters: edge_visits is the adjacency entries read per visit
# --------------------------------------------------------------------------

def _work_d1(g):
    return np.diff(g.row_ptr).astype(np.int64)


def _work_d2(g):
    """sum over u in N(v) of (1 + deg u): the hop-1 entry plus u's row."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    src = np.repeat(np.arange(g.n), deg)
    return np.bincount(src, weights=1 + deg[g.col], minlength=g.n).astype(np.int64)


def _work_pd2(b):
    """sum over the rows r of column c of (1 + deg r): the CSC entry plus the row."""
    rdeg = np.diff(b.row_ptr).astype(np.int64)
    cdeg = np.diff(b.col_ptr).astype(np.int64)
    src = np.repeat(np.arange(b.n_cols), cdeg)
    return np.bincount(src, weights=1 + rdeg[b.row_idx], minlength=b.n_cols).astype(np.int64)


@pytest.mark.parametrize("kind", ["d1", "d2", "pd2"])
def test_visit_counters_count_the_walk_of_every_round(kind):
    """Round by round, vertex_visits grows by the uncolored vertices and
    edge_visits by their work, counted here with numpy from the CSR/CSC
    alone (D2: each neighbour entry plus its row; PD2: each CSC entry plus
    the row's CSR entries).  The partial states come from the round cap."""
    if kind == "pd2":
        obj = gg.bipartite_powerlaw(3000, 800, 5, 2.1, seed=4)
        work, n, run = _work_pd2(obj), obj.n_cols, oracle.color_pd2
    else:
        obj = gg.erdos_renyi(1500, 9, 3)
        work, n = (_work_d1(obj) if kind == "d1" else _work_d2(obj)), obj.n
        run = oracle.color_d1 if kind == "d1" else oracle.color_d2
    full = run(obj, seed=2)
    assert full.vertex_visits == sum(full.worklist)
    prev_colors = np.zeros(n, dtype=np.int32)
    prev_v = prev_e = 0
    for k in range(1, full.rounds + 1):
        r = run(obj, seed=2, max_rounds=k)
        unc = prev_colors == 0
        assert r.vertex_visits - prev_v == int(unc.sum())
        assert r.edge_visits - prev_e == int(work[unc].sum()), f"round {k}"
        prev_colors, prev_v, prev_e = r.colors, r.vertex_visits, r.edge_visits
    assert (prev_v, prev_e) == (full.vertex_visits, full.edge_visits)
    # closed forms of one full pass: D2 nnz + sum deg^2, PD2 nnz + sum row-deg^2
    if kind == "d2":
        assert int(work.sum()) == obj.nnz + int((np.diff(obj.row_ptr).astype(np.int64) ** 2).sum())
    if kind == "pd2":
        assert int(work.sum()) == obj.nnz + int((np.diff(obj.row_ptr).astype(np.int64) ** 2).sum())


# --------------------------------------------------------------------------
# recolorDegrees (Section 3.3; Algorithm 4): key = (deg, p, gid)
# --------------------------------------------------------------------------

def test_golden_path_recolor_degrees():
    with open(os.path.join(GOLDEN, "path6_recolor_degrees.json")) as f:
        fx = json.load(f)
    g = gg.from_edge_list(fx["n"], fx["edges"])
    r = oracle.color_d1(g, prio=np.array(fx["prio"], np.uint32), recolor_degrees=True)
    assert r.colors.tolist() == fx["colors"]
    assert r.rounds == fx["rounds"] and r.worklist == fx["worklist"]


@pytest.mark.parametrize("m", [2, 3, 9])
def test_recolor_degrees_star_center_wins(m):
    """The center has the lowest priority but the highest degree: it keeps
    color 1 in round 1 and every leaf takes 2 in round 2 (without degrees
    the leaves take 1 and the center 2)."""
    g = gg.star(m)
    prio = np.arange(m + 1, dtype=np.uint32)[::-1].copy()   # vertex 0 (center) lowest
    prio[0] = 0
    r = oracle.color_d1(g, prio=prio, recolor_degrees=True)
    assert r.colors.tolist() == [1] + [2] * m and r.rounds == 2
    base = oracle.color_d1(g, prio=prio)
    assert base.colors.tolist() == [2] + [1] * m


@pytest.mark.parametrize("m,k", [(1, 3), (2, 5), (4, 7)])
def test_recolor_degrees_complete_bipartite(m, k):
    """K_{m,k} with m < k: the m-side has degree k > m, so whatever the
    priorities it keeps color 1 and the k-side takes 2, in two rounds."""
    edges = [(a, m + b) for a in range(m) for b in range(k)]
    g = gg.from_edge_list(m + k, edges)
    for seed in range(4):
        r = oracle.color_d1(g, seed=seed, recolor_degrees=True)
        assert r.colors.tolist() == [1] * m + [2] * k and r.rounds == 2


@pytest.mark.parametrize("make", [lambda: gg.complete(7), lambda: gg.cycle(31), lambda: gg.matching(9)])
def test_recolor_degrees_regular_graph_is_the_baseline(make):
    g = make()
    for seed in range(3):
        a = oracle.color_d1(g, seed=seed, recolor_degrees=True)
        b = oracle.color_d1(g, seed=seed)
        assert np.array_equal(a.colors, b.colors) and a.rounds == b.rounds


def _rank_priority(deg, p):
    """Explicit priorities that order vertices by (deg, p, id): the baseline
    rule with these priorities must equal recolorDegrees."""
    order = np.lexsort((np.arange(deg.size), p.astype(np.int64), deg.astype(np.int64)))
    rank = np.empty(deg.size, np.uint32)
    rank[order] = np.arange(deg.size, dtype=np.uint32)
    return rank


@pytest.mark.parametrize("kind", ["d1", "d2", "pd2"])
def test_recolor_degrees_is_baseline_with_degree_ranked_priorities(kind):
    """Degrees counted here with numpy (D1/D2: adjacency row lengths; PD2:
    rows per column), priorities from the pinned hash: the degree rule equals
    the baseline rule under the (deg, p, id) rank, on graphs with many equal
    degrees and with hubs."""
    for seed in range(3):
        if kind == "pd2":
            b = gg.bipartite_powerlaw(2500, 600, 5, 2.1, seed=seed)
            deg = np.diff(b.col_ptr)
            p = oracle.priorities(b.n_cols, seed)
            a = oracle.color_pd2(b, seed=seed, recolor_degrees=True)
            c = oracle.color_pd2(b, prio=_rank_priority(deg, p))
        else:
            g = gg.rmat(10, 8, seed=seed) if seed else gg.erdos_renyi(1200, 7, seed)
            deg = np.diff(g.row_ptr)
            p = oracle.priorities(g.n, seed)
            run = oracle.color_d1 if kind == "d1" else oracle.color_d2
            a = run(g, seed=seed, recolor_degrees=True)
            c = run(g, prio=_rank_priority(deg, p))
        assert np.array_equal(a.colors, c.colors) and a.rounds == c.rounds and a.worklist == c.worklist


def test_recolor_degrees_certificates():
    """Proper, first-fit complete, at most deg + 1, rounds >= colors."""
    for seed in range(4):
        g = gg.rmat(11, 8, seed=seed + 10)
        r = oracle.color_d1(g, seed=seed, recolor_degrees=True)
        # key-local maxima under (deg, p, id) take color 1
        _check_d1_certificate(g, r, prio=_rank_priority(np.diff(g.row_ptr), oracle.priorities(g.n, seed)))


# --------------------------------------------------------------------------
# resume, relabeling
# --------------------------------------------------------------------------

@pytest.mark.parametrize("stop", [1, 2, 4])
def test_resume_from_partial_state(stop):
    g = gg.erdos_renyi(3000, 12, 7)
    full = oracle.color_d1(g, seed=5)
    part = oracle.color_d1(g, seed=5, max_rounds=stop)
    assert not part.converged and part.rounds == stop
    assert np.all(part.colors[part.colors > 0] == full.colors[part.colors > 0])
    rest = oracle.color_d1(g, seed=5, init=part.colors)
    assert np.array_equal(rest.colors, full.colors)
    assert rest.rounds + stop == full.rounds
    assert rest.worklist == full.worklist[stop:]


def test_relabel_equivariance():
    rng = np.random.default_rng(11)
    g = gg.erdos_renyi(500, 10, 3)
    prio = rng.permutation(g.n).astype(np.uint32)
    perm = rng.permutation(g.n)
    h = gg.relabel(g, perm)
    prio_h = np.empty_like(prio)
    prio_h[perm] = prio
    a = oracle.color_d1(g, prio=prio).colors
    b = oracle.color_d1(h, prio=prio_h).colors
    assert np.array_equal(b[perm], a)


# --------------------------------------------------------------------------
# ghost variant (one rank's step of Algorithm 2)
# --------------------------------------------------------------------------

def _ghost_case(seed, layers, parts=4, n=3000, ef=8):
    g = gg.erdos_renyi(n, ef, seed)
    owner = gg.hash_partition(n, parts, seed)
    delta = int(g.degrees().max())
    gcol = gg.ghost_colors_uniform(n, delta, seed + 1)
    return g, gg.ghost_local_graph(g, owner, 0, layers, gcol)


def test_ghost_without_ghosts_equals_d1():
    g = gg.erdos_renyi(2000, 10, 2)
    owner = np.zeros(g.n, np.int32)
    lg = gg.ghost_local_graph(g, owner, 0, 1, np.ones(g.n, np.int32))
    assert lg.n_ghost == 0
    r = oracle.color_d1_ghost(lg, seed=9)
    assert np.array_equal(r.colors, oracle.color_d1(g, seed=9).colors)
    assert r.boundary_conflicts == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ghost_invariants(seed):
    g, lg = _ghost_case(seed, 1)
    _, lg2 = _ghost_case(seed, 2)
    r = oracle.color_d1_ghost(lg, seed=seed)
    r2 = oracle.color_d1_ghost(lg2, seed=seed)
    assert np.array_equal(r.colors, r2.colors)                  # ghosts are fixed: layer 2 unread
    assert np.array_equal(r.remote_loser, r2.remote_loser[:lg.n_ghost]) if lg.n_ghost == lg2.n_g1 else True
    assert r.boundary_conflicts > 0
    c = r.colors
    no = lg.n_owned
    keys = np.array([oracle.priority(int(x), seed) for x in lg.gid], dtype=np.int64)
    gc = lg.ghost_colors
    assert np.all(c >= 1)
    for v in range(no):
        nb = lg.col[lg.row_ptr[v]:lg.row_ptr[v + 1]]
        own = nb[nb < no]
        gh = nb[nb >= no]
        assert c[v] not in set(c[own].tolist())                 # owned-owned proper
        for u in gh:
            if c[v] == gc[u - no]:                              # surviving boundary pair:
                assert keys[v] > keys[u]                         # owned keeps it ...
                assert r.remote_loser[u - no] == 1               # ... and the ghost is flagged
    assert r.remote_losers == int(r.remote_loser.sum())


def test_ghost_phase1_is_ghost_blind_d1_of_owned_subgraph():
    g, lg = _ghost_case(4, 1)
    no = lg.n_owned
    src = np.repeat(np.arange(no), np.diff(lg.row_ptr))
    keep = lg.col < no
    sub = gg.csr_from_pairs(no, src[keep], lg.col[keep], True)
    # with every ghost colored 0-impossible (huge color), phase 2 finds no
    # conflicts and the result is D1 of the owned subgraph under gid keys
    lg.ghost_colors = np.full(lg.n_ghost, 1 << 30, np.int32)
    r = oracle.color_d1_ghost(lg, seed=4)
    prio = np.array([oracle.priority(int(x), 4) for x in lg.gid[:no]], dtype=np.uint32)
    ref = oracle.color_d1(sub, prio=prio)
    # prio ties are impossible (bijective hash), so gid order does not matter
    assert np.array_equal(r.colors, ref.colors)
    assert r.boundary_conflicts == 0


@pytest.mark.parametrize("seed,ncolors", [(5, 3), (6, 0), (7, 2)])
def test_ghost_reduces_to_d1_steps(seed, ncolors):
    """The ghost variant rebuilt from D1 pieces on explicitly constructed
    graphs: phase 1 = D1 of the owned subgraph; phase 2 recounted with numpy
    over the owned-ghost edges; phase 3 = D1 with an initial partial coloring
    on the owned + ghost graph where ghosts carry their fixed colors."""
    g, lg = _ghost_case(seed, 1, parts=3, n=2500)
    if ncolors:
        lg.ghost_colors = np.random.default_rng(seed).integers(1, ncolors + 1, lg.n_ghost).astype(np.int32)
    no, m = lg.n_owned, lg.n_owned + lg.n_ghost
    keys = np.array([oracle.priority(int(x), seed) for x in lg.gid], dtype=np.uint32)
    src = np.repeat(np.arange(no), np.diff(lg.row_ptr))
    own = lg.col < no
    sub = gg.csr_from_pairs(no, src[own], lg.col[own], True)
    c1 = oracle.color_d1(sub, prio=keys[:no]).colors
    gs, gv = src[~own], lg.col[~own] - no
    eq = c1[gs] == lg.ghost_colors[gv]
    k64 = keys.astype(np.int64)
    lose = np.zeros(no, bool)
    lose[gs[eq & (k64[gv + no] > k64[gs])]] = True
    flag = np.zeros(lg.n_ghost, np.uint8)
    flag[gv[eq & (k64[gs] > k64[gv + no])]] = 1
    aug = gg.csr_from_pairs(m, src, lg.col, True)
    init = np.concatenate([np.where(lose, 0, c1), lg.ghost_colors]).astype(np.int32)
    c3 = oracle.color_d1(aug, prio=keys, init=init).colors
    r = oracle.color_d1_ghost(lg, seed=seed)
    assert r.boundary_conflicts == int(eq.sum())
    assert np.array_equal(r.remote_loser, flag)
    assert np.array_equal(r.colors, c3[:no])
    assert np.array_equal(c3[no:], lg.ghost_colors)
    if ncolors:
        assert lose.any()
