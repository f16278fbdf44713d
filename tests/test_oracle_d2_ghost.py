"""Pins of the oracle's distance-2 and partial distance-2 ghost step
(Section 3.5, Algorithm 5 over a rank's owned vertices; Section 3.6): it is
the distance-1 ghost step on the square graph G^2 (D2) or on the column
intersection graph A^T A (PD2) — built here with scipy — with the same owners
and ghost colors."""
import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle


def _square(g):
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    s = ((a @ a) + a).tocoo()
    keep = s.row != s.col
    return gg.csr_from_pairs(g.n, s.row[keep], s.col[keep], True)


def _intersection(b):
    a = sp.csr_matrix((np.ones(b.nnz), b.col_idx, b.row_ptr), shape=(b.n_rows, b.n_cols))
    s = (a.T @ a).tocoo()
    keep = s.row != s.col
    return gg.csr_from_pairs(b.n_cols, s.row[keep], s.col[keep], True)


def _same_step(r, ref, lg_gid, ref_gid, n_owned):
    assert np.array_equal(lg_gid[:n_owned], ref_gid[:n_owned])          # owned in gid order in both
    assert np.array_equal(r.colors, ref.colors)
    assert (r.boundary_conflicts, r.remote_losers, r.rounds, r.vertex_visits) == \
        (ref.boundary_conflicts, ref.remote_losers, ref.rounds, ref.vertex_visits)
    flagged = set(lg_gid[n_owned:][r.remote_loser == 1].tolist())
    assert flagged == set(ref_gid[n_owned:][ref.remote_loser == 1].tolist())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_d2_ghost_is_d1_ghost_of_the_square(seed):
    rng = np.random.default_rng(seed)
    for g in (gg.erdos_renyi(1500, 5, seed), gg.stencil((12, 11, 10), 7), gg.rmat(10, 4, seed)):
        owner = gg.hash_partition(g.n, 3, seed) if seed != 2 else rng.integers(0, 3, g.n).astype(np.int32)
        gcol = rng.integers(1, 6, g.n).astype(np.int32)
        lg = gg.ghost_local_graph(g, owner, 0, 2, gcol)
        r = oracle.color_d2_ghost(lg, seed=seed)
        sq = gg.ghost_local_graph(_square(g), owner, 0, 1, gcol)
        ref = oracle.color_d1_ghost(sq, seed=seed)
        assert sq.n_ghost == lg.n_ghost                  # the two-hop ghosts are the two layers
        _same_step(r, ref, lg.gid, sq.gid, lg.n_owned)
        assert r.boundary_conflicts > 0


@pytest.mark.parametrize("seed", [1, 2])
def test_pd2_ghost_is_d1_ghost_of_the_intersection_graph(seed):
    rng = np.random.default_rng(seed + 10)
    b = gg.bipartite_powerlaw(3000, 1200, 5, 2.1, seed)
    owner = gg.hash_partition(b.n_cols, 4, seed)
    gcol = rng.integers(1, 8, b.n_cols).astype(np.int32)
    lp = gg.pd2_local_pattern(b, owner, 0, gcol)
    r = oracle.color_pd2_ghost(lp, seed=seed)
    ig = gg.ghost_local_graph(_intersection(b), owner, 0, 1, gcol)
    ref = oracle.color_d1_ghost(ig, seed=seed)
    assert ig.n_ghost == lp.n_ghost
    _same_step(r, ref, lp.gid, ig.gid, lp.n_owned)
    assert r.boundary_conflicts > 0


def test_one_rank_is_the_plain_method():
    g = gg.stencil((14, 13, 12), 7)
    lg = gg.ghost_local_graph(g, np.zeros(g.n, np.int32), 0, 2, np.ones(g.n, np.int32))
    assert lg.n_ghost == 0
    assert np.array_equal(oracle.color_d2_ghost(lg, seed=4).colors, oracle.color_d2(g, seed=4).colors)
    b = gg.bipartite_powerlaw(2000, 700, 6, 2.1, 5)
    lp = gg.pd2_local_pattern(b, np.zeros(b.n_cols, np.int32), 0, np.ones(b.n_cols, np.int32))
    assert lp.n_ghost == 0
    assert np.array_equal(oracle.color_pd2_ghost(lp, seed=4).colors, oracle.color_pd2(b, seed=4).colors)


def test_slab_partition_invariants():
    dims = (20, 20, 24)
    g = gg.stencil(dims, 7)
    owner = gg.slab_partition(dims, 4)
    assert np.array_equal(np.bincount(owner), [g.n // 4] * 4)
    gcol = np.random.default_rng(3).integers(1, 10, g.n).astype(np.int32)
    lg = gg.ghost_local_graph(g, owner, 1, 2, gcol)           # a middle slab: ghosts on both sides
    r = oracle.color_d2_ghost(lg, seed=6)
    no = lg.n_owned
    keys = np.array([oracle.priority(int(x), 6) for x in lg.gid], dtype=np.int64)
    C = r.colors
    sq = _square(g)
    for v in range(no):
        gv = lg.gid[v]
        for x in sq.col[sq.row_ptr[gv]:sq.row_ptr[gv + 1]]:
            if owner[x] == 1:
                assert C[v] != C[np.searchsorted(lg.gid[:no], x)]     # owned pairs within distance 2 differ
            elif C[v] == gcol[x]:                                      # surviving boundary pair
                j = np.nonzero(lg.gid[no:] == x)[0][0]
                assert keys[v] > keys[no + j] and r.remote_loser[j] == 1
