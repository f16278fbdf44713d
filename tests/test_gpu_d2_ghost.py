"""GPU parity of the distance-2 and partial distance-2 ghost steps
(color_d2_ghost, color_pd2_ghost; Section 3.5 Algorithm 5 over a rank's owned
vertices, Section 3.6) against the oracle, bit for bit: 7-point meshes in
slabs (the paper's mesh partition), hash partitions of random and power-law
graphs, power-law patterns by column hash, every pull-engine mapping."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_00075_amd as m
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def same(got, rl, st, ref, what):
    assert np.array_equal(got, ref.colors), what
    assert np.array_equal(rl, ref.remote_loser), what
    assert (st.boundary_conflicts, st.remote_losers) == (ref.boundary_conflicts, ref.remote_losers), what
    assert (st.rounds, st.vertex_visits, st.edge_visits, st.num_colors) == \
        (ref.rounds, ref.vertex_visits, ref.edge_visits, ref.num_colors), what
    assert st.worklist == ref.worklist[:len(st.worklist)], what


MAPPINGS = [{}, dict(bin_hi=(2, 8, 16, 40), lanes=(1, 2, 64), split_chunks=3),
            dict(bin_hi=(1, 2, 3, 4), lanes=(8, 32, 4), split_chunks=7)]
# phase 1 on the library's choice, the pull engine, the incremental engine
# with its tail kernel (a low threshold so that small graphs reach it) and
# with per-round launches only
ENGINES = [dict(engine=0), dict(engine=1), dict(engine=2, tail_threshold=1 << 20), dict(engine=2, flags=2)]


def configs():
    for mp in MAPPINGS:
        yield mp
    for en in ENGINES:
        yield en
    yield dict(MAPPINGS[1], engine=2)


def d2_cases():
    dims = (32, 30, 48)
    mesh = gg.stencil(dims, 7)
    yield "mesh slab 1 of 4", mesh, gg.slab_partition(dims, 4), 1, 25
    yield "mesh slab 0 of 8", mesh, gg.slab_partition(dims, 8), 0, 25
    er = gg.erdos_renyi(8000, 6, 2)
    yield "ER hash", er, gg.hash_partition(er.n, 3, 2), 0, 30
    rm = gg.rmat(12, 4, 3)
    yield "R-MAT hash", rm, gg.hash_partition(rm.n, 4, 3), 2, 60


@pytest.mark.parametrize("which", range(4))
def test_d2_ghost_matches_oracle(gc, which):
    name, g, owner, part, ncol = list(d2_cases())[which]
    gcol = np.random.default_rng(which).integers(1, ncol + 1, g.n).astype(np.int32)
    lg = gg.ghost_local_graph(g, owner, part, 2, gcol)
    ref = oracle.color_d2_ghost(lg, seed=7)
    assert ref.boundary_conflicts > 0
    for mp in configs():
        c, rl, st = gc.color_d2_ghost(lg.n_owned, lg.n_ghost, lg.n_g1, dev(lg.row_ptr), dev(lg.col), dev(lg.gid),
                                      dev(lg.ghost_colors), seed=7, params=gc.Params(**mp), trace_cap=4096)
        torch.cuda.synchronize()
        same(c.cpu().numpy(), rl.cpu().numpy(), st, ref, f"{name} {mp}")


@pytest.mark.parametrize("seed", [1, 2])
def test_pd2_ghost_matches_oracle(gc, seed):
    b = gg.bipartite_powerlaw(40000, 10000, 6, 2.1, seed)
    owner = gg.hash_partition(b.n_cols, 4, seed)
    gcol = np.random.default_rng(seed).integers(1, 40, b.n_cols).astype(np.int32)
    lp = gg.pd2_local_pattern(b, owner, seed % 4, gcol)
    ref = oracle.color_pd2_ghost(lp, seed=seed)
    assert ref.boundary_conflicts > 0
    for mp in configs():
        c, rl, st = gc.color_pd2_ghost(lp.n_owned, lp.n_ghost, lp.n_rows, dev(lp.col_ptr), dev(lp.row_idx),
                                       dev(lp.row_ptr), dev(lp.col_idx), dev(lp.gid), dev(lp.ghost_colors),
                                       seed=seed, params=gc.Params(**mp), trace_cap=4096)
        torch.cuda.synchronize()
        same(c.cpu().numpy(), rl.cpu().numpy(), st, ref, f"PD2 seed {seed} {mp}")


def test_ghost2_without_ghosts_is_the_plain_call(gc):
    g = gg.stencil((20, 18, 16), 7)
    lg = gg.ghost_local_graph(g, np.zeros(g.n, np.int32), 0, 2, np.ones(g.n, np.int32))
    c, rl, st = gc.color_d2_ghost(lg.n_owned, 0, 0, dev(lg.row_ptr), dev(lg.col), dev(lg.gid), None, seed=3)
    c2, _ = gc.color_d2(dev(g.row_ptr), dev(g.col), seed=3)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), c2.cpu().numpy()) and st.boundary_conflicts == 0


def test_pd2_ghost_heavy_owned_columns(gc):
    """The heaviest columns owned by the rank: their lists (first hop above
    1,024 rows) are built as bitmap sets, which keep owned members only."""
    b = gg.bipartite_powerlaw(60000, 8000, 6, 2.1, 5)
    deg = np.diff(b.col_ptr)
    owner = gg.hash_partition(b.n_cols, 4, 5)
    owner[np.argsort(deg)[-12:]] = 0
    assert deg[owner == 0].max() > 1024
    gcol = np.random.default_rng(5).integers(1, 80, b.n_cols).astype(np.int32)
    lp = gg.pd2_local_pattern(b, owner, 0, gcol)
    ref = oracle.color_pd2_ghost(lp, seed=4)
    for mp in ENGINES:
        c, rl, st = gc.color_pd2_ghost(lp.n_owned, lp.n_ghost, lp.n_rows, dev(lp.col_ptr), dev(lp.row_idx),
                                       dev(lp.row_ptr), dev(lp.col_idx), dev(lp.gid), dev(lp.ghost_colors),
                                       seed=4, params=gc.Params(**mp), trace_cap=4096)
        torch.cuda.synchronize()
        same(c.cpu().numpy(), rl.cpu().numpy(), st, ref, f"PD2 heavy {mp}")
        if mp.get("engine") == 2:
            assert st.engine == gc.ENGINE_INCREMENTAL


def test_d2_ghost_heavy_hubs(gc):
    """D2 on an R-MAT part whose hubs have first hops above 1,024 entries."""
    g = gg.rmat(13, 8, 6)
    owner = gg.hash_partition(g.n, 8, 6)
    deg = g.degrees()
    owner[np.argsort(deg)[-8:]] = 1
    assert deg[owner == 1].max() > 1024
    gcol = np.random.default_rng(6).integers(1, 200, g.n).astype(np.int32)
    lg = gg.ghost_local_graph(g, owner, 1, 2, gcol)
    ref = oracle.color_d2_ghost(lg, seed=2)
    for mp in ENGINES:
        c, rl, st = gc.color_d2_ghost(lg.n_owned, lg.n_ghost, lg.n_g1, dev(lg.row_ptr), dev(lg.col), dev(lg.gid),
                                      dev(lg.ghost_colors), seed=2, params=gc.Params(**mp), trace_cap=4096)
        torch.cuda.synchronize()
        same(c.cpu().numpy(), rl.cpu().numpy(), st, ref, f"D2 hubs {mp}")
