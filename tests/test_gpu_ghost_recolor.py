"""GPU parity of tentative ghost recoloring (COLOR_FLAG_GHOST_RECOLOR;
Section 3.2 save/restore of ghost colors, Section 3.4 second layer): the
ghost step and Algorithm 2 over several ranks against the oracle, bit for
bit, with one and two layers, hash key and recolorDegrees, fresh and
resumed steps, unknown ghost colors, and every pull-engine mapping."""
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


def case(seed, layers, ncolors=4, scale=15):
    g = gg.rmat(scale, 8, seed)
    owner = gg.hash_partition(g.n, 4, seed)
    gcol = np.random.default_rng(seed).integers(1, ncolors + 1, g.n).astype(np.int32)
    lg = gg.ghost_local_graph(g, owner, 0, layers, gcol)
    gdeg = g.degrees()[lg.gid[lg.n_owned:]].astype(np.int32)
    return g, lg, gdeg


def step(gc, lg, gdeg, seed, flags, init=None, gcolors=None, **pk):
    gcolors = lg.ghost_colors if gcolors is None else gcolors
    colors, rl, st = gc.color_d1_ghost_step(
        lg.n_owned, lg.n_ghost, lg.layers, lg.n_g1, dev(lg.row_ptr), dev(lg.col), dev(lg.gid), dev(gcolors),
        seed=seed, ghost_degree=dev(gdeg), init_owned=None if init is None else dev(init),
        params=gc.Params(flags=flags, **pk), trace_cap=4096)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), rl.cpu().numpy(), st


def same(got, rl, st, ref, what):
    assert np.array_equal(got, ref.colors), what
    assert np.array_equal(rl, ref.remote_loser), what
    assert st.boundary_conflicts == ref.boundary_conflicts and st.remote_losers == ref.remote_losers, what
    assert (st.rounds, st.vertex_visits, st.edge_visits) == (ref.rounds, ref.vertex_visits, ref.edge_visits), what
    assert st.worklist == ref.worklist[:len(st.worklist)], what


MAPPINGS = [{}, dict(bin_hi=(2, 4, 8, 16), lanes=(1, 2, 64), split_chunks=3),
            dict(bin_hi=(1, 2, 3, 4), lanes=(8, 32, 4), split_chunks=7)]


@pytest.mark.parametrize("degrees", [False, True], ids=["hash-key", "recolor-degrees"])
@pytest.mark.parametrize("layers", [1, 2])
def test_ghost_step_with_tentative_ghost_recoloring(gc, layers, degrees):
    g, lg, gdeg = case(3, layers)
    ref = oracle.color_d1_ghost(lg, seed=3, recolor_degrees=degrees, ghost_degree=gdeg, ghost_recolor=True)
    assert ref.remote_losers > 50
    flags = gc.COLOR_FLAG_GHOST_RECOLOR | (gc.COLOR_FLAG_RECOLOR_DEGREES if degrees else 0)
    for mp in MAPPINGS:
        got, rl, st = step(gc, lg, gdeg, 3, flags, **mp)
        same(got, rl, st, ref, f"layers {layers} {mp}")
    fixed = oracle.color_d1_ghost(lg, seed=3, recolor_degrees=degrees, ghost_degree=gdeg)
    assert not np.array_equal(fixed.colors, ref.colors)   # the option changes the result here


@pytest.mark.parametrize("layers", [1, 2])
def test_resumed_step_with_unknown_ghosts(gc, layers):
    """A later iteration of Algorithm 2: committed owned colors, new ghost
    colors of which some are not known yet (0: never recolored, never a
    constraint)."""
    g, lg, gdeg = case(4, layers)
    first = oracle.color_d1_ghost(lg, seed=4)
    new = np.random.default_rng(2).integers(0, 4, lg.n_ghost).astype(np.int32)
    lg2 = gg.LocalGraph(**{**lg.__dict__, "ghost_colors": new})
    ref = oracle.color_d1_ghost(lg2, seed=4, init_owned=first.colors, ghost_recolor=True)
    got, rl, st = step(gc, lg, gdeg, 4, gc.COLOR_FLAG_GHOST_RECOLOR, init=first.colors, gcolors=new)
    same(got, rl, st, ref, f"resumed, layers {layers}")


@pytest.mark.parametrize("layers", [1, 2])
def test_distributed_with_tentative_ghost_recoloring(gc, layers):
    g = gg.rmat(15, 16, 6)
    owner = gg.hash_partition(g.n, 8, 3)
    zeros = np.zeros(g.n, np.int32)
    locs = [gg.ghost_local_graph(g, owner, p, layers, zeros) for p in range(8)]
    ref = oracle.color_d1_distributed(locs, seed=5, ghost_recolor=True)
    homes = gg.ghost_homes(locs)
    parts = [dict(n_owned=lg.n_owned, n_ghost=lg.n_ghost, layers=lg.layers, n_g1=lg.n_g1, row_ptr=dev(lg.row_ptr),
                  col_idx=dev(lg.col), gid=dev(lg.gid), ghost_owner=dev(o), ghost_index=dev(i))
             for lg, (o, i) in zip(locs, homes)]
    outs, st = gc.color_d1_distributed(parts, seed=5, params=gc.Params(flags=gc.COLOR_FLAG_GHOST_RECOLOR))
    for p in range(8):
        assert np.array_equal(outs[p].cpu().numpy(), ref.colors[p]), p
    assert st.conflicts == ref.conflicts and st.exchanged == ref.exchanged and st.rounds_total == ref.rounds
