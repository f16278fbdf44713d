"""GPU parity of the recolorDegrees key (Section 3.3; Algorithm 4 with
recolorDegrees set): key(v) = (deg(v), p(v), gid(v)), so the lower-degree
vertex of a conflict is recolored.  The HIP path (COLOR_FLAG_RECOLOR_DEGREES
through the C-ABI) against the CPU oracle's recolor_degrees option, bit for
bit, on every engine; the ghost step with the ghosts' degrees and with a
committed starting state (a later iteration of Algorithm 2)."""
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


def dev(a, dtype=np.int32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


# (engine, extra flags): incremental with its tail kernel, incremental with
# per-round launches only, pull
ENGINES = [(2, 0), (2, 2), (1, 0)]


def P(gc, engine, flags, **kw):
    return gc.Params(engine=engine, flags=gc.COLOR_FLAG_RECOLOR_DEGREES | flags, **kw)


def same(got, st, ref, what):
    if not np.array_equal(got, ref.colors):
        bad = np.nonzero(got != ref.colors)[0]
        raise AssertionError(f"{what}: {bad.size} colors differ, first at {bad[:5]}: "
                             f"gpu {got[bad[:5]]} oracle {ref.colors[bad[:5]]}")
    assert st.rounds == ref.rounds, f"{what}: rounds {st.rounds} vs {ref.rounds}"
    assert st.worklist == ref.worklist[:len(st.worklist)], what
    assert st.vertex_visits == ref.vertex_visits, what
    assert st.edge_visits == ref.edge_visits, what
    assert st.num_colors == ref.num_colors, what


GRAPHS = {
    "er_10k": lambda: gg.erdos_renyi(10000, 16, 1),
    "rmat14": lambda: gg.rmat(14, 16, 2),
    "rmat16_ef8": lambda: gg.rmat(16, 8, 3),
    "stencil27_20": lambda: gg.stencil((20, 21, 19), 27),
    "mycielski_8": lambda: gg.mycielski(8),
}


@pytest.mark.parametrize("engine,flags", ENGINES, ids=["incremental", "incremental-no-tail", "pull"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_d1_recolor_degrees(gc, name, engine, flags):
    g = GRAPHS[name]()
    ref = oracle.color_d1(g, seed=5, recolor_degrees=True)
    colors, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=5, params=P(gc, engine, flags), trace_cap=4096)
    torch.cuda.synchronize()
    same(colors.cpu().numpy(), st, ref, name)
    # the option changes the result on every one of these graphs
    assert not np.array_equal(ref.colors, oracle.color_d1(g, seed=5).colors)


@pytest.mark.parametrize("engine,flags", ENGINES, ids=["incremental", "incremental-no-tail", "pull"])
def test_d1_recolor_degrees_split_bins(gc, engine, flags):
    """Every mapping of the pull engine (narrow groups, whole workgroups and
    split vertices) and narrow incremental bins give the same coloring."""
    g = gg.rmat(15, 16, 7)
    ref = oracle.color_d1(g, seed=1, recolor_degrees=True)
    for kw in (dict(bin_hi=(2, 4, 8, 16), lanes=(1, 2, 64), split_chunks=3),
               dict(bin_hi=(1, 2, 3, 4), lanes=(8, 32, 4), split_chunks=7)):
        colors, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=1, params=P(gc, engine, flags, **kw),
                                 trace_cap=4096)
        torch.cuda.synchronize()
        same(colors.cpu().numpy(), st, ref, f"rmat15 {kw}")


@pytest.mark.parametrize("engine,flags", ENGINES, ids=["incremental", "incremental-no-tail", "pull"])
def test_d1_recolor_degrees_explicit_priorities_with_ties(gc, engine, flags):
    """Explicit priorities with many ties: the library's second sort (by
    degree after (p, gid)) decides; equal degree and equal p fall to gid."""
    g = gg.erdos_renyi(6000, 12, 4)
    prio = (np.arange(g.n, dtype=np.uint64) % 7).astype(np.uint32)
    ref = oracle.color_d1(g, seed=1, prio=prio, recolor_degrees=True)
    colors, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=1, prio=dev(prio.view(np.int32)),
                             params=P(gc, engine, flags), trace_cap=4096)
    torch.cuda.synchronize()
    same(colors.cpu().numpy(), st, ref, "ER prio ties")


@pytest.mark.parametrize("engine,flags", ENGINES, ids=["incremental", "incremental-no-tail", "pull"])
def test_d2_recolor_degrees(gc, engine, flags):
    for g in (gg.stencil((17, 15, 13), 7), gg.erdos_renyi(3000, 6, 2), gg.rmat(11, 4, 3)):
        ref = oracle.color_d2(g, seed=2, recolor_degrees=True)
        colors, st = gc.color_d2(dev(g.row_ptr), dev(g.col), seed=2, params=P(gc, engine, flags), trace_cap=4096)
        torch.cuda.synchronize()
        same(colors.cpu().numpy(), st, ref, f"D2 n={g.n}")


@pytest.mark.parametrize("engine,flags", ENGINES, ids=["incremental", "incremental-no-tail", "pull"])
def test_pd2_recolor_degrees(gc, engine, flags):
    for b in (gg.bipartite_powerlaw(20000, 5000, 6, 2.1, 3), gg.bipartite_powerlaw(4000, 4000, 8, 2.5, 4)):
        ref = oracle.color_pd2(b, seed=3, recolor_degrees=True)
        colors, st = gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx), seed=3,
                                  params=P(gc, engine, flags), trace_cap=4096)
        torch.cuda.synchronize()
        same(colors.cpu().numpy(), st, ref, f"PD2 {b.n_rows}x{b.n_cols}")


def _ghost_case(seed, layers):
    g = gg.rmat(15, 8, seed)
    owner = gg.hash_partition(g.n, 4, seed)
    gcol = gg.ghost_colors_uniform(g.n, int(g.degrees().max()), seed + 1)
    lg = gg.ghost_local_graph(g, owner, 0, layers, gcol)
    gdeg = g.degrees()[lg.gid[lg.n_owned:]].astype(np.int32)
    return g, lg, gdeg


def _ghost_step(gc, lg, gdeg, seed, init=None, gcolors=None, degrees=True):
    gcolors = lg.ghost_colors if gcolors is None else gcolors
    params = gc.Params(flags=gc.COLOR_FLAG_RECOLOR_DEGREES if degrees else 0)
    colors, rl, st = gc.color_d1_ghost_step(
        lg.n_owned, lg.n_ghost, lg.layers, lg.n_g1, dev(lg.row_ptr), dev(lg.col), dev(lg.gid), dev(gcolors),
        seed=seed, ghost_degree=dev(gdeg), init_owned=None if init is None else dev(init), params=params,
        trace_cap=4096)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), rl.cpu().numpy(), st


@pytest.mark.parametrize("layers", [1, 2])
def test_ghost_step_recolor_degrees(gc, layers):
    g, lg, gdeg = _ghost_case(3, layers)
    ref = oracle.color_d1_ghost(lg, seed=3, recolor_degrees=True, ghost_degree=gdeg)
    colors, rl, st = _ghost_step(gc, lg, gdeg, 3)
    assert np.array_equal(colors, ref.colors)
    assert np.array_equal(rl, ref.remote_loser)
    assert st.boundary_conflicts == ref.boundary_conflicts > 0
    assert st.remote_losers == ref.remote_losers
    assert st.rounds == ref.rounds and st.num_colors == ref.num_colors
    assert st.vertex_visits == ref.vertex_visits


def test_ghost_step_resumes_from_committed_colors(gc):
    """A later iteration of Algorithm 2: the owned colors of the first step
    are committed, the ghosts carry new colors (some 0 = not known), and only
    the boundary is judged and repaired; with and without degrees."""
    g, lg, gdeg = _ghost_case(4, 1)
    rng = np.random.default_rng(9)
    for degrees in (False, True):
        first = oracle.color_d1_ghost(lg, seed=4, recolor_degrees=degrees, ghost_degree=gdeg)
        new_gc = rng.integers(0, 4, lg.n_ghost).astype(np.int32)   # many conflicts, some unknown ghosts
        lg2 = gg.LocalGraph(**{**lg.__dict__, "ghost_colors": new_gc})
        ref = oracle.color_d1_ghost(lg2, seed=4, init_owned=first.colors, recolor_degrees=degrees,
                                    ghost_degree=gdeg)
        colors, rl, st = _ghost_step(gc, lg, gdeg, 4, init=first.colors, gcolors=new_gc, degrees=degrees)
        assert np.array_equal(colors, ref.colors)
        assert np.array_equal(rl, ref.remote_loser)
        assert st.boundary_conflicts == ref.boundary_conflicts > 100
        assert st.rounds == ref.rounds and st.vertex_visits == ref.vertex_visits


def test_flag_rejections(gc):
    g, lg, gdeg = _ghost_case(5, 1)
    params = gc.Params(flags=gc.COLOR_FLAG_RECOLOR_DEGREES)
    with pytest.raises(gc.ColorError) as e:   # no ghost degrees to key the ghosts by
        gc.color_d1_ghost(lg.n_owned, lg.n_ghost, 1, 0, dev(lg.row_ptr), dev(lg.col), dev(lg.gid),
                          dev(lg.ghost_colors), seed=5, params=params)
    assert e.value.code == -1
    h = gg.erdos_renyi(200, 4, 1)
    with pytest.raises(gc.ColorError) as e:   # batched jobs carry no degree option
        gc.color_batch([dict(kind=gc.KIND_D1, row_ptr=dev(h.row_ptr), col_idx=dev(h.col))], params=params)
    assert e.value.code == -1
