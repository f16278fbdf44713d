"""Full-size parity on the benchmark graphs, in the launch configuration the
benchmark times (library defaults, both engines where the library has two),
against the oracle's results stored as SHA-256 digests of the color arrays
plus the round statistics by tests/golden/make_golden.py, which calls only
the oracle:

* 27-point stencil 128^3 (D1), R-MAT scale 22 (D1), 7-point stencil 96^3 (D2);
* the 4,000,000 x 1,000,000 power-law PD2 pattern (about half an hour of
  oracle time on one core), plus properties that hold at any size;
* one rank's ghost step on part 0 of R-MAT scale 24 split 16 ways, with one
  and with two ghost layers (colors, remote-loser flags, conflict counts).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_00075_amd as m
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def check_golden(colors, st, ref, what):
    digest = hashlib.sha256(np.ascontiguousarray(colors, dtype=np.int32).tobytes()).hexdigest()
    assert digest == ref["colors_sha256"], f"{what}: colors differ from the oracle's"
    assert st.rounds == ref["rounds"], what
    assert st.num_colors == ref["num_colors"], what
    assert st.vertex_visits == ref["vertex_visits"], what
    assert st.edge_visits == ref["edge_visits"], what
    assert st.worklist == ref["worklist"][:len(st.worklist)], what


@pytest.mark.parametrize("engine", [1, 2], ids=["pull", "incremental"])
def test_stencil27_128_d1(gc, engine):
    g = gg.stencil((128, 128, 128), 27)
    ref = golden("stencil27_128_d1_seed1")
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    c, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=1, params=gc.Params(engine=engine), trace_cap=4096)
    check_golden(c.cpu().numpy(), st, ref, f"27pt 128^3 engine {engine}")


@pytest.mark.parametrize("engine", [1, 2], ids=["pull", "incremental"])
def test_rmat22_d1(gc, engine):
    g = gg.rmat(22, 16, seed=1)
    ref = golden("rmat22_d1_seed1")
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    c, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=1, params=gc.Params(engine=engine), trace_cap=4096)
    check_golden(c.cpu().numpy(), st, ref, f"R-MAT 22 engine {engine}")


@pytest.mark.parametrize("engine", [1, 2], ids=["pull", "incremental"])
def test_stencil7_96_d2(gc, engine):
    g = gg.stencil((96, 96, 96), 7)
    ref = golden("stencil7_96_d2_seed1")
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    c, st = gc.color_d2(dev(g.row_ptr), dev(g.col), seed=1, params=gc.Params(engine=engine), trace_cap=4096)
    check_golden(c.cpu().numpy(), st, ref, f"7pt 96^3 D2 engine {engine}")


def test_pd2_4m_by_1m(gc):
    b = gg.bipartite_powerlaw(4_000_000, 1_000_000, 8, 2.1, seed=1)
    ref = golden("pd2_4m_1m_seed1")
    assert (b.n_rows, b.n_cols, b.nnz) == (ref["n_rows"], ref["n"], ref["nnz"])
    args = (dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx))
    out = {}
    for engine in (1, 2):
        c, st = gc.color_pd2(*args, seed=1, params=gc.Params(engine=engine), trace_cap=4096)
        out[engine] = (c.cpu().numpy(), st)
        check_golden(out[engine][0], st, ref, f"PD2 4M x 1M engine {engine}")
    (c1, s1), (c2, s2) = out[1], out[2]
    assert (s1.rounds, s1.num_colors, s1.vertex_visits, s1.edge_visits) == \
        (s2.rounds, s2.num_colors, s2.vertex_visits, s2.edge_visits)
    colors = c1
    assert colors.min() >= 1 and colors.max() == s1.num_colors
    assert s1.rounds >= s1.num_colors  # a vertex committed in round r has color <= r
    # every row has 8 columns: their colors must be pairwise distinct
    rc = np.sort(colors[b.col_idx].reshape(-1, 8), axis=1)
    assert np.all(rc[:, 1:] != rc[:, :-1]), "two columns of a row share a color"
    # first-fit certificate on sampled columns: every smaller color occurs
    # among the columns sharing a row with it
    rng = np.random.default_rng(7)
    for c in rng.choice(b.n_cols, size=300, replace=False):
        rows = b.row_idx[b.col_ptr[c]:b.col_ptr[c + 1]]
        nb = np.concatenate([b.col_idx[b.row_ptr[r]:b.row_ptr[r + 1]] for r in rows]) if rows.size else \
            np.zeros(0, np.int32)
        nb = nb[nb != c]
        seen = set(colors[nb].tolist())
        assert all(x in seen for x in range(1, colors[c])), f"column {c}: color {colors[c]} not first fit"


@pytest.fixture(scope="module")
def rmat24_parts():
    """R-MAT 24 ef16 seed 1 split 16 ways by hash, ghost colors per global id
    (the workload the golden digests were written for)."""
    g = gg.rmat(24, 16, seed=1)
    delta = int(g.degrees().max())
    owner = gg.hash_partition(g.n, 16, seed=7)
    gcol = gg.ghost_colors_uniform(g.n, delta, seed=11)
    return g, owner, gcol


@pytest.mark.parametrize("layers", [1, 2])
def test_rmat24_part0_ghost(gc, rmat24_parts, layers):
    g, owner, gcol = rmat24_parts
    lg = gg.ghost_local_graph(g, owner, 0, layers, gcol, sort_rows=False)
    ref = golden(f"rmat24_part0_l{layers}")
    assert (lg.n_owned, lg.n_ghost, lg.n_g1, lg.nnz) == (ref["n"], ref["n_ghost"], ref["n_g1"], ref["nnz"])
    colors, rl, st = gc.color_d1_ghost(lg.n_owned, lg.n_ghost, lg.layers, lg.n_g1, dev(lg.row_ptr), dev(lg.col),
                                       dev(lg.gid), dev(lg.ghost_colors), seed=1, trace_cap=4096)
    check_golden(colors.cpu().numpy(), st, ref, f"R-MAT 24 part 0, {layers} layer(s)")
    flags = hashlib.sha256(np.ascontiguousarray(rl.cpu().numpy(), dtype=np.uint8).tobytes()).hexdigest()
    assert flags == ref["remote_loser_sha256"]
    assert (st.boundary_conflicts, st.remote_losers) == (ref["boundary_conflicts"], ref["remote_losers"])
