"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit for
bit (colors, round count and per-round worklist sizes), on seeded inputs that
span many tiles, ragged tails, every degree bin and the degenerate cases."""
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


ENGINE = {"id": 0, "flags": 0}


@pytest.fixture(autouse=True, scope="module", params=[(2, 0), (2, 2), (1, 0)],
                ids=["incremental", "incremental-no-tail", "pull"])
def engine(request):
    """Every parity case runs on both engines (2 = incremental, 1 = pull); the
    incremental engine both with its cooperative tail kernel (the default: it
    takes over once the worklist is small, which is every round of most of
    these graphs) and with per-round launches only (COLOR_FLAG_NO_TAIL = 2)."""
    ENGINE["id"], ENGINE["flags"] = request.param
    yield request.param
    ENGINE["id"], ENGINE["flags"] = 0, 0


def with_engine(gc, kw):
    p = kw.get("params")
    if p is None:
        p = gc.Params()
    p.engine = ENGINE["id"]
    p.flags |= ENGINE["flags"]
    kw["params"] = p
    return kw


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def run_d1(gc, g, seed=1, **kw):
    with_engine(gc, kw)
    colors, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=seed, trace_cap=4096, **kw)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), st


def run_d2(gc, g, seed=1, **kw):
    with_engine(gc, kw)
    colors, st = gc.color_d2(dev(g.row_ptr), dev(g.col), seed=seed, trace_cap=4096, **kw)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), st


def run_pd2(gc, b, seed=1, **kw):
    with_engine(gc, kw)
    colors, st = gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx), seed=seed,
                              trace_cap=4096, **kw)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), st


def same(got, st, ref, what=""):
    if not np.array_equal(got, ref.colors):
        bad = np.nonzero(got != ref.colors)[0]
        raise AssertionError(f"{what}: {bad.size} colors differ, first at {bad[:5]}: "
                             f"gpu {got[bad[:5]]} oracle {ref.colors[bad[:5]]}")
    assert st.rounds == ref.rounds, f"{what}: rounds {st.rounds} vs {ref.rounds}"
    assert st.worklist == ref.worklist[:len(st.worklist)], what
    assert st.vertex_visits == ref.vertex_visits, what
    assert st.edge_visits == ref.edge_visits, f"{what}: edge visits {st.edge_visits} vs {ref.edge_visits}"
    assert st.num_colors == ref.num_colors, what


# Bin settings that push small graphs through every mapping: sub-wavefront
# groups of every width, whole wavefronts, whole workgroups and split vertices.
BIN_VARIANTS = [
    None,
    dict(bin_hi=(2, 4, 8, 16), lanes=(1, 2, 64), split_chunks=3),
    dict(bin_hi=(1, 2, 3, 4), lanes=(8, 32, 4), split_chunks=7),
    dict(bin_hi=(1000, 2000, 3000, 4000), lanes=(64, 64, 64)),
    dict(bin_hi=(0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff), lanes=(1, 1, 1)),
    dict(bin_hi=(1, 1, 1, 1), split_chunks=64),
]


def params(gc, v, **extra):
    if v is None and not extra:
        return None
    kw = dict(v or {})
    kw.update(extra)
    return gc.Params(**kw)


def test_priority_matches_oracle_for_all_ids_below_2_24(gc):
    n = 1 << 24
    for seed in (1, 0xDEADBEEF):
        got = gc.color_priority(n, seed=seed).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.priorities(n, seed))


def test_d1_er_config(gc):
    g = gg.erdos_renyi(10000, 16, 1)
    got, st = run_d1(gc, g, seed=1)
    ref = oracle.color_d1(g, seed=1)
    same(got, st, ref, "ER 10k")
    assert st.edge_visits == ref.edge_visits
    assert st.engine == ENGINE["id"]


@pytest.mark.parametrize("vi", range(len(BIN_VARIANTS)))
def test_d1_bin_invariance(gc, vi):
    g = gg.rmat(12, 8, 3)
    ref = oracle.color_d1(g, seed=7)
    got, st = run_d1(gc, g, seed=7, params=params(gc, BIN_VARIANTS[vi]))
    same(got, st, ref, f"rmat12 variant {vi}")


@pytest.mark.parametrize("seed", range(5))
def test_d1_random_graphs(gc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    g = gg.erdos_renyi(n, float(rng.uniform(0.5, 40)), seed) if n > 1 else gg.complete(1)
    ref = oracle.color_d1(g, seed=seed)
    got, st = run_d1(gc, g, seed=seed, params=params(gc, BIN_VARIANTS[seed % len(BIN_VARIANTS)]))
    same(got, st, ref, f"ER n={n}")


@pytest.mark.parametrize("name", ["empty", "single", "edgeless", "K64", "K200", "star", "path", "matching",
                                  "mycielski8"])
def test_d1_special_graphs(gc, name):
    g = {
        "empty": gg.csr_from_pairs(0, np.array([], np.int64), np.array([], np.int64)),
        "single": gg.complete(1),
        "edgeless": gg.csr_from_pairs(777, np.array([], np.int64), np.array([], np.int64)),
        "K64": gg.complete(64),
        "K200": gg.complete(200),
        "star": gg.star(5000),
        "path": gg.path(1001),
        "matching": gg.matching(300),
        "mycielski8": gg.mycielski(8),
    }[name]
    ref = oracle.color_d1(g, seed=3)
    for v in (None, BIN_VARIANTS[1], BIN_VARIANTS[5]):
        got, st = run_d1(gc, g, seed=3, params=params(gc, v))
        same(got, st, ref, name)


def test_d1_explicit_priorities_and_ties(gc):
    g = gg.erdos_renyi(2000, 12, 5)
    rng = np.random.default_rng(2)
    for prio in (rng.integers(0, 1 << 32, g.n, dtype=np.uint64).astype(np.uint32),
                 rng.integers(0, 4, g.n).astype(np.uint32)):     # many ties: gid decides
        ref = oracle.color_d1(g, prio=prio)
        p = torch.from_numpy(prio.view(np.int32)).cuda()
        got, st = run_d1(gc, g, prio=p)
        same(got, st, ref, "prio")


@pytest.mark.parametrize("stop", [1, 3])
def test_d1_partial_state_and_resume(gc, stop):
    g = gg.rmat(11, 8, 9)
    full = oracle.color_d1(g, seed=4)
    part = oracle.color_d1(g, seed=4, max_rounds=stop)
    got, st = run_d1(gc, g, seed=4, params=gc.Params(max_rounds=stop), allow_partial=True)
    assert not st.converged
    assert np.array_equal(got, part.colors)
    init = torch.from_numpy(part.colors).cuda()
    got2, st2 = run_d1(gc, g, seed=4, init_colors=init)
    assert np.array_equal(got2, full.colors)
    assert st2.rounds == full.rounds - stop


@pytest.mark.parametrize("dims", [(9, 7, 5), (20, 17, 13)])
def test_d1_stencil27(gc, dims):
    g = gg.stencil(dims, 27)
    ref = oracle.color_d1(g, seed=2)
    got, st = run_d1(gc, g, seed=2)
    same(got, st, ref, f"27pt {dims}")


# --------------------------------------------------------------------------- D2

@pytest.mark.parametrize("dims", [(5, 4, 3), (17, 13, 11)])
def test_d2_stencil7(gc, dims):
    g = gg.stencil(dims, 7)
    ref = oracle.color_d2(g, seed=1)
    for v in (None, BIN_VARIANTS[1], BIN_VARIANTS[2]):
        got, st = run_d2(gc, g, seed=1, params=params(gc, v))
        same(got, st, ref, f"D2 7pt {dims}")


@pytest.mark.parametrize("seed", range(3))
def test_d2_random(gc, seed):
    g = gg.rmat(10, 4, seed + 20)
    ref = oracle.color_d2(g, seed=seed)
    got, st = run_d2(gc, g, seed=seed, params=params(gc, BIN_VARIANTS[seed * 2 % len(BIN_VARIANTS)]))
    same(got, st, ref, "D2 rmat10")


def test_d2_special(gc):
    for g in (gg.star(300), gg.complete(1), gg.path(50), gg.csr_from_pairs(0, np.array([], np.int64),
                                                                             np.array([], np.int64))):
        ref = oracle.color_d2(g, seed=9)
        got, st = run_d2(gc, g, seed=9)
        same(got, st, ref, "D2 special")


# -------------------------------------------------------------------------- PD2

@pytest.mark.parametrize("seed", range(3))
def test_pd2_powerlaw(gc, seed):
    b = gg.bipartite_powerlaw(20000, 5000, 8, 2.1, seed)
    ref = oracle.color_pd2(b, seed=seed)
    for v in (None, BIN_VARIANTS[1], BIN_VARIANTS[5]):
        got, st = run_pd2(gc, b, seed=seed, params=params(gc, v))
        same(got, st, ref, "PD2")


def test_pd2_square_pattern_and_single_row(gc):
    b = gg.square_pattern_bipartite(gg.erdos_renyi(3000, 6, 2))
    ref = oracle.color_pd2(b, seed=2)
    got, st = run_pd2(gc, b, seed=2)
    same(got, st, ref, "PD2 square")
    b1 = gg.bipartite_from_dense(np.ones((1, 100), dtype=bool))
    ref1 = oracle.color_pd2(b1, seed=2)
    got1, st1 = run_pd2(gc, b1, seed=2)
    same(got1, st1, ref1, "PD2 single row")


def test_pd2_heavy_columns(gc):
    """Columns in more than 1024 rows: the incremental engine builds their
    two-hop lists as duplicate-free sets through bitmaps."""
    rng = np.random.default_rng(5)
    n_rows, n_cols = 3000, 4000
    a = np.zeros((n_rows, n_cols), dtype=bool)
    a[:, 0] = True        # column 0 in every row
    a[:1500, 1] = True    # column 1 in half of them
    for r in range(n_rows):
        a[r, 2 + rng.choice(n_cols - 2, 3, replace=False)] = True
    b = gg.bipartite_from_dense(a)
    ref = oracle.color_pd2(b, seed=4)
    got, st = run_pd2(gc, b, seed=4)
    same(got, st, ref, "PD2 heavy columns")


def test_d2_heavy_vertex(gc):
    """A vertex of degree 1025 (its two-hop list built as a bitmap set by the
    incremental engine) whose leaves also form a path: a D2 clique of 1026."""
    leaves = 1025
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, leaves)]
    g = gg.from_edge_list(leaves + 1, edges)
    ref = oracle.color_d2(g, seed=6)
    got, st = run_d2(gc, g, seed=6)
    same(got, st, ref, "D2 heavy vertex")


# ------------------------------------------------------------------------ ghost

def _ghost_case(seed, layers, n=20000, parts=4):
    g = gg.rmat(int(np.log2(n)) + 1, 8, seed)
    owner = gg.hash_partition(g.n, parts, seed)
    gcol = gg.ghost_colors_uniform(g.n, int(g.degrees().max()), seed + 1)
    return gg.ghost_local_graph(g, owner, 0, layers, gcol)


@pytest.mark.parametrize("layers", [1, 2])
@pytest.mark.parametrize("seed", [1, 2])
def test_ghost_parity(gc, layers, seed):
    lg = _ghost_case(seed, layers)
    ref = oracle.color_d1_ghost(lg, seed=seed)
    for v in (None, BIN_VARIANTS[1]):
        colors, rl, st = gc.color_d1_ghost(lg.n_owned, lg.n_ghost, lg.layers, lg.n_g1, dev(lg.row_ptr),
                                           dev(lg.col), dev(lg.gid), dev(lg.ghost_colors), seed=seed,
                                           params=params(gc, v), trace_cap=4096)
        torch.cuda.synchronize()
        assert np.array_equal(colors.cpu().numpy(), ref.colors)
        assert np.array_equal(rl.cpu().numpy(), ref.remote_loser)
        assert st.boundary_conflicts == ref.boundary_conflicts
        assert st.remote_losers == ref.remote_losers
        assert st.rounds == ref.rounds
        assert st.num_colors == ref.num_colors


def test_ghost_many_conflicts(gc):
    lg = _ghost_case(3, 1)
    lg.ghost_colors = np.random.default_rng(3).integers(1, 3, lg.n_ghost).astype(np.int32)
    ref = oracle.color_d1_ghost(lg, seed=3)
    colors, rl, st = gc.color_d1_ghost(lg.n_owned, lg.n_ghost, 1, 0, dev(lg.row_ptr), dev(lg.col),
                                       dev(lg.gid), dev(lg.ghost_colors), seed=3)
    assert np.array_equal(colors.cpu().numpy(), ref.colors)
    assert np.array_equal(rl.cpu().numpy(), ref.remote_loser)
    assert st.boundary_conflicts == ref.boundary_conflicts > 100


# ------------------------------------------------------------------- validation

def test_validate_rejects_bad_graphs(gc):
    g = gg.erdos_renyi(500, 6, 1)
    P = gc.Params(flags=gc.COLOR_FLAG_VALIDATE)
    got, st = run_d1(gc, g, seed=1, params=P)   # a good graph passes
    assert np.array_equal(got, oracle.color_d1(g, seed=1).colors)
    bad = g.col.copy()
    bad[10] = g.n + 5                              # out of range
    with pytest.raises(gc.ColorError) as e:
        gc.color_d1(dev(g.row_ptr), dev(bad), params=P)
    assert e.value.code == -2
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    asym = gg.csr_from_pairs(g.n, src[:-1], g.col[:-1], False)  # drop one direction
    with pytest.raises(gc.ColorError):
        gc.color_d1(dev(asym.row_ptr), dev(asym.col), params=P)
    loop = g.col.copy()
    loop[g.row_ptr[3]] = 3                         # self-loop
    with pytest.raises(gc.ColorError):
        gc.color_d1(dev(g.row_ptr), dev(loop), params=P)
    b = gg.bipartite_powerlaw(300, 100, 4, 2.1, 1)
    got, st = run_pd2(gc, b, seed=1, params=P)
    assert np.array_equal(got, oracle.color_pd2(b, seed=1).colors)
    ri = b.row_idx.copy()
    ri[0], ri[1] = ri[1], ri[0]
    with pytest.raises(gc.ColorError):
        gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(ri), params=P)


def test_streams_are_independent(gc):
    g1 = gg.erdos_renyi(5000, 10, 1)
    g2 = gg.rmat(12, 8, 2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c1, _ = gc.color_d1(dev(g1.row_ptr), dev(g1.col), seed=1, stream=s,
                            params=gc.Params(engine=ENGINE["id"]))
    c2, _ = gc.color_d1(dev(g2.row_ptr), dev(g2.col), seed=2, params=gc.Params(engine=ENGINE["id"]))
    torch.cuda.synchronize()
    assert np.array_equal(c1.cpu().numpy(), oracle.color_d1(g1, seed=1).colors)
    assert np.array_equal(c2.cpu().numpy(), oracle.color_d1(g2, seed=2).colors)


# ------------------------------------------------------------ larger graphs

@pytest.mark.parametrize("split_hi", [65536, 2048, 512])
def test_d1_rmat18_heavy_bins(gc, split_hi):
    """R-MAT scale 18 (hubs of degree ~10^4): block and split bins at scale."""
    g = gg.rmat(18, 16, 5)
    ref = oracle.color_d1(g, seed=3)
    P = gc.Params(bin_hi=(12, 96, min(2048, split_hi // 2), split_hi), split_chunks=16)
    for rep in range(2):
        got, st = run_d1(gc, g, seed=3, params=P)
        same(got, st, ref, f"rmat18 split>{split_hi} rep {rep}")


def test_pd2_medium(gc):
    b = gg.bipartite_powerlaw(100000, 25000, 8, 2.1, 4)
    ref = oracle.color_pd2(b, seed=5)
    got, st = run_pd2(gc, b, seed=5)
    same(got, st, ref, "PD2 100k x 25k")


def test_device_buffers_rewritten_between_calls(gc):
    """The same device buffers hold a different graph on each call, rewritten
    by device-side copies right before the call (as a batching or serving
    caller recycling its buffers would do)."""
    graphs = [gg.rmat(13, 8, s) for s in range(4)]
    nmax = max(g.n for g in graphs)
    emax = max(g.nnz for g in graphs)
    rp_buf = torch.zeros(nmax + 1, dtype=torch.int32, device="cuda")
    ci_buf = torch.zeros(emax, dtype=torch.int32, device="cuda")
    out = torch.zeros(nmax, dtype=torch.int32, device="cuda")
    for rep in range(3):
        for i, g in enumerate(graphs):
            src_rp, src_ci = dev(g.row_ptr), dev(g.col)
            rp_buf[:g.n + 1].copy_(src_rp)
            ci_buf[:g.nnz].copy_(src_ci)
            c, st = gc.color_d1(rp_buf[:g.n + 1], ci_buf[:g.nnz], seed=i + 1, out=out[:g.n],
                                params=gc.Params(engine=ENGINE["id"]))
            torch.cuda.synchronize()
            assert np.array_equal(c.cpu().numpy(), oracle.color_d1(g, seed=i + 1).colors), (rep, i)


def test_library_engine_choice(gc):
    """The library's own choice: pull on regular meshes, incremental on skewed
    graphs and on long two-hop walks; both give the oracle's coloring."""
    for g, want in ((gg.stencil((24, 20, 16), 27), 1), (gg.rmat(14, 16, 2), 2)):
        colors, st = gc.color_d1(dev(g.row_ptr), dev(g.col), seed=5)
        assert st.engine == want
        assert np.array_equal(colors.cpu().numpy(), oracle.color_d1(g, seed=5).colors)
    # D2: short two-hop walks (7-point stencil) pull, long ones (ER, mean degree 20) incremental
    for g, want in ((gg.stencil((20, 18, 16), 7), 1), (gg.erdos_renyi(1500, 20.0, 4), 2)):
        colors, st = gc.color_d2(dev(g.row_ptr), dev(g.col), seed=5)
        assert st.engine == want
        assert np.array_equal(colors.cpu().numpy(), oracle.color_d2(g, seed=5).colors)


def test_concurrent_calls_on_two_streams(gc):
    """Two host threads color different graphs on two streams at the same
    time (each call holds its own workspace from the per-device pool); both
    results equal the oracle, repeated so that the calls overlap."""
    import threading
    a = gg.rmat(16, 16, 4)
    b = gg.bipartite_powerlaw(60000, 15000, 8, 2.1, 3)
    ra = oracle.color_d1(a, seed=2)
    rb = oracle.color_pd2(b, seed=2)
    da = (dev(a.row_ptr), dev(a.col))
    db = (dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx))
    torch.cuda.synchronize()
    errors = []

    def work(which):
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                for _ in range(6):
                    if which == 0:
                        c, st = gc.color_d1(*da, seed=2, stream=s, params=gc.Params(engine=ENGINE["id"]))
                        ok = np.array_equal(c.cpu().numpy(), ra.colors) and st.rounds == ra.rounds
                    else:
                        c, st = gc.color_pd2(*db, seed=2, stream=s, params=gc.Params(engine=ENGINE["id"]))
                        ok = np.array_equal(c.cpu().numpy(), rb.colors) and st.rounds == rb.rounds
                    if not ok:
                        errors.append(which)
        except Exception as ex:  # noqa: BLE001 - reported below
            errors.append(repr(ex))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert not errors, errors
