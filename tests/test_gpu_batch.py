"""GPU parity of the batched persistent form (color_batch) and its
autotuner: every job's coloring, rounds, visit counts and color count equal
the CPU oracle's (small jobs) and the single-graph call's (all jobs), for
mixed D1/D2/PD2 streams, degenerate jobs, every degree bin, and every tuned
mapping."""
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


def job_of(gc, spec):
    if spec.kind == gc.KIND_PD2:
        b = spec.pattern
        return {"kind": spec.kind, "row_ptr": dev(b.row_ptr), "col_idx": dev(b.col_idx),
                "col_ptr": dev(b.col_ptr), "row_idx": dev(b.row_idx), "seed": spec.seed}
    g = spec.graph
    return {"kind": spec.kind, "row_ptr": dev(g.row_ptr), "col_idx": dev(g.col), "seed": spec.seed}


def single(gc, spec):
    """The single-graph call of the job's kind."""
    if spec.kind == gc.KIND_PD2:
        b = spec.pattern
        c, st = gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx), seed=spec.seed)
    elif spec.kind == gc.KIND_D2:
        c, st = gc.color_d2(dev(spec.graph.row_ptr), dev(spec.graph.col), seed=spec.seed)
    else:
        c, st = gc.color_d1(dev(spec.graph.row_ptr), dev(spec.graph.col), seed=spec.seed)
    return c.cpu().numpy(), st


def ref_of(spec):
    if spec.kind == 3:
        return oracle.color_pd2(spec.pattern, seed=spec.seed)
    if spec.kind == 2:
        return oracle.color_d2(spec.graph, seed=spec.seed)
    return oracle.color_d1(spec.graph, seed=spec.seed)


def oracle_ok(spec, limit=3_000_000):
    """Small enough for the oracle: an estimate of its two-hop work."""
    g = spec.graph
    if g.n == 0:
        return True
    d = g.nnz / g.n
    walk = g.n * d if spec.kind == 1 else g.n * d * (d + 1)
    return g.n <= 5_000 and walk <= limit


def two_level_star(hubs, leaves):
    """A center joined to `hubs` hubs, each hub joined to `leaves` leaves."""
    edges = [(0, h) for h in range(1, hubs + 1)]
    nxt = hubs + 1
    for h in range(1, hubs + 1):
        for _ in range(leaves):
            edges.append((h, nxt))
            nxt += 1
    return gg.from_edge_list(nxt, edges)


def check_same(got, st, colors, ref_st, what):
    if not np.array_equal(got, colors):
        bad = np.nonzero(got != colors)[0]
        raise AssertionError(f"{what}: {bad.size} colors differ, first at {bad[:5]}")
    assert st.rounds == ref_st.rounds, f"{what}: rounds {st.rounds} vs {ref_st.rounds}"
    assert st.num_colors == ref_st.num_colors, what
    assert st.vertex_visits == ref_st.vertex_visits, what
    assert st.edge_visits == ref_st.edge_visits, what


def spec_d1(g, seed=1, kind=1):
    pat = gg.square_pattern_bipartite(g) if kind == 3 else None
    return gg.JobSpec(kind, "fixed", g, pat, seed=seed)


def test_batch_mixed_stream_vs_oracle_and_single(gc):
    specs = gg.job_stream(48, seed=11, n_min=50, n_max=20_000)
    outs, stats = gc.color_batch([job_of(gc, s) for s in specs])
    torch.cuda.synchronize()
    for i, (s, o, st) in enumerate(zip(specs, outs, stats)):
        got = o.cpu().numpy()
        what = f"job {i} kind {s.kind} {s.family} n={s.graph.n}"
        # jobs with long two-hop walks go to the single-graph incremental engine
        assert st.engine == gc.ENGINE_BATCH or (s.kind != 1 and st.engine == gc.ENGINE_INCREMENTAL)
        if oracle_ok(s):
            r = ref_of(s)
            check_same(got, st, r.colors, r, what + " vs oracle")
        c1, st1 = single(gc, s)
        check_same(got, st, c1, st1, what + " vs single-graph call")


def test_batch_degenerate_and_heavy_jobs(gc):
    specs = [
        spec_d1(gg.complete(1)),              # one vertex, no edges
        spec_d1(gg.Graph(0, np.zeros(1, np.int32), np.zeros(0, np.int32))),  # empty
        spec_d1(gg.erdos_renyi(300, 0.0, 3)),  # edgeless
        spec_d1(gg.complete(70)),               # K_70: 70 rounds
        spec_d1(gg.star(3000)),                 # hub of degree 3000: a workgroup vertex (bin 3)
        spec_d1(two_level_star(90, 100), kind=2),  # D2: the center's walk (9180) is a workgroup vertex
        spec_d1(gg.star(600), kind=3),          # PD2 over the star's square pattern
        spec_d1(gg.mycielski(6), seed=5),
        spec_d1(gg.path(1000), kind=2, seed=9),
        spec_d1(gg.stencil((13, 11, 7), 27), seed=4),
    ]
    outs, stats = gc.color_batch([job_of(gc, s) for s in specs])
    torch.cuda.synchronize()
    for i, (s, o, st) in enumerate(zip(specs, outs, stats)):
        r = ref_of(s)
        check_same(o.cpu().numpy(), st, r.colors, r, f"job {i} n={s.graph.n} kind {s.kind}")
        if s.graph.n == 0:
            assert st.rounds == 0 and st.num_colors == 0


def test_batch_empty_list(gc):
    outs, stats = gc.color_batch([])
    assert outs == [] and stats == []


def test_batch_workspace_reuse_and_order(gc):
    """Two different batches in a row, then the first again in reverse
    order: results depend only on each job."""
    a = gg.job_stream(12, seed=3, n_min=100, n_max=30_000)
    b = gg.job_stream(20, seed=4, n_min=100, n_max=8_000)
    oa, _ = gc.color_batch([job_of(gc, s) for s in a])
    ob, _ = gc.color_batch([job_of(gc, s) for s in b])
    oa2, _ = gc.color_batch([job_of(gc, s) for s in reversed(a)])
    torch.cuda.synchronize()
    for x, y in zip(oa, reversed(oa2)):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    for s, o in zip(b, ob):
        if oracle_ok(s, 1_000_000):
            assert np.array_equal(o.cpu().numpy(), ref_of(s).colors)


def test_batch_geometry_invariance(gc):
    """A grid of 8 workgroups gives the same colorings as the full grid."""
    specs = gg.job_stream(10, seed=21, n_min=500, n_max=20_000)
    full, sf = gc.color_batch([job_of(gc, s) for s in specs])
    small, ss = gc.color_batch([job_of(gc, s) for s in specs], params=gc.Params(max_workgroups=8))
    torch.cuda.synchronize()
    for x, y, a, b in zip(full, small, sf, ss):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        assert (a.rounds, a.vertex_visits, a.edge_visits) == (b.rounds, b.vertex_visits, b.edge_visits)


def test_batch_round_cap(gc):
    specs = [spec_d1(gg.complete(40)), spec_d1(gg.path(10))]
    with pytest.raises(gc.ColorError) as ei:
        gc.color_batch([job_of(gc, s) for s in specs], params=gc.Params(max_rounds=5))
    assert ei.value.code == gc.COLOR_ENOCONVERGE


def test_batch_validate_rejects_bad_graph(gc):
    g = gg.path(50)
    col = g.col.copy()
    col[3] = 3  # row 2 becomes [3, 3]: a duplicate, and the edge 1-2 loses its mirror
    bad = {"kind": 1, "row_ptr": dev(g.row_ptr), "col_idx": dev(col)}
    good = job_of(gc, spec_d1(gg.path(50)))
    with pytest.raises(gc.ColorError) as ei:
        gc.color_batch([good, bad], params=gc.Params(flags=gc.COLOR_FLAG_VALIDATE))
    assert ei.value.code == gc.COLOR_EGRAPH


def test_autotune_keeps_colorings(gc):
    """The autotuner compares every candidate's colors itself (EMISMATCH
    otherwise); after it records a mapping, batches still match the oracle."""
    gc.color_autotune_reset()
    er = spec_d1(gg.erdos_renyi(20_000, 24.0, 8), seed=2)
    p = gc.color_autotune(job_of(gc, er), reps=1)
    assert all(x in (1, 2, 4, 8, 16, 32, 64) for x in p.lanes)
    d2 = spec_d1(gg.stencil((20, 20, 20), 7), kind=2, seed=3)
    gc.color_autotune(job_of(gc, d2), reps=1)
    specs = [er, d2, spec_d1(gg.erdos_renyi(5_000, 20.0, 9), seed=4)]
    outs, stats = gc.color_batch([job_of(gc, s) for s in specs])
    torch.cuda.synchronize()
    for s, o, st in zip(specs, outs, stats):
        r = ref_of(s)
        check_same(o.cpu().numpy(), st, r.colors, r, f"tuned n={s.graph.n}")
    gc.color_autotune_reset()
