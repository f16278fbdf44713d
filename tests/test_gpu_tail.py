"""The incremental engine's cooperative tail kernel (all remaining rounds in
one launch, grid barriers between the color and detect steps) against the
per-round launches (COLOR_FLAG_NO_TAIL) and the oracle: identical colorings,
round counts, visit counts and per-round worklist sizes wherever the switch
happens, identical partial states at a round cap inside the tail, resume from
initial colors, and small grids."""
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


def run(gc, kind, graph, seed, params, **kw):
    if kind == "pd2":
        b = graph
        c, st = gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx), seed=seed,
                             params=params, trace_cap=4096, **kw)
    elif kind == "d2":
        c, st = gc.color_d2(dev(graph.row_ptr), dev(graph.col), seed=seed, params=params, trace_cap=4096, **kw)
    else:
        c, st = gc.color_d1(dev(graph.row_ptr), dev(graph.col), seed=seed, params=params, trace_cap=4096, **kw)
    torch.cuda.synchronize()
    return c.cpu().numpy(), st


def oracle_of(kind, graph, seed, **kw):
    if kind == "pd2":
        return oracle.color_pd2(graph, seed=seed, **kw)
    if kind == "d2":
        return oracle.color_d2(graph, seed=seed, **kw)
    return oracle.color_d1(graph, seed=seed, **kw)


CASES = {
    "rmat15_d1": ("d1", lambda: gg.rmat(15, 16, seed=3)),
    "er_d2": ("d2", lambda: gg.erdos_renyi(4000, 12.0, 5)),
    "stencil7_d2": ("d2", lambda: gg.stencil((17, 13, 11), 7)),
    "powerlaw_pd2": ("pd2", lambda: gg.bipartite_powerlaw(20_000, 6_000, 6, 2.1, seed=2)),
}


def same_run(a, sa, b, sb, what):
    assert np.array_equal(a, b), f"{what}: colors differ"
    # (list_visits, pushes and the byte counts are not compared: how much of a
    # loser's list its compaction drops depends on which neighbours committing
    # in the same round it already sees, which varies from run to run)
    for f in ("rounds", "num_colors", "vertex_visits", "edge_visits"):
        assert getattr(sa, f) == getattr(sb, f), f"{what}: {f} {getattr(sa, f)} vs {getattr(sb, f)}"
    assert sa.worklist == sb.worklist, what
    assert (sa.tail_bytes > 0) == (sa.tail_rounds > 0)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("threshold", [1, 1 << 30], ids=["last-vertex", "all-rounds"])
def test_tail_matches_per_round_and_oracle(gc, case, threshold):
    kind, make = CASES[case]
    g = make()
    ref = oracle_of(kind, g, 7)
    base, sb = run(gc, kind, g, 7, gc.Params(engine=2, flags=gc.COLOR_FLAG_NO_TAIL))
    got, st = run(gc, kind, g, 7, gc.Params(engine=2, tail_threshold=threshold))
    assert sb.tail_rounds == 0 and sb.tail_bytes == 0
    assert np.array_equal(got, ref.colors), f"{case}: colors differ from the oracle's"
    assert st.rounds == ref.rounds and st.worklist == list(ref.worklist)[:len(st.worklist)]
    same_run(got, st, base, sb, case)
    if threshold == 1 << 30:
        assert st.tail_rounds == st.rounds and st.color_launches == 0


def test_tail_mid_run_switch(gc):
    """Per-round launches first, the tail kernel for the rest: same results,
    and the switch does happen part-way on these graphs."""
    mid = 0
    for case in sorted(CASES):
        kind, make = CASES[case]
        g = make()
        ref = oracle_of(kind, g, 7)
        for threshold in (500, 2000):
            got, st = run(gc, kind, g, 7, gc.Params(engine=2, tail_threshold=threshold))
            assert np.array_equal(got, ref.colors), f"{case} threshold {threshold}"
            assert st.rounds == ref.rounds and st.worklist == list(ref.worklist)[:len(st.worklist)]
            assert st.vertex_visits == ref.vertex_visits and st.edge_visits == ref.edge_visits
            mid += 0 < st.tail_rounds < st.rounds
    assert mid >= 4, "the tail kernel never took over part-way"


@pytest.mark.parametrize("cap", [1, 2, 5])
def test_tail_round_cap_partial_state_and_resume(gc, cap):
    g = gg.rmat(12, 8, seed=9)
    full = oracle.color_d1(g, seed=4)
    part = oracle.color_d1(g, seed=4, max_rounds=cap)
    got, st = run(gc, "d1", g, 4, gc.Params(engine=2, max_rounds=cap, tail_threshold=1 << 30), allow_partial=True)
    assert not st.converged
    assert st.rounds == cap and st.tail_rounds == cap
    assert np.array_equal(got, part.colors)
    # resume inside the tail from the partial coloring (round 1 then reads
    # initial colors: no uniform shortcut)
    got2, st2 = run(gc, "d1", g, 4, gc.Params(engine=2, tail_threshold=1 << 30),
                    init_colors=torch.from_numpy(part.colors).cuda())
    assert np.array_equal(got2, full.colors)
    assert st2.rounds == full.rounds - cap


def test_tail_small_grid_and_timing(gc):
    g = gg.rmat(14, 16, seed=5)
    ref = oracle.color_d1(g, seed=2)
    for mw in (8, 24, 0):
        got, st = run(gc, "d1", g, 2, gc.Params(engine=2, max_workgroups=mw, tail_threshold=1 << 30,
                                                flags=gc.COLOR_FLAG_KERNEL_TIMING))
        assert np.array_equal(got, ref.colors), f"max_workgroups {mw}"
        assert st.rounds == ref.rounds and st.tail_rounds == ref.rounds
        assert st.tail_kernel_ns > 0 and st.color_kernel_ns == 0 and st.detect_kernel_ns == 0


def test_tail_repeated_calls_reuse_barrier_state(gc):
    """The barrier words and error flags are reset by every call: many calls
    in a row (of different sizes) all finish and agree with the oracle."""
    graphs = [gg.rmat(10 + (i % 4), 8, seed=i) for i in range(12)]
    for i, g in enumerate(graphs):
        ref = oracle.color_d1(g, seed=i)
        got, st = run(gc, "d1", g, i, gc.Params(engine=2))
        assert np.array_equal(got, ref.colors), f"graph {i}"
        assert st.tail_rounds >= 1


@pytest.mark.parametrize("name", list(CASES))
def test_tail_checkin_gives_up_and_rounds_continue(gc, name):
    """tail_checkin_us = -1: the tail kernel's workgroups never wait for each
    other, so every tail launch gives up at its entry check-in (forced from
    the host: every kernel still exits normally), changes nothing, and the
    remaining rounds run as per-round launches with the same result."""
    kind, make = CASES[name]
    g = make()
    ref = oracle_of(kind, g, 4)
    c, st = run(gc, kind, g, 4, gc.Params(engine=gc.ENGINE_INCREMENTAL, tail_checkin_us=-1))
    assert st.tail_fallbacks == 1 and st.tail_rounds == 0
    assert np.array_equal(c, ref.colors)
    assert st.rounds == ref.rounds and st.worklist == ref.worklist[:len(st.worklist)]
    assert st.vertex_visits == ref.vertex_visits and st.edge_visits == ref.edge_visits
    c2, st2 = run(gc, kind, g, 4, gc.Params(engine=gc.ENGINE_INCREMENTAL))
    assert st2.tail_fallbacks == 0 and st2.tail_rounds > 0
    assert np.array_equal(c2, ref.colors)


def test_tail_next_to_a_device_filling_batch_launch(gc):
    """A single-graph call with the tail kernel on one stream while another
    host thread runs the batched engine's persistent launch on another stream.
    Whether the tail's workgroups find each other resident or fall back to
    per-round launches depends on timing; either way both results equal the
    oracle."""
    import threading
    jobs_graphs = [gg.erdos_renyi(20000 + 1000 * i, 24, 10 + i) for i in range(24)]
    jobs = [dict(kind=gc.KIND_D1, row_ptr=dev(h.row_ptr), col_idx=dev(h.col), seed=1) for h in jobs_graphs]
    g = gg.rmat(17, 16, seed=5)
    rp, ci = dev(g.row_ptr), dev(g.col)
    torch.cuda.synchronize()
    out = {}

    def batch():
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            cols, _ = gc.color_batch(jobs, stream=s)
            s.synchronize()
            out["batch"] = [c.cpu().numpy() for c in cols]

    def single():
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            c, st = gc.color_d1(rp, ci, seed=3, stream=s, params=gc.Params(engine=gc.ENGINE_INCREMENTAL),
                                trace_cap=4096)
            s.synchronize()
            out["single"] = (c.cpu().numpy(), st)

    threads = [threading.Thread(target=batch), threading.Thread(target=single)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert "batch" in out and "single" in out
    ref = oracle.color_d1(g, seed=3)
    c, st = out["single"]
    assert np.array_equal(c, ref.colors) and st.rounds == ref.rounds
    assert st.tail_rounds > 0 or st.tail_fallbacks == 1
    for h, col in zip(jobs_graphs, out["batch"]):
        assert np.array_equal(col, oracle.color_d1(h, seed=1).colors)
