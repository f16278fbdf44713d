"""GPU parity of the served form: jobs submitted to a continuous-batching
server (HBM-footprint admission, slots, epochs with parking) come back with
the same colorings as alone, also when the budget forces queueing and the
arena is reused many times."""
import time

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


def submit(srv, s):
    if s.kind == 3:
        b = s.pattern
        return srv.submit(3, b.row_ptr, b.col_idx, b.col_ptr, b.row_idx, seed=s.seed)
    return srv.submit(s.kind, s.graph.row_ptr, s.graph.col, seed=s.seed)


def ref_of(s):
    if s.kind == 3:
        return oracle.color_pd2(s.pattern, seed=s.seed)
    if s.kind == 2:
        return oracle.color_d2(s.graph, seed=s.seed)
    return oracle.color_d1(s.graph, seed=s.seed)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def single(gc, s):
    """The single-graph call of the job's kind (device arrays)."""
    if s.kind == 3:
        b = s.pattern
        c, st = gc.color_pd2(dev(b.row_ptr), dev(b.col_idx), dev(b.col_ptr), dev(b.row_idx), seed=s.seed)
    elif s.kind == 2:
        c, st = gc.color_d2(dev(s.graph.row_ptr), dev(s.graph.col), seed=s.seed)
    else:
        c, st = gc.color_d1(dev(s.graph.row_ptr), dev(s.graph.col), seed=s.seed)
    return c.cpu().numpy(), st


def oracle_ok(s, limit=1_000_000):
    g = s.graph
    if g.n == 0:
        return True
    d = g.nnz / g.n
    return (g.n * d if s.kind == 1 else g.n * d * (d + 1)) <= limit


def walk(s):
    """The server's estimate of a job's two-hop walk per visit."""
    g = s.graph
    d = g.nnz / max(g.n, 1)
    return d * (d + 1)  # square patterns: column and row degrees are the vertex degrees


def footprint(s):
    """An upper bound of the server's arena bytes for the job: CSR (+CSC),
    colors, and the batched engine's 16 bytes per vertex, or for a heavy-lane
    job the single-graph incremental engine's buffers (two list arrays of
    the two-hop walk, bitsets, worklists and per-vertex arrays)."""
    g = s.graph
    nnz = g.nnz
    b = 4 * (g.n + 1) + 4 * nnz + 4 * g.n + 16 * g.n
    if s.kind == 3:
        b += 4 * (g.n + 1) + 4 * nnz
    if s.kind != 1 and walk(s) >= 128:
        deg = np.diff(g.row_ptr).astype(np.int64)
        walk_entries = int((deg * deg).sum()) + nnz
        b += 9 * walk_entries + 200 * g.n + (1 << 20)
    return b


def test_server_queueing_and_reuse_match_oracle(gc):
    specs = gg.job_stream(40, seed=5, n_min=100, n_max=6_000)
    budget = 3 * max(footprint(s) for s in specs) + (1 << 20)
    srv = gc.ColorServer(budget, max_slots=6)
    try:
        ids, codes = [], []
        for s in specs:
            jid, rc = submit(srv, s)
            ids.append(jid)
            codes.append(rc)
        assert gc.COLOR_EQUEUED in codes  # the budget and slots force waiting
        pending = dict(zip(ids, specs))
        done = {}
        deadline = time.monotonic() + 60.0
        while pending and time.monotonic() < deadline:
            for jid in list(pending):
                r = srv.poll(jid)
                if r is not None:
                    done[jid] = r
                    del pending[jid]
        assert not pending, "jobs never finished: " + ", ".join(
            f"{j} ({s.family} kind {s.kind} n={s.graph.n})" for j, s in pending.items())
        engines = {done[j][1].engine for j in ids}
        assert gc.ENGINE_BATCH in engines
        if any(s.kind != 1 and walk(s) >= 128 for s in specs):  # long two-hop walks: the heavy lane
            assert gc.ENGINE_INCREMENTAL in engines
        for jid, s in zip(ids, specs):
            colors, st = done[jid]
            ref = ref_of(s) if oracle_ok(s) else None
            if ref is None:  # too large for the oracle here: the single-graph call
                c1, ref = single(gc, s)
                ref.colors = c1
            assert np.array_equal(colors, ref.colors), f"job {jid} {s.family} kind {s.kind} n={s.graph.n}"
            assert st.rounds == ref.rounds and st.num_colors == ref.num_colors
            assert st.vertex_visits == ref.vertex_visits and st.edge_visits == ref.edge_visits
    finally:
        srv.close()


def test_server_mix_equals_alone(gc):
    """A job served among others equals the same job served alone."""
    specs = gg.job_stream(16, seed=8, n_min=1_000, n_max=40_000)
    srv = gc.ColorServer(1 << 30, max_slots=16)
    try:
        ids = [submit(srv, s)[0] for s in specs]
        srv.drain()
        mixed = [srv.poll(j) for j in ids]
        alone = []
        for s in specs:
            jid, _ = submit(srv, s)
            srv.drain()
            alone.append(srv.poll(jid))
        for (cm, sm), (ca, sa), s in zip(mixed, alone, specs):
            assert np.array_equal(cm, ca), f"{s.family} kind {s.kind} n={s.graph.n}"
            assert sm.rounds == sa.rounds
    finally:
        srv.close()


def test_server_errors(gc):
    srv = gc.ColorServer(1 << 16, max_slots=2)
    try:
        big = gg.stencil((64, 64), 9)
        with pytest.raises(gc.ColorError) as ei:
            srv.submit(1, big.row_ptr, big.col)
        assert ei.value.code == gc.COLOR_E2BIG
        srv._keep[12345] = 1  # an id the server never issued
        with pytest.raises(gc.ColorError) as ei:
            srv.poll(12345)
        assert ei.value.code == gc.COLOR_EINVAL
        # a job of 0 vertices completes with an empty coloring
        jid, _ = srv.submit(1, np.zeros(1, np.int32), np.zeros(0, np.int32))
        srv.drain()
        colors, st = srv.poll(jid)
        assert colors.size == 0 and st.rounds == 0
    finally:
        srv.close()


def test_server_heavy_job_within_budget(gc):
    """A heavy-lane job (dense D2: long two-hop walks) keeps the single-graph
    engine's lists inside the server's arena: a budget that fits its CSR but
    not its lists refuses it at submit (COLOR_E2BIG); a budget that fits both
    serves it, with the coloring of the plain call."""
    g = gg.erdos_renyi(3000, 48, 7)
    spec = gg.JobSpec(kind=2, family="er", graph=g, pattern=None, seed=3)
    assert walk(spec) >= 128
    small = 4 * (g.n + 1) + 4 * g.nnz + 4 * g.n + 16 * g.n + (1 << 16)
    srv = gc.ColorServer(small, max_slots=4)
    try:
        with pytest.raises(gc.ColorError) as ei:
            srv.submit(2, g.row_ptr, g.col, seed=3)
        assert ei.value.code == gc.COLOR_E2BIG
    finally:
        srv.close()
    srv = gc.ColorServer(footprint(spec) + (1 << 20), max_slots=4)
    try:
        jid, _ = srv.submit(2, g.row_ptr, g.col, seed=3)
        srv.drain()
        colors, st = srv.poll(jid)
        assert st.engine == gc.ENGINE_INCREMENTAL
        ref = oracle.color_d2(g, seed=3)
        assert np.array_equal(colors, ref.colors) and st.rounds == ref.rounds
    finally:
        srv.close()
