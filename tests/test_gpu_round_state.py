"""The state after every round, not only the final coloring (Section 3,
Algorithm 2's loop stopped after r rounds): with a round cap of r the
committed colors equal the oracle's after r rounds, for every r before the
last round, on D1, D2 and PD2 and on every engine: pull, incremental with
per-round launches, and incremental with its tail kernel running from the
first round (small rounds are where the tail hands light vertices to whole
workgroups).  The per-round worklist sizes agree up to the cap, and a few of
the partial states are resumed to the full coloring."""
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


def engine_params(gc, engine, **kw):
    if engine == "pull":
        return gc.Params(engine=gc.ENGINE_PULL, **kw)
    if engine == "incremental":
        return gc.Params(engine=gc.ENGINE_INCREMENTAL, flags=gc.COLOR_FLAG_NO_TAIL, **kw)
    return gc.Params(engine=gc.ENGINE_INCREMENTAL, tail_threshold=1 << 30, **kw)


CASES = {
    "rmat11_d1": ("d1", lambda: gg.rmat(11, 8, seed=9)),
    "er600_d2": ("d2", lambda: gg.erdos_renyi(600, 8.0, 3)),
    "powerlaw_pd2": ("pd2", lambda: gg.bipartite_powerlaw(3000, 800, 6, 2.1, seed=4)),
}


@pytest.mark.parametrize("engine", ["pull", "incremental", "tail"])
@pytest.mark.parametrize("case", list(CASES))
def test_state_after_every_round(gc, case, engine):
    kind, make = CASES[case]
    g = make()
    seed = 6
    full = oracle_of(kind, g, seed)
    R = full.rounds
    assert R >= 4, f"{case}: too few rounds to test ({R})"
    resume_at = {1, R // 2, R - 1}
    for cap in range(1, R):
        part = oracle_of(kind, g, seed, max_rounds=cap)
        got, st = run(gc, kind, g, seed, engine_params(gc, engine, max_rounds=cap), allow_partial=True)
        what = f"{case} {engine} cap {cap}"
        assert not st.converged, what
        assert np.array_equal(got, part.colors), what
        assert st.rounds == cap == part.rounds, what
        assert st.worklist == list(full.worklist)[:cap], what
        if cap in resume_at:
            got2, st2 = run(gc, kind, g, seed, engine_params(gc, engine), init_colors=dev(part.colors))
            assert np.array_equal(got2, full.colors), f"{what} resumed"
            assert st2.rounds == R - cap, f"{what} resumed"
    got, st = run(gc, kind, g, seed, engine_params(gc, engine, max_rounds=R))
    assert np.array_equal(got, full.colors) and st.rounds == R
