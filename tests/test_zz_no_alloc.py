"""The no-allocation entry point (color_d1_noalloc) against color_d1 through
the C-ABI: identical colors and statistics on two calls in a row, the second
on a smaller graph (the static scratch array keeps the first call's contents,
so whatever must start cleared is cleared by the call itself), and against
the oracle."""
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


def _both(gc, g, seed):
    rp, ci = dev(g.row_ptr), dev(g.col)
    a, sa = gc.color_d1_noalloc(rp, ci, seed=seed, trace_cap=4096)
    b, sb = gc.color_d1(rp, ci, seed=seed, trace_cap=4096)
    torch.cuda.synchronize()
    return a.cpu().numpy(), sa, b.cpu().numpy(), sb


def _same(a, sa, b, sb, what):
    assert np.array_equal(a, b), what
    assert (sa.num_colors, sa.rounds, sa.vertex_visits, sa.edge_visits) == \
        (sb.num_colors, sb.rounds, sb.vertex_visits, sb.edge_visits), what
    assert sa.worklist == sb.worklist, what


def test_noalloc_matches_color_d1_on_two_calls_second_smaller(gc):
    big = gg.rmat(19, 16, 3)          # hubs in the workgroup bin, ragged bins
    small = gg.erdos_renyi(10000, 16, 1)
    for g, seed, what in ((big, 2, "R-MAT 19"), (small, 1, "ER 10k")):
        a, sa, b, sb = _both(gc, g, seed)
        _same(a, sa, b, sb, what)
        ref = oracle.color_d1(g, seed=seed)
        assert np.array_equal(a, ref.colors), what
        assert sa.rounds == ref.rounds and sa.worklist == ref.worklist, what


def test_noalloc_limits(gc):
    g = gg.erdos_renyi(gc.NOALLOC_MAX_N, 4, 5)     # exactly the largest size
    a, sa, b, sb = _both(gc, g, 5)
    _same(a, sa, b, sb, "n = NOALLOC_MAX_N")
    n = gc.NOALLOC_MAX_N + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(gc.ColorError) as e:
        gc.color_d1_noalloc(rp, ci)
    assert e.value.code == gc.COLOR_ESCRATCH
    with pytest.raises(gc.ColorError) as e:
        gc.color_d1_noalloc(rp[:11], ci, params=gc.Params(flags=gc.COLOR_FLAG_RECOLOR_DEGREES))
    assert e.value.code == -1
