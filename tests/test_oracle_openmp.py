"""The oracle built with OpenMP (the benchmark's all-core CPU baseline) gives
the plain build's results: rounds are synchronous, so running the per-vertex
loops of a round on several threads cannot change colors or counters."""
import numpy as np
import pytest

import graphgen as gg
import oracle


def _same(a, b):
    assert np.array_equal(a.colors, b.colors)
    assert (a.rounds, a.num_colors, a.vertex_visits, a.edge_visits) == \
        (b.rounds, b.num_colors, b.vertex_visits, b.edge_visits)
    assert a.worklist == b.worklist


@pytest.mark.parametrize("degrees", [False, True])
def test_openmp_build_matches_plain_build(degrees):
    assert oracle.threads() == 1
    for g in (gg.rmat(15, 16, 1), gg.stencil((40, 40, 40), 27), gg.erdos_renyi(30000, 12, 2)):
        _same(oracle.color_d1(g, seed=3, recolor_degrees=degrees),
              oracle.color_d1(g, seed=3, recolor_degrees=degrees, omp=True))
    g = gg.stencil((30, 30, 30), 7)
    _same(oracle.color_d2(g, seed=2, recolor_degrees=degrees),
          oracle.color_d2(g, seed=2, recolor_degrees=degrees, omp=True))
    b = gg.bipartite_powerlaw(40000, 10000, 8, 2.1, 1)
    _same(oracle.color_pd2(b, seed=1, recolor_degrees=degrees),
          oracle.color_pd2(b, seed=1, recolor_degrees=degrees, omp=True))
