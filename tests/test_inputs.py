"""The seeded input generators against the workload recipes they stand for:
mesh sizes by closed form, the R-MAT and Erdos-Renyi preprocessing (no
self-loops, no duplicates, symmetric), the power-law pattern's exact row
length and column-degree tail, the batch/serve stream's kind and family mix,
size distribution and Poisson arrivals, and the partition and ghost-color
helpers of the distributed inputs.  None of this is the method's arithmetic:
the generators only produce the arrays both sides are given."""
import math

import numpy as np
import pytest

import graphgen as gg


def stencil_entries(dims, points):
    """Directed CSR entries of a non-periodic stencil mesh, counted from the
    offsets: along offset o there are prod(d_i - |o_i|) neighbour pairs, and
    each pair is stored once per endpoint."""
    dims = tuple(dims) + (1,) * (3 - len(dims))
    rng3 = (-1, 0, 1)
    if points in (5, 9):
        offs = [(dx, dy, 0) for dx in rng3 for dy in rng3 if (dx, dy) != (0, 0)]
    else:
        offs = [(dx, dy, dz) for dx in rng3 for dy in rng3 for dz in rng3 if (dx, dy, dz) != (0, 0, 0)]
    if points in (5, 7):
        offs = [o for o in offs if sum(map(abs, o)) == 1]
    total = 0
    for o in offs:
        total += math.prod(max(d - abs(x), 0) for d, x in zip(dims, o))
    return total


def test_bench_mesh_sizes():
    # the 27-point 128^3 D1 mesh and the 7-point 96^3 D2 mesh
    assert stencil_entries((128, 128, 128), 27) == 53_645_816
    assert stencil_entries((96, 96, 96), 7) == 5_253_120


@pytest.mark.parametrize("dims,points", [((7, 5, 3), 27), ((4, 3, 2), 7), ((9, 4), 9), ((6, 11), 5),
                                         ((20, 21, 19), 27), ((17, 13, 11), 7)])
def test_stencil_matches_closed_form(dims, points):
    g = gg.stencil(dims, points)
    gg.check_csr(g)
    assert g.n == math.prod(dims)
    assert g.nnz == stencil_entries(dims, points)
    if min(dims) >= 3:   # there is an interior vertex, with every neighbour
        assert g.degrees().max() == points - 1


def test_rmat_preprocessing_and_skew():
    g = gg.rmat(12, 16, seed=3)
    gg.check_csr(g)   # symmetric, sorted, no self-loops, no duplicates
    assert g.n == 1 << 12
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()   # the power-law head the R-MAT parameters give
    assert (deg == 0).any()              # isolated vertices are kept
    h = gg.rmat(12, 16, seed=3)
    assert np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col, h.col)
    k = gg.rmat(12, 16, seed=4)
    assert not (k.nnz == g.nnz and np.array_equal(k.col, g.col))


def test_erdos_renyi_mean_degree():
    g = gg.erdos_renyi(20_000, 16.0, 7)
    gg.check_csr(g)
    # G(n, p): the edge count is binomial, its standard deviation is about
    # 0.03 % of the mean here
    assert abs(g.nnz / g.n - 16.0) < 0.1


def test_powerlaw_pattern_rows_and_tail():
    b = gg.bipartite_powerlaw(200_000, 50_000, 8, 2.1, seed=2)
    assert np.array_equal(np.diff(b.row_ptr), np.full(b.n_rows, 8))
    cols = b.col_idx.reshape(b.n_rows, 8)
    assert (np.diff(cols, axis=1) > 0).all()          # distinct, sorted
    assert cols.min() >= 0 and cols.max() < b.n_cols
    # the CSC is the transpose of the CSR
    rows = np.repeat(np.arange(b.n_rows), 8)
    order = np.lexsort((rows, b.col_idx))
    assert np.array_equal(b.row_idx, rows[order])
    assert np.array_equal(np.diff(b.col_ptr), np.bincount(b.col_idx, minlength=b.n_cols))
    # column degrees against their rank follow the Zipf weights
    # (j+1)^(-1/(gamma-1)): slope -1/1.1 on a log-log scale, away from the
    # head (where a row's distinct columns cap the degree) and the tail
    # (where counts are small)
    d = np.sort(np.diff(b.col_ptr))[::-1].astype(np.float64)
    r = np.arange(30, 3000)
    slope = np.polyfit(np.log(r + 1), np.log(d[r]), 1)[0]
    assert abs(slope + 1 / 1.1) < 0.06, slope


def test_job_stream_mix_sizes_and_arrivals():
    jobs = gg.job_stream(3000, seed=11, n_min=100, n_max=400, rate=50.0)
    kinds = np.array([j.kind for j in jobs])
    fams = np.array([j.family for j in jobs])
    for k, p in ((1, 0.7), (2, 0.2), (3, 0.1)):
        assert abs((kinds == k).mean() - p) < 0.03, (k, (kinds == k).mean())
    for f in ("er", "stencil", "rmat"):
        assert abs((fams == f).mean() - 1 / 3) < 0.03, (f, (fams == f).mean())
    assert set(fams[kinds != 1]) <= {"er", "stencil"}   # D2/PD2 never on R-MAT
    assert all((j.pattern is not None) == (j.kind == 3) for j in jobs)
    # ER jobs keep the drawn size: log-uniform on [n_min, n_max]
    n_er = np.array([j.graph.n for j in jobs if j.family == "er"])
    assert n_er.min() >= 100 and n_er.max() <= 400
    assert abs((n_er < math.sqrt(100 * 400)).mean() - 0.5) < 0.05
    # Poisson arrivals: nondecreasing, mean gap 1/rate
    t = np.array([j.arrival for j in jobs])
    assert (np.diff(t) >= 0).all()
    assert abs(np.diff(t).mean() * 50.0 - 1.0) < 0.06
    for j in jobs[:200]:
        gg.check_csr(j.graph)


def test_hash_partition_and_ghost_colors():
    own = gg.hash_partition(100_000, 16, 5)
    counts = np.bincount(own, minlength=16)
    assert own.min() >= 0 and own.max() < 16
    assert abs(counts / (100_000 / 16) - 1).max() < 0.05
    assert np.array_equal(own, gg.hash_partition(100_000, 16, 5))
    assert not np.array_equal(own, gg.hash_partition(100_000, 16, 6))
    gc = gg.ghost_colors_uniform(50_000, 9, 3)
    assert gc.min() == 1 and gc.max() == 10           # [1, Delta + 1]
    assert abs(np.bincount(gc)[1:] / (50_000 / 10) - 1).max() < 0.1
