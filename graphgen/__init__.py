"""Seeded synthetic input generators shared by the oracle tests, the GPU tests
and the benchmark.

This module builds graphs and nothing else: it holds none of the coloring
method's arithmetic (no priority hash, no first-fit, no conflict rule).  Every
array it returns is plain int32 CSR/CSC data (or a per-vertex input drawn from
a seeded numpy Generator), so the oracle and the GPU library consume the same
bytes without sharing any code.

Graph classes follow the paper's workload classes (Section 4, Table 1): PDE
meshes (3D stencils, standing in for the hexahedral weak-scaling meshes and
the SuiteSparse PDE matrices), power-law social/synthetic graphs (R-MAT,
standing in for kron_g500 / social networks) and a bipartite power-law pattern
for partial distance-2 coloring (standing in for Hamrle3 / patents of
Table 2).  The paper's preprocessing (no self-loops, no multi-edges,
Section 4) is applied to every generated graph.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph", "Bipartite", "csr_from_pairs", "erdos_renyi", "stencil", "rmat",
    "bipartite_powerlaw", "square_pattern_bipartite", "complete", "path",
    "star", "matching", "cycle", "mycielski", "from_edge_list", "hash_partition",
    "ghost_local_graph", "ghost_colors_uniform", "random_small_graph",
    "check_csr", "to_dense", "relabel",
]


@dataclass
class Graph:
    """Symmetric CSR graph: row_ptr int32[n+1], col int32[nnz], rows sorted."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


@dataclass
class Bipartite:
    """Sparse pattern A (n_rows x n_cols) in both CSR (rows) and CSC (cols)."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])


# ----------------------------------------------------------------------------
# CSR assembly
# ----------------------------------------------------------------------------

def csr_from_pairs(n: int, u: np.ndarray, v: np.ndarray, symmetrize: bool = True,
                   name: str = "") -> Graph:
    """CSR from an edge list; drops self-loops and duplicates (Section 4
    preprocessing), optionally symmetrizes, sorts every row."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if symmetrize:
        u, v = np.concatenate([u, v]), np.concatenate([v, u])
    key = u * np.int64(n) + v
    del u, v
    key = np.unique(key)
    src = (key // n).astype(np.int64)
    dst = (key % n).astype(np.int32)
    del key
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise OverflowError("nnz does not fit int32 offsets")
    return Graph(n, row_ptr.astype(np.int32), dst, name)


def from_edge_list(n: int, edges, name: str = "") -> Graph:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return csr_from_pairs(n, e[:, 0], e[:, 1], True, name)


def check_csr(g: Graph, symmetric: bool = True) -> None:
    """Input contract: monotone row_ptr, in-range sorted columns, no self-loops,
    no duplicates, symmetric adjacency."""
    rp, col, n = g.row_ptr.astype(np.int64), g.col.astype(np.int64), g.n
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == col.shape[0]
    assert np.all(np.diff(rp) >= 0)
    if col.size:
        assert col.min() >= 0 and col.max() < n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert not np.any(src == col), "self-loop"
    key = src * n + col
    assert np.all(np.diff(key) > 0), "unsorted row or duplicate edge"
    if symmetric:
        rkey = np.sort(col * n + src)
        assert np.array_equal(rkey, key), "asymmetric adjacency"


def to_dense(g: Graph) -> np.ndarray:
    a = np.zeros((g.n, g.n), dtype=bool)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[src, g.col] = True
    return a


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    return csr_from_pairs(g.n, perm[src], perm[g.col.astype(np.int64)], False, g.name)


# ----------------------------------------------------------------------------
# Small closed-form graphs (test inputs)
# ----------------------------------------------------------------------------

def complete(n: int) -> Graph:
    i, j = np.triu_indices(n, 1)
    return csr_from_pairs(n, i, j, True, f"K{n}")


def path(n: int) -> Graph:
    i = np.arange(n - 1)
    return csr_from_pairs(n, i, i + 1, True, f"P{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return csr_from_pairs(n, i, (i + 1) % n, True, f"C{n}")


def star(m: int) -> Graph:
    """K_{1,m}: centre 0, leaves 1..m."""
    return csr_from_pairs(m + 1, np.zeros(m, np.int64), np.arange(1, m + 1), True, f"S{m}")


def matching(pairs: int) -> Graph:
    i = np.arange(pairs) * 2
    return csr_from_pairs(2 * pairs, i, i + 1, True, f"M{pairs}")


def mycielski(k: int) -> Graph:
    """Mycielski graph M_k (M_2 = K_2): triangle-free with chromatic number k.
    From G on v_1..v_n add twins u_i adjacent to N(v_i) and a hub w adjacent to
    every u_i (the textbook construction)."""
    assert k >= 2
    n = 2
    edges = [(0, 1)]
    for _ in range(k - 2):
        new = list(edges)
        for (a, b) in edges:
            new.append((a, n + b))
            new.append((b, n + a))
        hub = 2 * n
        for i in range(n):
            new.append((n + i, hub))
        edges = new
        n = 2 * n + 1
    return from_edge_list(n, edges, f"Mycielski{k}")


def random_small_graph(n: int, p: float, rng: np.random.Generator) -> Graph:
    a = rng.random((n, n)) < p
    i, j = np.nonzero(np.triu(a, 1))
    return csr_from_pairs(n, i, j, True)


# ----------------------------------------------------------------------------
# Workload generators
# ----------------------------------------------------------------------------

def erdos_renyi(n: int, mean_degree: float, seed: int) -> Graph:
    """G(n, p) with p = mean_degree/(n-1): the number of edges is drawn from
    the binomial over all unordered pairs, then that many distinct pairs are
    drawn uniformly (exactly G(n, p))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = n * (n - 1) // 2
    p = mean_degree / (n - 1)
    m = int(rng.binomial(pairs, p))
    if pairs <= 1 << 27:
        idx = rng.choice(pairs, size=m, replace=False)
    else:  # large n: draw with replacement and redraw duplicates
        idx = np.unique(rng.integers(0, pairs, size=m, dtype=np.int64))
        while idx.size < m:
            extra = rng.integers(0, pairs, size=m - idx.size, dtype=np.int64)
            idx = np.unique(np.concatenate([idx, extra]))
    idx = np.asarray(idx, dtype=np.int64)
    # unrank pair index -> (i, j), i < j, row-major over the upper triangle
    i = (n - 2 - np.floor(np.sqrt(-8.0 * idx + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    start = i * (2 * n - i - 1) // 2
    # fix rounding at row boundaries
    lo = idx < start
    while np.any(lo):
        i[lo] -= 1
        start = i * (2 * n - i - 1) // 2
        lo = idx < start
    nxt = (i + 1) * (2 * n - i - 2) // 2
    hi = idx >= nxt
    while np.any(hi):
        i[hi] += 1
        start = i * (2 * n - i - 1) // 2
        nxt = (i + 1) * (2 * n - i - 2) // 2
        hi = idx >= nxt
    j = idx - start + i + 1
    return csr_from_pairs(n, i, j, True, f"ER(n={n},d={mean_degree})")


def stencil(dims, points: int) -> Graph:
    """Non-periodic stencil mesh.  dims = (X, Y) or (X, Y, Z); id = x + X*(y + Y*z).
    points: 5 / 9 for 2D, 7 / 27 for 3D.  Rows come out sorted because the
    offsets are visited in increasing linear-offset order."""
    dims = tuple(int(d) for d in dims)
    if len(dims) == 2:
        dims = dims + (1,)
        assert points in (5, 9)
        offs = [(dx, dy, 0) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (dx, dy) != (0, 0) and (points == 9 or abs(dx) + abs(dy) == 1)]
    else:
        assert points in (7, 27)
        offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (dx, dy, dz) != (0, 0, 0) and (points == 27 or abs(dx) + abs(dy) + abs(dz) == 1)]
    X, Y, Z = dims
    n = X * Y * Z
    offs.sort(key=lambda o: o[0] + X * (o[1] + Y * o[2]))
    ids = np.arange(n, dtype=np.int64)
    x = ids % X
    y = (ids // X) % Y
    z = ids // (X * Y)
    deg = np.zeros(n, dtype=np.int64)
    masks = []
    for (dx, dy, dz) in offs:
        m = (x + dx >= 0) & (x + dx < X) & (y + dy >= 0) & (y + dy < Y) & (z + dz >= 0) & (z + dz < Z)
        masks.append(m)
        deg += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    fill = row_ptr[:-1].copy()
    for (dx, dy, dz), m in zip(offs, masks):
        off = dx + X * (dy + Y * dz)
        src = ids[m]
        col[fill[src]] = (src + off).astype(np.int32)
        fill[src] += 1
    name = f"stencil{points}pt({'x'.join(str(d) for d in dims if d > 1 or len(dims) == 3)})"
    return Graph(n, row_ptr.astype(np.int32), col, name)


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, permute: bool = True, chunk: int = 1 << 24, progress=None) -> Graph:
    """R-MAT (Chakrabarti et al.) with m = edge_factor * 2^scale samples, no
    noise, a seeded vertex-id permutation (Graph500 practice), then the
    Section 4 preprocessing: self-loops dropped, symmetrized, deduplicated.
    Isolated vertices are kept."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << scale
    m = edge_factor * n
    ab, abc = a + b, a + b + c
    us, vs = [], []
    done = 0
    while done < m:
        k = min(chunk, m - done)
        u = np.zeros(k, dtype=np.int64)
        v = np.zeros(k, dtype=np.int64)
        for level in range(scale):
            r = rng.random(k, dtype=np.float32)
            bit = np.int64(1) << (scale - 1 - level)
            down = r >= ab          # quadrants c, d: source bit set
            right = ((r >= a) & (r < ab)) | (r >= abc)   # quadrants b, d: target bit set
            u += down * bit
            v += right * bit
        us.append(u)
        vs.append(v)
        done += k
        if progress:
            progress(f"rmat s{scale}: {done}/{m} samples")
    u = np.concatenate(us)
    v = np.concatenate(vs)
    del us, vs
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        u = perm[u]
        v = perm[v]
    if progress:
        progress(f"rmat s{scale}: building the CSR")
    return csr_from_pairs(n, u, v, True, f"RMAT(s={scale},ef={edge_factor})")


def _csc_from_csr(n_rows, n_cols, row_ptr, col_idx):
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(row_ptr.astype(np.int64)))
    order = np.lexsort((rows, col_idx.astype(np.int64)))
    row_idx = rows[order].astype(np.int32)
    counts = np.bincount(col_idx, minlength=n_cols)
    col_ptr = np.zeros(n_cols + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    return col_ptr.astype(np.int32), row_idx


def bipartite_powerlaw(n_rows: int, n_cols: int, per_row: int, gamma: float, seed: int) -> Bipartite:
    """Sparse pattern with exactly per_row distinct columns per row, columns
    drawn from Zipf weights w_j ~ (j+1)^(-1/(gamma-1)) (column-degree tail
    exponent gamma), followed by a seeded column permutation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.arange(1, n_cols + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cols = np.searchsorted(cdf, rng.random((n_rows, per_row))).astype(np.int64)
    np.minimum(cols, n_cols - 1, out=cols)
    while True:
        cols.sort(axis=1)
        dup = np.zeros_like(cols, dtype=bool)
        dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        redraw = np.searchsorted(cdf, rng.random(nd)).astype(np.int64)
        cols[dup] = np.minimum(redraw, n_cols - 1)
    perm = rng.permutation(n_cols).astype(np.int64)
    cols = np.sort(perm[cols], axis=1).astype(np.int32)
    row_ptr = (np.arange(n_rows + 1, dtype=np.int64) * per_row).astype(np.int32)
    col_idx = cols.reshape(-1)
    col_ptr, row_idx = _csc_from_csr(n_rows, n_cols, row_ptr, col_idx)
    return Bipartite(n_rows, n_cols, row_ptr, col_idx, col_ptr, row_idx,
                     f"bipartite({n_rows}x{n_cols},{per_row}/row,gamma={gamma})")


def square_pattern_bipartite(g: Graph) -> Bipartite:
    """The bipartite graph B(V_s, V_t, E_B) of a square pattern: one bipartite
    edge per directed entry (Section 3.6).  Rows are the nets."""
    col_ptr, row_idx = _csc_from_csr(g.n, g.n, g.row_ptr, g.col)
    return Bipartite(g.n, g.n, g.row_ptr, g.col, col_ptr, row_idx, g.name + "-pattern")


def bipartite_from_dense(a: np.ndarray) -> Bipartite:
    a = np.asarray(a, dtype=bool)
    n_rows, n_cols = a.shape
    counts = a.sum(axis=1)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = np.nonzero(a)[1].astype(np.int32)
    col_ptr, row_idx = _csc_from_csr(n_rows, n_cols, row_ptr.astype(np.int32), col_idx)
    return Bipartite(n_rows, n_cols, row_ptr.astype(np.int32), col_idx, col_ptr, row_idx)


# ----------------------------------------------------------------------------
# Distributed share: partition + ghost layers (Section 2.4, Section 3.4)
# ----------------------------------------------------------------------------

def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea, Flood 2014) on uint64."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def hash_partition(n: int, parts: int, seed: int) -> np.ndarray:
    """owner(v) = splitmix64(v + seed*2^32) mod parts: a vertex-id hash partition."""
    v = np.arange(n, dtype=np.uint64) + (np.uint64(seed) << np.uint64(32))
    return (_splitmix64(v) % np.uint64(parts)).astype(np.int32)


def ghost_colors_uniform(n: int, delta: int, seed: int) -> np.ndarray:
    """Per-GID ghost colors, uniform over Delta+1 colors, 1-based: [1, Delta+1].
    Drawn per global id so every viewer sees the same color for a vertex."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(1, delta + 2, size=n, dtype=np.int64).astype(np.int32)


@dataclass
class LocalGraph:
    """One rank's local graph G_l = {V_l + V_g, E_l + E_g} in local ids:
    owned vertices [0, n_owned) in increasing GID order, then the first ghost
    layer G1, then (two layers) the second layer G2.  row_ptr has n_owned rows
    (one layer) or n_owned + n_g1 rows (two layers)."""
    n_owned: int
    n_ghost: int
    n_g1: int
    layers: int
    row_ptr: np.ndarray
    col: np.ndarray
    gid: np.ndarray
    ghost_colors: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def ghost_local_graph(g: Graph, owner: np.ndarray, part: int, layers: int,
                      global_colors: np.ndarray, sort_rows: bool = True) -> LocalGraph:
    assert layers in (1, 2)
    rp = g.row_ptr.astype(np.int64)
    owned = np.nonzero(owner == part)[0].astype(np.int64)
    n_o = owned.size
    deg = rp[owned + 1] - rp[owned]
    idx = np.repeat(rp[owned], deg) + (np.arange(deg.sum()) - np.repeat(np.cumsum(deg) - deg, deg))
    nbr = g.col[idx].astype(np.int64)
    g1 = np.unique(nbr[owner[nbr] != part])
    gids = [owned, g1]
    if layers == 2:
        d1 = rp[g1 + 1] - rp[g1]
        idx1 = np.repeat(rp[g1], d1) + (np.arange(d1.sum()) - np.repeat(np.cumsum(d1) - d1, d1))
        nbr1 = g.col[idx1].astype(np.int64)
        cand = np.unique(nbr1[owner[nbr1] != part])
        g2 = np.setdiff1d(cand, g1, assume_unique=True)
        gids.append(g2)
    gid = np.concatenate(gids)
    local = np.full(g.n, -1, dtype=np.int64)
    local[gid] = np.arange(gid.size)
    row_vertices = owned if layers == 1 else np.concatenate([owned, g1])
    d = rp[row_vertices + 1] - rp[row_vertices]
    ridx = np.repeat(rp[row_vertices], d) + (np.arange(d.sum()) - np.repeat(np.cumsum(d) - d, d))
    lcol = local[g.col[ridx].astype(np.int64)]
    assert np.all(lcol >= 0)
    if sort_rows:  # columns of every row in increasing local id
        src = np.repeat(np.arange(row_vertices.size, dtype=np.int64), d)
        order = np.lexsort((lcol, src))
        lcol = lcol[order]
    lcol = lcol.astype(np.int32)
    row_ptr = np.zeros(row_vertices.size + 1, dtype=np.int64)
    np.cumsum(d, out=row_ptr[1:])
    n_g = gid.size - n_o
    return LocalGraph(n_o, int(n_g), int(g1.size), layers, row_ptr.astype(np.int32), lcol,
                      gid.astype(np.int32), global_colors[gid[n_o:]].astype(np.int32))


def slab_partition(dims, parts: int) -> np.ndarray:
    """Block partition of a stencil mesh (id = x + X (y + Y z)) along its last
    axis into `parts` slabs of consecutive planes."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    z = np.arange(n, dtype=np.int64) // (n // dims[-1])
    return (z * parts // dims[-1]).astype(np.int32)


@dataclass
class LocalPattern:
    """One rank's share of a partial distance-2 problem: owned columns
    [0, n_owned) in increasing GID order, then ghost columns (columns that
    share a row with an owned column); the local rows are the rows touching
    an owned column.  col_ptr/row_idx: the owned columns' rows (local row
    ids); row_ptr/col_idx: the local rows' columns (local column ids)."""
    n_owned: int
    n_ghost: int
    n_rows: int
    col_ptr: np.ndarray
    row_idx: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    gid: np.ndarray
    ghost_colors: np.ndarray


def pd2_local_pattern(b: Bipartite, owner_cols: np.ndarray, part: int, global_colors: np.ndarray) -> LocalPattern:
    cp = b.col_ptr.astype(np.int64)
    owned = np.nonzero(owner_cols == part)[0].astype(np.int64)
    d = cp[owned + 1] - cp[owned]
    idx = np.repeat(cp[owned], d) + (np.arange(d.sum()) - np.repeat(np.cumsum(d) - d, d))
    rows_of_owned = b.row_idx[idx].astype(np.int64)
    lrows = np.unique(rows_of_owned)
    rp = b.row_ptr.astype(np.int64)
    rd = rp[lrows + 1] - rp[lrows]
    ridx = np.repeat(rp[lrows], rd) + (np.arange(rd.sum()) - np.repeat(np.cumsum(rd) - rd, rd))
    cols_of_rows = b.col_idx[ridx].astype(np.int64)
    ghosts = np.unique(cols_of_rows[owner_cols[cols_of_rows] != part])
    gid = np.concatenate([owned, ghosts])
    lcol = np.full(b.n_cols, -1, dtype=np.int64)
    lcol[gid] = np.arange(gid.size)
    lrow = np.full(b.n_rows, -1, dtype=np.int64)
    lrow[lrows] = np.arange(lrows.size)
    col_ptr = np.zeros(owned.size + 1, dtype=np.int64)
    np.cumsum(d, out=col_ptr[1:])
    row_ptr = np.zeros(lrows.size + 1, dtype=np.int64)
    np.cumsum(rd, out=row_ptr[1:])
    return LocalPattern(int(owned.size), int(ghosts.size), int(lrows.size), col_ptr.astype(np.int32),
                        lrow[rows_of_owned].astype(np.int32), row_ptr.astype(np.int32),
                        lcol[cols_of_rows].astype(np.int32), gid.astype(np.int32),
                        global_colors[ghosts].astype(np.int32))


def ghost_homes(locals_):
    """Where every rank's ghosts are owned: per rank (owner rank, index among
    that rank's owned vertices) as int32 arrays, found by global id."""
    gid = np.concatenate([lg.gid[:lg.n_owned].astype(np.int64) for lg in locals_])
    rank = np.concatenate([np.full(lg.n_owned, r, np.int64) for r, lg in enumerate(locals_)])
    idx = np.concatenate([np.arange(lg.n_owned, dtype=np.int64) for lg in locals_])
    order = np.argsort(gid)
    sorted_gid = gid[order]
    out = []
    for lg in locals_:
        g = lg.gid[lg.n_owned:].astype(np.int64)
        at = order[np.searchsorted(sorted_gid, g)]
        assert np.array_equal(gid[at], g), "a ghost is owned by no rank"
        out.append((rank[at].astype(np.int32), idx[at].astype(np.int32)))
    return out


# ---------------------------------------------------------------------------
# Stream of jobs for the batched and served forms
# ---------------------------------------------------------------------------

@dataclass
class JobSpec:
    """One job of a batch or served stream.  kind 1 = D1, 2 = D2, 3 = PD2
    (graph adjacency used as a square pattern); arrival in seconds."""
    kind: int
    family: str
    graph: Graph
    pattern: Bipartite | None
    seed: int
    arrival: float = 0.0


def job_stream(count: int, seed: int, n_min: int = 1_000, n_max: int = 1_000_000,
               rate: float | None = None) -> list:
    """count jobs.  n ~ log-uniform [n_min, n_max]; kind D1/D2/PD2 with
    probability 0.7/0.2/0.1; family in {ER (mean degree U{8..64}), stencil
    (2D 5/9-point or 3D 7/27-point, side = round(n^(1/dim))), R-MAT (scale =
    round(log2 n), edge factor U{8..16})}, each with probability 1/3 overall.
    D2 and PD2 jobs use the ER and stencil families only (a D2 coloring of a
    power-law graph needs at least max-degree + 1 rounds), so the kind is
    drawn first and a D1 job is R-MAT with probability (1/3) / 0.7 = 10/21,
    ER or stencil with 11/42 each; a D2/PD2 job is ER or stencil with 1/2
    each.  rate: Poisson arrivals (jobs/s), else all arrive at 0."""
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        u = rng.uniform()
        kind = 1 if u < 0.7 else (2 if u < 0.9 else 3)
        f = rng.uniform()
        if kind == 1:
            fam = "rmat" if f < 10 / 21 else ("er" if f < 10 / 21 + 11 / 42 else "stencil")
        else:
            fam = "er" if f < 0.5 else "stencil"
        gseed = int(rng.integers(0, 2**31 - 1))
        if fam == "er":
            g = erdos_renyi(n, float(rng.integers(8, 65)), gseed)
        elif fam == "stencil":
            pts = (5, 9, 7, 27)[int(rng.integers(0, 4))]
            dim = 2 if pts in (5, 9) else 3
            side = max(2, int(round(n ** (1.0 / dim))))
            g = stencil((side,) * dim, pts)
        else:
            g = rmat(max(4, int(round(math.log2(n)))), int(rng.integers(8, 17)), gseed)
        pat = square_pattern_bipartite(g) if kind == 3 else None
        if rate:
            t += float(rng.exponential(1.0 / rate))
        jobs.append(JobSpec(kind, fam, g, pat, seed=i + 1, arrival=t))
    return jobs
