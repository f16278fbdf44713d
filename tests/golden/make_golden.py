#!/usr/bin/env python3
"""Writes the oracle's results on the full-size benchmark graphs as small
JSON summaries (a SHA-256 of the color array plus the round statistics), so
that GPU tests can check full-size runs without rerunning the slow oracle.

Calls only the CPU oracle and the seeded generators.  Usage (repo root):
    python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def sha(a, dtype=np.int32):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def summary(r, g_n, nnz, how):
    return {"how": how, "n": int(g_n), "nnz": int(nnz), "num_colors": int(r.num_colors), "rounds": int(r.rounds),
            "vertex_visits": int(r.vertex_visits), "edge_visits": int(r.edge_visits),
            "worklist": [int(x) for x in r.worklist],
            "colors_sha256": sha(r.colors)}


def _graph_case(how, make, kind):
    def run():
        g = make()
        r = {"d1": oracle.color_d1, "d2": oracle.color_d2}[kind](g, seed=1)
        return summary(r, g.n, g.nnz, how)
    return run


def _pd2_case():
    how = "gg.bipartite_powerlaw(4_000_000, 1_000_000, 8, 2.1, seed=1); oracle.color_pd2(b, seed=1)"
    b = gg.bipartite_powerlaw(4_000_000, 1_000_000, 8, 2.1, seed=1)
    r = oracle.color_pd2(b, seed=1)
    s = summary(r, b.n_cols, b.nnz, how)
    s["n_rows"] = int(b.n_rows)
    return s


def ghost_workload(scale=24):
    """The one-rank workload: R-MAT `scale` ef16 seed 1, 16-way hash
    partition (seed 7), ghost colors uniform in [1, maxdeg+1] (seed 11)."""
    g = gg.rmat(scale, 16, seed=1)
    delta = int(g.degrees().max())
    owner = gg.hash_partition(g.n, 16, seed=7)
    gcol = gg.ghost_colors_uniform(g.n, delta, seed=11)
    return g, owner, gcol, delta


def _ghost_cases(scale):
    """Both layer counts of part 0 from one generated graph."""
    how = (f"gg.rmat({scale}, 16, seed=1); owner = gg.hash_partition(n, 16, seed=7); "
           f"gc = gg.ghost_colors_uniform(n, maxdeg, seed=11); lg = gg.ghost_local_graph(g, owner, 0, L, gc, "
           f"sort_rows=False); oracle.color_d1_ghost(lg, seed=1)")
    g, owner, gcol, delta = ghost_workload(scale)
    out = {}
    for layers in (1, 2):
        lg = gg.ghost_local_graph(g, owner, 0, layers, gcol, sort_rows=False)
        t = time.time()
        r = oracle.color_d1_ghost(lg, seed=1)
        s = summary(r, lg.n_owned, lg.nnz, how.replace("L,", f"{layers},"))
        s.update({"n_ghost": int(lg.n_ghost), "n_g1": int(lg.n_g1), "owned_row_nnz": int(lg.row_ptr[lg.n_owned]),
                  "maxdeg": delta, "boundary_conflicts": int(r.boundary_conflicts),
                  "remote_losers": int(r.remote_losers), "remote_loser_sha256": sha(r.remote_loser, np.uint8),
                  "oracle_seconds": round(time.time() - t, 1)})
        out[f"rmat{scale}_part0_l{layers}"] = s
        del lg
    return out


CASES = {
    "rmat22_d1_seed1": _graph_case("gg.rmat(22, 16, seed=1); oracle.color_d1(g, seed=1)",
                                   lambda: gg.rmat(22, 16, seed=1), "d1"),
    "stencil7_96_d2_seed1": _graph_case("gg.stencil((96, 96, 96), 7); oracle.color_d2(g, seed=1)",
                                        lambda: gg.stencil((96, 96, 96), 7), "d2"),
    "stencil27_128_d1_seed1": _graph_case("gg.stencil((128, 128, 128), 27); oracle.color_d1(g, seed=1)",
                                          lambda: gg.stencil((128, 128, 128), 27), "d1"),
    "pd2_4m_1m_seed1": _pd2_case,
}
# cases that write several files from one run
MULTI = {"rmat24_part0": lambda: _ghost_cases(24)}


def write(name, s):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(s, f)
    print(name, s["num_colors"], s["rounds"], s.get("oracle_seconds"), flush=True)


def main():
    names = sys.argv[1:] or list(CASES) + list(MULTI)
    oracle.build()
    for name in names:
        t = time.time()
        if name in MULTI:
            for k, s in MULTI[name]().items():
                write(k, s)
            continue
        s = CASES[name]()
        s["oracle_seconds"] = round(time.time() - t, 1)
        write(name, s)


if __name__ == "__main__":
    main()
