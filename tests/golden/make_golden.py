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


def summary(r, g_n, nnz, how):
    colors = np.ascontiguousarray(r.colors, dtype=np.int32)
    return {"how": how, "n": int(g_n), "nnz": int(nnz), "num_colors": int(r.num_colors), "rounds": int(r.rounds),
            "vertex_visits": int(r.vertex_visits), "edge_visits": int(r.edge_visits),
            "worklist": [int(x) for x in r.worklist],
            "colors_sha256": hashlib.sha256(colors.tobytes()).hexdigest()}


CASES = {
    "rmat22_d1_seed1": lambda: ("gg.rmat(22, 16, seed=1); oracle.color_d1(g, seed=1)",
                                gg.rmat(22, 16, seed=1), "d1"),
    "stencil7_96_d2_seed1": lambda: ("gg.stencil((96, 96, 96), 7); oracle.color_d2(g, seed=1)",
                                     gg.stencil((96, 96, 96), 7), "d2"),
    "stencil27_128_d1_seed1": lambda: ("gg.stencil((128, 128, 128), 27); oracle.color_d1(g, seed=1)",
                                       gg.stencil((128, 128, 128), 27), "d1"),
}


def main():
    names = sys.argv[1:] or list(CASES)
    oracle.build()
    for name in names:
        how, g, kind = CASES[name]()
        t = time.time()
        r = oracle.color_d1(g, seed=1) if kind == "d1" else oracle.color_d2(g, seed=1)
        s = summary(r, g.n, g.nnz, how)
        s["oracle_seconds"] = round(time.time() - t, 1)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(s, f)
        print(name, s["num_colors"], s["rounds"], s["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main()
