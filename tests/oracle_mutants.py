"""Mutation check of the oracle's pins.

Each mutant plants one plausible mistake in a copy of the oracle (its C
source or its Python driver of Algorithm 2), and the CPU pin suite must fail
on it.  Run from the repository root (no GPU needed):

    python tests/oracle_mutants.py             # every mutant, 4 at a time
    python tests/oracle_mutants.py -k ghost    # the mutants whose name has "ghost"

For each mutant the script copies oracle/, graphgen/ and tests/ into a
temporary directory, applies the change there, and runs
`pytest -x -m "not gpu"` on the oracle's pin files in that copy; the
repository itself is never modified.  The unmutated copy runs first and must
pass.  Exit status 1 if any mutant survives.  Not collected by pytest (its
name does not start with test_): it takes a few minutes.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_distributed.py",
             "tests/test_oracle_ghost_recolor.py", "tests/test_oracle_d2_ghost.py"]

C = "oracle/oracle.c"
PY = "oracle/__init__.py"

# (name, file, text to replace (must occur once), replacement, the mistake)
# A mutant listed in EQUIVALENT changes the code but not what it computes,
# for the reason given there: the pins must pass on it.
MUTANTS = [
    ("fmix32_shift", C, "h ^= h >> 13;", "h ^= h >> 12;",
     "a wrong shift in the MurmurHash3 finalizer"),
    ("seed_mix", C, "orc_fmix32(seed ^ 0x9E3779B9u)", "orc_fmix32(seed)",
     "the seed not mixed with the constant"),
    ("loser_direction", C, "return k->p[a] > k->p[b];", "return k->p[a] < k->p[b];",
     "the higher key loses (the paper's direction instead of the reading taken)"),
    ("tie_break", C, "return k->gid[a] > k->gid[b];", "return k->gid[a] < k->gid[b];",
     "ties of p broken toward the lower id"),
    ("degree_direction", C, "return k->deg[a] > k->deg[b];", "return k->deg[a] < k->deg[b];",
     "recolorDegrees recolors the higher-degree vertex"),
    ("pd2_degree_source", C, "g->kind == 3 ? g->col_ptr : g->row_ptr", "g->row_ptr",
     "a PD2 column's degree read from the row pointers"),
    ("d2_self_kept", C, "if (x != v) list_push(l, x);", "list_push(l, x);",
     "v itself left in its distance-2 neighbourhood"),
    ("d2_first_hop_dropped", C, "list_push(l, u);\n            visits++;", "visits++;",
     "the distance-1 neighbours left out of the distance-2 neighbourhood"),
    ("pd2_self_kept", C, "if (c != v) list_push(l, c);", "list_push(l, c);",
     "a column left in its own partial distance-2 neighbourhood"),
    ("d2_visits_hop2", C, "visits++;\n                if (x != v)", "if (x != v)",
     "second-hop entries not counted as edge visits"),
    ("first_fit_ignores_1", C, "if (c > 0 && c < m) used[c] = 1;", "if (c > 1 && c < m) used[c] = 1;",
     "first fit blind to color 1"),
    ("detect_committed_too", C, "if (!in_w[u]) continue;", "",
     "committed neighbours' stale tentative colors judged as conflicts"),
    ("detect_reads_committed", C, "if (T[u] == T[v] && key_greater", "if (colors[u] == T[v] && key_greater",
     "detect compares against committed instead of tentative colors"),
    ("color_reads_tentative", C, "T[v] = first_fit(&nbt, colors,", "T[v] = first_fit(&nbt, T,",
     "the color step reads this round's tentative colors (not the snapshot)"),
    ("trace_index", C, "st->worklist_trace[round0 + r - 1] = W.len", "st->worklist_trace[round0 + r] = W.len",
     "the worklist trace shifted by one round"),
    ("vertex_visits", C, "st->vertex_visits += W.len;", "st->vertex_visits += W.len - 1;",
     "vertex visits undercounted"),
    ("ghost_loser_direction", C, "if (key_greater(&rc.keys, u, v))\n                loser[v] = 1;",
     "if (key_greater(&rc.keys, v, u))\n                loser[v] = 1;",
     "D1 ghost step: the owned vertex loses to a lower-key ghost"),
    ("ghost_conflicts_uncounted", C,
     "if (owned_colors[v] != ghost_colors[u - n_owned]) continue;\n            if (st) st->boundary_conflicts++;",
     "if (owned_colors[v] != ghost_colors[u - n_owned]) continue;",
     "D1 ghost step: boundary conflicts not counted"),
    ("ghost_phase3_blind", C, "rc.ignore_from = m;\n        r3 = run_rounds", "rc.ignore_from = n_owned;\n        r3 = run_rounds",
     "D1 ghost step: phase 3 ignores the ghosts' colors"),
    ("ghost_recolor_keeps_loser_color", C, "local[n_owned + j] = glose[j] ? 0 : ghost_colors[j];",
     "local[n_owned + j] = ghost_colors[j];",
     "tentative ghost recoloring: a losing ghost keeps its color as a constraint"),
    ("d2_ghost_pairs_repeated", C, "if (x < n_owned || seen[x - n_owned] == v) continue;",
     "if (x < n_owned) continue;",
     "D2/PD2 ghost step: an owned-ghost pair counted once per path"),
    ("d2_ghost_phase3_blind", C, "rc.ghost_col = ghost_colors;\n    r3 = run_rounds", "rc.ghost_col = none;\n    r3 = run_rounds",
     "D2/PD2 ghost step: phase 3 ignores the ghosts' colors"),
    ("dist_restart_each_step", PY, "r = step(p, gc[p], colors[p])", "r = step(p, gc[p], None)",
     "Algorithm 2: every iteration recolors from scratch instead of from the committed colors"),
    ("dist_sends_everything", PY, "np.count_nonzero(a != b)", "a.size",
     "Algorithm 2: every ghost copy counted as sent in every exchange"),
    ("dist_stops_early", PY, "if total == 0 or len(conflicts) > max_iterations:",
     "if total <= 2 or len(conflicts) > max_iterations:",
     "Algorithm 2: the loop stops with one conflicting cut edge left (counted once on each side)"),
    ("gid_ignored", C, "g[v] = gid ? (uint32_t)gid[v] : (uint32_t)v;", "g[v] = (uint32_t)v;",
     "ghost steps key vertices by local instead of global ids"),
    ("ghost_degree_zero", C, ": (int64_t)extra_deg[v - n_rows];", ": (int64_t)0;",
     "recolorDegrees: a ghost's reported degree ignored"),
    ("remote_loser_never", C, "glose[u - n_owned] = 1;", "(void)0;",
     "D1 ghost step: a ghost that loses a conflict is never flagged"),
    ("d2_ghost_phase1_sees_ghosts", C, "rc.ghost_col = none;\n    rc.ignore_from = m;", "rc.ghost_col = ghost_colors;\n    rc.ignore_from = m;",
     "D2/PD2 ghost step: phase 1 reads the ghosts' colors"),
    ("round_cap_off_by_one", C, "while (W.len > 0 && r < rc->max_rounds)", "while (W.len > 0 && r <= rc->max_rounds)",
     "a round cap of r runs r + 1 rounds"),
]

EQUIVALENT = {
    "d2_self_kept": "v's own color is 0 while it is in the worklist, and no vertex has a greater key "
                    "than itself, so v in its own neighbourhood changes neither step",
    "pd2_self_kept": "as d2_self_kept, for a column in its own neighbourhood",
    "detect_committed_too": "a committed neighbour's tentative color is its committed color, which the "
                            "worklist vertex's first fit avoided, so it never ties",
}


def run_copy(name, file=None, old=None, new=None):
    """Runs the pin files in a patched copy; returns (name, passed, seconds, tail)."""
    t0 = time.time()
    with tempfile.TemporaryDirectory(prefix=f"mut_{name}_") as d:
        for sub in ("oracle", "graphgen", "tests"):
            shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                            ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp*"))
        if file:
            path = os.path.join(d, file)
            with open(path) as f:
                text = f.read()
            if text.count(old) != 1:
                return name, None, 0.0, f"the text to replace occurs {text.count(old)} times"
            with open(path, "w") as f:
                f.write(text.replace(old, new))
        env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
        # a pin that runs far longer than it does on the oracle (a mutant
        # that stops converging) fails by its time limit
        p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "--timeout", "120", "-m", "not gpu", *PIN_FILES], cwd=d, env=env,
                           capture_output=True, text=True, timeout=3600)
        tail = (p.stdout.strip().splitlines() or [""])[-1]
        return name, p.returncode == 0, time.time() - t0, tail


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("-k", default="", help="only mutants whose name contains this")
    ap.add_argument("-j", type=int, default=4, help="mutants run at once")
    args = ap.parse_args()
    name, ok, secs, tail = run_copy("unmutated")
    print(f"unmutated: {'pass' if ok else 'FAIL'} ({secs:.0f} s) {tail}", flush=True)
    if not ok:
        sys.exit(2)
    chosen = [m for m in MUTANTS if args.k in m[0]]
    survivors = []
    with ThreadPoolExecutor(max_workers=args.j) as ex:
        futs = {ex.submit(run_copy, m[0], m[1], m[2], m[3]): m for m in chosen}
        for fut in futs:
            m = futs[fut]
            name, ok, secs, tail = fut.result()
            if ok is None:
                verdict = "NOT APPLIED"
                survivors.append(name)
            elif name in EQUIVALENT:
                verdict = "equivalent" if ok else "EQUIV-FAIL"
                if not ok:
                    survivors.append(name)
            elif ok:
                verdict = "SURVIVED"
                survivors.append(name)
            else:
                verdict = "killed"
            why = f"  (equivalent: {EQUIVALENT[name]})" if name in EQUIVALENT else ""
            print(f"{name:34s} {verdict:11s} {secs:5.0f} s  {m[4]}{why}  [{tail}]", flush=True)
    n_eq = sum(1 for m in chosen if m[0] in EQUIVALENT)
    print(f"{len(chosen) - n_eq - len(survivors)} of {len(chosen) - n_eq} mutants killed, "
          f"{n_eq} equivalent mutants pass as they must", flush=True)
    sys.exit(1 if survivors else 0)


if __name__ == "__main__":
    main()
