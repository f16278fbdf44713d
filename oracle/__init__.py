"""Python access to the C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the benchmark's CPU-baseline leg.  The GPU library never imports, links or
calls anything here, and nothing here imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
TRACE_ROUNDS = 4096
RECOLOR_DEGREES = 1   # key(v) = (deg(v), p(v), gid(v)): recolorDegrees (Section 3.3, Algorithm 4)
GHOST_RECOLOR = 2     # ghost step: losing ghosts recolored tentatively, then restored (Section 3.2)


_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = False, omp: bool = False) -> str:
    """Compile oracle.c with gcc: plain -O2, single thread (what the tests
    use), or with omp=True the same source with -fopenmp (the benchmark's
    all-core CPU baseline; identical results)."""
    src = os.path.join(_HERE, "oracle.c")
    so = _SO_OMP if omp else _SO
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + f".tmp{os.getpid()}"
        flags = ["-fopenmp"] if omp else ["-Wno-unknown-pragmas"]
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", *flags, "-fPIC", "-shared",
                               "-o", tmp, src])
        os.replace(tmp, so)
    return so


class _Stats(ctypes.Structure):
    _fields_ = [("num_colors", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("vertex_visits", ctypes.c_int64), ("edge_visits", ctypes.c_int64),
                ("boundary_conflicts", ctypes.c_int64), ("remote_losers", ctypes.c_int64),
                ("worklist_trace", ctypes.c_int64 * TRACE_ROUNDS)]


@dataclass
class Result:
    colors: np.ndarray
    num_colors: int
    rounds: int
    vertex_visits: int
    edge_visits: int
    boundary_conflicts: int = 0
    remote_losers: int = 0
    remote_loser: np.ndarray | None = None
    worklist: list = field(default_factory=list)
    converged: bool = True


_libs = {}


def lib(omp: bool = False):
    if omp not in _libs:
        l = ctypes.CDLL(build(omp=omp))
        P = ctypes.c_void_p
        l.orc_threads.restype = ctypes.c_int
        l.orc_threads.argtypes = []
        l.orc_fmix32.restype = ctypes.c_uint32
        l.orc_fmix32.argtypes = [ctypes.c_uint32]
        l.orc_priority.restype = ctypes.c_uint32
        l.orc_priority.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        l.orc_priorities.restype = None
        l.orc_priorities.argtypes = [ctypes.c_int32, ctypes.c_uint32, P]
        sig = [ctypes.c_int32, P, P, ctypes.c_uint32, P, P, ctypes.c_int32, P, P, ctypes.c_int]
        for name in ("orc_color_d1", "orc_color_d2"):
            getattr(l, name).restype = ctypes.c_int
            getattr(l, name).argtypes = sig
        l.orc_color_pd2.restype = ctypes.c_int
        l.orc_color_pd2.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_uint32,
                                    P, P, ctypes.c_int32, P, P, ctypes.c_int]
        l.orc_color_d1_ghost.restype = ctypes.c_int
        l.orc_color_d1_ghost.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, P, P, P, P, ctypes.c_uint32, P, P, P, P, P,
                                         ctypes.c_int]
        l.orc_color_d2_ghost.restype = ctypes.c_int
        l.orc_color_d2_ghost.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P,
                                         ctypes.c_uint32, P, P, P, ctypes.c_int]
        l.orc_serial_greedy.restype = None
        l.orc_serial_greedy.argtypes = [ctypes.c_int32, P, P, P, P]
        _libs[omp] = l
    return _libs[omp]


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _result(colors, st, ret, remote=None) -> Result:
    nr = min(st.rounds, TRACE_ROUNDS)
    return Result(colors, st.num_colors, st.rounds, st.vertex_visits, st.edge_visits,
                  st.boundary_conflicts, st.remote_losers, remote,
                  list(st.worklist_trace[:nr]), ret == 0)


def threads(omp: bool = False) -> int:
    """Threads the oracle's per-vertex loops use (1 for the plain build)."""
    return int(lib(omp).orc_threads())


def fmix32(h: int) -> int:
    return int(lib().orc_fmix32(h & 0xFFFFFFFF))


def priority(gid: int, seed: int) -> int:
    return int(lib().orc_priority(gid & 0xFFFFFFFF, seed & 0xFFFFFFFF))


def priorities(n: int, seed: int) -> np.ndarray:
    """p(i) for i in [0, n)."""
    out = np.empty(n, dtype=np.uint32)
    lib().orc_priorities(n, seed & 0xFFFFFFFF, _ptr(out))
    return out


def _flags(recolor_degrees):
    return RECOLOR_DEGREES if recolor_degrees else 0


def _prio_init(prio, init):
    p = None if prio is None else np.ascontiguousarray(prio, dtype=np.uint32)
    i = None if init is None else _i32(init)
    return p, i


def color_d1(g, seed: int = 1, prio=None, init=None, max_rounds: int = 0,
             recolor_degrees: bool = False, omp: bool = False) -> Result:
    rp, col = _i32(g.row_ptr), _i32(g.col)
    p, i = _prio_init(prio, init)
    out = np.zeros(g.n, dtype=np.int32)
    st = _Stats()
    ret = lib(omp).orc_color_d1(g.n, _ptr(rp), _ptr(col), seed & 0xFFFFFFFF, _ptr(p), _ptr(i),
                             max_rounds, _ptr(out), ctypes.byref(st), _flags(recolor_degrees))
    return _result(out, st, ret)


def color_d2(g, seed: int = 1, prio=None, init=None, max_rounds: int = 0,
             recolor_degrees: bool = False, omp: bool = False) -> Result:
    rp, col = _i32(g.row_ptr), _i32(g.col)
    p, i = _prio_init(prio, init)
    out = np.zeros(g.n, dtype=np.int32)
    st = _Stats()
    ret = lib(omp).orc_color_d2(g.n, _ptr(rp), _ptr(col), seed & 0xFFFFFFFF, _ptr(p), _ptr(i),
                             max_rounds, _ptr(out), ctypes.byref(st), _flags(recolor_degrees))
    return _result(out, st, ret)


def color_pd2(b, seed: int = 1, prio=None, init=None, max_rounds: int = 0,
              recolor_degrees: bool = False, omp: bool = False) -> Result:
    arrs = [_i32(x) for x in (b.row_ptr, b.col_idx, b.col_ptr, b.row_idx)]
    p, i = _prio_init(prio, init)
    out = np.zeros(b.n_cols, dtype=np.int32)
    st = _Stats()
    ret = lib(omp).orc_color_pd2(b.n_rows, b.n_cols, *[_ptr(a) for a in arrs], seed & 0xFFFFFFFF,
                              _ptr(p), _ptr(i), max_rounds, _ptr(out), ctypes.byref(st),
                              _flags(recolor_degrees))
    return _result(out, st, ret)


def color_d1_ghost(lg, seed: int = 1, init_owned=None, recolor_degrees: bool = False,
                   ghost_degree=None, ghost_recolor: bool = False) -> Result:
    """One rank's step.  init_owned: committed owned colors to start from (a
    later iteration of Algorithm 2); ghost_degree: the ghosts' degrees, needed
    with recolor_degrees; ghost_recolor: losing ghosts are recolored
    tentatively with the owned losers, then restored (Section 3.2)."""
    rp, col, gid, gc = (_i32(x) for x in (lg.row_ptr, lg.col, lg.gid, lg.ghost_colors))
    init = None if init_owned is None else _i32(init_owned)
    gdeg = None if ghost_degree is None else _i32(ghost_degree)
    if recolor_degrees and lg.n_ghost > 0 and gdeg is None:
        raise ValueError("recolor_degrees needs the ghosts' degrees")
    out = np.zeros(lg.n_owned, dtype=np.int32)
    remote = np.zeros(max(lg.n_ghost, 1), dtype=np.uint8)
    st = _Stats()
    ret = lib().orc_color_d1_ghost(lg.n_owned, lg.n_ghost, lg.layers, lg.n_g1, _ptr(rp), _ptr(col),
                                   _ptr(gid), _ptr(gc), seed & 0xFFFFFFFF, _ptr(init), _ptr(gdeg),
                                   _ptr(out), _ptr(remote), ctypes.byref(st),
                                   _flags(recolor_degrees) | (GHOST_RECOLOR if ghost_recolor else 0))
    return _result(out, st, ret, remote[:lg.n_ghost].copy())


def color_d2_ghost(lg, seed: int = 1) -> Result:
    """One rank's distance-2 step on a two-layer local graph (graphgen
    LocalGraph with layers = 2): reading R9 of oracle.c."""
    rp, col, gid, gc = (_i32(x) for x in (lg.row_ptr, lg.col, lg.gid, lg.ghost_colors))
    out = np.zeros(lg.n_owned, dtype=np.int32)
    remote = np.zeros(max(lg.n_ghost, 1), dtype=np.uint8)
    st = _Stats()
    ret = lib().orc_color_d2_ghost(2, lg.n_owned, lg.n_ghost, _ptr(rp), _ptr(col), _ptr(rp), _ptr(col), _ptr(gid),
                                   _ptr(gc), seed & 0xFFFFFFFF, _ptr(out), _ptr(remote), ctypes.byref(st), 0)
    return _result(out, st, ret, remote[:lg.n_ghost].copy())


def color_pd2_ghost(lp, seed: int = 1) -> Result:
    """One rank's partial distance-2 step on its local pattern (graphgen
    LocalPattern: owned columns' rows, the local rows' columns)."""
    arrs = [_i32(x) for x in (lp.col_ptr, lp.row_idx, lp.row_ptr, lp.col_idx, lp.gid, lp.ghost_colors)]
    out = np.zeros(lp.n_owned, dtype=np.int32)
    remote = np.zeros(max(lp.n_ghost, 1), dtype=np.uint8)
    st = _Stats()
    ret = lib().orc_color_d2_ghost(3, lp.n_owned, lp.n_ghost, *[_ptr(a) for a in arrs], seed & 0xFFFFFFFF,
                                   _ptr(out), _ptr(remote), ctypes.byref(st), 0)
    return _result(out, st, ret, remote[:lp.n_ghost].copy())


def serial_greedy(g, order) -> np.ndarray:
    rp, col, o = _i32(g.row_ptr), _i32(g.col), _i32(order)
    out = np.zeros(g.n, dtype=np.int32)
    lib().orc_serial_greedy(g.n, _ptr(rp), _ptr(col), _ptr(o), _ptr(out))
    return out


@dataclass
class DistResult:
    colors: list              # per rank: its owned vertices' colors (local order)
    detects: int              # conflict detections run (the last one found none)
    iterations: int           # Algorithm 2's while-loop iterations (recolorings)
    conflicts: list           # per detection: conflicts summed over the ranks (the Allreduce)
    exchanged: list           # per exchange: ghost copies whose color was sent
    rounds: int               # on-node rounds summed over ranks and steps


def _exchange_map(locals_):
    """For every rank's ghosts: the rank owning each ghost and its index among
    that rank's owned vertices (found by global id)."""
    gids = np.concatenate([np.asarray(lg.gid[:lg.n_owned], dtype=np.int64) for lg in locals_])
    part = np.concatenate([np.full(lg.n_owned, p, dtype=np.int64) for p, lg in enumerate(locals_)])
    index = np.concatenate([np.arange(lg.n_owned, dtype=np.int64) for lg in locals_])
    order = np.argsort(gids, kind="stable")
    sg = gids[order]
    maps = []
    for lg in locals_:
        g = np.asarray(lg.gid[lg.n_owned:], dtype=np.int64)
        pos = np.searchsorted(sg, g)
        if g.size and (np.any(pos >= sg.size) or np.any(sg[np.minimum(pos, sg.size - 1)] != g)):
            raise ValueError("a ghost is owned by no rank")
        maps.append((part[order[pos]], index[order[pos]]))
    return maps


def color_d1_distributed(locals_, seed: int = 1, recolor_degrees: bool = False, ghost_degrees=None,
                         max_iterations: int = 100000, ghost_recolor: bool = False) -> DistResult:
    """Algorithm 2 (Section 3), its ranks emulated one after another.

    Every rank first colors its owned vertices without ghost information (its
    ghosts' colors are not known yet: 0).  Then, until the conflicts summed
    over all ranks are zero: the ranks send their owned boundary colors to the
    ranks holding ghost copies (every ghost copy the first time, later only
    the copies whose color changed), and every rank runs one step of
    color_d1_ghost from its committed colors: it detects the conflicts of its
    owned-ghost edges against the received colors (the lower key loses,
    Algorithm 4) and recolors its losers with the ghosts' colors as fixed
    constraints.  Every rank reads only the colors sent in the last exchange,
    so the order in which the ranks run does not matter.
    locals_: one graphgen.LocalGraph per rank; ghost_degrees: per rank, its
    ghosts' global degrees (recolor_degrees only)."""
    P = len(locals_)
    maps = _exchange_map(locals_)
    gdeg = ghost_degrees if ghost_degrees is not None else [None] * P

    def step(p, gcolors, init):
        lg = locals_[p]
        view = type(lg)(**{**lg.__dict__, "ghost_colors": np.asarray(gcolors, dtype=np.int32)})
        return color_d1_ghost(view, seed=seed, init_owned=init, recolor_degrees=recolor_degrees,
                              ghost_degree=gdeg[p], ghost_recolor=ghost_recolor)

    rounds = 0
    colors = []
    for p in range(P):          # initial coloring: no ghost colors known yet
        r = step(p, np.zeros(locals_[p].n_ghost, np.int32), None)
        colors.append(r.colors)
        rounds += r.rounds
    gc = [colors_of(colors, m) for m in maps]
    exchanged = [int(sum(lg.n_ghost for lg in locals_))]
    conflicts = []
    while True:
        total = 0
        new = []
        for p in range(P):
            r = step(p, gc[p], colors[p])
            total += r.boundary_conflicts
            rounds += r.rounds
            new.append(r.colors)
        colors = new
        conflicts.append(int(total))
        if total == 0 or len(conflicts) > max_iterations:
            break
        nxt = [colors_of(colors, m) for m in maps]
        exchanged.append(int(sum(int(np.count_nonzero(a != b)) for a, b in zip(nxt, gc))))
        gc = nxt
    return DistResult(colors, len(conflicts), len(conflicts) - 1, conflicts, exchanged, rounds)


def colors_of(colors, m):
    """The colors a rank receives for its ghosts: owner rank's owned color."""
    part, index = m
    out = np.zeros(part.size, dtype=np.int32)
    for q in np.unique(part):
        sel = part == q
        out[sel] = colors[int(q)][index[sel]]
    return out
