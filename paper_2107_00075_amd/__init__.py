"""MI355X-native speculative graph coloring (distance-1, distance-2, partial
distance-2, and one rank's ghost-layer step) after Bogle et al., "Parallel
Graph Coloring Algorithms for Distributed GPU Environments".

The functions here have the names of the C-ABI entry points of
libgraphcolor.so (include/graphcolor.h) and only marshal arguments: graphs
are int32 torch tensors on a ROCm device, outputs are allocated with torch,
and every step of the coloring runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

from ._binding import (COLOR_E2BIG, COLOR_EGRAPH, COLOR_EINVAL, COLOR_EMISMATCH, COLOR_ENOCONVERGE, COLOR_ESCRATCH,
                       NOALLOC_MAX_N,
                       COLOR_EPENDING, COLOR_EQUEUED, COLOR_FLAG_KERNEL_TIMING, COLOR_FLAG_NO_TAIL,
                       COLOR_FLAG_GHOST_RECOLOR, COLOR_FLAG_RECOLOR_DEGREES, COLOR_FLAG_VALIDATE, COLOR_OK, ENGINE_AUTO, ENGINE_BATCH, ENGINE_INCREMENTAL, ENGINE_PULL,
                       EXPORTED, KIND_D1, KIND_D2, KIND_PD2, CDistStats, CHostJob, CJob, ColorError, CParams, CPart,
                       CStats, Params,
                       Stats, lib, strerror)

__all__ = [
    "color_d1", "color_d2", "color_pd2", "color_d1_ghost", "color_d1_ghost_step", "color_priority", "color_batch",
    "color_d1_noalloc", "NOALLOC_MAX_N", "COLOR_ESCRATCH", "color_d1_distributed", "DistStats",
    "color_d2_ghost", "color_pd2_ghost",
    "color_autotune", "color_autotune_reset", "ColorServer", "Params", "Stats", "ColorError", "lib",
    "strerror", "EXPORTED", "COLOR_FLAG_VALIDATE", "COLOR_FLAG_NO_TAIL", "COLOR_FLAG_KERNEL_TIMING",
    "COLOR_FLAG_RECOLOR_DEGREES", "COLOR_FLAG_GHOST_RECOLOR",
    "ENGINE_AUTO", "ENGINE_PULL", "ENGINE_INCREMENTAL", "ENGINE_BATCH", "KIND_D1", "KIND_D2", "KIND_PD2",
]


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, dtype=None, n=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a ROCm device")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    if t.numel() == 0:  # an empty array still needs a valid (never read) address
        t = _placeholder(t.device)
    return ctypes.c_void_p(t.data_ptr())


_PLACEHOLDERS = {}


def _placeholder(device):
    torch = _torch()
    key = str(device)
    if key not in _PLACEHOLDERS:
        _PLACEHOLDERS[key] = torch.zeros(16, dtype=torch.int32, device=device)
    return _PLACEHOLDERS[key]


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _stats(trace_cap):
    st = CStats()
    buf = None
    if trace_cap:
        buf = (ctypes.c_int64 * trace_cap)()
        st.worklist_trace = ctypes.cast(buf, ctypes.POINTER(ctypes.c_int64))
        st.trace_cap = trace_cap
    return st, buf


def _to_stats(st, buf) -> Stats:
    out = Stats(st.num_colors, st.rounds, st.vertex_visits, st.edge_visits, st.boundary_conflicts,
                st.remote_losers, st.kernel_launches, st.color_kernel_ns, st.detect_kernel_ns,
                st.color_launches, st.detect_launches, st.engine, st.list_visits, st.pushes,
                st.color_bytes, st.detect_bytes, st.tail_rounds, st.tail_kernel_ns, st.tail_bytes,
                st.tail_fallbacks)
    if buf is not None:
        out.worklist = list(buf[:min(st.rounds, len(buf))])
    return out


def _params(params):
    if params is None:
        return None
    return ctypes.byref(params.to_c())


def _check(rc, what, allow_noconverge=False):
    if rc == COLOR_OK or (allow_noconverge and rc == COLOR_ENOCONVERGE):
        return
    raise ColorError(rc, what)


def _graph_args(row_ptr, col_idx):
    torch = _torch()
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n+1 entries")
    return n, _dev_ptr(row_ptr, "row_ptr", torch.int32), _dev_ptr(col_idx, "col_idx", torch.int32)


def _color_sym(fn, row_ptr, col_idx, seed, prio, init_colors, out, params, stream, trace_cap,
               allow_partial):
    torch = _torch()
    n, rp, ci = _graph_args(row_ptr, col_idx)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    st, buf = _stats(trace_cap)
    if prio is not None and prio.element_size() != 4:
        raise TypeError("prio must hold 32-bit values")
    rc = fn(n, rp, ci, seed & 0xFFFFFFFF, _dev_ptr(prio, "prio", None, n),
            _dev_ptr(init_colors, "init_colors", torch.int32, n), _dev_ptr(out, "colors", torch.int32, n),
            ctypes.byref(st), _params(params), _stream(stream))
    _check(rc, fn.__name__, allow_partial)
    s = _to_stats(st, buf)
    s.converged = rc == COLOR_OK
    return out, s


def color_d1(row_ptr, col_idx, seed=1, prio=None, init_colors=None, out=None, params=None,
             stream=None, trace_cap=0, allow_partial=False):
    """Distance-1 coloring of a symmetric int32 CSR graph on the GPU.
    Returns (colors int32 tensor, Stats)."""
    return _color_sym(lib().color_d1, row_ptr, col_idx, seed, prio, init_colors, out, params, stream,
                      trace_cap, allow_partial)


def color_d1_noalloc(row_ptr, col_idx, seed=1, prio=None, init_colors=None, out=None, params=None,
                     stream=None, trace_cap=0, allow_partial=False):
    """color_d1 without any allocation inside the library (graphs of up to
    NOALLOC_MAX_N vertices; `out` should be passed by callers that cannot
    allocate either).  Returns (colors int32 tensor, Stats)."""
    return _color_sym(lib().color_d1_noalloc, row_ptr, col_idx, seed, prio, init_colors, out, params, stream,
                      trace_cap, allow_partial)


def color_d2(row_ptr, col_idx, seed=1, prio=None, init_colors=None, out=None, params=None,
             stream=None, trace_cap=0, allow_partial=False):
    """Distance-2 coloring of a symmetric int32 CSR graph on the GPU."""
    return _color_sym(lib().color_d2, row_ptr, col_idx, seed, prio, init_colors, out, params, stream,
                      trace_cap, allow_partial)


def color_pd2(row_ptr, col_idx, col_ptr, row_idx, seed=1, prio=None, init_colors=None, out=None,
              params=None, stream=None, trace_cap=0, allow_partial=False):
    """Partial distance-2 coloring of the columns of a sparse pattern given in
    CSR (row_ptr, col_idx) and CSC (col_ptr, row_idx)."""
    torch = _torch()
    n_rows = row_ptr.numel() - 1
    n_cols = col_ptr.numel() - 1
    if out is None:
        out = torch.empty(max(n_cols, 0), dtype=torch.int32, device=col_ptr.device)
    st, buf = _stats(trace_cap)
    i32 = torch.int32
    rc = lib().color_pd2(n_rows, n_cols, _dev_ptr(row_ptr, "row_ptr", i32), _dev_ptr(col_idx, "col_idx", i32),
                         _dev_ptr(col_ptr, "col_ptr", i32), _dev_ptr(row_idx, "row_idx", i32),
                         seed & 0xFFFFFFFF, _dev_ptr(prio, "prio", None, n_cols),
                         _dev_ptr(init_colors, "init_colors", i32, n_cols),
                         _dev_ptr(out, "col_colors", i32, n_cols), ctypes.byref(st), _params(params),
                         _stream(stream))
    _check(rc, "color_pd2", allow_partial)
    s = _to_stats(st, buf)
    s.converged = rc == COLOR_OK
    return out, s


def color_d1_ghost(n_owned, n_ghost, layers, n_g1, row_ptr, col_idx, gid, ghost_colors, seed=1,
                   out=None, remote_loser=True, params=None, stream=None, trace_cap=0):
    """One rank's step of the distributed D1 method on its local graph
    (owned vertices, then ghosts).  Returns (owned colors, remote-loser flags
    uint8 tensor or None, Stats)."""
    torch = _torch()
    i32 = torch.int32
    dev = row_ptr.device
    if out is None:
        out = torch.empty(max(n_owned, 0), dtype=i32, device=dev)
    rl = torch.empty(max(n_ghost, 1), dtype=torch.uint8, device=dev) if remote_loser else None
    st, buf = _stats(trace_cap)
    rc = lib().color_d1_ghost(n_owned, n_ghost, layers, n_g1, _dev_ptr(row_ptr, "row_ptr", i32),
                              _dev_ptr(col_idx, "col_idx", i32), _dev_ptr(gid, "gid", i32),
                              _dev_ptr(ghost_colors, "ghost_colors", i32) if n_ghost > 0 else None,
                              seed & 0xFFFFFFFF, _dev_ptr(out, "owned_colors", i32, n_owned),
                              _dev_ptr(rl, "remote_loser") if rl is not None else None,
                              ctypes.byref(st), _params(params), _stream(stream))
    _check(rc, "color_d1_ghost")
    return out, (rl[:n_ghost] if rl is not None else None), _to_stats(st, buf)


def color_d1_ghost_step(n_owned, n_ghost, layers, n_g1, row_ptr, col_idx, gid, ghost_colors, seed=1,
                        ghost_degree=None, init_owned=None, out=None, remote_loser=True, params=None,
                        stream=None, trace_cap=0):
    """One iteration of Algorithm 2 for one rank: color_d1_ghost with the
    ghosts' current colors (0 = not known yet), their degrees (needed with
    COLOR_FLAG_RECOLOR_DEGREES) and the rank's committed owned colors to
    start from.  Returns (owned colors, remote-loser flags or None, Stats)."""
    torch = _torch()
    i32 = torch.int32
    dev = row_ptr.device
    if out is None:
        out = torch.empty(max(n_owned, 0), dtype=i32, device=dev)
    rl = torch.empty(max(n_ghost, 1), dtype=torch.uint8, device=dev) if remote_loser else None
    st, buf = _stats(trace_cap)
    rc = lib().color_d1_ghost_step(n_owned, n_ghost, layers, n_g1, _dev_ptr(row_ptr, "row_ptr", i32),
                                   _dev_ptr(col_idx, "col_idx", i32), _dev_ptr(gid, "gid", i32),
                                   _dev_ptr(ghost_colors, "ghost_colors", i32, n_ghost) if n_ghost > 0 else None,
                                   _dev_ptr(ghost_degree, "ghost_degree", i32, n_ghost) if n_ghost > 0 else None,
                                   seed & 0xFFFFFFFF, _dev_ptr(init_owned, "init_owned", i32, n_owned),
                                   _dev_ptr(out, "owned_colors", i32, n_owned),
                                   _dev_ptr(rl, "remote_loser") if rl is not None else None,
                                   ctypes.byref(st), _params(params), _stream(stream))
    _check(rc, "color_d1_ghost_step")
    return out, (rl[:n_ghost] if rl is not None else None), _to_stats(st, buf)


def color_d2_ghost(n_owned, n_ghost, n_g1, row_ptr, col_idx, gid, ghost_colors, seed=1, out=None,
                   remote_loser=True, params=None, stream=None, trace_cap=0):
    """One rank's distance-2 step on its two-layer local graph.  Returns
    (owned colors, remote-loser flags or None, Stats)."""
    torch = _torch()
    i32 = torch.int32
    dev = row_ptr.device
    if out is None:
        out = torch.empty(max(n_owned, 0), dtype=i32, device=dev)
    rl = torch.empty(max(n_ghost, 1), dtype=torch.uint8, device=dev) if remote_loser else None
    st, buf = _stats(trace_cap)
    rc = lib().color_d2_ghost(n_owned, n_ghost, n_g1, _dev_ptr(row_ptr, "row_ptr", i32),
                              _dev_ptr(col_idx, "col_idx", i32), _dev_ptr(gid, "gid", i32),
                              _dev_ptr(ghost_colors, "ghost_colors", i32, n_ghost) if n_ghost > 0 else None,
                              seed & 0xFFFFFFFF, _dev_ptr(out, "owned_colors", i32, n_owned),
                              _dev_ptr(rl, "remote_loser") if rl is not None else None,
                              ctypes.byref(st), _params(params), _stream(stream))
    _check(rc, "color_d2_ghost")
    return out, (rl[:n_ghost] if rl is not None else None), _to_stats(st, buf)


def color_pd2_ghost(n_owned, n_ghost, n_rows, col_ptr, row_idx, row_ptr, col_idx, gid, ghost_colors, seed=1,
                    out=None, remote_loser=True, params=None, stream=None, trace_cap=0):
    """One rank's partial distance-2 step on its local pattern.  Returns
    (owned column colors, remote-loser flags or None, Stats)."""
    torch = _torch()
    i32 = torch.int32
    dev = col_ptr.device
    if out is None:
        out = torch.empty(max(n_owned, 0), dtype=i32, device=dev)
    rl = torch.empty(max(n_ghost, 1), dtype=torch.uint8, device=dev) if remote_loser else None
    st, buf = _stats(trace_cap)
    rc = lib().color_pd2_ghost(n_owned, n_ghost, n_rows, _dev_ptr(col_ptr, "col_ptr", i32),
                               _dev_ptr(row_idx, "row_idx", i32), _dev_ptr(row_ptr, "row_ptr", i32),
                               _dev_ptr(col_idx, "col_idx", i32), _dev_ptr(gid, "gid", i32),
                               _dev_ptr(ghost_colors, "ghost_colors", i32, n_ghost) if n_ghost > 0 else None,
                               seed & 0xFFFFFFFF, _dev_ptr(out, "owned_colors", i32, n_owned),
                               _dev_ptr(rl, "remote_loser") if rl is not None else None,
                               ctypes.byref(st), _params(params), _stream(stream))
    _check(rc, "color_pd2_ghost")
    return out, (rl[:n_ghost] if rl is not None else None), _to_stats(st, buf)


class DistStats:
    """Statistics of color_d1_distributed (see color_dist_stats)."""

    def __init__(self, c, conflicts, exchanged):
        self.detects = c.detects
        self.iterations = c.iterations
        self.num_colors = c.num_colors
        self.exchanged_total = c.exchanged_total
        self.rounds_total = c.rounds_total
        self.conflicts = conflicts
        self.exchanged = exchanged


def color_d1_distributed(parts, seed=1, max_detects=0, params=None, stream=None, trace_cap=4096):
    """Algorithm 2 over the ranks in `parts` (list of dicts: n_owned, n_ghost,
    layers, n_g1 and device tensors row_ptr, col_idx, gid, ghost_owner,
    ghost_index, optional ghost_degree and out).  Returns (list of owned color
    tensors, DistStats)."""
    torch = _torch()
    i32 = torch.int32
    arr = (CPart * max(len(parts), 1))()
    outs = []
    for i, q in enumerate(parts):
        o = q.get("out")
        if o is None:
            o = torch.empty(max(q["n_owned"], 1), dtype=i32, device=q["row_ptr"].device)
        outs.append(o[:q["n_owned"]])
        ng = q["n_ghost"]
        arr[i].n_owned, arr[i].n_ghost, arr[i].layers, arr[i].n_g1 = q["n_owned"], ng, q["layers"], q["n_g1"]
        arr[i].row_ptr = _dev_ptr(q["row_ptr"], "row_ptr", i32)
        arr[i].col_idx = _dev_ptr(q["col_idx"], "col_idx", i32)
        arr[i].gid = _dev_ptr(q["gid"], "gid", i32)
        arr[i].ghost_owner = _dev_ptr(q["ghost_owner"], "ghost_owner", i32, ng) if ng > 0 else None
        arr[i].ghost_index = _dev_ptr(q["ghost_index"], "ghost_index", i32, ng) if ng > 0 else None
        gd = q.get("ghost_degree")
        arr[i].ghost_degree = _dev_ptr(gd, "ghost_degree", i32, ng) if (gd is not None and ng > 0) else None
        arr[i].owned_colors = _dev_ptr(o, "out", i32)
    st = CDistStats()
    ct = (ctypes.c_int64 * trace_cap)()
    et = (ctypes.c_int64 * trace_cap)()
    st.trace_cap = trace_cap
    st.conflicts_trace = ctypes.cast(ct, ctypes.POINTER(ctypes.c_int64))
    st.exchanged_trace = ctypes.cast(et, ctypes.POINTER(ctypes.c_int64))
    rc = lib().color_d1_distributed(len(parts), arr, seed & 0xFFFFFFFF, max_detects, ctypes.byref(st),
                                    _params(params), _stream(stream))
    _check(rc, "color_d1_distributed", allow_noconverge=True)
    nd = min(st.detects, trace_cap)
    return outs, DistStats(st, list(ct[:nd]), list(et[:min(nd, trace_cap)]))


def color_priority(n, seed=1, gid=None, device="cuda", stream=None):
    """p(v) as the kernels compute it, for v < n (or for gid[0..n))."""
    torch = _torch()
    out = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    rc = lib().color_priority(n, _dev_ptr(gid, "gid", torch.int32, n), seed & 0xFFFFFFFF,
                              _dev_ptr(out, "out"), _stream(stream))
    _check(rc, "color_priority")
    return out[:n]


def _job_structs(jobs):
    torch = _torch()
    n_jobs = len(jobs)
    arr = (CJob * max(n_jobs, 1))()
    outs = []
    i32 = torch.int32
    for i, j in enumerate(jobs):
        kind = j["kind"]
        if kind == KIND_PD2:
            n = j["col_ptr"].numel() - 1
            n_rows = j["row_ptr"].numel() - 1
        else:
            n = j["row_ptr"].numel() - 1
            n_rows = n
        o = j.get("out")
        if o is None:
            o = torch.empty(max(n, 1), dtype=i32, device=j["row_ptr"].device)
        outs.append(o[:n])
        arr[i].kind = kind
        arr[i].n = n
        arr[i].n_rows = n_rows
        arr[i].seed = j.get("seed", 1) & 0xFFFFFFFF
        arr[i].row_ptr = _dev_ptr(j["row_ptr"], "row_ptr", i32)
        arr[i].col_idx = _dev_ptr(j["col_idx"], "col_idx", i32)
        arr[i].col_ptr = _dev_ptr(j.get("col_ptr"), "col_ptr", i32)
        arr[i].row_idx = _dev_ptr(j.get("row_idx"), "row_idx", i32)
        arr[i].colors = _dev_ptr(o, "colors", i32)
    return arr, outs


def color_batch(jobs, params=None, stream=None):
    """Colors many graphs in one persistent launch.  jobs: list of dicts with
    kind (KIND_*), and device tensors row_ptr, col_idx (+ col_ptr, row_idx for
    PD2), seed, optional out.  Returns (list of color tensors, list of Stats)."""
    n_jobs = len(jobs)
    arr, outs = _job_structs(jobs)
    stats = (CStats * max(n_jobs, 1))()
    rc = lib().color_batch(n_jobs, arr, stats, _params(params), _stream(stream))
    _check(rc, "color_batch")
    return outs, [_to_stats(stats[i], None) for i in range(n_jobs)]


def color_autotune(job, reps=2, stream=None):
    """Times candidate mappings of `job` (a color_batch job dict) in the
    batched engine and records the fastest for its kind and degree class.
    Returns the chosen Params (bin_hi, lanes)."""
    arr, _ = _job_structs([job])
    best = CParams()
    rc = lib().color_autotune(arr, int(reps), ctypes.byref(best), _stream(stream))
    _check(rc, "color_autotune")
    return Params(bin_hi=tuple(best.bin_hi), lanes=tuple(best.lanes))


def color_autotune_reset():
    _check(lib().color_autotune_reset(), "color_autotune_reset")


class ColorServer:
    """Continuous-batching coloring server (HBM-footprint admission)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64):
        err = ctypes.c_int(0)
        self._h = lib().color_server_create(hbm_budget_bytes, max_slots, ctypes.byref(err))
        if not self._h:
            raise ColorError(err.value, "color_server_create")
        self._keep = {}

    def submit(self, kind, row_ptr, col_idx, col_ptr=None, row_idx=None, seed=1):
        """Host numpy int32 arrays.  Returns (job id, status code)."""
        import numpy as np
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.int32)
                for a in (row_ptr, col_idx, col_ptr, row_idx)]
        j = CHostJob()
        j.kind = kind
        if kind == KIND_PD2:
            j.n = arrs[2].size - 1
            j.n_rows = arrs[0].size - 1
        else:
            j.n = arrs[0].size - 1
            j.n_rows = j.n
        j.seed = seed & 0xFFFFFFFF
        ptrs = [None if a is None else a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        j.row_ptr, j.col_idx, j.col_ptr, j.row_idx = ptrs
        jid = ctypes.c_uint64(0)
        rc = lib().color_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid))
        if rc not in (COLOR_OK, COLOR_EQUEUED):
            raise ColorError(rc, "color_server_submit")
        self._keep[jid.value] = j.n
        return jid.value, rc

    def poll(self, job_id):
        """Returns (colors numpy array, Stats) when done, None while pending."""
        import numpy as np
        n = self._keep[job_id]
        out = np.empty(max(n, 1), dtype=np.int32)
        st = CStats()
        rc = lib().color_server_poll(self._h, job_id, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        if rc == COLOR_EPENDING:
            return None
        _check(rc, "color_server_poll")
        del self._keep[job_id]
        return out[:n], _to_stats(st, None)

    def drain(self):
        _check(lib().color_server_drain(self._h), "color_server_drain")

    def close(self):
        if self._h:
            lib().color_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
