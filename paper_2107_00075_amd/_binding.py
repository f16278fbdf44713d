"""ctypes binding of libgraphcolor.so: argument marshalling only.

Every step of the coloring runs in the library's HIP kernels; this module
only turns torch tensors into device pointers, fills the C structs and maps
return codes to exceptions.  If the shared library is missing the import of
any entry point raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgraphcolor.so")

COLOR_OK = 0
COLOR_EINVAL = -1
COLOR_EGRAPH = -2
COLOR_EOVERFLOW = -3
COLOR_ENOMEM = -4
COLOR_EHIP = -5
COLOR_ENOCONVERGE = -6
COLOR_E2BIG = -7
COLOR_EMISMATCH = -8
COLOR_ESCRATCH = -9
NOALLOC_MAX_N = 1 << 20
COLOR_EQUEUED = 1
COLOR_EPENDING = 2

COLOR_FLAG_VALIDATE = 0x1
COLOR_FLAG_NO_TAIL = 0x2
COLOR_FLAG_KERNEL_TIMING = 0x4
COLOR_FLAG_RECOLOR_DEGREES = 0x8
COLOR_FLAG_GHOST_RECOLOR = 0x10

KIND_D1, KIND_D2, KIND_PD2 = 1, 2, 3
ENGINE_AUTO, ENGINE_PULL, ENGINE_INCREMENTAL, ENGINE_BATCH = 0, 1, 2, 3

EXPORTED = [
    "color_d1", "color_d2", "color_pd2", "color_d1_ghost", "color_d1_ghost_step", "color_priority",
    "color_batch", "color_server_create", "color_server_submit", "color_server_poll",
    "color_server_drain", "color_server_destroy", "color_release_workspace", "color_strerror",
    "color_autotune", "color_autotune_reset", "color_d1_noalloc", "color_d1_distributed",
    "color_d2_ghost", "color_pd2_ghost",
]


class ColorError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class CStats(ctypes.Structure):
    _fields_ = [("num_colors", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("vertex_visits", ctypes.c_int64), ("edge_visits", ctypes.c_int64),
                ("boundary_conflicts", ctypes.c_int64), ("remote_losers", ctypes.c_int64),
                ("worklist_trace", ctypes.POINTER(ctypes.c_int64)), ("trace_cap", ctypes.c_int32),
                ("kernel_launches", ctypes.c_int32), ("color_kernel_ns", ctypes.c_int64),
                ("detect_kernel_ns", ctypes.c_int64), ("color_launches", ctypes.c_int32),
                ("detect_launches", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("tail_rounds", ctypes.c_int32), ("list_visits", ctypes.c_int64),
                ("pushes", ctypes.c_int64), ("color_bytes", ctypes.c_int64),
                ("detect_bytes", ctypes.c_int64), ("tail_kernel_ns", ctypes.c_int64),
                ("tail_bytes", ctypes.c_int64), ("tail_fallbacks", ctypes.c_int32)]


class CParams(ctypes.Structure):
    _fields_ = [("bin_hi", ctypes.c_int32 * 4), ("lanes", ctypes.c_int32 * 3),
                ("split_chunks", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("rounds_per_poll", ctypes.c_int32), ("tail_threshold", ctypes.c_int32),
                ("max_workgroups", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("engine", ctypes.c_int32), ("tail_checkin_us", ctypes.c_int32)]


class CPart(ctypes.Structure):
    _fields_ = [("n_owned", ctypes.c_int32), ("n_ghost", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("n_g1", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("gid", ctypes.c_void_p), ("ghost_owner", ctypes.c_void_p), ("ghost_index", ctypes.c_void_p),
                ("ghost_degree", ctypes.c_void_p), ("owned_colors", ctypes.c_void_p)]


class CDistStats(ctypes.Structure):
    _fields_ = [("detects", ctypes.c_int32), ("iterations", ctypes.c_int32), ("num_colors", ctypes.c_int32),
                ("trace_cap", ctypes.c_int32), ("conflicts_trace", ctypes.POINTER(ctypes.c_int64)),
                ("exchanged_trace", ctypes.POINTER(ctypes.c_int64)), ("exchanged_total", ctypes.c_int64),
                ("rounds_total", ctypes.c_int64)]


class CJob(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p), ("colors", ctypes.c_void_p)]


class CHostJob(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p)]


@dataclass
class Stats:
    num_colors: int = 0
    rounds: int = 0
    vertex_visits: int = 0
    edge_visits: int = 0
    boundary_conflicts: int = 0
    remote_losers: int = 0
    kernel_launches: int = 0
    color_kernel_ns: int = 0
    detect_kernel_ns: int = 0
    color_launches: int = 0
    detect_launches: int = 0
    engine: int = 0
    list_visits: int = 0
    pushes: int = 0
    color_bytes: int = 0
    detect_bytes: int = 0
    tail_rounds: int = 0
    tail_kernel_ns: int = 0
    tail_bytes: int = 0
    tail_fallbacks: int = 0
    converged: bool = True
    worklist: list = field(default_factory=list)


@dataclass
class Params:
    """Tuning knobs (none changes a coloring, except the flag
    COLOR_FLAG_RECOLOR_DEGREES, which selects the recolorDegrees key).
    0 = library default."""
    bin_hi: tuple = (0, 0, 0, 0)
    lanes: tuple = (0, 0, 0)
    split_chunks: int = 0
    max_rounds: int = 0
    rounds_per_poll: int = 0
    tail_threshold: int = 0
    max_workgroups: int = 0
    flags: int = 0
    engine: int = 0
    tail_checkin_us: int = 0

    def to_c(self) -> CParams:
        p = CParams()
        for i, x in enumerate(self.bin_hi):
            p.bin_hi[i] = int(x)
        for i, x in enumerate(self.lanes):
            p.lanes[i] = int(x)
        p.split_chunks = self.split_chunks
        p.max_rounds = self.max_rounds
        p.rounds_per_poll = self.rounds_per_poll
        p.tail_threshold = self.tail_threshold
        p.max_workgroups = self.max_workgroups
        p.flags = self.flags
        p.engine = self.engine
        p.tail_checkin_us = self.tail_checkin_us
        return p


_lib = None


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2107_00075_amd.build)")
        l = ctypes.CDLL(LIB_PATH)
        P, I32, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        SP = ctypes.POINTER(CStats)
        PP = ctypes.POINTER(CParams)
        for name in ("color_d1", "color_d2", "color_d1_noalloc"):
            f = getattr(l, name)
            f.restype = ctypes.c_int
            f.argtypes = [I32, P, P, U32, P, P, P, SP, PP, P]
        l.color_pd2.restype = ctypes.c_int
        l.color_pd2.argtypes = [I32, I32, P, P, P, P, U32, P, P, P, SP, PP, P]
        l.color_d1_ghost.restype = ctypes.c_int
        l.color_d1_ghost.argtypes = [I32, I32, I32, I32, P, P, P, P, U32, P, P, SP, PP, P]
        l.color_d1_ghost_step.restype = ctypes.c_int
        l.color_d1_ghost_step.argtypes = [I32, I32, I32, I32, P, P, P, P, P, U32, P, P, P, SP, PP, P]
        l.color_d1_distributed.restype = ctypes.c_int
        l.color_d1_distributed.argtypes = [I32, ctypes.POINTER(CPart), U32, I32, ctypes.POINTER(CDistStats), PP, P]
        l.color_d2_ghost.restype = ctypes.c_int
        l.color_d2_ghost.argtypes = [I32, I32, I32, P, P, P, P, U32, P, P, SP, PP, P]
        l.color_pd2_ghost.restype = ctypes.c_int
        l.color_pd2_ghost.argtypes = [I32, I32, I32, P, P, P, P, P, P, U32, P, P, SP, PP, P]
        l.color_priority.restype = ctypes.c_int
        l.color_priority.argtypes = [I32, P, U32, P, P]
        l.color_batch.restype = ctypes.c_int
        l.color_batch.argtypes = [I32, ctypes.POINTER(CJob), SP, PP, P]
        l.color_server_create.restype = P
        l.color_server_create.argtypes = [ctypes.c_size_t, I32, ctypes.POINTER(ctypes.c_int)]
        l.color_server_submit.restype = ctypes.c_int
        l.color_server_submit.argtypes = [P, ctypes.POINTER(CHostJob), ctypes.POINTER(ctypes.c_uint64)]
        l.color_server_poll.restype = ctypes.c_int
        l.color_server_poll.argtypes = [P, ctypes.c_uint64, P, SP]
        l.color_server_drain.restype = ctypes.c_int
        l.color_server_drain.argtypes = [P]
        l.color_server_destroy.restype = ctypes.c_int
        l.color_server_destroy.argtypes = [P]
        l.color_autotune.restype = ctypes.c_int
        l.color_autotune.argtypes = [ctypes.POINTER(CJob), I32, PP, P]
        l.color_autotune_reset.restype = ctypes.c_int
        l.color_autotune_reset.argtypes = []
        l.color_release_workspace.restype = ctypes.c_int
        l.color_release_workspace.argtypes = []
        l.color_strerror.restype = ctypes.c_char_p
        l.color_strerror.argtypes = [ctypes.c_int]
        _lib = l
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().color_strerror(code).decode()
    except RuntimeError:
        return f"error {code}"
