"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every entry point include/graphcolor.h declares, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "graphcolor.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(color_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2107_00075_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libgraphcolor.so is not built (run __graft_entry__.build())")
    return _binding.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("color_d1", "color_d2", "color_pd2", "color_d1_ghost", "color_batch",
                     "color_server_create", "color_server_submit", "color_server_poll",
                     "color_server_destroy", "color_strerror", "color_priority"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2107_00075_amd import _binding
    raw = ctypes.CDLL(_binding.LIB_PATH)
    for name in _declared():
        assert hasattr(raw, name), name
    assert set(_declared()) == set(_binding.EXPORTED)


def test_no_undeclared_c_entry_points(lib):
    """Every unmangled function the library exports is one the header
    declares (the C++ internals stay mangled or hidden)."""
    import shutil
    import subprocess
    from paper_2107_00075_amd import _binding
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", _binding.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {parts[2] for parts in (line.split() for line in out.splitlines())
                if len(parts) == 3 and parts[1] == "T" and not parts[2].startswith("_Z")}
    assert exported == set(_declared())


def test_strerror(lib):
    from paper_2107_00075_amd import _binding as b
    assert lib.color_strerror(0) == b"ok"
    for code in (b.COLOR_EINVAL, b.COLOR_EGRAPH, b.COLOR_EOVERFLOW, b.COLOR_ENOMEM, b.COLOR_EHIP,
                 b.COLOR_ENOCONVERGE, b.COLOR_E2BIG, b.COLOR_EQUEUED, b.COLOR_EPENDING, b.COLOR_ESCRATCH):
        assert lib.color_strerror(code) not in (b"ok", b"unknown error")
    assert lib.color_strerror(12345) == b"unknown error"


def test_bad_arguments_rejected_on_host(lib):
    from paper_2107_00075_amd import _binding as b
    assert lib.color_d1(-1, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_d2(5, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_pd2(-2, 3, None, None, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_d1_ghost(4, 2, 3, 0, None, None, None, None, 1, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_d1_ghost(4, 2, 1, 5, None, None, None, None, 1, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_priority(-1, None, 1, None, None) == b.COLOR_EINVAL
    assert lib.color_batch(-1, None, None, None, None) == b.COLOR_EINVAL
    step = lib.color_d1_ghost_step
    assert step(4, 2, 3, 0, None, None, None, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    assert step(-1, 0, 1, 0, None, None, None, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    # recolorDegrees with ghosts but no ghost degrees
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks come first
    pr = b.CParams()
    pr.flags = b.COLOR_FLAG_RECOLOR_DEGREES
    assert step(4, 2, 1, 0, fake, fake, fake, fake, None, 1, None, fake, None, None, ctypes.byref(pr),
                None) == b.COLOR_EINVAL
    assert lib.color_d1_ghost(4, 2, 1, 0, fake, fake, fake, fake, 1, fake, None, None, ctypes.byref(pr),
                              None) == b.COLOR_EINVAL
    assert lib.color_batch(1, None, None, ctypes.byref(pr), None) == b.COLOR_EINVAL
    assert lib.color_d1_distributed(0, None, 1, 0, None, None, None) == b.COLOR_EINVAL
    parts = (b.CPart * 1)()
    parts[0].n_owned, parts[0].n_ghost = 4, 2   # ghosts without owner / index arrays
    assert lib.color_d1_distributed(1, parts, 1, 0, None, None, None) == b.COLOR_EINVAL
    # the no-allocation entry point: sizes beyond its scratch, flags it cannot honour
    assert lib.color_d1_noalloc(b.NOALLOC_MAX_N + 1, fake, fake, 1, None, None, fake, None, None,
                                None) == b.COLOR_ESCRATCH
    assert lib.color_d1_noalloc(-1, None, None, 1, None, None, None, None, None, None) == b.COLOR_EINVAL
    assert lib.color_d1_noalloc(10, fake, fake, 1, None, None, fake, None, ctypes.byref(pr),
                                None) == b.COLOR_EINVAL


def test_batch_and_server_arguments_rejected_on_host(lib):
    from paper_2107_00075_amd import _binding as b
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks come first
    jobs = (b.CJob * 2)()
    for j in jobs:
        j.kind, j.n, j.n_rows, j.seed = 1, 10, 10, 1
        j.row_ptr = j.col_idx = j.colors = fake
    jobs[1].kind = 7
    assert lib.color_batch(2, jobs, None, None, None) == b.COLOR_EINVAL
    jobs[1].kind = 1
    jobs[1].n = (1 << 23) + 1
    assert lib.color_batch(2, jobs, None, None, None) == b.COLOR_EOVERFLOW
    jobs[1].n = 5
    jobs[1].colors = None
    assert lib.color_batch(2, jobs, None, None, None) == b.COLOR_EINVAL
    jobs[1].colors = fake
    jobs[1].kind = 3  # PD2 without the CSC arrays
    assert lib.color_batch(2, jobs, None, None, None) == b.COLOR_EINVAL
    assert lib.color_batch(-1, jobs, None, None, None) == b.COLOR_EINVAL
    assert lib.color_batch(0, None, None, None, None) == b.COLOR_OK
    assert lib.color_autotune(None, 1, None, None) == b.COLOR_EINVAL
    jobs[0].n = 0
    assert lib.color_autotune(jobs, 1, None, None) == b.COLOR_EINVAL
    err = ctypes.c_int(0)
    assert not lib.color_server_create(0, 4, ctypes.byref(err))
    assert err.value == b.COLOR_EINVAL
    assert not lib.color_server_create(1 << 20, 0, ctypes.byref(err))
    assert err.value == b.COLOR_EINVAL
    assert lib.color_server_submit(None, None, None) == b.COLOR_EINVAL
    assert lib.color_server_poll(None, 1, None, None) == b.COLOR_EINVAL
    assert lib.color_server_drain(None) == b.COLOR_EINVAL
    assert lib.color_server_destroy(None) == b.COLOR_OK
    assert lib.color_strerror(b.COLOR_EMISMATCH)
