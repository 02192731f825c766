"""Host-only checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rp.h", "rp_serve.h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rp_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_abi():
    names = _declared()
    for want in ("rp_load_graph", "rp_prune", "rp_prune_sweep", "rp_search", "rp_free_graph",
                 "rp_last_error"):
        assert want in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2602_08097_amd import rp

    if not os.path.exists(rp.LIB_PATH):
        pytest.fail("librp.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(rp.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(rp.EXPORTS) == _declared()
    lib.rp_last_error.restype = ctypes.c_char_p
    assert lib.rp_last_error() == b""


def test_null_arguments_are_rejected_without_a_device():
    from paper_2602_08097_amd import rp

    lib = rp.load_library()
    h = ctypes.c_void_p()
    assert lib.rp_load_graph(None, 1, 10, 4, None, None, 4, 0, None, ctypes.byref(h)) == 1
    assert b"points" in lib.rp_last_error()
    assert lib.rp_load_graph(None, 7, 10, 4, None, None, 4, 0, None, ctypes.byref(h)) == 1
    assert b"dtype" in lib.rp_last_error()
    assert lib.rp_load_graph(None, 1, 10, 4, None, None, 4, 10, None, ctypes.byref(h)) == 2
    assert lib.rp_prune(None, rp.Alpha(6, 5), 4, None, None, None) == 5


def test_server_arguments_are_rejected_without_a_device():
    from paper_2602_08097_amd import rp

    lib = rp.load_library()
    h = ctypes.c_void_p()
    assert lib.rp_server_create(None, 1 << 20, 4, 64, 0, ctypes.byref(h)) == 5
    assert lib.rp_server_create(None, 1 << 20, 4, 64, 0, None) == 1
    req = rp.Request(rp.REQ_PRUNE, rp.Alpha(6, 5), 8, None, 0, 0, 0, None, None, None, 0)
    assert lib.rp_server_submit(None, ctypes.byref(req)) == 5
    comp = (rp.Completion * 4)()
    assert lib.rp_server_poll(None, comp, 4, 0) == -1
    st = rp.ServerStats()
    assert lib.rp_server_stats_get(None, ctypes.byref(st)) == 5
    lib.rp_server_destroy(None)


def test_oracle_library_is_separate():
    """The oracle is its own gcc-built library; it shares no source with csrc/."""
    import oracle

    assert os.path.dirname(oracle.lib_path()) != os.path.join(ROOT, "paper_2602_08097_amd")
    csrc = os.path.join(ROOT, "paper_2602_08097_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "rpo_" not in text and "oracle" not in text.lower(), f
