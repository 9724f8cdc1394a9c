"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports
every function include/xct.h declares; argument errors need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xct.h")
LIB = os.path.join(ROOT, "paper_2009_07226_amd", "libxct.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xct_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("xct_build_matrix", "xct_project", "xct_backproject", "xct_cgls", "xct_free_matrix",
                     "xct_matrix_info", "xct_last_error", "xct_cgls_workspace_bytes", "xct_spmm_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libxct.so has not been built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_device():
    import paper_2009_07226_amd as xct
    L = xct.lib()
    h = ctypes.c_void_p()
    assert L.xct_build_matrix(0, 10, 10, 0, None, None, ctypes.byref(h)) == -1
    assert b"n must be" in L.xct_last_error()
    assert L.xct_build_matrix(8, 10, 10, 7, None, None, ctypes.byref(h)) == -1
    assert L.xct_project(None, None, None, 1, 0, None, None) == -1
    assert L.xct_cgls(None, None, 0, None, 1, 1, None, None, None, None) == -1
    assert L.xct_spmm_workspace_bytes(None, 4) == 0
    assert L.xct_stream_workspace_bytes(None, 0, 4, 0) == 0
    assert L.xct_project_streamed(None, None, None, 1, 1, 0, None, None, None, None) == -1
    assert L.xct_backproject_streamed(None, None, None, 1, 1, 0, None, None, None, None) == -1
    assert L.xct_cgls_workspace_bytes(None, 4, 3) == 0
    assert L.xct_pgrad_workspace_bytes(None, 4) == 0
    assert L.xct_projected_gradient(None, None, None, 1, 1, None, 0.0, 0.1, 1, None, None) == -1
    assert b"NULL" in L.xct_last_error()
    g = ctypes.c_double()
    assert L.xct_read_bandwidth(None, 1 << 20, 1, ctypes.byref(g), None) == -1
    assert L.xct_profile_read(None, None) == -1
    assert L.xct_count_nonfinite(None, 4, 0, None, None) == -1
    assert L.xct_device_memory(None, None) == -1
    # no matrix built in this process: the library holds no device memory
    assert xct.device_memory() == {"buffers": 0, "bytes": 0}


def test_workspace_checks_in_the_binding():
    # a caller-supplied workspace is checked before the C ABI (which takes no
    # size) could write past it: device, contiguity and byte count
    import torch
    from paper_2009_07226_amd import xct as binding
    dev = torch.device("cpu")
    binding._require_workspace(torch.empty(64, dtype=torch.uint8), 64, dev)
    binding._require_workspace(torch.empty(16, dtype=torch.float32), 64, dev)  # 64 bytes
    with pytest.raises(ValueError, match="needs 65"):
        binding._require_workspace(torch.empty(64, dtype=torch.uint8), 65, dev)
    with pytest.raises(ValueError, match="must be on"):
        binding._require_workspace(torch.empty(64, dtype=torch.uint8), 1, torch.device("cuda", 0))
    with pytest.raises(ValueError, match="contiguous"):
        binding._require_workspace(torch.empty(8, 8, dtype=torch.uint8).t(), 1, dev)
    with pytest.raises(TypeError):
        binding._require_workspace(bytearray(64), 1, dev)


def _header_struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\}\s*" + name + r"\s*;", text, flags=re.S).group(1)
    return [(t, f) for t, f in re.findall(r"\b(int|int32_t|int64_t|double)\s+(\w+)\s*;", body)]


def test_binding_structs_match_the_header():
    """The ctypes mirrors of the header's option and statistics structs have
    the same fields in the same order and types."""
    import ctypes as C
    from paper_2009_07226_amd import xct
    ctype = {"int": C.c_int, "int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double}
    for cname, py in (("xct_build_opts", xct.BuildOpts),):
        want = [(f, ctype[t]) for t, f in _header_struct_fields(cname)]
        got = [(f, t) for f, t in py._fields_]
        assert [f for f, _ in got] == [f for f, _ in want], (cname, got, want)
        assert all(C.sizeof(a) == C.sizeof(b) for (_, a), (_, b) in zip(got, want))
