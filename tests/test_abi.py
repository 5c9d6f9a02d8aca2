"""The C-ABI library loads and exports every entry point include/ipc.h
declares; the product and the oracle share no code. No compute calls: these
run without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipc.h")
PKG = os.path.join(ROOT, "paper_2411_04776_amd")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"IPC_API\s+[\w\s\*]*?\b((?:ipc|ipcx)_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ipc_create_scene", "ipc_step", "ipc_read_surface", "ipc_batch_submit"):
        assert required in names
    assert len(names) >= 25


def test_library_exports_every_declared_symbol():
    from paper_2411_04776_amd import ipc
    if not os.path.exists(ipc.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(ipc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared names
    assert sorted(ipc.EXPORTED) == declared_functions()


def test_status_strings_without_gpu():
    from paper_2411_04776_amd import ipc
    if not os.path.exists(ipc.LIB_PATH):
        pytest.skip("library not built")
    L = ipc.lib()
    assert L.ipc_status_str(0) == b"ok"
    assert b"bad mesh" in L.ipc_status_str(ipc.IPC_E_BAD_MESH)


def _sources(d, exts):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(exts):
                yield os.path.join(root, f)


def test_product_and_oracle_share_no_code():
    for path in _sources(PKG, (".py", ".hip", ".h", ".cpp")):
        text = open(path).read()
        assert "ipc_oracle" not in text and "import oracle" not in text and "from oracle" not in text, path
    for path in _sources(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        text = open(path).read()
        assert "paper_2411_04776_amd" not in text.replace("paper_2411_04776_amd/scenes", ""), path
        assert "ipc.h" not in text and "ipc_internal" not in text, path


def test_binding_structs_match_the_library():
    """The ctypes layouts of the boundary's structs have the sizes the
    library was compiled with (fields appended on one side only would shift
    every later field)."""
    from paper_2411_04776_amd import ipc
    if not os.path.exists(ipc.LIB_PATH):
        pytest.skip("library not built")
    out = (ctypes.c_int64 * 5)()
    assert ipc.lib().ipcx_struct_sizes(out) == 0
    mine = [ctypes.sizeof(t) for t in (ipc.ipc_scene_desc, ipc.ipc_runtime, ipc.ipc_step_req, ipc.ipc_step_stats,
                                       ipc.ipc_height_map_spec)]
    assert list(out) == mine, (list(out), mine)
