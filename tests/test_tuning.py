"""The library's tuning-file reader (host only, no GPU): a scene takes the
class with the largest min_verts not above its vertex count; values are
clamped to what the kernels support; unknown keys and a trailing
measurements section are ignored; no file (or an empty path) gives the
built-in defaults."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def query(path, sizes):
    code = ("import json, sys; sys.path.insert(0, %r); from paper_2411_04776_amd import ipc; "
            "print(json.dumps([ipc.tuning_for(n) for n in %r]))" % (ROOT, list(sizes)))
    env = dict(os.environ, IPC_TUNING_FILE=path)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tuning_file_classes(tmp_path):
    from paper_2411_04776_amd import ipc
    if not os.path.exists(ipc.LIB_PATH):
        pytest.skip("library not built")
    f = tmp_path / "tuning.json"
    f.write_text(json.dumps({
        "classes": [
            {"min_verts": 65536, "name": "large", "spmv_one_lane_rows": 0, "mas_target": 192,
             "pcg_first_chunk": 0.75, "pcg_later_chunk": 0.125, "pcg_list_quantile": 3.0},
            {"min_verts": 0, "name": "small", "spmv_one_lane_rows": 131072, "mas_target": 4096,
             "pcg_first_chunk": 1.0, "pcg_later_chunk": 0.25}],
        "measurements": [{"min_verts": 99, "mas_target": 1}]}))
    small, edge, large = query(str(f), [1000, 65535, 65536])
    assert small == edge
    assert small["spmv_one_lane_rows"] == 131072 and small["mas_target"] == 256   # clamped to the group cap
    assert small["pcg_first_chunk"] == 1.0 and small["from_file"]
    assert large["spmv_one_lane_rows"] == 0 and large["mas_target"] == 192 and large["pcg_later_chunk"] == 0.125
    assert large["pcg_list_quantile"] == 1.0 and small["pcg_list_quantile"] == 0.25   # clamped; default


def test_no_tuning_file_gives_defaults(tmp_path):
    from paper_2411_04776_amd import ipc
    if not os.path.exists(ipc.LIB_PATH):
        pytest.skip("library not built")
    for path in ("", str(tmp_path / "missing.json")):
        (d,) = query(path, [5000])
        assert d == {"spmv_one_lane_rows": 65536, "mas_target": 256, "pcg_first_chunk": 0.875,
                     "pcg_later_chunk": 0.25, "from_file": False, "pcg_list_quantile": 0.25}
