"""Host-only checks of the C ABI (no GPU): the library loads, exports every
function its header declares, and its pure-host calls behave."""
import ctypes
import glob
import os
import math

import numpy as np
import pytest

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import _lib


def test_exports_every_declared_symbol():
    lib = rfi.load()
    declared = _lib.header_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(_lib._SIGS), "binding and header disagree"


def test_version_and_status_strings():
    lib = rfi.load()
    assert b"gfx950" in lib.rfi_version()
    for code in (0, -1, -2, -3, -4, -6):
        assert lib.rfi_status_string(code)


def test_layout_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        L = rng.integers(0, 100000, n)
        W = rng.integers(1, 65537, n)
        so, wo, nw, total = rfi.layout(L, W)
        so2, wo2, nw2 = oracle.layout(L, W)
        assert np.array_equal(so, so2) and np.array_equal(wo, wo2) and nw == nw2
        assert total == int(so[-1]) + (int(L[-1]) + 63) // 64 * 64


def test_layout_rejects():
    lib = rfi.load()
    L = np.array([10], np.int64)
    for W in (0, 65537, -3):
        Wa = np.array([W], np.int32)
        assert lib.rfi_layout(1, L.ctypes.data, Wa.ctypes.data, None, None, None) == -1
    Lb = np.array([-1], np.int64)
    Wa = np.array([4], np.int32)
    assert lib.rfi_layout(1, Lb.ctypes.data, Wa.ctypes.data, None, None, None) == -1


def test_validate():
    base = 1 << 20  # pretend device addresses: validate never dereferences
    ok = dict(elem_size=1, x_ptr=base, y_ptr=base + (1 << 16), lengths=[4096, 100],
              windows=[4096, 10], k=[3.0, 2.5], mode=[0, 2])
    assert _lib.validate(**ok) == 0
    assert _lib.validate(**{**ok, "y_ptr": ok["x_ptr"]}) == 0  # in place
    assert _lib.validate(**{**ok, "x_ptr": base + 1}) == -2
    assert _lib.validate(**{**ok, "y_ptr": base + 16}) == -1  # partial overlap
    assert _lib.validate(**{**ok, "k": [3.0, math.inf]}) == -1
    assert _lib.validate(**{**ok, "k": [3.0, 1e4 + 1]}) == -1
    assert _lib.validate(**{**ok, "k": [-0.1, 1.0]}) == -1
    assert _lib.validate(**{**ok, "mode": [0, 3]}) == -1
    assert _lib.validate(**{**ok, "windows": [0, 10]}) == -1
    assert _lib.validate(**{**ok, "elem_size": 4}) == -1
    assert _lib.validate(**{**ok, "x_ptr": 0}) == -1
    assert _lib.validate(**{**ok, "lengths": [0, 0], "x_ptr": 0, "y_ptr": 0}) == 0
    # stats overlapping the output
    assert _lib.validate(**{**ok, "stats_ptr": ok["y_ptr"]}) == -1
    assert _lib.validate(**{**ok, "stats_ptr": base + (1 << 18)}) == 0
    assert _lib.validate(**{**ok, "stats_ptr": base + (1 << 18) + 4}) == -2


def test_no_cpu_fallback():
    """Without a device the filter entry point must fail, not compute."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = rfi.load()
    h = ctypes.c_void_p()
    L = np.array([4096], np.int64)
    W = np.array([4096], np.int32)
    K = np.array([3.0], np.float32)
    M = np.array([1], np.int32)
    rc = lib.rfi_plan_create(1, 1, L.ctypes.data, W.ctypes.data, K.ctypes.data, M.ctypes.data, 0,
                             ctypes.byref(h))
    assert rc != 0


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: --gpus above 1 exits with a message, before touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_profile_summaries_parse():
    # every committed profile summary names its command and, for the traffic
    # summary, the calibration and the kernel-source hash bench.py checks
    from paper_1710_08576_amd import profiling
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    mds = sorted(glob.glob(os.path.join(root, "profiles", "*.md")))
    assert mds
    for fn in mds:
        text = open(fn).read()
        assert "rocprofv3" in text, fn
    summ = profiling.load_summary(os.path.join(root, "profiles", "i8_w4096_plain_scale.md"))
    assert summ["calibration"]["copy_bytes"] > 0
    assert len(summ["kernel_source_sha256"]) == 64


def test_tune_table_json_round_trip(tmp_path):
    """rfi_tune_load reads the JSON that rfi_tune_save writes (host only):
    hand-written entries come back with the same keys and choices, malformed
    files are refused whole."""
    import json
    src = tmp_path / "tune_in.json"
    entries = [
        {"arch": "gfx950", "signature": "0000000300003e01", "schedule": "fused", "tiles_per_wg": 1,
         "wg_per_cu": 8, "ms": 0.23},
        {"arch": "gfx950", "signature": "0000000000000802", "schedule": "one_launch_persist",
         "tiles_per_wg": 2, "wg_per_cu": 0, "ms": 0.5},
        {"arch": "gfx942", "signature": "0000000000000801", "schedule": "split", "tiles_per_wg": 1,
         "wg_per_cu": 6, "ms": 1.0},
    ]
    src.write_text(json.dumps({"format": "rfimad autotune 1", "entries": entries}, indent=1))
    rfi.tune_load(str(src))
    out = tmp_path / "tune_out.json"
    rfi.tune_save(str(out))
    got = json.loads(out.read_text())["entries"]
    keyed = {(e["arch"], e["signature"]): e for e in got}
    for e in entries:
        g = keyed[(e["arch"], e["signature"])]
        for k in ("schedule", "tiles_per_wg", "wg_per_cu"):
            assert g[k] == e[k], (e, g)
        assert g["ms"] == pytest.approx(e["ms"], rel=1e-5)
    # readable fields of the signature: int8, classes 512..16384 but 1024
    g = keyed[("gfx950", "0000000300003e01")]
    assert g["elem_size"] == 1 and g["window_classes"] == [1024, 2048, 4096, 8192, 16384]
    assert g["noise"] is True and g["generic_items"] is True and g["irregular_windows"] is False
    # a second save of the loaded file is identical
    out2 = tmp_path / "tune_out2.json"
    rfi.tune_load(str(out))
    rfi.tune_save(str(out2))
    assert json.loads(out2.read_text()) == json.loads(out.read_text())
    # malformed: unknown schedule, bad tiles per workgroup, not a table, missing file
    for bad in ('{"entries": [{"arch": "gfx950", "signature": "1", "schedule": "nope", '
                '"tiles_per_wg": 1, "wg_per_cu": 8}]}',
                '{"entries": [{"arch": "gfx950", "signature": "1", "schedule": "fused", '
                '"tiles_per_wg": 3, "wg_per_cu": 8}]}',
                '[1, 2, 3]'):
        f = tmp_path / "bad.json"
        f.write_text(bad)
        with pytest.raises(rfi.RfiError):
            rfi.tune_load(str(f))
    with pytest.raises(rfi.RfiError):
        rfi.tune_load(str(tmp_path / "missing.json"))


def test_kernel_source_hash_ignores_comments(tmp_path):
    # the hash that ties a profile to the kernels it was taken on changes
    # with the code and not with comments or layout
    import shutil
    from paper_1710_08576_amd import profiling
    for rel in profiling.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(profiling.HERE, rel), dst)
    h0 = profiling.kernel_source_hash(str(tmp_path))
    assert h0 == profiling.kernel_source_hash()
    k = tmp_path / "csrc" / "rfi_kernels.hip"
    text = k.read_text()
    k.write_text("// a new comment\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n", 3))
    assert profiling.kernel_source_hash(str(tmp_path)) == h0
    d = tmp_path / "csrc" / "rfi_device.hpp"
    d.write_text(d.read_text() + "\nstatic const int extra_code = 1;\n")
    assert profiling.kernel_source_hash(str(tmp_path)) != h0
