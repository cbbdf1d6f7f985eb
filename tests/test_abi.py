"""The C-ABI library loads and exports every entry point that the public
headers declare (no compute calls: no GPU needed)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2501_12928_amd", "libeor.so")


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(eor_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared()
    for required in ("eor_create", "eor_destroy", "eor_precompute", "eor_loglike_batch",
                     "eor_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libeor.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libeor.so not built")
def test_argument_errors_without_gpu():
    import paper_2501_12928_amd as eor
    L = eor.lib()
    assert L.eor_create(0, None) == eor.EOR_ERR_ARG
    assert b"NULL" in L.eor_last_error()
    assert L.eor_loglike_batch(None, 1, None, None, None, None) == eor.EOR_ERR_ARG
    assert L.eor_precompute(None, 1, 1, None, 1, None, None, 0, None, None, None, 0, None) == eor.EOR_ERR_ARG
    assert eor.version().startswith("eor")
    # forward model: sizes, NULL arrays, leading dimension, norm (refused before any device work)
    x = np.zeros(4)
    p = x.ctypes.data
    assert L.eor_forward_model(0, 1, 1, 1, 1, p, p, p, p, p, p, 1.0, p, 1, None) == eor.EOR_ERR_ARG
    assert L.eor_forward_model(1, 1, 1, 2, 2, p, p, p, p, p, p, 1.0, p, 3, None) == eor.EOR_ERR_ARG
    assert L.eor_forward_model(1, 1, 1, 1, 1, p, None, p, p, p, p, 1.0, p, 1, None) == eor.EOR_ERR_ARG
    assert L.eor_forward_model(1, 1, 1, 1, 1, p, p, p, p, p, p, float("inf"), p, 1, None) == eor.EOR_ERR_ARG
    # every size within its own limit and under 2^31 tiles, but 2^20 x 4194240 entries of G
    assert L.eor_forward_model(1, 1 << 20, 1, 65535 * 64, 1, p, p, p, p, p, p, 1.0, p, 65535 * 64,
                               None) == eor.EOR_ERR_ARG
    assert b"2^40" in L.eor_last_error()
    # out-of-core likelihood: sizes, bin map, fixed variances and the device budget are checked first
    A = np.zeros((4, 4), dtype=np.complex128)
    db = np.zeros(4, dtype=np.complex128)
    bins = np.array([0, 0, 1, -1], dtype=np.int32)
    fv = np.array([0.0, 0.0, 0.0, 1e4])
    th = np.zeros((1, 2))
    out = np.zeros(1)
    inf_ = np.zeros(1, dtype=np.int32)
    args = lambda n, b, f, nb, lanes=0: (0, n, A.ctypes.data, 4, db.ctypes.data, 0.0, 0.0, 2, b.ctypes.data,
                                         f.ctypes.data, None, 1, th.ctypes.data, nb, lanes, out.ctypes.data,
                                         inf_.ctypes.data)
    assert L.eor_loglike_host(*args(0, bins, fv, 1 << 30)) == eor.EOR_ERR_ARG
    assert L.eor_loglike_host(*args(4, np.array([0, 2, 1, -1], dtype=np.int32), fv, 1 << 30)) == eor.EOR_ERR_ARG
    assert L.eor_loglike_host(*args(4, bins, np.zeros(4), 1 << 30)) == eor.EOR_ERR_ARG
    assert L.eor_loglike_host(*args(4, bins, fv, 1024)) == eor.EOR_ERR_OOM
    assert L.eor_loglike_host(*args(4, bins, fv, 1 << 30, 5)) == eor.EOR_ERR_ARG
    assert L.eor_loglike_host(*args(4, bins, fv, 1 << 30, -1)) == eor.EOR_ERR_ARG


def _moved(N, J):
    """Tiles over the host link per theta for N tile rows in passes of J."""
    t = N * (N + 1) // 2
    for j0 in range(0, N, J):
        j1 = min(N, j0 + J)
        t += j0 * (N - j0) + (j1 - j0) * (N - j1)
    return t


def test_out_of_core_plan():
    """The out-of-core schedule, computed on the host without a device call:
    pass width from the device budget per lane (a lane's tiles in whole
    full-height tile columns, less min(4, half) of them for the window of
    earlier columns), the automatic lane count, and the host <-> device bytes
    per theta (A once, every earlier tile column's rows below a pass once per
    pass, and rows j1 .. N-1 of each pass's columns written back)."""
    import paper_2501_12928_amd as eor
    tile = 64 * 64 * 16
    N = 64
    # one lane at 256 MiB, n = 4096: 4091 tiles after the vectors = 63 columns -> 59 per pass
    p = eor.loglike_host_plan(4096, 12, 256 << 20, lanes=1)
    assert p["lanes"] == 1 and p["cols_per_pass"] == 59
    assert p["window_tiles"] == 4091 - 59 * N
    assert p["link_bytes"] == _moved(N, 59) * tile
    # automatic: four lanes would leave 1020 tiles each (< 2 x 8 x 64), three leave 1361 = 21 columns -> 17
    p = eor.loglike_host_plan(4096, 12, 256 << 20)
    assert p["lanes"] == 3 and p["cols_per_pass"] == 17 and p["window_tiles"] == 1361 - 17 * N
    assert p["link_bytes"] == _moved(N, 17) * tile
    # two lanes leave 2044 = 31 columns -> 27
    p = eor.loglike_host_plan(4096, 12, 256 << 20, lanes=2)
    assert p["lanes"] == 2 and p["cols_per_pass"] == 27 and p["window_tiles"] == 2044 - 27 * N
    assert p["link_bytes"] == _moved(N, 27) * tile
    # 64 tile rows, passes of 27: A 2080 tiles, earlier rows 27 x 37 + 54 x 10, written back 27 x 37 + 27 x 10
    assert _moved(N, 27) == 2080 + 999 + 540 + 999 + 270
    # the smallest budget of the GPU tests (n = 333: 6 tile rows, 14 tiles): one lane, one column per pass
    p = eor.loglike_host_plan(333, 4, 14 * tile)
    assert p == {"lanes": 1, "cols_per_pass": 1, "window_tiles": 6,
                 "link_bytes": _moved(6, 1) * tile}
    # a roomy budget: four lanes, each holding the whole matrix in one pass
    p = eor.loglike_host_plan(333, 4, 1 << 30)
    assert p["lanes"] == 4 and p["cols_per_pass"] == 6 and p["link_bytes"] == 21 * tile  # A only
    # explicit lanes that do not fit, and arguments out of range
    L = eor.lib()
    assert L.eor_loglike_host_plan(333, 4, 14 * tile, 2, None, None, None, None) == eor.EOR_ERR_OOM
    assert L.eor_loglike_host_plan(333, 4, 1 << 30, 5, None, None, None, None) == eor.EOR_ERR_ARG
    assert L.eor_loglike_host_plan(0, 4, 1 << 30, 0, None, None, None, None) == eor.EOR_ERR_ARG


def test_product_package_does_not_reference_oracle():
    """The product path never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2501_12928_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".h", ".cpp")):
            text = open(path).read()
            assert "import oracle" not in text and "from oracle" not in text, path
            assert "liboracle" not in text and "oracle.c" not in text, path
