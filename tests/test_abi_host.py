"""Host-side checks of the C ABI: the library loads, exports every function
that include/mcd.h declares, and its argument validation needs no GPU."""
import ctypes

import pytest

M = pytest.importorskip("paper_2412_12382_amd.mcd")


def test_exports_every_declared_function():
    L = M.lib()
    names = M.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing


def test_status_strings():
    for code, name in M.STATUS.items():
        assert M.mcd_status_string(code) == name


def test_sizes_validation():
    st, ws = M.mcd_graph_build_sizes(1000, 100)
    assert st >= 8 * 101 + 2 * 4 * 1000 + 2 * 4 * 100 and ws > 3 * 8 * 1000
    with pytest.raises(M.MCDError) as ei:
        M.mcd_graph_build_sizes(-1, 10)
    assert ei.value.status == -1
    with pytest.raises(M.MCDError) as ei:
        M.mcd_graph_build_sizes(10, 1 << 31)
    assert ei.value.status == -3


def test_null_arguments_rejected_without_device():
    L = M.lib()
    assert L.mcd_ctx_create(0, None, None) == -1
    assert L.mcd_graph_info(None, None, None, None, None) == -1
    assert L.mcd_triangles(None, None, None, 0) == -1
    assert L.mcd_run(None, 0, M.mcd_rational(1, 2), None, None, None, 0) == -1


def test_no_device_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert M.lib().mcd_ctx_create(0, None, ctypes.byref(h)) == -5


def test_kept_segments_constant_matches_header():
    import re
    text = open(M.HEADER).read()
    v = int(re.search(r"#define MCD_KEPT_SEGMENTS (\d+)", text).group(1))
    assert v == M.KEPT_SEGMENTS
