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
    # the largest input: 2^31 - 1 raw pairs, n below 2^31 - 1
    st, ws = M.mcd_graph_build_sizes((1 << 31) - 1, (1 << 31) - 2)
    assert st > 8 * ((1 << 31) - 1) and ws > 8 * ((1 << 31) - 1)
    for pairs, n in (((1 << 31), 10), (10, (1 << 31) - 1)):
        with pytest.raises(M.MCDError) as ei:
            M.mcd_graph_build_sizes(pairs, n)
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


def _checkpoint_bytes(params, mean, std, lo, hi, margin=0.25, version=1, grid=(64, 9, 7, 900), shape=(66, 64, 8513)):
    """A picker checkpoint laid out as include/mcd.h documents it, with the
    IEEE CRC-32 of zlib."""
    import struct
    import zlib

    import numpy as np
    head = b"MCDPICK\0" + struct.pack("<IIII", version, *shape) + struct.pack("<ii", grid[0], 0)
    head += struct.pack("<qqq", *grid[1:]) + struct.pack("<fI", margin, 0)
    assert len(head) == 64
    body = np.concatenate([np.asarray(a, "<f4") for a in (params, mean, std, lo, hi)]).tobytes()
    data = head + body
    return data + struct.pack("<I", zlib.crc32(data))


def test_picker_checkpoint_checks_on_host(tmp_path):
    import numpy as np
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.1, 8513).astype(np.float32)
    mean, std = rng.normal(0, 1, 66), rng.uniform(0.5, 2, 66)
    lo, hi = -np.ones(66), np.ones(66)
    good = _checkpoint_bytes(p, mean, std, lo, hi)
    assert len(good) == 64 + 4 * (8513 + 4 * 66) + 4
    path = tmp_path / "picker.ckpt"

    def status(data):
        path.write_bytes(data)
        try:
            M.mcd_picker_check_file(str(path))
            return 0
        except M.MCDError as e:
            return e.status

    assert status(good) == 0
    flipped = bytearray(good)
    flipped[64 + 4 * 100] ^= 0x10  # one bit of a weight: the CRC no longer matches
    bad_std = std.copy()
    bad_std[3] = 0.0
    nan_p = p.copy()
    nan_p[7] = np.nan
    cases = {
        "bit flip": bytes(flipped),
        "truncated": good[:-1],
        "trailing byte": good + b"\0",
        "bad magic": b"MCDPICX\0" + good[8:],
        "version 2": _checkpoint_bytes(p, mean, std, lo, hi, version=2),
        "other grid": _checkpoint_bytes(p, mean, std, lo, hi, grid=(64, 9, 7, 1000)),
        "other shape": _checkpoint_bytes(p, mean, std, lo, hi, shape=(66, 32, 8513)),
        "zero std": _checkpoint_bytes(p, mean, bad_std, lo, hi),
        "nan weight": _checkpoint_bytes(nan_p, mean, std, lo, hi),
        "negative margin": _checkpoint_bytes(p, mean, std, lo, hi, margin=-0.5),
        "empty": b"",
    }
    for name, data in cases.items():
        assert status(data) == -9, name
    missing = tmp_path / "absent.ckpt"
    with pytest.raises(M.MCDError) as ei:
        M.mcd_picker_check_file(str(missing))
    assert ei.value.status == -9
    assert M.lib().mcd_picker_check_file(None) == -1
    assert M.mcd_status_string(-9) == "MCD_ERR_CHECKPOINT"


def test_picker_calls_reject_null_without_device():
    L = M.lib()
    assert L.mcd_picker_create(None, 0, None) == -1
    assert L.mcd_picker_pick(None, None, 0, None, 1, None, 0, None, None, None, None, None, None, 0) == -1
    assert L.mcd_picker_load(None, b"x") == -1
    assert L.mcd_picker_save(None, b"x") == -1
    assert L.mcd_picker_destroy(None) == 0


def test_tune_cache_file_checks_on_host(tmp_path):
    import json
    entry = {"arch": "gfx950:sramecc+:xnack-", "tune_version": 2, "log2_n": 20, "log2_m": 23, "ms": 12.5,
             "params": {"tc_chunk": 512, "tc_lds_max": 4096, "tc_packed_range": 1048574, "tc_window_max": 262144,
                        "tc_window_occupancy": 1, "sweep_shape": 0}}
    good = {"format": "mcd-tune-cache", "version": 1, "entries": [entry]}
    path = tmp_path / "tune.json"

    def status(text):
        path.write_text(text)
        try:
            M.mcd_tune_cache_check_file(str(path))
            return 0
        except M.MCDError as e:
            return e.status

    assert status(json.dumps(good)) == 0
    assert status(json.dumps({"format": "mcd-tune-cache", "version": 1, "entries": []})) == 0
    bad_param = json.loads(json.dumps(good))
    bad_param["entries"][0]["params"]["tc_chunk"] = "512"
    no_arch = json.loads(json.dumps(good))
    del no_arch["entries"][0]["arch"]
    cases = {
        "truncated": json.dumps(good)[:-3],
        "trailing text": json.dumps(good) + " x",
        "other format": json.dumps(dict(good, format="something-else")),
        "version 2": json.dumps(dict(good, version=2)),
        "entries not a list": json.dumps(dict(good, entries={})),
        "string parameter": json.dumps(bad_param),
        "entry without arch": json.dumps(no_arch),
        "not an object": "[1, 2, 3]",
        "empty": "",
        "deep nesting": "[" * 64 + "]" * 64,
    }
    for name, text in cases.items():
        assert status(text) == -9, name
    M.mcd_tune_cache_check_file(str(tmp_path / "absent.json"))  # a missing file is an empty cache
    L = M.lib()
    assert L.mcd_tune_cache_check_file(None) == -1
    assert L.mcd_tune_cache_load(None, None, b"x", None) == -1
    assert L.mcd_tune_cache_store(None, None, b"x", ctypes.c_float(1.0)) == -1
