"""CPU-side checks of the C-ABI library: it loads, exports every function
declared in include/b64.h, and its pure-host functions and argument checks
behave as documented (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

from paper_1704_00605_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "b64.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(b64_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"


def test_library_is_gfx950_code_object():
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_length_functions(L):
    for n in range(0, 100):
        assert L.b64_encoded_len(n) == 4 * -(-n // 3)
        assert L.b64_decoded_max(n) == 3 * (n // 4)
        nopad = L.b64_encoded_len_mode(n, _lib.MODE_NOPAD)
        assert nopad == 4 * (n // 3) + ((n % 3) + 1 if n % 3 else 0)
        assert L.b64_decoded_max_mode(n, _lib.MODE_NOPAD) == 3 * (n // 4) + max(0, n % 4 - 1)
    assert L.b64_encoded_len(-1) == _lib.BAD_ARG
    assert L.b64_decoded_max(-5) == _lib.BAD_ARG
    assert L.b64_encoded_len((1 << 40) + 1) == 4 * -(-((1 << 40) + 1) // 3)


def test_argument_errors_need_no_gpu(L):
    err = ctypes.c_int64(0)
    assert L.b64_encode_ex(None, 0, None, 0, None) == 0
    assert L.b64_encode_ex(None, 10, None, 0, None) == _lib.BAD_ARG
    assert L.b64_encode_ex(None, 0, None, 7, None) == _lib.BAD_ARG
    assert "alphabet" in _lib.last_error()
    assert L.b64_encode_ex(None, -1, None, 0, None) == _lib.BAD_ARG
    assert L.b64_decode_ex(None, 0, None, ctypes.byref(err), 0, None) == 0 and err.value == -1
    assert L.b64_decode_ex(None, 8, None, None, 0, None) == _lib.BAD_ARG
    assert L.b64_decode_ex(None, 0, None, ctypes.byref(err),
                           _lib.MODE_STRICT | _lib.MODE_NOPAD, None) == _lib.BAD_ARG
    assert L.b64_decode_async(None, 4, None, 0, None, None, None) == _lib.BAD_ARG
    assert L.b64_batch_workspace_bytes(-1) == _lib.BAD_ARG
    assert L.b64_batch_workspace_bytes(0) > 0
    assert L.b64_batch_workspace_bytes(100000) >= 8 * 100001
    assert L.b64_encode_batch(None, None, -1, None, None, None, None, None, 0, None, None) == _lib.BAD_ARG
    assert L.b64_encode_batch(None, None, 0, None, None, None, None, None, 0, None, None) == 0
    assert L.b64_decode_ws_workspace_bytes(-1) == _lib.BAD_ARG
    assert L.b64_decode_ws_workspace_bytes(1 << 30) >= 8 * ((1 << 30) // 2048)
    assert L.b64_decode_ws(None, 0, None, ctypes.byref(err), 0, None) == 0 and err.value == -1
    assert L.b64_decode_ws(None, 4, None, ctypes.byref(err), _lib.MODE_STRICT, None) == _lib.BAD_ARG
    assert L.b64_decode_ws(None, 1 << 38, None, ctypes.byref(err), 0, None) == _lib.BAD_ARG
    assert L.b64_decode_ws_async(None, 8, None, 0, None, None, None, 0, None) == _lib.BAD_ARG
    assert L.b64_decode_ws_async(None, 0, None, 0, None, None, None, 0, None) == _lib.BAD_ARG  # empty input, no slots
    for d, m in ((0, 3), (1, 2), (0, -1)):
        assert L.b64_set_single_tune(d, ctypes.byref(_lib.Tune(block=0, units_per_lane=0, grid=0, layout=m))) == _lib.BAD_ARG
    assert L.b64_set_single_tune(0, ctypes.byref(_lib.Tune(block=0, units_per_lane=0, grid=0, layout=0))) == 0
    ws_bad = _lib.Tune(block=384, units_per_lane=2, grid=0, layout=0)
    assert L.b64_set_ws_tune(ctypes.byref(ws_bad)) == _lib.BAD_ARG
    bad = _lib.Tune(block=100, units_per_lane=0, grid=0, layout=0)
    assert L.b64_set_single_tune(0, ctypes.byref(bad)) == _lib.BAD_ARG
    assert L.b64_set_single_tune(5, ctypes.byref(bad)) == _lib.BAD_ARG


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.B64Error):
        _lib.lib()


def test_batch_slots_host_layout(L):
    """b64_batch_slots against the length law written out: encoded lengths
    (padded and unpadded), decode capacities rounded to 4-byte slots."""
    import numpy as np
    from paper_1704_00605_amd import codec

    rng = np.random.default_rng(3)
    lens = np.concatenate([np.arange(0, 70), rng.integers(0, 1 << 40, 50)]).astype(np.int64)
    flags = rng.integers(0, 8, lens.size).astype(np.uint8)
    nopad = (flags & _lib.FLAG_NOPAD) != 0
    need, oo = codec.batch_slots(_lib.DIR_ENCODE, lens, flags)
    enc_pad = 4 * ((lens + 2) // 3)
    enc_nopad = 4 * (lens // 3) + np.where(lens % 3, lens % 3 + 1, 0)
    assert np.array_equal(need, np.where(nopad, enc_nopad, enc_pad))
    assert oo[0] == 0 and np.array_equal(np.diff(oo), enc_pad)
    need, oo = codec.batch_slots(_lib.DIR_DECODE, lens, flags)
    cap = 3 * (lens // 4) + np.where(nopad & (lens % 4 >= 2), lens % 4 - 1, 0)
    assert np.array_equal(need, cap)
    assert np.array_equal(np.diff(oo), (cap + 3) // 4 * 4)
    need, oo = codec.batch_slots(_lib.DIR_DECODE, np.zeros(0, np.int64))
    assert need.size == 0 and oo.tolist() == [0]
    with pytest.raises(_lib.B64Error):
        codec.batch_slots(_lib.DIR_ENCODE, np.array([5, -1], np.int64))
