"""ctypes binding of ``libb64hip.so`` (declarations in ``include/b64.h``).

Argument marshalling only: every step of encoding and decoding runs in the
library's gfx950 kernels. Loading fails loudly when the library is missing.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libb64hip.so")

OK = 0
INVALID_INPUT = -1
BAD_ARG = -2
HIP_ERROR = -3
POOL_FULL = -4
TIMEOUT = -5

ALPHABET_STD = 0
ALPHABET_URL = 1
MODE_STRICT = 0x100
MODE_NOPAD = 0x200

FLAG_URL = 0x01
FLAG_STRICT = 0x02
FLAG_NOPAD = 0x04

DIR_ENCODE = 0
DIR_DECODE = 1

NOALLOC_MAX_MESSAGES = 1 << 20


class Tune(ctypes.Structure):
    """``b64_tune``: launch shape of the persistent batched kernels."""
    _fields_ = [("block", ctypes.c_int32), ("units_per_lane", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("layout", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    """``b64_server_cfg``."""
    _fields_ = [("max_batch", ctypes.c_int32), ("tick_us", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("capture", ctypes.c_int32), ("idle_sleep_us", ctypes.c_int32), ("block", ctypes.c_int32),
                ("units_per_lane", ctypes.c_int32), ("grid", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("time_scale", ctypes.c_double), ("max_seconds", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    """``b64_server_stats``."""
    _fields_ = [("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("launched_requests", ctypes.c_int64), ("pool_waits", ctypes.c_int64),
                ("max_inflight_batches", ctypes.c_int64), ("bytes_in", ctypes.c_int64),
                ("bytes_out", ctypes.c_int64), ("peak_pool_bytes", ctypes.c_int64),
                ("wall_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_i64, _i32, _p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
_pi64 = ctypes.POINTER(ctypes.c_int64)
_ptune = ctypes.POINTER(Tune)

# name -> (restype, argtypes); mirrors include/b64.h
SIGNATURES = {
    "b64_encoded_len": (_i64, [_i64]),
    "b64_encoded_len_mode": (_i64, [_i64, _i32]),
    "b64_decoded_max": (_i64, [_i64]),
    "b64_decoded_max_mode": (_i64, [_i64, _i32]),
    "b64_encode": (_i64, [_p, _i64, _p]),
    "b64_decode": (_i64, [_p, _i64, _p, _pi64]),
    "b64_encode_ex": (_i64, [_p, _i64, _p, _i32, _p]),
    "b64_decode_ex": (_i64, [_p, _i64, _p, _pi64, _i32, _p]),
    "b64_decode_async": (_i32, [_p, _i64, _p, _i32, _p, _p, _p]),
    "b64_decode_ws_workspace_bytes": (_i64, [_i64]),
    "b64_decode_ws_async": (_i32, [_p, _i64, _p, _i32, _p, _p, _p, _i64, _p]),
    "b64_decode_ws": (_i64, [_p, _i64, _p, _pi64, _i32, _p]),
    "b64_set_ws_tune": (_i32, [_ptune]),
    "b64_batch_out_offsets": (_i32, [_i32, _p, _i64, _p, _p, _p]),
    "b64_batch_slots": (_i32, [_i32, _p, _p, _i64, _p, _p]),
    "b64_batch_workspace_bytes": (_i64, [_i64]),
    "b64_encode_batch": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p, _i64, _ptune, _p]),
    "b64_decode_batch": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p, _p, _i64, _ptune, _p]),
    "b64_decode_batch_noalloc": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p, _ptune, _p]),
    "b64_encode_each": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p]),
    "b64_decode_each": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p, _p]),
    "b64_set_single_tune": (_i32, [_i32, _ptune]),
    "b64_encode_batch_gather": (_i32, [_p, _p, _p, _i64, _p, _p, _p, _p, _p, _i64, _ptune, _p]),
    "b64_decode_batch_gather": (_i32, [_p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _i64, _ptune, _p]),
    "b64_graph_create_batch": (_i32, [_i32, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _i64, _ptune,
                                      ctypes.POINTER(_p)]),
    "b64_graph_update_batch": (_i32, [_p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _i64, _ptune]),
    "b64_graph_launch": (_i32, [_p, _p]),
    "b64_graph_destroy": (_i32, [_p]),
    "b64_pool_create": (_i32, [_i64, _i64, ctypes.POINTER(_p)]),
    "b64_pool_alloc": (_i32, [_p, _i64, _pi64]),
    "b64_pool_free": (_i32, [_p, _i64]),
    "b64_pool_free_bytes": (_i64, [_p]),
    "b64_pool_peak_bytes": (_i64, [_p]),
    "b64_pool_destroy": (_i32, [_p]),
    "b64_server_run": (_i32, [ctypes.POINTER(ServerCfg), _i64, _p, _p, _p, _p, _p, _p, _i64, _p, _i64,
                              _p, _p, _p, _p, _p, _p, ctypes.POINTER(ServerStats)]),
    "b64_last_error": (ctypes.c_char_p, []),
    "b64_device_cus": (_i32, []),
}

_lib = None


class B64Error(RuntimeError):
    pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise B64Error(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().b64_last_error().decode()


def check(rc, what):
    """Raise on argument / runtime errors (codes -2, -3)."""
    if rc in (BAD_ARG, HIP_ERROR):
        raise B64Error(f"{what}: {last_error()} (code {rc})")
    return rc
