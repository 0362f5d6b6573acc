"""Torch-facing API of the gfx950 base64 codec.

PyTorch only supplies device memory and streams: every function here passes
tensor pointers and sizes to ``libb64hip.so`` (see ``include/b64.h``), whose
HIP kernels do all the work (Algorithm 1 encoding and validating Algorithm 2
decoding of Section 2 of the paper).
"""
import ctypes

import torch

from . import _lib
from ._lib import (ALPHABET_STD, ALPHABET_URL, DIR_DECODE, DIR_ENCODE, FLAG_NOPAD, FLAG_STRICT,
                   FLAG_URL, MODE_NOPAD, MODE_STRICT, NOALLOC_MAX_MESSAGES, B64Error, Tune, check, lib)

__all__ = [
    "encode", "decode", "decode_async", "encoded_len", "decoded_max", "batch_out_offsets", "batch_slots",
    "encode_batch", "decode_batch", "decode_batch_noalloc", "encode_batch_gather", "decode_batch_gather", "encode_each", "decode_each",
    "workspace_bytes", "Workspace", "set_single_tune", "decode_ws", "decode_ws_async", "ws_workspace_bytes",
    "set_ws_tune",
    "ALPHABET_STD", "ALPHABET_URL", "MODE_STRICT", "MODE_NOPAD", "FLAG_URL", "FLAG_STRICT",
    "FLAG_NOPAD", "DIR_ENCODE", "DIR_DECODE", "Tune", "B64Error",
]


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_u8(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError(f"{name} must be a uint8 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _tune(t):
    if t is None:
        return None
    if isinstance(t, Tune):
        return ctypes.byref(t)
    tt = Tune(**{k: int(v) for k, v in dict(t).items() if k in ("block", "units_per_lane", "grid", "layout")})
    return ctypes.byref(tt)


def encoded_len(n, mode=0):
    return check(lib().b64_encoded_len_mode(int(n), int(mode)), "encoded_len")


def decoded_max(m, mode=0):
    return check(lib().b64_decoded_max_mode(int(m), int(mode)), "decoded_max")


def encode(src, alphabet=ALPHABET_STD, out=None, stream=None):
    """Encode a uint8 CUDA tensor; returns the characters (uint8 CUDA tensor).

    ``alphabet`` may carry ``MODE_NOPAD``. Asynchronous on ``stream``."""
    src = _dev_u8(src, "src")
    n = src.numel()
    m = encoded_len(n, alphabet & ~0xff)
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.uint8, device=src.device)
    else:
        _dev_u8(out, "out")
        if out.numel() < m:
            raise ValueError("out is too small")
    r = lib().b64_encode_ex(_ptr(src), n, _ptr(out), int(alphabet), _stream(stream))
    check(r, "b64_encode_ex")
    return out[:m]


def decode(src, alphabet=ALPHABET_STD, out=None, stream=None):
    """Validating decode of a uint8 CUDA tensor of characters.

    Returns ``(bytes_tensor, -1)`` on success or ``(None, err_off)`` with the
    first offending index. Waits for ``stream`` to read the verdict."""
    src = _dev_u8(src, "src")
    n = src.numel()
    cap = decoded_max(n, alphabet & ~0xff)
    if out is None:
        out = torch.empty(max(cap, 1), dtype=torch.uint8, device=src.device)
    else:
        _dev_u8(out, "out")
        if out.numel() < cap:
            raise ValueError("out is too small")
    err = ctypes.c_int64(-1)
    r = lib().b64_decode_ex(_ptr(src), n, _ptr(out), ctypes.byref(err), int(alphabet), _stream(stream))
    check(r, "b64_decode_ex")
    if r < 0:
        return None, err.value
    return out[:r], -1


def decode_async(src, out, result, alphabet=ALPHABET_STD, stream=None):
    """Non-blocking decode: ``result`` is an int64 CUDA tensor of 2 slots that
    receives (length | -1, -1 | first offending index)."""
    src = _dev_u8(src, "src")
    _dev_u8(out, "out")
    if out.numel() < decoded_max(src.numel(), alphabet & ~0xff):
        raise ValueError("out is too small")
    _result_slots(result)
    rp = result.data_ptr()
    r = lib().b64_decode_async(_ptr(src), src.numel(), _ptr(out), int(alphabet),
                               ctypes.c_void_p(rp), ctypes.c_void_p(rp + 8), _stream(stream))
    check(r, "b64_decode_async")


def ws_workspace_bytes(n):
    return check(lib().b64_decode_ws_workspace_bytes(int(n)), "b64_decode_ws_workspace_bytes")


def decode_ws(src, alphabet=ALPHABET_STD, out=None, stream=None):
    """Whitespace-tolerant decode (space, LF, CR removed first). Returns
    ``(bytes_tensor, -1)`` or ``(None, err_off)`` with the first offending
    index in the coordinates of ``src``. Waits for ``stream``."""
    src = _dev_u8(src, "src")
    n = src.numel()
    cap = decoded_max(n)
    if out is None:
        out = torch.empty(max(cap, 1), dtype=torch.uint8, device=src.device)
    else:
        _dev_u8(out, "out")
        if out.numel() < cap:
            raise ValueError("out is too small")
    err = ctypes.c_int64(-1)
    r = lib().b64_decode_ws(_ptr(src), n, _ptr(out), ctypes.byref(err), int(alphabet), _stream(stream))
    check(r, "b64_decode_ws")
    if r < 0:
        return None, err.value
    return out[:r], -1


def decode_ws_async(src, out, result, workspace, alphabet=ALPHABET_STD, stream=None):
    """Non-blocking whitespace-tolerant decode; ``result`` (int64 CUDA, 2
    slots) receives (length | -1, -1 | first offending original index).
    ``workspace`` is a uint8 CUDA tensor of at least ws_workspace_bytes(n)."""
    src = _dev_u8(src, "src")
    _dev_u8(out, "out")
    _dev_u8(workspace, "workspace")
    n = src.numel()
    if out.numel() < decoded_max(n):
        raise ValueError("out is too small")
    if workspace.numel() < ws_workspace_bytes(n):
        raise ValueError("workspace is too small")
    _result_slots(result)
    rp = result.data_ptr()
    r = lib().b64_decode_ws_async(_ptr(src), n, _ptr(out), int(alphabet), ctypes.c_void_p(rp),
                                  ctypes.c_void_p(rp + 8), _ptr(workspace), workspace.numel(),
                                  _stream(stream))
    check(r, "b64_decode_ws_async")


def set_ws_tune(block=0, chunks_per_lane=0):
    """Launch shape of the whitespace-tolerant decode (see b64_set_ws_tune):
    block threads and 16-byte input chunks per lane per tile; zero keeps the
    current value."""
    t = Tune(block=block, units_per_lane=chunks_per_lane, grid=0, layout=0)
    check(lib().b64_set_ws_tune(ctypes.byref(t)), "b64_set_ws_tune")


def set_single_tune(direction, block=0, units_per_lane=0, blocks_per_cu=0, char_map=0):
    """Launch shape and character map of the single-buffer kernels (see
    b64_set_single_tune); char_map 0 LDS tables, 1 register maps, 2 (encode)
    pair table."""
    t = Tune(block=block, units_per_lane=units_per_lane, grid=blocks_per_cu, layout=char_map)
    check(lib().b64_set_single_tune(int(direction), ctypes.byref(t)), "b64_set_single_tune")


# ----------------------------------------------------------------- batches --

def _i64_dev(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int64 CUDA tensor")
    return t


def _i64_slots(t, n, name):
    """A caller's int64 device array that the kernels index up to n - 1."""
    _i64_dev(t, name)
    if t.numel() < n:
        raise ValueError(f"{name} needs at least {n} entries")
    return t


def _flags_dev(flags, N):
    """Per-message flags: None (standard alphabet, padded) or one uint8 per
    message on the device."""
    if flags is None:
        return None
    if not isinstance(flags, torch.Tensor) or flags.dtype != torch.uint8 or not flags.is_cuda \
            or not flags.is_contiguous():
        raise TypeError("flags must be a contiguous uint8 CUDA tensor")
    if flags.numel() < N:
        raise ValueError(f"flags needs one byte per message ({N})")
    return flags


def _result_slots(result):
    if not isinstance(result, torch.Tensor) or result.dtype != torch.int64 or result.numel() < 2 \
            or not result.is_cuda or not result.is_contiguous():
        raise TypeError("result must be a contiguous int64 CUDA tensor with 2 slots")


def workspace_bytes(N):
    return check(lib().b64_batch_workspace_bytes(int(N)), "workspace_bytes")


def batch_out_offsets(direction, in_off, flags=None, stream=None):
    """Device exclusive scan of the per-message output sizes (N+1 int64)."""
    in_off = _i64_dev(in_off, "in_off")
    N = in_off.numel() - 1
    flags = _flags_dev(flags, N)
    out_off = torch.empty(N + 1, dtype=torch.int64, device=in_off.device)
    r = lib().b64_batch_out_offsets(int(direction), _ptr(in_off), N, _ptr(out_off),
                                    _ptr(flags), _stream(stream))
    check(r, "b64_batch_out_offsets")
    return out_off


class Workspace:
    """A reusable device workspace for the batched calls (grows on demand,
    outside the launch path). Calls that pass no workspace share one default
    per device, which suits calls on one stream; calls that may run at the
    same time on different streams need a Workspace each."""

    def __init__(self, device=None):
        self.buf = None
        self.device = device

    def get(self, N, device):
        need = workspace_bytes(N)
        if self.buf is None or self.buf.numel() < need or self.buf.device != device:
            self.buf = torch.empty(need, dtype=torch.uint8, device=device)
        return self.buf


_default_ws = {}


def _ws(ws, N, device):
    if ws is None:
        ws = _default_ws.setdefault(device, Workspace(device))
    return ws.get(N, device)


def encode_batch(src, in_off, out_off=None, flags=None, dst=None, out_len=None, tune=None,
                 workspace=None, stream=None, total_out=None, validate=True):
    """Encode N packed messages in one persistent launch.

    Returns ``(dst, out_off, out_len)``. ``total_out`` (host int, the last
    entry of out_off) avoids a device read when ``dst`` is allocated here."""
    src = _dev_u8(src, "src")
    in_off = _i64_dev(in_off, "in_off")
    N = in_off.numel() - 1
    dev = src.device
    flags = _flags_dev(flags, N)
    if out_off is None:
        out_off = batch_out_offsets(DIR_ENCODE, in_off, flags, stream)
    else:
        _i64_slots(out_off, N, "out_off")
    if dst is None:
        tot = int(out_off[-1].item()) if total_out is None else int(total_out)
        dst = torch.empty(max(tot, 1), dtype=torch.uint8, device=dev)
    if out_len is None:
        out_len = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    _i64_slots(out_len, N, "out_len")
    _dev_u8(dst, "dst")
    if validate:
        _validate_packed(src, in_off, out_off, dst, DIR_ENCODE, flags)
    ws = _ws(workspace, N, dev)
    r = lib().b64_encode_batch(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off), _ptr(flags),
                               _ptr(out_len), _ptr(ws), ws.numel(), _tune(tune), _stream(stream))
    check(r, "b64_encode_batch")
    return dst, out_off, out_len[:N]


def decode_batch(src, in_off, out_off=None, flags=None, dst=None, out_len=None, err_off=None,
                 tune=None, workspace=None, stream=None, total_out=None, validate=True):
    """Decode N packed messages in one persistent launch.

    Returns ``(dst, out_off, out_len, err_off)``; per message out_len is the
    length or -1 and err_off is -1 or the offset inside the message."""
    src = _dev_u8(src, "src")
    in_off = _i64_dev(in_off, "in_off")
    N = in_off.numel() - 1
    dev = src.device
    flags = _flags_dev(flags, N)
    if out_off is None:
        out_off = batch_out_offsets(DIR_DECODE, in_off, flags, stream)
    else:
        _i64_slots(out_off, N, "out_off")
    if dst is None:
        tot = int(out_off[-1].item()) if total_out is None else int(total_out)
        dst = torch.empty(max(tot, 1), dtype=torch.uint8, device=dev)
    if out_len is None:
        out_len = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    if err_off is None:
        err_off = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    _i64_slots(out_len, N, "out_len")
    _i64_slots(err_off, N, "err_off")
    _dev_u8(dst, "dst")
    if validate:
        _validate_packed(src, in_off, out_off, dst, DIR_DECODE, flags)
    ws = _ws(workspace, N, dev)
    r = lib().b64_decode_batch(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off), _ptr(flags),
                               _ptr(out_len), _ptr(err_off), _ptr(ws), ws.numel(), _tune(tune),
                               _stream(stream))
    check(r, "b64_decode_batch")
    return dst, out_off, out_len[:N], err_off[:N]


def decode_batch_noalloc(src, in_off, out_off, dst, out_len, err_off, flags=None, tune=None, stream=None,
                         validate=True):
    """``b64_decode_batch_noalloc``: decode_batch with every buffer supplied by
    the caller and the planning workspace taken from the library's static
    device array (no allocation; at most NOALLOC_MAX_MESSAGES messages; calls
    overlapping on one device race). Returns ``(out_len, err_off)`` views."""
    src = _dev_u8(src, "src")
    in_off = _i64_dev(in_off, "in_off")
    N = in_off.numel() - 1
    flags = _flags_dev(flags, N)
    _i64_slots(out_off, N, "out_off")
    _i64_slots(out_len, N, "out_len")
    _i64_slots(err_off, N, "err_off")
    _dev_u8(dst, "dst")
    if validate:
        _validate_packed(src, in_off, out_off, dst, DIR_DECODE, flags)
    r = lib().b64_decode_batch_noalloc(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off), _ptr(flags),
                                       _ptr(out_len), _ptr(err_off), _tune(tune), _stream(stream))
    check(r, "b64_decode_batch_noalloc")
    return out_len[:N], err_off[:N]


def _validate_packed(src, in_off, out_off, dst, direction, flags=None):
    """Host-side check of a packed batch before launch (reads the offsets
    back): offsets non-decreasing and inside src, output slots inside dst."""
    import numpy as np
    o = in_off.cpu().numpy()
    if o.size < 1 or np.any(np.diff(o) < 0) or o[0] < 0 or o[-1] > src.numel():
        raise ValueError("in_off must be non-decreasing and inside src")
    lens = np.diff(o)
    oo = out_off.cpu().numpy()
    _check_slots(oo[: lens.size], lens, direction, flags, dst)


def batch_slots(direction, lens, flags=None):
    """Host form of the batch slot layout (``b64_batch_slots``): for message
    lengths ``lens`` and per-message flags (host arrays), returns (need,
    out_off): the bytes the kernels may write per message and the N+1 slot
    offsets that ``b64_batch_out_offsets`` computes on the device."""
    import numpy as np
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    N = lens.size
    if fl is not None and fl.size < N:
        raise ValueError(f"flags needs one byte per message ({N})")
    need = np.empty(max(N, 1), np.int64)
    oo = np.empty(N + 1, np.int64)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    check(lib().b64_batch_slots(int(direction), P(lens) if N else None, None if fl is None else P(fl), N,
                                P(need), P(oo)), "b64_batch_slots")
    return need[:N], oo


def _host_flags(flags):
    return None if flags is None else flags.cpu().numpy()


def _check_slots(oo, lens, direction, flags, dst):
    import numpy as np
    need, _ = batch_slots(direction, lens, _host_flags(flags))
    if lens.size and (np.any(oo < 0) or np.any(oo + need > dst.numel())):
        raise ValueError("output slots fall outside dst")


def _validate_gather(src, in_begin, in_len, out_off, dst, direction, flags=None):
    import numpy as np
    b = in_begin.cpu().numpy()
    n = in_len.cpu().numpy()
    if b.size != n.size or np.any(n < 0) or np.any(b < 0) or np.any(b + n > src.numel()):
        raise ValueError("every message span must lie inside src")
    _check_slots(out_off.cpu().numpy(), n, direction, flags, dst)


def _gather_out_off(in_len, direction, flags, device):
    """Output slots laid out as b64_batch_out_offsets lays them out, computed
    by the library on the host from the lengths."""
    _, oo = batch_slots(direction, in_len.cpu().numpy(), _host_flags(flags))
    return torch.from_numpy(oo[:-1].copy()).to(device), int(oo[-1])


def encode_batch_gather(src, in_begin, in_len, out_off=None, flags=None, dst=None, out_len=None,
                        tune=None, workspace=None, stream=None, validate=True):
    """Encode messages src[in_begin[i], in_begin[i] + in_len[i]) (device int64
    arrays) in one persistent launch. Returns (dst, out_off, out_len)."""
    src = _dev_u8(src, "src")
    in_begin = _i64_dev(in_begin, "in_begin")
    in_len = _i64_dev(in_len, "in_len")
    N = in_begin.numel()
    if in_len.numel() != N:
        raise ValueError("in_begin and in_len differ in length")
    dev = src.device
    flags = _flags_dev(flags, N)
    if out_off is None:
        out_off, total = _gather_out_off(in_len, DIR_ENCODE, flags, dev)
        if dst is None:
            dst = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
    else:
        _i64_slots(out_off, N, "out_off")
    if out_len is None:
        out_len = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    _i64_slots(out_len, N, "out_len")
    _dev_u8(dst, "dst")
    if validate:
        _validate_gather(src, in_begin, in_len, out_off, dst, DIR_ENCODE, flags)
    ws = _ws(workspace, N, dev)
    r = lib().b64_encode_batch_gather(_ptr(src), _ptr(in_begin), _ptr(in_len), N, _ptr(dst), _ptr(out_off),
                                      _ptr(flags), _ptr(out_len), _ptr(ws), ws.numel(), _tune(tune),
                                      _stream(stream))
    check(r, "b64_encode_batch_gather")
    return dst, out_off, out_len[:N]


def decode_batch_gather(src, in_begin, in_len, out_off=None, flags=None, dst=None, out_len=None,
                        err_off=None, tune=None, workspace=None, stream=None, validate=True):
    """Decode messages src[in_begin[i], in_begin[i] + in_len[i]) in one
    persistent launch. Returns (dst, out_off, out_len, err_off)."""
    src = _dev_u8(src, "src")
    in_begin = _i64_dev(in_begin, "in_begin")
    in_len = _i64_dev(in_len, "in_len")
    N = in_begin.numel()
    if in_len.numel() != N:
        raise ValueError("in_begin and in_len differ in length")
    dev = src.device
    flags = _flags_dev(flags, N)
    if out_off is None:
        out_off, total = _gather_out_off(in_len, DIR_DECODE, flags, dev)
        if dst is None:
            dst = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
    else:
        _i64_slots(out_off, N, "out_off")
    if out_len is None:
        out_len = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    if err_off is None:
        err_off = torch.empty(max(N, 1), dtype=torch.int64, device=dev)
    _i64_slots(out_len, N, "out_len")
    _i64_slots(err_off, N, "err_off")
    _dev_u8(dst, "dst")
    if validate:
        _validate_gather(src, in_begin, in_len, out_off, dst, DIR_DECODE, flags)
    ws = _ws(workspace, N, dev)
    r = lib().b64_decode_batch_gather(_ptr(src), _ptr(in_begin), _ptr(in_len), N, _ptr(dst), _ptr(out_off),
                                      _ptr(flags), _ptr(out_len), _ptr(err_off), _ptr(ws), ws.numel(),
                                      _tune(tune), _stream(stream))
    check(r, "b64_decode_batch_gather")
    return dst, out_off, out_len[:N], err_off[:N]


def _host_i64(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _host_u8(a):
    import numpy as np
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def encode_each(src, h_in_off, h_out_off, dst, out_len, h_flags=None, stream=None):
    """Baseline: one single-buffer launch per message (host offsets)."""
    a, pa = _host_i64(h_in_off)
    b, pb = _host_i64(h_out_off)
    f, pf = _host_u8(h_flags)
    r = lib().b64_encode_each(_ptr(src), pa, a.size - 1, _ptr(dst), pb, pf, _ptr(out_len), _stream(stream))
    check(r, "b64_encode_each")


def decode_each(src, h_in_off, h_out_off, dst, out_len, err_off, h_flags=None, stream=None):
    """Baseline: one single-buffer launch per message (host offsets)."""
    a, pa = _host_i64(h_in_off)
    b, pb = _host_i64(h_out_off)
    f, pf = _host_u8(h_flags)
    r = lib().b64_decode_each(_ptr(src), pa, a.size - 1, _ptr(dst), pb, pf, _ptr(out_len),
                              _ptr(err_off), _stream(stream))
    check(r, "b64_decode_each")
