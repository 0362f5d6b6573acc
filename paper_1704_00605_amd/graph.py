"""HIP graphs of batched codec calls (``b64_graph_*`` in ``include/b64.h``).

A graph holds the planning, codec and verdict kernels of one batched call;
replaying it costs one graph launch instead of three or four kernel launches.
"""
import ctypes

import torch

from . import codec
from ._lib import DIR_DECODE, DIR_ENCODE, check, lib


class BatchGraph:
    """Captured ``encode_batch`` / ``decode_batch`` over fixed buffers."""

    def __init__(self, direction, src, in_off, out_off, dst, out_len, err_off=None, flags=None,
                 tune=None):
        if direction not in (DIR_ENCODE, DIR_DECODE):
            raise ValueError("bad direction")
        self.direction = direction
        self._bufs = None
        self._ws = None
        self._tune = None
        self.handle = ctypes.c_void_p()
        args, keep = self._args(src, in_off, out_off, dst, out_len, err_off, flags, tune)
        check(lib().b64_graph_create_batch(direction, *args, ctypes.byref(self.handle)),
              "b64_graph_create_batch")
        self._bufs, self._ws, self._tune = keep

    def _args(self, src, in_off, out_off, dst, out_len, err_off, flags, tune):
        """C arguments of a capture, and what the graph must keep alive (held
        only once the capture or update succeeded)."""
        codec._dev_u8(src, "src")
        codec._dev_u8(dst, "dst")
        codec._i64_dev(in_off, "in_off")
        N = in_off.numel() - 1
        codec._i64_slots(out_off, N, "out_off")
        codec._i64_slots(out_len, N, "out_len")
        if self.direction == DIR_DECODE:
            if err_off is None:
                raise ValueError("decode graphs need err_off")
            codec._i64_slots(err_off, N, "err_off")
        flags = codec._flags_dev(flags, N)
        ws = codec.Workspace().get(N, src.device)
        t = codec.Tune(**dict(tune)) if tune is not None and not isinstance(tune, codec.Tune) else tune
        p = codec._ptr
        args = (p(src), p(in_off), N, p(dst), p(out_off), p(flags), p(out_len), p(err_off), p(ws), ws.numel(),
                ctypes.byref(t) if t is not None else None)
        return args, ((src, in_off, out_off, dst, out_len, err_off, flags), ws, t)

    def update(self, src, in_off, out_off, dst, out_len, err_off=None, flags=None, tune=None):
        args, keep = self._args(src, in_off, out_off, dst, out_len, err_off, flags, tune)
        check(lib().b64_graph_update_batch(self.handle, *args), "b64_graph_update_batch")
        self._bufs, self._ws, self._tune = keep

    def launch(self, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        check(lib().b64_graph_launch(self.handle, ctypes.c_void_p(stream.cuda_stream)), "b64_graph_launch")

    def close(self):
        if self.handle:
            lib().b64_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
