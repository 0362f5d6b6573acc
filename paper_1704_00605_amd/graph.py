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
        self.handle = ctypes.c_void_p()
        args = self._args(src, in_off, out_off, dst, out_len, err_off, flags, tune)
        check(lib().b64_graph_create_batch(direction, *args, ctypes.byref(self.handle)),
              "b64_graph_create_batch")

    def _args(self, src, in_off, out_off, dst, out_len, err_off, flags, tune):
        N = in_off.numel() - 1
        if self.direction == DIR_DECODE and err_off is None:
            raise ValueError("decode graphs need err_off")
        ws = codec.Workspace().get(N, src.device)
        # keep every captured buffer alive as long as the graph
        self._bufs = (src, in_off, out_off, dst, out_len, err_off, flags)
        self._ws = ws
        self._tune = codec.Tune(**dict(tune)) if tune is not None and not isinstance(tune, codec.Tune) else tune
        p = codec._ptr
        return (p(src), p(in_off), N, p(dst), p(out_off), p(flags), p(out_len), p(err_off), p(ws), ws.numel(),
                ctypes.byref(self._tune) if self._tune is not None else None)

    def update(self, src, in_off, out_off, dst, out_len, err_off=None, flags=None, tune=None):
        args = self._args(src, in_off, out_off, dst, out_len, err_off, flags, tune)
        check(lib().b64_graph_update_batch(self.handle, *args), "b64_graph_update_batch")

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
