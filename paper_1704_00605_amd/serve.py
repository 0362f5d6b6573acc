"""Continuous-batching serving of encode/decode requests (``b64_server_run``).

The request loop itself is native (``csrc/b64_runtime.cpp``): arrivals are
admitted in order when the device pool can hold their output, admitted
requests of one direction are launched together on one of several streams,
completions are polled per batch and release pool memory. This module builds
the device-resident request banks, turns a seeded arrival trace into request
descriptors, runs the loop and summarises latency and throughput.

Banks: a random byte corpus for encode requests; for decode requests its
base64 text (a valid unpadded encoding, so any slice starting at a multiple
of 4 characters is a valid encoding) and a corrupted copy of that text with
one character outside the alphabet every ``corrupt_stride`` characters.
"""
import ctypes

import numpy as np
import torch

from . import codec, workloads
from ._lib import ServerCfg, ServerStats, check, lib
from .pool import DevicePool


class Banks:
    def __init__(self, corpus_bytes=1 << 30, seed=40, device="cuda:0", corrupt_stride=1 << 18):
        corpus_bytes -= corpus_bytes % 3
        rng = np.random.default_rng(seed)
        self.device = device
        self.corpus = torch.from_numpy(workloads.random_bytes(rng, corpus_bytes)).to(device)
        T = corpus_bytes // 3 * 4
        self.text_len = T
        self.dec = torch.empty(2 * T, dtype=torch.uint8, device=device)
        codec.encode(self.corpus, out=self.dec[:T])
        self.dec[T:].copy_(self.dec[:T])
        # one injected character per stride, at a seeded position inside it
        k = T // corrupt_stride
        pos = np.arange(k, dtype=np.int64) * corrupt_stride + rng.integers(0, corrupt_stride, k)
        ranks = rng.integers(0, 192, k)
        # never '=': an injected '=' at the end of a request's slice could be valid padding
        vals = np.array([workloads.corruption_byte(r, 0, T - 1, T) for r in ranks], np.uint8)
        self.inject_pos = pos
        self.inject_val = vals
        self.dec[T + torch.from_numpy(pos).to(device)] = torch.from_numpy(vals).to(device)
        torch.cuda.synchronize()


def build_requests(trace, banks, seed=41):
    """Request descriptors (host arrays) for a trace from workloads.serving_trace.

    Encode request of size s: bytes corpus[b, b + s) at a uniform byte offset.
    Decode request of payload size s: 4 * ceil(s / 3) characters of the text
    bank starting at a uniform multiple of 4; corrupted decodes take a slice of
    the corrupted bank placed so that an injected character sits at a uniform
    relative position inside it."""
    rng = np.random.default_rng(seed)
    n = trace["t_arrival"].size
    op = trace["op"].astype(np.uint8)
    size = trace["size"].astype(np.int64)
    C = banks.corpus.numel()
    T = banks.text_len
    text_len, _ = codec.batch_slots(codec.DIR_ENCODE, size)
    in_len = np.where(op == 0, size, text_len).astype(np.int64)
    in_begin = np.zeros(n, dtype=np.int64)
    enc = op == 0
    in_begin[enc] = (rng.uniform(size=int(enc.sum())) * (C - size[enc] + 1)).astype(np.int64)
    dec = ~enc
    L = in_len[dec]
    in_begin[dec] = 4 * (rng.uniform(size=int(dec.sum())) * ((T - L) // 4 + 1)).astype(np.int64)
    bad = np.nonzero(trace["corrupt"] & dec)[0]
    if bad.size:
        pick = banks.inject_pos[rng.integers(0, banks.inject_pos.size, bad.size)]
        Lb = in_len[bad]
        rel = np.floor(trace["corrupt_u"][bad] * Lb).astype(np.int64)
        # slices start at multiples of 4: round down, unless that pushes the
        # injected character past the end of the slice
        start = (pick - rel) // 4 * 4
        start = np.where(pick - start >= Lb, start + 4, start)
        start = np.clip(start, 0, (T - Lb) // 4 * 4)
        in_begin[bad] = T + start
    return {"t_arrival": trace["t_arrival"].astype(np.float64), "op": op, "in_begin": in_begin,
            "in_len": in_len, "flags": np.zeros(n, dtype=np.uint8)}


def run(requests, banks, pool, max_batch=2048, tick_us=200, streams=4, capture=False,
        time_scale=1.0, max_seconds=120.0, tune=None, idle_sleep_us=0):
    """Runs the native serving loop. Returns (per-request results, stats)."""
    n = requests["t_arrival"].size
    cfg = ServerCfg(max_batch=max_batch, tick_us=tick_us, streams=streams, capture=int(capture),
                    idle_sleep_us=idle_sleep_us, block=0, units_per_lane=0, grid=0, layout=1,
                    time_scale=time_scale, max_seconds=max_seconds)
    if tune:
        cfg.block = tune.get("block", 0)
        cfg.units_per_lane = tune.get("units_per_lane", 0)
        cfg.grid = tune.get("grid", 0)
        cfg.layout = tune.get("layout", 1)
    t_arr = np.ascontiguousarray(requests["t_arrival"], dtype=np.float64)
    op = np.ascontiguousarray(requests["op"], dtype=np.uint8)
    ib = np.ascontiguousarray(requests["in_begin"], dtype=np.int64)
    il = np.ascontiguousarray(requests["in_len"], dtype=np.int64)
    fl = np.ascontiguousarray(requests["flags"], dtype=np.uint8)
    if not all(a.ndim == 1 and a.size == n for a in (t_arr, op, ib, il, fl)):
        raise ValueError("every per-request array needs one entry per request")
    t_done = np.empty(n, np.float64)
    out_off = np.empty(n, np.int64)
    out_len = np.empty(n, np.int64)
    err = np.empty(n, np.int64)
    st = ServerStats()
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    torch.cuda.synchronize()
    if pool.buf.numel() < pool.capacity:
        raise ValueError("pool buffer smaller than the pool capacity")
    rc = lib().b64_server_run(ctypes.byref(cfg), n, P(t_arr), P(op), P(ib), P(il), P(fl),
                              ctypes.c_void_p(banks.corpus.data_ptr()), banks.corpus.numel(),
                              ctypes.c_void_p(banks.dec.data_ptr()), banks.dec.numel(),
                              pool.handle, ctypes.c_void_p(pool.base_ptr()), P(t_done), P(out_off),
                              P(out_len), P(err), ctypes.byref(st))
    check(rc, "b64_server_run")
    res = {"t_done": t_done, "out_off": out_off, "out_len": out_len, "err_off": err, "rc": rc}
    return res, st.as_dict()


def summarize(requests, res, stats, time_scale=1.0):
    lat = res["t_done"] - requests["t_arrival"] * time_scale
    done = res["t_done"] >= 0
    lat = lat[done]
    bytes_in = int(requests["in_len"][done].sum())
    span = float(res["t_done"][done].max() - (requests["t_arrival"][done].min() * time_scale))
    return {
        "requests": int(done.sum()),
        "throughput_GBps": round(bytes_in / span / 1e9, 3),
        "requests_per_s": round(done.sum() / span, 1),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "max_ms": round(float(lat.max()) * 1e3, 4),
        "batches": stats["batches"],
        "mean_batch": round(stats["launched_requests"] / max(stats["batches"], 1), 1),
        "pool_waits": stats["pool_waits"],
        "peak_pool_MiB": round(stats["peak_pool_bytes"] / 2**20, 1),
        "max_inflight_batches": stats["max_inflight_batches"],
        "invalid_requests": int((res["err_off"][done] >= 0).sum()),
    }


__all__ = ["Banks", "DevicePool", "build_requests", "run", "summarize"]
