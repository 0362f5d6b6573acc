"""Autotuner for the persistent batched kernels.

Searches the work layout (grid-stride tiles, one contiguous range of 64-unit
groups per wave, or staged tiles whose input goes through LDS) and the launch
shape (threads per workgroup, units per lane, workgroups in the grid; for the
staged layout also one workgroup per tile, counted on the host from the
message lengths) of ``b64_encode_batch`` /
``b64_decode_batch`` on the actual batch, timing each candidate with HIP events, and caches the winner in
a JSON file keyed by architecture, compute-unit count, direction and a coarse signature
of the batch (message count, total bytes and the log2 histogram of message
lengths). The tile of one workgroup step is ``block * units_per_lane``
units of 12 bytes (encode) or 16 characters (decode); how many messages share
a workgroup step follows from it and the size histogram and is reported as
``msgs_per_wg_step``.
"""
import json
import os
import time

import numpy as np
import torch

from . import codec

# per layout: (blocks, units per lane, workgroups per compute unit)
SPACE = {
    0: ((256, 512, 1024), (1, 2, 4), (8, 16, 32)),
    # finer per-wave shares balance the uneven per-message costs better
    1: ((64, 128, 256), (1, 2, 4), (16, 32, 64, 128)),
}
DEFAULT = {"block": 512, "units_per_lane": 2, "grid_per_cu": 32, "layout": 0}


def cache_path():
    p = os.environ.get("B64HIP_TUNE_CACHE")
    if p:
        return p
    home = os.path.expanduser("~")
    d = os.path.join(home, ".cache", "b64hip")
    try:
        os.makedirs(d, exist_ok=True)
        return os.path.join(d, "tune.json")
    except OSError:
        return os.path.join("/tmp", "b64hip_tune.json")


def signature(in_off_host):
    lens = np.diff(np.asarray(in_off_host, dtype=np.int64))
    N = lens.size
    hist = np.bincount(np.minimum(np.log2(np.maximum(lens, 1)).astype(np.int64), 40), minlength=41)
    frac = np.round(hist / max(N, 1), 2)
    return {"N_log2": int(np.log2(max(N, 1))), "bytes_log2": int(np.log2(max(int(lens.sum()), 1))),
            "hist": [float(x) for x in frac]}


def _device_key():
    # architecture and compute-unit count (the marketing name can differ
    # between processes, e.g. under a profiler)
    props = torch.cuda.get_device_properties(0)
    return f"{getattr(props, 'gcnArchName', 'unknown')}|cus{props.multi_processor_count}"


def _key(direction, sig):
    return f"{_device_key()}|dir{direction}|{json.dumps(sig, sort_keys=True)}"


def load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c):
    """Atomic replace through a per-process temporary file, so that processes
    saving at once never interleave their writes (the last one wins)."""
    p = cache_path()
    tmp = f"{p}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1)
    os.replace(tmp, p)


# staged layout (2): 256-thread workgroups, units per lane, and either one
# workgroup per tile (counted from the batch's lengths on the host) or a
# grid of 32 workgroups per CU walking the tiles
STAGED_UNITS = (1, 2, 4, 8)


def staged_tiles(direction, in_off_host, units_per_lane):
    """Tiles of the staged layout for a packed batch (known on the host)."""
    unit = 12 if direction == codec.DIR_ENCODE else 16
    lens = np.diff(np.asarray(in_off_host, dtype=np.int64))
    U = int((-(-lens // unit)).sum())
    T = 256 * units_per_lane
    return max(1, -(-U // T))


def candidates(cus, direction=None, in_off_host=None):
    out = [dict(block=b, units_per_lane=u, grid=g * cus, layout=lay)
           for lay, (blocks, units, grids) in SPACE.items() for b in blocks for u in units for g in grids]
    for u in STAGED_UNITS:
        grids = {32 * cus}
        if in_off_host is not None and direction is not None:
            grids.add(min(staged_tiles(direction, in_off_host, u), 1 << 20))
        out += [dict(block=256, units_per_lane=u, grid=g, layout=2) for g in sorted(grids)]
    return out


def time_call(fn, reps):
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))


def tune(direction, src, in_off, flags=None, in_off_host=None, reps=3, cands=None, use_cache=True,
         verbose=False):
    """Best launch shape for this batch; returns (tune dict, report)."""
    if in_off_host is None:
        in_off_host = in_off.cpu().numpy()
    sig = signature(in_off_host)
    key = _key(direction, sig)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]["tune"], cache[key]
    N = in_off.numel() - 1
    cus = codec.lib().b64_device_cus()
    out_off = codec.batch_out_offsets(direction, in_off, flags)
    total = int(out_off[-1].item())
    dst = torch.empty(max(total, 1), dtype=torch.uint8, device=src.device)
    out_len = torch.empty(max(N, 1), dtype=torch.int64, device=src.device)
    err = torch.empty(max(N, 1), dtype=torch.int64, device=src.device)
    ws = codec.Workspace()
    results = []
    t0 = time.perf_counter()
    for c in cands or candidates(cus, direction, in_off_host):
        if direction == codec.DIR_ENCODE:
            fn = lambda: codec.encode_batch(src, in_off, out_off, flags, dst, out_len, tune=c, workspace=ws,
                                            validate=False)
        else:
            fn = lambda: codec.decode_batch(src, in_off, out_off, flags, dst, out_len, err, tune=c, workspace=ws,
                                            validate=False)
        ms = time_call(fn, reps)
        results.append((ms, c))
        if verbose:
            print(f"  {c} {ms:.4f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    units = in_off_host[-1] - in_off_host[0]
    unit = 12 if direction == codec.DIR_ENCODE else 16
    tile_units = best["block"] * best["units_per_lane"]
    msg_units = np.maximum(-(-np.diff(np.asarray(in_off_host)) // unit), 1)
    entry = {
        "tune": best, "ms": round(best_ms, 4), "worst_ms": round(results[-1][0], 4),
        "default_ms": None, "candidates": len(results), "tuning_s": round(time.perf_counter() - t0, 2),
        "msgs_per_wg_step": round(float(tile_units / msg_units.mean()), 2),
        "bytes": int(units), "signature": sig,
    }
    for ms, c in results:
        if (c["block"], c["units_per_lane"], c["grid"], c["layout"]) == (
                DEFAULT["block"], DEFAULT["units_per_lane"], DEFAULT["grid_per_cu"] * cus, DEFAULT["layout"]):
            entry["default_ms"] = round(ms, 4)
    if use_cache:
        cache[key] = entry
        save_cache(cache)
    return best, entry


# --------------------------------------------------------- single buffer --
# Candidates of the single-buffer kernels: character map (0 LDS byte tables,
# 1 register maps on v_perm_b32, 2 LDS pair table for encoding) x launch shape
# (block, units per lane, workgroups per CU with -1 = one per tile).
SINGLE_SHAPES = ((512, 2, -1), (256, 4, -1), (1024, 2, -1), (256, 4, 8), (512, 2, 16), (1024, 2, 4))
SINGLE_MAPS = {codec.DIR_ENCODE: (0, 1, 2), codec.DIR_DECODE: (0, 1)}


def tune_single(direction, size, reps=5, use_cache=True, apply=True, seed=8):
    """Best (block, units_per_lane, blocks_per_cu, char_map) of the
    single-buffer kernel for inputs of `size` bytes (encode) or characters
    (decode), timed on seeded random data with HIP events; cached per device
    and power-of-two size class. Applies the winner unless apply=False."""
    key = f"single|{_device_key()}|dir{direction}|log2size{int(np.log2(max(size, 1)))}"
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tune"]
    else:
        dev = torch.device("cuda:0")
        rng = np.random.default_rng(seed)
        n = size if direction == codec.DIR_ENCODE else size // 4 * 3
        x = torch.from_numpy(rng.integers(0, 256, max(n, 1), dtype=np.uint8)).to(dev)
        text = codec.encode(x)
        out = torch.empty(codec.decoded_max(text.numel()), dtype=torch.uint8, device=dev)
        res = torch.zeros(2, dtype=torch.int64, device=dev)
        results = []
        for cm in SINGLE_MAPS[direction]:
            for b, u, g in SINGLE_SHAPES:
                codec.set_single_tune(direction, b, u, g, cm)
                if direction == codec.DIR_ENCODE:
                    fn = lambda: codec.encode(x, out=text)
                else:
                    fn = lambda: codec.decode_async(text, out, res)
                results.append((time_call(fn, reps), {"block": b, "units_per_lane": u, "blocks_per_cu": g,
                                                       "char_map": cm}))
        results.sort(key=lambda r: r[0])
        best = results[0][1]
        if use_cache:
            cache[key] = {"tune": best, "ms": round(results[0][0], 5), "worst_ms": round(results[-1][0], 5),
                          "candidates": len(results)}
            save_cache(cache)
    if apply:
        codec.set_single_tune(direction, best["block"], best["units_per_lane"], best["blocks_per_cu"],
                              best["char_map"])
    else:
        codec.set_single_tune(direction, 512 if direction == codec.DIR_ENCODE else 256, 2, -1, 0)
    return best
