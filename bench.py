#!/usr/bin/env python3
"""Benchmark of the gfx950 base64 codec (one GPU).

Default workload (one step): a 1 GiB buffer of uniform random bytes (seed 1)
is encoded to 1,431,655,768 characters, the text is decoded back, and a copy
of the text with one byte outside the alphabet at 99.9% of its length is
decoded (verdict: -1 at that offset). Inputs are resident in HBM before the
timed region; verdicts and the round trip are verified after it.

Prints ONE JSON line. ``value`` is the step's input throughput
(bytes + characters + characters per second, GB/s). ``roofline`` reports the
dominant kernel's algorithmic HBM bytes per launch (input + output) over its
average launch duration from HIP events on its stream, against the MI355X HBM
peak of 8 TB/s. ``cpu_baseline`` times the plain CPU oracle on a bounded
sample on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "encode/decode GB/s & %HBM peak; batched vs per-msg launch; p50/p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_single_1GiB.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_batched_ws.json")


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=1 << 30, help="payload bytes (default 1 GiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mib", type=int, default=1024)
    ap.add_argument("--quick", action="store_true",
                    help="only the timed 1 GiB step (skip the 1 MiB latency, batched and serving reports)")
    ap.add_argument("--only", default="",
                    help="comma list of extra reports to run: latency,uneven,heavy,maps,files,mime,serving")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-per-message", action="store_true",
                    help="skip the per-message-launch baseline of the batched reports (for kernel traces)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain int32 copy kernel (1 GiB in, 1 GiB out) three times; "
                         "its HBM counter readings scale the codec's counter readings")
    return ap.parse_args()


def calibrate_copy():
    import torch

    dev = torch.device("cuda:0")
    a = torch.zeros((1 << 30) // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4,
                      "launches": 3}), flush=True)


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(payload, text, sample_mib):
    """The oracle (plain scalar C) on a bounded sample: all host threads over
    the first sample_mib MiB, and one thread over the first 128 MiB. Same step
    shape as the GPU step (encode n, decode m twice); median of >= 5 reps."""
    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def measure(nb, th, min_reps, budget_s):
        x = payload[:nb]
        t = text[: (nb // 3) * 4]
        te, td = [], []
        t_start = time.perf_counter()
        while len(te) < min_reps or (time.perf_counter() - t_start < budget_s and len(te) < 20):
            t0 = time.perf_counter()
            e = oracle.encode(x, threads=th)
            t1 = time.perf_counter()
            n, err, _ = oracle.decode(t, threads=th)
            t2 = time.perf_counter()
            assert err == -1 and n == nb and np.array_equal(e, t)
            te.append(t1 - t0)
            td.append(t2 - t1)
        return nb, t.size, float(np.median(te)), float(np.median(td)), float(min(te)), float(min(td)), len(te)

    nb = min(payload.size, (sample_mib << 20) // 3 * 3)
    nb, nt, me, md, be, bd, reps = measure(nb, threads, 5, 8.0)
    n1 = min(payload.size, (128 << 20) // 3 * 3)
    n1, nt1, me1, md1, _, _, reps1 = measure(n1, 1, 5, 0.0)
    step_bytes = nb + 2 * nt
    return {
        "value": round(step_bytes / (me + 2 * md) / 1e9, 3),
        "unit": "GB/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"first {nb} bytes of the 1 GiB payload and their {nt} characters, encode + 2x decode "
                  f"(the GPU step's shape), median of {reps} reps on {threads} threads; one-thread figures "
                  f"over the first {n1} bytes, median of {reps1} reps; plain C -O2",
        "cpu_model": _cpu_model(),
        "encode_GBps": round(nb / me / 1e9, 3),
        "decode_GBps": round(nt / md / 1e9, 3),
        "encode_GBps_best": round(nb / be / 1e9, 3),
        "decode_GBps_best": round(nt / bd / 1e9, 3),
        "one_thread": {"value": round((n1 + 2 * nt1) / (me1 + 2 * md1) / 1e9, 3),
                       "encode_GBps": round(n1 / me1 / 1e9, 3), "decode_GBps": round(nt1 / md1 / 1e9, 3)},
    }


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "this codec build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1704_00605_amd import codec, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.size
    progress("generating the 1 GiB workload")
    w = workloads.single_at_fraction(n, seed=1, frac=0.999)
    payload = w["payload"]
    x = torch.from_numpy(payload).to(dev)
    m = codec.encoded_len(n)
    text = torch.empty(m, dtype=torch.uint8, device=dev)
    out = torch.empty(codec.decoded_max(m), dtype=torch.uint8, device=dev)
    out_bad = torch.empty_like(out)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    res_bad = torch.zeros(2, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    # corrupted copy of the text (prepared once, outside the timed region)
    codec.encode(x, out=text)
    bad = text.clone()
    pos = int(np.floor(0.999 * m))
    bad[pos] = workloads.corruption_byte(w["corrupt_rank"], 0, pos, m)
    torch.cuda.synchronize()

    def step(ev=None):
        if ev: ev[0].record(stream)
        codec.encode(x, out=text, stream=stream)
        if ev: ev[1].record(stream)
        codec.decode_async(text, out, res, stream=stream)
        if ev: ev[2].record(stream)
        codec.decode_async(bad, out_bad, res_bad, stream=stream)
        if ev: ev[3].record(stream)

    progress("timed steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # verification (after the timed region)
    r = res.cpu().tolist()
    rb = res_bad.cpu().tolist()
    ok = r == [n, -1] and rb == [-1, pos] and torch.equal(out[:n], x)
    if not ok:
        print(f"VERIFICATION FAILED: decode={r} corrupted={rb} expected pos {pos}", file=sys.stderr)
        sys.exit(1)

    enc_t = [e[0].elapsed_time(e[1]) for e in evs]
    dec_t = [e[1].elapsed_time(e[2]) for e in evs]
    decb_t = [e[2].elapsed_time(e[3]) for e in evs]
    enc_ms, dec_ms, decb_ms = (float(np.mean(v)) for v in (enc_t, dec_t, decb_t))
    step_ms = wall * 1e3 / args.steps
    algo_bytes = n + m  # same for both directions: read input, write output
    enc_bw = algo_bytes / (enc_ms * 1e-3) / 1e9
    dec_bw = algo_bytes / (dec_ms * 1e-3) / 1e9
    # dominant kernel: the one with the largest share of the step (decode runs twice)
    dominant = "decode" if 2 * dec_ms >= enc_ms else "encode"
    ach = dec_bw if dominant == "decode" else enc_bw
    traffic = stored_traffic(dominant, n)
    line = {
        "metric": METRIC,
        "value": round((n + 2 * m) / (step_ms * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "single-buffer codec: 1 GiB uniform random bytes (seed 1) encoded, decoded, "
                        "and a copy with an invalid byte at 99.9% decoded",
            "bytes": n, "chars": m, "invalid_at": pos, "alphabet": "standard, padded",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_{'dec' if dominant == 'decode' else 'enc'}_single",
            "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": algo_bytes,
        },
        "encode": {"ms": round(enc_ms, 4), "median_ms": round(float(np.median(enc_t)), 4),
                   "min_ms": round(min(enc_t), 4), "input_GBps": round(n / enc_ms / 1e6, 1),
                   "hbm_GBps": round(enc_bw, 1), "hbm_frac": round(enc_bw / HBM_PEAK_GBPS, 4)},
        "decode": {"ms": round(dec_ms, 4), "median_ms": round(float(np.median(dec_t)), 4),
                   "min_ms": round(min(dec_t), 4), "input_GBps": round(m / dec_ms / 1e6, 1),
                   "hbm_GBps": round(dec_bw, 1), "hbm_frac": round(dec_bw / HBM_PEAK_GBPS, 4)},
        "decode_invalid": {"ms": round(decb_ms, 4), "err_off": pos},
        "paper_context": "AVX2 on i7-6700 (Skylake, 3.4 GHz, 1 core): ~0.25 cycles/byte "
                         "(~13.6 GB/s) encode and decode; Chrome 2.7 / 1.8 cycles/byte",
    }
    text_h = text.cpu().numpy() if not args.no_cpu_baseline else None
    del x, out, out_bad, bad, text
    torch.cuda.empty_cache()
    if not args.quick:
        wanted = set(filter(None, args.only.split(","))) or {"latency", "uneven", "heavy", "maps", "files", "mime", "serving"}
        if "latency" in wanted:
            progress("1 MiB latency")
            line["latency_1MiB"] = report_latency_1mib()
        if "uneven" in wanted:
            progress("100,000 uneven messages, batched vs per-message")
            line["batched_uneven_100k"] = report_batched("uneven", not args.no_per_message)
            torch.cuda.empty_cache()
        if "heavy" in wanted:
            progress("8,192-message heavy mix, batched vs per-message (autotuned)")
            line["batched_heavy_mix_8k"] = report_batched("heavy", not args.no_per_message)
            torch.cuda.empty_cache()
        if "maps" in wanted:
            progress("character-map variants of the single-buffer kernels")
            line["char_maps"] = report_maps()
            torch.cuda.empty_cache()
        if "files" in wanted:
            progress("file-size workload (decode per file)")
            line["table7_files"] = report_files()
            torch.cuda.empty_cache()
        if "mime" in wanted:
            progress("whitespace-tolerant decode, MIME lines")
            line["ws_decode_mime"] = report_ws()
            torch.cuda.empty_cache()
        if "serving" in wanted:
            progress("serving, Poisson 200,000 requests/s")
            line["serving_poisson_200k"] = report_serving(args.serve_seconds)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(payload, text_h, args.cpu_sample_mib)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- reports --

def _events_ms(fn, reps, stream):
    """Median device time of one call of fn over reps back-to-back calls on
    stream (HIP events between consecutive calls). A spin kernel queued first
    keeps the device behind the host, so that the calls run back to back and
    an interval is device time, not the host's time to issue a call; the
    spin is lengthened until it is still running when the host has issued
    every call."""
    import torch
    fn()
    torch.cuda.synchronize()
    spin = 200_000 * reps
    for _ in range(4):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        with torch.cuda.stream(stream):
            torch.cuda._sleep(spin)
        ev[0].record(stream)
        for i in range(reps):
            fn()
            ev[i + 1].record(stream)
        behind = not ev[0].query()
        torch.cuda.synchronize()
        if behind:
            break
        spin *= 4
    return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))


def _wall_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def report_latency_1mib():
    """1 MiB single buffer (seed 0): launch/latency bound and cache resident."""
    import torch
    from paper_1704_00605_amd import codec, workloads

    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    w = workloads.single(1 << 20, seed=0)
    x = torch.from_numpy(w["payload"]).to(dev)
    n = x.numel()
    m = codec.encoded_len(n)
    t = torch.empty(m, dtype=torch.uint8, device=dev)
    o = torch.empty(codec.decoded_max(m), dtype=torch.uint8, device=dev)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    codec.encode(x, out=t)
    bad = t.clone()
    pos = min(int(np.floor(w["corrupt_u"] * m)), m - 1)
    bad[pos] = workloads.corruption_byte(w["corrupt_rank"], 0, pos, m)
    enc_ms = _events_ms(lambda: codec.encode(x, out=t), 50, s)
    dec_ms = _events_ms(lambda: codec.decode_async(t, o, res), 50, s)
    dec_sync_ms = _wall_ms(lambda: codec.decode(t, out=o), 50)
    verdict = codec.decode(bad, out=o)[1]
    assert verdict == pos and torch.equal(codec.decode(t, out=o)[0], x)
    return {
        "workload": "1 MiB uniform random bytes (seed 0), standard alphabet; cache resident, launch bound",
        "encode_us": round(enc_ms * 1e3, 2), "decode_async_us": round(dec_ms * 1e3, 2),
        "decode_sync_call_us": round(dec_sync_ms * 1e3, 2),
        "encode_input_GBps": round(n / enc_ms / 1e6, 1), "decode_input_GBps": round(m / dec_ms / 1e6, 1),
        "invalid_byte_at": pos, "note": "%HBM peak not meaningful at this size (L2/MALL resident)",
    }


def report_batched(which, per_message=True):
    """The 100,000 uneven messages ("uneven") or the 8,192-message heavy mix
    ("heavy"): one persistent launch per direction over the packed batch
    (plan + codec kernels, eager and as a HIP graph, default and autotuned
    launch shape) against one single-buffer launch per message."""
    import torch
    from paper_1704_00605_amd import autotune, codec, workloads
    from paper_1704_00605_amd.graph import BatchGraph

    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    if which == "uneven":
        w = workloads.uneven()
        name = "100,000 messages, lengths log-uniform in [1, 65536] (seed 2), standard alphabet, 1% corrupted"
    else:
        w = workloads.heavy_mix()
        name = ("8,192 messages: 819 uniform in [1 MiB, 16 MiB] + 7,373 uniform in [16 B, 4 KiB] (seed 3), "
                "per-message std/url flag, 0.5% corrupted")
    off_h = w["in_off"]
    N = off_h.size - 1
    flags_h = w["flags"]
    src = torch.from_numpy(w["payload"]).to(dev)
    del w["payload"]
    in_off = torch.from_numpy(off_h).to(dev)
    flags = torch.from_numpy(flags_h).to(dev)
    out = {"workload": name, "messages": N, "input_bytes": int(off_h[-1])}
    for direction, label in ((codec.DIR_ENCODE, "encode"), (codec.DIR_DECODE, "decode")):
        if direction == codec.DIR_DECODE:
            # decode input: the encoded batch with the seeded corruptions
            text_off = enc_off
            toff_h = text_off.cpu().numpy()
            text = enc_dst
            ids, u, rk = w["corrupt_ids"], w["corrupt_u"], w["corrupt_rank"]
            lens = np.diff(toff_h)[ids]
            pos = np.minimum(np.floor(u * lens).astype(np.int64), np.maximum(lens - 1, 0))
            vals = [workloads.corruption_byte(r, int(flags_h[i]), int(p), int(L)) for r, i, p, L in zip(rk, ids, pos, lens)]
            keep = lens > 0
            text[torch.from_numpy((toff_h[ids] + pos)[keep]).to(dev)] = torch.tensor(np.array(vals, np.uint8)[keep], device=dev)
            bsrc, boff, boff_h = text, text_off, toff_h
        else:
            bsrc, boff, boff_h = src, in_off, off_h
        out_off = codec.batch_out_offsets(direction, boff, flags)
        total = int(out_off[-1].item())
        dst = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
        out_len = torch.empty(N, dtype=torch.int64, device=dev)
        err = torch.empty(N, dtype=torch.int64, device=dev)
        ws = codec.Workspace()
        if direction == codec.DIR_ENCODE:
            run = lambda tn=None: codec.encode_batch(bsrc, boff, out_off, flags, dst, out_len, tune=tn,
                                                     workspace=ws, validate=False)
        else:
            run = lambda tn=None: codec.decode_batch(bsrc, boff, out_off, flags, dst, out_len, err, tune=tn,
                                                     workspace=ws, validate=False)
        run()
        torch.cuda.synchronize()
        base_ms = _events_ms(run, 10, s)
        best, entry = autotune.tune(direction, bsrc, boff, flags, in_off_host=boff_h, reps=3)
        tuned_ms = _events_ms(lambda: run(best), 10, s)
        tuned_wall = _wall_ms(lambda: run(best), 5)
        g = BatchGraph(direction, bsrc, boff, out_off, dst, out_len,
                       err if direction == codec.DIR_DECODE else None, flags, tune=best)
        graph_ms = _events_ms(g.launch, 10, s)
        graph_wall = _wall_ms(g.launch, 5)
        g.close()
        # verdicts of the batch (checked against the per-message launches below)
        b_len = out_len.cpu().numpy().copy()
        b_err = err.cpu().numpy().copy() if direction == codec.DIR_DECODE else None
        oo_h = out_off.cpu().numpy()
        each_wall, same = None, None
        if per_message:
            dst2 = torch.empty_like(dst)
            ol2 = torch.empty(N, dtype=torch.int64, device=dev)
            er2 = torch.empty(N, dtype=torch.int64, device=dev)
            if direction == codec.DIR_ENCODE:
                each = lambda: codec.encode_each(bsrc, boff_h, oo_h, dst2, ol2, h_flags=flags_h)
            else:
                each = lambda: codec.decode_each(bsrc, boff_h, oo_h, dst2, ol2, er2, h_flags=flags_h)
            each_wall = _wall_ms(each, 2)
            same = bool(np.array_equal(ol2.cpu().numpy(), b_len))
            if direction == codec.DIR_DECODE:
                same = same and bool(np.array_equal(er2.cpu().numpy(), b_err))
            else:
                same = same and bool(torch.equal(dst2, dst))
            del dst2
        algo = int(boff_h[-1] - boff_h[0]) + total
        out[label] = {
            "batched_ms": round(tuned_ms, 4), "batched_default_shape_ms": round(base_ms, 4),
            "batched_wall_ms": round(tuned_wall, 4), "graph_replay_ms": round(graph_ms, 4),
            "graph_wall_ms": round(graph_wall, 4),
            "per_message_wall_ms": None if each_wall is None else round(each_wall, 4),
            "speedup_vs_per_message": None if each_wall is None else round(each_wall / tuned_wall, 2),
            "input_GBps": round((boff_h[-1] - boff_h[0]) / tuned_ms / 1e6, 1),
            "hbm_GBps_algorithmic": round(algo / tuned_ms / 1e6, 1),
            "hbm_frac": round(algo / tuned_ms / 1e6 / HBM_PEAK_GBPS, 4),
            "tune": best, "msgs_per_wg_step": entry.get("msgs_per_wg_step"),
            "same_verdicts_as_per_message": same,
            "hbm_traffic": stored_batch_traffic(f"{which}.{label}", batch_kernel_name(direction, best),
                                                best.get("block"), best.get("grid")),
        }
        if direction == codec.DIR_ENCODE:
            enc_dst, enc_off = dst, out_off
            out["encode"]["invalid_messages"] = 0
        else:
            out["decode"]["invalid_messages"] = int((b_err >= 0).sum())
    return out


def report_maps():
    """Character-map variants of the single-buffer kernels (0 LDS byte
    tables, 1 register maps on v_perm_b32, 2 LDS pair table for encoding),
    each at its best launch shape, at three sizes: 1 GiB (HBM-bound), 64 MiB
    and 4 MiB (cache-resident when repeated), HIP events, median of reps."""
    import torch
    from paper_1704_00605_amd import codec

    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    rng = np.random.default_rng(7)
    shapes = [(512, 2, -1), (256, 2, -1), (1024, 2, 4)]
    out = {}
    for size in (1 << 30, 64 << 20, 4 << 20):
        x = torch.from_numpy(rng.integers(0, 256, size, dtype=np.uint8)).to(dev)
        m = codec.encoded_len(size)
        t = torch.empty(m, dtype=torch.uint8, device=dev)
        o = torch.empty(codec.decoded_max(m), dtype=torch.uint8, device=dev)
        res = torch.zeros(2, dtype=torch.int64, device=dev)
        codec.encode(x, out=t)
        want = t.clone()
        reps = 10 if size >= (1 << 30) else 50
        row = {}
        for direction, maps in ((0, (0, 1, 2)), (1, (0, 1))):
            for cm in maps:
                best = None
                for b, u, g in shapes:
                    codec.set_single_tune(direction, b, u, g, cm)
                    if direction == 0:
                        ms = _events_ms(lambda: codec.encode(x, out=t, stream=s), reps, s)
                        ok = torch.equal(t, want)
                    else:
                        ms = _events_ms(lambda: codec.decode_async(t, o, res, stream=s), reps, s)
                        ok = res.tolist() == [size, -1] and torch.equal(o[:size], x)
                    if best is None or ms < best[0]:
                        best = (ms, (b, u, g), ok)
                key = ("encode" if direction == 0 else "decode") + f"_map{cm}"
                row[key] = {"us": round(best[0] * 1e3, 2), "hbm_GBps": round((size + m) / best[0] / 1e6, 1),
                            "shape": list(best[1]), "verified": bool(best[2])}
            codec.set_single_tune(direction, 512 if direction == 0 else 256, 2, -1, 0)
        out[f"{size >> 20}MiB"] = row
        del x, t, o, want
    from paper_1704_00605_amd import autotune
    out["autotuner_pick"] = {f"{d}_{sz >> 20}MiB": autotune.tune_single(0 if d == "encode" else 1, sz, apply=False)
                             for d in ("encode", "decode") for sz in (4 << 20, 64 << 20)}
    out["maps"] = {"0": "LDS byte tables", "1": "register maps on v_perm_b32 (range offsets / nibble bitsets)",
                   "2": "LDS pair table, 4096 entries (encode)"}
    return out


def report_files():
    """Decode of synthetic texts at the six sizes of the paper's decoding
    table: per-call latency (HIP events, median of 200), input GB/s, GPU
    cycles per input byte (whole chip at 2.4 GHz, the analogue of the table's
    single-core cycles per byte), a device-to-device copy of the same text,
    and all six decoded as one batch."""
    import torch
    from paper_1704_00605_amd import codec, workloads

    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    files = workloads.table7_files()
    rows, texts = [], []
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    for name, size, payload in files:
        x = torch.from_numpy(payload).to(dev)
        t = codec.encode(x)
        texts.append(t)
        L = t.numel()
        out = torch.empty(codec.decoded_max(L), dtype=torch.uint8, device=dev)
        cp = torch.empty_like(t)
        dec_ms = _events_ms(lambda: codec.decode_async(t, out, res, stream=s), 200, s)
        ok = res.tolist() == [x.numel(), -1] and torch.equal(out[: x.numel()], x)
        enc_ms = _events_ms(lambda: codec.encode(x, out=t, stream=s), 200, s)
        copy_ms = _events_ms(lambda: cp.copy_(t), 200, s)
        rows.append({"file": name, "stated_bytes": size, "text_bytes": L,
                     "decode_us": round(dec_ms * 1e3, 2), "decode_input_GBps": round(L / dec_ms / 1e6, 2),
                     "decode_gpu_cycles_per_byte": round(dec_ms * 1e-3 * 2.4e9 / L, 3),
                     "encode_us": round(enc_ms * 1e3, 2), "copy_us": round(copy_ms * 1e3, 2),
                     "verified": bool(ok)})
    # the six texts as one batch
    lens = np.array([t.numel() for t in texts], np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    packed = torch.cat(texts)
    in_off = torch.from_numpy(off).to(dev)
    out_off = codec.batch_out_offsets(codec.DIR_DECODE, in_off)
    dst = torch.empty(int(out_off[-1].item()), dtype=torch.uint8, device=dev)
    ol = torch.empty(lens.size, dtype=torch.int64, device=dev)
    er = torch.empty(lens.size, dtype=torch.int64, device=dev)
    ws = codec.Workspace()
    tune = {"layout": 1}
    batch_ms = _events_ms(lambda: codec.decode_batch(packed, in_off, out_off, None, dst, ol, er, tune=tune,
                                                     workspace=ws, validate=False), 200, s)
    ok = (er.cpu().numpy() == -1).all() and np.array_equal(ol.cpu().numpy(), [f[2].size for f in files])
    return {"workload": "uniform random payloads (seed 6) whose texts have the sizes of the paper's decoding "
                        "table (2,357 and 1,355 rounded down to multiples of 4)",
            "files": rows, "batch_of_six_decode_us": round(batch_ms * 1e3, 2), "batch_verified": bool(ok),
            "note": "launch-latency bound: every text fits in cache; compare decode_us with copy_us"}


def report_ws():
    """Whitespace-tolerant decode (Appendix B) of a 1 GiB payload's base64 text
    cut into 76-character CRLF lines (MIME), against the plain decode of the
    same text without line breaks."""
    import torch
    from paper_1704_00605_amd import codec, workloads

    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream()
    w = workloads.mime_1gib()
    x = torch.from_numpy(w["payload"]).to(dev)
    del w["payload"]
    n = x.numel()
    m = codec.encoded_len(n)
    text = codec.encode(x)
    lines = -(-m // 76)
    wrapped = torch.empty(m + 2 * lines, dtype=torch.uint8, device=dev)
    full = m // 76
    v = wrapped[: full * 78].view(full, 78)
    v[:, :76] = text[: full * 76].view(full, 76)
    v[:, 76] = 13
    v[:, 77] = 10
    rest = m - full * 76
    if rest:
        wrapped[full * 78: full * 78 + rest] = text[full * 76:]
        wrapped[full * 78 + rest:] = torch.tensor([13, 10], dtype=torch.uint8, device=dev)
    nw = wrapped.numel()
    out = torch.empty(3 * (nw // 4), dtype=torch.uint8, device=dev)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = torch.empty(codec.ws_workspace_bytes(nw), dtype=torch.uint8, device=dev)
    ws_ms = _events_ms(lambda: codec.decode_ws_async(wrapped, out, res, ws, stream=s), 20, s)
    ok = res.tolist() == [n, -1] and torch.equal(out[:n], x)
    plain_ms = _events_ms(lambda: codec.decode_async(text, out, res, stream=s), 20, s)
    algo = nw + n
    return {
        "workload": "1 GiB uniform random bytes (seed 5) -> base64 text in 76-character CRLF lines "
                    f"({nw} bytes, {nw - m} of them line breaks)",
        "ms": round(ws_ms, 4), "input_GBps": round(nw / ws_ms / 1e6, 1),
        "hbm_GBps_algorithmic": round(algo / ws_ms / 1e6, 1),
        "hbm_frac": round(algo / ws_ms / 1e6 / HBM_PEAK_GBPS, 4),
        "plain_decode_same_text_ms": round(plain_ms, 4),
        "verified": bool(ok),
        "hbm_traffic": {"count_pass": stored_batch_traffic("mime.count"),
                        "decode_pass": stored_batch_traffic("mime.decode")},
    }


def serving_mismatches(req, res, banks):
    """Requests whose result differs from its closed form: an encode writes
    4 * ceil(n / 3) characters; a decode of a clean slice (symbols only,
    length a multiple of 4) gives 3 / 4 of its length and no error; a decode
    of a slice of the corrupted bank stops at the first injected byte inside
    it (the generator never injects '='). Counted over completed requests."""
    op, il, ib = req["op"], req["in_len"], req["in_begin"]
    enc = op == 0
    T = banks.text_len
    want_len = np.where(enc, 4 * ((il + 2) // 3), 3 * (il // 4)).astype(np.int64)
    want_err = np.full(il.size, -1, np.int64)
    bad = np.nonzero(~enc & (ib >= T))[0]
    if bad.size:
        inj = np.asarray(banks.inject_pos, np.int64)
        s0 = ib[bad] - T
        k = np.searchsorted(inj, s0)
        pos = inj[np.minimum(k, inj.size - 1)]
        inside = (k < inj.size) & (pos >= s0) & (pos < s0 + il[bad])
        want_err[bad] = np.where(inside, pos - s0, -1)
        want_len[bad] = np.where(inside, -1, want_len[bad])
    done = res["t_done"] >= 0
    mism = ((res["out_len"] != want_len) | (res["err_off"] != want_err)) & done
    return int(mism.sum()), int(bad.size)


SERVER = dict(max_batch=4096, tick_us=25, streams=4)


def report_serving(seconds, sweep=True):
    """Serving: Poisson arrivals at 200,000/s, 50/50 encode/decode, sizes
    log-uniform in [64 B, 1 MiB], 1% of decodes corrupted; device pool capped
    at 8 GiB with admission by free memory. Every request's verdict and
    length are checked in closed form. Then a sweep of the arrival rate (same
    generator, 1 s of traffic each) for the highest rate whose p99 latency
    stays under 1 ms."""
    import torch
    from paper_1704_00605_amd import serve, workloads
    from paper_1704_00605_amd.pool import DevicePool

    banks = serve.Banks(corpus_bytes=1 << 30, seed=40)
    tr = workloads.serving_trace(rate=200_000.0, seconds=seconds, seed=4)
    req = serve.build_requests(tr, banks, seed=41)
    pool = DevicePool(8 << 30)
    # a 25 us batching tick: the lowest p99 of a sweep over 250..0 us at this
    # rate (throughput unchanged)
    res, st = serve.run(req, banks, pool, **SERVER, max_seconds=seconds * 6 + 30)
    summ = serve.summarize(req, res, st)
    mism, ncorrupt = serving_mismatches(req, res, banks)
    summ.update({"workload": f"Poisson 200,000 req/s for {seconds:g} s (seed 4), 50/50 encode/decode, "
                             "sizes log-uniform [64 B, 1 MiB], 1% of decodes corrupted",
                 "server": {**SERVER, "layout": "per-wave ranges"},
                 "offered_GBps": round(float(req['in_len'].sum()) / seconds / 1e9, 3),
                 "pool_GiB": 8, "rc": res["rc"],
                 "verified_requests": int((res["t_done"] >= 0).sum()), "verdict_mismatches": mism,
                 "corrupted_requests": ncorrupt})
    if sweep:
        rows = []
        best = None
        for rate in (200_000, 400_000, 800_000, 1_600_000, 3_200_000, 6_400_000, 12_800_000, 25_600_000):
            progress(f"serving sweep: {rate} requests/s")
            trr = workloads.serving_trace(rate=float(rate), seconds=1.0, seed=4)
            rq = serve.build_requests(trr, banks, seed=41)
            rr, sr = serve.run(rq, banks, pool, **SERVER, max_seconds=60)
            sm = serve.summarize(rq, rr, sr)
            mm, _ = serving_mismatches(rq, rr, banks)
            row = {"rate": rate, "requests": sm["requests"], "throughput_GBps": sm["throughput_GBps"],
                   "requests_per_s": sm["requests_per_s"], "p50_ms": sm["p50_ms"], "p99_ms": sm["p99_ms"],
                   "mean_batch": sm["mean_batch"], "pool_waits": sm["pool_waits"],
                   "peak_pool_MiB": sm["peak_pool_MiB"], "verdict_mismatches": mm, "rc": rr["rc"]}
            rows.append(row)
            if rr["rc"] == 0 and sm["p99_ms"] < 1.0:
                best = row
        summ["rate_sweep"] = {"seconds_each": 1.0, "rows": rows,
                              "highest_rate_p99_under_1ms": None if best is None else best["rate"],
                              "throughput_GBps_at_that_rate": None if best is None else best["throughput_GBps"]}
    del pool, banks
    torch.cuda.empty_cache()
    return summ


def stored_traffic(direction, n):
    """HBM bytes per launch of the single-buffer kernel of `direction`, from
    the committed counter summary, or None when that summary was taken on
    another size or on other kernel sources."""
    try:
        tf = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    entry = tf.get(direction)
    if not entry or tf.get("size") != n or tf.get("kernel_hash") != kernel_hash():
        return None
    return entry.get("bytes_per_launch")


def sources_hash(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        p = os.path.join(ROOT, "paper_1704_00605_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def batch_kernel_name(direction, tune):
    """Name of the batched codec kernel a launch shape runs (layout 2:
    k_batch_s<dir, units>; 1: k_*_batch_w<units>; 0: k_*_batch_t<units>)."""
    upl = tune.get("units_per_lane") or 2
    layout = tune.get("layout", 0)
    if layout == 2:
        return f"k_batch_s<{direction}, {upl}>"
    d = "enc" if direction == 0 else "dec"
    return f"k_{d}_batch_{'w' if layout == 1 else 't'}<{upl}>"


def stored_batch_traffic(key, kernel=None, block=None, grid=None):
    """HBM bytes per launch and their ratio to the payload for one batched or
    whitespace configuration (key such as "uneven.encode" or "mime.decode"),
    from the committed counter summary; None when the summary was taken on
    other kernel sources or another kernel or launch shape."""
    try:
        tf = json.load(open(BATCH_TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = tf.get("entries", {}).get(key)
    if not e:
        return None
    files = ["b64_modes.hpp", "b64_device.hpp", "b64_ws.hip" if key.startswith("mime") else "b64_batch.hip"]
    want = tf.get("ws_kernel_hash" if key.startswith("mime") else "batch_kernel_hash")
    if want != sources_hash(files):
        return None
    if kernel is not None and e.get("kernel") != kernel:
        return None
    if block is not None and grid is not None and kernel and "batch_s" not in kernel and \
            (e.get("block") != block or e.get("grid_threads") != block * grid):
        return None
    return {"bytes_per_launch": e["bytes_per_launch"], "algorithmic_bytes": e["algorithmic_bytes"],
            "ratio": e["ratio_to_algorithmic"], "kernel": e["kernel"],
            "from": "profiles/hbm_traffic_batched_ws.json"}


def kernel_hash():
    """Hash of the sources of the single-buffer kernels (the dominant kernels of
    the step), to tie stored counter readings to the code they were taken on."""
    import hashlib

    h = hashlib.sha256()
    for f in ("b64_modes.hpp", "b64_device.hpp", "b64_single.hip"):
        p = os.path.join(ROOT, "paper_1704_00605_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
