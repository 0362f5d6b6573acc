"""The serving workload at full size and rate (Poisson arrivals at 200,000
requests/s for 10 s, seed 4; sizes log-uniform in [64 B, 1 MiB]; 1% of the
decodes corrupted), every request checked against the oracle: characters,
decoded bytes, lengths and error offsets.

All outputs of 10 s of traffic do not fit in the 8 GiB pool at once, so the
trace is served in consecutive windows whose outputs fit; each window runs in
real time at the trace's own arrival times and keeps its outputs in the pool
(capture), which are then compared with the oracle's outputs written at the
same pool offsets."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import serve, workloads
from paper_1704_00605_amd.pool import DevicePool

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def _windows(blocks, limit):
    """Consecutive index ranges whose summed pool blocks stay within limit."""
    out, a, acc = [], 0, 0
    for i, b in enumerate(blocks):
        if acc + b > limit and i > a:
            out.append((a, i))
            a, acc = i, 0
        acc += b
    out.append((a, blocks.size))
    return out


@pytest.mark.timeout(900)
def test_serving_full_trace_every_request_against_oracle():
    th = _host_threads()
    banks = serve.Banks(corpus_bytes=1 << 30, seed=40)
    tr = workloads.serving_trace(rate=200_000.0, seconds=10.0, seed=4)
    req = serve.build_requests(tr, banks, seed=41)
    n = req["op"].size
    assert n > 1_900_000
    # the oracle's inputs: the corpus, and the decode bank rebuilt from the
    # oracle's own text of the corpus plus the generator's injected bytes;
    # the device banks must hold exactly these bytes
    corpus = banks.corpus.cpu().numpy()
    T = banks.text_len
    text = oracle.encode(corpus, threads=th)
    assert text.size == T
    dech = np.concatenate([text, text])
    del text
    dech[T + banks.inject_pos] = banks.inject_val
    assert torch.equal(banks.dec, torch.from_numpy(dech).to(DEV))

    op, ib, il = req["op"], req["in_begin"], req["in_len"]
    cap = np.where(op == 0, 4 * ((il + 2) // 3), 3 * (il // 4) + 2).astype(np.int64)
    pool_bytes = 8 << 30
    blocks = np.maximum(256, 2 ** np.ceil(np.log2(np.maximum(cap, 1)))).astype(np.int64)
    wins = _windows(blocks, pool_bytes - (pool_bytes >> 4))
    pool = DevicePool(pool_bytes)
    checked = invalid = 0
    for k, (a, b) in enumerate(wins):
        sub = {key: v[a:b] for key, v in req.items()}
        sub["t_arrival"] = sub["t_arrival"] - sub["t_arrival"][0]
        pool.buf.zero_()
        res, st = serve.run(sub, banks, pool, max_batch=4096, tick_us=25, streams=4, capture=True,
                            max_seconds=120)
        assert res["rc"] == 0 and st["completed"] == b - a, (k, a, b, res["rc"])
        oo = res["out_off"]
        used = int((oo + cap[a:b]).max())
        exp = np.zeros(used, np.uint8)
        e = sub["op"] == 0
        d = ~e
        wl_e = oracle.encode_gather(corpus, sub["in_begin"][e], sub["in_len"][e], oo[e], exp, threads=th)
        wl_d, we_d = oracle.decode_gather(dech, sub["in_begin"][d], sub["in_len"][d], oo[d], exp, threads=th)
        assert np.array_equal(res["out_len"][e], wl_e) and (res["err_off"][e] == -1).all(), k
        assert np.array_equal(res["out_len"][d], wl_d), k
        assert np.array_equal(res["err_off"][d], we_d), k
        # the output of an invalid decode is unspecified: clear it on the device
        bad = np.nonzero(d)[0][we_d >= 0]
        for r in bad:
            pool.buf[oo[r]:oo[r] + cap[a + r]].zero_()
        assert torch.equal(pool.buf[:used], torch.from_numpy(exp).to(DEV)), k
        for off in oo:
            pool.free(int(off))
        assert pool.free_bytes() == pool_bytes
        checked += b - a
        invalid += bad.size
        print(f"window {k + 1}/{len(wins)}: requests {a}..{b} equal the oracle "
              f"({bad.size} invalid decodes)", flush=True)
    assert checked == n
    assert invalid == int(tr["corrupt"].sum())
