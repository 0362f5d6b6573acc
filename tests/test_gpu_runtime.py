"""GPU tests of the runtime around the kernels: gather batches, HIP-graph
replay and update, and the continuous-batching serving loop (results in the
mix equal results alone; admission by free pool memory)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import _lib, codec, serve, workloads
from paper_1704_00605_amd.graph import BatchGraph
from paper_1704_00605_amd.pool import DevicePool

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
E, D = codec.DIR_ENCODE, codec.DIR_DECODE


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a if a.flags.writeable else a.copy()).to(DEV)


def host(t):
    return t.cpu().numpy()


def gather_call(direction, bank, begin, lens, flags=None):
    """Gather batch through the C ABI via the checked Python wrappers (they
    validate every message span against the bank before launching)."""
    fl = dev(flags) if flags is not None else None
    if direction == E:
        dst, out_off, out_len = codec.encode_batch_gather(bank, dev(begin), dev(lens), flags=fl)
        err = None
    else:
        dst, out_off, out_len, err = codec.decode_batch_gather(bank, dev(begin), dev(lens), flags=fl)
    torch.cuda.synchronize()
    return host(dst), host(out_off), host(out_len), None if err is None else host(err)


def test_gather_batches_match_oracle():
    rng = np.random.default_rng(0)
    bank_h = rng.integers(0, 256, 3 << 20, dtype=np.uint8)
    bank = dev(bank_h)
    N = 3000
    lens = np.where(rng.uniform(size=N) < 0.05, rng.integers(10_000, 300_000, N), rng.integers(0, 500, N)).astype(np.int64)
    begin = (rng.uniform(size=N) * (bank_h.size - lens)).astype(np.int64)  # overlapping, any alignment
    flags = rng.integers(0, 2, N).astype(np.uint8)
    dst, out_off, out_len, _ = gather_call(E, bank, begin, lens, flags)
    texts = []
    for i in range(N):
        w = oracle.encode(bank_h[begin[i]:begin[i] + lens[i]], int(flags[i]))
        assert out_len[i] == w.size and np.array_equal(dst[out_off[i]:out_off[i] + w.size], w), i
        texts.append(w)
    # decode gather over a text bank holding the encodings (some corrupted)
    tl = np.array([t.size for t in texts], np.int64)
    tb = np.zeros(tl.size, np.int64)
    tb[1:] = np.cumsum(tl)[:-1]
    text = np.concatenate(texts)
    for i in rng.choice(N, 60, replace=False):
        if tl[i]:
            text[tb[i] + rng.integers(0, tl[i])] = ord("#")
    order = rng.permutation(N)  # messages in any order
    dst, out_off, out_len, err = gather_call(D, dev(text), tb[order], tl[order], flags[order])
    for k, i in enumerate(order):
        w = oracle.decode(text[tb[i]:tb[i] + tl[i]], int(flags[i]))
        assert (out_len[k], err[k]) == w[:2], (i, k)
        if w[0] > 0:
            assert np.array_equal(dst[out_off[k]:out_off[k] + w[0]], w[2])


@pytest.mark.parametrize("direction", [E, D])
def test_graph_replays_match_eager(direction):
    w = workloads.uneven(count=20_000, seed=5)
    data, off = w["payload"], w["in_off"]
    if direction == D:
        data, off, _ = oracle.encode_batch(data, off)
        workloads.corrupt_text(data, off, w["corrupt_ids"][:200] % 20_000, w["corrupt_u"][:200],
                               w["corrupt_rank"][:200])
    src, in_off = dev(data), dev(off)
    out_off = codec.batch_out_offsets(direction, in_off)
    total = int(out_off[-1].item())
    N = off.size - 1
    dst = torch.zeros(total, dtype=torch.uint8, device=DEV)
    out_len = torch.zeros(N, dtype=torch.int64, device=DEV)
    err = torch.zeros(N, dtype=torch.int64, device=DEV)
    if direction == E:
        ed, _, el = codec.encode_batch(src, in_off, out_off)
        eager = (ed.clone(), el.clone(), None)
    else:
        ed, _, el, ee = codec.decode_batch(src, in_off, out_off)
        eager = (ed.clone(), el.clone(), ee.clone())
    g = BatchGraph(direction, src, in_off, out_off, dst, out_len, err if direction == D else None)
    for rep in range(4):
        dst.zero_()
        out_len.fill_(-7)
        err.fill_(-7)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(out_len, eager[1]), rep
        if direction == E:
            assert torch.equal(dst, eager[0]), rep
        else:
            assert torch.equal(err, eager[2]), rep
            valid = host(eager[2]) < 0
            oo, ol = host(out_off), host(eager[1])
            m = np.zeros(total, bool)
            for i in np.nonzero(valid)[0][:2000]:
                m[oo[i]:oo[i] + ol[i]] = True
            assert np.array_equal(host(dst)[m], host(eager[0])[m]), rep
        _ = torch.randn(1000, device=DEV).sum().item()  # unrelated eager work between replays
    # update to a different batch (smaller N) and replay
    off2 = off[:5001] - off[0]
    src2 = dev(data[: off2[-1]])
    in2 = dev(off2)
    oo2 = codec.batch_out_offsets(direction, in2)
    dst2 = torch.zeros(int(oo2[-1].item()) + 1, dtype=torch.uint8, device=DEV)
    ol2 = torch.zeros(5000, dtype=torch.int64, device=DEV)
    er2 = torch.zeros(5000, dtype=torch.int64, device=DEV)
    g.update(src2, in2, oo2, dst2, ol2, er2 if direction == D else None)
    for rep in range(2):
        g.launch()
        torch.cuda.synchronize()
        if direction == E:
            want, _, wl = oracle.encode_batch(data[: off2[-1]], off2)
            assert np.array_equal(host(dst2)[: want.size], want) and np.array_equal(host(ol2), wl)
        else:
            _, _, wl, we = oracle.decode_batch(data[: off2[-1]], off2)
            assert np.array_equal(host(ol2), wl) and np.array_equal(host(er2), we)
    g.close()


@pytest.mark.parametrize("direction", [E, D])
def test_graph_update_across_planning_topologies(direction):
    """A captured batch re-pointed from 3,000 messages to 1,200,000 (whose
    planning takes one more pass, so the update re-instantiates the graph)
    and back; every replay against the oracle."""
    rng = np.random.default_rng(31 + direction)

    def batch(N):
        lens = rng.integers(0, 30, N)
        off = np.zeros(N + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, int(off[-1]), dtype=np.uint8)
        if direction == D:
            data, off, _ = oracle.encode_batch(data, off)
            data = data.copy()
            hit = rng.choice(N, N // 100, replace=False)
            hit = hit[np.diff(off)[hit] > 0]
            data[off[hit]] = ord("#")
        src, in_off = dev(data), dev(off)
        out_off = codec.batch_out_offsets(direction, in_off)
        dst = torch.zeros(int(out_off[-1].item()) + 1, dtype=torch.uint8, device=DEV)
        ol = torch.full((N,), -7, dtype=torch.int64, device=DEV)
        er = torch.full((N,), -7, dtype=torch.int64, device=DEV)
        return data, off, (src, in_off, out_off, dst, ol, er if direction == D else None)

    def check(data, off, args):
        g.launch()
        torch.cuda.synchronize()
        if direction == E:
            want, _, wl = oracle.encode_batch(data, off)
            assert np.array_equal(host(args[4]), wl) and np.array_equal(host(args[3])[:want.size], want)
        else:
            _, _, wl, we = oracle.decode_batch(data, off)
            assert np.array_equal(host(args[4]), wl) and np.array_equal(host(args[5]), we)
            assert (we >= 0).sum() > 0

    small = batch(3000)
    g = BatchGraph(direction, *small[2])
    check(*small)
    big = batch(1_200_000)
    g.update(*big[2])
    for _ in range(2):
        check(*big)
    small2 = batch(2000)
    g.update(*small2[2])
    check(*small2)
    g.close()


def _small_trace(n_target, rate, hi, seed, corrupt=0.05):
    tr = workloads.serving_trace(rate=rate, seconds=n_target / rate, lo=64, hi=hi, seed=seed, corrupt_frac=corrupt)
    return tr


def _alone(banks, req, r, pool_like=None):
    op, b, n = int(req["op"][r]), int(req["in_begin"][r]), int(req["in_len"][r])
    if op == 0:
        out = codec.encode(banks.corpus[b:b + n]) if n else torch.empty(0, dtype=torch.uint8, device=DEV)
        return out, out.numel(), -1
    out, err = codec.decode(banks.dec[b:b + n])
    return out, (-1 if out is None else out.numel()), err


def test_serving_results_same_alone_and_in_mix():
    banks = serve.Banks(corpus_bytes=48 << 20, seed=7, corrupt_stride=1 << 16)
    tr = _small_trace(4000, 100_000.0, 256 << 10, seed=8, corrupt=0.05)
    req = serve.build_requests(tr, banks, seed=9)
    pool = DevicePool(2 << 30)
    res, st = serve.run(req, banks, pool, max_batch=256, tick_us=100, streams=3, capture=True)
    assert res["rc"] == 0 and st["completed"] == req["op"].size
    assert st["max_inflight_batches"] >= 1
    summ = serve.summarize(req, res, st)
    assert summ["invalid_requests"] > 0
    pb = host(pool.buf[: int((res["out_off"] + 4 * ((req["in_len"] + 2) // 3)).max())])
    rng = np.random.default_rng(1)
    check = np.unique(np.concatenate([rng.choice(req["op"].size, 400, replace=False),
                                      np.nonzero(res["err_off"] >= 0)[0]]))
    for r in check:
        out, n, err = _alone(banks, req, r)
        assert (res["out_len"][r], res["err_off"][r]) == (n, err), r
        if n > 0:
            assert np.array_equal(pb[res["out_off"][r]:res["out_off"][r] + n], host(out)), r
    # and the alone results agree with the oracle on a sample
    dech = None
    for r in check[:40]:
        op, b, n = int(req["op"][r]), int(req["in_begin"][r]), int(req["in_len"][r])
        if op == 1:
            if dech is None:
                dech = host(banks.dec)
            w = oracle.decode(dech[b:b + n])
            assert (res["out_len"][r], res["err_off"][r]) == w[:2]


def test_serving_admission_waits_for_free_memory():
    banks = serve.Banks(corpus_bytes=24 << 20, seed=10, corrupt_stride=1 << 16)
    tr = _small_trace(600, 200_000.0, 1 << 20, seed=11, corrupt=0.02)
    req = serve.build_requests(tr, banks, seed=12)
    pool = DevicePool(4 << 20)  # room for a few outputs only
    res, st = serve.run(req, banks, pool, max_batch=64, tick_us=50, streams=2, capture=False, time_scale=0.0)
    assert res["rc"] == 0
    assert st["completed"] == req["op"].size and st["pool_waits"] > 0
    assert st["peak_pool_bytes"] <= 4 << 20
    assert pool.free_bytes() == 4 << 20
    for r in np.random.default_rng(2).choice(req["op"].size, 60, replace=False):
        _, n, err = _alone(banks, req, r)
        assert (res["out_len"][r], res["err_off"][r]) == (n, err), r


def test_serving_rejects_request_larger_than_pool():
    banks = serve.Banks(corpus_bytes=6 << 20, seed=13)
    req = {"t_arrival": np.array([0.0, 0.0]), "op": np.array([0, 0], np.uint8),
           "in_begin": np.array([0, 0], np.int64), "in_len": np.array([100, 3 << 20], np.int64),
           "flags": np.zeros(2, np.uint8)}
    pool = DevicePool(1 << 20)
    res, st = serve.run(req, banks, pool, max_batch=8, tick_us=10, streams=1, time_scale=0.0, max_seconds=20)
    assert res["rc"] == _lib.POOL_FULL
    assert res["t_done"][0] >= 0 and res["t_done"][1] < 0
