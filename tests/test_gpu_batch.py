"""GPU parity of the batched codec (persistent kernels over a packed offsets
table) and of the per-message baseline, against the oracle, per message:
output bytes, out_len and error offset relative to the message start."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import codec, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
E, D = codec.DIR_ENCODE, codec.DIR_DECODE


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a if a.flags.writeable else a.copy()).to(DEV)


def host(t):
    return t.cpu().numpy()


def packed(lens, seed, base=0):
    rng = np.random.default_rng(seed)
    lens = np.asarray(lens, dtype=np.int64)
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    off += base
    data = rng.integers(0, 256, int(off[-1]) + 7, dtype=np.uint8)
    return data, off


def check_encode(data, off, flags=None, tune=None):
    want, want_off, want_len = oracle.encode_batch(data, off - off[0] if off[0] else off,
                                                   flags) if off[0] == 0 else (None, None, None)
    if off[0] != 0:
        # messages start at in_off[0] > 0: the oracle sees the same bytes
        want, want_off, want_len = oracle.encode_batch(data[off[0]:], off - off[0], flags)
    fl = None if flags is None else dev(flags)
    dst, out_off, out_len = codec.encode_batch(dev(data), dev(off), flags=fl, tune=tune)
    assert np.array_equal(host(out_off), want_off)
    assert np.array_equal(host(out_len), want_len)
    assert np.array_equal(host(dst)[: want.size], want)
    return dst, out_off


def dec_slots(toff, flags=None):
    """Decode slot layout: capacity rounded up to a multiple of 4."""
    lens = np.diff(toff)
    fl = np.zeros(lens.size, np.uint8) if flags is None else flags
    cap = 3 * (lens // 4) + np.where(fl & 4, np.maximum(lens % 4 - 1, 0), 0)
    slot = (cap + 3) // 4 * 4
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(slot, out=off[1:])
    return off


def segments(buf, starts, lens):
    """Concatenation of buf[starts[i] : starts[i] + lens[i]] over i."""
    lens = np.maximum(lens, 0)
    if lens.sum() == 0:
        return np.zeros(0, buf.dtype)
    idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(lens.sum())
    return buf[idx]


def check_decode(text, toff, flags=None, tune=None):
    want, want_off, want_len, want_err = oracle.decode_batch(text, toff, flags)
    fl = None if flags is None else dev(flags)
    dst, out_off, out_len, err = codec.decode_batch(dev(text), dev(toff), flags=fl, tune=tune)
    assert np.array_equal(host(out_off), dec_slots(toff, flags))
    gl, ge = host(out_len), host(err)
    bad = np.nonzero((gl != want_len) | (ge != want_err))[0]
    assert bad.size == 0, f"{bad.size} messages differ, first {bad[:5]}: got {gl[bad[:5]]},{ge[bad[:5]]} want {want_len[bad[:5]]},{want_err[bad[:5]]}"
    # decoded bytes of valid messages; the rest of each slot (and the whole
    # slot of an invalid message) is unspecified
    ok = want_len > 0
    got_b = segments(host(dst), host(out_off)[:-1][ok], want_len[ok])
    want_b = segments(want, want_off[:-1][ok], want_len[ok])
    assert np.array_equal(got_b, want_b)
    return gl, ge


def encode_text(data, off, flags=None):
    t, toff, _ = oracle.encode_batch(data[off[0]:], off - off[0], flags)
    return t, toff


@pytest.mark.parametrize("lens", [
    [0], [1], [5], [12], [13], [0, 0, 0], [3] * 1000, list(range(0, 300)),
    [1 << 20], [0, 1 << 20, 0, 7], [64 * 12 * 3 + 1] * 5,
])
def test_encode_batch_shapes(lens):
    data, off = packed(lens, len(lens))
    check_encode(data, off)


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_encode_batch_random_mix_with_alphabets(layout):
    rng = np.random.default_rng(1)
    for trial in range(6):
        N = int(rng.integers(1, 3000))
        lens = np.where(rng.uniform(size=N) < 0.05, rng.integers(5000, 300_000, N), rng.integers(0, 200, N))
        data, off = packed(lens, trial)
        flags = rng.integers(0, 2, N).astype(np.uint8)
        check_encode(data, off, flags, tune=dict(layout=layout))


STAGED_SHAPES = [dict(layout=2, units_per_lane=u, grid=g) for u in (1, 2, 4, 8) for g in (0, 3, 1 << 16)]


@pytest.mark.parametrize("tune", STAGED_SHAPES, ids=lambda t: f"upl{t['units_per_lane']}-grid{t['grid']}")
def test_staged_layout_shapes(tune):
    """The staged layout (tiles of 256 x units_per_lane units, input through
    LDS) at every units-per-lane value, with a grid of 3 workgroups (many
    tiles per workgroup), the default and one workgroup per tile: a mix of
    empty, tiny and long messages at every start alignment (in_off[0] = 5),
    per-message alphabets and padding modes, some decodes corrupted."""
    rng = np.random.default_rng(31 + tune["units_per_lane"])
    N = 1500
    lens = np.where(rng.uniform(size=N) < 0.04, rng.integers(3000, 60_000, N), rng.integers(0, 90, N))
    lens[rng.choice(N, 100, replace=False)] = 0
    data, off = packed(lens, 31, base=5)
    flags = rng.choice([0, 1, 4, 5], N).astype(np.uint8)  # std/url x padded/unpadded
    texts = [oracle.encode_nopad(data[off[i]:off[i + 1]], flags[i] & 1) if flags[i] & 4
             else oracle.encode(data[off[i]:off[i + 1]], flags[i] & 1) for i in range(N)]
    dst, out_off, out_len = codec.encode_batch(dev(data), dev(off), flags=dev(flags), tune=tune)
    d, oo, ol = host(dst), host(out_off), host(out_len)
    for i in range(N):
        assert ol[i] == texts[i].size and np.array_equal(d[oo[i]:oo[i] + ol[i]], texts[i]), (i, tune)
    for i in rng.choice(N, 60, replace=False):
        if texts[i].size:
            texts[i] = texts[i].copy()
            texts[i][rng.integers(0, texts[i].size)] = workloads.corruption_byte(
                int(rng.integers(0, 192)), int(flags[i] & 1), 0, texts[i].size)
    tl = np.array([t.size for t in texts], np.int64)
    toff = np.zeros(N + 1, np.int64)
    np.cumsum(tl, out=toff[1:])
    text = np.concatenate(texts)
    dflags = np.where(flags & 4, flags, flags | 2).astype(np.uint8)  # strict on the padded ones
    dst, out_off, out_len, err = codec.decode_batch(dev(text), dev(toff), flags=dev(dflags), tune=tune)
    d, oo, ol, oe = host(dst), host(out_off), host(out_len), host(err)
    for i in range(N):
        t = texts[i]
        w = oracle.decode_nopad(t, dflags[i] & 1) if dflags[i] & 4 else oracle.decode_strict(t, dflags[i] & 1)
        assert (ol[i], oe[i]) == w[:2], (i, tune)
        if w[0] > 0:
            assert np.array_equal(d[oo[i]:oo[i] + w[0]], w[2]), (i, tune)


def test_staged_layout_dense_tiles_and_long_message():
    """Tiles that start more than 256 messages (1-byte messages: the per-lane
    path), and one 60 MB message whose tiles outnumber the tile table (N +
    4096 entries) at 256 units per tile (the searched path), in both
    directions, against the oracle."""
    for lens in ([1] * 5000 + [7] * 3000, [60_000_000], [0, 3] * 2000 + [50_000_000, 5]):
        data, off = packed(lens, len(lens))
        for upl in (1, 4):
            tune = dict(layout=2, units_per_lane=upl, grid=0)
            check_encode(data, off, tune=tune)
            text, toff = encode_text(data, off)
            text[toff[-2] + (toff[-1] - toff[-2]) // 2] = ord("*")
            check_decode(text, toff, tune=tune)


def test_staged_layout_falls_back_for_gather():
    """Gather batches have no single input range per tile: the staged layout
    falls back to per-wave ranges and still matches the oracle."""
    rng = np.random.default_rng(8)
    src = rng.integers(0, 256, 300_000, dtype=np.uint8)
    N = 400
    ln = rng.integers(0, 3000, N).astype(np.int64)
    ib = rng.integers(0, src.size - 3000, N).astype(np.int64)
    dst, oo, ol = codec.encode_batch_gather(dev(src), dev(ib), dev(ln), tune=dict(layout=2, units_per_lane=4))
    d, oo = host(dst), host(oo)
    for i in range(N):
        want = oracle.encode(src[ib[i]:ib[i] + ln[i]])
        assert np.array_equal(d[oo[i]:oo[i] + want.size], want), i


def test_encode_batch_unaligned_starts():
    # in_off[0] > 0 and odd offsets put every message at a different alignment
    data, off = packed(np.random.default_rng(3).integers(0, 5000, 500), 3, base=3)
    check_encode(data, off)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("shape", [dict(block=64, units_per_lane=1, grid=1), dict(block=1024, units_per_lane=8, grid=3),
                                   dict(block=256, units_per_lane=4, grid=4096), dict(block=128, units_per_lane=2, grid=17)])
def test_batch_launch_shapes_agree(shape, layout):
    tune = dict(shape, layout=layout)
    rng = np.random.default_rng(9)
    lens = np.concatenate([rng.integers(0, 100, 2000), rng.integers(10_000, 100_000, 30)])
    rng.shuffle(lens)
    data, off = packed(lens, 9)
    check_encode(data, off, tune=tune)
    text, toff = encode_text(data, off)
    check_decode(text, toff, tune=tune)


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_decode_batch_valid_and_corrupted(layout):
    rng = np.random.default_rng(2)
    for trial in range(5):
        N = int(rng.integers(1, 4000))
        lens = np.where(rng.uniform(size=N) < 0.03, rng.integers(4000, 200_000, N), rng.integers(0, 300, N))
        data, off = packed(lens, 100 + trial)
        flags = rng.integers(0, 2, N).astype(np.uint8)
        text, toff = encode_text(data, off, flags)
        k = max(1, N // 20)
        ids = rng.choice(N, size=k, replace=False)
        workloads.corrupt_text(text, toff, ids, rng.uniform(size=k), rng.integers(0, 192, k), flags)
        gl, ge = check_decode(text, toff, flags, tune=dict(layout=layout))
        assert (ge >= 0).sum() >= 1


def test_decode_batch_garbage_lengths_and_padding():
    """Messages of every length 0..70 made of random symbols, '=' and other
    bytes: exercises length errors, misplaced padding and tails."""
    rng = np.random.default_rng(4)
    pool = np.frombuffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/==-_*\n", np.uint8)
    msgs = []
    for L in range(0, 71):
        for rep in range(8):
            m = pool[rng.integers(0, 64, L)].copy()  # symbols only
            if rep % 4 == 1 and L >= 2:
                m[-1] = ord("=")
            if rep % 4 == 2 and L >= 2:
                m[-2:] = ord("=")
            if rep % 4 == 3 and L:
                m[rng.integers(0, L)] = pool[rng.integers(0, pool.size)]
            msgs.append(m)
    lens = np.array([m.size for m in msgs], dtype=np.int64)
    toff = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=toff[1:])
    text = np.concatenate(msgs)
    for layout in (0, 1, 2):
        check_decode(text, toff, tune=dict(layout=layout))
        check_decode(text, toff, np.ones(lens.size, np.uint8), tune=dict(layout=layout))


def test_batch_matches_single_and_each():
    rng = np.random.default_rng(6)
    lens = rng.integers(0, 3000, 300)
    data, off = packed(lens, 6)
    flags = rng.integers(0, 2, lens.size).astype(np.uint8)
    dst, out_off = check_encode(data, off, flags)
    # per-message launches give the same bytes
    dst2 = torch.zeros_like(dst)
    ol2 = torch.zeros(lens.size, dtype=torch.int64, device=DEV)
    codec.encode_each(dev(data), off, host(out_off), dst2, ol2, h_flags=flags)
    torch.cuda.synchronize()
    assert torch.equal(dst, dst2)
    assert np.array_equal(host(ol2), 4 * ((lens + 2) // 3))
    text, toff = encode_text(data, off, flags)
    for i in rng.choice(lens.size, 10, replace=False):
        t = text[toff[i]:toff[i + 1]]
        out, err = codec.decode(dev(t) if t.size else torch.empty(0, dtype=torch.uint8, device=DEV), int(flags[i]))
        assert err == -1 and np.array_equal(host(out), data[off[i]:off[i + 1]])
    k = 15
    ids = rng.choice(lens.size, size=k, replace=False)
    workloads.corrupt_text(text, toff, ids, rng.uniform(size=k), rng.integers(0, 192, k), flags)
    gl, ge = check_decode(text, toff, flags)
    doff = dec_slots(toff)
    ddst = torch.zeros(max(int(doff[-1]), 1), dtype=torch.uint8, device=DEV)
    dl = torch.zeros(lens.size, dtype=torch.int64, device=DEV)
    de = torch.zeros(lens.size, dtype=torch.int64, device=DEV)
    codec.decode_each(dev(text), toff, doff, ddst, dl, de, h_flags=flags)
    torch.cuda.synchronize()
    assert np.array_equal(host(dl), gl) and np.array_equal(host(de), ge)


def test_per_message_modes_in_batch():
    """Per-message flags: URL alphabet, unpadded, strict."""
    rng = np.random.default_rng(12)
    N = 600
    lens = rng.integers(0, 80, N)
    data, off = packed(lens, 12)
    flags = rng.choice([0, 1, 4, 5], N).astype(np.uint8)  # std/url x padded/unpadded
    dst, out_off, out_len = codec.encode_batch(dev(data), dev(off), flags=dev(flags))
    d, oo, ol = host(dst), host(out_off), host(out_len)
    texts = []
    for i in range(N):
        x = data[off[i]:off[i + 1]]
        w = oracle.encode_nopad(x, flags[i] & 1) if flags[i] & 4 else oracle.encode(x, flags[i] & 1)
        assert ol[i] == w.size and np.array_equal(d[oo[i]:oo[i] + w.size], w), i
        texts.append(w)
    # decode them back; strict flag on the padded ones; some corrupted
    dflags = np.where(flags & 4, flags, flags | 2).astype(np.uint8)
    for i in rng.choice(N, 40, replace=False):
        if texts[i].size:
            t = texts[i].copy()
            t[rng.integers(0, t.size)] = ord("*")
            texts[i] = t
    tl = np.array([t.size for t in texts], np.int64)
    toff = np.zeros(N + 1, np.int64)
    np.cumsum(tl, out=toff[1:])
    text = np.concatenate(texts)
    dst, out_off, out_len, err = codec.decode_batch(dev(text), dev(toff), flags=dev(dflags))
    d, oo, ol, oe = host(dst), host(out_off), host(out_len), host(err)
    for i in range(N):
        t = texts[i]
        if dflags[i] & 4:
            w = oracle.decode_nopad(t, dflags[i] & 1)
        else:
            w = oracle.decode_strict(t, dflags[i] & 1)
        assert (ol[i], oe[i]) == w[:2], (i, dflags[i], bytes(t))
        if w[0] >= 0:
            assert np.array_equal(d[oo[i]:oo[i] + w[0]], w[2])


def test_uneven_100k_messages():
    w = workloads.uneven()
    data, off = w["payload"], w["in_off"]
    assert off.size == 100_001
    lens = np.diff(off)
    assert set(np.unique(lens % 3)) == {0, 1, 2}
    check_encode(data, off)
    text, toff = encode_text(data, off)
    applied = workloads.corrupt_text(text, toff, w["corrupt_ids"], w["corrupt_u"], w["corrupt_rank"])
    assert len(applied) == 1000
    gl, ge = check_decode(text, toff)
    for m_id, pos, b in applied:
        assert ge[m_id] >= 0 and ge[m_id] <= pos


@pytest.mark.parametrize("tune", [None, dict(layout=2, units_per_lane=4, grid=0)])
def test_heavy_mix_scaled(tune):
    """The heavy-tailed mix with per-message alphabets at reduced count
    (large messages 1-4 MiB) so the oracle finishes in seconds."""
    w = workloads.heavy_mix(count=1024, n_large=102, large=(1 << 20, 4 << 20), seed=3)
    data, off, flags = w["payload"], w["in_off"], w["flags"]
    check_encode(data, off, flags, tune=tune)
    text, toff = encode_text(data, off, flags)
    workloads.corrupt_text(text, toff, w["corrupt_ids"], w["corrupt_u"], w["corrupt_rank"], flags)
    check_decode(text, toff, flags, tune=tune)


def _host_threads():
    import os
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


# the launch shapes the benchmark timed on the 100,000-message batch (per-wave
# ranges, 128 lanes x 4 units; 32,768 / 16,384 workgroups)
UNEVEN_TIMED = {E: dict(layout=1, block=128, units_per_lane=4, grid=32768),
                D: dict(layout=1, block=128, units_per_lane=4, grid=16384)}


@pytest.mark.parametrize("shape", ["timed", "autotuned", "staged"])
def test_uneven_100k_in_timed_shapes(shape):
    """The 100,000-message batch in the launch shape the benchmark times (the
    recorded per-wave shape, and the autotuner's pick for this device, cache
    bypassed): every message's characters, lengths, verdicts, error offsets
    and decoded bytes against the oracle."""
    from paper_1704_00605_amd import autotune

    w = workloads.uneven()
    data, off = w["payload"], w["in_off"]
    if shape == "timed":
        te, td = UNEVEN_TIMED[E], UNEVEN_TIMED[D]
    elif shape == "staged":
        te = td = dict(layout=2, units_per_lane=4, grid=0)
    else:
        te, _ = autotune.tune(E, dev(data), dev(off), None, in_off_host=off, reps=1, use_cache=False)
    check_encode(data, off, tune=te)
    text, toff = encode_text(data, off)
    applied = workloads.corrupt_text(text, toff, w["corrupt_ids"], w["corrupt_u"], w["corrupt_rank"])
    assert len(applied) == 1000
    if shape == "autotuned":
        td, _ = autotune.tune(D, dev(text), dev(toff), None, in_off_host=toff, reps=1, use_cache=False)
    gl, ge = check_decode(text, toff, tune=td)
    assert (ge >= 0).sum() == 1000


@pytest.mark.parametrize("tune", [None, dict(layout=1, block=128, units_per_lane=4, grid=16384),
                                  dict(layout=2, units_per_lane=4, grid=0)])
def test_three_million_short_messages(tune):
    """3,000,000 messages of 0-40 bytes (a tenth of them empty): more
    planning chunks than each chunk can sum the totals of its predecessors
    for, so the chunk totals take their own scan pass. Every message's
    characters, lengths, verdicts, error offsets and decoded bytes against
    the oracle, with 5,000 messages corrupted for the decode."""
    rng = np.random.default_rng(21)
    lens = rng.integers(0, 41, 3_000_000)
    lens[rng.random(lens.size) < 0.1] = 0
    data, off = packed(lens, 22)
    check_encode(data, off, tune=tune)
    text, toff = encode_text(data, off)
    text = text.copy()
    tl = np.diff(toff)
    ids = rng.choice(np.flatnonzero(tl > 0), 5000, replace=False)
    text[toff[ids] + (rng.random(ids.size) * tl[ids]).astype(np.int64)] = ord("*")
    gl, ge = check_decode(text, toff, tune=tune)
    assert (ge >= 0).sum() == 5000 and np.array_equal(np.sort(np.flatnonzero(ge >= 0)), np.sort(ids))


def test_heavy_mix_8192_full_size_against_oracle():
    """The heavy-tailed mix at full size (8,192 messages, 7.25 GB, per-message
    alphabets, 41 corrupted) in the autotuned launch shape, as timed: the
    whole batch of characters equals the threaded oracle's batch, every
    message's length, verdict and error offset equals the oracle's, and every
    valid message's decoded bytes equal the oracle's decoded bytes."""
    from paper_1704_00605_amd import autotune

    th = _host_threads()
    w = workloads.heavy_mix()
    data, off, flags = w["payload"], w["in_off"], w["flags"]
    N = off.size - 1
    want_t, want_toff, want_tl = oracle.encode_batch(data, off, flags, threads=th)
    src, in_off, fl = dev(data), dev(off), dev(flags)
    tune_e, _ = autotune.tune(E, src, in_off, fl, in_off_host=off, reps=1, use_cache=False)
    text, toff_d, tl = codec.encode_batch(src, in_off, flags=fl, tune=tune_e)
    toff = host(toff_d)
    assert np.array_equal(toff, want_toff) and np.array_equal(host(tl)[:N], want_tl)
    assert torch.equal(text[: want_t.size], dev(want_t))
    del src
    # corruptions as the benchmark applies them, on the oracle's text and on
    # the device text alike
    ids, u, rk = w["corrupt_ids"], w["corrupt_u"], w["corrupt_rank"]
    tlen = np.diff(toff)
    pos = np.minimum(np.floor(u * tlen[ids]).astype(np.int64), np.maximum(tlen[ids] - 1, 0))
    vals = np.array([workloads.corruption_byte(int(r), int(flags[i]), int(p), int(tlen[i]))
                     for r, i, p in zip(rk, ids, pos)], np.uint8)
    want_t[toff[ids] + pos] = vals
    text[dev(toff[ids] + pos)] = dev(vals)
    wd, wdo, wl, we = oracle.decode_batch(want_t, want_toff, flags, threads=th)
    del want_t
    bad = np.zeros(N, bool)
    bad[ids] = True
    assert (we[bad] >= 0).all() and (we[~bad] == -1).all()
    tune_d, _ = autotune.tune(D, text, toff_d, fl, in_off_host=toff, reps=1, use_cache=False)
    out, oo_d, ol, er = codec.decode_batch(text, toff_d, flags=fl, tune=tune_d)
    oo, gl, ge = host(oo_d), host(ol)[:N], host(er)[:N]
    assert np.array_equal(gl, wl) and np.array_equal(ge, we)
    del text
    wdd = dev(wd)
    del wd
    for i in np.nonzero(wl > 0)[0]:
        assert torch.equal(out[oo[i]:oo[i] + wl[i]], wdd[wdo[i]:wdo[i] + wl[i]]), i


def test_bindings_reject_bad_arguments_before_launch():
    """Flags, result and slot arrays of the wrong type or too short for N are
    refused on the host (the kernels would read or write past them); a valid
    call still works afterwards."""
    from paper_1704_00605_amd.graph import BatchGraph

    data, off = packed([5, 7, 0, 12], seed=40)
    src, in_off = dev(data), dev(off)
    N = off.size - 1
    i64 = lambda k: torch.empty(k, dtype=torch.int64, device=DEV)
    with pytest.raises(TypeError):
        codec.encode_batch(src, in_off, flags=dev(np.zeros(N, np.int32)))
    with pytest.raises(ValueError):
        codec.encode_batch(src, in_off, flags=dev(np.zeros(N - 1, np.uint8)))
    with pytest.raises(TypeError):
        codec.batch_out_offsets(E, in_off, flags=dev(np.zeros(N, np.int64)))
    with pytest.raises(ValueError):
        codec.encode_batch(src, in_off, out_len=i64(N - 1))
    with pytest.raises(ValueError):
        codec.encode_batch(src, in_off, out_off=i64(N - 1))
    text, toff, _ = codec.encode_batch(src, in_off)
    with pytest.raises(ValueError):
        codec.decode_batch(text, toff, err_off=i64(N - 1))
    with pytest.raises(ValueError):
        codec.decode_batch_gather(text, toff[:-1].contiguous(), i64(N - 1))
    with pytest.raises(TypeError):
        codec.decode_async(text[:8], torch.empty(6, dtype=torch.uint8, device=DEV), i64(4)[::2])
    oo = codec.batch_out_offsets(D, toff)
    with pytest.raises(ValueError):
        BatchGraph(D, text, toff, oo, torch.empty(64, dtype=torch.uint8, device=DEV), i64(N), i64(N - 1))
    check_encode(data, off)


def test_out_offsets_scan_sizes():
    rng = np.random.default_rng(7)
    for N in [0, 1, 2, 1023, 1024, 1025, 5000, 100_000]:
        lens = rng.integers(0, 100, N).astype(np.int64)
        off = np.zeros(N + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        fl = rng.choice([0, 4], N).astype(np.uint8)
        e = host(codec.batch_out_offsets(E, dev(off)))
        d = host(codec.batch_out_offsets(D, dev(off), flags=dev(fl) if N else None))
        we = np.zeros(N + 1, np.int64)
        np.cumsum(4 * ((lens + 2) // 3), out=we[1:])
        assert np.array_equal(e, we) and np.array_equal(d, dec_slots(off, fl))


@pytest.mark.parametrize("alphabet", [0, 1])
def test_rejection_sweep_as_one_batch(alphabet):
    """All 256 byte values at 7 position classes (first, second, third,
    interior, n-3, n-2, n-1 of a 96-character text) as 1,792 messages of one
    batched decode: verdicts and bytes equal the oracle's per message."""
    rng = np.random.default_rng(30 + alphabet)
    base = oracle.encode(rng.integers(0, 256, 72, dtype=np.uint8), alphabet)
    n = base.size
    msgs = []
    for v in range(256):
        for pos in (0, 1, 2, 41, n - 3, n - 2, n - 1):
            t = base.copy()
            t[pos] = v
            msgs.append(t)
    text = np.concatenate(msgs)
    toff = np.arange(len(msgs) + 1, dtype=np.int64) * n
    flags = np.full(len(msgs), alphabet, np.uint8)
    gl, ge = check_decode(text, toff, flags)
    assert (ge >= 0).sum() > 1000


@pytest.mark.parametrize("layout", [0, 1])
def test_batch_misaligned_user_output_slots(layout):
    """Caller-chosen output slots at any alignment (gaps of 0..3 bytes
    between slots, destination view shifted by one byte): every message's
    output equals the oracle's and no byte between slots is written."""
    rng = np.random.default_rng(40 + layout)
    N = 700
    lens = np.where(rng.uniform(size=N) < 0.05, rng.integers(3000, 60_000, N), rng.integers(0, 400, N))
    data, off = packed(lens, 40 + layout)
    text, toff = encode_text(data, off)
    for direction in (0, 1):
        src, in_off = (data, off) if direction == 0 else (text, toff)
        n_in = np.diff(in_off)
        size = 4 * ((n_in + 2) // 3) if direction == 0 else 3 * (n_in // 4)
        gap = rng.integers(0, 4, N)
        out_off = np.zeros(N + 1, np.int64)
        np.cumsum(size + gap, out=out_off[1:])
        base = torch.full((int(out_off[-1]) + 8,), 0xAB, dtype=torch.uint8, device=DEV)
        dst = base[1:]
        oo = dev(out_off)
        tune = dict(layout=layout)
        if direction == 0:
            codec.encode_batch(dev(src), dev(in_off), oo, dst=dst, tune=tune)
            want, want_off, want_len = oracle.encode_batch(src, in_off)
        else:
            _, _, gl, ge = codec.decode_batch(dev(src), dev(in_off), oo, dst=dst, tune=tune)
            want, want_off, want_len, want_err = oracle.decode_batch(src, in_off)
            assert np.array_equal(host(gl), want_len) and np.array_equal(host(ge), want_err)
        got = host(dst)
        for i in range(N):
            L = int(want_len[i])
            if L > 0:
                assert np.array_equal(got[out_off[i]:out_off[i] + L], want[want_off[i]:want_off[i] + L]), (direction, i)
            # the gap after the slot's capacity is untouched
            assert (got[out_off[i] + size[i]:out_off[i + 1]] == 0xAB).all(), (direction, i)
        assert host(base)[0] == 0xAB


@pytest.mark.parametrize("layout", [0, 1])
def test_groups_spanning_more_than_64_messages(layout):
    """Runs of empty messages between short ones, so that one 64-unit group
    spans hundreds of messages: the per-lane search must go past its first
    window of 64 message starts. Short messages of both alphabets, and a long
    one after the runs so the single-buffer step resumes."""
    rng = np.random.default_rng(50 + layout)
    lens = []
    for _ in range(1500):
        lens += [0] * int(rng.integers(0, 200))
        lens.append(int(rng.integers(1, 40)))
    lens.append(200_000)
    lens += [0] * 300 + [5]
    flags = rng.integers(0, 2, len(lens)).astype(np.uint8)
    data, off = packed(lens, 60 + layout)
    for tune in (dict(layout=layout), dict(layout=layout, block=256, units_per_lane=4)):
        check_encode(data, off, flags, tune=tune)
        text, toff = encode_text(data, off, flags)
        check_decode(text, toff, flags, tune=tune)
