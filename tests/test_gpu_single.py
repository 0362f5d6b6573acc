"""GPU parity of the single-buffer codec against the oracle (bit-exact:
characters, bytes, return length and error offset), through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import codec, workloads

pytestmark = pytest.mark.gpu

STD, URL = codec.ALPHABET_STD, codec.ALPHABET_URL
NOPAD, STRICT = codec.MODE_NOPAD, codec.MODE_STRICT
DEV = "cuda:0"

# sizes around lane units (12 B / 16 chars), waves, the default tiles (encode
# 512 lanes x 2 units = 12,288 B; decode 256 lanes x 2 units = 8,192
# characters = 6,144 B), several tiles, the one-workgroup decode limit
# (16,384 interior units = 262,144 characters = 196,608 B) and ragged tails
SIZES = sorted(set(list(range(0, 70)) + [95, 96, 97, 767, 768, 769, 1023, 1024, 1025,
                                         6143, 6144, 6145, 12287, 12288, 12289, 16383, 16384, 16385,
                                         24575, 24576, 24577, 49151, 49152, 49153,
                                         196_605, 196_606, 196_607, 196_608, 196_609, 196_611, 196_614,
                                         3 * 4096 * 4 + 5, 200_003, 1_000_001]))


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a if a.flags.writeable else a.copy()).to(DEV)


def host(t):
    return t.cpu().numpy()


def rnd(n, seed):
    return np.random.default_rng(seed).integers(0, 256, n, dtype=np.uint8)


def oracle_mode(alphabet):
    return alphabet & 0xff


@pytest.mark.parametrize("alphabet", [STD, URL, STD | NOPAD, URL | NOPAD])
def test_encode_matches_oracle(alphabet):
    for n in SIZES:
        x = rnd(n, n)
        got = host(codec.encode(dev(x), alphabet))
        if alphabet & NOPAD:
            want = oracle.encode_nopad(x, alphabet & 0xff)
        else:
            want = oracle.encode(x, alphabet & 0xff)
        assert np.array_equal(got, want), (n, alphabet)


@pytest.mark.parametrize("alphabet", [STD, URL])
def test_decode_valid_matches_oracle(alphabet):
    for n in SIZES:
        x = rnd(n, n + 1)
        t = oracle.encode(x, alphabet)
        out, err = codec.decode(dev(t), alphabet)
        assert err == -1, (n, err)
        assert np.array_equal(host(out), x), n


def test_decode_unpadded_and_strict():
    for n in SIZES[:80] + [1000, 1001, 1002, 50_000]:
        x = rnd(n, 3 * n + 7)
        t = oracle.encode_nopad(x)
        out, err = codec.decode(dev(t), STD | NOPAD)
        want = oracle.decode_nopad(t)
        assert (err, -1 if out is None else out.numel()) == (want[1], want[0])
        assert np.array_equal(host(out), want[2])
        tp = oracle.encode(x)
        out, err = codec.decode(dev(tp), STD | STRICT)
        assert err == -1 and np.array_equal(host(out), x)
    for s in [b"Zh==", b"Zm9=", b"Zm8=", b"Zg==", b"QUJD" * 5 + b"Zh==", b"Z@==", b"QUJD" * 7 + b"Zm9="]:
        want = oracle.decode_strict(s)
        out, err = codec.decode(dev(np.frombuffer(s, np.uint8)), STD | STRICT)
        assert (out.numel() if out is not None else -1, err) == want[:2], s
    for s in [b"Zg", b"Zm9", b"Zg=", b"Z", b"ZmZmZ", b"QUJDRA", b"QUJD=A"]:
        want = oracle.decode_nopad(s)
        out, err = codec.decode(dev(np.frombuffer(s, np.uint8)), STD | NOPAD)
        assert (out.numel() if out is not None else -1, err) == want[:2], s


@pytest.mark.parametrize("alphabet", [STD, URL])
def test_strict_mode_every_leftover_symbol(alphabet):
    """Appendix A on the GPU: every symbol in the position holding the
    leftover bits, for both padded endings, after 0, 3 and 4 full quads (the
    final quad in different places of a 16-character unit), as one batched
    decode with per-message strict flags and as single-buffer calls; verdicts,
    lengths and bytes equal the oracle's strict decode."""
    syms = [oracle.symbol(v, alphabet) for v in range(64)]
    rng = np.random.default_rng(40 + alphabet)
    msgs = []
    for k in (0, 3, 4):
        prefix = bytes(oracle.encode(rng.integers(0, 256, 3 * k, dtype=np.uint8), alphabet))
        for v in range(64):
            msgs.append(prefix + bytes([syms[5], syms[v]]) + b"==")
            msgs.append(prefix + bytes([syms[5], syms[9], syms[v]]) + b"=")
    text = np.frombuffer(b"".join(msgs), np.uint8).copy()
    toff = np.zeros(len(msgs) + 1, np.int64)
    np.cumsum([len(m) for m in msgs], out=toff[1:])
    flags = np.full(len(msgs), alphabet | codec.FLAG_STRICT, np.uint8)
    out, oo, gl, ge = codec.decode_batch(dev(text), dev(toff), flags=dev(flags))
    gl, ge, oo, ob = host(gl), host(ge), host(oo), host(out)
    n_bad = 0
    for i, m in enumerate(msgs):
        want = oracle.decode_strict(np.frombuffer(m, np.uint8), alphabet)
        assert (gl[i], ge[i]) == want[:2], (i, m)
        if want[0] >= 0:
            assert bytes(ob[oo[i]:oo[i] + want[0]]) == bytes(want[2])
        n_bad += want[0] < 0
        if i % 7 == 0:
            got, err = codec.decode(dev(np.frombuffer(m, np.uint8)), alphabet | STRICT)
            assert (-1 if got is None else got.numel(), err) == want[:2], m
    assert 0 < n_bad < len(msgs)


@pytest.mark.parametrize("alphabet", [STD, URL])
def test_unpadded_mode_every_final_symbol(alphabet):
    """The unpadded mode (Section 2) on the GPU: every symbol as the last
    character of a final group of 2 or 3 characters (leftover bits accepted,
    as in the padded mode without Appendix A), after 0, 3 and 4 full quads,
    as one batched decode whose messages also carry the strict flag (ignored
    for unpadded messages) and as single-buffer calls; equal to the oracle's
    unpadded decode."""
    syms = [oracle.symbol(v, alphabet) for v in range(64)]
    rng = np.random.default_rng(50 + alphabet)
    msgs = []
    for k in (0, 3, 4):
        prefix = bytes(oracle.encode(rng.integers(0, 256, 3 * k, dtype=np.uint8), alphabet))
        for v in range(64):
            msgs.append(prefix + bytes([syms[5], syms[v]]))
            msgs.append(prefix + bytes([syms[5], syms[9], syms[v]]))
    text = np.frombuffer(b"".join(msgs), np.uint8).copy()
    toff = np.zeros(len(msgs) + 1, np.int64)
    np.cumsum([len(m) for m in msgs], out=toff[1:])
    flags = np.full(len(msgs), alphabet | codec.FLAG_NOPAD | codec.FLAG_STRICT, np.uint8)
    out, oo, gl, ge = codec.decode_batch(dev(text), dev(toff), flags=dev(flags))
    gl, ge, oo, ob = host(gl), host(ge), host(oo), host(out)
    for i, m in enumerate(msgs):
        want = oracle.decode_nopad(np.frombuffer(m, np.uint8), alphabet)
        assert want[1] == -1 and (gl[i], ge[i]) == want[:2], (i, m)
        assert bytes(ob[oo[i]:oo[i] + want[0]]) == bytes(want[2])
        if i % 7 == 0:
            got, err = codec.decode(dev(np.frombuffer(m, np.uint8)), alphabet | NOPAD)
            assert err == -1 and bytes(host(got)) == bytes(want[2]), m


def test_padding_and_length_readings():
    cases = [b"", b"Zg==", b"Zh==", b"Zm8=", b"Zg==AAAA", b"AB=C", b"Zg=", b"Z===", b"====",
             b"=AAA", b"A", b"AB", b"ABC", b"AB\x80D", b"AB D", b"A@C", b"QUJD" * 4 + b"Zg==",
             b"QUJD" * 4 + b"Z===", b"QUJD" * 4 + b"Zg=A", b"QUJD" * 3 + b"Zg==",
             b"QUJD" * 8 + b"=", b"QUJD" * 8 + b"==", b"QUJD" * 5 + b"A", b"QU=D" * 5]
    for s in cases:
        want = oracle.decode(s)
        out, err = codec.decode(dev(np.frombuffer(s, np.uint8)) if s else torch.empty(0, dtype=torch.uint8, device=DEV))
        got_len = -1 if out is None else out.numel()
        assert (got_len, err) == want[:2], s
        if out is not None:
            assert bytes(host(out)) == bytes(want[2])


@pytest.mark.parametrize("alphabet", [STD, URL])
def test_rejection_sweep_all_bytes_and_positions(alphabet):
    """Every byte value at every position class of texts whose lengths put
    the position in an interior unit, a tail unit and the padding quad."""
    rng = np.random.default_rng(21)
    for n_bytes in (30, 31, 32, 100, 3 * 64):
        x = rng.integers(0, 256, n_bytes, dtype=np.uint8)
        t = oracle.encode(x, alphabet)
        m = t.size
        positions = sorted(set([0, 1, 15, 16, 17, m // 2, m - 17, m - 16, m - 5, m - 4, m - 3, m - 2, m - 1]))
        for pos in positions:
            if not 0 <= pos < m:
                continue
            for b in range(256):
                tt = t.copy()
                tt[pos] = b
                want = oracle.decode(tt, alphabet)
                out, err = codec.decode(dev(tt), alphabet)
                assert ((-1 if out is None else out.numel()), err) == want[:2], (n_bytes, pos, b)


def test_injected_errors_and_minimum_offset():
    rng = np.random.default_rng(5)
    for n in [100, 1000, 12289, 100_000, 1_000_003]:
        x = rnd(n, n)
        t = oracle.encode(x)
        for _ in range(6):
            tt = t.copy()
            k = int(rng.integers(1, 5))
            pos = rng.integers(0, t.size, size=k)
            for p in pos:
                tt[p] = workloads.corruption_byte(int(rng.integers(0, 192)), 0, int(p), t.size)
            want = oracle.decode(tt)
            out, err = codec.decode(dev(tt))
            assert ((-1 if out is None else out.numel()), err) == want[:2], (n, pos)


@pytest.mark.parametrize("soff,doff", [(1, 0), (0, 1), (2, 3), (3, 2), (5, 7), (13, 15), (4, 8)])
def test_misaligned_subbuffers(soff, doff):
    # 1,000,003 bytes: decode leaves the one-workgroup kernel (256 KiB and below)
    for n in [0, 1, 2, 3, 11, 12, 13, 100, 4097, 100_001, 1_000_003]:
        x = rnd(n, n + soff)
        big = torch.zeros(n + 64, dtype=torch.uint8, device=DEV)
        big[soff:soff + n] = dev(x) if n else big[:0]
        m = oracle.encoded_len(n)
        outbig = torch.full((m + 64,), 0xAB, dtype=torch.uint8, device=DEV)
        got = codec.encode(big[soff:soff + n], STD, out=outbig[doff:doff + m])
        assert np.array_equal(host(got), oracle.encode(x)), (n, soff, doff)
        ob = host(outbig)
        assert np.all(ob[:doff] == 0xAB) and np.all(ob[doff + m:] == 0xAB)  # no stray writes
        t = oracle.encode(x)
        tb = torch.zeros(m + 64, dtype=torch.uint8, device=DEV)
        tb[soff:soff + m] = dev(t) if m else tb[:0]
        cap = oracle.decoded_max(m)
        db = torch.full((cap + 64,), 0xCD, dtype=torch.uint8, device=DEV)
        out, err = codec.decode(tb[soff:soff + m], STD, out=db[doff:doff + cap])
        assert err == -1 and np.array_equal(host(out), x), (n, soff, doff)
        dbh = host(db)
        assert np.all(dbh[:doff] == 0xCD) and np.all(dbh[doff + n:] == 0xCD)


# (block, units per lane, blocks per CU; -1 = one workgroup per tile)
SPLIT_SHAPES = [(256, 2, -1), (64, 1, -1), (1024, 8, -1), (512, 4, 1), (128, 2, 3)]


@pytest.mark.parametrize("shape", SPLIT_SHAPES, ids=[f"{b}x{u}_g{g}" for b, u, g in SPLIT_SHAPES])
def test_misaligned_destination_whole_dword_runs(shape):
    """A destination that is not 4-byte aligned is written in whole dwords per
    wave, each wave rebuilding the last word of the unit before its own: every
    launch shape (one-shot and grid-stride, guarded last tiles), every
    character map, sizes around the tile edges, against the oracle, with
    guard bytes on both sides of the output."""
    b, u, g = shape
    try:
        for n in [13, 12 * 64 + 1, 12 * 64 * 5 + 11, 100_003, 1_000_001]:
            x = rnd(n, n + b)
            t = oracle.encode(x)
            m = t.size
            for doff in (1, 2, 3):
                for char_map in (0, 1, 2):
                    codec.set_single_tune(0, b, u, g, char_map)
                    outbig = torch.full((m + 16,), 0xAB, dtype=torch.uint8, device=DEV)
                    codec.encode(dev(x), out=outbig[doff:doff + m])
                    ob = host(outbig)
                    assert np.array_equal(ob[doff:doff + m], t), (n, doff, char_map)
                    assert np.all(ob[:doff] == 0xAB) and np.all(ob[doff + m:] == 0xAB)
                for char_map in (0, 1):
                    codec.set_single_tune(1, b, u, g, char_map)
                    cap = oracle.decoded_max(m)
                    db = torch.full((cap + 16,), 0xCD, dtype=torch.uint8, device=DEV)
                    out, err = codec.decode(dev(t), out=db[doff:doff + cap])
                    assert err == -1 and np.array_equal(host(out), x), (n, doff, char_map)
                    dbh = host(db)
                    assert np.all(dbh[:doff] == 0xCD) and np.all(dbh[doff + n:] == 0xCD)
                    bad = t.copy()
                    bad[m // 2] = ord("?")
                    got, err = codec.decode(dev(bad), out=db[doff:doff + cap])
                    assert (got, err) == (None, oracle.decode(bad)[1]), (n, doff, char_map)
    finally:
        codec.set_single_tune(0, 512, 2, -1, 0)
        codec.set_single_tune(1, 256, 2, -1, 0)


def test_decode_writes_nothing_past_the_decoded_length():
    for n in [1, 2, 4, 5, 100, 1001]:
        x = rnd(n, 99 + n)
        t = oracle.encode(x)
        cap = oracle.decoded_max(t.size)
        buf = torch.full((cap + 32,), 0x5A, dtype=torch.uint8, device=DEV)
        out, err = codec.decode(dev(t), out=buf[:cap])
        b = host(buf)
        assert np.array_equal(b[:n], x) and np.all(b[n:] == 0x5A)


def test_async_decode_slots():
    res = torch.zeros(2, dtype=torch.int64, device=DEV)
    for n in [0, 1, 50, 100_000]:
        x = rnd(n, n)
        t = oracle.encode(x)
        tt = t.copy()
        if t.size:
            tt[t.size // 3] = ord("*")
        for txt in (t, tt):
            out = torch.empty(oracle.decoded_max(txt.size) + 1, dtype=torch.uint8, device=DEV)
            src = dev(txt) if txt.size else torch.empty(0, dtype=torch.uint8, device=DEV)
            codec.decode_async(src, out, res)
            torch.cuda.synchronize()
            want = oracle.decode(txt)
            assert tuple(host(res)) == want[:2]


def test_all_2_24_triples_closed_form():
    i = np.arange(1 << 24, dtype=np.uint32)
    buf = np.stack([(i >> 16) & 255, (i >> 8) & 255, i & 255], axis=1).astype(np.uint8).reshape(-1)
    for alphabet in (STD, URL):
        t = codec.encode(dev(buf), alphabet)
        assert np.array_equal(host(t), oracle.encode(buf, alphabet))
        out, err = codec.decode(t, alphabet)
        assert err == -1 and torch.equal(out, dev(buf))


def test_one_mib_seed0():
    w = workloads.single(1 << 20, seed=0)
    x = w["payload"]
    t = codec.encode(dev(x))
    want = oracle.encode(x)
    assert t.numel() == 1_398_104 and np.array_equal(host(t), want)
    out, err = codec.decode(t)
    assert err == -1 and np.array_equal(host(out), x)
    tt = want.copy()
    applied = workloads.corrupt_text(tt, np.array([0, tt.size]), [0], [w["corrupt_u"]], [w["corrupt_rank"]])
    (_, pos, _b), = applied
    ow = oracle.decode(tt)
    assert ow[:2] == (-1, pos)
    out, err = codec.decode(dev(tt))
    assert (out, err) == (None, pos)


def _host_threads():
    """Host threads for the threaded oracle (the machine's CPU share is 16)."""
    import os
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def test_one_gib_full_against_oracle():
    """1 GiB (seed 1) in the benchmark's launch shape and calls: the whole
    encoded text equals the oracle's text, the whole decoded output
    (asynchronous decode, as timed) equals the oracle's decode of its own
    text, and with the invalid byte at 99.9% of the text both the oracle and
    the GPU report -1 at exactly that offset."""
    th = _host_threads()
    n = 1 << 30
    w = workloads.single_at_fraction(n, seed=1, frac=0.999)
    xh = w["payload"]
    want_t = oracle.encode(xh, threads=th)
    assert want_t.size == 1_431_655_768
    x = dev(xh)
    m = codec.encoded_len(n)
    t = torch.empty(m, dtype=torch.uint8, device=DEV)
    codec.encode(x, out=t)
    assert torch.equal(t, dev(want_t))
    ow = oracle.decode(want_t, threads=th)
    assert ow[:2] == (n, -1)
    out = torch.empty(codec.decoded_max(m), dtype=torch.uint8, device=DEV)
    res = torch.zeros(2, dtype=torch.int64, device=DEV)
    codec.decode_async(t, out, res)
    torch.cuda.synchronize()
    assert host(res).tolist() == [n, -1]
    assert torch.equal(out[:n], dev(ow[2]))
    del ow
    pos = int(np.floor(0.999 * m))
    assert pos == 1_430_224_112
    b = workloads.corruption_byte(w["corrupt_rank"], 0, pos, m)
    want_t[pos] = b
    t[pos] = b
    ow = oracle.decode(want_t, threads=th)
    assert ow[:2] == (-1, pos)
    codec.decode_async(t, out, res)
    torch.cuda.synchronize()
    assert host(res).tolist() == [-1, pos]
    got, err = codec.decode(t)
    assert got is None and err == pos


def test_table7_file_sizes_match_oracle():
    """Texts at the six sizes of the paper's decoding table (synthetic
    payloads): encode and decode agree with the oracle byte for byte."""
    from paper_1704_00605_amd import workloads
    for name, size, payload in workloads.table7_files():
        t = codec.encode(torch.from_numpy(payload).to("cuda:0"))
        want = oracle.encode(payload)
        assert t.numel() == size // 4 * 4 and np.array_equal(t.cpu().numpy(), want), name
        out, err = codec.decode(t)
        w = oracle.decode(want)
        assert err == -1 and out.numel() == w[0] and np.array_equal(out.cpu().numpy(), w[2]), name


def test_single_buffer_beyond_4gib():
    """5 GiB (byte offsets above 2^32): the whole text equals the oracle's
    encoding of the same bytes, the whole decoded output equals the oracle's
    decode of that text, and an injected byte near the end is found at its
    index by both."""
    th = _host_threads()
    n = 5 << 30
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda:0", generator=g)
    t = codec.encode(x)
    m = t.numel()
    assert m == 4 * -(-n // 3)
    want_t = oracle.encode(host(x), threads=th)
    assert want_t.size == m
    assert torch.equal(t, dev(want_t))
    ow = oracle.decode(want_t, threads=th)
    assert ow[:2] == (n, -1)
    out, err = codec.decode(t)
    assert err == -1 and out.numel() == n and torch.equal(out, dev(ow[2]))
    del out, ow
    pos = m - 4097
    t[pos] = ord("*")
    want_t[pos] = ord("*")
    assert oracle.decode(want_t, threads=th)[:2] == (-1, pos)
    out, err = codec.decode(t)
    assert out is None and err == pos


def _chunk_payload(i, size):
    """Chunk i of a payload generated on the device chunk by chunk (seed 40 + i)."""
    g = torch.Generator(device=DEV)
    g.manual_seed(40 + i)
    return torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=g)


def _need_device_bytes(b):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < b:
        pytest.skip(f"needs {b / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")


def test_launch_shape_beyond_2_32_work_items():
    """A payload of more than 2^32 encode units (51.5 GB) at 1,024 lanes x 1
    unit with one workgroup per tile: that grid would hold more than 2^32
    work-items, more than one launch takes, so it is capped and the kernels
    stride over the remaining tiles. The decode of the text (also more than
    2^32 units) gives back every byte of the payload, and windows of the
    text, last unit included, equal the oracle's encoding of the same
    bytes."""
    CH = 3 << 30                                     # payload chunk (a multiple of 3)
    n = 12 * ((1 << 32) + (1 << 20)) + 7             # 4,296,015,872 units + 7 bytes
    m = 4 * -(-n // 3)
    _need_device_bytes(n + m + n + (8 << 30))
    chunks = [(i, min(CH, n - o)) for i, o in enumerate(range(0, n, CH))]
    x = torch.empty(n, dtype=torch.uint8, device=DEV)
    for i, size in chunks:
        x[i * CH:i * CH + size] = _chunk_payload(i, size)
    try:
        for d in (0, 1):
            codec.set_single_tune(d, 1024, 1, -1, 0)
        t = codec.encode(x)
        assert t.numel() == m
        windows = [0, 3 * (1 << 31), 12 * ((1 << 32) - 5), n - n % 3 - 3 * 4096, n - n % 3 - 3]
        want = [(a, oracle.encode(host(x[a:min(a + 3 * 4096, n)]))) for a in windows]
        want.append((n - n % 3, oracle.encode(host(x[n - n % 3:]))))  # the padded final group
        del x
        for a, w in want:
            assert np.array_equal(host(t[4 * a // 3:4 * a // 3 + w.size]), w), a
        out, err = codec.decode(t)
        assert err == -1 and out.numel() == n
        del t
        for i, size in chunks:
            assert torch.equal(out[i * CH:i * CH + size], _chunk_payload(i, size)), i
    finally:
        codec.set_single_tune(0, 512, 2, -1, 0)
        codec.set_single_tune(1, 256, 2, -1, 0)
        torch.cuda.empty_cache()


def test_plain_entry_points_on_the_null_stream():
    """b64_encode / b64_decode (Section 2, Algorithms 1 and 2) called through
    ctypes as declared: device buffers, the NULL stream, a host err_off. The
    1 MiB seed-0 payload, its text, the copy with an invalid byte at the
    seeded position, and a text whose length is not a multiple of 4."""
    import ctypes

    from paper_1704_00605_amd import _lib

    L = _lib.lib()
    w = workloads.single(1 << 20, seed=0)
    x = w["payload"]
    want_t = oracle.encode(x)
    m = want_t.size
    xd = dev(x)
    td = torch.zeros(m, dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    assert L.b64_encode(ctypes.c_void_p(xd.data_ptr()), x.size, ctypes.c_void_p(td.data_ptr())) == m
    assert np.array_equal(host(td), want_t)
    out = torch.zeros(oracle.decoded_max(m), dtype=torch.uint8, device=DEV)
    err = ctypes.c_int64(7)
    r = L.b64_decode(ctypes.c_void_p(td.data_ptr()), m, ctypes.c_void_p(out.data_ptr()), ctypes.byref(err))
    assert (r, err.value) == (x.size, -1) and np.array_equal(host(out)[: x.size], x)
    pos = min(int(np.floor(w["corrupt_u"] * m)), m - 1)
    bad = want_t.copy()
    bad[pos] = workloads.corruption_byte(w["corrupt_rank"], 0, pos, m)
    bd = dev(bad)
    r = L.b64_decode(ctypes.c_void_p(bd.data_ptr()), m, ctypes.c_void_p(out.data_ptr()), ctypes.byref(err))
    assert (r, err.value) == (_lib.INVALID_INPUT, pos) == oracle.decode(bad)[:2]
    # length error: 4k + 3 symbols (the padded final quad cut off) -> -1 at n
    k = m - 5
    r = L.b64_decode(ctypes.c_void_p(td.data_ptr()), k, ctypes.c_void_p(out.data_ptr()), ctypes.byref(err))
    assert (r, err.value) == oracle.decode(want_t[:k])[:2] == (-1, k)
    # ... and cut inside the padding: the '=' left at index m - 2 is then invalid
    r = L.b64_decode(ctypes.c_void_p(td.data_ptr()), m - 1, ctypes.c_void_p(out.data_ptr()), ctypes.byref(err))
    assert (r, err.value) == oracle.decode(want_t[: m - 1])[:2] == (-1, m - 2)


def test_device_slot_scan_equals_host_layout():
    """b64_batch_out_offsets (in-place device scan) equals b64_batch_slots
    (host) for batch sizes around its chunk boundaries, with mixed flags,
    and the slot sizes equal the length law."""
    rng = np.random.default_rng(77)
    for N in [0, 1, 2, 2047, 2048, 2049, 4096, 6143, 100_000, (1 << 21) + 5]:
        lens = rng.integers(0, 5000, N).astype(np.int64)
        off = np.zeros(N + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        flags = rng.integers(0, 8, N).astype(np.uint8)
        for d in (codec.DIR_ENCODE, codec.DIR_DECODE):
            got = host(codec.batch_out_offsets(d, dev(off), dev(flags) if N else None))
            need, want = codec.batch_slots(d, lens, flags)
            assert np.array_equal(got, want), (N, d)
            if d == codec.DIR_ENCODE:
                assert np.array_equal(np.diff(want), 4 * ((lens + 2) // 3))
            else:
                assert np.all(np.diff(want) >= need) and np.all(np.diff(want) % 4 == 0)
