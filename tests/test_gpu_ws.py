"""Whitespace-tolerant decode (Appendix B: space, LF and CR are removed before
decoding) on the GPU against the oracle's decode_ws, which strips, decodes
and reports errors in the coordinates of the original input."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import codec, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [(256, 1), (256, 2), (256, 4), (256, 8), (512, 1), (512, 2), (512, 4), (1024, 1), (1024, 2)]


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a if a.flags.writeable else a.copy()).to(DEV)


def gpu_ws(a, alphabet=0, shift=0):
    """decode_ws of host bytes `a`, placed `shift` bytes into a device buffer."""
    buf = torch.zeros(a.size + shift + 4, dtype=torch.uint8, device=DEV)
    if a.size:
        buf[shift:shift + a.size] = dev(a)
    out, err = codec.decode_ws(buf[shift:shift + a.size], alphabet)
    return (-1, err, None) if out is None else (out.numel(), -1, out.cpu().numpy())


def injected(rank, pos, m, alphabet=0):
    """A byte outside the alphabet that is not removed as whitespace."""
    while True:
        b = workloads.corruption_byte(rank % 192, alphabet, pos, m)
        if b not in workloads.WS_BYTES:
            return b
        rank += 1


def check(a, alphabet=0, shift=0):
    want = oracle.decode_ws(a, alphabet)
    got = gpu_ws(a, alphabet, shift)
    assert got[:2] == want[:2], (got[:2], want[:2], a.size)
    if want[0] > 0:
        assert np.array_equal(got[2], want[2])
    return want


@pytest.fixture(autouse=True)
def default_shape():
    yield
    codec.set_ws_tune(256, 2)


def test_ws_small_random_cases():
    rng = np.random.default_rng(0)
    for trial in range(400):
        L = int(rng.integers(0, 400))
        text = oracle.encode(rng.integers(0, 256, L, dtype=np.uint8))
        a, _ = workloads.sprinkle_ws(rng, text, float(rng.choice([0, 0.05, 0.3, 0.9])))
        if rng.uniform() < 0.3 and a.size:
            a[rng.integers(0, a.size)] = rng.choice([ord("="), ord("#"), ord("A"), 0x80, ord("-"), 9, 0, 0x1F, 0x21])
        if rng.uniform() < 0.1 and a.size:
            a = a[:-1]
        check(a)


@pytest.mark.parametrize("shape", SHAPES)
def test_ws_multi_tile_layouts_every_shape(shape):
    codec.set_ws_tune(*shape)
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, 200_003, dtype=np.uint8)
    text = oracle.encode(x)
    for width, eol in ((76, b"\r\n"), (64, b"\n")):
        a, _ = workloads.wrap_lines(text, width, eol)
        w = check(a)
        assert w[0] == x.size and np.array_equal(w[2], x)
    a, _ = workloads.sprinkle_ws(rng, text, 0.2, run_max=5)
    check(a)


def test_ws_every_dword_keep_pattern():
    """Each aligned dword of the input keeps the bytes of one of the 16
    kept/removed patterns, dword i taking pattern (7 i + i // 16) mod 16, so
    every pattern follows stripped runs of every length mod 4 and sits in
    every lane and tile position; the removed bytes cycle through space, LF
    and CR."""
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, 150_000, dtype=np.uint8)
    text = oracle.encode(x)
    i = np.arange(2 * text.size // 4 + 64)
    pat = (7 * i + i // 16) % 16
    kept = ((pat[:, None] >> np.arange(4)) & 1).astype(bool).ravel()
    where = np.flatnonzero(kept)[:text.size]
    a = workloads.WS_BYTES[np.arange(kept.size) % 3].copy()
    a[where] = text
    a = a[:where[-1] + 1 + 37]                          # ends inside a dword
    for shape in ((256, 1), (256, 2), (1024, 2)):
        codec.set_ws_tune(*shape)
        w = check(a)
        assert w[1] == -1 and w[0] == x.size and np.array_equal(w[2], x)
        check(a, shift=3)                               # dwords of the input no longer aligned


def test_ws_long_whitespace_runs_across_tiles():
    # runs longer than any tile: tiles with no kept byte, quads and padding
    # split across such tiles
    rng = np.random.default_rng(2)
    for shape in ((256, 1), (1024, 2)):
        codec.set_ws_tune(*shape)
        for L in (1, 2, 3, 4, 5, 1000, 4099):
            text = oracle.encode(rng.integers(0, 256, L, dtype=np.uint8))
            parts = []
            for i, ch in enumerate(text):
                if rng.uniform() < 0.2:
                    parts.append(workloads.WS_BYTES[rng.integers(0, 3, int(rng.integers(1, 20_000)))])
                parts.append(np.array([ch], np.uint8))
            parts.append(workloads.WS_BYTES[rng.integers(0, 3, 50_000)])
            a = np.concatenate(parts)
            w = check(a)
            assert w[1] == -1


def test_ws_all_whitespace_and_empty():
    for n in (0, 1, 3, 4, 5000, 70_000):
        a = workloads.WS_BYTES[np.arange(n) % 3]
        assert gpu_ws(a)[:2] == (0, -1)
        check(a)


@pytest.mark.parametrize("case", [
    b"Zg==", b"Zg=\n=", b"Zg\r\n==\r\n", b"Z g = =", b"Zg=X", b"Zg==Zg==", b"Z===", b"Zm9v\nYg",
    b"Zm9vYg=", b"=", b"==", b"Zh==", b"Zm9v YmFy", b"Zm9v\tYmFy", b"QUJD\n\n\n\nREVG\n",
    b"Zg==\t", b"Zg=\t=", b"Z\x00g==", b"Zg\x1f=", b"Zm9v\x0bYmFy==",
])
def test_ws_padding_and_length_readings(case):
    a = np.frombuffer(case, np.uint8).copy()
    check(a)


def test_ws_errors_in_original_coordinates():
    rng = np.random.default_rng(3)
    text = oracle.encode(rng.integers(0, 256, 150_000, dtype=np.uint8))
    a, pos = workloads.wrap_lines(text, 76, b"\r\n")
    for trial in range(40):
        b = a.copy()
        j = int(rng.integers(0, text.size))
        b[pos[j]] = injected(int(rng.integers(0, 192)), j, text.size)
        w = check(b)
        assert w[:2] == (-1, int(pos[j]))
    # a tab in place of a line's CR is not removed: an error at its index
    b = a.copy()
    b[pos[76 * 3 - 1] + 1] = ord("\t")
    assert check(b)[:2] == (-1, int(pos[76 * 3 - 1]) + 1)
    # two errors: the first in original order wins
    b = a.copy()
    b[pos[9000]] = ord("*")
    b[pos[100]] = ord("=")
    assert check(b)[:2] == (-1, int(pos[100]))


def test_ws_url_alphabet_and_misaligned_buffers():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, 90_001, dtype=np.uint8)
    text = oracle.encode(x, 1)
    a, _ = workloads.wrap_lines(text, 64, b"\n")
    for shift in (0, 1, 2, 3):
        w = check(a, alphabet=1, shift=shift)
        assert np.array_equal(w[2], x)
    b = a.copy()
    b[10] = ord("+")  # standard-only symbol
    check(b, alphabet=1)
    # unaligned output view
    out = torch.zeros(3 * (a.size // 4) + 3, dtype=torch.uint8, device=DEV)
    got, err = codec.decode_ws(dev(a), 1, out=out[1:])
    assert err == -1 and np.array_equal(got.cpu().numpy(), x)
    assert out[0].item() == 0


def test_ws_async_reuses_workspace_and_writes_nothing_past_the_length():
    rng = np.random.default_rng(5)
    ws = torch.empty(codec.ws_workspace_bytes(1 << 20), dtype=torch.uint8, device=DEV)
    res = torch.zeros(2, dtype=torch.int64, device=DEV)
    for L in (700_000, 123, 50_001, 0, 1):
        x = rng.integers(0, 256, L, dtype=np.uint8)
        a, _ = workloads.wrap_lines(oracle.encode(x), 76, b"\r\n")
        out = torch.full((3 * (a.size // 4) + 64,), 0xEE, dtype=torch.uint8, device=DEV)
        codec.decode_ws_async(dev(a), out, res, ws)
        torch.cuda.synchronize()
        assert res.tolist() == [L, -1]
        o = out.cpu().numpy()
        assert np.array_equal(o[:L], x) and (o[L:] == 0xEE).all()


def test_ws_async_captured_in_a_graph():
    """decode_ws_async enqueues kernels only (an empty input too), so it
    records into a HIP graph; the graph (an empty input, a valid text and a
    text with an invalid byte, each with its own workspace) is replayed
    three times with eager decodes of other texts between the replays, and
    every replay's verdicts and bytes equal the oracle's."""
    rng = np.random.default_rng(8)
    x = rng.integers(0, 256, 300_001, dtype=np.uint8)
    a, pos = workloads.wrap_lines(oracle.encode(x), 76, b"\r\n")
    bad = a.copy()
    bad[pos[123_457]] = ord("*")
    texts = [np.zeros(0, np.uint8), a, bad]
    want = [oracle.decode_ws(t) for t in texts]
    assert [w[:2] for w in want] == [(0, -1), (x.size, -1), (-1, int(pos[123_457]))]
    srcs = [dev(t) if t.size else torch.zeros(1, dtype=torch.uint8, device=DEV)[:0] for t in texts]
    outs = [torch.zeros(3 * (t.size // 4) + 4, dtype=torch.uint8, device=DEV) for t in texts]
    wss = [torch.empty(codec.ws_workspace_bytes(t.size), dtype=torch.uint8, device=DEV) for t in texts]
    res = torch.zeros(6, dtype=torch.int64, device=DEV)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for k in range(3):
                codec.decode_ws_async(srcs[k], outs[k], res[2 * k:2 * k + 2], wss[k], stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        res.fill_(7)
        for o in outs:
            o.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        for k in range(3):
            assert tuple(res[2 * k:2 * k + 2].tolist()) == want[k][:2], (r, k)
        assert np.array_equal(outs[1][:x.size].cpu().numpy(), x)
        y = rng.integers(0, 256, 5000 + r, dtype=np.uint8)
        check(workloads.wrap_lines(oracle.encode(y), 64, b"\n")[0])


def test_ws_mime_1gib_properties():
    """Full-size MIME text (1 GiB payload, 76-character CRLF lines): the decode
    returns the payload; with one injected byte it reports that byte's
    original index. Both hold by construction at any size."""
    w = workloads.mime_1gib()
    x = torch.from_numpy(w["payload"]).to(DEV)
    del w["payload"]
    m = codec.encoded_len(x.numel())
    text = codec.encode(x)
    lines = -(-m // 76)
    wrapped = torch.empty(m + 2 * lines, dtype=torch.uint8, device=DEV)
    full = m // 76
    v = wrapped[: full * 78].view(full, 78)
    v[:, :76] = text[: full * 76].view(full, 76)
    v[:, 76] = 13
    v[:, 77] = 10
    rest = m - full * 76
    if rest:
        wrapped[full * 78: full * 78 + rest] = text[full * 76:]
        wrapped[full * 78 + rest:] = torch.tensor([13, 10], dtype=torch.uint8, device=DEV)
    del text
    out, err = codec.decode_ws(wrapped)
    assert err == -1 and out.numel() == x.numel() and torch.equal(out, x)
    j = min(int(w["corrupt_u"] * m), m - 3)
    p = j + 2 * (j // 76)
    wrapped[p] = injected(w["corrupt_rank"], j, m)
    del out
    out, err = codec.decode_ws(wrapped)
    assert out is None and err == p


def test_ws_every_control_byte_is_an_error():
    """Bytes at or below 0x20 other than space, LF and CR are invalid
    (Appendix B removes only those three): each one, at random places of a
    multi-tile text without padding, is reported at its own index."""
    rng = np.random.default_rng(7)
    text = oracle.encode(rng.integers(0, 256, 60_000, dtype=np.uint8))
    a, _ = workloads.wrap_lines(text, 76, b"\r\n")
    for shape in ((256, 1), (256, 2)):
        codec.set_ws_tune(*shape)
        for b in range(0x21):
            if b in (0x0A, 0x0D, 0x20):
                continue
            for _ in range(3):
                c = a.copy()
                j = int(rng.integers(0, a.size))
                c[j] = b
                assert check(c)[:2] == (-1, j), (shape, b, j)


@pytest.mark.parametrize("shape", [(256, 1), (512, 2), (256, 8)])
def test_ws_marks_next_to_tile_boundaries(shape):
    """Invalid bytes and '=' just before and after tile boundaries, where the
    last kept bytes of a tile form a partial quad that the next tile decodes."""
    codec.set_ws_tune(*shape)
    tile = shape[0] * 16 * shape[1]
    rng = np.random.default_rng(8)
    text = oracle.encode(rng.integers(0, 256, 5 * tile, dtype=np.uint8))
    a, _ = workloads.sprinkle_ws(rng, text, 0.03)
    for t in range(1, a.size // tile):
        for d in range(-5, 5):
            j = t * tile + d
            if a[j] in workloads.WS_BYTES:
                continue
            for bad in (ord("*"), ord("="), 0x80):
                c = a.copy()
                c[j] = bad
                check(c)


def test_ws_beyond_4gib():
    """A 4.5 GB MIME text (byte offsets above 2^32): the whitespace-tolerant
    decode returns the payload; an invalid byte and, separately, a misplaced
    '=' past 2^32 are reported at their original indexes; sampled lines
    decode as the oracle decodes them."""
    n = 3_400_000_001
    g = torch.Generator(device=DEV)
    g.manual_seed(12)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, device=DEV, generator=g)
    text = codec.encode(x)
    m = text.numel()
    full = m // 76
    rest = m - full * 76
    wrapped = torch.empty(m + 2 * (full + (1 if rest else 0)), dtype=torch.uint8, device=DEV)
    v = wrapped[: full * 78].view(full, 78)
    v[:, :76] = text[: full * 76].view(full, 76)
    v[:, 76] = 13
    v[:, 77] = 10
    if rest:
        wrapped[full * 78: full * 78 + rest] = text[full * 76:]
        wrapped[full * 78 + rest:] = torch.tensor([13, 10], dtype=torch.uint8, device=DEV)
    del text
    assert wrapped.numel() > (1 << 32)
    out, err = codec.decode_ws(wrapped)
    assert err == -1 and out.numel() == n and torch.equal(out, x)
    # sampled lines past 2^32 against the oracle
    for line in (full - 3, (1 << 32) // 78 + 5):
        seg = wrapped[line * 78: line * 78 + 3 * 78].cpu().numpy()
        want = oracle.decode_ws(seg)
        assert want[1] == -1
        assert np.array_equal(out[line * 57: line * 57 + want[0]].cpu().numpy(), want[2])
    del out
    p = (1 << 32) + 78 * 1000 + 17
    keep = int(wrapped[p].item())
    wrapped[p] = ord("*")
    out, err = codec.decode_ws(wrapped)
    assert out is None and err == p
    wrapped[p] = ord("=")
    out, err = codec.decode_ws(wrapped)
    assert out is None and err == p
    wrapped[p] = keep


def _chunk_payload(i, size):
    """Chunk i of a payload generated on the device chunk by chunk (seed 60 + i)."""
    g = torch.Generator(device=DEV)
    g.manual_seed(60 + i)
    return torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=g)


def test_ws_decode_pass_beyond_2_32_work_items():
    """A MIME text of more than 2^36 bytes (76-character CRLF lines) at 256
    lanes x one 16-byte chunk: one workgroup per 4 KiB tile would put more
    than 2^32 work-items (more than one launch takes) into the decode pass,
    so it runs as two launches over the tiles. Every decoded byte equals the
    payload (generated on the device chunk by chunk); lines at the start,
    middle and end decode as the oracle decodes them; an invalid byte in
    the second launch's tiles is reported at its index."""
    LINE, PL = 78, 57                     # characters per line, payload bytes per line
    L = (1 << 36) // LINE + 4096          # lines
    nw, n = LINE * L, PL * L
    torch.cuda.empty_cache()
    if torch.cuda.mem_get_info()[0] < nw + n + (8 << 30):
        pytest.skip("needs about 120 GiB of free device memory")
    K = 1 << 24                           # lines per chunk
    wrapped = torch.empty(nw, dtype=torch.uint8, device=DEV)
    w2 = wrapped.view(L, LINE)
    for c, l0 in enumerate(range(0, L, K)):
        k = min(K, L - l0)
        w2[l0:l0 + k, :76] = codec.encode(_chunk_payload(c, PL * k)).view(k, 76)
    w2[:, 76] = 13
    w2[:, 77] = 10
    try:
        codec.set_ws_tune(256, 1)
        out, err = codec.decode_ws(wrapped)
        assert err == -1 and out.numel() == n
        for c, l0 in enumerate(range(0, L, K)):
            k = min(K, L - l0)
            assert torch.equal(out[PL * l0:PL * (l0 + k)], _chunk_payload(c, PL * k)), c
        for line in (0, L // 2, L - 3):
            want = oracle.decode_ws(wrapped[LINE * line:LINE * (line + 3)].cpu().numpy())
            assert want[:2] == (3 * PL, -1)
            assert np.array_equal(out[PL * line:PL * (line + 3)].cpu().numpy(), want[2])
        del out
        p = LINE * (L - 13) + 5           # a symbol in a tile past the first launch's
        assert p // 4096 >= ((1 << 32) - 1) // 256
        wrapped[p] = ord("*")
        want = oracle.decode_ws(wrapped[LINE * (L - 14):LINE * (L - 11)].cpu().numpy())
        assert want[:2] == (-1, p - LINE * (L - 14))
        out, err = codec.decode_ws(wrapped)
        assert out is None and err == p
    finally:
        del wrapped, w2
        torch.cuda.empty_cache()
