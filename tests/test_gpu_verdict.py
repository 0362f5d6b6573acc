"""One-launch verdicts of the single-buffer decode above the one-workgroup
size: the workgroup that finishes last forms (length, -1) or (-1, first
offending index) from a per-stream verdict cell and returns the cell to rest.
Every verdict and every decoded byte is compared with the oracle, over runs
of back-to-back calls on one stream (each call finds the cell at rest), on
several streams at once (one cell each), in several launch shapes (one-shot
and grid-stride grids), and under graph capture (no cell: two launches)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import codec, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
STD, URL, NOPAD = codec.ALPHABET_STD, codec.ALPHABET_URL, codec.MODE_NOPAD


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).copy()).to(DEV)


def _cases():
    """(name, text, alphabet): all above 2,048 interior units (32 KiB of
    text), so with a verdict cell none takes the one-workgroup kernel. Up to
    1 MiB of text the default shape's grid fits one workgroup per CU; 5 MiB
    takes the larger workgroups; 40 MiB is past the one-launch limit
    (32 MiB)."""
    rng = np.random.default_rng(77)
    x = rng.integers(0, 256, 1 << 20, dtype=np.uint8)
    t = oracle.encode(x)                                    # 1,398,104 characters
    multi = t.copy()
    for p in (17, t.size // 2 + 5, t.size - 3):             # first, middle and final units
        multi[p] = ord("*")
    late = t.copy()
    late[t.size - 1] = ord("#")                             # only the final unit is wrong
    mid = t.copy()
    mid[700_001] = workloads.corruption_byte(5, 0, 700_001, t.size)
    y = rng.integers(0, 256, 1_000_001, dtype=np.uint8)
    padded = oracle.encode(y)                               # ends in '=='
    short_len = padded[:262_165]                            # length 1 mod 4: error at n - 1 or earlier
    nopad = oracle.encode_nopad(y, URL)                     # 1,333,335 characters
    big = oracle.encode(rng.integers(0, 256, 5 * (1 << 20) + 7, dtype=np.uint8))
    # 40 MiB of text: beyond the one-launch grids, two launches on any stream
    huge = oracle.encode(rng.integers(0, 256, 30 * (1 << 20) + 2, dtype=np.uint8))
    huge[huge.size - 900_000] = ord("!")
    # 100,000 characters (6,249 interior units): one workgroup without a
    # cell, the multi-workgroup one-launch grid with one
    z = rng.integers(0, 256, 75_000, dtype=np.uint8)
    small = oracle.encode(z)
    small_bad = small.copy()
    small_bad[66_666] = ord("-")
    return [("valid_1MiB", t, STD), ("three_errors", multi, STD), ("final_unit_error", late, STD),
            ("one_error", mid, STD), ("padded", padded, STD), ("bad_length", short_len, STD),
            ("url_nopad", nopad, URL | NOPAD), ("valid_5MiB", big, STD), ("error_40MiB", huge, STD),
            ("valid_100k", small, STD), ("error_100k", small_bad, STD)]


CASES = _cases()
WANT = [oracle.decode_nopad(t, a & 0xff) if a & NOPAD else oracle.decode(t, a & 0xff) for _, t, a in CASES]
_TEXTS = []


def text(i):
    """Device copy of CASES[i]'s text (made on first use)."""
    if not _TEXTS:
        _TEXTS.extend(dev(t) for _, t, _a in CASES)
    return _TEXTS[i]

# (block, units per lane, blocks per CU; -1 = one workgroup per tile)
SHAPES = [(256, 2, -1), (64, 1, 1), (1024, 8, -1), (256, 4, 2), (512, 1, -1)]


@pytest.fixture
def restore_tune():
    yield
    codec.set_single_tune(1, 256, 2, -1, 0)


def _enqueue(order, stream):
    """Enqueues decode_async of CASES[i] for i in order on stream, each into
    its own output buffer and result slots; nothing waits in between."""
    jobs = []
    with torch.cuda.stream(stream):
        for i in order:
            _, t, a = CASES[i]
            out = torch.full((codec.decoded_max(t.size, a & ~0xff) + 16,), 0xEE, dtype=torch.uint8, device=DEV)
            res = torch.full((2,), 12345, dtype=torch.int64, device=DEV)
            codec.decode_async(text(i), out, res, a, stream=stream)
            jobs.append((i, out, res))
    return jobs


def _check(jobs):
    torch.cuda.synchronize()
    for i, out, res in jobs:
        name = CASES[i][0]
        want = WANT[i]
        assert tuple(res.cpu().tolist()) == want[:2], name
        if want[1] == -1:
            n = want[0]
            assert torch.equal(out[:n], dev(want[2])), name


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{b}x{u}_g{g}" for b, u, g in SHAPES])
def test_back_to_back_on_one_stream(shape, restore_tune):
    codec.set_single_tune(1, *shape, 0)
    s = torch.cuda.Stream()
    order = [0, 1, 0, 5, 2, 4, 1, 3, 8, 6, 7, 9, 10, 2, 8, 0, 10, 9]
    _check(_enqueue(order, s))
    # the synchronous call on the same stream shares its cell
    for i in (1, 0, 2):
        got, err = codec.decode(text(i), CASES[i][2], stream=s)
        assert ((-1 if got is None else got.numel()), err) == WANT[i][:2], CASES[i][0]


def test_several_streams_at_once():
    streams = [torch.cuda.Stream() for _ in range(4)]
    jobs = []
    for k in range(3):
        for j, s in enumerate(streams):
            jobs += _enqueue([(j + k + r) % len(CASES) for r in range(3)], s)
    _check(jobs)


def test_default_stream_and_sync_calls():
    jobs = _enqueue(list(range(len(CASES))), torch.cuda.default_stream())
    _check(jobs)
    for i in range(len(CASES)):
        got, err = codec.decode(text(i), CASES[i][2])
        assert ((-1 if got is None else got.numel()), err) == WANT[i][:2], CASES[i][0]


def test_captured_decode_replays():
    """A stream under capture gets no verdict cell; the captured two-launch
    decode is replayed with eager one-launch decodes between the replays."""
    i_bad, i_ok, i_sbad, i_sok = 1, 0, 10, 9
    out = torch.empty(codec.decoded_max(CASES[i_ok][1].size) + 16, dtype=torch.uint8, device=DEV)
    out_s = torch.empty(codec.decoded_max(CASES[i_sok][1].size) + 16, dtype=torch.uint8, device=DEV)
    res = torch.full((8,), 7, dtype=torch.int64, device=DEV)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            codec.decode_async(text(i_bad), out, res[2:4], stream=s)
            codec.decode_async(text(i_ok), out, res[0:2], stream=s)
            codec.decode_async(text(i_sbad), out_s, res[6:8], stream=s)
            codec.decode_async(text(i_sok), out_s, res[4:6], stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        res.fill_(7)
        out.fill_(0)
        out_s.fill_(0)
        g.replay()
        _check(_enqueue([r % len(CASES), 3, 10], torch.cuda.current_stream()))
        for i, k in ((i_ok, 0), (i_bad, 2), (i_sok, 4), (i_sbad, 6)):
            assert tuple(res[k:k + 2].cpu().tolist()) == WANT[i][:2], CASES[i][0]
        assert torch.equal(out[:WANT[i_ok][0]], dev(WANT[i_ok][2]))
        assert torch.equal(out_s[:WANT[i_sok][0]], dev(WANT[i_sok][2]))


def test_per_thread_default_stream_takes_no_cell():
    """The per-thread default stream is one handle for many streams, so it
    gets no verdict cell: its decodes take the two-launch path (and the
    one-workgroup kernel below 256 KiB). Every verdict is checked after a
    device-wide synchronisation."""
    import ctypes
    from paper_1704_00605_amd._lib import lib
    per_thread = ctypes.c_void_p(2)  # hipStreamPerThread
    torch.cuda.synchronize()
    jobs = []
    for i in (0, 1, 8, 9, 10, 5, 0):
        _, t, a = CASES[i]
        out = torch.empty(codec.decoded_max(t.size, a & ~0xff) + 16, dtype=torch.uint8, device=DEV)
        res = torch.full((2,), 12345, dtype=torch.int64, device=DEV)
        torch.cuda.synchronize()
        rp = res.data_ptr()
        rc = lib().b64_decode_async(ctypes.c_void_p(text(i).data_ptr()), t.size, ctypes.c_void_p(out.data_ptr()),
                                    int(a), ctypes.c_void_p(rp), ctypes.c_void_p(rp + 8), per_thread)
        assert rc == 0
        jobs.append((i, out, res))
    _check(jobs)
