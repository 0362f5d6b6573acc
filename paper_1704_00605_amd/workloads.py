"""Seeded synthetic workloads (input generators only).

This module is shared by the tests, the benchmark and the oracle-side checks.
It holds no codec arithmetic: it draws random payload bytes, message lengths,
alphabet flags, arrival times and corruption choices with numpy's PCG64, in a
fixed order per workload, and it can overwrite one byte of a text buffer.

Workload recipes (payloads are uniform random bytes, as in the paper's
random-input experiment of Section 5):

* ``single(n, seed)``: one buffer of ``n`` bytes (1 MiB, seed 0; 1 GiB, seed 1).
* ``uneven(...)``: 100,000 messages, lengths log-uniform in [1, 65536], seed 2;
  1% of the decode inputs get one invalid byte.
* ``heavy_mix(...)``: 8,192 messages, seed 3: 819 lengths uniform in
  [1 MiB, 16 MiB] and 7,373 in [16 B, 4 KiB], shuffled; per-message alphabet
  flag (0 standard, 1 URL-safe); 0.5% of messages corrupted.
* ``serving_trace(...)``: Poisson arrivals at 200,000/s for 10 s, seed 4;
  50/50 encode/decode; sizes log-uniform in [64 B, 1 MiB]; 1% of decodes
  corrupted.

Log-uniform in [a, b] means ``clip(floor(exp(U(ln a, ln(b + 1)))), a, b)``.

Corruption draws a byte that is not one of the 64 symbols of the message's
alphabet (so '=' and the other alphabet's two extra symbols are candidates),
at a uniform position; when '=' would land on one of the last two positions
(where it can be legal padding) the next candidate is taken instead.
"""
import numpy as np

_LETTERS_DIGITS = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789"
_EXTRA = {0: b"+/", 1: b"-_"}


def non_symbols(alphabet):
    """The 192 byte values outside the 64 symbols of ``alphabet``, ascending."""
    sym = set(_LETTERS_DIGITS) | set(_EXTRA[alphabet])
    return np.array([b for b in range(256) if b not in sym], dtype=np.uint8)


_NON = {0: non_symbols(0), 1: non_symbols(1)}


def log_uniform(rng, count, a, b):
    u = rng.uniform(np.log(a), np.log(b + 1), size=count)
    return np.clip(np.floor(np.exp(u)), a, b).astype(np.int64)


def random_bytes(rng, n):
    return rng.integers(0, 256, size=n, dtype=np.uint8)


def offsets(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def corruption_byte(rank, alphabet, pos, m):
    """The injected byte for a uniform draw ``rank`` in [0, 192)."""
    cands = _NON[int(alphabet)]
    b = cands[int(rank) % cands.size]
    if b == ord("=") and pos >= m - 2:
        b = cands[(int(rank) + 1) % cands.size]
    return int(b)


def corrupt_text(text, text_off, msg_ids, u, ranks, flags=None):
    """Overwrite one byte in each listed message of a packed text buffer.

    ``text`` is a host uint8 array (modified in place), ``text_off`` the int64
    offsets of the messages in it, ``u`` uniform draws in [0, 1) for the
    position and ``ranks`` draws in [0, 192) for the byte. Returns the list of
    (message, position within the message, byte) applied; messages of length
    0 are skipped."""
    applied = []
    for j, m_id in enumerate(msg_ids):
        m_id = int(m_id)
        lo, hi = int(text_off[m_id]), int(text_off[m_id + 1])
        m = hi - lo
        if m == 0:
            continue
        pos = min(int(np.floor(u[j] * m)), m - 1)
        alph = 0 if flags is None else int(flags[m_id])
        b = corruption_byte(ranks[j], alph, pos, m)
        text[lo + pos] = b
        applied.append((m_id, pos, b))
    return applied


def single(n, seed):
    """Config of one buffer: payload, and a (u, rank) draw for the injected
    byte at a uniform position of the encoded text."""
    rng = np.random.default_rng(seed)
    x = random_bytes(rng, n)
    u = float(rng.uniform())
    rank = int(rng.integers(0, 192))
    return {"payload": x, "alphabet": 0, "corrupt_u": u, "corrupt_rank": rank}


def single_at_fraction(n, seed, frac):
    """One buffer whose injected byte sits at ``floor(frac * m)``."""
    w = single(n, seed)
    w["corrupt_u"] = frac
    return w


def uneven(count=100_000, lo=1, hi=65536, seed=2, corrupt_frac=0.01):
    rng = np.random.default_rng(seed)
    lens = log_uniform(rng, count, lo, hi)
    off = offsets(lens)
    payload = random_bytes(rng, int(off[-1]))
    k = int(round(corrupt_frac * count))
    ids = np.sort(rng.choice(count, size=k, replace=False))
    u = rng.uniform(size=k)
    ranks = rng.integers(0, 192, size=k)
    return {"payload": payload, "in_off": off, "flags": np.zeros(count, np.uint8),
            "corrupt_ids": ids, "corrupt_u": u, "corrupt_rank": ranks}


def heavy_mix(count=8192, n_large=819, large=(1 << 20, 16 << 20), small=(16, 4096), seed=3,
              corrupt_frac=0.005):
    rng = np.random.default_rng(seed)
    n_small = count - n_large
    big = rng.integers(large[0], large[1] + 1, size=n_large)
    sml = rng.integers(small[0], small[1] + 1, size=n_small)
    lens = np.concatenate([big, sml]).astype(np.int64)
    rng.shuffle(lens)
    flags = rng.integers(0, 2, size=count).astype(np.uint8)
    off = offsets(lens)
    payload = random_bytes(rng, int(off[-1]))
    k = int(round(corrupt_frac * count))
    ids = np.sort(rng.choice(count, size=k, replace=False))
    u = rng.uniform(size=k)
    ranks = rng.integers(0, 192, size=k)
    return {"payload": payload, "in_off": off, "flags": flags,
            "corrupt_ids": ids, "corrupt_u": u, "corrupt_rank": ranks}


def serving_trace(rate=200_000.0, seconds=10.0, lo=64, hi=1 << 20, seed=4, corrupt_frac=0.01):
    """Arrival times (s), op (0 encode, 1 decode), payload sizes (bytes of the
    raw message), and corruption draws for decode requests."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 16)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    n = t.size
    op = rng.integers(0, 2, size=n).astype(np.uint8)
    size = log_uniform(rng, n, lo, hi)
    corrupt = (rng.uniform(size=n) < corrupt_frac) & (op == 1)
    u = rng.uniform(size=n)
    ranks = rng.integers(0, 192, size=n)
    return {"t_arrival": t, "op": op, "size": size, "corrupt": corrupt,
            "corrupt_u": u, "corrupt_rank": ranks}


# ------------------------------------------------------ whitespace layouts --
# Text layouts for the whitespace-tolerant decode (Appendix B removes space,
# line feed and carriage return before decoding). These only move bytes
# around: a text is cut into lines, or whitespace bytes are inserted.
WS_BYTES = np.frombuffer(b" \n\r", dtype=np.uint8)


def wrap_lines(text, width=76, eol=b"\r\n"):
    """Text cut into lines of `width` characters, each followed by `eol`
    (MIME uses 76 and CRLF, PEM 64 and LF); the last line may be shorter and
    also ends with `eol`. Returns (wrapped, original index of every kept
    character)."""
    text = np.asarray(text, dtype=np.uint8)
    eol = np.frombuffer(eol, dtype=np.uint8)
    m = text.size
    lines = -(-m // width)
    e = eol.size
    out = np.empty(m + lines * e, dtype=np.uint8)
    idx = np.arange(m, dtype=np.int64)
    pos = idx + (idx // width) * e
    out[pos] = text
    ends = np.minimum((np.arange(lines, dtype=np.int64) + 1) * width, m)
    starts = ends + np.arange(lines, dtype=np.int64) * e
    for j in range(e):
        out[starts + j] = eol[j]
    return out, pos


def sprinkle_ws(rng, text, density, run_max=3):
    """Inserts, before each character independently with probability
    `density`, a run of 1..run_max whitespace bytes drawn from WS_BYTES.
    Returns (new text, new index of every original character)."""
    text = np.asarray(text, dtype=np.uint8)
    m = text.size
    runs = np.where(rng.uniform(size=m) < density, rng.integers(1, run_max + 1, m), 0).astype(np.int64)
    pos = np.arange(m, dtype=np.int64) + np.cumsum(runs)
    total = m + int(runs.sum())
    out = WS_BYTES[rng.integers(0, 3, total)]
    out[pos] = text
    return out, pos


def mime_1gib(seed=5):
    """Whitespace workload: 1 GiB of uniform random bytes (seed 5) whose
    base64 text is cut into 76-character CRLF lines (MIME)."""
    rng = np.random.default_rng(seed)
    return {"payload": random_bytes(rng, 1 << 30), "width": 76, "eol": b"\r\n",
            "corrupt_u": float(rng.uniform()), "corrupt_rank": int(rng.integers(0, 192))}


# ---------------------------------------------------------- file sizes --
# Base64 text sizes of the six files of the paper's decoding table (Section
# 5, Table 7: three JPEG images, a text quote, two PNG images). The files are
# not available; uniform random payloads stand in for them. A padded text has
# a length divisible by 4, so 2,357 and 1,355 round down to 2,356 and 1,352.
TABLE7_SIZES = (("lena [jpg]", 141_020), ("peppers [jpg]", 12_640), ("mandril [jpg]", 329_632),
                ("Moby Dick [text]", 1_484), ("google logo [png]", 2_357), ("bing social icons [png]", 1_355))


def table7_files(seed=6):
    """[(name, stated size, payload)]: a payload of 3 * L / 4 - 1 random
    bytes encodes to a text of exactly L = 4 * floor(size / 4) characters
    ending in one '='."""
    rng = np.random.default_rng(seed)
    out = []
    for name, size in TABLE7_SIZES:
        L = size // 4 * 4
        out.append((name, size, random_bytes(rng, 3 * L // 4 - 1)))
    return out
