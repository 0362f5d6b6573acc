"""Character-map variants of the single-buffer kernels (LDS byte tables,
register maps on v_perm_b32 after Section 4's range offsets and Algorithm 3,
and the LDS pair table) against the oracle: every variant must give the
same bytes and the same verdicts."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import codec, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ENC_MAPS = [0, 1, 2]
DEC_MAPS = [0, 1]


@pytest.fixture(autouse=True)
def restore_defaults():
    yield
    codec.set_single_tune(0, 512, 2, -1, 0)
    codec.set_single_tune(1, 256, 2, -1, 0)


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a if a.flags.writeable else a.copy()).to(DEV)


@pytest.mark.parametrize("grid", [-1, 8])
@pytest.mark.parametrize("char_map", ENC_MAPS)
def test_encode_maps_match_oracle(char_map, grid):
    codec.set_single_tune(0, 256, 2, grid, char_map)
    rng = np.random.default_rng(char_map)
    for n in (1, 11, 12, 13, 777, 12 * 512 * 2 + 5, 1_000_003):
        x = rng.integers(0, 256, n, dtype=np.uint8)
        for alphabet in (0, 1):
            got = codec.encode(dev(x), alphabet).cpu().numpy()
            assert np.array_equal(got, oracle.encode(x, alphabet)), (n, alphabet)
    # unaligned source and destination
    x = rng.integers(0, 256, 100_001, dtype=np.uint8)
    buf = torch.zeros(x.size + 3, dtype=torch.uint8, device=DEV)
    buf[1:1 + x.size] = dev(x)
    out = torch.zeros(codec.encoded_len(x.size) + 2, dtype=torch.uint8, device=DEV)
    codec.encode(buf[1:1 + x.size], out=out[2:])
    assert np.array_equal(out[2:].cpu().numpy(), oracle.encode(x))


@pytest.mark.parametrize("char_map", ENC_MAPS)
def test_encode_maps_brute_force_triples(char_map):
    """All 2^24 three-byte groups (big-endian counter): quad i of the text is
    B(i>>18) B(i>>12&63) B(i>>6&63) B(i&63) (closed form, both alphabets)."""
    codec.set_single_tune(0, 0, 0, 0, char_map)
    i = np.arange(1 << 24, dtype=np.uint32)
    x = np.stack([(i >> 16) & 255, (i >> 8) & 255, i & 255], axis=1).astype(np.uint8).reshape(-1)
    for alphabet, sym in ((0, b"+/"), (1, b"-_")):
        B = np.frombuffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789" + sym, np.uint8)
        got = codec.encode(dev(x), alphabet).cpu().numpy().reshape(-1, 4)
        assert np.array_equal(got[:, 0], B[i >> 18]) and np.array_equal(got[:, 1], B[(i >> 12) & 63])
        assert np.array_equal(got[:, 2], B[(i >> 6) & 63]) and np.array_equal(got[:, 3], B[i & 63])


@pytest.mark.parametrize("char_map", DEC_MAPS)
def test_decode_maps_every_byte_value_everywhere(char_map):
    """Each of the 256 byte values at interior positions of every lane slot:
    valid symbols decode, everything else is rejected at its index."""
    codec.set_single_tune(1, 256, 2, 0, char_map)
    rng = np.random.default_rng(10 + char_map)
    base = oracle.encode(rng.integers(0, 256, 3 * 4096, dtype=np.uint8))
    m = base.size
    for alphabet in (0, 1):
        text = oracle.encode(oracle.decode(base)[2], alphabet)
        for v in range(256):
            pos = int(rng.integers(0, m - 64))
            t = text.copy()
            t[pos] = v
            want = oracle.decode(t, alphabet)
            out, err = codec.decode(dev(t), alphabet)
            got = (-1 if out is None else out.numel(), err)
            assert got == want[:2], (v, pos, alphabet)
            if out is not None:
                assert np.array_equal(out.cpu().numpy(), want[2])


@pytest.mark.parametrize("char_map", DEC_MAPS)
def test_decode_maps_random_sizes_modes_and_injected_errors(char_map):
    codec.set_single_tune(1, 512, 2, -1, char_map)
    rng = np.random.default_rng(20 + char_map)
    for n in (3, 4, 15, 16, 17, 1000, 16 * 1024 + 7, 900_001):
        x = rng.integers(0, 256, n, dtype=np.uint8)
        for alphabet, mode in ((0, 0), (1, 0), (0, 0x100), (1, 0x200)):
            t = oracle.encode_nopad(x, alphabet) if mode == 0x200 else oracle.encode(x, alphabet)
            out, err = codec.decode(dev(t), alphabet | mode)
            assert err == -1 and np.array_equal(out.cpu().numpy(), x), (n, alphabet, mode)
            if t.size > 8:
                j = int(rng.integers(0, t.size - 3))
                b = t.copy()
                b[j] = workloads.corruption_byte(int(rng.integers(0, 192)), alphabet, j, t.size)
                fn = oracle.decode_nopad if mode == 0x200 else (oracle.decode_strict if mode == 0x100 else oracle.decode)
                want = fn(b, alphabet)
                out, err = codec.decode(dev(b), alphabet | mode)
                assert ((-1 if out is None else out.numel()), err) == want[:2], (n, alphabet, mode, j)
