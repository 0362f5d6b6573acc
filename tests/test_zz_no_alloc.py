"""The allocation-free batched decode (b64_decode_batch_noalloc) against the
workspace form (b64_decode_batch) it varies, through the C ABI: two calls in
a row on the library's static scratch array, the second with fewer messages,
each compared with the workspace form and with the oracle (lengths, error
offsets, decoded bytes). Sizes beyond the stated maximum are refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1704_00605_amd import _lib, codec, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).copy()).to(DEV)


def _batch(N, seed):
    rng = np.random.default_rng(seed)
    lens = workloads.log_uniform(rng, N, 1, 20_000)
    off = np.zeros(N + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    data = rng.integers(0, 256, int(off[-1]), dtype=np.uint8)
    flags = rng.integers(0, 2, N).astype(np.uint8)
    text, toff, _ = oracle.encode_batch(data, off, flags)
    ids = rng.choice(N, max(1, N // 50), replace=False)
    workloads.corrupt_text(text, toff, ids, rng.uniform(size=ids.size), rng.integers(0, 192, ids.size), flags)
    return text, toff, flags


def _run(fn, text, toff, flags, tune):
    src, in_off, fl = dev(text), dev(toff), dev(flags)
    N = toff.size - 1
    out_off = codec.batch_out_offsets(codec.DIR_DECODE, in_off, fl)
    dst = torch.full((int(out_off[-1].item()) + 1,), 0x77, dtype=torch.uint8, device=DEV)
    ol = torch.full((N,), -7, dtype=torch.int64, device=DEV)
    er = torch.full((N,), -7, dtype=torch.int64, device=DEV)
    fn(src, in_off, out_off, fl, dst, ol, er, tune)
    torch.cuda.synchronize()
    return dst.cpu().numpy(), out_off.cpu().numpy(), ol.cpu().numpy(), er.cpu().numpy()


def _noalloc(src, in_off, out_off, fl, dst, ol, er, tune):
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    t = None if tune is None else ctypes.byref(_lib.Tune(**tune))
    rc = _lib.lib().b64_decode_batch_noalloc(P(src), P(in_off), in_off.numel() - 1, P(dst), P(out_off), P(fl),
                                             P(ol), P(er), t, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, _lib.last_error()


def _with_workspace(src, in_off, out_off, fl, dst, ol, er, tune):
    codec.decode_batch(src, in_off, out_off, fl, dst, ol, er, tune=tune, validate=False)


@pytest.mark.parametrize("tune", [None, dict(block=128, units_per_lane=4, grid=4096, layout=1)])
def test_noalloc_decode_equals_workspace_form_two_calls(tune):
    for N, seed in ((40_000, 1), (3_001, 2)):  # the second call is smaller
        text, toff, flags = _batch(N, seed)
        got = _run(_noalloc, text, toff, flags, tune)
        ref = _run(_with_workspace, text, toff, flags, tune)
        wd, wo, wl, we = oracle.decode_batch(text, toff, flags)
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3]), N
        assert np.array_equal(got[2], wl) and np.array_equal(got[3], we), N
        assert (we >= 0).sum() >= N // 50
        oo = got[1]
        for i in np.nonzero(wl > 0)[0]:
            assert np.array_equal(got[0][oo[i]:oo[i] + wl[i]], ref[0][oo[i]:oo[i] + wl[i]]), (N, i)
            assert np.array_equal(got[0][oo[i]:oo[i] + wl[i]], wd[wo[i]:wo[i] + wl[i]]), (N, i)


def test_noalloc_at_its_maximum_batch():
    """Exactly the largest batch the call accepts (1,048,576 messages of 0-30
    characters of text, many of them invalid), against the workspace form
    and the oracle: every length, error offset and decoded byte."""
    N = _lib.NOALLOC_MAX_MESSAGES
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 31, N)
    toff = np.zeros(N + 1, np.int64)
    np.cumsum(lens, out=toff[1:])
    # random symbols: a message is invalid when its length is 1 mod 4 or its
    # last symbol leaves nonzero bits unused (most of the messages here)
    symbols = np.frombuffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/", np.uint8)
    text = symbols[rng.integers(0, 64, int(toff[-1]))]
    flags = np.zeros(N, np.uint8)
    got = _run(_noalloc, text, toff, flags, None)
    ref = _run(_with_workspace, text, toff, flags, None)
    wd, wo, wl, we = oracle.decode_batch(text, toff, flags)
    assert np.array_equal(got[2], wl) and np.array_equal(got[3], we)
    assert np.array_equal(ref[2], wl) and np.array_equal(ref[3], we)
    assert (we >= 0).sum() > N // 10 and (wl > 0).sum() > N // 10
    ok = wl > 0
    idx_got = np.repeat(got[1][:-1][ok] - np.concatenate([[0], np.cumsum(wl[ok])[:-1]]), wl[ok]) + \
        np.arange(wl[ok].sum())
    idx_want = np.repeat(wo[:-1][ok] - np.concatenate([[0], np.cumsum(wl[ok])[:-1]]), wl[ok]) + \
        np.arange(wl[ok].sum())
    assert np.array_equal(got[0][idx_got], wd[idx_want])
    assert np.array_equal(ref[0][idx_got], wd[idx_want])


def test_noalloc_refuses_batches_beyond_its_maximum():
    L = _lib.lib()
    N = _lib.NOALLOC_MAX_MESSAGES + 1
    rc = L.b64_decode_batch_noalloc(None, None, N, None, None, None, None, None, None, None)
    assert rc == _lib.BAD_ARG and "at most" in _lib.last_error()
    assert L.b64_decode_batch_noalloc(None, None, 0, None, None, None, None, None, None, None) == 0
