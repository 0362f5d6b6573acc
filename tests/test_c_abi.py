"""The C ABI from C: tests/c/b64_abi_client.c is compiled with gcc against
include/b64.h alone and linked to libb64hip.so. On the CPU it checks the
pure-host functions and argument errors; on the GPU it calls b64_encode and
b64_decode (the two calls of the paper's problem statement, Section 2,
Algorithms 1 and 2) on the NULL stream, and its outputs are compared with
the oracle's."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1704_00605_amd import _lib, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "b64_abi_client.c")
LIBDIR = os.path.dirname(_lib.LIB_PATH)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    exe = str(tmp_path_factory.mktemp("abi") / "b64_abi_client")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-isystem", os.path.join(ROCM, "include"), SRC,
           "-o", exe, "-L", LIBDIR, "-lb64hip", f"-Wl,-rpath,{LIBDIR}",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    subprocess.run(cmd, check=True)
    return exe


def test_header_compiles_as_c_and_host_calls_work(client):
    r = subprocess.run([client, "host"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "host checks: ok" in r.stdout


def _run_gpu(client, tmp_path, payload, pos, byte):
    p_in = tmp_path / "payload.bin"
    p_text = tmp_path / "text.bin"
    p_out = tmp_path / "bytes.bin"
    payload.tofile(p_in)
    print(f"C client: {payload.size} bytes, invalid byte {byte} at {pos}", flush=True)
    r = subprocess.run([client, "gpu", str(p_in), str(p_text), str(p_out), str(pos), str(byte)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    kv = dict(tok.split("=") for tok in r.stdout.split())
    return ({k: int(v) for k, v in kv.items()}, np.fromfile(p_text, np.uint8), np.fromfile(p_out, np.uint8))


@pytest.mark.gpu
def test_c_client_encode_decode_against_oracle(client, tmp_path):
    """1 MiB of seed-0 bytes: b64_encode's text and length, b64_decode's
    bytes, length and -1, and for the copy with a byte outside the alphabet
    at a seeded position, B64_INVALID_INPUT with that offset; all equal to the
    oracle. Also a payload whose text has a padded ending and a tiny one."""
    w = workloads.single(1 << 20, seed=0)
    x = w["payload"]
    want_t = oracle.encode(x)
    m = want_t.size
    pos = min(int(np.floor(w["corrupt_u"] * m)), m - 1)
    byte = workloads.corruption_byte(w["corrupt_rank"], 0, pos, m)
    for payload, p, b in [(x, pos, byte), (x[:1000], 1001, ord("*")), (x[:1], 0, ord("\n"))]:
        want_t = oracle.encode(payload)
        wl, we, wb = oracle.decode(want_t)
        bad = want_t.copy()
        if p < bad.size:
            bad[p] = b
        ob = oracle.decode(bad)
        kv, text, got = _run_gpu(client, tmp_path, payload, p, b)
        assert kv["enc_len"] == want_t.size and np.array_equal(text, want_t)
        assert (kv["dec_len"], kv["dec_err"]) == (wl, we) and np.array_equal(got, wb)
        assert (kv["bad_len"], kv["bad_err"]) == ob[:2]
        if p < bad.size:
            assert ob[:2] == (-1, p)
