"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs a spread of inputs in a child process: every
one- and two-byte tail, random messages of every residue, corrupted and
padded texts, the strict, unpadded, whitespace and batched forms, and the
threaded wrappers. Any out-of-bounds access or undefined behaviour aborts
the child."""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle
from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    with oracle.using(SO):
        for v in range(256):
            for a in (0, 1):
                x = np.array([v], np.uint8)
                assert oracle.decode(oracle.encode(x, a), a)[2].tolist() == [v]
        rng = np.random.default_rng(0)
        for n in list(range(0, 80)) + [1000, 4097, 65537]:
            x = rng.integers(0, 256, n, dtype=np.uint8)
            for a in (0, 1):
                t = oracle.encode(x, a)
                assert oracle.decode(t, a)[2].tobytes() == x.tobytes()
                assert oracle.decode_nopad(oracle.encode_nopad(x, a), a)[2].tobytes() == x.tobytes()
                if t.size:
                    b = t.copy(); b[rng.integers(0, t.size)] = ord('*')
                    oracle.decode(b, a); oracle.decode_strict(b, a)
                    oracle.decode(t[:-1], a); oracle.decode_nopad(t[:-1], a)
                    ws = np.insert(t, rng.integers(0, t.size, 5), np.uint8(10))
                    assert oracle.decode_ws(ws, a)[2].tobytes() == x.tobytes()
        for junk in (b"", b"=", b"==", b"===", b"A=B=", b"Zg=", b"Zh==", b"Zg==Zg==", b"\\n\\n", b"\\xff\\x00"):
            j = np.frombuffer(junk, np.uint8).copy()
            oracle.decode(j); oracle.decode_strict(j); oracle.decode_nopad(j); oracle.decode_ws(j)
        lens = rng.integers(0, 300, 200)
        off = np.zeros(lens.size + 1, np.int64); np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, int(off[-1]), dtype=np.uint8)
        t, toff, _ = oracle.encode_batch(data, off)
        oracle.decode_batch(t, toff)
        big = rng.integers(0, 256, 3 << 20, dtype=np.uint8)
        bt = oracle.encode(big, threads=4)
        assert oracle.decode(bt, threads=4)[2].tobytes() == big.tobytes()
        assert oracle.decode(bt[:-3], threads=4)[:2] == oracle.decode(bt[:-3])[:2]
    print("sanitized oracle ok")
""")


@pytest.mark.skipif(_runtime("libasan.so") is None or _runtime("libubsan.so") is None,
                    reason="gcc sanitizer runtimes not installed")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    obuild.build(["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                  "-g", "-O1"], out=so)
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so") + ":" + _runtime("libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = f"ROOT = {ROOT!r}\nSO = {so!r}\n" + CHILD
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "sanitized oracle ok" in p.stdout
