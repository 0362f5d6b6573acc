import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def golden_lines(name):
    """Non-comment, non-empty lines of a golden fixture."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.lstrip().startswith("#")]


def golden_kv(name):
    """``key: a, b, c`` lines -> {key: [tokens]} (repeated keys -> list of lists)."""
    out = {}
    for ln in golden_lines(name):
        k, _, v = ln.partition(":")
        toks = [t.strip() for t in v.replace(",", " ").split()]
        out.setdefault(k.strip(), []).append(toks)
    return out


def ints(tokens):
    return [int(t, 0) for t in tokens]


@pytest.fixture(scope="session")
def table1():
    """Table 1 as parsed from the fixture: list of (value, code, char)."""
    rows = []
    for ln in golden_lines("table1_alphabet.txt"):
        v, code, ch = ln.split()
        rows.append((int(v), int(code, 16), ch))
    return rows


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible in this process")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
