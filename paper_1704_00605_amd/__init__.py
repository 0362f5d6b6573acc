"""b64hip: base64 encoding and validating decoding on AMD MI355X (gfx950).

A from-scratch GPU implementation of the method of Muła & Lemire, "Faster
Base64 Encoding and Decoding using AVX2 Instructions" (arXiv 1704.00605):
Algorithm 1 encoding and validating Algorithm 2 decoding (Section 2), single
buffer and batched, behind the C ABI of ``include/b64.h``.

Submodules are imported lazily so that the input generators
(``workloads``) can be used without loading the GPU library.
"""
import importlib

__all__ = ["codec", "workloads", "build"]


def __getattr__(name):
    if name in ("codec", "workloads", "build", "_lib", "graph", "autotune", "serve", "pool"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
