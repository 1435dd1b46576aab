"""Exact planted (l, d) motif search (Skip-Brute-Force) on AMD Instinct MI355X.

The search runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/pms.h`` (``libpms.so``, built in-tree by ``build.py``).  The Python
side only marshals arguments: see ``native`` for the binding and ``serve`` for
the continuous-batching request server.  Nothing here falls back to a CPU
path; importing ``native`` without the built library raises.
"""
import importlib

__all__ = ["native"]


def __getattr__(name):
    if name in ("native", "serve", "benchmarks"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
