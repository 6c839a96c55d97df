"""MI355X-native batched search over small sorted float64 tables.

For each target x and a sorted table a[0..n), the library returns
idx(x) = #{i : a[i] < x} - 1 (the index of the largest entry below x, -1 if
none), computed by hand-written gfx950 HIP kernels behind the C ABI in
``include/searchsorted.h``.  ``binding`` holds the Python marshalling layer;
``inputs`` the seeded synthetic workloads.

The binding is imported lazily so that the input generators can be used on
machines without the HIP library.
"""
from __future__ import annotations

__all__ = ["binding", "inputs"]


def __getattr__(name):
    if name in ("binding", "inputs"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
