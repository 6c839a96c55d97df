"""Seeded synthetic workloads for the batched sorted search.

The paper searches the density axis of one SESAME material (Sec. 4: 111
values, 0 to 5.4e4 g/cc, of which the positive part spans 3e-6 .. 5.4e4) with
5e6 targets drawn over 1e-10 .. 1e10.  That table is not available here, so
every workload is synthetic, with the same structure: small, sorted,
log-distributed float64 tables and many more targets than table entries.

This module holds no part of the search method.  It draws numbers (through
the counter-based generator in ``csrc/inputs.c``) and lays them out; the
device library and the CPU oracle both consume the same bytes.

Recipes (log-uniform on [lo, hi] means 10^(log10 lo + u (log10 hi - log10 lo))
with u uniform on [0, 1)):

* paper shape: n = 110 log-spaced entries on [3e-6, 5.4e4] with 10% jitter;
  targets log-uniform on [1e-10, 1e10] (about half fall outside the table).
* ``single64``: n = 64, a_i = 10^(-6 + 10 i / 63) (1 + 0.1 (2 u_i - 1)), sorted;
  1e6 targets log-uniform on [0.5 a_0, 2 a_63].
* ``single``: n in {100, 300, 1000} sorted i.i.d. log-uniform draws on
  [1e-8, 1e6] with both ends pinned; 1e8 targets, either i.i.d. log-uniform on
  [0.5e-8, 2e6] ("random") or a sorted random walk in log space ("smooth").
* ``batched``: 512 tables, n_t uniform on {20..2000}, each on [10^p, 10^q]
  with p < q uniform on (-10, 8) and q - p >= 1; query counts round(10^U(4,7)).
* ``learned``: n = 2000 sorted log-uniform draws on [1e-8, 1e6]; 1e8 targets.
* ``paired``: 4096 materials with a density table (n uniform on {50..4000})
  and a temperature table (n uniform on {20..1000}), ranges as for
  ``batched``; pair counts proportional to 10^U(0,3), summing to 1e9.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SS_INPUTS_LIB selects another build of the generators (the sanitizer build).
_LIB_PATH = os.environ.get("SS_INPUTS_LIB") or os.path.join(_HERE, "_lib", "libssinputs.so")
_lib = None

# stream ids (one independent counter stream per use)
S_TABLE, S_TARGETS, S_WALK, S_SIZES, S_RANGES, S_COUNTS, S_SEGMENTS = 1, 2, 3, 4, 5, 6, 7
S_TABLE2, S_SEGMENTS2 = 8, 9


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import _build
        _build.build_inputs()
    lib = ctypes.CDLL(_LIB_PATH)
    P, U64, I64, D, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.ssin_word.argtypes = [U64, U64, U64]
    lib.ssin_word.restype = U64
    lib.ssin_u01.argtypes = [U64, U64, U64]
    lib.ssin_u01.restype = D
    lib.ssin_uniform.argtypes = [U64, U64, U64, I64, P, I]
    lib.ssin_log_uniform.argtypes = [U64, U64, U64, D, D, I64, P, I]
    lib.ssin_sorted_log_table.argtypes = [U64, U64, I64, D, D, I, P]
    lib.ssin_jittered_log_table.argtypes = [U64, U64, I64, D, D, D, P]
    lib.ssin_smooth_walk.argtypes = [U64, U64, D, D, I64, P, I]
    lib.ssin_smooth_walk.restype = I
    lib.ssin_log_uniform_segments.argtypes = [U64, U64, P, P, P, ctypes.c_int32, P, I]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _out(count: int, out: np.ndarray | None) -> np.ndarray:
    if out is None:
        return np.empty(count, dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape[0] >= count
    return out


def uniform(seed: int, stream: int, count: int, k0: int = 0, threads: int = 0, out=None):
    o = _out(count, out)
    _load().ssin_uniform(seed, stream, k0, count, _ptr(o), threads)
    return o[:count]


def log_uniform(seed: int, stream: int, lo: float, hi: float, count: int, k0: int = 0,
                threads: int = 0, out=None):
    o = _out(count, out)
    _load().ssin_log_uniform(seed, stream, k0, lo, hi, count, _ptr(o), threads)
    return o[:count]


def sorted_log_table(seed: int, n: int, lo: float, hi: float, pin_ends: bool = True,
                     stream: int = S_TABLE):
    o = np.empty(n, dtype=np.float64)
    _load().ssin_sorted_log_table(seed, stream, n, lo, hi, int(pin_ends), _ptr(o))
    return o


def jittered_log_table(seed: int, n: int, e0: float, e1: float, jitter: float,
                       stream: int = S_TABLE):
    o = np.empty(n, dtype=np.float64)
    _load().ssin_jittered_log_table(seed, stream, n, e0, e1, jitter, _ptr(o))
    return o


def smooth_walk(seed: int, lo: float, hi: float, m: int, threads: int = 0, out=None,
                stream: int = S_WALK):
    o = _out(m, out)
    if _load().ssin_smooth_walk(seed, stream, lo, hi, m, _ptr(o), threads) != 0:
        raise MemoryError("smooth_walk")
    return o[:m]


def log_uniform_segments(seed: int, stream: int, off, lo, hi, threads: int = 0, out=None):
    off = np.ascontiguousarray(off, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    nseg = off.shape[0] - 1
    o = _out(int(off[-1]), out)
    _load().ssin_log_uniform_segments(seed, stream, _ptr(off), _ptr(lo), _ptr(hi), nseg, _ptr(o),
                                      threads)
    return o[:int(off[-1])]


# ---------------------------------------------------------------------------
# workload recipes
# ---------------------------------------------------------------------------

def paper_shape_table(seed: int = 110):
    """Stand-in for the searched density axis: 110 entries on [3e-6, 5.4e4]."""
    t = jittered_log_table(seed, 110, np.log10(3e-6), np.log10(5.4e4), 0.1)
    t[0], t[-1] = 3e-6, 5.4e4
    t.sort()
    return t


def paper_shape_targets(m: int, seed: int = 5, threads: int = 0, out=None):
    """The paper's targets for that table: i.i.d. log-uniform on [1e-10, 1e10],
    so that about half fall outside [3e-6, 5.4e4]."""
    return log_uniform(seed, S_TARGETS, 1e-10, 1e10, m, threads=threads, out=out)


def single64_table(seed: int = 64):
    return jittered_log_table(seed, 64, -6.0, 4.0, 0.1)


def single_table(n: int, seed: int = 1000):
    return sorted_log_table(seed + n, n, 1e-8, 1e6, pin_ends=True)


def table_targets(table: np.ndarray, m: int, seed: int, kind: str = "random", threads: int = 0,
                  out=None):
    """Targets over [0.5 a_0, 2 a_{n-1}], i.i.d. log-uniform or a smooth walk."""
    lo, hi = 0.5 * float(table[0]), 2.0 * float(table[-1])
    if kind == "random":
        return log_uniform(seed, S_TARGETS, lo, hi, m, threads=threads, out=out)
    if kind == "smooth":
        return smooth_walk(seed, lo, hi, m, threads=threads, out=out)
    raise ValueError(kind)


def _ranges(seed: int, stream: int, count: int):
    """(p, q) per table: uniform on (-10, 8), p < q, redrawn until q - p >= 1."""
    lib = _load()
    p = np.empty(count)
    q = np.empty(count)
    for t in range(count):
        k = 0
        while True:
            a = -10.0 + 18.0 * lib.ssin_u01(seed, stream, (t << 20) + k)
            b = -10.0 + 18.0 * lib.ssin_u01(seed, stream, (t << 20) + k + 1)
            k += 2
            lo_e, hi_e = min(a, b), max(a, b)
            if hi_e - lo_e >= 1.0:
                break
        p[t], q[t] = lo_e, hi_e
    return p, q


def _int_uniform(seed: int, stream: int, count: int, lo: int, hi: int):
    """Integers uniform on {lo..hi}."""
    u = uniform(seed, stream, count, threads=1)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


@dataclass
class Batch:
    """CSR layout of many tables and their target segments."""
    tables: np.ndarray          # float64, all tables back to back
    table_off: np.ndarray       # int64 [T+1]
    query_off: np.ndarray       # int64 [T+1]
    lo: np.ndarray = field(default=None)
    hi: np.ndarray = field(default=None)

    @property
    def num_tables(self) -> int:
        return self.table_off.shape[0] - 1

    @property
    def num_queries(self) -> int:
        return int(self.query_off[-1])

    def table(self, t: int) -> np.ndarray:
        return self.tables[self.table_off[t]:self.table_off[t + 1]]


def _tables_from(seed: int, sizes, p, q, stream: int):
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    tabs = np.empty(int(off[-1]), dtype=np.float64)
    for t, n in enumerate(sizes):
        tabs[off[t]:off[t + 1]] = sorted_log_table(seed * 7919 + t, int(n), 10.0 ** p[t],
                                                   10.0 ** q[t], pin_ends=True, stream=stream)
    return tabs, off


def batched_layout(seed: int = 512, num_tables: int = 512, nmin: int = 20, nmax: int = 2000,
                   qexp=(4.0, 7.0), query_scale: float = 1.0) -> Batch:
    sizes = _int_uniform(seed, S_SIZES, num_tables, nmin, nmax)
    p, q = _ranges(seed, S_RANGES, num_tables)
    tabs, toff = _tables_from(seed, sizes, p, q, S_TABLE)
    u = uniform(seed, S_COUNTS, num_tables, threads=1)
    counts = np.rint(10.0 ** (qexp[0] + (qexp[1] - qexp[0]) * u) * query_scale).astype(np.int64)
    qoff = np.zeros(num_tables + 1, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    lo = np.array([0.5 * tabs[toff[t]] for t in range(num_tables)])
    hi = np.array([2.0 * tabs[toff[t + 1] - 1] for t in range(num_tables)])
    return Batch(tabs, toff, qoff, lo, hi)


def batched_targets(batch: Batch, seed: int = 512, threads: int = 0, out=None,
                    stream: int = S_SEGMENTS):
    return log_uniform_segments(seed, stream, batch.query_off, batch.lo, batch.hi,
                                threads=threads, out=out)


def batched_smooth_targets(batch: Batch, seed: int = 513, threads: int = 0, out=None):
    """Each table's targets as one smooth increasing walk over its range (the
    single-table "smooth" order, per segment): targets that arrive sorted."""
    o = _out(batch.num_queries, out)
    for t in range(batch.num_tables):
        a, b = int(batch.query_off[t]), int(batch.query_off[t + 1])
        if b > a:
            smooth_walk(seed + t, float(batch.lo[t]), float(batch.hi[t]), b - a,
                        threads=threads, out=o[a:b])
    return o[:batch.num_queries]


def learned_table(seed: int = 2000, n: int = 2000):
    return sorted_log_table(seed, n, 1e-8, 1e6, pin_ends=True)


@dataclass
class Paired:
    rho: Batch
    temp: Batch

    @property
    def num_materials(self) -> int:
        return self.rho.num_tables

    @property
    def num_pairs(self) -> int:
        return self.rho.num_queries


def paired_layout(seed: int = 4096, materials: int = 4096, total_pairs: int = 10**9) -> Paired:
    n_rho = _int_uniform(seed, S_SIZES, materials, 50, 4000)
    n_t = _int_uniform(seed + 1, S_SIZES, materials, 20, 1000)
    pr, qr = _ranges(seed, S_RANGES, materials)
    pt, qt = _ranges(seed + 1, S_RANGES, materials)
    rtabs, roff = _tables_from(seed, n_rho, pr, qr, S_TABLE)
    ttabs, toff = _tables_from(seed + 1, n_t, pt, qt, S_TABLE2)
    w = 10.0 ** (3.0 * uniform(seed, S_COUNTS, materials, threads=1))
    share = w / w.sum() * total_pairs
    counts = np.floor(share).astype(np.int64)
    rem = int(total_pairs - counts.sum())
    if rem > 0:  # largest remainders first, ties by material id
        order = np.lexsort((np.arange(materials), -(share - counts)))
        counts[order[:rem]] += 1
    poff = np.zeros(materials + 1, dtype=np.int64)
    poff[1:] = np.cumsum(counts)
    rho = Batch(rtabs, roff, poff,
                np.array([0.5 * rtabs[roff[t]] for t in range(materials)]),
                np.array([2.0 * rtabs[roff[t + 1] - 1] for t in range(materials)]))
    temp = Batch(ttabs, toff, poff.copy(),
                 np.array([0.5 * ttabs[toff[t]] for t in range(materials)]),
                 np.array([2.0 * ttabs[toff[t + 1] - 1] for t in range(materials)]))
    return Paired(rho, temp)


@dataclass
class Interp:
    """Paired axes plus one value grid per material (row-major, density-major:
    values[voff[j] + a * n_t + b] is material j's value at (rho_a, T_b))."""
    pairs: Paired
    values: np.ndarray
    value_off: np.ndarray


def interp_layout(seed: int = 1024, materials: int = 1024, total_pairs: int = 10**9,
                  n_rho=(50, 150), n_t=(20, 100)) -> Interp:
    """Axes shaped like SESAME tables (about 100 x 60 points), the paired
    layout's ranges and pair counts, and a smooth synthetic value grid per
    material: f = c0 + c1 L + c2 M + c3 L M + 0.05 sin(7 L) with L = log10 rho,
    M = log10 T and coefficients drawn per material (numbers, not a method)."""
    base = paired_layout(seed=seed, materials=materials, total_pairs=total_pairs)
    nr = _int_uniform(seed, S_SIZES, materials, n_rho[0], n_rho[1])
    nt = _int_uniform(seed + 1, S_SIZES, materials, n_t[0], n_t[1])
    pr, qr = _ranges(seed, S_RANGES, materials)
    pt, qt = _ranges(seed + 1, S_RANGES, materials)
    rtabs, roff = _tables_from(seed, nr, pr, qr, S_TABLE)
    ttabs, toff = _tables_from(seed + 1, nt, pt, qt, S_TABLE2)
    for tabs, off in ((rtabs, roff), (ttabs, toff)):
        for j in range(materials):
            a = tabs[off[j]:off[j + 1]]
            assert np.all(a[1:] > a[:-1]), "axes must be strictly increasing"
    coef = uniform(seed, S_COUNTS + 10, 4 * materials, threads=1).reshape(materials, 4) * 2 - 1
    voff = np.zeros(materials + 1, dtype=np.int64)
    voff[1:] = np.cumsum(nr * nt)
    vals = np.empty(int(voff[-1]))
    for j in range(materials):
        L = np.log10(rtabs[roff[j]:roff[j + 1]])[:, None]
        Mv = np.log10(ttabs[toff[j]:toff[j + 1]])[None, :]
        c = coef[j]
        g = c[0] + c[1] * L + c[2] * Mv + c[3] * L * Mv + 0.05 * np.sin(7.0 * L)
        vals[voff[j]:voff[j + 1]] = g.reshape(-1)
    poff = base.rho.query_off
    rho = Batch(rtabs, roff, poff,
                np.array([0.5 * rtabs[roff[t]] for t in range(materials)]),
                np.array([2.0 * rtabs[roff[t + 1] - 1] for t in range(materials)]))
    temp = Batch(ttabs, toff, poff.copy(),
                 np.array([0.5 * ttabs[toff[t]] for t in range(materials)]),
                 np.array([2.0 * ttabs[toff[t + 1] - 1] for t in range(materials)]))
    return Interp(Paired(rho, temp), vals, voff)


def paired_targets(pairs: Paired, seed: int = 4096, threads: int = 0, out_rho=None, out_t=None):
    r = log_uniform_segments(seed, S_SEGMENTS, pairs.rho.query_off, pairs.rho.lo, pairs.rho.hi,
                             threads=threads, out=out_rho)
    t = log_uniform_segments(seed, S_SEGMENTS2, pairs.temp.query_off, pairs.temp.lo,
                             pairs.temp.hi, threads=threads, out=out_t)
    return r, t


def special_values():
    """Targets every implementation must handle exactly (see the contract)."""
    return np.array([
        np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308,
        2.2250738585072009e-308, 1e-300, 1.0, -1.0, 1.7976931348623157e308,
    ], dtype=np.float64)
