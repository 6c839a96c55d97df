"""CPU oracle for the batched sorted search -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the device library
and its Python binding) never imports, links or runs anything here, and this
package imports nothing from the product.

What it computes (plain definitions, each written out in ``oracle.c``):

* ``search_lt``: idx(x) = #{i : a[i] < x} - 1, the index of the largest table
  entry strictly less than the target (paper Sec. 1; strict "<" and -1 for
  "none").  Every search method of the library must return exactly this.
* ``search_le_clamped``: the paper's own convention (Sec. 3), the last index
  with a[i] <= x clamped to [0, n-1]; the library's SS_OPT_CONVENTION mode.
* ``interp_pairs``: bilinear interpolation of a material's value grid at each
  (rho, T) pair after the paired search, the step EOSPAC performs after it.
* ``check_bracket``: the per-target property a[i] < x <= a[i+1] (a[-1] = -inf,
  a[n] = +inf; NaN -> -1), which fixes idx uniquely and is O(1) per target.
* ``exponent_key`` / ``exponent_bins``: the exponent hash of Sec. 3.5 and the
  bin table indexed as in Eq. 3, in prefix-count form (see ``oracle.c``).
* ``log_hash_base`` / ``log_hash_key`` / ``log_hash_bins``: the logarithm hash
  of Sec. 3.4 (Eq. 1-3) in float64, keys clamped to [0, |H|-1], and its bin
  table in prefix-count form.
* ``mlp_forward`` (in ``learned.py``): the float64 forward pass of the
  1-32-32-1 ReLU position model of the learned index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# SS_ORACLE_LIB selects another build of oracle.c (the sanitizer build).
_LIB_PATH = os.environ.get("SS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (no fast-math, no flush-to-zero)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-shared", "-fPIC",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(outdir: str) -> str:
    """``oracle.c`` with AddressSanitizer and UndefinedBehaviorSanitizer
    (clang, so that one sanitizer runtime serves every instrumented
    library); load it by setting SS_ORACLE_LIB to the returned path."""
    os.makedirs(outdir, exist_ok=True)
    out = os.path.join(outdir, "liboracle.so")
    subprocess.check_call(
        ["/opt/rocm/llvm/bin/clang", "-O1", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-std=c11",
         "-D_GNU_SOURCE", "-fno-fast-math", "-shared", "-fPIC", "-pthread", "-o", out, _SRC,
         "-lm"])
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_default_threads.restype = ctypes.c_int
    D = ctypes.c_double
    lib.oracle_log_hash_base.argtypes = [D, D, I64]
    lib.oracle_log_hash_base.restype = D
    lib.oracle_log_hash_raw.argtypes = [D, D, D]
    lib.oracle_log_hash_raw.restype = I64
    lib.oracle_log_hash_keys.argtypes = [P, I64, D, D, I64, P]
    lib.oracle_log_hash_keys.restype = None
    lib.oracle_log_hash_bins.argtypes = [P, I64, I64, P]
    lib.oracle_log_hash_bins.restype = I64
    lib.oracle_interp_pairs.argtypes = [P, P, P, P, P, ctypes.c_int32, P, P, P, P, P]
    lib.oracle_interp_pairs.restype = None
    lib.oracle_search_le_clamped.argtypes = [P, I64, P, I64, P, ctypes.c_int]
    lib.oracle_search_le_clamped.restype = ctypes.c_int
    lib.oracle_search_lt.argtypes = [P, I64, P, I64, P, ctypes.c_int]
    lib.oracle_search_lt.restype = ctypes.c_int
    lib.oracle_search_lt_at.argtypes = [P, I64, P, P, I64, P, ctypes.c_int]
    lib.oracle_search_lt_at.restype = ctypes.c_int
    lib.oracle_search_lt_segments.argtypes = [P, P, P, P, ctypes.c_int32, P, ctypes.c_int]
    lib.oracle_search_lt_segments.restype = ctypes.c_int
    lib.oracle_check_bracket.argtypes = [P, I64, P, I64, P, ctypes.POINTER(I64), ctypes.c_int]
    lib.oracle_check_bracket.restype = I64
    lib.oracle_exponent_key.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.oracle_exponent_key.restype = I64
    lib.oracle_exponent_bins.argtypes = [P, I64, ctypes.c_int, P, I64, ctypes.POINTER(I64)]
    lib.oracle_exponent_bins.restype = I64
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return _load().oracle_default_threads()


def search_lt(table, targets, threads: int = 0, return_threads: bool = False):
    """idx[k] = #{i : table[i] < targets[k]} - 1, as int32."""
    lib = _load()
    a = _f64(table)
    x = _f64(targets)
    out = np.empty(x.shape[0], dtype=np.int32)
    used = lib.oracle_search_lt(_ptr(a), a.shape[0], _ptr(x), x.shape[0], _ptr(out), threads)
    return (out, used) if return_threads else out


def search_le_clamped(table, targets, threads: int = 0):
    """The paper's convention (Sec. 3): min(max(#{table <= x} - 1, 0), n - 1)
    as int32 (-1 for an empty table)."""
    lib = _load()
    a = _f64(table)
    x = _f64(targets)
    out = np.empty(x.shape[0], dtype=np.int32)
    lib.oracle_search_le_clamped(_ptr(a), a.shape[0], _ptr(x), x.shape[0], _ptr(out), threads)
    return out


def interp_pairs(rho_tables, rho_off, t_tables, t_off, pair_off, values, rho, temp):
    """Bilinear interpolation of each material's grid at its (rho, T) pairs
    after locating both cells (see ``oracle.c``); returns (f, scale)."""
    lib = _load()
    rt, tt, vals = _f64(rho_tables), _f64(t_tables), _f64(values)
    ro = np.ascontiguousarray(rho_off, dtype=np.int64)
    to = np.ascontiguousarray(t_off, dtype=np.int64)
    po = np.ascontiguousarray(pair_off, dtype=np.int64)
    r, t = _f64(rho), _f64(temp)
    M = ro.shape[0] - 1
    assert to.shape[0] == M + 1 and po.shape[0] == M + 1
    assert vals.shape[0] == int(np.sum(np.diff(ro) * np.diff(to)))
    out = np.empty(r.shape[0])
    scale = np.empty(r.shape[0])
    lib.oracle_interp_pairs(_ptr(rt), _ptr(ro), _ptr(tt), _ptr(to), _ptr(po), M, _ptr(vals),
                            _ptr(r), _ptr(t), _ptr(out), _ptr(scale))
    return out, scale


def search_lt_at(table, targets, positions, threads: int = 0):
    """The definition evaluated only at ``targets[positions]``."""
    lib = _load()
    a = _f64(table)
    x = _f64(targets)
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    if pos.size and (pos.min() < 0 or pos.max() >= x.shape[0]):
        raise IndexError("position out of range")
    out = np.empty(pos.shape[0], dtype=np.int32)
    lib.oracle_search_lt_at(_ptr(a), a.shape[0], _ptr(x), _ptr(pos), pos.shape[0], _ptr(out),
                            threads)
    return out


def search_lt_segments(tables, table_off, targets, query_off, threads: int = 0,
                       return_threads: bool = False):
    """Segment s searches tables[table_off[s]:table_off[s+1]] with its targets."""
    lib = _load()
    t = _f64(tables)
    toff = np.ascontiguousarray(table_off, dtype=np.int64)
    qoff = np.ascontiguousarray(query_off, dtype=np.int64)
    x = _f64(targets)
    nseg = toff.shape[0] - 1
    assert qoff.shape[0] == nseg + 1 and qoff[-1] == x.shape[0] and toff[-1] <= t.shape[0]
    out = np.empty(x.shape[0], dtype=np.int32)
    used = lib.oracle_search_lt_segments(_ptr(t), _ptr(toff), _ptr(x), _ptr(qoff), nseg,
                                         _ptr(out), threads)
    return (out, used) if return_threads else out


def check_bracket(table, targets, idx, threads: int = 0):
    """Returns (violations, first_bad_position or -1)."""
    lib = _load()
    a = _f64(table)
    x = _f64(targets)
    i = np.ascontiguousarray(idx, dtype=np.int32)
    assert i.shape[0] == x.shape[0]
    first = ctypes.c_int64(-1)
    bad = lib.oracle_check_bracket(_ptr(a), a.shape[0], _ptr(x), x.shape[0], _ptr(i),
                                   ctypes.byref(first), threads)
    if bad < 0:
        raise MemoryError("oracle_check_bracket")
    return int(bad), int(first.value)


def check_bracket_segments(tables, table_off, targets, query_off, idx, threads: int = 0):
    """Bracket check per segment; returns (violations, first_bad_position or -1)."""
    toff = np.asarray(table_off, dtype=np.int64)
    qoff = np.asarray(query_off, dtype=np.int64)
    bad_total, first_total = 0, -1
    for s in range(toff.shape[0] - 1):
        q0, q1 = int(qoff[s]), int(qoff[s + 1])
        if q1 <= q0:
            continue
        bad, first = check_bracket(tables[toff[s]:toff[s + 1]], targets[q0:q1], idx[q0:q1],
                                   threads)
        bad_total += bad
        if first >= 0 and first_total < 0:
            first_total = q0 + first
    return bad_total, first_total


def exponent_key(v: float, s: int) -> int:
    """Exponent-hash key of a non-negative double with s sub-bin bits."""
    return int(_load().oracle_exponent_key(float(v), int(s)))


def log_hash_base(xmin: float, xmax: float, H: int) -> float:
    """Eq. 1: b = 10^((log10 Xmax - log10 Xmin) / |H|)."""
    lib = _load()
    return float(lib.oracle_log_hash_base(float(xmin), float(xmax), int(H)))


def log_hash_raw(x: float, xmin: float, base: float) -> int:
    """Eq. 2 before clamping: floor(log_b x) - floor(log_b Xmin)."""
    return int(_load().oracle_log_hash_raw(float(x), float(xmin), float(base)))


def log_hash_key(x, xmin: float, xmax: float, H: int):
    """Eq. 2 clamped to [0, H-1] (x <= 0 and NaN: 0), for an array of x."""
    lib = _load()
    xv = _f64(np.atleast_1d(np.asarray(x, dtype=np.float64)))
    out = np.empty(xv.shape[0], dtype=np.int64)
    base = log_hash_base(xmin, xmax, H)
    lib.oracle_log_hash_keys(_ptr(xv), xv.shape[0], float(xmin), base, int(H), _ptr(out))
    return out


def log_hash_bins(table, H: int):
    """C with C[i] = #{j : hash(table[j]) < i}, i = 0..H (Eq. 3, prefix form)."""
    lib = _load()
    a = _f64(table)
    C = np.empty(int(H) + 1, dtype=np.int64)
    r = lib.oracle_log_hash_bins(_ptr(a), a.shape[0], int(H), _ptr(C))
    if r < 0:
        raise ValueError("log hash needs 0 < a[0] < a[n-1] < inf and H >= 1")
    return C


def exponent_bins(table, s: int, cap: int = 1 << 22):
    """(kmin, C) with C[b] = #{i : key(table[i]) - kmin < b}, b = 0..nb."""
    lib = _load()
    a = _f64(table)
    C = np.empty(cap, dtype=np.int64)
    kmin = ctypes.c_int64(0)
    nb = lib.oracle_exponent_bins(_ptr(a), a.shape[0], int(s), _ptr(C), cap, ctypes.byref(kmin))
    if nb < 0:
        raise ValueError("bin table unavailable (empty table or more than cap bins)")
    return int(kmin.value), C[:nb + 1].copy()
