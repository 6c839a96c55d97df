"""Thin ctypes binding over ``libsearchsorted.so`` (see include/searchsorted.h).

Argument marshalling only: tensors supply device pointers and sizes, torch's
current stream is handed to the library before each call, and every step of
the search runs in the library's HIP kernels.  There is no fallback: if the
library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SS_LIBRARY selects another build of the library (the sanitizer build).
LIB_PATH = os.environ.get("SS_LIBRARY") or os.path.join(_HERE, "_lib", "libsearchsorted.so")

SS_OK = 0
STATUS_NAMES = {
    -1: "SS_ERR_INVALID_ARG", -2: "SS_ERR_NOT_DEVICE_PTR", -3: "SS_ERR_NO_DEVICE",
    -4: "SS_ERR_HIP", -5: "SS_ERR_OOM", -6: "SS_ERR_UNSUPPORTED",
}

ALGO_AUTO, ALGO_BINARY, ALGO_BALLOT, ALGO_EXPHASH, ALGO_BINARY_GLOBAL = 0, 1, 2, 3, 4
ALGO_LEARNED, ALGO_LOGHASH, ALGO_SKIPLIST = 5, 6, 7
ALGO_NAMES = {ALGO_AUTO: "auto", ALGO_BINARY: "binary", ALGO_BALLOT: "ballot",
              ALGO_EXPHASH: "exphash", ALGO_BINARY_GLOBAL: "binary_global",
              ALGO_LEARNED: "learned", ALGO_LOGHASH: "loghash", ALGO_SKIPLIST: "skiplist"}
ALGO_IDS = {v: k for k, v in ALGO_NAMES.items()}

OPT_FORCE_ALGO, OPT_BUCKET_BITS, OPT_BUCKET_CAP = 1, 2, 3
OPT_BLOCK_SIZE, OPT_GRID_BLOCKS, OPT_CHECK_POINTERS = 4, 5, 6
OPT_TARGETS_PER_LANE = 7
OPT_PLAN_TILES, OPT_PLAN_LEARNED, OPT_LEARNED_STEPS, OPT_PLAN_XCD, OPT_PAIR_JOINT = 8, 9, 10, 11, 12
OPT_CONVENTION = 13
OPT_PLAN_ALGO = 14
OPT_PLAN_ORDER = 15
PLAN_LEARNED_TUNER, PLAN_LEARNED_ALL, PLAN_LEARNED_NONE = 0, 1, 2


class SearchSortedError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2112_03229_amd._build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    L.ss_last_error.restype = ctypes.c_char_p
    L.ss_version.restype = I
    L.ss_set_stream.argtypes = [P]
    L.ss_set_option.argtypes = [I, I64]
    L.ss_get_option.argtypes = [I, ctypes.POINTER(I64)]
    L.search_sorted_batch.argtypes = [P, I64, P, I64, P]
    L.ss_search_with.argtypes = [P, I64, P, I64, P, I, I]
    L.ss_validate_table.argtypes = [P, I64, ctypes.POINTER(I64)]
    L.ss_exphash_bins.argtypes = [P, I64, I, P, I64, ctypes.POINTER(I64)]
    for name in ("ss_set_stream", "ss_set_option", "ss_get_option", "search_sorted_batch",
                 "ss_search_with", "ss_validate_table", "ss_exphash_bins"):
        getattr(L, name).restype = I
    _register_extra(L)
    _lib = L
    return L


def _register_extra(L) -> None:
    """Signatures of the plan, paired and learned entry points (if present)."""
    P, I64, I32, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    sigs = {
        "ss_multi_plan_create": [P, P, I32, P, ctypes.POINTER(P)],
        "ss_multi_plan_create_learned": [P, P, I32, P, P, ctypes.POINTER(P)],
        "ss_multi_plan_create_sampled": [P, P, I32, P, P, ctypes.POINTER(P)],
        "ss_pair_plan_create_sampled": [P, P, P, P, I32, P, P, P, ctypes.POINTER(P)],
        "ss_multi_search": [P, P, P],
        "ss_plan_destroy": [P],
        "ss_plan_info": [P, I, P, I64],
        "ss_plan_fallbacks": [P, ctypes.POINTER(I64)],
        "ss_pair_plan_create": [P, P, P, P, I32, P, ctypes.POINTER(P)],
        "ss_pair_search": [P, P, P, P, P],
        "ss_tuner_calibrate": [],
        "ss_debug_violations": [ctypes.POINTER(I64)],
        "ss_debug_selftest": [],
        "ss_tuner_get": [P, I],
        "ss_tuner_set": [P, I],
        "ss_tuner_save": [ctypes.c_char_p],
        "ss_tuner_load": [ctypes.c_char_p],
        "ss_learned_build": [P, I64, P, ctypes.POINTER(P)],
        "ss_learned_from_weights": [P, I64, P, ctypes.POINTER(P)],
        "ss_learned_search": [P, P, I64, P],
        "ss_learned_info": [P, P, I],
        "ss_learned_fallbacks": [P, ctypes.POINTER(I64)],
        "ss_learned_error_bound": [P, ctypes.POINTER(I32)],
        "ss_learned_set_error_bound": [P, I32],
        "ss_learned_stats": [P, ctypes.POINTER(I64)],
        "ss_learned_predict": [P, P, I64, P],
        "ss_learned_weights": [P, P, I64],
        "ss_mlp_gradient": [P, I64, P, P, P],
        "ss_learned_destroy": [P],
        "ss_loghash_bins": [P, I64, I64, P, P],
        "ss_interp_plan_create": [P, P, P, P, I32, P, P, ctypes.POINTER(P)],
        "ss_interp_search": [P, P, P, P, P, P],
        "ss_multi_search_noalloc": [P, I64, P, I32, P, P, I64, P],
        "ss_plan_save": [P, ctypes.c_char_p],
        "ss_multi_plan_load": [ctypes.c_char_p, P, P, I32, P, ctypes.POINTER(P)],
        "ss_pair_plan_load": [ctypes.c_char_p, P, P, P, P, I32, P, ctypes.POINTER(P)],
        "ss_learned_save": [P, ctypes.c_char_p],
        "ss_learned_load": [P, I64, ctypes.c_char_p, ctypes.POINTER(P)],
    }
    for name, argtypes in sigs.items():
        fn = getattr(L, name, None)
        if fn is not None:
            fn.argtypes = argtypes
            fn.restype = I


def check(rc: int) -> None:
    if rc != SS_OK:
        raise SearchSortedError(rc, lib().ss_last_error().decode(errors="replace"))


def use_current_stream() -> None:
    """Routes subsequent library calls to torch's current stream."""
    lib().ss_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _need(t: torch.Tensor, dtype: torch.dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.numel() and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def set_option(opt: int, value: int) -> None:
    check(lib().ss_set_option(opt, value))


def get_option(opt: int) -> int:
    v = ctypes.c_int64()
    check(lib().ss_get_option(opt, ctypes.byref(v)))
    return v.value


def search_sorted_batch(table: torch.Tensor, targets: torch.Tensor,
                        out: torch.Tensor | None = None) -> torch.Tensor:
    """idx[k] = #{i : table[i] < targets[k]} - 1 (int32), on the GPU."""
    _need(table, torch.float64, "table")
    _need(targets, torch.float64, "targets")
    if out is None:
        out = torch.empty(targets.numel(), dtype=torch.int32, device=targets.device)
    _need(out, torch.int32, "out")
    if out.numel() != targets.numel():
        raise ValueError("out must have one entry per target")
    use_current_stream()
    check(lib().search_sorted_batch(_ptr(table), table.numel(), _ptr(targets), targets.numel(),
                                    _ptr(out)))
    return out


searchsorted_lt = search_sorted_batch


def search_with(table: torch.Tensor, targets: torch.Tensor, algo, bucket_bits: int = -1,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """search_sorted_batch with an explicit kernel ("binary", "ballot", "exphash", ...)."""
    if isinstance(algo, str):
        algo = ALGO_IDS[algo]
    _need(table, torch.float64, "table")
    _need(targets, torch.float64, "targets")
    if out is None:
        out = torch.empty(targets.numel(), dtype=torch.int32, device=targets.device)
    _need(out, torch.int32, "out")
    if out.numel() != targets.numel():
        raise ValueError("out must have one entry per target")
    use_current_stream()
    check(lib().ss_search_with(_ptr(table), table.numel(), _ptr(targets), targets.numel(),
                               _ptr(out), int(algo), int(bucket_bits)))
    return out


def validate_table(table: torch.Tensor) -> int:
    """-1 if sorted without NaN, else the first offending index (synchronous)."""
    _need(table, torch.float64, "table")
    bad = ctypes.c_int64()
    use_current_stream()
    check(lib().ss_validate_table(_ptr(table), table.numel(), ctypes.byref(bad)))
    return bad.value


def exphash_bins(table: torch.Tensor, bucket_bits: int = -1, cap: int = 1 << 16):
    """Exponent-hash bin table as built on the device: (info dict, counts)."""
    _need(table, torch.float64, "table")
    counts = torch.full((cap,), -7, dtype=torch.int32, device=table.device)
    info = (ctypes.c_int64 * 4)()
    use_current_stream()
    check(lib().ss_exphash_bins(_ptr(table), table.numel(), int(bucket_bits), _ptr(counts), cap,
                                info))
    s, kmin, nb, kmax_occ = (int(v) for v in info)
    return {"bits": s, "kmin": kmin, "nb": nb, "max_occupancy": kmax_occ}, counts[:nb + 1]


def loghash_bins(table: torch.Tensor, nb: int):
    """Logarithm-hash bin table as built on the device: (info dict, counts)."""
    _need(table, torch.float64, "table")
    counts = torch.full((int(nb) + 1,), -7, dtype=torch.int32, device=table.device)
    info = (ctypes.c_double * 6)()
    use_current_stream()
    check(lib().ss_loghash_bins(_ptr(table), table.numel(), int(nb), _ptr(counts), info))
    keys = ("nb", "max_occupancy", "e0", "lm0", "S", "phi")
    d = dict(zip(keys, (float(v) for v in info)))
    for k in ("nb", "max_occupancy", "e0"):
        d[k] = int(d[k])
    return d, counts


# ---------------------------------------------------------------------------
# plans: many tables (batched) and paired lookups
# ---------------------------------------------------------------------------

PLAN_ALGOS, PLAN_BITS, PLAN_SUMMARY, PLAN_COSTS, PLAN_BRACKETS = 1, 2, 3, 4, 5
SUMMARY_KEYS = ("tables", "tiles", "tiles_per_wg", "grid", "block", "lds_bytes",
                "max_bin", "graph_uses", "targets_per_lane", "learned_form")


def _host_offsets(off, name):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    if a.ndim != 1 or a.shape[0] < 2:
        raise ValueError(f"{name} must be a 1-D array of at least 2 offsets")
    return a


def _off_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Plan:
    _handle = None

    def close(self) -> None:
        if self._handle is not None and self._handle.value:
            lib().ss_plan_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fallbacks(self) -> int:
        v = ctypes.c_int64()
        use_current_stream()
        check(lib().ss_plan_fallbacks(self._handle, ctypes.byref(v)))
        return v.value

    def save(self, path: str) -> None:
        """Writes the plan's choices (ss_plan_save); reload with saved=path."""
        check(lib().ss_plan_save(self._handle, os.fsencode(path)))

    def info(self) -> dict:
        import numpy as np
        T = self.num_descriptors
        algos = np.zeros(T, dtype=np.int32)
        bits = np.zeros(T, dtype=np.int32)
        summ = np.zeros(len(SUMMARY_KEYS), dtype=np.int64)
        check(lib().ss_plan_info(self._handle, PLAN_ALGOS, _off_ptr(algos), T))
        check(lib().ss_plan_info(self._handle, PLAN_BITS, _off_ptr(bits), T))
        check(lib().ss_plan_info(self._handle, PLAN_SUMMARY, _off_ptr(summ), summ.size))
        costs = np.zeros(2 * T, dtype=np.float64)
        check(lib().ss_plan_info(self._handle, PLAN_COSTS, _off_ptr(costs), 2 * T))
        out = dict(zip(SUMMARY_KEYS, (int(v) for v in summ)))
        out["algos"] = algos
        out["bits"] = bits
        out["plain_ns"] = costs[0::2].copy()
        out["learned_ns"] = costs[1::2].copy()
        brackets = np.zeros(T, dtype=np.float64)
        check(lib().ss_plan_info(self._handle, PLAN_BRACKETS, _off_ptr(brackets), T))
        out["brackets"] = brackets
        return out


class MultiPlan(_Plan):
    """Many tables searched in one launch (see ss_multi_plan_create).  With
    models (a list of T LearnedIndex or None), each given model searches its
    table (ss_multi_plan_create_learned); the plan copies the models.  With
    sample (device float64 targets in the search layout) the tuner measures
    the targets' spread per table and may choose the ballot scan
    (ss_multi_plan_create_sampled)."""

    def __init__(self, tables: torch.Tensor, table_off, query_off, models=None,
                 saved: str | None = None, sample: torch.Tensor | None = None):
        _need(tables, torch.float64, "tables")
        self._toff = _host_offsets(table_off, "table_off")
        self._qoff = _host_offsets(query_off, "query_off")
        if self._toff.shape != self._qoff.shape:
            raise ValueError("table_off and query_off must have the same length")
        self.num_descriptors = self._toff.shape[0] - 1
        self.num_queries = int(self._qoff[-1])
        self._tables = tables  # referenced by the plan: keep alive
        h = ctypes.c_void_p()
        use_current_stream()
        if saved is not None:  # a plan saved with save(): no tuning or training
            check(lib().ss_multi_plan_load(os.fsencode(saved), _ptr(tables), _off_ptr(self._toff),
                                           self.num_descriptors, _off_ptr(self._qoff),
                                           ctypes.byref(h)))
        elif sample is not None:
            if models is not None:
                raise ValueError("sample and models cannot be combined")
            _need(sample, torch.float64, "sample")
            if sample.numel() != self.num_queries:
                raise ValueError(f"expected {self.num_queries} sample targets")
            check(lib().ss_multi_plan_create_sampled(_ptr(tables), _off_ptr(self._toff),
                                                     self.num_descriptors, _off_ptr(self._qoff),
                                                     _ptr(sample), ctypes.byref(h)))
        elif models is None:
            check(lib().ss_multi_plan_create(_ptr(tables), _off_ptr(self._toff),
                                             self.num_descriptors, _off_ptr(self._qoff),
                                             ctypes.byref(h)))
        else:
            if len(models) != self.num_descriptors:
                raise ValueError(f"expected {self.num_descriptors} models (or None entries)")
            arr = (ctypes.c_void_p * len(models))(
                *[None if mdl is None else mdl._handle.value for mdl in models])
            check(lib().ss_multi_plan_create_learned(_ptr(tables), _off_ptr(self._toff),
                                                     self.num_descriptors, _off_ptr(self._qoff),
                                                     arr, ctypes.byref(h)))
        self._handle = h

    def search(self, targets: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _need(targets, torch.float64, "targets")
        if targets.numel() != self.num_queries:
            raise ValueError(f"expected {self.num_queries} targets, got {targets.numel()}")
        if out is None:
            out = torch.empty(self.num_queries, dtype=torch.int32, device=targets.device)
        _need(out, torch.int32, "out")
        if out.numel() != self.num_queries:
            raise ValueError("out must have one entry per target")
        use_current_stream()
        check(lib().ss_multi_search(self._handle, _ptr(targets), _ptr(out)))
        return out


def multi_search_noalloc(tables: torch.Tensor, table_off: torch.Tensor, query_off: torch.Tensor,
                         targets: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Batched search without a plan (ss_multi_search_noalloc): table_off and
    query_off are device int64 tensors of T+1 offsets."""
    _need(tables, torch.float64, "tables")
    _need(table_off, torch.int64, "table_off")
    _need(query_off, torch.int64, "query_off")
    _need(targets, torch.float64, "targets")
    T = table_off.numel() - 1
    if query_off.numel() != T + 1:
        raise ValueError("table_off and query_off must have the same length")
    if out is None:
        out = torch.empty(targets.numel(), dtype=torch.int32, device=targets.device)
    _need(out, torch.int32, "out")
    if out.numel() != targets.numel():
        raise ValueError("out must have one entry per target")
    use_current_stream()
    check(lib().ss_multi_search_noalloc(_ptr(tables), tables.numel(), _ptr(table_off), T,
                                        _ptr(query_off), _ptr(targets), targets.numel(),
                                        _ptr(out)))
    return out


class PairPlan(_Plan):
    """Paired density/temperature lookups per material (ss_pair_plan_create;
    with sample=(rho, temp), ss_pair_plan_create_sampled)."""

    def __init__(self, rho_tables: torch.Tensor, rho_off, t_tables: torch.Tensor, t_off,
                 pair_off, saved: str | None = None, sample=None):
        _need(rho_tables, torch.float64, "rho_tables")
        _need(t_tables, torch.float64, "t_tables")
        self._roff = _host_offsets(rho_off, "rho_off")
        self._toff = _host_offsets(t_off, "t_off")
        self._poff = _host_offsets(pair_off, "pair_off")
        M = self._roff.shape[0] - 1
        if self._toff.shape[0] != M + 1 or self._poff.shape[0] != M + 1:
            raise ValueError("offset arrays must all have M+1 entries")
        self.num_materials = M
        self.num_descriptors = 2 * M
        self.num_queries = int(self._poff[-1])
        self._tables = (rho_tables, t_tables)
        h = ctypes.c_void_p()
        use_current_stream()
        if saved is not None:  # a plan saved with save(): no tuning or training
            check(lib().ss_pair_plan_load(os.fsencode(saved), _ptr(rho_tables),
                                          _off_ptr(self._roff), _ptr(t_tables),
                                          _off_ptr(self._toff), M, _off_ptr(self._poff),
                                          ctypes.byref(h)))
        elif sample is not None:
            s_rho, s_t = sample
            _need(s_rho, torch.float64, "sample rho")
            _need(s_t, torch.float64, "sample temp")
            if s_rho.numel() != self.num_queries or s_t.numel() != self.num_queries:
                raise ValueError(f"expected {self.num_queries} sample pairs")
            check(lib().ss_pair_plan_create_sampled(_ptr(rho_tables), _off_ptr(self._roff),
                                                    _ptr(t_tables), _off_ptr(self._toff), M,
                                                    _off_ptr(self._poff), _ptr(s_rho), _ptr(s_t),
                                                    ctypes.byref(h)))
        else:
            check(lib().ss_pair_plan_create(_ptr(rho_tables), _off_ptr(self._roff),
                                            _ptr(t_tables), _off_ptr(self._toff), M,
                                            _off_ptr(self._poff), ctypes.byref(h)))
        self._handle = h

    def search(self, rho: torch.Tensor, temp: torch.Tensor, out_rho: torch.Tensor | None = None,
               out_t: torch.Tensor | None = None):
        _need(rho, torch.float64, "rho")
        _need(temp, torch.float64, "temp")
        m = self.num_queries
        if rho.numel() != m or temp.numel() != m:
            raise ValueError(f"expected {m} pairs")
        if out_rho is None:
            out_rho = torch.empty(m, dtype=torch.int32, device=rho.device)
        if out_t is None:
            out_t = torch.empty(m, dtype=torch.int32, device=rho.device)
        _need(out_rho, torch.int32, "out_rho")
        _need(out_t, torch.int32, "out_t")
        use_current_stream()
        check(lib().ss_pair_search(self._handle, _ptr(rho), _ptr(temp), _ptr(out_rho),
                                   _ptr(out_t)))
        return out_rho, out_t


def debug_violations() -> int:
    """Bounds-check violations counted since the last call (device-checked
    library only; SearchSortedError SS_ERR_UNSUPPORTED otherwise)."""
    v = ctypes.c_int64()
    use_current_stream()
    check(lib().ss_debug_violations(ctypes.byref(v)))
    return v.value


def debug_selftest() -> None:
    """One deliberately clamped index in a one-thread kernel (device-checked
    library only): afterwards debug_violations() reports 1."""
    use_current_stream()
    check(lib().ss_debug_selftest())


# ---------------------------------------------------------------------------
# autotuner model
# ---------------------------------------------------------------------------

TUNER_KEYS = ("stream_gbs", "hash_base_ns", "hash_per_k_ns", "bin_base_ns", "bin_per_step_ns",
              "learned_base_ns", "calibrated", "bins_per_entry", "tiles_short", "tiles_long",
              "learned_per_step_ns", "ballot_base_ns", "ballot_per_entry_ns")


class InterpPlan(PairPlan):
    """Paired lookups followed by bilinear interpolation of each material's
    value grid (ss_interp_plan_create / ss_interp_search)."""

    def __init__(self, rho_tables: torch.Tensor, rho_off, t_tables: torch.Tensor, t_off,
                 pair_off, values: torch.Tensor):
        _need(rho_tables, torch.float64, "rho_tables")
        _need(t_tables, torch.float64, "t_tables")
        _need(values, torch.float64, "values")
        self._roff = _host_offsets(rho_off, "rho_off")
        self._toff = _host_offsets(t_off, "t_off")
        self._poff = _host_offsets(pair_off, "pair_off")
        M = self._roff.shape[0] - 1
        if self._toff.shape[0] != M + 1 or self._poff.shape[0] != M + 1:
            raise ValueError("offset arrays must all have M+1 entries")
        self.num_materials = M
        self.num_descriptors = 2 * M
        self.num_queries = int(self._poff[-1])
        self._tables = (rho_tables, t_tables, values)
        h = ctypes.c_void_p()
        use_current_stream()
        check(lib().ss_interp_plan_create(_ptr(rho_tables), _off_ptr(self._roff), _ptr(t_tables),
                                          _off_ptr(self._toff), M, _off_ptr(self._poff),
                                          _ptr(values), ctypes.byref(h)))
        self._handle = h

    def interpolate(self, rho: torch.Tensor, temp: torch.Tensor, out: torch.Tensor | None = None,
                    out_rho: torch.Tensor | None = None, out_t: torch.Tensor | None = None):
        _need(rho, torch.float64, "rho")
        _need(temp, torch.float64, "temp")
        m = self.num_queries
        if rho.numel() != m or temp.numel() != m:
            raise ValueError(f"expected {m} pairs")
        if out is None:
            out = torch.empty(m, dtype=torch.float64, device=rho.device)
        _need(out, torch.float64, "out")
        if (out_rho is None) != (out_t is None):
            raise ValueError("out_rho and out_t: both or neither")
        use_current_stream()
        check(lib().ss_interp_search(self._handle, _ptr(rho), _ptr(temp), _ptr(out),
                                     _ptr(out_rho), _ptr(out_t)))
        return out

    def search(self, *a, **k):
        raise TypeError("interpolation plan: use interpolate()")


def tuner_calibrate() -> dict:
    use_current_stream()
    check(lib().ss_tuner_calibrate())
    return tuner_get()


def tuner_get() -> dict:
    buf = (ctypes.c_double * len(TUNER_KEYS))()
    check(lib().ss_tuner_get(buf, len(TUNER_KEYS)))
    return dict(zip(TUNER_KEYS, list(buf)))


def tuner_set(**changes) -> dict:
    """Replaces named coefficients of the model (others unchanged)."""
    cur = tuner_get()
    unknown = set(changes) - set(TUNER_KEYS)
    if unknown:
        raise KeyError(sorted(unknown))
    cur.update(changes)
    buf = (ctypes.c_double * len(TUNER_KEYS))(*[float(cur[k]) for k in TUNER_KEYS])
    check(lib().ss_tuner_set(buf, len(TUNER_KEYS)))
    return tuner_get()


def tuner_save(path: str) -> None:
    check(lib().ss_tuner_save(os.fsencode(path)))


def tuner_load(path: str) -> None:
    check(lib().ss_tuner_load(os.fsencode(path)))


# ---------------------------------------------------------------------------
# learned index
# ---------------------------------------------------------------------------

MLP_PARAMS = 1153


class MlpOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("lr", ctypes.c_float), ("seed", ctypes.c_uint64)]


class LearnedIndex:
    """Per-table learned index (see ss_learned_build).  Build from a table
    (trains on the device) or from given weights."""

    def __init__(self, table: torch.Tensor, steps: int = 3000, lr: float = 0.01, seed: int = 1,
                 weights=None, path: str | None = None):
        import numpy as np
        _need(table, torch.float64, "table")
        self._table = table
        self.n = table.numel()
        h = ctypes.c_void_p()
        use_current_stream()
        if path is not None:
            check(lib().ss_learned_load(_ptr(table), self.n, os.fsencode(path), ctypes.byref(h)))
        elif weights is None:
            opts = MlpOpts(int(steps), float(lr), int(seed))
            check(lib().ss_learned_build(_ptr(table), self.n, ctypes.byref(opts), ctypes.byref(h)))
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32)
            if w.shape != (MLP_PARAMS,):
                raise ValueError(f"weights must have {MLP_PARAMS} entries")
            check(lib().ss_learned_from_weights(_ptr(table), self.n,
                                                w.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.byref(h)))
        self._handle = h

    @classmethod
    def load(cls, table: torch.Tensor, path: str) -> "LearnedIndex":
        """A model saved with save(), attached to `table` (E measured again)."""
        return cls(table, path=path)

    def save(self, path: str) -> None:
        check(lib().ss_learned_save(self._handle, os.fsencode(path)))

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib().ss_learned_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search(self, targets: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _need(targets, torch.float64, "targets")
        if out is None:
            out = torch.empty(targets.numel(), dtype=torch.int32, device=targets.device)
        _need(out, torch.int32, "out")
        if out.numel() != targets.numel():
            raise ValueError("out must have one entry per target")
        use_current_stream()
        check(lib().ss_learned_search(self._handle, _ptr(targets), targets.numel(), _ptr(out)))
        return out

    def predict(self, x: torch.Tensor) -> torch.Tensor:
        _need(x, torch.float64, "x")
        out = torch.empty(x.numel(), dtype=torch.float32, device=x.device)
        use_current_stream()
        check(lib().ss_learned_predict(self._handle, _ptr(x), x.numel(), _ptr(out)))
        return out

    def info(self) -> dict:
        buf = (ctypes.c_double * 10)()
        check(lib().ss_learned_info(self._handle, buf, 10))
        return {"E": int(buf[0]), "n": int(buf[1]), "steps": int(buf[2]), "loss": buf[3],
                "u0": buf[4], "inv": buf[5], "pieces": int(buf[6]),
                "bound_slots": int(buf[7]), "cells": int(buf[8]), "cell_scan": int(buf[9])}

    def fallbacks(self) -> int:
        v = ctypes.c_int64()
        use_current_stream()
        check(lib().ss_learned_fallbacks(self._handle, ctypes.byref(v)))
        return v.value

    def error_bound(self) -> int:
        v = ctypes.c_int32()
        check(lib().ss_learned_error_bound(self._handle, ctypes.byref(v)))
        return v.value

    def set_error_bound(self, E: int) -> None:
        """Replaces the bound the searches use (ss_learned_set_error_bound)."""
        check(lib().ss_learned_set_error_bound(self._handle, int(E)))

    def stats(self) -> int:
        """Fallbacks of the most recent search (ss_learned_stats)."""
        v = ctypes.c_int64()
        use_current_stream()
        check(lib().ss_learned_stats(self._handle, ctypes.byref(v)))
        return v.value

    def weights(self):
        import numpy as np
        w = np.empty(MLP_PARAMS, dtype=np.float32)
        check(lib().ss_learned_weights(self._handle, w.ctypes.data_as(ctypes.c_void_p),
                                       MLP_PARAMS))
        return w


def mlp_gradient(table: torch.Tensor, weights):
    """(loss, gradient) of the training loss at `weights`, from the device
    training kernel's arithmetic."""
    import numpy as np
    _need(table, torch.float64, "table")
    w = np.ascontiguousarray(weights, dtype=np.float32)
    g = np.empty(MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_double()
    use_current_stream()
    check(lib().ss_mlp_gradient(_ptr(table), table.numel(), w.ctypes.data_as(ctypes.c_void_p),
                                g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)))
    return loss.value, g
