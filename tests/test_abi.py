"""The C-ABI library loads and exports every declared symbol; host-side
argument checks reject bad calls before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(REPO, "include", "searchsorted.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^SS_API\s+[\w\s\*]*?\b(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2112_03229_amd import binding
    return binding.lib()


def test_header_declares_entry_points():
    syms = declared_symbols()
    for required in ("search_sorted_batch", "ss_search_with", "ss_last_error", "ss_set_stream",
                     "ss_set_option", "ss_get_option", "ss_validate_table", "ss_exphash_bins"):
        assert required in syms


def test_every_declared_symbol_is_exported(L):
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_version_and_options(L):
    from paper_2112_03229_amd import binding as b
    assert L.ss_version() >= 100
    assert b.get_option(b.OPT_FORCE_ALGO) == b.ALGO_AUTO
    b.set_option(b.OPT_BUCKET_BITS, 5)
    assert b.get_option(b.OPT_BUCKET_BITS) == 5
    b.set_option(b.OPT_BUCKET_BITS, -1)
    for opt, bad in ((b.OPT_FORCE_ALGO, 9), (b.OPT_BUCKET_BITS, 21), (b.OPT_BLOCK_SIZE, 100),
                     (b.OPT_CHECK_POINTERS, 2), (999, 0)):
        with pytest.raises(b.SearchSortedError) as e:
            b.set_option(opt, bad)
        assert e.value.code == -1
    assert b.get_option(b.OPT_BUCKET_BITS) == -1


def test_argument_errors_before_device_work(L):
    P = ctypes.c_void_p
    fake = P(0x10000)
    # negative sizes, n > INT32_MAX, null with count, misalignment, overlap
    assert L.search_sorted_batch(fake, -1, fake, 10, fake) == -1
    assert L.search_sorted_batch(fake, 10, fake, -5, fake) == -1
    assert L.search_sorted_batch(fake, 2**31, fake, 10, P(0x90000)) == -1
    assert L.search_sorted_batch(P(0), 10, fake, 10, P(0x90000)) == -1
    assert L.search_sorted_batch(fake, 10, P(0x20004), 10, P(0x90000)) == -1
    assert L.search_sorted_batch(fake, 10, P(0x20000), 10, P(0x20010)) == -1
    assert b"overlap" in L.ss_last_error()
    assert L.ss_search_with(fake, 10, P(0x20000), 10, P(0x90000), 7, -1) == -1
    assert L.ss_search_with(fake, 10, P(0x20000), 10, P(0x90000), 3, 25) == -1
    # m == 0 is a no-op that touches nothing
    assert L.search_sorted_batch(P(0), 0, P(0), 0, P(0)) == 0
    assert L.ss_exphash_bins(fake, 0, 0, fake, 16, None) == -1


def test_host_pointers_are_rejected(L):
    import numpy as np
    from paper_2112_03229_amd import binding as b
    a = np.arange(16, dtype=np.float64)
    x = np.arange(32, dtype=np.float64)
    out = np.zeros(32, dtype=np.int32)
    rc = L.search_sorted_batch(a.ctypes.data, 16, x.ctypes.data, 32, out.ctypes.data)
    # without a GPU the check reports a non-device pointer or no device;
    # either way a status code, never a crash
    assert rc in (-2, -3, -4)
    assert L.ss_last_error()
