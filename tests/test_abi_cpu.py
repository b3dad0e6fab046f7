"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and rejects bad arguments before touching
a device."""
import ctypes
import os
import re

import pytest

import paper_1304_0681_amd as sw

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hpgsw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function():
    L = sw.lib()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), f"{n} declared in hpgsw.h but not exported"


def test_null_and_invalid_arguments():
    L = sw.lib()
    assert L.sw_ctx_create(0, None) == sw.SW_E_INVALID
    assert L.sw_batch_score(None, None, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_batch_traceback(None, None, None, None, 0, None, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_pack2b(None, None, 0, None, None, None) == sw.SW_E_INVALID
    assert L.sw_select_windows(None, None, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_sole_windows(None, None, None, None, None, None, None) == sw.SW_E_INVALID
    assert L.sw_merge_best(None, 4, None, None, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_ctx_destroy(None) == sw.SW_E_INVALID


def test_no_device_reported(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = sw.lib().sw_ctx_create(0, ctypes.byref(h))
    assert st == sw.SW_E_NODEVICE
    assert sw.lib().sw_last_error(None)


def test_cigar_string_formatting():
    ops = [(3 << 4) | 4, (10 << 4) | 0, (1 << 4) | 2, (5 << 4) | 0, (2 << 4) | 1, (7 << 4) | 0]
    assert sw.sw_cigar_string(ops) == "3S10M1D5M2I7M"
    assert sw.sw_cigar_string([]) == ""
    buf = ctypes.create_string_buffer(4)
    a = (ctypes.c_uint32 * 1)((123 << 4) | 0)
    assert sw.lib().sw_cigar_string(a, 1, buf, 4) == -1


def test_new_stage_calls_reject_bad_arguments():
    """The seeker, stage B, CAL and junction calls refuse a missing context
    before touching a device, and the index size is checked on the host."""
    L = sw.lib()
    assert L.sw_seed_cals(None, None, None, None, None, 0, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_join_cals(None, None, 0, 0, 0, 0, 0, None, None, None) == sw.SW_E_INVALID
    assert L.sw_junctions_clear(None, None, None, 8, None) == sw.SW_E_INVALID
    assert L.sw_detect_junctions(None, None, None, 0, None, None, 0, 0, 40, None, None, 8, None,
                                 None, None) == sw.SW_E_INVALID
    assert L.sw_list_junctions(None, None, None, 8, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_kmer_index_build(None, None, 0, 15, None, 0, None) == sw.SW_E_INVALID
    assert L.sw_seed_regions(None, None, None, 0, None, None, 0, None, None) == sw.SW_E_INVALID
    assert L.sw_cal_seeker(None, None, None, 0, 0, 15, 0, 0, None, None, None) == sw.SW_E_INVALID
    assert L.sw_stage_b(None, None, None, None, 0, None, None, None) == sw.SW_E_INVALID
    # index sizes: 4 (4^k + 1) bytes of offsets, rounded to 256, plus 4 per k-mer
    assert sw.sw_kmer_index_bytes(1000, 4) == ((4 * 257 + 255) // 256) * 256 + 4 * 997
    assert sw.sw_kmer_index_bytes(4_000_000, 15) == 4 * (4 ** 15 + 1) + 252 + 4 * (4_000_000 - 14)
    assert sw.sw_kmer_index_bytes(3, 4) == 1280          # no k-mer at all
    for k in (3, 16):
        with pytest.raises(sw.SwError):
            sw.sw_kmer_index_bytes(1000, k)
    with pytest.raises(sw.SwError):
        sw.sw_kmer_index_bytes(1 << 33, 15)
