"""The C-ABI library loads and exports every function include/fht.h declares (no GPU)."""
import ctypes
import os
import re

import paper_2411_07351_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "fht.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fht_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(F.LIB_PATH)
    names = _declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(F.EXPORTED) == names


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert F.fht_status_string(code) != "unknown status"
    assert F.fht_status_string(42) == "unknown status"


def test_plan_queries_without_gpu():
    h = F.fht_plan_create(61, 47, F.FHT_U8, F.FHT_SPLIT_S, 15, None)
    try:
        assert F.fht_plan_out_elems(h) == 4 * 61 * 47
        assert [F.fht_plan_out_offset(h, q) for q in range(4)] == [0, 61 * 47, 2 * 61 * 47,
                                                                   3 * 61 * 47]
        assert F.fht_plan_num_launches(h) == 2
    finally:
        F.fht_plan_destroy(h)
    h = F.fht_plan_create(8, 3, F.FHT_F32, F.FHT_SPLIT_T, 0b0100, None)
    try:
        assert F.fht_plan_out_elems(h) == 24
        assert F.fht_plan_out_offset(h, 0) == -1 and F.fht_plan_out_offset(h, 2) == 0
        assert F.fht_plan_workspace_bytes(h) == 0
        assert F.fht_plan_num_passes(h, 0) == -1 and F.fht_plan_num_passes(h, 1) == 1
    finally:
        F.fht_plan_destroy(h)


def test_null_arguments_are_rejected():
    lib = ctypes.CDLL(F.LIB_PATH)
    lib.fht_forward.restype = ctypes.c_int32
    lib.fht_forward.argtypes = [ctypes.c_void_p] * 5
    assert lib.fht_forward(None, None, None, None, None) == -1
    lib.fht_batch_run.restype = ctypes.c_int32
    lib.fht_batch_run.argtypes = [ctypes.c_void_p] * 3
    assert lib.fht_batch_run(None, None, None) == -1
    lib.fht_plan_upload_programs.restype = ctypes.c_int32
    lib.fht_plan_upload_programs.argtypes = [ctypes.c_void_p]
    assert lib.fht_plan_upload_programs(None) == -1
    F.fht_plan_destroy(None)
    F.fht_batch_destroy(None)
