"""The C-ABI library loads and exports every function include/fht.h declares (no GPU)."""
import ctypes
import os
import re
import time

import numpy as np
import pytest

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
    lib.fht_batch_copy_images.restype = ctypes.c_int32
    lib.fht_batch_copy_images.argtypes = [ctypes.c_void_p] * 3
    assert lib.fht_batch_copy_images(None, None, None) == -1
    lib.fht_plan_upload_programs_many.restype = ctypes.c_int32
    lib.fht_plan_upload_programs_many.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    assert lib.fht_plan_upload_programs_many(None, 1) == -1
    assert lib.fht_plan_upload_programs_many(None, -1) == -1
    F.fht_plan_destroy(None)
    F.fht_batch_destroy(None)


def _wait(pool, ticket, timeout=60.0):
    t0 = time.monotonic()
    while True:
        state, h, st = F.fht_planner_poll(pool, ticket)
        if state != 0:
            return state, h, st
        assert time.monotonic() - t0 < timeout, "planner pool never finished"
        time.sleep(1e-3)


def _tables(h):
    out = []
    for v in (0, 1):
        for p in range(max(F.fht_plan_num_passes(h, v), 0)):
            t = F.fht_plan_pass_tables(h, v, p)
            out += [np.ascontiguousarray(t[k]).tobytes() for k in ("hdrs", "ops", "items")]
    return out


def test_planner_pool_makes_the_same_plans():
    """Plans from the native pool (host only) equal plans made directly."""
    pool = F.fht_planner_create(4, -1)
    try:
        shapes = [(64, 80, F.FHT_U8, 0), (1021, 333, F.FHT_F32, 1), (7, 3000, F.FHT_U8, 0),
                  (300, 300, F.FHT_F64, 0)] * 3
        tickets = [F.fht_planner_submit(pool, r, c, d, s) for r, c, d, s in shapes]
        assert tickets == list(range(len(shapes)))
        for (r, c, d, s), t in zip(shapes, tickets):
            state, h, st = _wait(pool, t)
            assert state == 1 and st == 0 and h
            ref = F.fht_plan_create(r, c, d, s, 15, None)
            try:
                assert F.fht_plan_out_elems(h) == F.fht_plan_out_elems(ref)
                assert _tables(h) == _tables(ref)
            finally:
                F.fht_plan_destroy(ref)
                F.fht_plan_destroy(h)
            assert F.fht_planner_poll(pool, t)[0] == -1  # taken once
        assert F.fht_planner_poll(pool, len(shapes))[0] == -1  # never issued
    finally:
        F.fht_planner_destroy(pool)


def test_planner_pool_errors():
    with pytest.raises(F.FhtError):
        F.fht_planner_create(0, -1)
    with pytest.raises(F.FhtError):
        F.fht_planner_create(2, -2)
    pool = F.fht_planner_create(2, -1)
    try:
        state, h, st = _wait(pool, F.fht_planner_submit(pool, 0, 5, F.FHT_U8, 0))
        assert state == 1 and F.STATUS[st] == "FHT_EINVAL" and not h
        state, h, st = _wait(pool, F.fht_planner_submit(pool, 5, 5, 9, 0))
        assert state == 1 and st != 0 and not h
    finally:
        F.fht_planner_destroy(pool)
    # a pool destroyed with work queued drops it and frees unpolled plans
    pool = F.fht_planner_create(1, -1)
    for _ in range(20):
        F.fht_planner_submit(pool, 4000, 4000, F.FHT_U8, 0)
    F.fht_planner_destroy(pool)
    F.fht_planner_destroy(None)
    lib = ctypes.CDLL(F.LIB_PATH)
    lib.fht_planner_poll.restype = ctypes.c_int32
    lib.fht_planner_poll.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]
    assert lib.fht_planner_poll(None, 0, None, None) == -1


def test_planner_pool_without_a_device_reports_it():
    """device >= 0 on a host without that HIP device: every plan's poll
    reports FHT_ENODEV (the pool itself is created)."""
    pool = F.fht_planner_create(2, 250)
    try:
        state, h, st = _wait(pool, F.fht_planner_submit(pool, 64, 64, F.FHT_U8, 0))
        assert state == 1 and F.STATUS[st] == "FHT_ENODEV" and not h
    finally:
        F.fht_planner_destroy(pool)


def test_planner_pool_from_several_threads():
    """Submits and polls from four threads at once: tickets are unique and
    every plan arrives exactly once, at the thread that asked for it."""
    import threading
    pool = F.fht_planner_create(3, -1)
    got, errors = {}, []

    def client(k):
        try:
            mine = [(F.fht_planner_submit(pool, 40 + 7 * k + j, 90 + j, F.FHT_U8, j % 2), j)
                    for j in range(15)]
            for t, j in mine:
                state, h, st = _wait(pool, t)
                assert state == 1 and st == 0 and h
                assert F.fht_plan_out_elems(h) == 2 * 2 * (40 + 7 * k + j) * (90 + j)
                F.fht_plan_destroy(h)
                got[t] = k
        except Exception as e:  # reported below, in the test's thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    F.fht_planner_destroy(pool)
    assert not errors, errors
    assert sorted(got) == list(range(60))


def test_program_uploads_without_a_device():
    """With no HIP device both program uploads report FHT_ENODEV (also for an
    empty list) and leave the plan usable for host queries."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = F.fht_plan_create(64, 80, F.FHT_U8, 0, 15, None)
    try:
        for call in (lambda: F.fht_plan_upload_programs(h),
                     lambda: F.fht_plan_upload_programs_many([h, h]),
                     lambda: F.fht_plan_upload_programs_many([])):
            with pytest.raises(F.FhtError) as e:
                call()
            assert F.STATUS[e.value.status] == "FHT_ENODEV"
        assert F.fht_plan_out_elems(h) == 2 * 2 * 64 * 80
    finally:
        F.fht_plan_destroy(h)


def test_noalloc_entry_point_host_checks():
    """fht_forward_noalloc: null pointers are rejected, the header's scratch
    size is the binding's, and without a HIP device the call reports
    FHT_ENODEV before anything is enqueued."""
    with open(os.path.join(ROOT, "include", "fht.h")) as fh:
        m = re.search(r"#define FHT_NOALLOC_WS_BYTES \(\(size_t\)(\d+) \* (\d+) \* (\d+)\)", fh.read())
    assert m and int(m[1]) * int(m[2]) * int(m[3]) == F.NOALLOC_WS_BYTES
    lib = ctypes.CDLL(F.LIB_PATH)
    lib.fht_forward_noalloc.restype = ctypes.c_int32
    lib.fht_forward_noalloc.argtypes = [ctypes.c_void_p] * 4
    assert lib.fht_forward_noalloc(None, None, None, None) == -1
    h = F.fht_plan_create(61, 47, F.FHT_U8, F.FHT_SPLIT_S, 15, None)
    try:
        assert lib.fht_forward_noalloc(h, None, None, None) == -1
        import torch
        if not torch.cuda.is_available():
            assert F.STATUS[lib.fht_forward_noalloc(h, 16, 16, None)] == "FHT_ENODEV"
    finally:
        F.fht_plan_destroy(h)
