"""ctypes binding of ``libfht.so`` (declared in ``include/fht.h``).

The functions keep the C names and only marshal arguments: every step of the
transform runs in the HIP kernels of the library.  ``Plan`` and ``Batch`` wrap
them for torch tensors (torch supplies device memory and the stream).  If the
library has not been built, importing this module raises.
"""
from __future__ import annotations

import atexit
import collections
import contextlib
import ctypes
import os
from typing import Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfht.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2411_07351_amd/build.py`")

# torch first: the library must bind to the HIP runtime torch already loaded,
# because streams and device pointers are torch's.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# Destructors that run while the interpreter exits skip the C calls: the
# process frees everything then, and the HIP runtime may already be gone.
_EXITING = [False]
atexit.register(lambda: _EXITING.__setitem__(0, True))

__all__ = [
    "FHT_U8", "FHT_F32", "FHT_F64", "FHT_SPLIT_S", "FHT_SPLIT_T", "FHT_HDR_INTS", "QUADRANTS",
    "LIB_PATH", "EXPORTED", "FhtError", "fht_schedule", "Plan", "Batch", "hough",
    "fht_status_string", "fht_plan_create", "fht_plan_destroy", "fht_plan_out_elems",
    "fht_plan_out_offset", "fht_plan_workspace_bytes", "fht_plan_num_launches",
    "fht_plan_launch_info", "fht_plan_upload", "fht_forward", "fht_forward_launch", "fht_batch_create",
    "fht_batch_workspace_bytes", "fht_batch_num_launches", "fht_batch_run",
    "fht_batch_run_launch", "fht_batch_destroy", "fht_plan_num_passes", "fht_plan_pass_tables",
    "fht_batch_prepare", "fht_batch_tables_bytes", "fht_batch_upload", "fht_debug_fail_next",
    "fht_plan_adjoint_workspace_bytes", "fht_plan_adjoint_tasks", "fht_adjoint",
    "HoughFunction", "hough_autograd", "fht_peaks_workspace_bytes", "fht_peaks", "PEAK_DTYPE",
    "fht_plan_work", "fht_plan_launch_kernel", "fht_plan_workspace_bytes_many",
    "fht_forward_many", "fht_plan_adjoint_workspace_bytes_many", "fht_adjoint_many",
    "fht_plan_adjoint_num_passes", "fht_plan_adjoint_pass", "fht_batch_upload_staged",
    "fht_plan_upload_programs", "fht_planner_create", "fht_planner_submit", "fht_planner_poll",
    "fht_planner_destroy", "fht_plan_upload_programs_many", "fht_batch_copy_images", "STATUS",
    "fht_forward_noalloc", "NOALLOC_WS_BYTES",
]

FHT_U8, FHT_F32, FHT_F64 = 0, 1, 2
FHT_SPLIT_S, FHT_SPLIT_T = 0, 1
FHT_HDR_INTS = 32
QUADRANTS = ("V+", "V-", "H+", "H-")

STATUS = {0: "FHT_OK", -1: "FHT_EINVAL", -2: "FHT_EDTYPE", -3: "FHT_ENOMEM",
          -4: "FHT_EHIP", -5: "FHT_EBUSY", -6: "FHT_ENODEV"}

EXPORTED = (
    "fht_status_string", "fht_plan_create", "fht_plan_destroy", "fht_plan_out_elems",
    "fht_plan_out_offset", "fht_plan_workspace_bytes", "fht_plan_num_launches",
    "fht_plan_launch_info", "fht_plan_upload", "fht_forward", "fht_forward_launch", "fht_batch_create",
    "fht_batch_workspace_bytes", "fht_batch_num_launches", "fht_batch_run",
    "fht_batch_run_launch", "fht_batch_destroy", "fht_plan_num_passes", "fht_plan_pass_tables",
    "fht_batch_prepare", "fht_batch_tables_bytes", "fht_batch_upload", "fht_debug_fail_next",
    "fht_plan_adjoint_workspace_bytes", "fht_plan_adjoint_tasks", "fht_adjoint",
    "fht_peaks_workspace_bytes", "fht_peaks", "fht_plan_work", "fht_plan_launch_kernel",
    "fht_plan_workspace_bytes_many", "fht_forward_many", "fht_plan_adjoint_workspace_bytes_many",
    "fht_adjoint_many", "fht_plan_adjoint_num_passes", "fht_plan_adjoint_pass",
    "fht_batch_upload_staged", "fht_plan_upload_programs",
    "fht_planner_create", "fht_planner_submit", "fht_planner_poll", "fht_planner_destroy",
    "fht_plan_upload_programs_many", "fht_batch_copy_images", "fht_forward_noalloc",
)

# FHT_NOALLOC_WS_BYTES: the static scratch fht_forward_noalloc uses
NOALLOC_WS_BYTES = 64 * 1024 * 1024

# struct fht_peak
PEAK_DTYPE = np.dtype([("value", np.float32), ("quadrant", np.int32), ("t", np.int32),
                       ("s", np.int32)])


class fht_schedule(ctypes.Structure):
    _fields_ = [("s_tile", ctypes.c_int32), ("first_levels", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("lds_budget", ctypes.c_int32),
                ("t_tile", ctypes.c_int32), ("s_tile_first", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("threads_first", ctypes.c_int32)]


_vp, _i32, _u32, _i64, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                              ctypes.c_int64, ctypes.c_size_t)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_ppi32 = ctypes.POINTER(_pi32)


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("fht_status_string", ctypes.c_char_p, _i32)
_sig("fht_plan_create", _i32, ctypes.POINTER(_vp), _i32, _i32, _i32, _i32, _u32,
     ctypes.POINTER(fht_schedule))
_sig("fht_plan_destroy", None, _vp)
_sig("fht_plan_out_elems", _sz, _vp)
_sig("fht_plan_out_offset", _i64, _vp, _i32)
_sig("fht_plan_workspace_bytes", _sz, _vp)
_sig("fht_plan_num_launches", _i32, _vp)
_sig("fht_plan_launch_info", _i32, _vp, _i32, _pi32, ctypes.POINTER(_i64),
     ctypes.POINTER(_i64), _pi32)
_sig("fht_plan_work", _i32, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_sig("fht_plan_launch_kernel", ctypes.c_char_p, _vp, _i32)
_sig("fht_plan_workspace_bytes_many", _sz, _vp, _i32)
_sig("fht_forward_many", _i32, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp)
_sig("fht_plan_adjoint_workspace_bytes_many", _sz, _vp, _i32)
_sig("fht_adjoint_many", _i32, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp)
_sig("fht_plan_upload", _i32, _vp)
_sig("fht_forward", _i32, _vp, _vp, _vp, _vp, _vp)
_sig("fht_forward_noalloc", _i32, _vp, _vp, _vp, _vp)
_sig("fht_forward_launch", _i32, _vp, _i32, _vp, _vp, _vp, _vp)
_sig("fht_batch_create", _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32,
     ctypes.POINTER(_vp), ctypes.POINTER(_vp))
_sig("fht_batch_workspace_bytes", _sz, _vp)
_sig("fht_batch_num_launches", _i32, _vp)
_sig("fht_batch_run", _i32, _vp, _vp, _vp)
_sig("fht_batch_run_launch", _i32, _vp, _i32, _vp, _vp)
_sig("fht_batch_destroy", None, _vp)
_sig("fht_batch_prepare", _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32,
     ctypes.POINTER(_vp), ctypes.POINTER(_vp))
_sig("fht_batch_tables_bytes", _sz, _vp)
_sig("fht_batch_upload", _i32, _vp, _vp, _sz, _vp)
_sig("fht_debug_fail_next", None, _i32, _i32)
_sig("fht_batch_upload_staged", _i32, _vp, _vp, _sz, _vp, _vp)
_sig("fht_plan_upload_programs", _i32, _vp)
_sig("fht_batch_copy_images", _i32, _vp, ctypes.POINTER(_vp), _vp)
_sig("fht_plan_upload_programs_many", _i32, ctypes.POINTER(_vp), _i32)
_sig("fht_planner_create", _i32, _i32, _i32, ctypes.POINTER(_vp))
_sig("fht_planner_submit", _i32, _vp, _i32, _i32, _i32, _i32, _u32, ctypes.POINTER(fht_schedule),
     ctypes.POINTER(_i64))
_sig("fht_planner_poll", _i32, _vp, _i64, ctypes.POINTER(_vp), ctypes.POINTER(_i32))
_sig("fht_planner_destroy", None, _vp)
_sig("fht_plan_adjoint_workspace_bytes", _sz, _vp)
_sig("fht_plan_adjoint_tasks", _i32, _vp, _i32, _ppi32, _pi32, _pi32)
_sig("fht_adjoint", _i32, _vp, _vp, _vp, _vp, _vp)
_sig("fht_plan_adjoint_num_passes", _i32, _vp, _i32)
_sig("fht_plan_adjoint_pass", _i32, _vp, _i32, _i32, _pi32, _ppi32, _ppi32, _pi32)
_sig("fht_peaks_workspace_bytes", _sz, _i32)
_sig("fht_peaks", _i32, _vp, _vp, _i32, _i32, ctypes.c_double, _i32, _vp, _vp, _vp, _vp)
_sig("fht_plan_num_passes", _i32, _vp, _i32)
_sig("fht_plan_pass_tables", _i32, _vp, _i32, _i32, _ppi32, _pi32, _ppi32, _pi32, _ppi32,
     _pi32, _pi32)


class FhtError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({fht_status_string(status)})")


def _check(status: int, what: str) -> None:
    if status != 0:
        raise FhtError(status, what)


# ----------------------------------------------------------------- C names

def fht_status_string(status: int) -> str:
    return _lib.fht_status_string(status).decode()


def fht_plan_create(rows: int, cols: int, dtype: int, split: int, quadrant_mask: int = 15,
                    schedule: fht_schedule | None = None) -> int:
    h = _vp()
    sched = ctypes.byref(schedule) if schedule is not None else None
    _check(_lib.fht_plan_create(ctypes.byref(h), rows, cols, dtype, split, quadrant_mask, sched),
           "fht_plan_create")
    return h.value


def fht_plan_destroy(plan: int) -> None:
    _lib.fht_plan_destroy(plan)


def fht_plan_out_elems(plan: int) -> int:
    return _lib.fht_plan_out_elems(plan)


def fht_plan_out_offset(plan: int, q: int) -> int:
    return _lib.fht_plan_out_offset(plan, q)


def fht_plan_workspace_bytes(plan: int) -> int:
    return _lib.fht_plan_workspace_bytes(plan)


def fht_plan_num_launches(plan: int) -> int:
    return _lib.fht_plan_num_launches(plan)


def fht_plan_launch_info(plan: int, launch: int) -> dict:
    level, n = _i32(), _i32()
    bi, bo = _i64(), _i64()
    _check(_lib.fht_plan_launch_info(plan, launch, ctypes.byref(level), ctypes.byref(bi),
                                     ctypes.byref(bo), ctypes.byref(n)), "fht_plan_launch_info")
    return {"level": level.value, "bytes_in": bi.value, "bytes_out": bo.value,
            "n_items": n.value}


def fht_plan_work(plan: int) -> dict:
    tree, done = _i64(), _i64()
    _check(_lib.fht_plan_work(plan, ctypes.byref(tree), ctypes.byref(done)), "fht_plan_work")
    return {"adds_tree": tree.value, "adds_executed": done.value}


def fht_plan_launch_kernel(plan: int, launch: int) -> str:
    name = _lib.fht_plan_launch_kernel(plan, launch)
    if name is None:
        raise FhtError(-1, "fht_plan_launch_kernel")
    return name.decode()


def fht_plan_upload(plan: int) -> None:
    _check(_lib.fht_plan_upload(plan), "fht_plan_upload")


def fht_plan_upload_programs(plan: int) -> None:
    _check(_lib.fht_plan_upload_programs(plan), "fht_plan_upload_programs")


def fht_plan_upload_programs_many(plans) -> None:
    arr = (_vp * len(plans))(*plans)
    _check(_lib.fht_plan_upload_programs_many(arr, len(plans)), "fht_plan_upload_programs_many")


def fht_planner_create(threads: int, device: int = -1) -> int:
    h = _vp()
    _check(_lib.fht_planner_create(threads, device, ctypes.byref(h)), "fht_planner_create")
    return h.value


def fht_planner_submit(planner: int, rows: int, cols: int, dtype: int, split: int,
                       quadrant_mask: int = 15, schedule: fht_schedule | None = None) -> int:
    t = _i64()
    sched = ctypes.byref(schedule) if schedule is not None else None
    _check(_lib.fht_planner_submit(planner, rows, cols, dtype, split, quadrant_mask, sched,
                                   ctypes.byref(t)), "fht_planner_submit")
    return t.value


def fht_planner_poll(planner: int, ticket: int) -> tuple:
    """(state, plan handle or None, status): state 1 finished (the caller owns
    the plan), 0 pending, -1 unknown ticket."""
    h, st = _vp(), _i32()
    r = _lib.fht_planner_poll(planner, ticket, ctypes.byref(h), ctypes.byref(st))
    return r, h.value, st.value


def fht_planner_destroy(planner: int) -> None:
    _lib.fht_planner_destroy(planner)


def fht_forward(plan: int, d_img: int, d_out: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_forward(plan, d_img, d_out, d_ws, stream), "fht_forward")


def fht_plan_workspace_bytes_many(plan: int, n: int) -> int:
    return _lib.fht_plan_workspace_bytes_many(plan, n)


def fht_forward_noalloc(plan: int, d_img: int, d_out: int, stream: int | None) -> None:
    _check(_lib.fht_forward_noalloc(plan, d_img, d_out, stream), "fht_forward_noalloc")


def fht_forward_many(plan: int, n: int, d_imgs: int, img_stride: int, d_outs: int,
                     out_stride: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_forward_many(plan, n, d_imgs, img_stride, d_outs, out_stride, d_ws, stream),
           "fht_forward_many")


def fht_plan_adjoint_workspace_bytes_many(plan: int, n: int) -> int:
    return _lib.fht_plan_adjoint_workspace_bytes_many(plan, n)


def fht_adjoint_many(plan: int, n: int, d_gouts: int, gout_stride: int, d_gimgs: int,
                     gimg_stride: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_adjoint_many(plan, n, d_gouts, gout_stride, d_gimgs, gimg_stride, d_ws,
                                 stream), "fht_adjoint_many")


def fht_forward_launch(plan: int, launch: int, d_img: int, d_out: int, d_ws: int | None,
                       stream: int | None) -> None:
    _check(_lib.fht_forward_launch(plan, launch, d_img, d_out, d_ws, stream), "fht_forward_launch")


def fht_batch_create(plans: Sequence[int], d_imgs: Sequence[int], d_outs: Sequence[int]) -> int:
    n = len(plans)
    arr = ctypes.c_void_p * n
    h = _vp()
    _check(_lib.fht_batch_create(ctypes.byref(h), arr(*plans), n, arr(*d_imgs), arr(*d_outs)),
           "fht_batch_create")
    return h.value


def fht_batch_prepare(plans: Sequence[int], d_imgs: Sequence[int], d_outs: Sequence[int]) -> int:
    n = len(plans)
    arr = ctypes.c_void_p * n
    h = _vp()
    _check(_lib.fht_batch_prepare(ctypes.byref(h), arr(*plans), n, arr(*d_imgs), arr(*d_outs)),
           "fht_batch_prepare")
    return h.value


def fht_batch_copy_images(batch: int, srcs: Sequence, stream: int | None) -> None:
    arr = (_vp * len(srcs))(*srcs)
    _check(_lib.fht_batch_copy_images(batch, arr, stream), "fht_batch_copy_images")


def fht_batch_tables_bytes(batch: int) -> int:
    return _lib.fht_batch_tables_bytes(batch)


def fht_batch_upload(batch: int, d_tables: int, nbytes: int, stream: int | None) -> None:
    _check(_lib.fht_batch_upload(batch, d_tables, nbytes, stream), "fht_batch_upload")


def fht_batch_upload_staged(batch: int, d_tables: int, nbytes: int, h_staging: int,
                            stream: int | None) -> None:
    _check(_lib.fht_batch_upload_staged(batch, d_tables, nbytes, h_staging, stream),
           "fht_batch_upload_staged")


def fht_debug_fail_next(code: int, count: int = 1) -> None:
    _lib.fht_debug_fail_next(code, count)


def fht_batch_workspace_bytes(batch: int) -> int:
    return _lib.fht_batch_workspace_bytes(batch)


def fht_batch_num_launches(batch: int) -> int:
    return _lib.fht_batch_num_launches(batch)


def fht_batch_run(batch: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_batch_run(batch, d_ws, stream), "fht_batch_run")


def fht_batch_run_launch(batch: int, launch: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_batch_run_launch(batch, launch, d_ws, stream), "fht_batch_run_launch")


def fht_batch_destroy(batch: int) -> None:
    _lib.fht_batch_destroy(batch)


def fht_plan_adjoint_workspace_bytes(plan: int) -> int:
    return _lib.fht_plan_adjoint_workspace_bytes(plan)


def fht_plan_adjoint_tasks(plan: int, view: int) -> np.ndarray:
    """Copy of the adjoint's tasks of one lane view: (levels, lanes, 4) int32."""
    tasks, levels, lanes = _pi32(), _i32(), _i32()
    _check(_lib.fht_plan_adjoint_tasks(plan, view, ctypes.byref(tasks), ctypes.byref(levels),
                                       ctypes.byref(lanes)), "fht_plan_adjoint_tasks")
    n = levels.value * lanes.value * 4
    if n == 0:
        return np.zeros((levels.value, lanes.value, 4), dtype=np.int32)
    return np.ctypeslib.as_array(tasks, shape=(n,)).reshape(levels.value, lanes.value, 4).copy()


def fht_plan_adjoint_num_passes(plan: int, view: int) -> int:
    return _lib.fht_plan_adjoint_num_passes(plan, view)


def fht_plan_adjoint_pass(plan: int, view: int, pass_idx: int) -> dict:
    """Copy of one fused adjoint gather pass: levels, offs (lanes + 1), terms (n, 2)."""
    levels, nterms = _i32(), _i32()
    offs, terms = _pi32(), _pi32()
    _check(_lib.fht_plan_adjoint_pass(plan, view, pass_idx, ctypes.byref(levels), ctypes.byref(offs),
                                      ctypes.byref(terms), ctypes.byref(nterms)),
           "fht_plan_adjoint_pass")
    lanes = fht_plan_adjoint_tasks(plan, view).shape[1]
    o = np.ctypeslib.as_array(offs, shape=(lanes + 1,)).copy()
    t = (np.ctypeslib.as_array(terms, shape=(2 * nterms.value,)).reshape(-1, 2).copy()
         if nterms.value else np.zeros((0, 2), dtype=np.int32))
    return {"levels": levels.value, "offs": o, "terms": t}


def fht_adjoint(plan: int, d_gout: int, d_gimg: int, d_ws: int | None, stream: int | None) -> None:
    _check(_lib.fht_adjoint(plan, d_gout, d_gimg, d_ws, stream), "fht_adjoint")


def fht_peaks_workspace_bytes(capacity: int) -> int:
    return _lib.fht_peaks_workspace_bytes(capacity)


def fht_peaks(plan: int, d_out: int, k: int, radius: int, min_value: float, capacity: int,
              d_ws: int, d_peaks: int, d_found: int, stream: int | None) -> None:
    _check(_lib.fht_peaks(plan, d_out, k, radius, min_value, capacity, d_ws, d_peaks, d_found,
                          stream), "fht_peaks")


def fht_plan_num_passes(plan: int, view: int) -> int:
    return _lib.fht_plan_num_passes(plan, view)


def fht_plan_pass_tables(plan: int, view: int, pass_idx: int) -> dict:
    """Copies of one pass's host tables as NumPy arrays."""
    hdrs, ops, items = _pi32(), _pi32(), _pi32()
    nh, no, ni, s = _i32(), _i32(), _i32(), _i32()
    _check(_lib.fht_plan_pass_tables(plan, view, pass_idx, ctypes.byref(hdrs), ctypes.byref(nh),
                                     ctypes.byref(ops), ctypes.byref(no), ctypes.byref(items),
                                     ctypes.byref(ni), ctypes.byref(s)), "fht_plan_pass_tables")

    def arr(p, n, k):
        if n == 0:
            return np.zeros((0, k), dtype=np.int32)
        return np.ctypeslib.as_array(p, shape=(n * k,)).reshape(n, k).copy()

    return {"hdrs": arr(hdrs, nh.value, FHT_HDR_INTS), "ops": arr(ops, no.value, 4),
            "items": arr(items, ni.value, 4), "s_tile": s.value}


# ----------------------------------------------------------------- torch layer

def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    torch = _torch()
    table = {"u8": FHT_U8, "uint8": FHT_U8, torch.uint8: FHT_U8,
             "f32": FHT_F32, "float32": FHT_F32, torch.float32: FHT_F32,
             "f64": FHT_F64, "float64": FHT_F64, torch.float64: FHT_F64}
    if dtype not in table:
        raise ValueError(f"unsupported dtype {dtype!r}")
    return table[dtype]


def _split_code(split) -> int:
    table = {"S": FHT_SPLIT_S, "s": FHT_SPLIT_S, FHT_SPLIT_S: FHT_SPLIT_S,
             "T": FHT_SPLIT_T, "t": FHT_SPLIT_T, FHT_SPLIT_T: FHT_SPLIT_T}
    if split not in table:
        raise ValueError(f"unknown split {split!r}")
    return table[split]


def _stream_handle(stream) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _on(stream):
    """Context for the tensors a call allocates: on the stream its kernels run
    on, so the caching allocator never hands their memory to other work
    while those kernels may still use it."""
    if stream is None:
        return contextlib.nullcontext()
    return _torch().cuda.stream(stream)


class Plan:
    """A plan for rows x cols images (owns the C plan)."""

    def __init__(self, rows: int, cols: int, dtype="u8", split="S", quadrants=(0, 1, 2, 3),
                 schedule: dict | None = None):
        self.rows, self.cols = int(rows), int(cols)
        self.dtype_code = _dtype_code(dtype)
        self.split = _split_code(split)
        self.quadrants = tuple(sorted(set(int(q) for q in quadrants)))
        mask = 0
        for q in self.quadrants:
            mask |= 1 << q
        sched = fht_schedule(**schedule) if schedule else None
        self._setup(fht_plan_create(self.rows, self.cols, self.dtype_code, self.split, mask, sched))

    @classmethod
    def adopt(cls, handle: int, rows: int, cols: int, dtype="u8", split="S",
              quadrants=(0, 1, 2, 3)) -> "Plan":
        """Wraps (and takes ownership of) a plan made by the C library with
        these arguments, e.g. by fht_planner."""
        self = cls.__new__(cls)
        self.rows, self.cols = int(rows), int(cols)
        self.dtype_code = _dtype_code(dtype)
        self.split = _split_code(split)
        self.quadrants = tuple(sorted(set(int(q) for q in quadrants)))
        self._setup(handle)
        return self

    def _setup(self, handle: int) -> None:
        torch = _torch()
        self.handle = handle
        self.in_dtype = (torch.uint8, torch.float32, torch.float64)[self.dtype_code]
        self.out_dtype = (torch.int32, torch.float32, torch.float64)[self.dtype_code]
        self.out_elems = fht_plan_out_elems(self.handle)
        self.ws_bytes = fht_plan_workspace_bytes(self.handle)
        self.shapes = {q: ((self.rows, self.cols) if q < 2 else (self.cols, self.rows))
                       for q in self.quadrants}
        self.offsets = {q: fht_plan_out_offset(self.handle, q) for q in self.quadrants}

    def __del__(self, _exiting=_EXITING, _destroy=_lib.fht_plan_destroy):
        h = getattr(self, "handle", None)
        if h and not _exiting[0]:
            _destroy(h)
        self.handle = None

    def new_out(self, device=None):
        torch = _torch()
        return torch.empty(self.out_elems, dtype=self.out_dtype, device=device or "cuda")

    def new_ws(self, device=None):
        torch = _torch()
        return torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device or "cuda")

    def split_out(self, out) -> list:
        """Views of the flat output, one (W, H) tensor per selected quadrant."""
        res = []
        for q in self.quadrants:
            W, H = self.shapes[q]
            off = self.offsets[q]
            res.append(out[off:off + W * H].view(W, H))
        return res

    def check_image(self, img) -> None:
        if not img.is_cuda or not img.is_contiguous():
            raise ValueError("image must be a contiguous device tensor")
        if img.dtype != self.in_dtype or tuple(img.shape) != (self.rows, self.cols):
            raise ValueError(f"image must be {self.in_dtype} of shape {(self.rows, self.cols)}")

    def forward(self, img, out=None, ws=None, stream=None) -> list:
        self.check_image(img)
        with _on(stream):
            if out is None:
                out = self.new_out(img.device)
            if ws is None and self.ws_bytes:
                ws = self.new_ws(img.device)
        if out.numel() < self.out_elems or out.dtype != self.out_dtype or not out.is_contiguous():
            raise ValueError("output buffer has the wrong size or dtype")
        if self.ws_bytes and ws.numel() * ws.element_size() < self.ws_bytes:
            raise ValueError("workspace too small")
        fht_forward(self.handle, img.data_ptr(), out.data_ptr(),
                    ws.data_ptr() if ws is not None else None, _stream_handle(stream))
        return self.split_out(out)


    def adjoint(self, gout, gimg=None, ws=None, stream=None):
        """Image gradient for the output gradient `gout` (flat, fht_forward's
        output layout; float plans only)."""
        torch = _torch()
        if not gout.is_cuda or not gout.is_contiguous() or gout.dtype != self.out_dtype \
                or gout.numel() < self.out_elems:
            raise ValueError("output gradient must be a contiguous device tensor of the "
                             "plan's output size and dtype")
        abytes = fht_plan_adjoint_workspace_bytes(self.handle)
        with _on(stream):
            if gimg is None:
                gimg = torch.empty((self.rows, self.cols), dtype=self.in_dtype, device=gout.device)
            if ws is None and abytes:
                ws = torch.empty(abytes, dtype=torch.uint8, device=gout.device)
        fht_adjoint(self.handle, gout.data_ptr(), gimg.data_ptr(),
                    ws.data_ptr() if ws is not None else None, _stream_handle(stream))
        return gimg


    def forward_many(self, imgs, outs=None, ws=None, stream=None):
        """Forward transform of a same-shape batch imgs (n x rows x cols,
        contiguous): returns outs (n x out_elems), one launch per pass for all."""
        torch = _torch()
        if not imgs.is_cuda or not imgs.is_contiguous() or imgs.dim() != 3 \
                or tuple(imgs.shape[1:]) != (self.rows, self.cols) or imgs.dtype != self.in_dtype:
            raise ValueError(f"images must be contiguous {self.in_dtype} of shape "
                             f"(n, {self.rows}, {self.cols}) on the device")
        n = imgs.shape[0]
        wbytes = fht_plan_workspace_bytes_many(self.handle, n)
        with _on(stream):
            if outs is None:
                outs = torch.empty((n, self.out_elems), dtype=self.out_dtype, device=imgs.device)
            if ws is None and wbytes:
                ws = torch.empty(wbytes, dtype=torch.uint8, device=imgs.device)
        if outs.shape != (n, self.out_elems) or outs.dtype != self.out_dtype or not outs.is_contiguous():
            raise ValueError("outputs must be a contiguous (n, out_elems) tensor of the output dtype")
        fht_forward_many(self.handle, n, imgs.data_ptr(), imgs.stride(0) * imgs.element_size(),
                         outs.data_ptr(), outs.stride(0) * outs.element_size(),
                         ws.data_ptr() if ws is not None else None, _stream_handle(stream))
        return outs

    def adjoint_many(self, gouts, gimgs=None, ws=None, stream=None):
        """Image gradients (n x rows x cols) for output gradients gouts
        (n x out_elems, contiguous; float plans only)."""
        torch = _torch()
        if not gouts.is_cuda or not gouts.is_contiguous() or gouts.dim() != 2 \
                or gouts.shape[1] != self.out_elems or gouts.dtype != self.out_dtype:
            raise ValueError("output gradients must be a contiguous (n, out_elems) device tensor")
        n = gouts.shape[0]
        wbytes = fht_plan_adjoint_workspace_bytes_many(self.handle, n)
        with _on(stream):
            if gimgs is None:
                gimgs = torch.empty((n, self.rows, self.cols), dtype=self.in_dtype,
                                    device=gouts.device)
            if ws is None and wbytes:
                ws = torch.empty(wbytes, dtype=torch.uint8, device=gouts.device)
        fht_adjoint_many(self.handle, n, gouts.data_ptr(), gouts.stride(0) * gouts.element_size(),
                         gimgs.data_ptr(), gimgs.stride(0) * gimgs.element_size(),
                         ws.data_ptr() if ws is not None else None, _stream_handle(stream))
        return gimgs

    def peaks(self, out, k: int = 32, radius: int = 3, min_value: float = 0.0,
              capacity: int = 1 << 16, stream=None):
        """The k strongest local maxima of the output `out` (see fht_peaks):
        a NumPy array of PEAK_DTYPE records, strongest first, and the number
        of candidates found."""
        torch = _torch()
        if not out.is_cuda or not out.is_contiguous() or out.numel() < self.out_elems:
            raise ValueError("output must be a contiguous device tensor of the plan's size")
        with _on(stream):
            ws = torch.empty(fht_peaks_workspace_bytes(capacity), dtype=torch.uint8,
                             device=out.device)
            rec = torch.zeros(k * PEAK_DTYPE.itemsize, dtype=torch.uint8, device=out.device)
            found = torch.zeros(2, dtype=torch.int32, device=out.device)
        fht_peaks(self.handle, out.data_ptr(), k, radius, float(min_value), capacity, ws.data_ptr(),
                  rec.data_ptr(), found.data_ptr(), _stream_handle(stream))
        if stream is not None:
            stream.synchronize()
        n, cands = (int(v) for v in found.cpu())
        return rec.cpu().numpy().view(PEAK_DTYPE)[:n].copy(), cands


class HoughFunction(torch.autograd.Function):
    """Differentiable forward transform of one float image (rows x cols) or a
    batch of same-shape images (n x rows x cols): returns the flat output (all
    quadrants; n x out_elems for a batch); the backward pass is the library's
    adjoint (``fht_adjoint`` / ``fht_adjoint_many``)."""

    @staticmethod
    def forward(ctx, img, plan):
        ctx.plan = plan
        img = img.contiguous()
        if img.dim() == 2:
            out = plan.new_out(img.device)
            plan.forward(img, out)
            return out
        return plan.forward_many(img)

    @staticmethod
    def backward(ctx, gout):
        gout = gout.contiguous()
        if gout.dim() == 1:
            return ctx.plan.adjoint(gout), None
        return ctx.plan.adjoint_many(gout), None


def hough_autograd(img, split="S", quadrants=(0, 1, 2, 3)) -> list:
    """`hough` with gradients for one image (rows x cols) or a same-shape batch
    (n x rows x cols): one tensor per quadrant, (W, H) or (n, W, H), views of
    one flat output whose backward runs the library's adjoint."""
    shape = tuple(img.shape[-2:])
    plan = _cached_plan(shape, img.dtype, split, quadrants)
    out = HoughFunction.apply(img, plan)
    if img.dim() == 2:
        return plan.split_out(out)
    res = []
    for q in plan.quadrants:
        W, H = plan.shapes[q]
        off = plan.offsets[q]
        res.append(out[:, off:off + W * H].view(-1, W, H))
    return res


class Batch:
    """Many images (one plan each) run as one launch per fused pass."""

    def __init__(self, plans: Sequence[Plan], imgs, outs, defer_upload: bool = False):
        """With ``defer_upload`` the device tables are not allocated here:
        ``upload(tables, stream)`` copies them into a caller tensor of at least
        ``tables_bytes`` bytes (nothing here then allocates or synchronises the
        device)."""
        if not (len(plans) == len(imgs) == len(outs)) or not plans:
            raise ValueError("plans, images and outputs must be non-empty and of equal length")
        for p, img, out in zip(plans, imgs, outs):
            p.check_image(img)
            if out.numel() < p.out_elems or out.dtype != p.out_dtype or not out.is_contiguous():
                raise ValueError("output buffer has the wrong size or dtype")
        self.plans = list(plans)      # keep the plans alive as long as the batch
        self.imgs, self.outs = list(imgs), list(outs)
        make = fht_batch_prepare if defer_upload else fht_batch_create
        self.handle = make([p.handle for p in plans], [i.data_ptr() for i in imgs],
                           [o.data_ptr() for o in outs])
        self.ws_bytes = fht_batch_workspace_bytes(self.handle)
        self.num_launches = fht_batch_num_launches(self.handle)
        self.tables_bytes = fht_batch_tables_bytes(self.handle)
        self.tables = None

    @classmethod
    def from_pointers(cls, plans: Sequence[Plan], img_ptrs: Sequence[int],
                      out_ptrs: Sequence[int]) -> "Batch":
        """A deferred-upload batch over raw device pointers (image i: rows x
        cols pixels of its plan's dtype, output i: ``out_elems`` elements of
        its output dtype), for callers that manage the buffers themselves;
        nothing checks their sizes.  The caller keeps the buffers alive."""
        if not (len(plans) == len(img_ptrs) == len(out_ptrs)) or not plans:
            raise ValueError("plans, images and outputs must be non-empty and of equal length")
        self = cls.__new__(cls)
        self.plans = list(plans)
        self.imgs = self.outs = None
        self.handle = fht_batch_prepare([p.handle for p in plans], list(img_ptrs), list(out_ptrs))
        self.ws_bytes = fht_batch_workspace_bytes(self.handle)
        self.num_launches = fht_batch_num_launches(self.handle)
        self.tables_bytes = fht_batch_tables_bytes(self.handle)
        self.tables = None
        return self

    def copy_images(self, srcs: Sequence, stream=None) -> None:
        """Enqueue the copies of every image from srcs[i] (a pinned host or a
        device address; None: in place) in one call."""
        fht_batch_copy_images(self.handle, srcs, _stream_handle(stream))

    def upload(self, tables, stream=None, staging=None) -> None:
        """Enqueue the copy of the device tables into `tables` (a device tensor
        of at least ``tables_bytes`` bytes, kept alive with the batch); with
        `staging` (a pinned host tensor as large) the copy goes through it and
        does not wait for the stream."""
        if tables.numel() * tables.element_size() < self.tables_bytes:
            raise ValueError("table buffer too small")
        if staging is None:
            fht_batch_upload(self.handle, tables.data_ptr(), self.tables_bytes, _stream_handle(stream))
        else:
            if staging.numel() * staging.element_size() < self.tables_bytes or not staging.is_pinned():
                raise ValueError("staging buffer too small or not pinned")
            fht_batch_upload_staged(self.handle, tables.data_ptr(), self.tables_bytes,
                                    staging.data_ptr(), _stream_handle(stream))
            self.staging = staging
        self.tables = tables

    def __del__(self, _exiting=_EXITING, _destroy=_lib.fht_batch_destroy):
        h = getattr(self, "handle", None)
        if h and not _exiting[0]:
            _destroy(h)
        self.handle = None

    def new_ws(self, device=None):
        torch = _torch()
        return torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device or "cuda")

    def run(self, ws, stream=None) -> None:
        if self.ws_bytes and ws.numel() * ws.element_size() < self.ws_bytes:
            raise ValueError("workspace too small")
        fht_batch_run(self.handle, ws.data_ptr() if ws is not None else None,
                      _stream_handle(stream))

    def capture(self, ws):
        """Record the batch's launches into a HIP graph (``torch.cuda.CUDAGraph``).

        ``graph.replay()`` then enqueues the whole batch at once.  The graph
        holds raw pointers: keep this batch, its images, outputs and ``ws``
        alive while it is used.
        """
        torch = _torch()
        if self.ws_bytes and ws.numel() * ws.element_size() < self.ws_bytes:
            raise ValueError("workspace too small")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run(ws)  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.run(ws)
        return graph


# Plans of `hough` and `hough_autograd`, least recently used first.  A plan
# dropped from here lives on while a tensor's autograd graph still holds it.
PLAN_CACHE_SIZE = 64
_plan_cache: "collections.OrderedDict" = collections.OrderedDict()


def _cached_plan(shape, dtype, split, quadrants) -> Plan:
    key = (tuple(shape), dtype, _split_code(split), tuple(sorted(set(quadrants))))
    plan = _plan_cache.get(key)
    if plan is None:
        plan = Plan(shape[0], shape[1], dtype, split, quadrants)
        _plan_cache[key] = plan
        while len(_plan_cache) > PLAN_CACHE_SIZE:
            _plan_cache.popitem(last=False)
    else:
        _plan_cache.move_to_end(key)
    return plan


def hough(img, split="S", quadrants=(0, 1, 2, 3)) -> list:
    """Transform one device image; returns one (W, H) tensor per quadrant."""
    return _cached_plan(img.shape, img.dtype, split, quadrants).forward(img)
