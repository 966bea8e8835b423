"""Python binding of libfunnel (the C ABI in include/funnel.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.  The
library must have been built (``python -m paper_1904_09409_amd.build``); there
is no fallback path, and a missing library raises at load time.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfunnel.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "funnel.h")

FT_OK = 0
FT_ERR_INVALID_ARG = 1
FT_ERR_UNSUPPORTED_SIZE = 2
FT_ERR_MISALIGNED = 3
FT_ERR_WORKSPACE_TOO_SMALL = 4
FT_ERR_NO_DEVICE = 5
FT_ERR_HIP = 6
FT_ERR_OUT_OF_MEMORY = 7

FT_SPACE_REGULAR = 1
FT_SPACE_INVERSE = 2
FT_SPACE_BOTH = 3
FT_PREC_FP32 = 0
FT_PREC_BF16X3 = 1
FT_PREC_FP16X3 = 2
FT_PLAN_NVMT_CHIRPZ = 1
FT_VOL_SPACE_Z = 1
FT_VOL_SPACE_X = 2
FT_VOL_SPACE_Y = 4
FT_VOL_SPACE_ALL = 7
VOLUME_SPACE_NAMES = ("z", "x", "y")
FT_PEAK_CLAMP_BORDER = 1
FT_PEAK_KEEP_PAD_BOUNDARY = 2
FT_GRAPH_FORWARD = 1
FT_GRAPH_ADJOINT = 2
FT_SCHEDULE_CLASS_STREAMS = 0
FT_SCHEDULE_QUEUE = 1
# tile variants per launch (funnel_plan_set_variant): 0-7 register tiles,
# 8-10 LDS-resident tiles (column passes); 0-3 register and 4-5 LDS-resident
# tiles (row passes)
MAX_VARIANTS = 12


class ft_plan_desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("padded_len", ctypes.c_int32), ("spaces", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ft_image_desc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("image_offset", ctypes.c_int64), ("plane_offset", ctypes.c_int64)]


class ft_volume_desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("depth", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("padded_len", ctypes.c_int32), ("spaces", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class ft_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_float),
                ("bytes_per_launch", ctypes.c_double)]


class ft_tune_result(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("variant", ctypes.c_int32), ("n_tried", ctypes.c_int32),
                ("ms", ctypes.c_float), ("ms_default", ctypes.c_float)]


PEAK_DTYPE = np.dtype([("image", np.int32), ("space", np.int32), ("row", np.int32), ("col", np.int32),
                       ("value", np.float32), ("slope", np.float32), ("intercept", np.float32)])
PEAK_WORDS = PEAK_DTYPE.itemsize // 4   # 7 x 4 bytes
LINE_CHECK_DTYPE = np.dtype([("profile", np.float32, (7,)), ("contrast", np.float32), ("length", np.int32),
                             ("verified", np.int32)])
LINE_CHECK_WORDS = LINE_CHECK_DTYPE.itemsize // 4   # 10 x 4 bytes
REFINED_DTYPE = np.dtype([("col", np.float32), ("row", np.float32), ("value", np.float32), ("slope", np.float32),
                          ("intercept", np.float32), ("shift", np.float32)])
REFINED_WORDS = REFINED_DTYPE.itemsize // 4   # 6 x 4 bytes
PLANE_PEAK_DTYPE = np.dtype([("volume", np.int32), ("space", np.int32), ("z", np.int32), ("row", np.int32),
                             ("col", np.int32), ("value", np.float32), ("a", np.float32), ("b", np.float32),
                             ("c", np.float32)])
PLANE_PEAK_WORDS = PLANE_PEAK_DTYPE.itemsize // 4   # 9 x 4 bytes


class FunnelError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {msg}")


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfunnel.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1904_09409_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i32, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_uint32
    sigs = {
        "funnel_plan_create": ([ctypes.POINTER(ft_plan_desc), ctypes.POINTER(vp)], ctypes.c_int),
        "funnel_plan_destroy": ([vp], None),
        "funnel_plan_create_ragged": ([ctypes.POINTER(ft_image_desc), i32, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "funnel_buffer_elems": ([vp, ctypes.POINTER(sz), ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_plan_classes": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_plan_set_schedule": ([vp, i32], ctypes.c_int),
        "funnel_plan_schedule": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_graph_create": ([vp, u32, vp, vp, vp, vp, vp, sz, ctypes.POINTER(vp)], ctypes.c_int),
        "funnel_graph_launch": ([vp, vp], ctypes.c_int),
        "funnel_graph_destroy": ([vp], None),
        "funnel_workspace_size": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_plane_elems": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_padded_len": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_forward": ([vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "funnel_adjoint": ([vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "funnel_peaks_workspace_size": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_peaks": ([vp, vp, i32, ctypes.c_float, i32, u32, vp, vp, vp, sz, vp], ctypes.c_int),
        "funnel_peaks_noalloc": ([vp, vp, i32, ctypes.c_float, i32, u32, vp, vp, vp], ctypes.c_int),
        "funnel_verify": ([vp, vp, vp, vp, i32, i32, ctypes.c_float, i32, vp, vp], ctypes.c_int),
        "funnel_refine_workspace_size": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_refine": ([vp, vp, vp, vp, i32, i32, vp, vp, sz, vp], ctypes.c_int),
        "funnel_profile_enable": ([vp, i32], ctypes.c_int),
        "funnel_profile_read": ([vp, ctypes.POINTER(ft_kernel_time), i32, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_profile_disable": ([vp], ctypes.c_int),
        "funnel_autotune": ([vp, vp, ctypes.POINTER(ft_tune_result), i32, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_plan_variants": ([vp, ctypes.POINTER(i32), i32], ctypes.c_int),
        "funnel_plan_set_variant": ([vp, i32, i32], ctypes.c_int),
        "funnel_volume_plan_create": ([ctypes.POINTER(ft_volume_desc), ctypes.POINTER(vp)], ctypes.c_int),
        "funnel_volume_plan_destroy": ([vp], None),
        "funnel_volume_padded_len": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "funnel_volume_workspace_size": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_volume_param_elems": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_volume_forward": ([vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "funnel_volume_peaks_workspace_size": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "funnel_volume_peaks": ([vp, vp, i32, ctypes.c_float, i32, u32, vp, vp, vp, sz, vp], ctypes.c_int),
        "funnel_volume_variants": ([vp, ctypes.POINTER(i32), i32], ctypes.c_int),
        "funnel_volume_set_variant": ([vp, i32, i32], ctypes.c_int),
        "funnel_volume_autotune": ([vp, vp, ctypes.POINTER(ft_tune_result), i32, ctypes.POINTER(i32)],
                                   ctypes.c_int),
        "funnel_volume_profile_enable": ([vp, i32], ctypes.c_int),
        "funnel_volume_profile_read": ([vp, ctypes.POINTER(ft_kernel_time), i32, ctypes.POINTER(i32)],
                                       ctypes.c_int),
        "funnel_volume_profile_disable": ([vp], ctypes.c_int),
        "funnel_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "funnel_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions the public header declares."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(funnel_[a-z_]+)\s*\(", text)))


def status_string(status: int) -> str:
    return load_library().funnel_status_string(int(status)).decode()


def last_error() -> str:
    return load_library().funnel_last_error().decode()


def _check(status: int, where: str):
    if status != FT_OK:
        raise FunnelError(status, where, last_error())


def _ptr(t) -> int:
    return int(t.data_ptr())


def _need(t, name: str, dtype, numel: int, device) -> None:
    """The C calls take bare device pointers, so the extent, type and place of
    every tensor are checked here: a short or foreign buffer raises instead of
    being written past its end."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


# ------------------------------------------------------------------ raw ABI (same names)

def funnel_plan_create(batch: int, rows: int, cols: int, padded_len: int = 0,
                       spaces: int = FT_SPACE_BOTH, precision: int = FT_PREC_FP32, flags: int = 0) -> int:
    lib = load_library()
    d = ft_plan_desc(batch, rows, cols, padded_len, spaces, precision, flags)
    h = ctypes.c_void_p()
    _check(lib.funnel_plan_create(ctypes.byref(d), ctypes.byref(h)), "funnel_plan_create")
    return h.value


def funnel_plan_destroy(plan: int) -> None:
    load_library().funnel_plan_destroy(plan)


def funnel_plan_create_ragged(shapes, image_offsets, plane_offsets, spaces: int = FT_SPACE_BOTH) -> int:
    n = len(shapes)
    arr = (ft_image_desc * n)()
    for i, ((r, c), io, po) in enumerate(zip(shapes, image_offsets, plane_offsets)):
        arr[i] = ft_image_desc(int(r), int(c), int(io), int(po))
    h = ctypes.c_void_p()
    _check(load_library().funnel_plan_create_ragged(arr, n, spaces, ctypes.byref(h)), "funnel_plan_create_ragged")
    return h.value


def funnel_buffer_elems(plan: int) -> tuple[int, int]:
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().funnel_buffer_elems(plan, ctypes.byref(a), ctypes.byref(b)), "funnel_buffer_elems")
    return a.value, b.value


def funnel_plan_classes(plan: int) -> int:
    v = ctypes.c_int32()
    _check(load_library().funnel_plan_classes(plan, ctypes.byref(v)), "funnel_plan_classes")
    return v.value


def funnel_plan_set_schedule(plan: int, schedule: int) -> None:
    _check(load_library().funnel_plan_set_schedule(plan, int(schedule)), "funnel_plan_set_schedule")


def funnel_plan_schedule(plan: int) -> int:
    v = ctypes.c_int32()
    _check(load_library().funnel_plan_schedule(plan, ctypes.byref(v)), "funnel_plan_schedule")
    return v.value


def funnel_graph_create(plan: int, what: int, images=None, planes=None, d_planes=None, d_images=None,
                        ws=None) -> int:
    h = ctypes.c_void_p()
    ptr = lambda t: None if t is None else _ptr(t)
    _check(load_library().funnel_graph_create(plan, what, ptr(images), ptr(planes), ptr(d_planes), ptr(d_images),
                                              _ptr(ws), ws.numel() * ws.element_size(), ctypes.byref(h)),
           "funnel_graph_create")
    return h.value


def funnel_graph_launch(graph: int, stream=None) -> None:
    _check(load_library().funnel_graph_launch(graph, _stream(stream)), "funnel_graph_launch")


def funnel_graph_destroy(graph: int) -> None:
    load_library().funnel_graph_destroy(graph)


def funnel_workspace_size(plan: int) -> int:
    v = ctypes.c_size_t()
    _check(load_library().funnel_workspace_size(plan, ctypes.byref(v)), "funnel_workspace_size")
    return v.value


def funnel_plane_elems(plan: int) -> int:
    v = ctypes.c_size_t()
    _check(load_library().funnel_plane_elems(plan, ctypes.byref(v)), "funnel_plane_elems")
    return v.value


def funnel_padded_len(plan: int) -> int:
    v = ctypes.c_int32()
    _check(load_library().funnel_padded_len(plan, ctypes.byref(v)), "funnel_padded_len")
    return v.value


def funnel_forward(plan: int, images, planes, ws, stream=None) -> None:
    _check(load_library().funnel_forward(plan, _ptr(images), _ptr(planes), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)), "funnel_forward")


def funnel_adjoint(plan: int, d_planes, d_images, ws, stream=None) -> None:
    _check(load_library().funnel_adjoint(plan, _ptr(d_planes), _ptr(d_images), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)), "funnel_adjoint")


def funnel_peaks_workspace_size(plan: int, K: int) -> int:
    v = ctypes.c_size_t()
    _check(load_library().funnel_peaks_workspace_size(plan, K, ctypes.byref(v)), "funnel_peaks_workspace_size")
    return v.value


def funnel_peaks(plan: int, planes, K: int, threshold: float, radius: int, flags: int,
                 peaks, n_found, ws, stream=None) -> None:
    _check(load_library().funnel_peaks(plan, _ptr(planes), int(K), float(threshold), int(radius), int(flags),
                                       _ptr(peaks), _ptr(n_found), _ptr(ws), ws.numel() * ws.element_size(),
                                       _stream(stream)), "funnel_peaks")


def funnel_peaks_noalloc(plan: int, planes, K: int, threshold: float, radius: int, flags: int,
                         peaks, n_found, stream=None) -> None:
    _check(load_library().funnel_peaks_noalloc(plan, _ptr(planes), int(K), float(threshold), int(radius),
                                               int(flags), _ptr(peaks), _ptr(n_found), _stream(stream)),
           "funnel_peaks_noalloc")


def funnel_verify(plan: int, images, peaks, n_found, K: int, half_width: int, min_contrast: float,
                  min_length: int, out, stream=None) -> None:
    _check(load_library().funnel_verify(plan, _ptr(images), _ptr(peaks), _ptr(n_found), int(K), int(half_width),
                                        float(min_contrast), int(min_length), _ptr(out), _stream(stream)),
           "funnel_verify")


def funnel_refine_workspace_size(plan: int, K: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().funnel_refine_workspace_size(plan, int(K), ctypes.byref(n)), "funnel_refine_workspace_size")
    return n.value


def funnel_refine(plan: int, images, peaks, n_found, K: int, iters: int, out, ws, stream=None) -> None:
    _check(load_library().funnel_refine(plan, _ptr(images), _ptr(peaks), _ptr(n_found), int(K), int(iters), _ptr(out),
                                        _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), "funnel_refine")


def funnel_profile_enable(plan: int, max_records: int) -> None:
    _check(load_library().funnel_profile_enable(plan, int(max_records)), "funnel_profile_enable")


def funnel_profile_read(plan: int, cap: int = 64) -> list[dict]:
    """Per-kernel event times recorded since profiling was enabled (or last read)."""
    arr = (ft_kernel_time * cap)()
    n = ctypes.c_int32()
    _check(load_library().funnel_profile_read(plan, arr, cap, ctypes.byref(n)), "funnel_profile_read")
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                 bytes_per_launch=arr[i].bytes_per_launch) for i in range(n.value)]


def funnel_profile_disable(plan: int) -> None:
    _check(load_library().funnel_profile_disable(plan), "funnel_profile_disable")


def funnel_autotune(plan: int, stream=None, cap: int = 64) -> list[dict]:
    arr = (ft_tune_result * cap)()
    n = ctypes.c_int32()
    _check(load_library().funnel_autotune(plan, _stream(stream), arr, cap, ctypes.byref(n)), "funnel_autotune")
    return [dict(name=arr[i].name.decode(), variant=arr[i].variant, n_tried=arr[i].n_tried, ms=arr[i].ms,
                 ms_default=arr[i].ms_default) for i in range(n.value)]


def funnel_plan_variants(plan: int) -> list[int]:
    n = 12 * funnel_plan_classes(plan)
    arr = (ctypes.c_int32 * n)()
    _check(load_library().funnel_plan_variants(plan, arr, n), "funnel_plan_variants")
    return list(arr)


def funnel_plan_set_variant(plan: int, role: int, variant: int) -> None:
    _check(load_library().funnel_plan_set_variant(plan, int(role), int(variant)), "funnel_plan_set_variant")


# volumes (App. A)

def funnel_volume_plan_create(batch: int, depth: int, rows: int, cols: int, padded_len: int = 0,
                              spaces: int = FT_VOL_SPACE_Z, flags: int = 0) -> int:
    lib = load_library()
    d = ft_volume_desc(batch, depth, rows, cols, padded_len, spaces, flags)
    h = ctypes.c_void_p()
    _check(lib.funnel_volume_plan_create(ctypes.byref(d), ctypes.byref(h)), "funnel_volume_plan_create")
    return h.value


def funnel_volume_plan_destroy(plan: int) -> None:
    load_library().funnel_volume_plan_destroy(plan)


def funnel_volume_padded_len(plan: int) -> int:
    n = ctypes.c_int32()
    _check(load_library().funnel_volume_padded_len(plan, ctypes.byref(n)), "funnel_volume_padded_len")
    return n.value


def funnel_volume_param_elems(plan: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().funnel_volume_param_elems(plan, ctypes.byref(n)), "funnel_volume_param_elems")
    return n.value


def funnel_volume_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().funnel_volume_workspace_size(plan, ctypes.byref(n)), "funnel_volume_workspace_size")
    return n.value


def funnel_volume_forward(plan: int, volumes, params, ws, stream=None) -> None:
    _check(load_library().funnel_volume_forward(plan, _ptr(volumes), _ptr(params), _ptr(ws),
                                                ws.numel() * ws.element_size(), _stream(stream)),
           "funnel_volume_forward")


def funnel_volume_peaks_workspace_size(plan: int, K: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().funnel_volume_peaks_workspace_size(plan, int(K), ctypes.byref(n)),
           "funnel_volume_peaks_workspace_size")
    return n.value


def funnel_volume_peaks(plan: int, params, K: int, threshold: float, radius: int, flags: int,
                        peaks, n_found, ws, stream=None) -> None:
    _check(load_library().funnel_volume_peaks(plan, _ptr(params), int(K), float(threshold), int(radius), int(flags),
                                              _ptr(peaks), _ptr(n_found), _ptr(ws), ws.numel() * ws.element_size(),
                                              _stream(stream)),
           "funnel_volume_peaks")


def funnel_volume_variants(plan: int) -> list[int]:
    """Tile variant of each role, 4 per space (z, x, y), -1 for spaces the plan does not compute."""
    arr = (ctypes.c_int32 * 12)()
    _check(load_library().funnel_volume_variants(plan, arr, 12), "funnel_volume_variants")
    return list(arr)


def funnel_volume_set_variant(plan: int, role: int, variant: int) -> None:
    _check(load_library().funnel_volume_set_variant(plan, int(role), int(variant)), "funnel_volume_set_variant")


def funnel_volume_autotune(plan: int, stream=None, cap: int = 8) -> list[dict]:
    arr = (ft_tune_result * cap)()
    n = ctypes.c_int32()
    _check(load_library().funnel_volume_autotune(plan, _stream(stream), arr, cap, ctypes.byref(n)),
           "funnel_volume_autotune")
    return [dict(name=arr[i].name.decode(), variant=arr[i].variant, n_tried=arr[i].n_tried, ms=arr[i].ms,
                 ms_default=arr[i].ms_default) for i in range(n.value)]


def funnel_volume_profile_enable(plan: int, max_records: int) -> None:
    _check(load_library().funnel_volume_profile_enable(plan, int(max_records)), "funnel_volume_profile_enable")


def funnel_volume_profile_read(plan: int, cap: int = 16) -> list[dict]:
    arr = (ft_kernel_time * cap)()
    n = ctypes.c_int32()
    _check(load_library().funnel_volume_profile_read(plan, arr, cap, ctypes.byref(n)), "funnel_volume_profile_read")
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                 bytes_per_launch=arr[i].bytes_per_launch) for i in range(n.value)]


def funnel_volume_profile_disable(plan: int) -> None:
    _check(load_library().funnel_volume_profile_disable(plan), "funnel_volume_profile_disable")


# ------------------------------------------------------------------ convenience layer

@dataclass
class PlaneViews:
    regular: object = None   # torch view [B, Np, M]
    inverse: object = None   # torch view [B, Np, N]


class FunnelPlan:
    """A plan plus its workspace for a fixed batch shape on the current device."""

    def __init__(self, batch: int, rows: int, cols: int, padded_len: int = 0,
                 spaces: int = FT_SPACE_BOTH, precision: int = FT_PREC_FP32, nvmt: str = "linear"):
        import torch
        if nvmt not in ("linear", "chirpz"):
            raise ValueError(f"nvmt must be 'linear' or 'chirpz' (got {nvmt!r})")
        self.batch, self.N, self.M, self.spaces = batch, rows, cols, spaces
        self.precision, self.nvmt = precision, nvmt
        flags = FT_PLAN_NVMT_CHIRPZ if nvmt == "chirpz" else 0
        self.handle = funnel_plan_create(batch, rows, cols, padded_len, spaces, precision, flags)
        self.Np = funnel_padded_len(self.handle)
        self.plane_elems = funnel_plane_elems(self.handle)
        self.device = torch.device("cuda", torch.cuda.current_device())
        ws = funnel_workspace_size(self.handle)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                funnel_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def nspaces(self) -> int:
        return 2 if self.spaces == FT_SPACE_BOTH else 1

    def new_planes(self):
        import torch
        return torch.empty((self.batch, self.plane_elems), dtype=torch.float32, device=self.device)

    def views(self, planes) -> PlaneViews:
        v = PlaneViews()
        off = 0
        if self.spaces & FT_SPACE_REGULAR:
            n = self.Np * self.M
            v.regular = planes[:, off:off + n].view(self.batch, self.Np, self.M)
            off += n
        if self.spaces & FT_SPACE_INVERSE:
            n = self.Np * self.N
            v.inverse = planes[:, off:off + n].view(self.batch, self.Np, self.N)
        return v

    def _check_images(self, images, name="images"):
        import torch
        _need(images, name, torch.float32, self.batch * self.N * self.M, self.device)
        if tuple(images.shape) != (self.batch, self.N, self.M):
            raise ValueError(f"{name} must have shape {(self.batch, self.N, self.M)}")

    def _check_planes(self, planes, name="planes"):
        import torch
        _need(planes, name, torch.float32, self.batch * self.plane_elems, self.device)

    def _check_peaks(self, rec, cnt, words=PEAK_WORDS):
        import torch
        if rec.dim() != 4 or rec.shape[:2] != (self.batch, self.nspaces) or rec.shape[3] != words:
            raise ValueError(f"peak records must have shape ({self.batch}, {self.nspaces}, K, {words})")
        _need(rec, "peak records", torch.int32, rec.shape[0] * rec.shape[1] * rec.shape[2] * words, self.device)
        _need(cnt, "peak counts", torch.int32, self.batch * self.nspaces, self.device)

    def forward(self, images, planes=None, stream=None):
        self._check_images(images)
        if planes is None:
            planes = self.new_planes()
        self._check_planes(planes)
        funnel_forward(self.handle, images, planes, self.ws, stream)
        return planes

    def adjoint(self, d_planes, d_images=None, stream=None):
        import torch
        d_planes = d_planes.reshape(self.batch, self.plane_elems)
        if not d_planes.is_contiguous():
            d_planes = d_planes.contiguous()
        self._check_planes(d_planes, "d_planes")
        if d_images is None:
            d_images = torch.empty((self.batch, self.N, self.M), dtype=torch.float32, device=self.device)
        self._check_images(d_images, "d_images")
        funnel_adjoint(self.handle, d_planes, d_images, self.ws, stream)
        return d_images

    def peaks(self, planes, K: int = 16, threshold: float = 0.0, radius: int = 1, flags: int = 0,
              stream=None):
        """Returns (records int32 [B, nspaces, K, 7] on the device, counts int32 [B, nspaces])."""
        import torch
        self._check_planes(planes)
        ws = torch.empty(max(funnel_peaks_workspace_size(self.handle, K), 256), dtype=torch.uint8,
                         device=self.device)
        rec = torch.empty((self.batch, self.nspaces, K, PEAK_WORDS), dtype=torch.int32, device=self.device)
        cnt = torch.empty((self.batch, self.nspaces), dtype=torch.int32, device=self.device)
        funnel_peaks(self.handle, planes, K, threshold, radius, flags, rec, cnt, ws, stream)
        return rec, cnt

    def peaks_noalloc(self, planes, rec, cnt, threshold: float = 0.0, radius: int = 1, flags: int = 0,
                      stream=None) -> None:
        """peaks() into caller-provided records rec int32 [B, nspaces, K, 7]
        and counts cnt int32 [B, nspaces], with the library's static scratch
        instead of a workspace: nothing is allocated (funnel_peaks_noalloc;
        calls that overlap on one GPU share the scratch and must not)."""
        self._check_planes(planes)
        self._check_peaks(rec, cnt)
        funnel_peaks_noalloc(self.handle, planes, rec.shape[2], threshold, radius, flags, rec, cnt, stream)

    def verify(self, images, rec, cnt, half_width: int = 3, min_contrast: float = 0.1, min_length: int = 32,
               stream=None):
        """Sec. 4.5 line verification of peak lists from peaks(): returns the
        ft_line_check records as int32 [B, nspaces, K, 10] on the device
        (checks_to_numpy() reads them)."""
        import torch
        self._check_images(images)
        self._check_peaks(rec, cnt)
        out = torch.empty((rec.shape[0], rec.shape[1], rec.shape[2], LINE_CHECK_WORDS), dtype=torch.int32,
                          device=self.device)
        funnel_verify(self.handle, images, rec, cnt, rec.shape[2], half_width, min_contrast, min_length, out, stream)
        return out

    def refine(self, images, rec, cnt, iters: int = 4, stream=None):
        """Sub-cell refinement of peak lists from peaks(): ft_refined records
        as float32 [B, nspaces, K, 6] on the device (refined_to_numpy() reads
        them)."""
        import torch
        self._check_images(images)
        self._check_peaks(rec, cnt)
        K = rec.shape[2]
        ws = torch.empty(funnel_refine_workspace_size(self.handle, K), dtype=torch.uint8, device=self.device)
        out = torch.empty((rec.shape[0], rec.shape[1], K, REFINED_WORDS), dtype=torch.float32, device=self.device)
        funnel_refine(self.handle, images, rec, cnt, K, iters, out, ws, stream)
        return out


class RaggedPlan:
    """A plan for a batch of images of different sizes, packed back to back
    (each image's floats, then each image's plane block, 16-byte aligned)."""

    def __init__(self, shapes, spaces: int = FT_SPACE_BOTH):
        import torch
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        self.spaces = spaces
        self.nspaces = 2 if spaces == FT_SPACE_BOTH else 1
        self.image_offsets, self.plane_offsets = [], []
        io = po = 0
        for (r, c) in self.shapes:
            self.image_offsets.append(io)
            self.plane_offsets.append(po)
            io += (r * c + 3) // 4 * 4
            np_ = r + c
            pf = (np_ * c if spaces & FT_SPACE_REGULAR else 0) + (np_ * r if spaces & FT_SPACE_INVERSE else 0)
            po += (pf + 3) // 4 * 4
        self.handle = funnel_plan_create_ragged(self.shapes, self.image_offsets, self.plane_offsets, spaces)
        self.image_floats, self.plane_floats = funnel_buffer_elems(self.handle)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(max(funnel_workspace_size(self.handle), 256), dtype=torch.uint8, device=self.device)
        self.batch = len(self.shapes)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                funnel_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def schedule(self) -> int:
        return funnel_plan_schedule(self.handle)

    def set_schedule(self, schedule: int) -> None:
        """FT_SCHEDULE_CLASS_STREAMS or FT_SCHEDULE_QUEUE (one persistent
        launch per pass kind over a work queue of all classes' tiles)."""
        funnel_plan_set_schedule(self.handle, schedule)

    def pack(self, images):
        """List of [N, M] float32 arrays -> one flat device tensor."""
        import torch
        buf = np.zeros(self.image_floats, dtype=np.float32)
        for img, off in zip(images, self.image_offsets):
            buf[off:off + img.size] = np.asarray(img, dtype=np.float32).ravel()
        return torch.from_numpy(buf).to(self.device)

    def unpack_images(self, flat):
        h = flat.cpu().numpy()
        return [h[o:o + r * c].reshape(r, c) for (r, c), o in zip(self.shapes, self.image_offsets)]

    def unpack_planes(self, flat):
        """Flat planes tensor -> list of (regular or None, inverse or None) numpy arrays."""
        h = flat.cpu().numpy()
        out = []
        for (r, c), o in zip(self.shapes, self.plane_offsets):
            np_ = r + c
            reg = inv = None
            if self.spaces & FT_SPACE_REGULAR:
                reg = h[o:o + np_ * c].reshape(np_, c)
                o += np_ * c
            if self.spaces & FT_SPACE_INVERSE:
                inv = h[o:o + np_ * r].reshape(np_, r)
            out.append((reg, inv))
        return out

    def new_planes(self):
        import torch
        return torch.zeros(self.plane_floats, dtype=torch.float32, device=self.device)

    def forward(self, images_flat, planes=None, stream=None):
        import torch
        _need(images_flat, "images", torch.float32, self.image_floats, self.device)
        if planes is None:
            planes = self.new_planes()
        _need(planes, "planes", torch.float32, self.plane_floats, self.device)
        funnel_forward(self.handle, images_flat, planes, self.ws, stream)
        return planes

    def adjoint(self, d_planes, d_images=None, stream=None):
        import torch
        _need(d_planes, "d_planes", torch.float32, self.plane_floats, self.device)
        if d_images is None:
            d_images = torch.zeros(self.image_floats, dtype=torch.float32, device=self.device)
        _need(d_images, "d_images", torch.float32, self.image_floats, self.device)
        funnel_adjoint(self.handle, d_planes, d_images, self.ws, stream)
        return d_images

    def peaks(self, planes, K: int = 16, threshold: float = 0.0, radius: int = 1, flags: int = 0, stream=None):
        import torch
        _need(planes, "planes", torch.float32, self.plane_floats, self.device)
        ws = torch.empty(max(funnel_peaks_workspace_size(self.handle, K), 256), dtype=torch.uint8,
                         device=self.device)
        rec = torch.empty((self.batch, self.nspaces, K, PEAK_WORDS), dtype=torch.int32, device=self.device)
        cnt = torch.empty((self.batch, self.nspaces), dtype=torch.int32, device=self.device)
        funnel_peaks(self.handle, planes, K, threshold, radius, flags, rec, cnt, ws, stream)
        return rec, cnt

    def verify(self, images, rec, cnt, half_width: int = 3, min_contrast: float = 0.1, min_length: int = 32,
               stream=None):
        """Sec. 4.5 line verification of peak lists from peaks(): returns the
        ft_line_check records as int32 [B, nspaces, K, 10] on the device
        (checks_to_numpy() reads them)."""
        import torch
        _need(images, "images", torch.float32, self.image_floats, self.device)
        if rec.dim() != 4 or rec.shape[:2] != (self.batch, self.nspaces) or rec.shape[3] != PEAK_WORDS:
            raise ValueError(f"peak records must have shape ({self.batch}, {self.nspaces}, K, {PEAK_WORDS})")
        _need(rec, "peak records", torch.int32, rec.numel(), self.device)
        _need(cnt, "peak counts", torch.int32, self.batch * self.nspaces, self.device)
        out = torch.empty((rec.shape[0], rec.shape[1], rec.shape[2], LINE_CHECK_WORDS), dtype=torch.int32,
                          device=self.device)
        funnel_verify(self.handle, images, rec, cnt, rec.shape[2], half_width, min_contrast, min_length, out, stream)
        return out


class FunnelGraph:
    """An executable graph of a plan's forward and/or adjoint on fixed buffers."""

    def __init__(self, plan, what: int, images=None, planes=None, d_planes=None, d_images=None):
        self.handle = funnel_graph_create(plan.handle, what, images, planes, d_planes, d_images, plan.ws)
        self._keep = (plan, images, planes, d_planes, d_images)

    def launch(self, stream=None):
        funnel_graph_launch(self.handle, stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                funnel_graph_destroy(h)
            except Exception:
                pass
            self.handle = None


def refined_to_numpy(out):
    """Device ft_refined records [B, nspaces, K, 6] -> numpy structured array [B, nspaces, K]."""
    a = np.ascontiguousarray(out.cpu().numpy())
    return a.view(REFINED_DTYPE).reshape(a.shape[:3])


def checks_to_numpy(out):
    """Device ft_line_check records [B, nspaces, K, 10] -> numpy structured array [B, nspaces, K]."""
    a = np.ascontiguousarray(out.cpu().numpy())
    return a.view(LINE_CHECK_DTYPE).reshape(a.shape[:3])


def peaks_to_numpy(rec, cnt) -> list:
    """Device peak records -> list (per image) of lists (per space) of numpy records."""
    r = rec.cpu().numpy()
    c = cnt.cpu().numpy()
    out = []
    for b in range(r.shape[0]):
        per = []
        for s in range(r.shape[1]):
            per.append(np.ascontiguousarray(r[b, s, :c[b, s]]).view(PEAK_DTYPE).reshape(-1))
        out.append(per)
    return out


def _autograd():
    import torch

    class FunnelTransform(torch.autograd.Function):
        """planes = F(images); the backward applies the hand-written adjoint.
        The operator is linear, so nothing is saved for the backward."""

        @staticmethod
        def forward(ctx, images, plan: FunnelPlan):
            ctx.plan = plan
            return plan.forward(images.contiguous())

        @staticmethod
        def backward(ctx, grad_planes):
            return ctx.plan.adjoint(grad_planes.contiguous()), None

    return FunnelTransform


_FT = None


def funnel_transform(images, plan: FunnelPlan):
    """Differentiable forward: ``planes = funnel_transform(images, plan)``."""
    global _FT
    if _FT is None:
        _FT = _autograd()
    return _FT.apply(images, plan)


class VolumePlan:
    """A volume plan (App. A) plus its workspace for a fixed batch shape on
    the current device.  ``spaces``: FT_VOL_SPACE_Z (planes within 45 degrees
    of the z axis), _X, _Y or FT_VOL_SPACE_ALL."""

    def __init__(self, batch: int, depth: int, rows: int, cols: int, padded_len: int = 0,
                 spaces: int = FT_VOL_SPACE_Z):
        import torch
        self.batch, self.Nz, self.Ny, self.Nx, self.spaces = batch, depth, rows, cols, spaces
        self.handle = funnel_volume_plan_create(batch, depth, rows, cols, padded_len, spaces)
        self.Lp = self.Nzp = funnel_volume_padded_len(self.handle)
        self.param_elems = funnel_volume_param_elems(self.handle)
        self.device = torch.device("cuda", torch.cuda.current_device())
        ws = funnel_volume_workspace_size(self.handle)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)
        # (name, rows, cols) of the spaces computed, in their order in the parameter block
        geo = {"z": (depth, rows, cols), "x": (cols, depth, rows), "y": (rows, depth, cols)}
        self.space_list = [(n, geo[n][1], geo[n][2]) for i, n in enumerate(VOLUME_SPACE_NAMES) if spaces & (1 << i)]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                funnel_volume_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def nspaces(self) -> int:
        return len(self.space_list)

    def new_params(self):
        import torch
        return torch.empty((self.batch, self.param_elems), dtype=torch.float32, device=self.device)

    def views(self, params) -> dict:
        """Per space name, the parameter volumes as [B, Lp, rows, cols] views."""
        out, off = {}, 0
        for name, r, c in self.space_list:
            n = self.Lp * r * c
            out[name] = params[:, off:off + n].view(self.batch, self.Lp, r, c)
            off += n
        return out

    def forward(self, volumes, params=None, stream=None):
        import torch
        _need(volumes, "volumes", torch.float32, self.batch * self.Nz * self.Ny * self.Nx, self.device)
        if tuple(volumes.shape) != (self.batch, self.Nz, self.Ny, self.Nx):
            raise ValueError(f"volumes must have shape {(self.batch, self.Nz, self.Ny, self.Nx)}")
        if params is None:
            params = self.new_params()
        _need(params, "params", torch.float32, self.batch * self.param_elems, self.device)
        funnel_volume_forward(self.handle, volumes, params, self.ws, stream)
        return params

    def peaks(self, params, K: int = 16, threshold: float = 0.0, radius: int = 1, flags: int = 0, stream=None):
        """Returns (records int32 [B, nspaces, K, 9] on the device, counts int32 [B, nspaces])."""
        import torch
        _need(params, "params", torch.float32, self.batch * self.param_elems, self.device)
        ws = torch.empty(max(funnel_volume_peaks_workspace_size(self.handle, K), 256), dtype=torch.uint8,
                         device=self.device)
        rec = torch.empty((self.batch, self.nspaces, K, PLANE_PEAK_WORDS), dtype=torch.int32, device=self.device)
        cnt = torch.empty((self.batch, self.nspaces), dtype=torch.int32, device=self.device)
        funnel_volume_peaks(self.handle, params, K, threshold, radius, flags, rec, cnt, ws, stream)
        return rec, cnt

    def autotune(self, stream=None) -> list[dict]:
        return funnel_volume_autotune(self.handle, stream, cap=12)


def plane_peaks_to_numpy(rec, cnt):
    """Device plane-peak records -> list (per volume) of lists (per space) of numpy records."""
    r = rec.cpu().numpy()
    c = cnt.cpu().numpy()
    return [[np.ascontiguousarray(r[b, s, :c[b, s]]).view(PLANE_PEAK_DTYPE).reshape(-1) for s in range(r.shape[1])]
            for b in range(r.shape[0])]
