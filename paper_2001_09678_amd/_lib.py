"""ctypes view of include/mpv.h. Loading fails loudly when the HIP library is missing:
there is no CPU fallback anywhere in the product path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpv.so")

MPV_OK, MPV_ERR_INVALID_ARG, MPV_ERR_UNSUPPORTED, MPV_ERR_WORKSPACE, MPV_ERR_OVERFLOW, MPV_ERR_DEVICE = range(6)
MPV_AGG_U16, MPV_AGG_I32 = 0, 1
MPV_MERGE_SUM, MPV_MERGE_LAYERED, MPV_MERGE_LAYERED_OCC = 0, 1, 2
MPV_PROP_NEAREST, MPV_PROP_PAPER = 0, 1
MPV_DATA_CENSUS, MPV_DATA_SSIM = 0, 1
MPV_MAX_BLOCK = 32
MPV_BAND_LANES_LINE = 1
MPV_MAX_LEVELS = 4
MPV_MAX_DISP = 256
MPV_MAX_WIDTH = 4096
MPV_ROAD_MAX_HEIGHT = 4096
MPV_PYRAMID_NOALLOC_MAX_BYTES = 144 << 20
STAGE_DOWNSAMPLE, STAGE_CENSUS, STAGE_SCAN, STAGE_REDUCE, STAGE_PROPAGATE = range(5)


class Image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int32)]


class Band(C.Structure):
    _fields_ = [("lo", C.c_void_p), ("len", C.c_void_p), ("cap", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("num_disp", C.c_int32), ("census_radius", C.c_int32), ("num_paths", C.c_int32),
                ("lambda_", C.c_int32), ("tau", C.c_int32), ("lr_max_diff", C.c_int32),
                ("agg_type", C.c_int32), ("merge", C.c_int32), ("grad_sigma", C.c_int32),
                ("data_term", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("full_lanes", C.c_int32), ("band_lanes", C.c_int32),
                ("order", C.c_int32)]


class PyramidParams(C.Structure):
    _fields_ = [("base", Params), ("levels", C.c_int32), ("band_radius", C.c_int32),
                ("sched", Schedule), ("propagation", C.c_int32), ("block", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("left", Image), ("right", Image), ("num_disp", C.c_int32), ("disp", C.c_void_p),
                ("disp_right", C.c_void_p), ("disp_raw", C.c_void_p)]


class PyramidOut(C.Structure):
    _fields_ = [("disp", C.c_void_p), ("disp_raw", C.c_void_p), ("disp_right", C.c_void_p),
                ("level_raw", C.c_void_p * MPV_MAX_LEVELS)]


class MPVError(RuntimeError):
    def __init__(self, status: int, what: str):
        name = lib().mpv_status_string(status).decode()
        super().__init__(f"{what}: {name}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run paper_2001_09678_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_size_t
        i32, u32 = C.c_int32, C.c_uint32
        sigs = {
            "mpv_status_string": ([i32], C.c_char_p),
            "mpv_census": ([C.POINTER(Image), P, P], i32),
            "mpv_downsample": ([C.POINTER(Image), P, P], i32),
            "mpv_cost": ([C.POINTER(Params), C.POINTER(Image), C.POINTER(Image), C.POINTER(Band), P, P], i32),
            "mpv_aggregate": ([C.POINTER(Params), P, i32, i32, C.POINTER(Band), u32, P, P], i32),
            "mpv_disparity": ([C.POINTER(Params), P, i32, i32, C.POINTER(Band), P, P, P, P], i32),
            "mpv_pyramid_workspace_bytes": ([C.POINTER(PyramidParams), i32, i32], S),
            "mpv_pyramid": ([C.POINTER(PyramidParams), C.POINTER(Image), C.POINTER(Image),
                             C.POINTER(PyramidOut), P, S, P], i32),
            "mpv_pyramid_noalloc": ([C.POINTER(PyramidParams), C.POINTER(Image), C.POINTER(Image),
                                     C.POINTER(PyramidOut), P], i32),
            "mpv_match_workspace_bytes": ([C.POINTER(Params), i32, i32, C.POINTER(Band)], S),
            "mpv_match": ([C.POINTER(Params), C.POINTER(Image), C.POINTER(Image), C.POINTER(Band),
                           P, P, P, P, S, P], i32),
            "mpv_set_timing_events": ([i32, i32, P, P], i32),
            "mpv_vdisparity": ([P, i32, i32, i32, i32, P, P], i32),
            "mpv_udisparity": ([P, i32, i32, i32, i32, P, P], i32),
            "mpv_road_workspace_bytes": ([i32, i32], S),
            "mpv_road": ([P, i32, i32, i32, P, P, P, S, P], i32),
            "mpv_batch_create": ([C.POINTER(PyramidParams), C.POINTER(BatchItem), i32, C.POINTER(P)], i32),
            "mpv_batch_workspace_bytes": ([P], S),
            "mpv_batch_bind": ([P, P, S, P], i32),
            "mpv_batch_run": ([P, P], i32),
            "mpv_batch_run_graph": ([P, P], i32),
            "mpv_batch_run_items": ([P, P, i32, P], i32),
            "mpv_batch_destroy": ([P], None),
            "mpv_lb_coarse_workspace_bytes": ([C.POINTER(Params), i32, i32], S),
            "mpv_lb_coarse": ([C.POINTER(Params), C.POINTER(Image), C.POINTER(Image), P, P, P, P, S, P], i32),
            "mpv_lb_packed_elems": ([i32, i32], S),
            "mpv_lb_packed_bwd_elems": ([i32, i32], S),
            "mpv_lb_pack": ([P, i32, i32, P, P, P], i32),
            "mpv_lb_conv": ([P, i32, i32, i32, i32, P, P, i32, i32, P, i32, P, i32, i32, P], i32),
            "mpv_lb_dw_workspace_bytes": ([i32, i32, i32, i32, i32], S),
            "mpv_lb_conv_dw": ([P, P, i32, i32, i32, i32, i32, i32, P, P, P, S, P], i32),
            "mpv_lb_loss": ([P, P, P, i32, i32, i32, i32, i32, C.c_float, C.c_float, P, P, P], i32),
            "mpv_lb_adam": ([P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, i32, P], i32),
            "mpv_lb_bands": ([P, P, i32, i32, i32, i32, i32, C.c_float, P, P, P, P], i32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != MPV_OK:
        raise MPVError(status, what)
