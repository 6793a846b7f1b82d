"""ctypes binding of libtrhip.so (include/trhip.h): argument marshalling only.

Every computation happens in the HIP library; this module converts Python /
numpy / torch arguments into the C structures and raw pointers of the ABI.
The library must have been built (``paper_2510_25660_amd.build``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libtrhip.so")

TRHIP_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "HIP", 4: "UNSUPPORTED", 5: "BAD_HANDLE"}

FLAG_PIXEL_CENTRE = 1 << 0
FLAG_ACCUMULATE = 1 << 1
FLAG_FROZEN_PROPOSAL = 1 << 2
FLAG_NLOS_AREA_SAMPLING = 1 << 3
FLAG_DETERMINISTIC = 1 << 4

BUILDERS = {"ploc": 0, "lbvh": 1}

KERNELS = {"auto": 0, "path": 1, "wavefront": 2, "deferred": 3}

EXPORTED_SYMBOLS = (
    "trhip_scene_create", "trhip_scene_destroy", "trhip_scene_get_info", "trhip_render_transient",
    "trhip_render_transient_backward", "trhip_render_transient_counted", "trhip_status_string",
    "trhip_last_error", "trhip_version", "trhip_batch_create", "trhip_batch_render", "trhip_batch_get_info",
    "trhip_batch_destroy", "trhip_poisson_noise", "trhip_render_phasor", "trhip_render_transient_tangent",
    "trhip_render_transient_records", "trhip_numerics_probe", "trhip_render_transient_noalloc",
)

PROBES = {"sincos2pi": 0, "log1m": 1, "philox": 2, "div": 3, "sqrt": 4}

COUNT_NAMES = ("nodes", "tris", "rays", "shadow_rays", "vertices", "draws", "contributions", "wave_nodes",
               "wave_tris", "wave_vertices")


# numpy layout of trhip_record
RECORD_FIELDS = [("pixel", "<u4"), ("sample", "<u4"), ("vertex", "<i4"), ("bin", "<i4"), ("value", "<f4"),
                 ("tof", "<f4"), ("tri", "<i4"), ("reserved", "<u4")]


class TrhipError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"trhip {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [
        ("vertices", C.POINTER(C.c_float)),
        ("n_vertices", C.c_uint32),
        ("indices", C.POINTER(C.c_uint32)),
        ("n_triangles", C.c_uint32),
        ("mat_type", C.POINTER(C.c_uint8)),
        ("albedo", C.POINTER(C.c_float)),
        ("roughness", C.POINTER(C.c_float)),
        ("light_pos", C.c_float * 3),
        ("light_intensity", C.c_float),
        ("sensor", C.c_int32),
        ("width", C.c_uint32),
        ("height", C.c_uint32),
        ("cam_origin", C.c_float * 3),
        ("cam_right", C.c_float * 3),
        ("cam_up", C.c_float * 3),
        ("cam_fwd", C.c_float * 3),
        ("tan_x", C.c_float),
        ("tan_y", C.c_float),
        ("scan_points", C.POINTER(C.c_float)),
        ("wall_normal", C.c_float * 3),
        ("wall_albedo", C.c_float),
        ("laser_power", C.c_float),
        ("sigma_t", C.c_float),
        ("medium_albedo", C.c_float),
        ("n_bins", C.c_uint32),
        ("bin_width", C.c_float),
        ("bin_start", C.c_float),
        ("camera_unwarp", C.c_int32),
        ("bvh_builder", C.c_int32),
        ("ior", C.POINTER(C.c_float)),
        ("delay", C.POINTER(C.c_float)),
        ("medium_ior", C.c_float),
    ]


class RenderDesc(C.Structure):
    _fields_ = [
        ("spp", C.c_uint32),
        ("sample_offset", C.c_uint32),
        ("norm_spp", C.c_uint32),
        ("max_depth", C.c_uint32),
        ("seed", C.c_uint64),
        ("stream_id", C.c_uint32),
        ("flags", C.c_uint32),
        ("albedo_override", C.c_void_p),
        ("roughness_override", C.c_void_p),
        ("tile_pixels", C.c_uint32),
        ("block_size", C.c_uint32),
        ("kernel", C.c_uint32),
    ]


class SceneInfo(C.Structure):
    _fields_ = [
        ("n_triangles", C.c_uint32),
        ("n_pixels", C.c_uint32),
        ("n_bins", C.c_uint32),
        ("bvh_internal_nodes", C.c_uint32),
        ("bvh_depth", C.c_uint32),
        ("box_pad", C.c_float),
        ("device_bytes", C.c_size_t),
    ]


class BatchOpts(C.Structure):
    _fields_ = [
        ("block_size", C.c_uint32),
        ("tile_pixels", C.c_uint32),
        ("groups_per_cu", C.c_uint32),
        ("kernel", C.c_uint32),
        ("autotune", C.c_int32),
    ]


class BatchInfo(C.Structure):
    _fields_ = [
        ("n_scenes", C.c_uint32),
        ("n_items", C.c_uint32),
        ("block_size", C.c_uint32),
        ("tile_pixels", C.c_uint32),
        ("groups", C.c_uint32),
        ("kernel", C.c_uint32),
        ("stack_depth", C.c_uint32),
        ("lds_bytes", C.c_size_t),
        ("candidates", C.c_uint32),
        ("tune_ms", C.c_float),
        ("best_ms", C.c_float),
        ("n_classes", C.c_uint32),
    ]


_lib = None


def lib():
    """Load libtrhip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libtrhip.so not built ({LIB_PATH}); run paper_2510_25660_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.trhip_scene_create.argtypes = [C.POINTER(SceneDesc), vp, C.POINTER(vp)]
        L.trhip_scene_create.restype = C.c_int
        L.trhip_scene_destroy.argtypes = [vp]
        L.trhip_scene_destroy.restype = C.c_int
        L.trhip_scene_get_info.argtypes = [vp, C.POINTER(SceneInfo)]
        L.trhip_scene_get_info.restype = C.c_int
        L.trhip_render_transient.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, vp, vp]
        L.trhip_render_transient.restype = C.c_int
        L.trhip_render_transient_backward.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, vp, vp, vp]
        L.trhip_render_transient_backward.restype = C.c_int
        L.trhip_render_transient_counted.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, vp,
                                                     C.POINTER(C.c_uint64), vp]
        L.trhip_render_transient_counted.restype = C.c_int
        L.trhip_batch_create.argtypes = [C.POINTER(vp), C.POINTER(RenderDesc), C.c_uint32, C.POINTER(vp),
                                         C.POINTER(BatchOpts), vp, C.POINTER(vp)]
        L.trhip_batch_create.restype = C.c_int
        L.trhip_batch_render.argtypes = [vp, vp]
        L.trhip_batch_render.restype = C.c_int
        L.trhip_batch_get_info.argtypes = [vp, C.POINTER(BatchInfo)]
        L.trhip_batch_get_info.restype = C.c_int
        L.trhip_batch_destroy.argtypes = [vp]
        L.trhip_batch_destroy.restype = C.c_int
        L.trhip_render_phasor.argtypes = [vp, C.POINTER(RenderDesc), C.POINTER(C.c_float), C.c_uint32, vp, vp, vp]
        L.trhip_render_phasor.restype = C.c_int
        L.trhip_render_transient_tangent.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, vp, vp, vp, vp]
        L.trhip_render_transient_tangent.restype = C.c_int
        L.trhip_render_transient_records.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, C.c_uint64,
                                                     C.POINTER(C.c_uint64), vp, vp, vp, vp]
        L.trhip_render_transient_records.restype = C.c_int
        L.trhip_render_transient_noalloc.argtypes = [vp, C.POINTER(RenderDesc), vp, vp, vp, vp]
        L.trhip_render_transient_noalloc.restype = C.c_int
        L.trhip_numerics_probe.argtypes = [C.c_int32, vp, vp, C.c_uint64, C.c_uint64, vp]
        L.trhip_numerics_probe.restype = C.c_int
        L.trhip_poisson_noise.argtypes = [vp, vp, C.c_uint64, C.c_float, C.c_uint64, vp]
        L.trhip_poisson_noise.restype = C.c_int
        L.trhip_status_string.argtypes = [C.c_int]
        L.trhip_status_string.restype = C.c_char_p
        L.trhip_last_error.argtypes = []
        L.trhip_last_error.restype = C.c_char_p
        L.trhip_version.argtypes = []
        L.trhip_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(status: int):
    if status != TRHIP_OK:
        raise TrhipError(status, lib().trhip_last_error().decode())
