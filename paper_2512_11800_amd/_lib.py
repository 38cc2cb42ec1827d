"""ctypes binding of libmb3dgs.so (argument marshalling only).

Mirrors the structs and entry points of include/mb3dgs.h. The library must
be built (``paper_2512_11800_amd.build.build()``); loading fails loudly when
it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmb3dgs.so")

MB_OK = 0
MB_ERR_ARG = -1
MB_ERR_UNSUPPORTED = -2
MB_ERR_WORKSPACE = -3
MB_ERR_HIP = -4
MB_MAX_CAMERAS = 16
MB_SAVED_FLOATS_PER_PIXEL = 8
MB_STAGE_COUNT = 10
MB_ENTRIES_ON_DEVICE = -1
STAGES = ("preprocess", "scan", "emit", "sort", "lists", "render_forward", "render_backward",
          "gradients", "mlp", "render_consume")


class MbGaussians(ctypes.Structure):
    _fields_ = [("n", c_int32), ("sh_degree", c_int32),
                ("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p),
                ("densities", c_void_p), ("colors", c_void_p)]


class MbCamera(ctypes.Structure):
    _fields_ = [("world_to_cam", c_float * 12), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32),
                ("t_near", c_float), ("background", c_float * 3)]


class MbOptions(ctypes.Structure):
    _fields_ = [("n_moments", c_int32), ("n_intervals", c_int32), ("kappa", c_float),
                ("conf_c", c_float), ("beta", c_float), ("eps", c_float), ("basis", c_int32),
                ("surrogate", c_void_p), ("full_coverage", c_int32), ("reserved", c_int32)]


class MbAdcParams(ctypes.Structure):
    _fields_ = [("min_opacity", c_float), ("grad_threshold", c_float), ("split_scale", c_float)]


class MbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mb3dgs error {code}: {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes) of every entry point declared in include/mb3dgs.h
SIGNATURES = [
    ("mb_default_options", None, [POINTER(MbOptions)]),
    ("mb_last_error", ctypes.c_char_p, []),
    ("mb_version", c_int32, []),
    ("mb_gauss_workspace_bytes", c_size_t, [c_int32, c_int32]),
    ("mb_pair_workspace_bytes", c_size_t, [c_int64, c_int32, c_int32, c_int32]),
    ("mb_pair_capacity", c_int64, [c_size_t, c_int32, c_int32, c_int32]),
    ("mb_entry_count", c_int32, [c_int32, c_int32, c_void_p, c_size_t, POINTER(c_int64), c_void_p]),
    ("mb_project", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), POINTER(MbOptions),
                             c_void_p, c_void_p]),
    ("mb_prepare", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32, POINTER(MbOptions),
                             c_void_p, c_size_t, POINTER(c_int64), c_void_p]),
    ("mb_render_forward", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                    POINTER(MbOptions), c_void_p, c_size_t, c_void_p, c_size_t,
                                    c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mb_render_forward_noalloc", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                            POINTER(MbOptions), c_void_p, c_void_p, c_void_p,
                                            POINTER(c_int64), c_void_p]),
    ("mb_table_workspace_bytes", c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    ("mb_render_forward_tabulated", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                              POINTER(MbOptions), c_void_p, c_size_t, c_void_p, c_size_t,
                                              c_int64, c_void_p, c_int32, c_void_p, c_size_t, c_void_p,
                                              c_void_p, c_void_p]),
    ("mb_mlp_param_count", c_int32, []),
    ("mb_mlp_packed_bytes", c_size_t, []),
    ("mb_mlp_workspace_bytes", c_size_t, [c_int64]),
    ("mb_mlp_pack", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("mb_mlp_forward", c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    ("mb_mlp_loss_grad", c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    ("mb_adam_step", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                               c_float, c_float, c_float, c_float, c_void_p]),
    ("mb_profile_enable", None, [c_int32]),
    ("mb_profile_read", c_int32, [POINTER(ctypes.c_double), POINTER(c_int64), c_int32]),
    ("mb_render_backward", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                     POINTER(MbOptions), c_void_p, c_size_t, c_void_p, c_size_t,
                                     c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mb_render_forward_harvest", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                            POINTER(MbOptions), c_void_p, c_size_t, c_void_p,
                                            c_size_t, c_int64, c_float, ctypes.c_uint32, c_void_p,
                                            c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mb_query_workspace_bytes", c_size_t, [c_int32, c_int32, c_int32, c_int64]),
    ("mb_render_forward_surrogate", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                              POINTER(MbOptions), c_void_p, c_size_t, c_void_p,
                                              c_size_t, c_int64, c_void_p, c_void_p, c_size_t,
                                              c_int64, c_void_p, c_void_p, c_void_p]),
    ("mb_query_workspace_bytes_backward", c_size_t, [c_int32, c_int32, c_int32, c_int64]),
    ("mb_dssim_workspace_bytes", c_size_t, [c_int32, c_int32, c_int32]),
    ("mb_l1_workspace_bytes", c_size_t, []),
    ("mb_l1", c_int32, [c_void_p, c_void_p, c_int64, c_float, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("mb_dssim", c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p, c_void_p,
                           c_void_p, c_size_t, c_void_p]),
    ("mb_view_independent_opacity", c_int32, [POINTER(MbGaussians), c_void_p, c_void_p]),
    ("mb_density_from_opacity", c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mb_adc_accumulate", c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mb_adc_workspace_bytes", c_size_t, [c_int32]),
    ("mb_adc_plan", c_int32, [POINTER(MbGaussians), c_void_p, c_void_p, POINTER(MbAdcParams), c_void_p,
                              c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("mb_adc_apply", c_int32, [POINTER(MbGaussians), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p]),
    ("mb_render_backward_surrogate", c_int32, [POINTER(MbGaussians), POINTER(MbCamera), c_int32,
                                               POINTER(MbOptions), c_void_p, c_size_t, c_void_p,
                                               c_size_t, c_int64, c_void_p, c_void_p, c_size_t,
                                               c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                               c_void_p, c_void_p, c_void_p, c_void_p]),
]


def load():
    """Load libmb3dgs.so (once) and declare its entry points."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2512_11800_amd.build.build() "
                           "(the HIP library is required, there is no CPU path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != MB_OK:
        msg = load().mb_last_error()
        raise MbError(rc, msg.decode() if msg else "")


def profile_enable(on: bool = True, stages=None):
    """Time every stage (``on``), none, or only the named ``stages``."""
    if stages is not None:
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
    else:
        mask = (1 << MB_STAGE_COUNT) - 1 if on else 0
    load().mb_profile_enable(mask)


def profile_read():
    """Stage totals since the last read: {stage: (ms, calls)} (waits for them)."""
    ms = (ctypes.c_double * MB_STAGE_COUNT)()
    calls = (c_int64 * MB_STAGE_COUNT)()
    load().mb_profile_read(ms, calls, MB_STAGE_COUNT)
    return {name: (ms[i], calls[i]) for i, name in enumerate(STAGES)}
