"""ctypes declarations of the libedgemask C ABI (include/edge_masks.h).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libedgemask.so")

EDGE_OK = 0
EDGE_ERR_INVALID = -1
EDGE_ERR_ALIGN = -2
EDGE_ERR_ALIAS = -3
EDGE_ERR_HIP = -4
EDGE_ERR_WORKSPACE = -5
EDGE_ERR_UNSUPPORTED = -6

EDGE_BORDER_WHITE = 0
EDGE_BORDER_BLACK = 1
EDGE_MODE_MASKS = 0
EDGE_MODE_FULL = 1
EDGE_FLAG_CLAUSE2_ONLY = 1 << 0
EDGE_FLAG_INVERT_OUT = 1 << 1
EDGE_FLAG_PLANNED = 1 << 2
EDGE_FLAG_PEEL_EDGE = 1 << 3
EDGE_PEEL_MAX_ITERATIONS = 30
EDGE_MAX_HEIGHT = 1 << 30
EDGE_BATCH_NOALLOC_MAX_IMAGES = 16384

c_i32, c_i64, c_u32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p


class EdgeImageDesc(ctypes.Structure):
    _fields_ = [("offset_words", c_i64), ("height", c_i32), ("width", c_i32),
                ("stride_words", c_i64)]


EDGE_CACHE_AUTO = 0
EDGE_CACHE_NORMAL = 1
EDGE_CACHE_STREAM = 2
EDGE_SHAPE_STRIP = 0
EDGE_SHAPE_TILE = 1
EDGE_SHAPE_TILE_XCD = 2
EDGE_SHAPE_BAND = 3
EDGE_SHAPE_BAND_XCD = 4
EDGE_TILE_MAX_ROWS = 16


class EdgeLaunchCfg(ctypes.Structure):
    _fields_ = [("vec_words", c_i32), ("rows_per_tile", c_i32), ("waves_per_block", c_i32),
                ("blocks_per_cu", c_i32), ("cache_policy", c_i32), ("shape", c_i32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d: dict) -> "EdgeLaunchCfg":
        return cls(int(d["vec_words"]), int(d["rows_per_tile"]), int(d["waves_per_block"]),
                   int(d.get("blocks_per_cu", 1)), int(d.get("cache_policy", EDGE_CACHE_AUTO)),
                   int(d.get("shape", EDGE_SHAPE_STRIP)))


class EdgeError(RuntimeError):
    """A libedgemask call returned an error status."""

    def __init__(self, status: int, message: str, hip_error: int = 0):
        super().__init__(f"{message} (status {status}" +
                         (f", hipError {hip_error})" if hip_error else ")"))
        self.status = status
        self.hip_error = hip_error


_SIGNATURES = {
    "edge_masks": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int, c_vp]),
    "edge_full": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int, c_u32,
                                 c_vp]),
    "edge_image_launch": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, c_u32, ctypes.POINTER(EdgeLaunchCfg), c_vp]),
    "edge_directions": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(EdgeLaunchCfg), c_vp]),
    "edge_threshold_pack": (ctypes.c_int, [c_vp, c_i64, ctypes.c_int, c_vp, c_i64, c_i64, c_i64,
                                           ctypes.c_int, c_vp]),
    "edge_threshold_edges": (ctypes.c_int, [c_vp, c_i64, ctypes.c_int, c_vp, c_i64, c_i64, c_i64,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int, c_u32,
                                            ctypes.POINTER(EdgeLaunchCfg), c_vp]),
    "edge_peel": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, c_u32, ctypes.POINTER(EdgeLaunchCfg), c_vp]),
    "edge_masks_staged": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_i64, c_i64, c_i64,
                                         ctypes.c_int, ctypes.c_int, c_vp]),
    "edge_default_cfg": (ctypes.c_int, [c_i64, c_i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(EdgeLaunchCfg)]),
    "edge_batch_workspace_bytes": (c_i64, [c_i32]),
    "edge_batch_check": (ctypes.c_int, [c_vp, c_i32, c_i64, ctypes.c_int]),
    "edge_batch": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i32, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, c_u32, ctypes.POINTER(EdgeLaunchCfg), c_vp, c_i64,
                                  c_vp]),
    "edge_batch_noalloc": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i32, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, c_u32,
                                          ctypes.POINTER(EdgeLaunchCfg), c_vp]),
    "edge_batch_plan": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i32, ctypes.c_int,
                                       ctypes.POINTER(EdgeLaunchCfg), c_vp, c_i64,
                                       ctypes.POINTER(c_i64)]),
    "edge_batch_graph_create": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i32, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, c_u32,
                                               ctypes.POINTER(EdgeLaunchCfg), c_vp, c_i64,
                                               ctypes.POINTER(c_vp)]),
    "edge_graph_launch": (ctypes.c_int, [c_vp, c_vp]),
    "edge_graph_destroy": (ctypes.c_int, [c_vp]),
    "edge_copy_bytes": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp]),
    "edge_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "edge_last_hip_error": (ctypes.c_int, []),
    "edge_abi_version": (ctypes.c_int, []),
}

ABI_VERSION = 2
_lib = None


def load() -> ctypes.CDLL:
    """Load libedgemask.so; raise ImportError when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built. Build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()'); there is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.edge_abi_version() != ABI_VERSION:
        raise ImportError("libedgemask.so ABI version mismatch; rebuild it")
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != EDGE_OK:
        lib = load()
        msg = lib.edge_status_string(status).decode()
        raise EdgeError(status, msg, lib.edge_last_hip_error() if status == EDGE_ERR_HIP else 0)
