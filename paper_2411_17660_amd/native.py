"""ctypes binding of libgsr.so (include/gsr.h): argument marshalling only.

Every step of the rasterizer runs in the library's HIP kernels; this module
passes device pointers, sizes and the current HIP stream, and raises on any
non-zero status.  There is no fallback: if the library is missing the import
of the binding fails.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

GSR_OK = 0
STATUS = {1: "INVALID_ARGUMENT", 2: "CAPACITY", 3: "OUT_OF_MEMORY", 4: "HIP_ERROR",
          5: "STATE", 6: "UNSUPPORTED"}
FLAG_NO_XCD_REMAP = 1
FLAG_TIMING = 2
FLAG_COUNT_PAIRS = 4
FLAG_MEDIAN_DEPTH = 8
STAGES = ["preprocess", "depth_sort", "offsets", "keygen", "tile_sort", "ranges",
          "composite_fwd", "loss", "composite_bwd", "preprocess_bwd"]

EXPORTS = ["gsr_create", "gsr_destroy", "gsr_last_error", "gsr_forward", "gsr_forward_surfel",
           "gsr_backward", "gsr_backward_surfel", "gsr_normal_consistency",
           "gsr_loss_l1", "gsr_loss_l1_noalloc", "gsr_step_l1", "gsr_loss_render", "gsr_step_render",
           "gsr_densify_stats", "gsr_mcmc_noise", "gsr_mcmc_relocate", "gsr_check_overflow", "gsr_debug_stats",
           "gsr_debug_timings", "gsr_debug_lists", "gsr_debug_grad2d", "gsr_debug_copy",
           "gsr_autotune",
           "gsr_adam_step"]
TILE_SHAPES = [(16, 16), (8, 8), (32, 8), (16, 8), (32, 16)]
LDS_BATCHES = [32, 64, 128]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float)]


class Settings(C.Structure):
    _fields_ = [("sh_degree", C.c_int32), ("background", C.c_float * 3),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("lds_batch", C.c_int32),
                ("key_capacity", C.c_int64), ("flags", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("n_records", C.c_int64), ("n_keys", C.c_int64), ("n_tiles", C.c_int64),
                ("n_pixels", C.c_int64), ("key_capacity", C.c_int64), ("epoch", C.c_uint32),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("n_pairs", C.c_int64),
                ("n_culled", C.c_int64), ("n_nonfinite", C.c_int64)]


class GsrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsr status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libgsr.so and declare its C signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2411_17660_amd/build.py "
                          "(the rasterizer has no non-HIP fallback)")
    # PyTorch ships its own HIP runtime; load it first so that libgsr binds to
    # that same runtime (same soname) instead of pulling in a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    V, I64, I32, F32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
    S = C.c_int32
    lib.gsr_create.argtypes = [C.POINTER(V), I32]
    lib.gsr_destroy.argtypes = [V]
    lib.gsr_last_error.argtypes = [V]
    lib.gsr_last_error.restype = C.c_char_p
    lib.gsr_forward.argtypes = [V, C.POINTER(Settings), I64, V, V, V, V, V, I32,
                                C.POINTER(Camera), V, V, V, V, V]
    lib.gsr_forward_surfel.argtypes = [V, C.POINTER(Settings), I64, V, V, V, V, V, I32,
                                       C.POINTER(Camera), V, V, V, V, V, V, V]
    lib.gsr_backward.argtypes = [V] + [V] * 9 + [V]
    lib.gsr_backward_surfel.argtypes = [V] + [V] * 11 + [V]
    lib.gsr_normal_consistency.argtypes = [V, I32, C.POINTER(Camera), V, V, V, F32, V, V, V, V,
                                           V]
    lib.gsr_loss_l1.argtypes = [V, V, V, F32, V, V, V, V, V]
    lib.gsr_loss_l1_noalloc.argtypes = [V, V, V, F32, V, V, V, V, V]
    lib.gsr_step_l1.argtypes = [V, C.POINTER(Settings), I64, V, V, V, V, V, I32,
                                C.POINTER(Camera), V, V, V, F32, V, V, V, V, V, V, V, V, V, V,
                                V]
    lib.gsr_loss_render.argtypes = [V, V, V, V, V, F32, F32, V, V, V, V, V, V]
    lib.gsr_step_render.argtypes = [V, C.POINTER(Settings), I64, V, V, V, V, V, I32,
                                    C.POINTER(Camera), V, V, V, F32, F32, V, V, V, V, V, V, V,
                                    V, V, V, V, V]
    lib.gsr_densify_stats.argtypes = [V, V, V, V]
    lib.gsr_mcmc_noise.argtypes = [V, I64, V, V, V, V, V, F32, V]
    lib.gsr_mcmc_relocate.argtypes = [V, I64, I32, V, V, V, V, V, V, V]
    lib.gsr_check_overflow.argtypes = [V, V]
    lib.gsr_debug_stats.argtypes = [V, C.POINTER(Stats), V]
    lib.gsr_debug_lists.argtypes = [V] + [V] * 8 + [V]
    lib.gsr_debug_grad2d.argtypes = [V, V, V]
    lib.gsr_debug_copy.argtypes = [V, V, V, C.c_uint64, V]
    lib.gsr_debug_timings.argtypes = [V, V, V]
    lib.gsr_adam_step.argtypes = [V, I64, I32, V, V, V, V, V, V, V, V, I32, V, V, V, V, F32, F32,
                                  F32, F32, F32, F32, V, V]
    lib.gsr_autotune.argtypes = [V, C.POINTER(Settings), I64, V, V, V, V, V, I32,
                                 C.POINTER(Camera), V, V, V, F32, I32, I32,
                                 C.POINTER(Settings), V, V]
    for name in EXPORTS:
        if name != "gsr_last_error":
            getattr(lib, name).restype = S
    _lib = lib
    return lib


def make_settings(sh_degree, background=(0.0, 0.0, 0.0), tile=(16, 16), key_capacity=0,
                  xcd_remap=True, lds_batch=0, timing=False, count_pairs=False, median=False):
    flags = (0 if xcd_remap else FLAG_NO_XCD_REMAP) | (FLAG_TIMING if timing else 0) | \
        (FLAG_COUNT_PAIRS if count_pairs else 0) | (FLAG_MEDIAN_DEPTH if median else 0)
    return Settings(int(sh_degree), (C.c_float * 3)(*[float(b) for b in background]),
                    int(tile[0]), int(tile[1]), int(lds_batch), int(key_capacity), flags)


def make_cameras(cams):
    """cams: sequence of (W, H, fx, fy, cx, cy[, near])."""
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        near = float(c[6]) if len(c) > 6 else 0.2
        arr[i] = Camera(int(c[0]), int(c[1]), float(c[2]), float(c[3]), float(c[4]),
                        float(c[5]), near)
    return arr
