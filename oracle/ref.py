"""ctypes wrapper of the FP64 CPU oracle (oracle/gsr_ref.c).

TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  Arrays are numpy; inputs are the exact FP32
values the GPU path receives, outputs are FP64.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class _Cam(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float)]


class _Set(C.Structure):
    _fields_ = [("sh_degree", C.c_int32), ("background", C.c_float * 3),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("n_threads", C.c_int32),
                ("depth_mode", C.c_int32)]

DEPTH_BLENDED, DEPTH_MEDIAN = 0, 1


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    _lib = declare(C.CDLL(_build.LIB))
    return _lib


def use_library(path):
    """Point the wrapper at another build of the oracle (the planted-mistake
    tests load mutated copies); returns the previous library handle."""
    global _lib
    prev = _lib
    _lib = declare(C.CDLL(path)) if isinstance(path, str) else path
    return prev


def declare(lib):
    P = C.c_void_p
    lib.ref_forward.argtypes = [C.POINTER(_Set), C.c_int64, P, P, P, P, P, C.c_int32,
                                C.POINTER(_Cam), P, P, P, P, C.POINTER(P)]
    lib.ref_forward.restype = C.c_int
    lib.ref_forward_f64.argtypes = lib.ref_forward.argtypes
    lib.ref_forward_f64.restype = C.c_int
    lib.ref_backward.argtypes = [P] + [P] * 9
    lib.ref_backward.restype = C.c_int
    lib.ref_free.argtypes = [P]
    lib.ref_free.restype = None
    for name in ("ref_num_keys", "ref_num_tiles", "ref_num_pixels", "ref_pairs_evaluated"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = C.c_int64
    lib.ref_decision_hash.argtypes = [P]
    lib.ref_decision_hash.restype = C.c_uint64
    lib.ref_records.argtypes = [P, P, P, P]
    lib.ref_records.restype = None
    lib.ref_tile_lists.argtypes = [P, P, P]
    lib.ref_tile_lists.restype = None
    lib.ref_pixel_info.argtypes = [P, P, P, P]
    lib.ref_pixel_info.restype = None
    lib.ref_screen_grads.argtypes = [P, P]
    lib.ref_screen_grads.restype = C.c_int
    lib.ref_quat_to_rotmat.argtypes = [P, P]
    lib.ref_sh_basis.argtypes = [C.c_int32, P, P]
    lib.ref_sh_basis_grad.argtypes = [C.c_int32, P, P]
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class RefForward:
    """Result of one oracle forward; holds the saved state for backward."""

    def __init__(self, scene, tile=(16, 16), threads=1, f64=False, median=False):
        lib = load()
        conv = (lambda a: np.ascontiguousarray(a, dtype=np.float64)) if f64 else _f32
        self.scene = scene
        n = int(scene.means.shape[0])
        F = len(scene.cams)
        self.n, self.F = n, F
        self.sizes = [(int(c[0]), int(c[1])) for c in scene.cams]  # (W, H)
        self._keep = [conv(scene.means), conv(scene.log_scales), conv(scene.quats),
                      conv(scene.opacity), conv(scene.sh), conv(scene.poses)]
        cams = (_Cam * F)(*[_Cam(int(c[0]), int(c[1]), *[float(v) for v in c[2:7]])
                            for c in scene.cams])
        self._cams = cams
        s = _Set(int(scene.sh_degree), (C.c_float * 3)(*[float(b) for b in scene.background]),
                 int(tile[0]), int(tile[1]), int(threads),
                 DEPTH_MEDIAN if median else DEPTH_BLENDED)
        self._set = s
        P = sum(w * h for w, h in self.sizes)
        self.P = P
        self._rgb = np.zeros(3 * P)
        self._depth = np.zeros(P)
        self._alpha = np.zeros(P)
        st = C.c_void_p()
        m, ls, q, o, sh, poses = self._keep
        fwd = lib.ref_forward_f64 if f64 else lib.ref_forward
        rc = fwd(C.byref(s), n, _p(m), _p(ls), _p(q), _p(o), _p(sh), F,
                             cams, _p(poses), _p(self._rgb), _p(self._depth),
                             _p(self._alpha), C.byref(st))
        if rc != 0:
            raise ValueError(f"oracle forward failed with status {rc}")
        self._st = st

    def __del__(self):
        if getattr(self, "_st", None) and _lib is not None:
            _lib.ref_free(self._st)
            self._st = None

    # ---- outputs, per frame ----
    def frames(self):
        """List of (rgb [3,H,W], depth [H,W], alpha [H,W]) per frame."""
        out, p = [], 0
        for (w, h) in self.sizes:
            out.append((self._rgb[3 * p:3 * (p + w * h)].reshape(3, h, w),
                        self._depth[p:p + w * h].reshape(h, w),
                        self._alpha[p:p + w * h].reshape(h, w)))
            p += w * h
        return out

    @property
    def rgb_flat(self):
        return self._rgb

    @property
    def depth_flat(self):
        return self._depth

    @property
    def alpha_flat(self):
        return self._alpha

    # ---- backward ----
    def backward(self, g_rgb, g_depth, g_alpha):
        lib = load()
        n, F = self.n, self.F
        K = (self.scene.sh_degree + 1) ** 2
        g_rgb = np.ascontiguousarray(g_rgb, dtype=np.float64).ravel()
        g_depth = np.ascontiguousarray(g_depth, dtype=np.float64).ravel()
        g_alpha = np.ascontiguousarray(g_alpha, dtype=np.float64).ravel()
        assert g_rgb.size == 3 * self.P and g_depth.size == self.P and g_alpha.size == self.P
        out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
                   opacity=np.zeros(n), sh=np.zeros((n, K, 3)), twist=np.zeros((F, 6)))
        rc = lib.ref_backward(self._st, _p(g_rgb), _p(g_depth), _p(g_alpha), _p(out["means"]),
                              _p(out["log_scales"]), _p(out["quats"]), _p(out["opacity"]),
                              _p(out["sh"]), _p(out["twist"]))
        if rc != 0:
            raise ValueError(f"oracle backward failed with status {rc}")
        return out

    def screen_grads(self):
        """[F*n, 10] screen-space gradients of the last backward: d/du, d/dv,
        d/dA, d/dB, d/dC of the conic, d/dopacity, d/dcolour (3), d/dz."""
        out = np.zeros((self.n * self.F, 10))
        rc = load().ref_screen_grads(self._st, _p(out))
        if rc != 0:
            raise ValueError(f"no backward has run (status {rc})")
        return out

    # ---- debug artefacts ----
    @property
    def K(self):
        return int(load().ref_num_keys(self._st))

    @property
    def n_tiles_total(self):
        return int(load().ref_num_tiles(self._st))

    @property
    def pairs(self):
        return int(load().ref_pairs_evaluated(self._st))

    @property
    def decision_hash(self):
        return int(load().ref_decision_hash(self._st))

    def records(self):
        M = self.n * self.F
        ints = np.zeros((M, 14), np.int32)
        bits = np.zeros(M, np.uint32)
        vals = np.zeros((M, 20))
        if M:
            load().ref_records(self._st, _p(ints), _p(bits), _p(vals))
        names = ["u", "v", "z", "A", "B", "C", "sxx", "sxy", "syy", "lmax", "radius",
                 "opacity", "c0", "c1", "c2", "raw0", "raw1", "raw2", "det", "tz"]
        d = {nm: vals[:, i] for i, nm in enumerate(names)}
        for i, nm in enumerate(["keep", "x_lo", "x_hi", "y_lo", "y_hi", "tx_lo", "tx_hi",
                                "ty_lo", "ty_hi", "n_tiles", "bx_lo", "bx_hi", "by_lo",
                                "by_hi"]):
            d[nm] = ints[:, i]
        d["depth_bits"] = bits
        return d

    def tile_lists(self):
        T = self.n_tiles_total
        start = np.zeros(T + 1, np.int64)
        ent = np.zeros(max(self.K, 1), np.int32)
        load().ref_tile_lists(self._st, _p(start), _p(ent))
        return start, ent[:self.K]

    def pixel_info(self):
        flags = np.zeros(self.P, np.uint8)
        nl = np.zeros(self.P, np.int32)
        tf = np.zeros(self.P)
        load().ref_pixel_info(self._st, _p(flags), _p(nl), _p(tf))
        return flags, nl, tf


def forward(scene, tile=(16, 16), threads=1, f64=False, median=False):
    """Oracle forward.  f64=True passes the scene arrays as FP64 (used by the
    finite-difference pins); otherwise they are the FP32 values.  median=True
    renders the median depth instead of the alpha-blended depth."""
    return RefForward(scene, tile=tile, threads=threads, f64=f64, median=median)


def quat_to_rotmat(q):
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    load().ref_quat_to_rotmat(_p(q), _p(R))
    return R.reshape(3, 3)


def sh_basis(degree, d):
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros((degree + 1) ** 2)
    load().ref_sh_basis(int(degree), _p(d), _p(out))
    return out


def sh_basis_grad(degree, d):
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(((degree + 1) ** 2) * 3)
    load().ref_sh_basis_grad(int(degree), _p(d), _p(out))
    return out.reshape(-1, 3)
