"""FP64 CPU oracle of the pencil-beam VMAT dose model (arXiv:2512.18863, §2.2).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  The arithmetic
lives in ``oracle.c`` (plain C, double precision); this module only marshals
numpy arrays through ctypes.  It shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

WEPL_PER_RAY = 0
WEPL_CENTRAL_AXIS = 1


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (host gcc, -O2, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Model(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("sx", ctypes.c_double), ("sy", ctypes.c_double), ("sz", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
        ("sad", ctypes.c_double), ("iso", ctypes.c_double * 3),
        ("n_leaf", ctypes.c_int), ("leaf_edges", ctypes.POINTER(ctypes.c_double)),
        ("field_limit", ctypes.c_double * 2),
        ("n_taps", ctypes.c_int), ("wepl_mode", ctypes.c_int),
        ("lat_step", ctypes.c_double), ("depth_step", ctypes.c_double),
        ("tau", ctypes.c_double), ("calib", ctypes.c_double),
        ("n_dd", ctypes.c_int), ("dd_step", ctypes.c_double), ("dd", ctypes.POINTER(ctypes.c_double)),
        ("kpoly", (ctypes.c_double * 4) * 4), ("kz_max", ctypes.c_double),
        ("fcorr", ctypes.c_int), ("pen_fwhm_u", ctypes.c_double), ("pen_fwhm_v", ctypes.c_double),
        ("hs_amp", ctypes.c_double), ("hs_sigma", ctypes.c_double), ("oar", ctypes.c_double * 2),
        ("coll_rot", ctypes.c_int),
    ]


_P = ctypes.POINTER(ctypes.c_double)


def _lib_handle():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        M = ctypes.POINTER(_Model)
        I, D = ctypes.c_int, ctypes.c_double
        sigs = {
            "or_fan_dims": (I, [M, ctypes.POINTER(I), _P]),
            "or_hu_to_density": (None, [ctypes.c_long, _P, _P, I, _P, _P]),
            "or_raster": (None, [M, _P, _P, _P]),
            "or_fluence_correct": (None, [M, _P, _P, I]),
            "or_rotate_fluence": (None, [M, D, _P, _P, I]),
            "or_rho_sample": (D, [M, _P, D, D, D]),
            "or_ca_depth": (None, [M, _P, D, _P]),
            "or_wepl": (None, [M, _P, D, _P]),
            "or_taps": (None, [M, D, D, _P]),
            "or_conv_plane": (None, [I, I, I, _P, _P, _P]),
            "or_gather": (None, [M, D, _P, _P]),
            "or_scatter": (None, [M, D, _P, _P]),
            "or_forward_cp": (None, [M, _P, D, D, _P, _P, _P, _P, _P, _P, _P, _P]),
            "or_forward": (None, [M, _P, I, _P, _P, _P, _P, _P, _P]),
            "or_backward": (None, [M, _P, I, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
            "or_raster_backward": (None, [M, _P, _P, _P, _P, _P]),
            "or_project": (None, [I, I, _P, _P, _P, D, D, D, D, D]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


class Model:
    """The problem description the oracle needs, built from an inputs.Case."""

    def __init__(self, case, n_taps=None, wepl_mode=None, coll_rot=None):
        m = case.machine
        nz, ny, nx = case.shape
        self.case = case
        self._edges = _f64(m.leaf_edges)
        self._dd = _f64(m.dd)
        s = _Model()
        s.nx, s.ny, s.nz = nx, ny, nz
        s.sx, s.sy, s.sz = case.spacing
        s.ox, s.oy, s.oz = case.origin
        s.sad = m.sad
        s.iso[:] = list(case.iso)
        s.n_leaf = m.n_leaf
        s.leaf_edges = _ptr(self._edges)
        s.field_limit[:] = list(case.field_limit)
        s.n_taps = case.n_taps if n_taps is None else n_taps
        s.wepl_mode = case.wepl_mode if wepl_mode is None else wepl_mode
        s.lat_step, s.depth_step = case.lat_step, case.depth_step
        s.tau, s.calib = m.tau, m.calib
        s.n_dd, s.dd_step, s.dd = len(self._dd), m.dd_step, _ptr(self._dd)
        for a in range(4):
            for b in range(4):
                s.kpoly[a][b] = float(m.kpoly[a][b])
        s.kz_max = m.kz_max
        s.fcorr = 1 if m.fcorr else 0
        s.pen_fwhm_u, s.pen_fwhm_v = m.pen_fwhm_u, m.pen_fwhm_v
        s.hs_amp, s.hs_sigma = m.hs_amp, m.hs_sigma
        s.oar[:] = [float(m.oar[0]), float(m.oar[1])]
        # a plan with collimator angles gets the square fan grid of the rotation
        s.coll_rot = (1 if getattr(case, "collimator", None) is not None else 0) if coll_rot is None \
            else (1 if coll_rot else 0)
        self.s = s
        dims = (ctypes.c_int * 3)()
        d0 = ctypes.c_double()
        if _lib_handle().or_fan_dims(ctypes.byref(s), dims, ctypes.byref(d0)) != 0:
            raise ValueError("invalid kernel size or steps")
        self.Nu, self.Nv, self.Nk = dims[0], dims[1], dims[2]
        self.d0 = d0.value
        self.n_leaf = m.n_leaf

    @property
    def ref(self):
        return ctypes.byref(self.s)

    @property
    def fan_shape(self):
        return (self.Nk, self.Nv, self.Nu)

    @property
    def vol_shape(self):
        return tuple(self.case.shape)


def hu_to_density(hu, hu_pts, rho_pts) -> np.ndarray:
    hu = _f64(hu)
    out = np.empty_like(hu)
    hp, rp = _f64(hu_pts), _f64(rho_pts)
    _lib_handle().or_hu_to_density(hu.size, _ptr(hu), _ptr(out), len(hp), _ptr(hp), _ptr(rp))
    return out


def density(model: Model) -> np.ndarray:
    m = model.case.machine
    return hu_to_density(model.case.hu, m.hu_pts, m.rho_pts)


def raster(model: Model, leaves, jaws) -> np.ndarray:
    F = np.empty((model.Nv, model.Nu))
    lv, jw = _f64(leaves), _f64(jaws)
    _lib_handle().or_raster(model.ref, _ptr(lv), _ptr(jw), _ptr(F))
    return F


def fluence_correct(model: Model, F, transpose: bool = False) -> np.ndarray:
    """Fluence corrections (source penumbra, head scatter, off-axis) of one map
    [Nv][Nu], or their adjoint."""
    F = _f64(F)
    out = np.empty_like(F)
    _lib_handle().or_fluence_correct(model.ref, _ptr(F), _ptr(out), 1 if transpose else 0)
    return out


def rotate_fluence(model: Model, coll_deg, F, transpose: bool = False) -> np.ndarray:
    """Collimator rotation of one map [Nv][Nu] (or its transpose)."""
    F = _f64(F)
    out = np.empty_like(F)
    _lib_handle().or_rotate_fluence(model.ref, float(coll_deg), _ptr(F), _ptr(out), 1 if transpose else 0)
    return out


def rho_sample(model: Model, rho, x, y, z) -> float:
    return _lib_handle().or_rho_sample(model.ref, _ptr(_f64(rho)), x, y, z)


def ca_depth(model: Model, rho, gantry) -> np.ndarray:
    z = np.empty(model.Nk)
    _lib_handle().or_ca_depth(model.ref, _ptr(_f64(rho)), float(gantry), _ptr(z))
    return z


def wepl(model: Model, rho, gantry) -> np.ndarray:
    W = np.empty(model.fan_shape)
    _lib_handle().or_wepl(model.ref, _ptr(_f64(rho)), float(gantry), _ptr(W))
    return W


def taps(model: Model, d_k, z_k) -> np.ndarray:
    n = model.s.n_taps
    K = np.empty((n, n))
    _lib_handle().or_taps(model.ref, float(d_k), float(z_k), _ptr(K))
    return K


def conv_plane(K, plane) -> np.ndarray:
    K, plane = _f64(K), _f64(plane)
    out = np.empty_like(plane)
    _lib_handle().or_conv_plane(plane.shape[0], plane.shape[1], K.shape[0], _ptr(K), _ptr(plane), _ptr(out))
    return out


def gather(model: Model, gantry, Dfan) -> np.ndarray:
    out = np.empty(model.vol_shape)
    _lib_handle().or_gather(model.ref, float(gantry), _ptr(_f64(Dfan)), _ptr(out))
    return out


def scatter(model: Model, gantry, g) -> np.ndarray:
    out = np.empty(model.fan_shape)
    _lib_handle().or_scatter(model.ref, float(gantry), _ptr(_f64(g)), _ptr(out))
    return out


def _coll(coll, n):
    if coll is None:
        return None
    c = _f64(coll).reshape(-1)
    assert len(c) == n
    return c


def forward_cp(model: Model, rho, gantry, leaves, jaws, coll: float = 0.0) -> dict:
    """Every intermediate of one control point (fan arrays in [Nk][Nv][Nu]; F in the
    beam frame)."""
    r = {
        "F": np.empty((model.Nv, model.Nu)),
        "z": np.empty(model.Nk),
        "W": np.empty(model.fan_shape),
        "P": np.empty(model.fan_shape),
        "Dfan": np.empty(model.fan_shape),
        "D": np.empty(model.vol_shape),
    }
    _lib_handle().or_forward_cp(model.ref, _ptr(_f64(rho)), float(gantry), float(coll), _ptr(_f64(leaves)),
                                _ptr(_f64(jaws)), _ptr(r["F"]), _ptr(r["z"]), _ptr(r["W"]), _ptr(r["P"]),
                                _ptr(r["Dfan"]), _ptr(r["D"]))
    return r


def forward(model: Model, rho, gantry, leaves, jaws, mu, coll=None) -> np.ndarray:
    """Plan dose; coll = per-control-point collimator angles (None: all 0)."""
    gantry, leaves, jaws, mu = _f64(gantry), _f64(leaves), _f64(jaws), _f64(mu)
    c = _coll(coll, len(gantry))
    dose = np.empty(model.vol_shape)
    _lib_handle().or_forward(model.ref, _ptr(_f64(rho)), len(gantry), _ptr(gantry), _ptr(c), _ptr(leaves),
                             _ptr(jaws), _ptr(mu), _ptr(dose))
    return dose


def backward(model: Model, rho, gantry, leaves, jaws, mu, g, coll=None):
    gantry, leaves, jaws, mu = _f64(gantry), _f64(leaves), _f64(jaws), _f64(mu)
    n = len(gantry)
    c = _coll(coll, n)
    gl = np.empty((n, 2, model.n_leaf))
    gj = np.empty((n, 4))
    gm = np.empty(n)
    _lib_handle().or_backward(model.ref, _ptr(_f64(rho)), n, _ptr(gantry), _ptr(c), _ptr(leaves), _ptr(jaws),
                              _ptr(mu), _ptr(_f64(g)), _ptr(gl), _ptr(gj), _ptr(gm))
    return gl, gj, gm


def raster_backward(model: Model, leaves, jaws, gF):
    gl = np.empty((2, model.n_leaf))
    gj = np.empty(4)
    _lib_handle().or_raster_backward(model.ref, _ptr(_f64(leaves)), _ptr(_f64(jaws)), _ptr(_f64(gF)),
                                     _ptr(gl), _ptr(gj))
    return gl, gj


def project(leaves, jaws, mu, leaf_limit, jaw_limit_x, jaw_limit_y, w_min, mu_min):
    lv, jw, m = _f64(leaves).copy(), _f64(jaws).copy(), _f64(mu).copy()
    _lib_handle().or_project(len(m), lv.shape[-1], _ptr(lv), _ptr(jw), _ptr(m), leaf_limit, jaw_limit_x,
                             jaw_limit_y, w_min, mu_min)
    return lv, jw, m
