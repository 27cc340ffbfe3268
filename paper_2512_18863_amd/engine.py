"""PyTorch binding of the HIP dose library (``libpdrt.so``, ``include/pdrt.h``).

Argument marshalling only: every step of the dose path runs in the library's
HIP kernels on the caller's current stream.  Torch provides device memory,
streams and the autograd hook.  There is no CPU fallback: if the library is
not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

from . import inputs as _inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdrt.so")

PDRT_OK = 0
CONV_FP32 = 0
CONV_BF16 = 1
WEPL_PER_RAY = 0
WEPL_CENTRAL_AXIS = 1
CACHE_F32 = 0
CACHE_BF16 = 1


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("sx", ctypes.c_double), ("sy", ctypes.c_double), ("sz", ctypes.c_double),
                ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double)]


class Beam(ctypes.Structure):
    _fields_ = [("sad_mm", ctypes.c_double), ("iso_mm", ctypes.c_double * 3),
                ("n_leaf_pairs", ctypes.c_int32), ("leaf_edges_mm", ctypes.POINTER(ctypes.c_double)),
                ("n_cp", ctypes.c_int32), ("gantry_deg", ctypes.c_void_p),
                ("field_limit_mm", ctypes.c_double * 2), ("collimator_deg", ctypes.c_void_p)]


class Spec(ctypes.Structure):
    _fields_ = [("n_taps", ctypes.c_int32), ("wepl_mode", ctypes.c_int32), ("conv_mode", ctypes.c_int32),
                ("lateral_step_mm", ctypes.c_double), ("depth_step_mm", ctypes.c_double),
                ("transmission", ctypes.c_double), ("calib", ctypes.c_double),
                ("n_dd", ctypes.c_int32), ("dd_step_mm", ctypes.c_double), ("dd", ctypes.c_void_p),
                ("kpoly", (ctypes.c_double * 4) * 4), ("kz_max_mm", ctypes.c_double),
                ("max_cp_batch", ctypes.c_int32),
                ("fluence_corr", ctypes.c_int32), ("pen_fwhm_mm", ctypes.c_double * 2),
                ("hs_amp", ctypes.c_double), ("hs_sigma_mm", ctypes.c_double), ("oar", ctypes.c_double * 2),
                ("march_scan", ctypes.c_int32)]


def set_fluence_corrections(s: "Spec", m) -> None:
    """Copy a machine's fluence-correction parameters into a Spec."""
    s.fluence_corr = 1 if m.fcorr else 0
    s.pen_fwhm_mm[:] = [float(m.pen_fwhm_u), float(m.pen_fwhm_v)]
    s.hs_amp, s.hs_sigma_mm = float(m.hs_amp), float(m.hs_sigma)
    s.oar[:] = [float(m.oar[0]), float(m.oar[1])]


class WsLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_size_t) for n in
                ("frame", "rho_t", "fluence", "depth", "vol0", "vol1", "adj", "comp", "fc_tmp", "box",
                 "cframe", "rot", "total")] + \
               [("batch", ctypes.c_int32)]


class Limits(ctypes.Structure):
    _fields_ = [("leaf_limit_mm", ctypes.c_double), ("jaw_limit_x_mm", ctypes.c_double),
                ("jaw_limit_y_mm", ctypes.c_double), ("w_min_mm", ctypes.c_double), ("mu_min", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "pdrt_fan_dims": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Beam), ctypes.POINTER(Spec),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "pdrt_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(Beam), ctypes.POINTER(Spec),
                                               ctypes.c_int32, ctypes.c_int32]),
    "pdrt_workspace_layout": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Beam), ctypes.POINTER(Spec),
                                             ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(WsLayout)]),
    "pdrt_hu_to_density": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _VP]),
    "pdrt_dose_forward": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.POINTER(Beam), _VP, _VP, _VP,
                                         ctypes.POINTER(Spec), _VP, _VP, ctypes.c_size_t, _VP]),
    "pdrt_dose_backward": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.POINTER(Beam), _VP, _VP, _VP,
                                          ctypes.POINTER(Spec), _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "pdrt_dose_forward_noalloc": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.POINTER(Beam), _VP, _VP, _VP,
                                                 ctypes.POINTER(Spec), _VP, _VP]),
    "pdrt_dose_forward_f64": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.POINTER(Beam), _VP, _VP, _VP,
                                             ctypes.POINTER(Spec), _VP, _VP, ctypes.c_size_t, _VP]),
    "pdrt_geometry_cache_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(Beam),
                                                    ctypes.POINTER(Spec), ctypes.c_int32]),
    "pdrt_geometry_cache_build": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.POINTER(Beam),
                                                 ctypes.POINTER(Spec), ctypes.c_int32, _VP, ctypes.c_size_t, _VP,
                                                 ctypes.c_size_t, _VP]),
    "pdrt_dose_forward_cached": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Beam), _VP, _VP, _VP,
                                                ctypes.POINTER(Spec), ctypes.c_int32, _VP, ctypes.c_size_t, _VP, _VP,
                                                ctypes.c_size_t, _VP]),
    "pdrt_dose_backward_cached": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Beam), _VP, _VP, _VP,
                                                 ctypes.POINTER(Spec), ctypes.c_int32, _VP, ctypes.c_size_t, _VP,
                                                 _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "pdrt_project_params": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, ctypes.POINTER(Limits),
                                           _VP, _VP, _VP, _VP]),
    "pdrt_project_params_backward": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP,
                                                    ctypes.POINTER(Limits), ctypes.c_int32, _VP, _VP, _VP, _VP, _VP,
                                                    _VP, _VP]),
    "pdrt_profile_begin": (ctypes.c_int, [ctypes.c_int32]),
    "pdrt_profile_end": (ctypes.c_int, [ctypes.POINTER(KernelTime), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "pdrt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pdrt_version": (ctypes.c_int, []),
}


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpdrt.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2512_18863_amd.build); there is no CPU fallback")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


class PdrtError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != PDRT_OK:
        raise PdrtError("%s failed: %s (%d)" % (what, lib().pdrt_status_string(status).decode(), status))


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dptr(t: torch.Tensor, dtype, device, shape=None, name="tensor") -> int:
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dtype, device))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


class DoseEngine:
    """One CT + beam geometry + kernel choice, ready to map (leaves, jaws, MU) to dose.

    The CT is converted to density on the GPU once; the workspace is allocated
    once (sized for forward + backward) and reused by every call.
    """

    def __init__(self, case: "_inputs.Case", *, n_taps: Optional[int] = None, conv: str = "fp32",
                 wepl_mode: Optional[int] = None, device="cuda", max_cp_batch: int = 0,
                 calib: Optional[float] = None, with_f64: bool = False, march_scan: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("DoseEngine needs a GPU")
        lib()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.case = case
        m = case.machine
        nz, ny, nx = case.shape
        self.vol_shape = (nz, ny, nx)
        self.n_cp = case.n_cp
        self.n_leaf = m.n_leaf
        g = Grid()
        g.nx, g.ny, g.nz = nx, ny, nz
        g.sx, g.sy, g.sz = case.spacing
        g.ox, g.oy, g.oz = case.origin
        self.grid = g
        self._edges = np.ascontiguousarray(m.leaf_edges, dtype=np.float64)
        dev = self.device
        self.gantry32 = torch.tensor(np.asarray(case.gantry), dtype=torch.float32, device=dev)
        self.dd32 = torch.tensor(np.asarray(m.dd), dtype=torch.float32, device=dev)
        b = Beam()
        b.sad_mm = m.sad
        b.iso_mm[:] = list(case.iso)
        b.n_leaf_pairs = m.n_leaf
        b.leaf_edges_mm = self._edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        b.n_cp = self.n_cp
        b.gantry_deg = self.gantry32.data_ptr()
        b.field_limit_mm[:] = list(case.field_limit)
        # collimator angles (None: all 0, no rotation)
        self.coll32 = None
        if getattr(case, "collimator", None) is not None:
            self.coll32 = torch.tensor(np.asarray(case.collimator), dtype=torch.float32, device=dev)
            b.collimator_deg = self.coll32.data_ptr()
        self.beam = b
        s = Spec()
        s.n_taps = case.n_taps if n_taps is None else n_taps
        s.wepl_mode = case.wepl_mode if wepl_mode is None else wepl_mode
        s.conv_mode = {"fp32": CONV_FP32, "bf16": CONV_BF16}[conv]
        s.lateral_step_mm, s.depth_step_mm = case.lat_step, case.depth_step
        s.transmission = m.tau
        s.calib = m.calib if calib is None else calib
        s.n_dd, s.dd_step_mm = len(m.dd), m.dd_step
        s.dd = self.dd32.data_ptr()
        for a in range(4):
            for c in range(4):
                s.kpoly[a][c] = float(m.kpoly[a][c])
        s.kz_max_mm = m.kz_max
        s.max_cp_batch = max_cp_batch
        s.march_scan = 1 if march_scan else 0
        set_fluence_corrections(s, m)
        self.spec = s
        dims = (ctypes.c_int32 * 3)()
        d0 = ctypes.c_double()
        _check(lib().pdrt_fan_dims(ctypes.byref(g), ctypes.byref(b), ctypes.byref(s), dims, ctypes.byref(d0)),
               "pdrt_fan_dims")
        self.Nu, self.Nv, self.Nk = dims[0], dims[1], dims[2]
        self.d0 = d0.value
        nbytes = lib().pdrt_workspace_bytes(ctypes.byref(g), ctypes.byref(b), ctypes.byref(s), 1, 4)
        if nbytes == 0:
            raise PdrtError("invalid problem")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        # CT -> density on the GPU
        hu = torch.tensor(np.ascontiguousarray(case.hu, dtype=np.float32), device=dev)
        self.rho = torch.empty_like(hu)
        hp = np.ascontiguousarray(m.hu_pts, dtype=np.float64)
        rp = np.ascontiguousarray(m.rho_pts, dtype=np.float64)
        _check(lib().pdrt_hu_to_density(ctypes.byref(g), hu.data_ptr(), self.rho.data_ptr(), len(hp),
                                        hp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        rp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        _stream_ptr(dev)), "pdrt_hu_to_density")
        self._f64 = None
        if with_f64:
            self._init_f64()
        self.cache = None
        self.cache_type = None

    # ------------------------------------------------------------------ helpers
    def _ptrs(self, leaves, jaws, mu, dtype=torch.float32):
        n, L, dev = self.n_cp, self.n_leaf, self.device
        return (_dptr(leaves, dtype, dev, (n, 2, L), "leaves"), _dptr(jaws, dtype, dev, (n, 4), "jaws"),
                _dptr(mu, dtype, dev, (n,), "mu"))

    def fan_shape(self):
        return (self.Nk, self.Nu, self.Nv)

    def layout(self, with_backward=1, elem=4) -> WsLayout:
        lay = WsLayout()
        _check(lib().pdrt_workspace_layout(ctypes.byref(self.grid), ctypes.byref(self.beam), ctypes.byref(self.spec),
                                           with_backward, elem, ctypes.byref(lay)), "pdrt_workspace_layout")
        return lay

    def ws_view(self, name: str, shape, dtype=torch.float32, elem=4, with_backward=1):
        """A view of an intermediate inside the workspace (valid after a call)."""
        lay = self.layout(with_backward, elem)
        off = getattr(lay, name)
        count = int(np.prod(shape))
        ws = self.ws if elem == 4 else self._f64["ws"]
        return ws[off:off + count * elem].view(dtype).view(*shape)

    # ------------------------------------------------------------------ geometry cache
    def build_cache(self, kind: str = "fp32") -> int:
        """Compute the plan-level geometry cache (central-axis depths and
        (SAD/d)^2 DD(W) of every beam-frame node, all control points); later
        forward / backward calls use it instead of the ray march.  Returns bytes."""
        ctype = {"fp32": CACHE_F32, "bf16": CACHE_BF16}[kind]
        nbytes = lib().pdrt_geometry_cache_bytes(ctypes.byref(self.grid), ctypes.byref(self.beam),
                                                 ctypes.byref(self.spec), ctype)
        if nbytes == 0:
            raise PdrtError("invalid problem for a geometry cache")
        self.cache = None
        cache = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _check(lib().pdrt_geometry_cache_build(ctypes.byref(self.grid), self.rho.data_ptr(), ctypes.byref(self.beam),
                                               ctypes.byref(self.spec), ctype, cache.data_ptr(), nbytes,
                                               self.ws.data_ptr(), self.ws.numel(), _stream_ptr(self.device)),
               "pdrt_geometry_cache_build")
        self.cache, self.cache_type = cache, ctype
        return nbytes

    def drop_cache(self):
        self.cache, self.cache_type = None, None

    # ------------------------------------------------------------------ calls
    def forward(self, leaves, jaws, mu, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        lp, jp, mp = self._ptrs(leaves, jaws, mu)
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
        op = _dptr(out, torch.float32, self.device, self.vol_shape, "out")
        if self.cache is not None:
            _check(lib().pdrt_dose_forward_cached(ctypes.byref(self.grid), ctypes.byref(self.beam), lp, jp, mp,
                                                  ctypes.byref(self.spec), self.cache_type, self.cache.data_ptr(),
                                                  self.cache.numel(), op, self.ws.data_ptr(), self.ws.numel(),
                                                  _stream_ptr(self.device)), "pdrt_dose_forward_cached")
            return out
        _check(lib().pdrt_dose_forward(ctypes.byref(self.grid), self.rho.data_ptr(), ctypes.byref(self.beam), lp, jp,
                                       mp, ctypes.byref(self.spec), op, self.ws.data_ptr(), self.ws.numel(),
                                       _stream_ptr(self.device)), "pdrt_dose_forward")
        return out

    def forward_noalloc(self, leaves, jaws, mu, out: torch.Tensor) -> torch.Tensor:
        """The forward through pdrt_dose_forward_noalloc: the library's static
        scratch instead of this engine's workspace; `out` is caller-allocated."""
        lp, jp, mp = self._ptrs(leaves, jaws, mu)
        op = _dptr(out, torch.float32, self.device, self.vol_shape, "out")
        _check(lib().pdrt_dose_forward_noalloc(ctypes.byref(self.grid), self.rho.data_ptr(), ctypes.byref(self.beam),
                                               lp, jp, mp, ctypes.byref(self.spec), op, _stream_ptr(self.device)),
               "pdrt_dose_forward_noalloc")
        return out

    def backward(self, leaves, jaws, mu, grad_dose):
        lp, jp, mp = self._ptrs(leaves, jaws, mu)
        gp = _dptr(grad_dose, torch.float32, self.device, self.vol_shape, "grad_dose")
        gl = torch.empty((self.n_cp, 2, self.n_leaf), dtype=torch.float32, device=self.device)
        gj = torch.empty((self.n_cp, 4), dtype=torch.float32, device=self.device)
        gm = torch.empty((self.n_cp,), dtype=torch.float32, device=self.device)
        if self.cache is not None:
            _check(lib().pdrt_dose_backward_cached(ctypes.byref(self.grid), ctypes.byref(self.beam), lp, jp, mp,
                                                   ctypes.byref(self.spec), self.cache_type, self.cache.data_ptr(),
                                                   self.cache.numel(), gp, gl.data_ptr(), gj.data_ptr(),
                                                   gm.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                                   _stream_ptr(self.device)), "pdrt_dose_backward_cached")
            return gl, gj, gm
        _check(lib().pdrt_dose_backward(ctypes.byref(self.grid), self.rho.data_ptr(), ctypes.byref(self.beam), lp, jp,
                                        mp, ctypes.byref(self.spec), gp, gl.data_ptr(), gj.data_ptr(), gm.data_ptr(),
                                        self.ws.data_ptr(), self.ws.numel(), _stream_ptr(self.device)),
               "pdrt_dose_backward")
        return gl, gj, gm

    def __call__(self, leaves, jaws, mu) -> torch.Tensor:
        """Differentiable dose (leaves, jaws, mu -> dose)."""
        return DoseFunction.apply(leaves, jaws, mu, self)

    # ------------------------------------------------------------------ FP64
    def _init_f64(self):
        dev = self.device
        gantry = torch.tensor(np.asarray(self.case.gantry), dtype=torch.float64, device=dev)
        dd = torch.tensor(np.asarray(self.case.machine.dd), dtype=torch.float64, device=dev)
        b = Beam.from_buffer_copy(self.beam)
        b.gantry_deg = gantry.data_ptr()
        coll = None
        if self.coll32 is not None:
            coll = torch.tensor(np.asarray(self.case.collimator), dtype=torch.float64, device=dev)
            b.collimator_deg = coll.data_ptr()
        s = Spec.from_buffer_copy(self.spec)
        s.dd = dd.data_ptr()
        s.conv_mode = CONV_FP32
        nbytes = lib().pdrt_workspace_bytes(ctypes.byref(self.grid), ctypes.byref(b), ctypes.byref(s), 0, 8)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._f64 = {"gantry": gantry, "dd": dd, "coll": coll, "beam": b, "spec": s, "ws": ws,
                     "rho": self.rho.to(torch.float64)}

    def set_density_f64(self, rho64: torch.Tensor):
        """Use an exact FP64 density for the FP64 path (default: the FP32 one widened)."""
        if self._f64 is None:
            self._init_f64()
        self._f64["rho"] = rho64.to(self.device, torch.float64).contiguous()

    def forward_f64(self, leaves, jaws, mu, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if self._f64 is None:
            self._init_f64()
        f = self._f64
        lp, jp, mp = self._ptrs(leaves, jaws, mu, torch.float64)
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float64, device=self.device)
        op = _dptr(out, torch.float64, self.device, self.vol_shape, "out")
        _check(lib().pdrt_dose_forward_f64(ctypes.byref(self.grid), f["rho"].data_ptr(), ctypes.byref(f["beam"]), lp,
                                           jp, mp, ctypes.byref(f["spec"]), op, f["ws"].data_ptr(), f["ws"].numel(),
                                           _stream_ptr(self.device)), "pdrt_dose_forward_f64")
        return out


def profile_begin(max_launches: int = 4096):
    """Start timing every kernel launch of the dose entry points with HIP events."""
    _check(lib().pdrt_profile_begin(max_launches), "pdrt_profile_begin")


def profile_end() -> dict:
    """Stop timing; returns {kernel name: (launches, total ms)}."""
    out = (KernelTime * 64)()
    n = ctypes.c_int32()
    _check(lib().pdrt_profile_end(out, 64, ctypes.byref(n)), "pdrt_profile_end")
    return {out[i].name.decode(): (out[i].launches, out[i].total_ms) for i in range(n.value)}


class DoseFunction(torch.autograd.Function):
    """dose = engine(leaves, jaws, mu) with the hand-written adjoint as backward.
    No beam-frame volume is saved: the backward recomputes per control point."""

    @staticmethod
    def forward(ctx, leaves, jaws, mu, engine):
        ctx.engine = engine
        ctx.save_for_backward(leaves, jaws, mu)
        return engine.forward(leaves.detach(), jaws.detach(), mu.detach())

    @staticmethod
    def backward(ctx, grad):
        leaves, jaws, mu = ctx.saved_tensors
        gl, gj, gm = ctx.engine.backward(leaves.detach(), jaws.detach(), mu.detach(), grad.contiguous())
        return gl, gj, gm, None


def project_params(leaves, jaws, mu, limits: dict, out=None):
    """Hardware-constrained projection (§2.2.1) on the GPU."""
    n, _, L = leaves.shape
    dev = leaves.device
    lim = Limits(limits["leaf"], limits["jaw_x"], limits["jaw_y"], limits["w_min"], limits["mu_min"])
    lo = torch.empty_like(leaves) if out is None else out[0]
    jo = torch.empty_like(jaws) if out is None else out[1]
    mo = torch.empty_like(mu) if out is None else out[2]
    _check(lib().pdrt_project_params(n, L, _dptr(leaves, torch.float32, dev, name="leaves"),
                                     _dptr(jaws, torch.float32, dev, name="jaws"),
                                     _dptr(mu, torch.float32, dev, name="mu"), ctypes.byref(lim), lo.data_ptr(),
                                     jo.data_ptr(), mo.data_ptr(), _stream_ptr(dev)), "pdrt_project_params")
    return lo, jo, mo


def project_params_backward(leaves, jaws, mu, limits: dict, g_leaves, g_jaws, g_mu, straight_through=True):
    n, _, L = leaves.shape
    dev = leaves.device
    lim = Limits(limits["leaf"], limits["jaw_x"], limits["jaw_y"], limits["w_min"], limits["mu_min"])
    ol, oj, om = torch.empty_like(g_leaves), torch.empty_like(g_jaws), torch.empty_like(g_mu)
    _check(lib().pdrt_project_params_backward(
        n, L, _dptr(leaves, torch.float32, dev, name="leaves"), _dptr(jaws, torch.float32, dev, name="jaws"),
        _dptr(mu, torch.float32, dev, name="mu"), ctypes.byref(lim), 1 if straight_through else 0,
        _dptr(g_leaves.contiguous(), torch.float32, dev, name="g_leaves"),
        _dptr(g_jaws.contiguous(), torch.float32, dev, name="g_jaws"),
        _dptr(g_mu.contiguous(), torch.float32, dev, name="g_mu"), ol.data_ptr(), oj.data_ptr(), om.data_ptr(),
        _stream_ptr(dev)), "pdrt_project_params_backward")
    return ol, oj, om


class ProjectFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, leaves, jaws, mu, limits, straight_through):
        ctx.limits, ctx.ste = limits, straight_through
        ctx.save_for_backward(leaves, jaws, mu)
        return project_params(leaves.detach(), jaws.detach(), mu.detach(), limits)

    @staticmethod
    def backward(ctx, gl, gj, gm):
        leaves, jaws, mu = ctx.saved_tensors
        ol, oj, om = project_params_backward(leaves, jaws, mu, ctx.limits, gl, gj, gm, ctx.ste)
        return ol, oj, om, None, None
