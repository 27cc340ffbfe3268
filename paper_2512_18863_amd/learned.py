"""Learned large-kernel correction: small-kernel dose + density -> large-kernel dose.

The paper's timings grow with the lateral kernel size (Table 5) and it suggests
optimising with smaller kernels first (§4.1).  This module trains a small 3-D
U-Net that maps the cheap 9 x 9 dose (plus the density) to the 61 x 61 dose,
with a second output that estimates its own error; when that estimate exceeds
1 % of the maximum dose inside the 10 % isodose, the plain 61 x 61 FP32 path is
run instead (its output is then returned bit for bit).

Network (channels-last BF16 activations, FP32 master weights, every layer a
hand-written HIP kernel from libpdrt.so):
    level 0 (L^3):     e1a 16->16, e1b 16->16                (input: dose*s, rho, 14 zeros)
    level 1 (L/2)^3:   e2a 16->32, e2b 32->32                after 2x2x2 average pooling
    level 2 (L/4)^3:   ba 32->64,  bb 64->64
    level 1:           d2a (64 up ++ 32 skip)->32, d2b 32->32
    level 0:           d1a (32 up ++ 16 skip)->16, d1b 16->16
    head (1x1x1):      pred = dose*s + h0(x), resid = h1(x)
with s = 1 / max(small-kernel dose).  All 3x3x3 convolutions are ReLU'd.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from . import engine as E
from . import inputs

LAYERS = [  # name, c1, c2, cout, level
    ("e1a", 16, 0, 16, 0), ("e1b", 16, 0, 16, 0),
    ("e2a", 16, 0, 32, 1), ("e2b", 32, 0, 32, 1),
    ("ba", 32, 0, 64, 2), ("bb", 64, 0, 64, 2),
    ("d2a", 64, 32, 32, 1), ("d2b", 32, 0, 32, 1),
    ("d1a", 32, 16, 16, 0), ("d1b", 16, 0, 16, 0),
]
HEAD_C = 16


def _lib():
    lib = E.lib()
    if not getattr(lib, "_net_sigs", False):
        V = ctypes.c_void_p
        I32 = ctypes.c_int32
        P = ctypes.POINTER
        sigs = {
            "pdrt_conv3d_kpad": (I32, [I32]),
            "pdrt_conv3d_prepare_weights": (ctypes.c_int, [I32, I32, V, V, V, V]),
            "pdrt_conv3d_forward": (ctypes.c_int, [P(Vol), I32, I32, V, V, I32, V, V, I32, V, V]),
            "pdrt_conv3d_backward_data": (ctypes.c_int, [P(Vol), I32, V, V, I32, I32, V, V, V, V]),
            "pdrt_conv3d_wgrad_ws_bytes": (ctypes.c_size_t, [I32, I32, I32]),
            "pdrt_conv3d_backward_weight": (ctypes.c_int, [P(Vol), I32, I32, V, V, I32, V, V, I32, V,
                                                           ctypes.c_size_t, V, V, V]),
            "pdrt_net_input": (ctypes.c_int, [I32, V, V, V, V, V]),
            "pdrt_net_reduce_ws_bytes": (ctypes.c_size_t, [I32]),
            "pdrt_net_input_backward": (ctypes.c_int, [I32, V, V, V, V, V, V, V, V, ctypes.c_size_t, V]),
            "pdrt_net_scale": (ctypes.c_int, [I32, V, V, V, V, ctypes.c_size_t, V]),
            "pdrt_scale_by": (ctypes.c_int, [I32, V, V, I32, V, V]),
            "pdrt_add_bf16": (ctypes.c_int, [ctypes.c_size_t, V, V, V, V]),
            "pdrt_pool2": (ctypes.c_int, [P(Vol), I32, V, V, I32, V]),
            "pdrt_upsample2": (ctypes.c_int, [P(Vol), I32, V, V, I32, V]),
            "pdrt_net_head": (ctypes.c_int, [I32, I32, V, V, V, V, V, V, V, V]),
            "pdrt_net_head_ws_bytes": (ctypes.c_size_t, [I32, I32]),
            "pdrt_net_head_backward": (ctypes.c_int, [I32, I32, V, V, V, V, V, V, ctypes.c_size_t, V, V]),
            "pdrt_net_loss_ws_bytes": (ctypes.c_size_t, [I32]),
            "pdrt_net_train_loss": (ctypes.c_int, [I32, V, V, V, V, V, ctypes.c_float, ctypes.c_float,
                                                   ctypes.c_float, V, V, V, ctypes.c_size_t, V, V]),
            "pdrt_net_fallback_stats": (ctypes.c_int, [I32, V, V, ctypes.c_float, V, V, ctypes.c_size_t, V]),
            "pdrt_adam_step": (ctypes.c_int, [ctypes.c_size_t, V, V, V, V, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_float, I32, V]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        lib._net_sigs = True
    return lib


class Vol(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


def _p(t):
    return None if t is None else t.data_ptr()


def _ck(st, what):
    E._check(st, what)


class Net3D:
    """The U-Net's parameters, optimiser state and activation buffers for one grid size."""

    def __init__(self, dims, device="cuda", seed=0):
        D, H, W = dims
        assert D % 4 == 0 and H % 4 == 0 and W % 4 == 0
        self.dev = torch.device(device)
        self.dims = [(D, H, W), (D // 2, H // 2, W // 2), (D // 4, H // 4, W // 4)]
        self.vols = [Vol(*d) for d in self.dims]
        self.npos = [int(np.prod(d)) for d in self.dims]
        lib = _lib()
        rng = np.random.default_rng(seed)
        # flat FP32 master parameters: per layer w[cout][27][cin] then b[cout]; head hw[2][16], hb[2]
        self.slices = {}
        chunks = []
        off = 0
        for (name, c1, c2, cout, lvl) in LAYERS:
            cin = c1 + c2
            fan_in = 27 * (2 if name == "e1a" else cin)
            w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(cout, 27, cin))
            if name == "e1a":
                w[:, :, 2:] = 0.0
            b = np.zeros(cout)
            chunks += [w.ravel(), b]
            self.slices[name] = (off, w.size, off + w.size, cout)
            off += w.size + cout
        hw = rng.normal(0.0, 1e-3, size=(2, HEAD_C))
        hb = np.array([0.0, 0.0])
        chunks += [hw.ravel(), hb]
        self.head_off = off
        off += hw.size + 2
        self.params = torch.tensor(np.concatenate(chunks), dtype=torch.float32, device=self.dev)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        # BF16 operand layouts per layer
        self.wt, self.wd = {}, {}
        for (name, c1, c2, cout, lvl) in LAYERS:
            cin = c1 + c2
            self.wt[name] = torch.empty(cout * lib.pdrt_conv3d_kpad(cin), dtype=torch.bfloat16, device=self.dev)
            self.wd[name] = torch.empty(cin * lib.pdrt_conv3d_kpad(cout), dtype=torch.bfloat16, device=self.dev)
        self.prepare()
        # activations (outputs of each layer), pooled / upsampled tensors, and their gradients
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        n0, n1, n2 = self.npos
        self.x0 = torch.empty(n0 * 16, **bf)
        self.act = {name: torch.empty(self.npos[lvl] * cout, **bf) for (name, c1, c2, cout, lvl) in LAYERS}
        self.p1 = torch.empty(n1 * 16, **bf)
        self.p2 = torch.empty(n2 * 32, **bf)
        self.u2 = torch.empty(n1 * 64, **bf)
        self.u1 = torch.empty(n0 * 32, **bf)
        self.gbuf = {k: torch.empty_like(v) for k, v in self.act.items()}
        self.gx0 = torch.empty_like(self.x0)
        self.gp1, self.gp2 = torch.empty_like(self.p1), torch.empty_like(self.p2)
        self.gu2, self.gu1 = torch.empty_like(self.u2), torch.empty_like(self.u1)
        self.gs1, self.gs2 = torch.empty(n0 * 16, **bf), torch.empty(n1 * 32, **bf)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.pred = torch.empty(n0, **f32)
        self.resid = torch.empty(n0, **f32)
        self.scale = torch.empty(1, **f32)
        self.argmax = torch.empty(1, dtype=torch.int32, device=self.dev)
        self._dose = None
        self.gp = torch.empty(n0, **f32)
        self.gr = torch.empty(n0, **f32)
        self.stats = torch.empty(2, **f32)
        self.loss = torch.empty(1, **f32)
        self.nsplit = [max(1, n // 4096) for n in self.npos]
        wsz = max(lib.pdrt_conv3d_wgrad_ws_bytes(cout, c1 + c2, self.nsplit[lvl]) for (_, c1, c2, cout, lvl) in LAYERS)
        wsz = max(wsz, lib.pdrt_net_head_ws_bytes(n0, HEAD_C), lib.pdrt_net_loss_ws_bytes(n0),
                  lib.pdrt_net_reduce_ws_bytes(n0))
        self.ws = torch.empty(wsz // 4 + 1, **f32)
        self.ws_bytes = self.ws.numel() * 4

    # -------------------------------------------------------------- parameters
    def w(self, name):
        o, n, bo, cout = self.slices[name]
        return self.params[o:o + n], self.params[bo:bo + cout]

    def gw(self, name):
        o, n, bo, cout = self.slices[name]
        return self.grads[o:o + n], self.grads[bo:bo + cout]

    def head(self):
        o = self.head_off
        return self.params[o:o + 2 * HEAD_C], self.params[o + 2 * HEAD_C:o + 2 * HEAD_C + 2]

    def prepare(self):
        lib, s = _lib(), self._s()
        for (name, c1, c2, cout, lvl) in LAYERS:
            w, _ = self.w(name)
            _ck(lib.pdrt_conv3d_prepare_weights(cout, c1 + c2, _p(w), _p(self.wt[name]), _p(self.wd[name]), s),
                "prepare_weights")

    def _s(self):
        return torch.cuda.current_stream(self.dev).cuda_stream

    # -------------------------------------------------------------- forward
    def _conv(self, name, x1, x2=None):
        lib = _lib()
        (_, c1, c2, cout, lvl) = next(l for l in LAYERS if l[0] == name)
        _, b = self.w(name)
        _ck(lib.pdrt_conv3d_forward(ctypes.byref(self.vols[lvl]), c1, c2, _p(x1), _p(x2), cout, _p(self.wt[name]),
                                    _p(b), 1, _p(self.act[name]), self._s()), "conv3d " + name)
        return self.act[name]

    def forward(self, dose, rho):
        """dose, rho: FP32 [D*H*W] device tensors (same grid).  Returns (pred, resid)
        normalised by the dose maximum (self.scale)."""
        lib, s = _lib(), self._s()
        n0 = self.npos[0]
        self._dose = dose
        _ck(lib.pdrt_net_scale(n0, _p(dose), _p(self.scale), _p(self.argmax), _p(self.ws), self.ws_bytes, s),
            "net_scale")
        _ck(lib.pdrt_net_input(n0, _p(dose), _p(self.scale), _p(rho), _p(self.x0), s), "net_input")
        a = self._conv("e1a", self.x0)
        s1 = self._conv("e1b", a)
        _ck(lib.pdrt_pool2(ctypes.byref(self.vols[0]), 16, _p(s1), _p(self.p1), 0, s), "pool")
        a = self._conv("e2a", self.p1)
        s2 = self._conv("e2b", a)
        _ck(lib.pdrt_pool2(ctypes.byref(self.vols[1]), 32, _p(s2), _p(self.p2), 0, s), "pool")
        a = self._conv("ba", self.p2)
        b = self._conv("bb", a)
        _ck(lib.pdrt_upsample2(ctypes.byref(self.vols[1]), 64, _p(b), _p(self.u2), 0, s), "up")
        a = self._conv("d2a", self.u2, s2)
        c2 = self._conv("d2b", a)
        _ck(lib.pdrt_upsample2(ctypes.byref(self.vols[0]), 32, _p(c2), _p(self.u1), 0, s), "up")
        a = self._conv("d1a", self.u1, s1)
        c1 = self._conv("d1b", a)
        hw, hb = self.head()
        _ck(lib.pdrt_net_head(n0, HEAD_C, _p(c1), _p(hw), _p(hb), _p(dose), _p(self.scale), _p(self.pred),
                              _p(self.resid), s), "head")
        return self.pred, self.resid

    # -------------------------------------------------------------- backward
    def _back(self, name, dy, x1, x2, dx1, dx2, weights: bool):
        """dy: gradient w.r.t. this layer's activated output; writes dx1 (++ dx2) and,
        if weights, the layer's weight and bias gradients."""
        lib, s = _lib(), self._s()
        (_, c1, c2, cout, lvl) = next(l for l in LAYERS if l[0] == name)
        y = self.act[name]
        if dx1 is not None:
            _ck(lib.pdrt_conv3d_backward_data(ctypes.byref(self.vols[lvl]), cout, _p(dy), _p(y), c1, c2,
                                              _p(self.wd[name]), _p(dx1), _p(dx2), s), "dgrad " + name)
        if weights:
            gw, gb = self.gw(name)
            _ck(lib.pdrt_conv3d_backward_weight(ctypes.byref(self.vols[lvl]), c1, c2, _p(x1), _p(x2), cout, _p(dy),
                                                _p(y), self.nsplit[lvl], _p(self.ws), self.ws_bytes, _p(gw), _p(gb),
                                                s), "wgrad " + name)

    def backward(self, gp, gr, dose_grad=None, weights=True):
        """Back-propagate dL/dpred (gp) and dL/dresid (gr, may be None); accumulates
        nothing: weight gradients are overwritten.  If dose_grad is given, writes
        dL/d dose (the input dose of the last forward, including its effect through
        the normalisation 1 / max dose) into it."""
        lib, s = _lib(), self._s()
        n0 = self.npos[0]
        hw, _ = self.head()
        dhead = self.grads[self.head_off:self.head_off + 2 * HEAD_C + 2] if weights else None
        g = self.gbuf
        _ck(lib.pdrt_net_head_backward(n0, HEAD_C, _p(self.act["d1b"]), _p(hw), _p(gp), _p(gr), _p(g["d1b"]),
                                       _p(self.ws), self.ws_bytes, _p(dhead), s), "head_bwd")
        self._back("d1b", g["d1b"], self.act["d1a"], None, g["d1a"], None, weights)
        self._back("d1a", g["d1a"], self.u1, self.act["e1b"], self.gu1, self.gs1, weights)
        _ck(lib.pdrt_upsample2(ctypes.byref(self.vols[0]), 32, _p(self.gu1), _p(g["d2b"]), 1, s), "up_bwd")
        self._back("d2b", g["d2b"], self.act["d2a"], None, g["d2a"], None, weights)
        self._back("d2a", g["d2a"], self.u2, self.act["e2b"], self.gu2, self.gs2, weights)
        _ck(lib.pdrt_upsample2(ctypes.byref(self.vols[1]), 64, _p(self.gu2), _p(g["bb"]), 1, s), "up_bwd")
        self._back("bb", g["bb"], self.act["ba"], None, g["ba"], None, weights)
        self._back("ba", g["ba"], self.p2, None, self.gp2, None, weights)
        _ck(lib.pdrt_pool2(ctypes.byref(self.vols[1]), 32, _p(self.gp2), _p(g["e2b"]), 1, s), "pool_bwd")
        _ck(lib.pdrt_add_bf16(g["e2b"].numel(), _p(g["e2b"]), _p(self.gs2), _p(g["e2b"]), s), "add")
        self._back("e2b", g["e2b"], self.act["e2a"], None, g["e2a"], None, weights)
        self._back("e2a", g["e2a"], self.p1, None, self.gp1, None, weights)
        _ck(lib.pdrt_pool2(ctypes.byref(self.vols[0]), 16, _p(self.gp1), _p(g["e1b"]), 1, s), "pool_bwd")
        _ck(lib.pdrt_add_bf16(g["e1b"].numel(), _p(g["e1b"]), _p(self.gs1), _p(g["e1b"]), s), "add")
        self._back("e1b", g["e1b"], self.act["e1a"], None, g["e1a"], None, weights)
        self._back("e1a", g["e1a"], self.x0, None, self.gx0 if dose_grad is not None else None, None, weights)
        if dose_grad is not None:
            _ck(lib.pdrt_net_input_backward(n0, _p(self.gx0), _p(gp), _p(self.scale), _p(self._dose), _p(self.pred),
                                            _p(self.argmax), _p(dose_grad), _p(self.ws), self.ws_bytes, s),
                "input_bwd")

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        # (the first layer's padding input channels are zero, so their weight gradients
        # vanish and those weights stay at their zero initialisation)
        self.t += 1
        _ck(_lib().pdrt_adam_step(self.params.numel(), _p(self.params), _p(self.grads), _p(self.m), _p(self.v), lr,
                                  b1, b2, eps, self.t, self._s()), "adam")
        self.prepare()

    def train_loss(self, target, mask, count, lam=1.0, quantile=0.0):
        lib, s = _lib(), self._s()
        n0 = self.npos[0]
        inv = 1.0 / max(1.0, float(count))
        _ck(lib.pdrt_net_train_loss(n0, _p(self.pred), _p(self.resid), _p(target), _p(self.scale), _p(mask), inv,
                                    lam, quantile, _p(self.gp), _p(self.gr), _p(self.ws), self.ws_bytes,
                                    _p(self.loss), s), "loss")
        return self.loss

    def resid_head_slices(self):
        """Index ranges of the error head's parameters (its weights and bias)."""
        o = self.head_off
        return (o + HEAD_C, o + 2 * HEAD_C), (o + 2 * HEAD_C + 1, o + 2 * HEAD_C + 2)

    def scale_error_head(self, k):
        """Multiply the error estimate by k > 0 (the head is linear in its weights)."""
        if not (k > 0.0 and math.isfinite(k)):
            raise ValueError("error-head scale must be positive and finite")
        for a, b in self.resid_head_slices():
            self.params[a:b] *= k
        self.prepare()

    def state(self):
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "t": self.t}

    def load(self, st):
        """Parameters (and, if present, the Adam state) from a dict or npz archive."""
        if "layers" in st and [str(x) for x in st["layers"]] != [l[0] for l in LAYERS]:
            raise ValueError("the stored network has a different layer list")
        p = np.asarray(st["params"], dtype=np.float32)
        if p.size != self.params.numel():
            raise ValueError("stored parameter count %d != %d" % (p.size, self.params.numel()))
        self.params.copy_(torch.tensor(p, device=self.dev))
        if "m" in st and "v" in st:
            self.m.copy_(torch.tensor(st["m"], device=self.dev))
            self.v.copy_(torch.tensor(st["v"], device=self.dev))
            self.t = int(st["t"])
        else:
            self.m.zero_()
            self.v.zero_()
            self.t = 0
        self.prepare()

    @classmethod
    def from_file(cls, path, dims, device="cuda"):
        net = cls(dims, device=device)
        with np.load(path) as st:
            net.load({k: st[k] for k in st.files})
        return net


# ---------------------------------------------------------------------- data


def pair(plan_index, small=9, large=61, device="cuda"):
    """(small-kernel dose, large-kernel dose, density) of a randomised 128^3 plan."""
    case = inputs.config_c4_plan(plan_index, n_taps=large)
    e_small = E.DoseEngine(case, n_taps=small, device=device)
    e_large = E.DoseEngine(case, n_taps=large, device=device)
    dev = e_small.device
    lv = torch.tensor(case.leaves, dtype=torch.float32, device=dev)
    jw = torch.tensor(case.jaws, dtype=torch.float32, device=dev)
    mu = torch.tensor(case.mu, dtype=torch.float32, device=dev)
    ds = e_small.forward(lv, jw, mu).reshape(-1)
    dl = e_large.forward(lv, jw, mu).reshape(-1)
    return ds, dl, e_small.rho.reshape(-1), case


def train(net: Net3D, plans, steps, lr=1e-3, log_every=50, lam=1.0, log=print, quantile=0.0, error_head_only=False):
    """Train on precomputed pairs [(ds, dl, rho, mask)], cycling through them.  With
    error_head_only the gradients of every parameter but the error head's are
    cleared before each update (the prediction is left as it is)."""
    t0 = time.perf_counter()
    hist = []
    keep = net.resid_head_slices() if error_head_only else None
    for it in range(steps):
        ds, dl, rho, mask, count = plans[it % len(plans)]
        net.forward(ds, rho)
        loss = net.train_loss(dl, mask, count, lam, quantile)
        net.backward(net.gp, net.gr, weights=True)
        if keep:
            (a0, a1), (b0, b1) = keep
            net.grads[:a0].zero_()
            net.grads[a1:b0].zero_()
            net.grads[b1:].zero_()
        net.adam(lr)
        if (it + 1) % log_every == 0 or it == 0:
            lv = float(loss)
            hist.append((it + 1, lv))
            log("[learned] step %d loss %.3e (%.1f s)" % (it + 1, lv, time.perf_counter() - t0))
    return hist


class LearnedDose:
    """Small-kernel engine + network, with the plain large-kernel engine as the
    fallback.  Forward returns the dose in the engine's units."""

    def __init__(self, net: Net3D, case, small=9, large=61, threshold=0.01, cutoff=0.1, mode="auto"):
        """mode: "auto" (fall back when the estimated error is too large), "always"
        or "never" (forced, for tests and timing)."""
        assert mode in ("auto", "always", "never")
        self.mode = mode
        self.net = net
        self.small = E.DoseEngine(case, n_taps=small)
        self.large = E.DoseEngine(case, n_taps=large)
        self.threshold = threshold
        self.cutoff = cutoff
        self.n = int(np.prod(case.shape))
        self.shape = case.shape
        self.out = torch.empty(self.n, dtype=torch.float32, device=self.small.device)
        self.dsmall = torch.empty(self.n, dtype=torch.float32, device=self.small.device)
        self.ddose = torch.empty(self.n, dtype=torch.float32, device=self.small.device)
        self.fell_back = False
        self.generation = 0

    def forward(self, lv, jw, mu):
        """The dose of (lv, jw, mu) as a new tensor.  The network keeps this call's
        activations (and the fallback decision) for `backward`, which therefore
        always differentiates the most recent forward; `self.generation` numbers
        the forwards so a caller can check the pairing (backward(..., generation=g))."""
        self.generation += 1
        lib, s = _lib(), torch.cuda.current_stream().cuda_stream
        self.small.forward(lv, jw, mu, out=self.dsmall.view(*self.shape))
        pred, resid = self.net.forward(self.dsmall, self.small.rho.reshape(-1))
        _ck(lib.pdrt_net_fallback_stats(self.n, _p(pred), _p(resid), self.cutoff, _p(self.net.stats), _p(self.net.ws),
                                        self.net.ws_bytes, s), "stats")
        if self.mode == "auto":
            st = self.net.stats.cpu()
            self.fell_back = bool(st[1] > self.threshold * st[0])
        else:
            self.fell_back = self.mode == "always"
        if self.fell_back:
            return self.large.forward(lv, jw, mu)
        _ck(lib.pdrt_scale_by(self.n, _p(pred), _p(self.net.scale), 1, _p(self.out), s), "scale")
        return self.out.view(*self.shape).clone()

    def backward(self, lv, jw, mu, g, generation=None):
        """Gradient of L with dL/d dose = g through the path the most recent forward
        took (the network's activations are that forward's); with `generation` given,
        raises if a later forward has replaced them."""
        if generation is not None and generation != self.generation:
            raise RuntimeError("LearnedDose.backward: forward %d was followed by forward %d; the network holds "
                               "the activations of the latest one only" % (generation, self.generation))
        if self.fell_back:
            return self.large.backward(lv, jw, mu, g)
        lib, s = _lib(), torch.cuda.current_stream().cuda_stream
        gflat = g.reshape(-1)
        # dose = pred / s  ->  dL/dpred = g / s
        _ck(lib.pdrt_scale_by(self.n, _p(gflat), _p(self.net.scale), 1, _p(self.net.gp), s), "scale")
        self.net.backward(self.net.gp, None, dose_grad=self.ddose, weights=False)
        return self.small.backward(lv, jw, mu, self.ddose.view(*self.shape))
