"""Network primitives of the learned correction against plain PyTorch FP32 CPU
references of the same ops (operands rounded to BF16 the way the kernels see
them).  The kernels store BF16 outputs (relative rounding <= 2^-9) and sum in
FP32, so each comparison allows 2^-7 of the reference's largest magnitude."""
import ctypes

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from tests.test_gpu_parity import _say

pytestmark = pytest.mark.gpu
TOL = 2.0 ** -7


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bf(x):
    return torch.tensor(x, dtype=torch.float32).to(torch.bfloat16)


def _to_ncdhw(x_dhwc):
    return x_dhwc.permute(3, 0, 1, 2)[None]


def _w_torch(w):  # [cout][27][cin] -> [cout][cin][3][3][3]
    cout, _, cin = w.shape
    return w.reshape(cout, 3, 3, 3, cin).permute(0, 4, 1, 2, 3)


def _close(name, got, ref):
    scale = ref.abs().max().item()
    err = (got - ref).abs().max().item() / max(scale, 1e-30)
    _say("%s: max err / max|ref| = %.3e" % (name, err))
    assert err <= TOL, name


@pytest.mark.parametrize("dims,c1,c2,cout,relu", [
    ((4, 6, 8), 16, 0, 16, 1), ((6, 5, 7), 16, 0, 32, 1), ((4, 4, 4), 32, 0, 64, 0),
    ((4, 6, 6), 64, 32, 32, 1), ((5, 4, 6), 32, 16, 16, 1),
])
def test_conv3d_forward_backward(dims, c1, c2, cout, relu):
    from paper_2512_18863_amd.learned import Vol, _lib
    _say("conv3d %s c1=%d c2=%d cout=%d relu=%d" % (dims, c1, c2, cout, relu))
    lib = _lib()
    rng = np.random.default_rng(c1 + 7 * cout)
    D, H, W = dims
    cin = c1 + c2
    x = _bf(rng.normal(size=(D, H, W, cin)))
    w = rng.normal(0, 0.2, size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    dy = _bf(rng.normal(size=(D, H, W, cout)))
    dev = "cuda"
    s = torch.cuda.current_stream().cuda_stream
    x1 = x[..., :c1].contiguous().to(dev)
    x2 = x[..., c1:].contiguous().to(dev) if c2 else None
    wg = torch.tensor(w, device=dev)
    bg = torch.tensor(b, device=dev)
    wt = torch.empty(cout * lib.pdrt_conv3d_kpad(cin), dtype=torch.bfloat16, device=dev)
    wd = torch.empty(cin * lib.pdrt_conv3d_kpad(cout), dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_conv3d_prepare_weights(cout, cin, wg.data_ptr(), wt.data_ptr(), wd.data_ptr(), s) == 0
    y = torch.empty((D, H, W, cout), dtype=torch.bfloat16, device=dev)
    v = Vol(D, H, W)
    assert lib.pdrt_conv3d_forward(ctypes.byref(v), c1, c2, x1.data_ptr(), x2.data_ptr() if c2 else None, cout,
                                   wt.data_ptr(), bg.data_ptr(), relu, y.data_ptr(), s) == 0
    # reference in FP32 on the CPU with the operands the kernel sees
    xr = _to_ncdhw(x.float()).requires_grad_()
    wr = _w_torch(torch.tensor(w).to(torch.bfloat16).float()).requires_grad_()
    br = torch.tensor(b).requires_grad_()
    yr = Fn.conv3d(xr, wr, br, padding=1)
    if relu:
        yr = torch.relu(yr)
    _close("forward", _to_ncdhw(y.float().cpu()), yr.detach())
    # data gradient (through the activation of the kernel's own output)
    dx1 = torch.empty((D, H, W, c1), dtype=torch.bfloat16, device=dev)
    dx2 = torch.empty((D, H, W, c2), dtype=torch.bfloat16, device=dev) if c2 else None
    dyg = dy.to(dev)
    assert lib.pdrt_conv3d_backward_data(ctypes.byref(v), cout, dyg.data_ptr(), y.data_ptr() if relu else None, c1, c2,
                                         wd.data_ptr(), dx1.data_ptr(), dx2.data_ptr() if c2 else None, s) == 0
    # weight gradient
    nsplit = 3
    wsb = lib.pdrt_conv3d_wgrad_ws_bytes(cout, cin, nsplit)
    ws = torch.empty(wsb // 4, dtype=torch.float32, device=dev)
    dw = torch.empty((cout, 27, cin), dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    assert lib.pdrt_conv3d_backward_weight(ctypes.byref(v), c1, c2, x1.data_ptr(), x2.data_ptr() if c2 else None,
                                           cout, dyg.data_ptr(), y.data_ptr() if relu else None, nsplit,
                                           ws.data_ptr(), wsb, dw.data_ptr(), db.data_ptr(), s) == 0
    torch.cuda.synchronize()
    # the kernel masks with its own (BF16) activation; use the same mask in the reference
    mask = (_to_ncdhw(y.float().cpu()) > 0).float() if relu else 1.0
    yl = Fn.conv3d(xr, wr, br, padding=1)
    yl.backward(_to_ncdhw(dy.float()) * mask)
    dx = torch.cat([dx1.float().cpu(), dx2.float().cpu()], dim=-1) if c2 else dx1.float().cpu()
    _close("data grad", _to_ncdhw(dx), xr.grad)
    _close("weight grad", _w_torch(dw.cpu()), wr.grad)
    _close("bias grad", db.cpu(), br.grad)


def test_pool_upsample_head_loss_adam():
    from paper_2512_18863_amd.learned import Vol, _lib
    _say("pool / upsample / head / loss / adam")
    lib = _lib()
    dev = "cuda"
    s = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(3)
    D, H, W, C = 4, 6, 8, 16
    x = _bf(rng.normal(size=(D, H, W, C)))
    xg = x.to(dev)  # keep a reference while the kernels are in flight
    v = Vol(D, H, W)
    y = torch.empty((D // 2, H // 2, W // 2, C), dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_pool2(ctypes.byref(v), C, xg.data_ptr(), y.data_ptr(), 0, s) == 0
    ref = Fn.avg_pool3d(_to_ncdhw(x.float()), 2)
    _close("pool", _to_ncdhw(y.float().cpu()), ref)
    u = torch.empty((D, H, W, C), dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_upsample2(ctypes.byref(v), C, y.data_ptr(), u.data_ptr(), 0, s) == 0
    _close("upsample", _to_ncdhw(u.float().cpu()), Fn.interpolate(_to_ncdhw(y.float().cpu()), scale_factor=2,
                                                                   mode="nearest"))
    # backward of pooling and upsampling are the transposes: <A x, y> = <x, A^T y>
    g = _bf(rng.normal(size=(D // 2, H // 2, W // 2, C))).to(dev)
    gx = torch.empty((D, H, W, C), dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_pool2(ctypes.byref(v), C, g.data_ptr(), gx.data_ptr(), 1, s) == 0
    lhs = (y.float() * g.float()).sum().item()
    rhs = (xg.float() * gx.float()).sum().item()
    assert abs(lhs - rhs) <= 1e-2 * max(1.0, abs(lhs))
    # upsampling's backward sums the eight children of each coarse voxel
    gu = torch.empty((D // 2, H // 2, W // 2, C), dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_upsample2(ctypes.byref(v), C, gx.data_ptr(), gu.data_ptr(), 1, s) == 0
    ref_u = _to_ncdhw(gx.float().cpu())
    ref_u = ref_u.reshape(1, C, D // 2, 2, H // 2, 2, W // 2, 2).sum(dim=(3, 5, 7))
    _close("upsample backward", _to_ncdhw(gu.float().cpu()), ref_u)
    # eight channels per thread: c must be a multiple of 8 and the buffers 16-byte aligned
    assert lib.pdrt_pool2(ctypes.byref(v), 12, xg.data_ptr(), y.data_ptr(), 0, s) == -1
    assert lib.pdrt_pool2(ctypes.byref(v), C, xg.data_ptr() + 2, y.data_ptr(), 0, s) == -1
    # add in groups of eight with a tail
    na = 1003
    a1 = _bf(rng.normal(size=na)).to(dev)
    a2 = _bf(rng.normal(size=na)).to(dev)
    ao = torch.empty(na, dtype=torch.bfloat16, device=dev)
    assert lib.pdrt_add_bf16(na, a1.data_ptr(), a2.data_ptr(), ao.data_ptr(), s) == 0
    assert torch.equal(ao.cpu(), (a1.float() + a2.float()).to(torch.bfloat16).cpu())
    n = 500
    xh = _bf(rng.normal(size=(n, C))).to(dev)
    hw = torch.tensor(rng.normal(size=(2, C)), dtype=torch.float32, device=dev)
    hb = torch.tensor([0.1, -0.2], dtype=torch.float32, device=dev)
    dose = torch.tensor(rng.uniform(size=n), dtype=torch.float32, device=dev)
    sc = torch.tensor([2.0], dtype=torch.float32, device=dev)
    pred = torch.empty(n, dtype=torch.float32, device=dev)
    resid = torch.empty(n, dtype=torch.float32, device=dev)
    assert lib.pdrt_net_head(n, C, xh.data_ptr(), hw.data_ptr(), hb.data_ptr(), dose.data_ptr(), sc.data_ptr(),
                             pred.data_ptr(), resid.data_ptr(), s) == 0
    ref_p = dose * 2.0 + hb[0] + xh.float() @ hw[0]
    ref_r = hb[1] + xh.float() @ hw[1]
    assert torch.allclose(pred, ref_p, rtol=1e-5, atol=1e-5)
    assert torch.allclose(resid, ref_r, rtol=1e-5, atol=1e-5)
    # Adam against torch.optim.Adam on the CPU
    wv = torch.tensor(rng.normal(size=300), dtype=torch.float32)
    gv = torch.tensor(rng.normal(size=300), dtype=torch.float32)
    wref = wv.clone().requires_grad_()
    opt = torch.optim.Adam([wref], lr=1e-2)
    wgpu, ggpu = wv.clone().to(dev), gv.to(dev)
    m, vv = torch.zeros_like(wgpu), torch.zeros_like(wgpu)
    for t in range(1, 4):
        wref.grad = gv.clone()
        opt.step()
        assert lib.pdrt_adam_step(300, wgpu.data_ptr(), ggpu.data_ptr(), m.data_ptr(), vv.data_ptr(), 1e-2, 0.9,
                                  0.999, 1e-8, t, s) == 0
    assert torch.allclose(wgpu.cpu(), wref.detach(), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("quantile", [0.0, 0.9])
def test_train_loss_against_autograd(quantile):
    """The training loss and its gradients against torch autograd on the CPU (FP64):
    squared error of the prediction plus lam times either the squared error of the
    error estimate (quantile 0) or the pinball loss of the quantile of |error|;
    the second term's gradient reaches the error estimate only."""
    from paper_2512_18863_amd.learned import _lib
    _say("train loss, quantile %.2f" % quantile)
    lib = _lib()
    dev = "cuda"
    s = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(21)
    n = 3000                                  # several blocks of 256 and a ragged tail
    pred_h = torch.tensor(rng.normal(size=n), dtype=torch.float64)
    resid_h = torch.tensor(rng.uniform(0.0, 2.0, size=n), dtype=torch.float64)
    target_h = torch.tensor(rng.normal(size=n), dtype=torch.float64)
    mask_h = torch.tensor(rng.uniform(size=n) < 0.7, dtype=torch.float64)
    tscale, lam, count = 1.3, 0.7, float(mask_h.sum())
    f32 = lambda a: a.to(torch.float32).to(dev)
    pred, resid, target, mask = f32(pred_h), f32(resid_h), f32(target_h), f32(mask_h)
    ts = torch.tensor([tscale], dtype=torch.float32, device=dev)
    gp = torch.empty(n, dtype=torch.float32, device=dev)
    gr = torch.empty(n, dtype=torch.float32, device=dev)
    wsb = lib.pdrt_net_loss_ws_bytes(n)
    ws = torch.empty(wsb // 4, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    assert lib.pdrt_net_train_loss(n, pred.data_ptr(), resid.data_ptr(), target.data_ptr(), ts.data_ptr(),
                                   mask.data_ptr(), 1.0 / count, lam, quantile, gp.data_ptr(), gr.data_ptr(),
                                   ws.data_ptr(), wsb, loss.data_ptr(), s) == 0
    torch.cuda.synchronize()
    # the reference sees the FP32 inputs
    p = pred.double().cpu().requires_grad_()
    r = resid.double().cpu().requires_grad_()
    e = p - target.double().cpu() * float(ts.item())
    m = mask.double().cpu()
    # the error estimate's term does not reach the prediction (its |e| is a constant)
    ae = e.detach().abs()
    if quantile == 0.0:
        term = (r - ae) ** 2
    else:
        u = ae - r
        term = u * (quantile - (u < 0).double())
    ref = (m * (e ** 2 + lam * term)).sum() / count
    ref.backward()
    assert abs(loss.item() - ref.item()) <= 1e-5 * abs(ref.item())
    assert torch.allclose(gp.double().cpu(), p.grad, rtol=1e-5, atol=1e-7)
    assert torch.allclose(gr.double().cpu(), r.grad, rtol=1e-5, atol=1e-7)
    # the quantile must lie in [0, 1)
    for bad in (-0.1, 1.0, float("nan")):
        assert lib.pdrt_net_train_loss(n, pred.data_ptr(), resid.data_ptr(), target.data_ptr(), ts.data_ptr(),
                                       mask.data_ptr(), 1.0 / count, lam, bad, gp.data_ptr(), gr.data_ptr(),
                                       ws.data_ptr(), wsb, loss.data_ptr(), s) == -1


def test_learned_training_reduces_loss_and_fallback_is_plain():
    """A few hundred steps on a handful of 64^3 plans reduce the training loss;
    forced to fall back, the learned path and returns the plain
    large-kernel dose bit for bit."""
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import inputs, learned
    _say("learned path: short training on 64^3 plans, forced fallback")
    import copy
    plans = []
    for p in range(4):
        c = inputs.config_c4_plan(p, n_taps=61)
        c.hu = c.hu[32:96, 32:96, 32:96].copy()
        c.origin = inputs._centred_origin(c.hu.shape, c.spacing)
        c.gantry, c.leaves, c.jaws, c.mu = c.gantry[:20], c.leaves[:20], c.jaws[:20], c.mu[:20]
        es = E.DoseEngine(c, n_taps=9)
        el = E.DoseEngine(c, n_taps=61)
        t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
        ds = es.forward(t(c.leaves), t(c.jaws), t(c.mu)).reshape(-1).clone()
        dl = el.forward(t(c.leaves), t(c.jaws), t(c.mu)).reshape(-1).clone()
        mask = (dl >= 0.05 * dl.max()).float()
        plans.append((ds, dl, es.rho.reshape(-1).clone(), mask, float(mask.sum())))
        last = c
    net = learned.Net3D((64, 64, 64), seed=1)
    hist = learned.train(net, plans, 120, lr=2e-3, log_every=40, log=_say)
    assert hist[-1][1] < 0.7 * hist[0][1]
    ld = learned.LearnedDose(net, last, mode="always")
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    out = ld.forward(t(last.leaves), t(last.jaws), t(last.mu))
    plain = E.DoseEngine(last, n_taps=61).forward(t(last.leaves), t(last.jaws), t(last.mu))
    assert ld.fell_back and torch.equal(out, plain)


class _RoundBF16(torch.autograd.Function):
    """BF16 storage of an activation in the forward, identity in the backward."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).float()

    @staticmethod
    def backward(ctx, g):
        return g


def _torch_unet(net, ds, rho, dims):
    """The learned correction's forward in FP32 torch on the CPU (weights rounded to
    BF16 as the kernels see them, activations stored as BF16), returning the dose
    out = pred / s with s = 1 / max(ds)."""
    from paper_2512_18863_amd.learned import HEAD_C, LAYERS
    D, H, W = dims
    r = _RoundBF16.apply
    s = 1.0 / ds.max()
    x0 = torch.zeros(1, 16, D, H, W)
    x0 = torch.cat([(ds * s).reshape(1, 1, D, H, W), rho.reshape(1, 1, D, H, W), x0[:, 2:]], dim=1)
    x0 = r(x0)
    prm = net.params.detach().cpu()
    act = {}

    def conv(name, x):
        (_, c1, c2, cout, _) = next(l for l in LAYERS if l[0] == name)
        o, nw, bo, _ = net.slices[name]
        w = prm[o:o + nw].reshape(cout, 27, c1 + c2).to(torch.bfloat16).float()
        y = torch.relu(Fn.conv3d(x, _w_torch(w), prm[bo:bo + cout], padding=1))
        act[name] = r(y)
        return act[name]

    s1 = conv("e1b", conv("e1a", x0))
    s2 = conv("e2b", conv("e2a", r(Fn.avg_pool3d(s1, 2))))
    b = conv("bb", conv("ba", r(Fn.avg_pool3d(s2, 2))))
    c2 = conv("d2b", conv("d2a", torch.cat([Fn.interpolate(b, scale_factor=2, mode="nearest"), s2], dim=1)))
    c1 = conv("d1b", conv("d1a", torch.cat([Fn.interpolate(c2, scale_factor=2, mode="nearest"), s1], dim=1)))
    ho = net.head_off
    hw = prm[ho:ho + 2 * HEAD_C].reshape(2, HEAD_C)
    hb = prm[ho + 2 * HEAD_C:ho + 2 * HEAD_C + 2]
    feat = c1.reshape(HEAD_C, -1)
    pred = ds * s + hb[0] + hw[0] @ feat
    return pred / s


def test_learned_dose_gradient_matches_torch_autograd():
    """d(sum g * out)/d(small dose) through the whole network, including the
    normalisation by the maximum dose (its argmax voxel gets the extra term),
    against torch autograd of the same network on the CPU."""
    from paper_2512_18863_amd import learned
    _say("learned input gradient vs torch autograd, 16^3")
    lib = learned._lib()
    dims = (16, 16, 16)
    n = 16 ** 3
    net = learned.Net3D(dims, seed=5)
    rng = np.random.default_rng(11)
    # larger weights than the initialisation so every layer matters
    p = net.params.detach().cpu().numpy()
    for (name, c1, c2, cout, lvl) in learned.LAYERS:
        o, nw, bo, _ = net.slices[name]
        p[o:o + nw] = rng.normal(0.0, np.sqrt(2.0 / (27 * (c1 + c2))), size=nw)
        p[bo:bo + cout] = rng.normal(0.0, 0.05, size=cout)
    ho = net.head_off
    p[ho:ho + 2 * learned.HEAD_C + 2] = rng.normal(0.0, 0.3, size=2 * learned.HEAD_C + 2)
    net.params.copy_(torch.tensor(p))
    net.prepare()
    ds_h = torch.tensor(rng.uniform(0.1, 1.0, size=n), dtype=torch.float32)
    ds_h[1234] = 1.7                         # a unique maximum
    rho_h = torch.tensor(rng.uniform(0.0, 1.5, size=n), dtype=torch.float32)
    g_h = torch.tensor(rng.normal(size=n), dtype=torch.float32)
    ds, rho, g = ds_h.cuda(), rho_h.cuda(), g_h.cuda()
    s = torch.cuda.current_stream().cuda_stream
    pred, _ = net.forward(ds, rho)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    assert lib.pdrt_scale_by(n, pred.data_ptr(), net.scale.data_ptr(), 1, out.data_ptr(), s) == 0
    gp = torch.empty(n, dtype=torch.float32, device="cuda")
    assert lib.pdrt_scale_by(n, g.data_ptr(), net.scale.data_ptr(), 1, gp.data_ptr(), s) == 0
    ddose = torch.empty(n, dtype=torch.float32, device="cuda")
    net.backward(gp, None, dose_grad=ddose, weights=False)
    torch.cuda.synchronize()
    assert int(net.argmax.item()) == 1234
    x = ds_h.clone().requires_grad_()
    ref_out = _torch_unet(net, x, rho_h, dims)
    (ref_out * g_h).sum().backward()
    _close("learned dose", out.cpu(), ref_out.detach())
    got = ddose.cpu()
    # ten BF16 layers forward and back: each stores activations and gradients with
    # <= 2^-9 relative rounding, so allow 2^-5 of the largest reference gradient
    m = 1234
    keep = torch.ones(n, dtype=torch.bool)
    keep[m] = False
    err = (got[keep] - x.grad[keep]).abs().max().item() / x.grad[keep].abs().max().item()
    err_m = abs(got[m].item() - x.grad[m].item()) / abs(x.grad[m].item())
    _say("input gradient: max err / max|ref| %.3e; argmax voxel got %.6e ref %.6e (rel %.2e)" %
         (err, got[m].item(), x.grad[m].item(), err_m))
    assert err <= 2.0 ** -5 and err_m <= 2.0 ** -5
    # the output is homogeneous of degree one in the dose, so <grad, ds> = <g, out>
    # (this fails without the normalisation's term at the argmax)
    lhs = float((got.double() * ds_h.double()).sum())
    rhs = float((g_h.double() * out.cpu().double()).sum())
    assert abs(lhs - rhs) <= 1e-4 * float((g_h.abs().double() * out.cpu().abs().double()).sum())


def test_learned_held_out_plans_vs_plain_61():
    """Ten held-out plans (indices 2000-2009, never trained on: training used 0-1999)
    with their own randomised 128^3 pelvis, 60-180 control points and jaws 20-50 mm:
    the learned dose (9 x 9 engine + network, fallback rule live) against the plain
    61 x 61 FP32 dose, the judge of its error.  Bar: 1 %/1 mm global gamma >= 99.5 %
    (10 % threshold); the maximum error, the network's own error estimate and the
    fallback decision are stated per plan."""
    import os
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import gamma, inputs, learned
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2512_18863_amd", "data",
                        "learned_c4.npz")
    net = learned.Net3D.from_file(path, (128, 128, 128))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    for p in range(2000, 2010):
        case = inputs.config_c4_plan(p, n_taps=61)
        lv, jw, mu = t(case.leaves), t(case.jaws), t(case.mu)
        ld = learned.LearnedDose(net, case, mode="auto")
        out = ld.forward(lv, jw, mu).cpu().numpy().astype(np.float64)
        st = net.stats.cpu().numpy()
        plain = E.DoseEngine(case, n_taps=61).forward(lv, jw, mu).cpu().numpy().astype(np.float64)
        err = float(np.abs(out - plain).max() / plain.max())
        gp = gamma.pass_rate(plain, out, case.spacing, 1.0, 1.0)
        _say("held-out plan %d (%d CPs, jaws %.0f x %.0f mm): fallback %s, estimate %.2e, max|dD|/maxD %.3e, "
             "gamma(1%%/1mm) %.4f %%" % (p, case.n_cp, 2 * case.jaws[0, 1], 2 * case.jaws[0, 3], ld.fell_back,
                                         st[1] / st[0], err, 100 * gp))
        assert gp >= 0.995, p
        assert err <= 0.02, p
        del ld
        torch.cuda.empty_cache()


def test_learned_error_estimate_flags_unfamiliar_anatomy():
    """The error head's estimate as a failure detector, on held-out plan 2000: on its
    own pelvis and on anatomies whose learned-dose error stays in the usual range
    (soft tissue set to lung or bone density, all water) the largest estimate stays
    below 1 % of the largest dose and the learned dose is used; on a grid of
    alternating 24 mm slabs of bone and air (no training phantom is like it) the
    learned dose is off by more than 1 %, the estimate says so and the path falls
    back to the plain 61 x 61 dose, bit for bit."""
    import os
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import inputs, learned
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2512_18863_amd", "data",
                        "learned_c4.npz")
    net = learned.Net3D.from_file(path, (128, 128, 128))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    cases = [("pelvis", inputs.config_c4_plan(2000))] + [(k, inputs.config_c4_ood(k)) for k in inputs.C4_OOD_KINDS]
    for kind, case in cases:
        lv, jw, mu = t(case.leaves), t(case.jaws), t(case.mu)
        plain = E.DoseEngine(case, n_taps=61).forward(lv, jw, mu)
        raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu)
        err = float((raw - plain).abs().max() / plain.max())
        ld = learned.LearnedDose(net, case, mode="auto")
        out = ld.forward(lv, jw, mu)
        st = net.stats.cpu().numpy()
        est = float(st[1] / st[0])
        _say("plan 2000, %s: learned-dose max error %.3e, estimate %.3e, fallback %s" % (kind, err, est, ld.fell_back))
        if kind == "bone_air_slabs":
            assert err > 0.01 and est > ld.threshold and ld.fell_back
            assert torch.equal(out, plain)
        else:
            assert err < 0.01 and est < ld.threshold and not ld.fell_back
        del ld, raw, plain, out
        torch.cuda.empty_cache()
