"""Index arithmetic of the BF16 lateral convolution (arXiv:2512.18863 §2.2.6,
Eq. 8, BF16 operands with FP32 accumulation), modelled on the CPU.

One workgroup computes one plane.  Forward: the input is zero outside the
aperture rectangle (the box) and every output within the box's reach (box +- h)
is computed, the rest of the plane written as zero; adjoint: only the outputs
inside the box, from the inputs in their reach.  Outputs come in 16 x 16 tiles,
register blocks of 6 x 3 tiles (forward, two wavefronts) or 2 x 2 tiles whose
tap rows four wavefronts split (adjoint); for each tap row p and 32-column K-step,
a row tile's A fragment (16 input rows x 32 columns from an LDS image) is used
only if its rows meet the input support, a column tile's B fragment (eight
entries per lane from one of two padded BF16 copies of the tap row, the second
shifted by one element) only if the K-step lies in its reach, lanes whose run is
wholly outside the band |c - n| <= h taking zeros.  Inputs that do not fit the
image are processed in row and column chunks.

This model follows the kernel's integer arithmetic and checks, for random plane
sizes, kernel sizes and boxes (typical, wide, at the plane's edges, empty), that
every image read lies inside the rows staged for its chunk and inside the image
capacity the host sizes, every tap row runs exactly once per block and chunk,
every tap-row read lies inside the padded row, and the result equals a direct correlation of the BF16-rounded input with the
BF16-rounded taps (exact products, so only the summation order differs).  It
needs no GPU.
"""
import math
import random

import numpy as np
import pytest
from scipy import ndimage


def bf16(x):
    """Round to nearest even BF16, returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def box_extent(F, D, c, N):
    fa, fb = -F / D + c - 0.5, F / D + c + 0.5
    lo, hi = max(0, math.floor(fa) - 1), min(N, math.ceil(fb) + 1)
    return hi - lo if hi > lo else 1


def host_plan(Nu, Nv, h, fwd, lat=3.0):
    """The launcher's sizing: NK, image rows, pitch, padded tap row, block shape."""
    Fu, Fv = ((Nu - 1) // 2 - h) * lat, ((Nv - 1) // 2 - h) * lat
    br = box_extent(Fu, lat, 0.5 * (Nu - 1), Nu)
    bc = box_extent(Fv, lat, 0.5 * (Nv - 1), Nv)
    in_cols = bc if fwd else min(bc + 2 * h, Nv)
    nk = min(3, max(1, (in_cols + 31) // 32))
    BR, BC, NWB, NWP = (6, 3, 2, 1) if fwd else (2, 2, 1, 4)
    out_rows = min(br + 2 * h, Nu) if fwd else br
    tr = (out_rows + 15) // 16
    in_rows = br if fwd else min(br + 2 * h, Nu)
    rows = max(min(in_rows + 30, 16 * tr + 2 * h), 31)
    pitch = 32 * nk + 8
    red_rows = (NWB * (NWP - 1) * BR * BC * 1024 + 2 * pitch - 1) // (2 * pitch)
    return dict(NK=nk, img_rows=max(rows, red_rows), pitch=pitch, L=2 * h + 16, X0=h + 8, BR=BR, BC=BC, NWP=NWP)


def model(inp, K, h, box, fwd, plan):
    """The kernel on one plane: returns the output (NaN where not written)."""
    Nu, Nv = inp.shape
    NK, L, X0, BR, BC, NWP = plan["NK"], plan["L"], plan["X0"], plan["BR"], plan["BC"], plan["NWP"]
    out = np.full((Nu, Nv), np.nan)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    empty = u1 <= u0 or v1 <= v0
    if fwd:
        ir0, ir1, ic0, ic1 = u0, u1, v0, v1
        or0, or1, oc0, oc1 = max(0, u0 - h), min(Nu, u1 + h), max(0, v0 - h), min(Nv, v1 + h)
        if empty:
            or0 = or1 = oc0 = oc1 = 0
        mask = np.ones((Nu, Nv), bool)
        mask[or0:or1, oc0:oc1] = False
        out[mask] = 0.0
        if empty:
            return out
    else:
        if empty:
            return out
        or0, or1, oc0, oc1 = u0, u1, v0, v1
        ir0, ir1, ic0, ic1 = max(0, u0 - h), min(Nu, u1 + h), max(0, v0 - h), min(Nv, v1 + h)
    # padded tap rows: T0[a][x] = K[a][|x - X0|] inside the band
    T0 = np.zeros((h + 1, L + 1))
    for a in range(h + 1):
        for x in range(L):
            qq = abs(x - X0)
            if qq <= h:
                T0[a, x] = bf16(K[a, qq])
    TR, TC = (or1 - or0 + 15) // 16, (oc1 - oc0 + 15) // 16
    KC = 32 * NK
    rows_all = min(ir1 - ir0 + 30, 16 * TR + 2 * h)
    rch = ir1 - ir0 if rows_all <= plan["img_rows"] else plan["img_rows"] - 30
    assert rch >= 1
    m = np.arange(16)
    nbc = (TC + BC - 1) // BC
    for blk in range(((TR + BR - 1) // BR) * nbc):
        rb, cb = (blk // nbc) * BR, (blk % nbc) * BC
        nr, nc = min(BR, TR - rb), min(BC, TC - cb)
        OI0, OJ0 = or0 + 16 * rb, oc0 + 16 * cb
        acc = np.zeros((nr, nc, 16, 16))
        for cr0 in range(ir0, ir1, rch):
            cr1 = min(ir1, cr0 + rch)
            for cc0 in range(ic0, ic1, KC):
                cc1 = min(ic1, cc0 + KC)
                IR0 = max(cr0 - 15, or0 - h)
                nrows = min(cr1 + 15, or0 + 16 * TR + h) - IR0
                assert 0 < nrows <= plan["img_rows"], (nrows, plan["img_rows"])
                img = np.zeros((nrows, KC))
                for rr in range(nrows):
                    i = IR0 + rr
                    if cr0 <= i < cr1:
                        img[rr, :cc1 - cc0] = bf16(inp[i, cc0:cc1])
                p_lo, p_hi = max(-h, cr0 - (OI0 + 16 * nr - 1)), min(h, cr1 - 1 - OI0)
                if p_hi < p_lo:
                    continue
                np_ = p_hi - p_lo + 1
                ran = []
                for wp in range(NWP):   # the parts split the tap rows: every p exactly once
                    pa, pz = p_lo + (np_ * wp) // NWP, p_lo + (np_ * (wp + 1)) // NWP
                    for p in range(pa, pz):
                        ap = abs(p)
                        ran.append(p)
                        B = {}
                        for t in range(BC):
                            n0 = OJ0 + 16 * t
                            for s in range(NK):
                                c0 = cc0 + 32 * s
                                Bm = np.zeros((32, 16))
                                for kq in range(4):
                                    x = c0 + 8 * kq - n0 - m + X0          # per column n0 + m
                                    live = (t < nc) & (c0 < cc1) & (x + 7 >= X0 - h) & (x <= X0 + h)
                                    for col in range(16):
                                        if live[col]:
                                            xs = x[col]
                                            # dword reads (xs >> 1) .. + 3 of the copy of parity xs & 1
                                            assert 0 <= xs and xs + 7 <= L - 1, (xs, L)
                                            assert (xs >> 1) + 3 <= L // 2 - 1
                                            Bm[8 * kq:8 * kq + 8, col] = T0[ap, xs:xs + 8]
                                B[(t, s)] = Bm
                        for r in range(nr):
                            i0 = OI0 + 16 * r
                            if i0 + p + 15 < cr0 or i0 + p >= cr1:
                                continue
                            rows = i0 + p + m - IR0
                            assert rows.min() >= 0 and rows.max() < nrows
                            for s in range(NK):
                                A = img[rows][:, 32 * s:32 * s + 32]
                                for t in range(nc):
                                    acc[r, t] += A @ B[(t, s)]
                assert sorted(ran) == list(range(p_lo, p_hi + 1))
        for r in range(nr):
            for t in range(nc):
                for e in range(16):
                    i = OI0 + 16 * r + e
                    if i >= or1:
                        continue
                    for c in range(16):
                        j = OJ0 + 16 * t + c
                        if j < oc1:
                            out[i, j] = acc[r, t, e, c]
    return out


def direct(inp, K, h, box, fwd):
    Nu, Nv = inp.shape
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    full = np.zeros((2 * h + 1, 2 * h + 1))
    for p in range(-h, h + 1):
        for q in range(-h, h + 1):
            full[p + h, q + h] = bf16(K[abs(p), abs(q)])
    x = bf16(inp)
    if fwd:
        xm = np.zeros_like(x)
        if u1 > u0 and v1 > v0:
            xm[u0:u1, v0:v1] = x[u0:u1, v0:v1]
        return ndimage.correlate(xm, full, mode="constant"), None
    ref = ndimage.correlate(x, full, mode="constant")
    sel = np.zeros((Nu, Nv), bool)
    if u1 > u0 and v1 > v0:
        sel[u0:u1, v0:v1] = True
    return ref, sel


def _taps(h, rng):
    a = np.arange(h + 1)
    return np.exp(-0.15 * np.hypot(a[:, None], a[None, :])) * rng.uniform(0.5, 1.0)


CASES = [
    # (Nu, Nv, h, box): the 128^3 benchmark geometry (89 x 89, n = 61, jaws +-40 mm)
    (89, 89, 30, (29, 59, 29, 59)),
    (89, 89, 30, (29, 59, 40, 41)),
    (89, 89, 30, (0, 89, 0, 89)),          # box = plane: chunked rows / columns
    (89, 89, 30, (29, 29, 30, 50)),        # empty
    (43, 43, 7, (14, 29, 15, 28)),         # n = 15 plane
    (63, 63, 15, (15, 48, 10, 52)),        # n = 31, wider than the field
    (71, 71, 15, (0, 9, 60, 71)),          # corner of the plane
    (37, 41, 4, (10, 27, 12, 29)),         # n = 9, rectangular plane
]


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
@pytest.mark.parametrize("fwd", [True, False], ids=["forward", "adjoint"])
def test_bf16_conv_model_matches_direct(case, fwd):
    Nu, Nv, h, box = case
    rng = np.random.default_rng(Nu * 131 + h + (7 if fwd else 0))
    inp = rng.uniform(0.0, 1.0, size=(Nu, Nv))
    K = _taps(h, rng)
    plan = host_plan(Nu, Nv, h, fwd)
    got = model(inp, K, h, box, fwd, plan)
    ref, sel = direct(inp, K, h, box, fwd)
    if fwd:
        assert not np.isnan(got).any()
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    else:
        assert not np.isnan(got[sel]).any()
        np.testing.assert_allclose(got[sel], ref[sel], rtol=1e-12, atol=1e-12)


def test_bf16_conv_model_random_boxes():
    rnd = random.Random(5)
    for it in range(6):
        h = rnd.choice([3, 6, 12, 30])
        N = rnd.randint(2 * h + 5, 2 * h + 50)
        M = rnd.randint(2 * h + 5, 2 * h + 50)
        a, b = sorted(rnd.randint(-3, N + 3) for _ in range(2))
        c, d = sorted(rnd.randint(-3, M + 3) for _ in range(2))
        fwd = it % 2 == 0
        rng = np.random.default_rng(it)
        inp = rng.uniform(size=(N, M))
        K = _taps(h, rng)
        plan = host_plan(N, M, h, fwd)
        got = model(inp, K, h, (a, b, c, d), fwd, plan)
        ref, sel = direct(inp, K, h, (a, b, c, d), fwd)
        if fwd:
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
        else:
            np.testing.assert_allclose(got[sel], ref[sel], rtol=1e-12, atol=1e-12)
