"""Index arithmetic of the FP32 forward convolution restricted to the aperture
rectangle (arXiv:2512.18863 §2.2.6, Eq. 8, with the fluence zero outside the jaw
opening), modelled on the CPU.

The kernel computes each 16 x 16 output tile as a sum over folded tap rows p
(input rows i + p and i - p added) and 16-column super-steps of a Toeplitz
product, running only the tap rows and super-steps that reach the input
rectangle, with the region's tile grid shifted to minimise that work.  Its LDS
image is placed at the rectangle: first row max(I - h, r0 - 15), first column the
last multiple-of-4 offset of J - h not above c0 - 18, capacity
min(min(Nu, 16 TI + 2h) + 30, 16 TI + 2h) rows by
min(min(Nv, 16 TJ + 2h) + 36, 16 TJ + 16 SS) columns, reused from one item to the
next with the previous rectangle cleared outside the new one.  Horizontally
adjacent tiles whose column windows start at the same input column are run as a
pair sharing the A operand, each with its own Toeplitz offset.

This model follows the same integer arithmetic and checks, for random planes,
kernel sizes and rectangles (inside, across and outside the plane, empty), that
every image read lies inside that capacity, every Toeplitz read inside the
extended tap row, every output is written exactly once, the two tiles of every
pair read the same input window, and the result equals a direct correlation of
the masked input.  It needs no GPU.
"""
import random

import numpy as np
import pytest
from scipy import ndimage

MT, RMAX = 16, 6
PAIRS = []  # (item, left tile column) of every horizontal pair formed


def region_shape(N):
    t = (N + MT - 1) // MT
    T = min(t, RMAX)
    return T, (t + T - 1) // T


def pitch_f32(cols):
    return ((cols + 7) // 16) * 16 + 8


def row_reach(X, lo, hi, h):
    """Tap rows of the plus side [a1, b1] and minus side [a2, b2] for tile rows X..X+15."""
    return max(0, lo - X - 15), min(h, hi - X - 1), max(0, X - hi + 1), min(h, X + 15 - lo)


def col_window(X, lo, hi, h, SS):
    """Column offset o (multiple of 4) and super-step count nu for tile columns X..X+15."""
    cb = X - h
    ca, cz = max(cb, lo), min(cb + 16 * SS - 1, hi - 1)
    if cz < ca:
        return 0, 0
    o = ((ca - cb) >> 2) << 2
    nu = (cz - cb - o + 16) >> 4
    return min(o, 16 * (SS - nu)), nu


def grid_offset(N, X0, T, lo, hi, h, SS, col):
    lo, hi = max(lo, 0), min(hi, N)
    gmin = max(-15, min(0, (N - X0) - MT * T))
    end = min(N, X0 + MT * T)
    best = None
    for cand in range(16):
        if -cand < gmin:
            continue
        cost = 0
        for t in range(RMAX):
            X = X0 - cand + MT * t
            if t >= T or X >= end or hi <= lo:
                continue
            if col:
                cost += col_window(X, lo, hi, h, SS)[1]
            else:
                a1, b1, a2, b2 = row_reach(X, lo, hi, h)
                n1 = b1 - a1 + 1 if a1 <= b1 else 0
                n2 = b2 - a2 + 1 if a2 <= b2 else 0
                ov = max(0, min(b1, b2) - max(a1, a2) + 1) if n1 and n2 else 0
                cost += n1 + n2 - ov
        key = (cost << 4) | cand
        best = key if best is None else min(best, key)
    return -(best & 15)


def segments(a1, b1, a2, b2, h):
    """Tap-row segments in increasing p with the fold sides each one loads."""
    out = []
    p = min(a1 if a1 <= b1 else h + 1, a2 if a2 <= b2 else h + 1)
    top = max(b1 if a1 <= b1 else -1, b2 if a2 <= b2 else -1)
    while p <= top:
        plus, minus = a1 <= p <= b1, a2 <= p <= b2
        e = top
        if plus:
            e = min(e, b1)
        elif p < a1 <= b1:
            e = min(e, a1 - 1)
        if minus:
            e = min(e, b2)
        elif p < a2 <= b2:
            e = min(e, a2 - 1)
        out.append((p, e, plus, minus))
        p = e + 1
    return out


def pair_roles(J0p, TJ, Nv, c0, c1, nr, h, SS):
    """Roles of the tile columns (1 left tile of a pair, -1 right tile, 0 alone):
    scanning from the left, columns j and j + 1 pair when their windows start at
    the same input column with the same super-step count."""
    def window(Jc):
        if not nr or Jc >= Nv:
            return 0, 0
        return col_window(Jc, c0, c1, h, SS)
    roles = [0] * TJ
    j = 0
    while j < TJ:
        oa, na = window(J0p + MT * j)
        ob, nb = window(J0p + MT * (j + 1)) if j + 1 < TJ else (0, 0)
        if j + 1 < TJ and na > 0 and nb == na and ob == oa - 16:
            roles[j], roles[j + 1] = 1, -1
            j += 2
        else:
            j += 1
    return roles


def image_capacity(Nu, Nv, h, TI, TJ, SS):
    rows = min(min(Nu, MT * TI + 2 * h) + 30, MT * TI + 2 * h)
    cols = min(min(Nv, MT * TJ + 2 * h) + 36, MT * TJ + 16 * SS)
    return rows, cols


def forward_in_box(inputs, K, boxes):
    """One region-resident image per region, items (input, box) in sequence."""
    Nu, Nv = inputs[0].shape
    h = (K.shape[0] - 1) // 2
    TI, ri = region_shape(Nu)
    TJ, rj = region_shape(Nv)
    SS = (16 + 2 * h + 15) // 16
    E = 16 * SS + 16
    rows, cols = image_capacity(Nu, Nv, h, TI, TJ, SS)
    kx = np.zeros((h + 1, E))
    for p in range(h + 1):
        for c in range(E):
            q = c - (h + 15)
            if -h <= q <= h:
                kx[p, c] = K[h + p, h + q] * (0.5 if p == 0 else 1.0)
    outs = [np.full((Nu, Nv), np.nan) for _ in inputs]
    m = np.arange(16)[:, None]
    cidx = np.arange(16)
    for reg in range(ri * rj):
        I0, J0 = (reg // rj) * TI * MT, (reg % rj) * TJ * MT
        img = np.zeros((rows, pitch_f32(cols)))
        prev = None
        for item, (inp, (u0, u1, v0, v1)) in enumerate(zip(inputs, boxes)):
            I0p = I0 + grid_offset(Nu, I0, TI, u0, u1, h, SS, False)
            J0p = J0 + grid_offset(Nv, J0, TJ, v0, v1, h, SS, True)
            r0 = max(max(0, I0p - h), u0)
            r1 = min(min(Nu, I0p + MT * TI + h), u1)
            c0 = max(max(0, J0p - h), v0)
            c1 = min(min(Nv, J0p + MT * TJ + h), v1)
            nr = r1 - r0 if (r1 > r0 and c1 > c0) else 0
            nc = c1 - c0 if nr else 1
            R0 = max(I0p - h, r0 - 15)
            C0 = (J0p - h) + ((max(0, c0 - 18 - (J0p - h)) >> 2) << 2)
            lr0, lc0 = r0 - R0, c0 - C0
            if nr:
                assert 0 <= lr0 and lr0 + nr <= rows and 0 <= lc0 and lc0 + nc <= cols
                img[lr0:lr0 + nr, lc0:lc0 + nc] = inp[r0:r0 + nr, c0:c0 + nc]
            if prev is not None:
                pr, pnr, pc, pnc = prev
                keep = np.zeros((pnr, pnc), dtype=bool)
                rr = np.arange(pr, pr + pnr)[:, None]
                cc = np.arange(pc, pc + pnc)[None, :]
                keep = (rr >= lr0) & (rr < lr0 + nr) & (cc >= lc0) & (cc < lc0 + nc)
                img[pr:pr + pnr, pc:pc + pnc][~keep] = 0.0
            prev = (lr0, nr, lc0, nc)
            roles = pair_roles(J0p, TJ, Nv, c0, c1, nr, h, SS)
            for tj in range(TJ - 1):
                if roles[tj] == 1:
                    # the pair's two tiles read the same input columns (one A operand),
                    # and the right tile's Toeplitz offset o - 16 is its own window offset
                    oL, nL = col_window(J0p + MT * tj, c0, c1, h, SS)
                    oR, nR = col_window(J0p + MT * (tj + 1), c0, c1, h, SS)
                    assert nL == nR > 0 and oR == oL - 16 >= 0
                    assert (J0p + MT * tj - h + oL) == (J0p + MT * (tj + 1) - h + oR)
                    PAIRS.append((item, tj))
            for ti in range(TI):
                for tj in range(TJ):
                    I, J = I0p + MT * ti, J0p + MT * tj
                    if I >= Nu or J >= Nv:
                        continue
                    a1, b1, a2, b2 = row_reach(I, r0, r0 + nr, h)
                    o, nu = col_window(J, c0, c1, h, SS) if nr else (0, 0)
                    assert o % 4 == 0 and o + 16 * nu <= 16 * SS
                    if nu == 0:
                        b1, b2 = a1 - 1, a2 - 1
                    acc = np.zeros((16, 16))
                    cbase = J - h - C0 + o
                    assert cbase % 4 == 0
                    for p0, p1, plus, minus in segments(a1, b1, a2, b2, h):
                        for p in range(p0, p1 + 1):
                            for u in range(nu):
                                colv = cbase + 16 * u + cidx[None, :]
                                assert colv.min() >= 0 and colv.max() < cols
                                A = np.zeros((16, 16))
                                for side, on in ((1, plus), (-1, minus)):
                                    if on:
                                        r = I + m - R0 + side * p
                                        assert r.min() >= 0 and r.max() < rows
                                        A += img[r, colv]
                                bi = o + 16 * u + cidx[:, None] + 15 - cidx[None, :]
                                assert bi.min() >= 0 and bi.max() < E
                                acc += A @ kx[p, bi]
                    out = outs[item]
                    for mm in range(16):
                        for nn in range(16):
                            i, j = I + mm, J + nn
                            if I0 <= i < Nu and J0 <= j < Nv:
                                assert np.isnan(out[i, j]), "output written twice"
                                out[i, j] = acc[mm, nn]
    return outs


def _reference(inp, K, box):
    u0, u1, v0, v1 = box
    masked = np.zeros_like(inp)
    ru, rv = slice(max(u0, 0), max(u1, 0)), slice(max(v0, 0), max(v1, 0))
    masked[ru, rv] = inp[ru, rv]
    return ndimage.correlate(masked, K, mode="constant")


def _symmetric_kernel(rng, h):
    K = rng.normal(size=(2 * h + 1, 2 * h + 1))
    K = K + K[::-1, :] + K[:, ::-1] + K[::-1, ::-1]
    return K + K.T


def _check(Nu, Nv, h, boxes, seed):
    rng = np.random.default_rng(seed)
    inputs = [rng.normal(size=(Nu, Nv)) for _ in boxes]
    K = _symmetric_kernel(rng, h)
    for inp, box, got in zip(inputs, boxes, forward_in_box(inputs, K, boxes)):
        assert not np.isnan(got).any(), "output not written"
        ref = _reference(inp, K, box)
        assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


def test_standard_plane_and_full_opening():
    """89 x 89 planes with n = 61: the benchmark's jaw opening, a shifted and a
    wider one, the whole plane, and a one-row slit, in sequence on one image."""
    del PAIRS[:]
    _check(89, 89, 30, [(30, 59, 30, 59), (28, 61, 31, 58), (0, 89, 0, 89), (44, 45, 10, 80)], seed=1)
    # at the benchmark's opening the inner tile columns pair up: (1, 2) and (3, 4)
    assert sorted(tj for item, tj in PAIRS if item == 0) == [1, 3]


def test_random_planes_and_rectangles():
    rnd = random.Random(7)
    for t in range(12):
        h = rnd.choice([2, 3, 6, 7, 9, 12])
        Nu, Nv = rnd.randint(5, 130), rnd.randint(5, 130)
        boxes = []
        for _ in range(3):
            u0 = rnd.randint(-5, Nu)
            v0 = rnd.randint(-5, Nv)
            boxes.append((u0, rnd.randint(u0, Nu + 5), v0, rnd.randint(v0, Nv + 5)))
        _check(Nu, Nv, h, boxes, seed=100 + t)


def test_image_capacity_fits_two_workgroups_at_the_benchmark_size():
    """89 x 89 beam-frame planes, n = 61: image and taps of one workgroup fit
    twice in a CU's 160 KB of LDS."""
    h, N = 30, 89
    TI, _ = region_shape(N)
    SS = (16 + 2 * h + 15) // 16
    rows, cols = image_capacity(N, N, h, TI, TI, SS)
    assert (rows, pitch_f32(cols)) == (119, 136)
    E = 16 * SS + 16
    lds = 4 * (rows * pitch_f32(cols) + (h + 1) * E + (h + 1) ** 2) + 16 + 4 * 9 * RMAX * RMAX
    assert 2 * lds <= 160 * 1024
    # the region-placed image would not
    region = 4 * ((MT * TI + 2 * h) * pitch_f32(MT * TI + 16 * SS) + (h + 1) * E + (h + 1) ** 2) + 16
    assert 2 * region > 160 * 1024
