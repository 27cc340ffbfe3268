"""CPU model of the windowed BF16 adjoint convolution's indexing
(paper_2512_18863_amd/csrc/conv_bf16.hip, k_conv_bf16_adj_win): pieces of at
most 2 x 2 output tiles at the rectangle's corner, each piece's BF16 image (plane
rows [I - h, I + 16 nI + h), the 32 NK columns from J - h, zero outside the
plane), the two padded copies of each tap row and the per-lane B runs of eight
taps read as four aligned words, the A fragments of eight image elements, and
the v_mfma_f32_16x16x32_bf16 lane layout, in FP64 on BF16-rounded operands,
compared with the direct convolution (§2.2.6, Eq. 8:
out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q]) of the rounded input and taps.  Every
tap-row word and image element read must lie inside its array."""
import numpy as np
import pytest

X0B = 32  # element x of a padded row holds the tap at |x - (h + X0B)|


def bf16(x):
    """Round float32 values to BF16 (nearest even), returned as float64."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def model(inp, box, h, kq):
    Nu, Nv = inp.shape
    NK = (32 + 2 * h + 31) // 32
    L2 = 16 * NK + 16
    # padded rows: element x -> K[p][|x - (h + X0B)|]
    T = np.zeros((h + 1, 2 * L2 + 2))
    for p in range(h + 1):
        for x in range(2 * L2 + 2):
            d = abs(x - (h + X0B))
            T[p, x] = bf16(kq[p, d]) if d <= h else 0.0
    out = np.full((Nu, Nv), np.nan)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    if not (u1 > u0 and v1 > v0):
        return out
    nI, nJ = (u1 - u0 + 15) // 16, (v1 - v0 + 15) // 16
    npi, npj = (nI + 1) // 2, (nJ + 1) // 2
    lanes = np.arange(64)
    m, kq_ = lanes & 15, lanes >> 4
    e8 = np.arange(8)
    for pp in range(npi * npj):
        pi, pj = pp // npj, pp % npj
        nIp, nJp = min(2, nI - 2 * pi), min(2, nJ - 2 * pj)
        r0, c0 = u0 + 32 * pi - h, v0 + 32 * pj - h
        nr, nc = 16 * nIp + 2 * h, 32 * NK
        rows, pitch = 32 + 2 * h, 32 * NK + 16
        assert nr <= rows and nc <= pitch - 16
        img = np.full((rows, pitch), np.nan)
        for r in range(nr):
            for c in range(nc):
                pr, pc = r0 + r, c0 + c
                img[r, c] = bf16(inp[pr, pc]) if 0 <= pr < Nu and 0 <= pc < Nv else 0.0
        acc = np.zeros((2, 2, 64, 4))
        for p in range(-h, h + 1):
            ap = abs(p)
            for s in range(NK):
                # B runs: lane (m, kq) of column tile t reads words x // 2 .. + 3 of the
                # copy of parity x & 1, i.e. elements x .. x + 7 of the padded row
                B = np.zeros((2, 64, 8))
                for t in range(nJp):
                    x = 32 * s + 8 * kq_ - 16 * t - m + X0B
                    assert x.min() >= 1 and (x // 2 + 3).max() < L2
                    B[t] = T[ap][x[:, None] + e8[None, :]]
                A = np.zeros((2, 64, 8))
                for r in range(nIp):
                    row = 16 * r + m + p + h
                    col = 32 * s + 8 * kq_
                    assert row.min() >= 0 and row.max() < nr and (col + 7).max() < nc
                    A[r] = img[row[:, None], col[:, None] + e8[None, :]]
                for r in range(nIp):
                    for t in range(nJp):
                        Am = np.zeros((16, 32))
                        Bm = np.zeros((32, 16))
                        for l in range(64):
                            Am[l & 15, 8 * (l >> 4):8 * (l >> 4) + 8] = A[r, l]
                            Bm[8 * (l >> 4):8 * (l >> 4) + 8, l & 15] = B[t, l]
                        D = Am @ Bm
                        for l in range(64):
                            acc[r, t, l] += D[4 * (l >> 4) + np.arange(4), l & 15]
        Ip, Jp = r0 + h, c0 + h
        for r in range(nIp):
            for t in range(nJp):
                for l in range(64):
                    j = Jp + 16 * t + (l & 15)
                    for e in range(4):
                        i = Ip + 16 * r + 4 * (l >> 4) + e
                        if i < Nu and j < Nv:
                            out[i, j] = acc[r, t, l, e]
    return out


def direct(inp, h, kq):
    Nu, Nv = inp.shape
    x = bf16(inp)
    out = np.zeros((Nu, Nv))
    pad = np.zeros((Nu + 2 * h, Nv + 2 * h))
    pad[h:h + Nu, h:h + Nv] = x
    for p in range(-h, h + 1):
        for q in range(-h, h + 1):
            out += bf16(kq[abs(p), abs(q)]) * pad[h + p:h + p + Nu, h + q:h + q + Nv]
    return out


CASES = [
    (89, 89, 30, (30, 59, 31, 58)),        # the benchmark plane: 61 taps, a 29 x 27 rectangle
    (40, 37, 6, (3, 38, 0, 21)),           # small kernel, several pieces each way
    (50, 47, 16, (20, 21, 46, 47)),        # one pixel in the last column
    (70, 66, 31, (25, 46, 20, 41)),        # four K-steps
    (30, 30, 8, (12, 12, 3, 20)),          # empty rectangle
]


@pytest.mark.parametrize("Nu,Nv,h,box", CASES)
def test_windowed_bf16_adjoint_matches_direct_convolution(Nu, Nv, h, box):
    rng = np.random.default_rng(Nu * 5 + h)
    inp = rng.normal(size=(Nu, Nv)).astype(np.float32)
    kq = rng.uniform(0.1, 1.0, size=(h + 1, h + 1)).astype(np.float32)
    got = model(inp, box, h, kq)
    ref = direct(inp, h, kq)
    written = ~np.isnan(got)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    if u1 > u0 and v1 > v0:
        assert written[u0:u1, v0:v1].all()
    else:
        assert not written.any()
    assert np.abs(got[written] - ref[written]).max(initial=0.0) <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("h", [1, 7, 15, 30, 47])
def test_tap_rows_rewritten_whole_for_every_plane(h):
    """The windowed BF16 adjoint's tap rows (taps_to_bf16_rows): both copies are
    cleared once per workgroup, then every plane writes tap K[p][q] (pair p <= q)
    at elements X0 + h +- q of row p and X0 + h +- p of row q, copy c at half-word
    x - c of a row of 2 L2 half-words (L2 = 16 NK + 17).  After any sequence of
    planes, every element within h of X0 + h holds the current plane's tap and
    every other element zero; each write stays inside its row; and every B run a
    lane reads (eight elements from x in [1, 32 NK + 24]) lies inside the row."""
    NK = (32 + 2 * h + 31) // 32
    L2 = 16 * NK + 17
    x0 = h + 32
    rows = [[[0] * (2 * L2) for _ in range(h + 1)] for _ in range(2)]    # cleared once

    for plane in range(3):
        def K(p, q):
            return 1 + plane * 10000 + p * 100 + q
        for q in range(h + 1):
            for p in range(q + 1):
                for c in range(2):
                    for r, d in ((p, q), (p, -q), (q, p), (q, -p)):
                        hw = x0 + d - c
                        assert 0 <= hw < 2 * L2
                        rows[c][r][hw] = K(p, q)
        for c in range(2):
            for r in range(h + 1):
                for hw in range(2 * L2):
                    d = abs(hw + c - x0)
                    want = K(min(r, d), max(r, d)) if d <= h else 0
                    assert rows[c][r][hw] == want, (plane, c, r, hw)
    # B runs: start x = 32 s + 8 kq - 16 t - m + 32 (s < NK, kq < 4, t < 2, m < 16),
    # read from the copy of x's parity as four words from word x >> 1
    for s in range(NK):
        for kq in range(4):
            for t in range(2):
                for m in range(16):
                    x = 32 * s + 8 * kq - 16 * t - m + 32
                    assert 1 <= x <= 32 * NK + 24
                    assert (x >> 1) + 3 < L2
