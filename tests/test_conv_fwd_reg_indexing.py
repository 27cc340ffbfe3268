"""CPU model of the register-resident forward convolution's indexing
(paper_2512_18863_amd/csrc/conv_fwd_reg.hip), FP32 and BF16 layouts: box chunks, the column groups in
reach of each output strip, the tap-row addresses (in range for every group, run
or not), the matrix instructions' lane layout and the DPP row
shifts that move each product p rows up and down, emulated lane by lane in FP64
and compared with the direct convolution of the masked input
(§2.2.6, Eq. 8: out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q]).  The DPP shifts are
modelled as row_shl:S (lane i takes lane i + S of its 16-lane row) and row_shr:S
(lane i takes lane i - S), zero where the source lies outside the row; the GPU
parity tests check the hardware against the oracle."""
import numpy as np
import pytest

QB = 2          # output blocks above and below a row chunk
NW_LANES = 64


def mfma(a_lane, b_lane):
    """D = A B for v_mfma_f32_16x16x4_f32 (KP = 1) and v_mfma_f32_16x16x32_bf16
    (KP = 8): lane l gives A[l & 15][KP (l >> 4) + e] and B[KP (l >> 4) + e][l & 15]
    for e < KP; lane l holds D[4 (l >> 4) + e][l & 15], e = 0..3."""
    KP = a_lane.shape[1]
    A = np.zeros((16, 4 * KP))
    B = np.zeros((4 * KP, 16))
    for l in range(64):
        A[l & 15, KP * (l >> 4):KP * (l >> 4) + KP] = a_lane[l]
        B[KP * (l >> 4):KP * (l >> 4) + KP, l & 15] = b_lane[l]
    D = A @ B
    out = np.zeros((64, 4))
    for l in range(64):
        for e in range(4):
            out[l, e] = D[4 * (l >> 4) + e, l & 15]
    return out


def row_shl(v, s):
    out = np.zeros_like(v)
    for l in range(64):
        if (l & 15) + s < 16:
            out[l] = v[l + s]
    return out


def row_shr(v, s):
    out = np.zeros_like(v)
    for l in range(64):
        if (l & 15) - s >= 0:
            out[l] = v[l - s]
    return out


def model(inp, box, h, kq, T, SU, bf):
    """The kernel's FP32 (bf False: groups of 16 columns, four K = 4 products) or
    BF16 (groups of 32 columns, one K = 32 product, eight taps per lane read from
    the row copy of the start's parity) indexing, with FP64 arithmetic."""
    Nu, Nv = inp.shape
    GW = 32 if bf else 16
    E, off = (2 * h + 96, h + 47) if bf else (2 * h + 62, h + 31)
    KP, MPG = (8, 1) if bf else (1, 4)      # K elements per lane and products per group
    kx = np.zeros((h + 1, E + 1))           # (entry E is the zero the second BF16 copy ends with)
    for p in range(h + 1):
        for x in range(E + 1):
            q = abs(x - off)
            kx[p, x] = kq[p, q] if q <= h else 0.0
    r0, r1, c0, c1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    plane = np.zeros((Nu, Nv))
    if r1 <= r0 or c1 <= c0:
        return plane
    NB = T + 2 * QB
    lanes = np.arange(64)
    n, kk = lanes & 15, lanes >> 4
    cw0, cw1 = max(0, c0 - h), min(Nv, c1 + h)
    njt = (cw1 - cw0 + 15) // 16
    nrc = (r1 - r0 + 16 * T - 1) // (16 * T)
    ncc = (c1 - c0 + GW * SU - 1) // (GW * SU)
    wpitch = 16 * ((Nv + 15) // 16) + 4
    win = np.zeros((Nu, wpitch))
    ev = np.arange(KP)
    for jt in range(njt):
        J = cw0 + 16 * jt
        assert J - cw0 + 16 <= wpitch
        for rc in range(nrc):
            R = r0 + 16 * T * rc
            O = np.zeros((NB, 64, 4))
            for cc in range(ncc):
                C = c0 + GW * SU * cc
                # B of group u, product s: lane (n, kk) column C + GW u + 4 kk + s (FP32)
                # or C + 32 u + 8 kk + e (BF16)
                B = np.zeros((T, SU, MPG, 64, KP))
                for t in range(T):
                    for u in range(SU):
                        for sm in range(MPG):
                            r = R + 16 * t + n
                            cols = (C + GW * u + 4 * kk + sm)[:, None] if not bf else \
                                (C + GW * u + 8 * kk)[:, None] + ev[None, :]
                            ok = (r[:, None] < r1) & (cols < c1)
                            rr = np.broadcast_to(r[:, None], cols.shape)
                            B[t, u, sm][ok] = inp[rr[ok], cols[ok]]
                nsu = min(SU, (c1 - C + GW - 1) // GW)
                lo, hi = J - h - C - (GW - 1), J + 15 + h - C
                ua = 0 if lo <= 0 else (lo + GW - 1) // GW
                ub = min(nsu - 1, hi // GW if hi >= 0 else -1)
                if ua > ub:
                    continue
                for p in range(h + 1):
                    S, Q = p & 15, p >> 4
                    A = np.zeros((SU, MPG, 64, KP))
                    for u in range(SU):
                        KL = 8 if bf else 4
                        base = C + GW * u + KL * kk - J - n + off if ua <= u <= ub else 15 + KL * kk - n
                        for sm in range(MPG):
                            x = (base + sm)[:, None] + ev[None, :]
                            assert x.min() >= 0 and x.max() < (E + 1 if bf else E), (x.min(), x.max(), E)
                            if bf:   # words (x >> 1) .. (x >> 1) + 3 of a copy of E / 2 words
                                assert ((base >> 1) + 3).max() < E // 2
                            A[u, sm] = kx[p, x]
                    for t in range(T):
                        y = np.zeros((64, 4))
                        # group 0 always (zero A when out of reach), the others when in reach
                        for u in sorted(set([0] + list(range(max(1, ua), ub + 1)))):
                            for sm in range(MPG):
                                y += mfma(A[u, sm], B[t, u, sm])
                        c = QB
                        if p == 0:
                            O[c + t] += y
                        elif S == 0:
                            O[c + t - Q] += y
                            O[c + t + Q] += y
                        else:
                            O[c + t - Q] += row_shl(y, S)
                            O[c + t - Q - 1] += row_shr(y, 16 - S)
                            O[c + t + Q] += row_shr(y, S)
                            O[c + t + Q + 1] += row_shl(y, 16 - S)
            for q in range(NB):
                row = R - 16 * QB + 16 * q + n
                for l in range(64):
                    if 0 <= row[l] < Nu:
                        col = J - cw0 + 4 * kk[l]
                        win[row[l], col:col + 4] += O[q, l]
    for j in range(cw0, min(Nv, cw0 + 16 * njt)):
        plane[:, j] = win[:, j - cw0]
    return plane


def direct(inp, box, h, kq):
    Nu, Nv = inp.shape
    m = np.zeros_like(inp)
    r0, r1, c0, c1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    m[r0:r1, c0:c1] = inp[r0:r1, c0:c1]
    out = np.zeros_like(inp)
    pad = np.zeros((Nu + 2 * h, Nv + 2 * h))
    pad[h:h + Nu, h:h + Nv] = m
    for p in range(-h, h + 1):
        for q in range(-h, h + 1):
            out += kq[abs(p), abs(q)] * pad[h + p:h + p + Nu, h + q:h + q + Nv]
    return out


CASES = [
    (89, 89, 30, (30, 59, 31, 58), 2, 2),      # the benchmark plane: 61 taps, a 29 x 27 rectangle
    (89, 89, 30, (0, 89, 0, 89), 2, 2),        # the whole plane: several chunks each way
    (40, 37, 6, (3, 38, 0, 21), 1, 1),         # small kernel, rectangle at the left edge, several chunks
    (50, 47, 16, (20, 21, 46, 47), 2, 2),      # one pixel in the last column, tap rows 16 = 16 + 0
    (45, 60, 17, (10, 40, 5, 55), 3, 3),       # one chunk each way with T = SU = 3 (FP32)
    (70, 66, 31, (25, 46, 20, 41), 1, 2),      # the largest half-width, 2 x 1 chunks
    (30, 30, 8, (12, 12, 3, 20), 2, 2),        # empty rectangle
]


@pytest.mark.parametrize("bf", [False, True], ids=["fp32", "bf16"])
@pytest.mark.parametrize("Nu,Nv,h,box,T,SU", CASES)
def test_register_forward_matches_direct_convolution(Nu, Nv, h, box, T, SU, bf):
    rng = np.random.default_rng(Nu * 7 + h)
    inp = rng.normal(size=(Nu, Nv))
    kq = rng.uniform(0.1, 1.0, size=(h + 1, h + 1))   # any table with K[p][q] = kq[|p|][|q|]
    got = model(inp, box, h, kq, T, SU if not bf else (SU + 1) // 2, bf)
    ref = direct(inp, box, h, kq)
    assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("h", [1, 2, 5, 16, 30, 31])
def test_bf16_tap_rows_written_once_inside_the_rows(h):
    """The BF16 forward's tap rows (two copies; copy c holds element x of row p at
    half-word x - c): each tap K[p][q] (pair p <= q) is written at elements off +- q
    of row p and off +- p of row q, whole words made only of elements farther than
    h from off are cleared, and the two elements beside the taps one by one.  Every
    half-word of every row must end up written, with the tap or zero, and no write
    may leave its row."""
    E, off = 2 * h + 96, h + 47
    W2 = E // 2
    rows = [[[None] * (2 * W2) for _ in range(h + 1)] for _ in range(2)]
    kq = {(p, q): 1.0 + p * 100 + q for p in range(h + 1) for q in range(h + 1)}

    def put(c, p, hw, v):
        assert 0 <= hw < 2 * W2
        old = rows[c][p][hw]
        assert old is None or old == v          # only equal values may meet
        rows[c][p][hw] = v

    for q in range(h + 1):
        for p in range(q + 1):
            v = kq[(p, q)]
            for c in range(2):
                put(c, p, off + q - c, v)
                put(c, p, off - q - c, v)
                put(c, q, off + p - c, v)
                put(c, q, off - p - c, v)
    xa, xb = off - h, off + h
    nl = [xa // 2, (xa - 1) // 2]
    ir = [xb // 2 + 1, (xb - 1) // 2 + 1]
    for p in range(h + 1):
        for c in range(2):
            for i in list(range(nl[c])) + list(range(ir[c], W2)):
                put(c, p, 2 * i, 0.0)
                put(c, p, 2 * i + 1, 0.0)
            for x in (xa - 1, xb + 1):
                if 0 <= x - c < 2 * W2:
                    put(c, p, x - c, 0.0)
    for c in range(2):
        for p in range(h + 1):
            for hw in range(2 * W2):
                x = hw + c
                want = kq[(min(p, abs(x - off)), max(p, abs(x - off)))] if abs(x - off) <= h else 0.0
                assert rows[c][p][hw] == want, (c, p, hw)
