"""CPU model of the windowed FP32 adjoint convolution's indexing
(paper_2512_18863_amd/csrc/conv_mfma.hip, k_conv_f32_adj_win): the covered tiles
at the box corner, their pieces, each piece's image window (zero outside the
plane), the folded tap rows and the Toeplitz operand read from the extended tap
row, in FP64, compared with the direct convolution (§2.2.6, Eq. 8:
out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q], K[p][q] = kq[|p|][|q|]) at every
output the model writes; the written outputs must cover the box inside the plane
and every image read must lie inside the window and the allocated image."""
import numpy as np
import pytest

MT = 16


def pitch_f32(cols):
    return ((cols + 7) // 16) * 16 + 8


def shape(Nu, Nv, h, nw=8, lds_max=160 * 1024):
    """The launcher's piece size and image shape (f32_adj_win_shape)."""
    half_u, half_v = (Nu - 1) // 2 - h, (Nv - 1) // 2 - h
    bu, bv = 2 * max(half_u, 0) + 4, 2 * max(half_v, 0) + 4
    WI = min(max((bu + MT - 1) // MT, 1), 4)
    WJ = min(max((bv + MT - 1) // MT, 1), 4)
    SS = (MT + 2 * h + 15) // 16
    E = 16 * SS + 16
    while True:
        rows = MT * WI + 2 * h
        pitch = pitch_f32(MT * (WJ - 1) + 16 * SS)
        lds = 4 * (rows * pitch + (h + 1) * E) + 16 + 4 * 256 * (nw - 1)
        if lds <= lds_max:
            return dict(WI=WI, WJ=WJ, SS=SS, E=E, rows=rows, pitch=pitch)
        if WI == 1 and WJ == 1:
            return None
        if WJ >= WI:
            WJ -= 1
        else:
            WI -= 1


def model(inp, box, h, kq, aw):
    Nu, Nv = inp.shape
    WI, WJ, SS, E = aw["WI"], aw["WJ"], aw["SS"], aw["E"]
    off = h + 15
    kx = np.zeros((h + 1, E))
    for p in range(h + 1):
        for c in range(E):
            q = c - off
            if -h <= q <= h:
                kx[p, c] = kq[p, abs(q)] * (0.5 if p == 0 else 1.0)
    out = np.full((Nu, Nv), np.nan)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    if not (u1 > u0 and v1 > v0):
        return out
    Jw = v0
    nI, nJ = (u1 - u0 + MT - 1) // MT, (v1 - Jw + MT - 1) // MT
    npi, npj = (nI + WI - 1) // WI, (nJ + WJ - 1) // WJ
    n = np.arange(16)
    x = np.arange(16 * SS)
    for pp in range(npi * npj):
        pi, pj = pp // npj, pp % npj
        nIp, nJp = min(WI, nI - WI * pi), min(WJ, nJ - WJ * pj)
        r0, c0 = u0 + MT * WI * pi - h, Jw + MT * WJ * pj - h
        nr, nc = MT * nIp + 2 * h, MT * (nJp - 1) + 16 * SS
        assert nr <= aw["rows"] and nc <= aw["pitch"]
        assert nc % 4 == 0                           # whole four-column groups
        img = np.full((aw["rows"], aw["pitch"]), np.nan)   # unstaged entries poison the sums
        for r in range(nr):
            for c in range(nc):
                pr, pc = r0 + r, c0 + c
                img[r, c] = inp[pr, pc] if 0 <= pr < Nu and 0 <= pc < Nv else 0.0
        for t in range(nIp * nJp):
            ti, tj = t // nJp, t % nJp
            oI, oJ = r0 + h + MT * ti, c0 + h + MT * tj
            acc = np.zeros((16, 16))
            for p in range(h + 1):
                rows_p = MT * ti + n + h + p
                rows_m = MT * ti + n + h - p
                assert rows_m.min() >= 0 and rows_p.max() < nr
                cols = MT * tj + x
                assert cols.max() < nc
                a = img[np.ix_(rows_p, cols)] + img[np.ix_(rows_m, cols)]   # A[m][x]
                bidx = x[:, None] + 15 - n[None, :]
                assert bidx.min() >= 0 and bidx.max() < E
                acc += a @ kx[p][bidx]                                      # B[x][n]
            for m in range(16):
                i = oI + m
                for nn in range(16):
                    j = oJ + nn
                    if 0 <= i < Nu and 0 <= j < Nv:
                        out[i, j] = acc[m, nn]
    return out


def direct(inp, h, kq):
    Nu, Nv = inp.shape
    out = np.zeros_like(inp)
    pad = np.zeros((Nu + 2 * h, Nv + 2 * h))
    pad[h:h + Nu, h:h + Nv] = inp
    for p in range(-h, h + 1):
        for q in range(-h, h + 1):
            out += kq[abs(p), abs(q)] * pad[h + p:h + p + Nu, h + q:h + q + Nv]
    return out


CASES = [
    (89, 89, 30, (30, 59, 31, 58)),        # the benchmark plane: 61 taps, a 29 x 27 rectangle
    (89, 89, 30, (0, 89, 0, 89)),          # the whole plane: several pieces each way
    (40, 37, 6, (3, 38, -5, 21)),          # small kernel, rectangle over the left edge
    (50, 47, 16, (20, 21, 46, 47)),        # one pixel in the last column
    (129, 129, 12, (7, 120, 9, 128)),      # a wide plane: 4 x 4 tiles a piece, 8 x 8 tiles
    (70, 66, 31, (25, 46, 20, 41)),        # the largest half-width of the register forward
    (200, 200, 60, (40, 160, 50, 150)),    # a kernel wide enough that the pieces shrink
    (30, 30, 8, (12, 12, 3, 20)),          # empty rectangle
    (61, 58, 9, (2, 30, 1, 57)),           # groups straddling both plane edges
]


@pytest.mark.parametrize("Nu,Nv,h,box", CASES)
def test_windowed_adjoint_matches_direct_convolution(Nu, Nv, h, box):
    rng = np.random.default_rng(Nu * 13 + h)
    inp = rng.normal(size=(Nu, Nv))
    kq = rng.uniform(0.1, 1.0, size=(h + 1, h + 1))
    aw = shape(Nu, Nv, h)
    assert aw is not None
    got = model(inp, box, h, kq, aw)
    ref = direct(inp, h, kq)
    written = ~np.isnan(got)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    if u1 > u0 and v1 > v0:
        assert written[u0:u1, v0:v1].all()
    else:
        assert not written.any()
    assert np.abs(got[written] - ref[written]).max(initial=0.0) <= 1e-10 * max(1.0, np.abs(ref).max())


def test_benchmark_shape_fits_two_workgroups_per_cu():
    aw = shape(89, 89, 30)
    assert (aw["WI"], aw["WJ"]) == (2, 2)
    lds = 4 * (aw["rows"] * aw["pitch"] + 31 * aw["E"]) + 16 + 4 * 256 * 7
    assert 2 * lds <= 160 * 1024


def stage(flat, it, n_items, Nu, Nv, w, nt=512, pitch=None):
    """The window staging of one piece (win_stage, load_group, mask_group,
    put_win): thread tid keeps column group tid % gw and walks rows tid // gw,
    + step, ...; the four-word load of a group reads flat[pr Nv + pc + e] (pc may
    lie outside [0, Nv - 4]), the batch's first and last planes load word by word.
    Returns the image and the set of flat indices read."""
    r0w, c0w, nr, nc = w
    gw = nc // 4
    step = nt // gw
    img = np.full((nr, nc), np.nan)
    reads = set()
    base = it * Nu * Nv
    edge = it == 0 or it == n_items - 1
    for tid in range(nt):
        r0, cg = divmod(tid, gw)
        if r0 >= step:
            continue
        pc = c0w + 4 * cg
        cmask = [0 <= pc + e < Nv for e in range(4)]
        for r in range(r0, nr, step):
            pr = r0w + r
            rok = 0 <= pr < Nu and any(cmask)
            off = base + (pr * Nv + pc if rok else 0)
            v = np.zeros(4)
            for e in range(4):
                if edge and not (rok and cmask[e]):
                    continue
                reads.add(off + e)
                v[e] = flat[off + e]
            for e in range(4):
                if not (rok and cmask[e]):
                    v[e] = 0.0
            assert np.isnan(img[r, 4 * cg:4 * cg + 4]).all()     # each group written once
            img[r, 4 * cg:4 * cg + 4] = v
    return img, reads


@pytest.mark.parametrize("Nu,Nv,h,box", [c for c in CASES if c[3][1] > c[3][0] and c[3][3] > c[3][2]])
def test_window_staging_reads_inside_the_batch(Nu, Nv, h, box):
    rng = np.random.default_rng(Nu + 3 * Nv + h)
    n_items = 3
    flat = rng.normal(size=n_items * Nu * Nv)
    aw = shape(Nu, Nv, h)
    u0, u1, v0, v1 = max(box[0], 0), min(box[1], Nu), max(box[2], 0), min(box[3], Nv)
    nI, nJ = (u1 - u0 + MT - 1) // MT, (v1 - v0 + MT - 1) // MT
    nIp, nJp = min(aw["WI"], nI), min(aw["WJ"], nJ)
    w = (u0 - h, v0 - h, MT * nIp + 2 * h, MT * (nJp - 1) + 16 * aw["SS"])
    for it in range(n_items):
        img, reads = stage(flat, it, n_items, Nu, Nv, w)
        plane = flat[it * Nu * Nv:(it + 1) * Nu * Nv].reshape(Nu, Nv)
        want = np.zeros((w[2], w[3]))
        for r in range(w[2]):
            for c in range(w[3]):
                pr, pc = w[0] + r, w[1] + c
                if 0 <= pr < Nu and 0 <= pc < Nv:
                    want[r, c] = plane[pr, pc]
        assert not np.isnan(img).any()
        assert np.array_equal(img, want)
        assert min(reads) >= 0 and max(reads) < flat.size
