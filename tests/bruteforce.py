"""Pure-Python FP64 brute force of the dose model for tiny grids.

Written independently of oracle.c from the same definitions (arXiv:2512.18863,
§2.2): no scans, no batching, no stored volumes.  Every fan-grid value a voxel
needs is rebuilt from scratch: the water-equivalent path length of a node is a
direct sum over all samples up to that node (O(Nk^2) per ray), the beam-frame
dose of a node is a direct sum over the kernel taps.  Intended for grids of a
few hundred voxels.
"""
from __future__ import annotations

import math
from functools import lru_cache


def _sincos_deg(deg):
    r = math.fmod(deg, 360.0)
    if r < 0:
        r += 360.0
    exact = {0.0: (0.0, 1.0), 90.0: (1.0, 0.0), 180.0: (0.0, -1.0), 270.0: (-1.0, 0.0)}
    if r in exact:
        return exact[r]
    a = math.radians(r)
    return math.sin(a), math.cos(a)


def _frac(x, a, b, D):
    """Share of the pixel [x - D/2, x + D/2] lying inside [a, b]."""
    o = min(b, x + D / 2) - max(a, x - D / 2)
    return o / D if o > 0 else 0.0


class BruteForce:
    def __init__(self, case, rho):
        self.c = case
        self.m = case.machine
        self.rho = rho                                  # numpy [nz][ny][nx]
        self.nz, self.ny, self.nx = rho.shape
        self.h = (case.n_taps - 1) // 2
        D = case.lat_step
        self.D, self.Dd = D, case.depth_step
        self.Nu = 2 * math.ceil((case.field_limit[0] + self.h * D) / D - 1e-9) + 1
        self.Nv = 2 * math.ceil((case.field_limit[1] + self.h * D) / D - 1e-9) + 1
        sx, sy, _ = case.spacing
        ox, oy, _ = case.origin
        corners_x = (ox - sx / 2, ox + (self.nx - 0.5) * sx)
        corners_y = (oy - sy / 2, oy + (self.ny - 0.5) * sy)
        R = max(math.hypot(x - case.iso[0], y - case.iso[1]) for x in corners_x for y in corners_y)
        self.d0 = self.m.sad - R
        self.Nk = math.ceil(2 * R / self.Dd - 1e-9) + 1

    # -- density at a patient point, trilinear in voxel index space, zero outside
    def density(self, x, y, z):
        c = self.c
        fx = (x - c.origin[0]) / c.spacing[0]
        fy = (y - c.origin[1]) / c.spacing[1]
        fz = (z - c.origin[2]) / c.spacing[2]
        x0, y0, z0 = math.floor(fx), math.floor(fy), math.floor(fz)
        s = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    ix, iy, iz = x0 + dx, y0 + dy, z0 + dz
                    if 0 <= ix < self.nx and 0 <= iy < self.ny and 0 <= iz < self.nz:
                        w = ((fx - x0) if dx else (1 - (fx - x0))) * \
                            ((fy - y0) if dy else (1 - (fy - y0))) * \
                            ((fz - z0) if dz else (1 - (fz - z0)))
                        s += w * float(self.rho[iz, iy, ix])
        return s

    # -- a point on ray (u, v) at the plane a distance d from the source
    def ray_point(self, sn, cs, d, u, v):
        sad, p = self.m.sad, self.c.iso
        src = (p[0] + sad * sn, p[1] - sad * cs, p[2])
        bx, by = -sn, cs
        ux, uy = cs, sn
        return (src[0] + d * (bx + u * ux / sad),
                src[1] + d * (by + u * uy / sad),
                src[2] + d * (v / sad))

    def u_of(self, i):
        return (i - (self.Nu - 1) / 2) * self.D

    def v_of(self, j):
        return (j - (self.Nv - 1) / 2) * self.D

    def depth_dose(self, W):
        dd, st = self.m.dd, self.m.dd_step
        x = W / st
        if x <= 0:
            return float(dd[0])
        if x >= len(dd) - 1:
            return float(dd[-1])
        i = math.floor(x)
        f = x - i
        return float(dd[i]) * (1 - f) + float(dd[i + 1]) * f

    def fluence(self, b, j, i):
        c, m = self.c, self.m
        L, D = m.n_leaf, self.D
        edges = m.leaf_edges
        lv, jw = c.leaves[b], c.jaws[b]
        u, v = self.u_of(i), self.v_of(j)
        jaw = _frac(u, jw[0], jw[1], D) * _frac(v, jw[2], jw[3], D)
        cover = 0.0
        opening = 0.0
        for l in range(L):
            w = _frac(v, edges[l], edges[l + 1], D)
            cover += w
            opening += w * _frac(u, lv[0][l], lv[1][l], D)
        return jaw * (m.tau * cover + (1 - m.tau) * opening)

    def plane_d(self, k):
        return self.d0 + k * self.Dd

    def wepl_node(self, b, k, j, i):
        sn, cs = _sincos_deg(float(self.c.gantry[b]))
        if self.c.wepl_mode == 1:      # central axis
            return sum(self.density(*self.ray_point(sn, cs, self.plane_d(kk), 0.0, 0.0)) * self.Dd
                       for kk in range(k + 1))
        u, v = self.u_of(i), self.v_of(j)
        step = self.Dd * math.sqrt(1 + (u * u + v * v) / self.m.sad ** 2)
        return sum(self.density(*self.ray_point(sn, cs, self.plane_d(kk), u, v)) * step
                   for kk in range(k + 1))

    def central_depth(self, b, k):
        sn, cs = _sincos_deg(float(self.c.gantry[b]))
        return sum(self.density(*self.ray_point(sn, cs, self.plane_d(kk), 0.0, 0.0)) * self.Dd
                   for kk in range(k + 1))

    def primary(self, b, k, j, i):
        if not (0 <= j < self.Nv and 0 <= i < self.Nu):
            return 0.0
        F = self.fluence(b, j, i)
        if F == 0.0:
            return 0.0
        d = self.plane_d(k)
        return F * (self.m.sad / d) ** 2 * self.depth_dose(self.wepl_node(b, k, j, i))

    def tap(self, b, k, p, q):
        m = self.m
        z = min(max(self.central_depth(b, k), 0.0), m.kz_max)

        def poly(c):
            return c[0] + c[1] * z + c[2] * z * z + c[3] * z ** 3
        A, a, B, bb = (poly(m.kpoly[r]) for r in range(4))
        norm = A / a + B / bb
        delta = self.D * self.plane_d(k) / m.sad
        if p == 0 and q == 0:
            r0 = delta / math.sqrt(math.pi)
            return (A / a * (1 - math.exp(-a * r0)) + B / bb * (1 - math.exp(-bb * r0))) / norm
        r = delta * math.sqrt(p * p + q * q)
        return delta ** 2 * (A * math.exp(-a * r) + B * math.exp(-bb * r)) / (2 * math.pi * r * norm)

    def beam_dose_node(self, b, k, j, i):
        h = self.h
        return sum(self.tap(b, k, p, q) * self.primary(b, k, j + p, i + q)
                   for p in range(-h, h + 1) for q in range(-h, h + 1))

    def voxel_dose_cp(self, b, iz, iy, ix):
        c, m = self.c, self.m
        sn, cs = _sincos_deg(float(c.gantry[b]))
        tx = c.origin[0] + ix * c.spacing[0] - c.iso[0]
        ty = c.origin[1] + iy * c.spacing[1] - c.iso[1]
        tz = c.origin[2] + iz * c.spacing[2] - c.iso[2]
        d = -sn * tx + cs * ty + m.sad
        u = m.sad * (cs * tx + sn * ty) / d
        v = m.sad * tz / d
        kc = (d - self.d0) / self.Dd
        jc = v / self.D + (self.Nv - 1) / 2
        ic = u / self.D + (self.Nu - 1) / 2
        k0, j0, i0 = math.floor(kc), math.floor(jc), math.floor(ic)
        s = 0.0
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    k, j, i = k0 + dk, j0 + dj, i0 + di
                    if 0 <= k < self.Nk and 0 <= j < self.Nv and 0 <= i < self.Nu:
                        w = ((kc - k0) if dk else (1 - (kc - k0))) * \
                            ((jc - j0) if dj else (1 - (jc - j0))) * \
                            ((ic - i0) if di else (1 - (ic - i0)))
                        if w != 0.0:
                            s += w * self._node(b, k, j, i)
        return s

    @lru_cache(maxsize=None)
    def _node(self, b, k, j, i):
        return self.beam_dose_node(b, k, j, i)

    def dose(self):
        import numpy as np
        out = np.zeros((self.nz, self.ny, self.nx))
        for iz in range(self.nz):
            for iy in range(self.ny):
                for ix in range(self.nx):
                    out[iz, iy, ix] = self.m.calib * sum(
                        float(self.c.mu[b]) * self.voxel_dose_cp(b, iz, iy, ix) for b in range(self.c.n_cp))
        return out
