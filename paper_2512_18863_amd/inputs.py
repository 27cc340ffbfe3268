"""Seeded synthetic inputs: machine tables, phantoms and VMAT plans.

This module only *describes* workloads.  It holds none of the dose model's
arithmetic, so both the HIP engine and the FP64 oracle can consume the same
inputs without sharing any computation.

The paper's measurements use clinical prostate cohorts and commissioned beam
data that are not available here (§2.4-2.5); the workloads below stand in for
them with the same structure: a pelvis-like CT (water body, two femurs, a gas
pocket), a prostate-sized target with rectum and bladder, and VMAT arcs of
control points spaced 2-4 degrees apart.

Conventions: lengths in mm, angles in degrees, arrays row-major with x
fastest ([nz][ny][nx]); the isocentre sits at the grid centre, voxel centres at
(i - (N-1)/2) * spacing.  Seeds follow 1000 * config + purpose.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

WEPL_PER_RAY = 0
WEPL_CENTRAL_AXIS = 1


# --------------------------------------------------------------------------- machine


@dataclass
class Machine:
    """A synthetic 10 MV-like machine description (the commissioned data of §2.4 are
    not available, so every table here is synthetic)."""

    sad: float = 1000.0
    n_leaf: int = 60
    leaf_width: float = 5.0
    tau: float = 0.002                    # MLC transmission (§2.2.2)
    calib: float = 1.0                    # dose per MU
    # HU -> relative density calibration points
    hu_pts: np.ndarray = field(default_factory=lambda: np.array([-1000.0, 0.0, 1500.0]))
    rho_pts: np.ndarray = field(default_factory=lambda: np.array([0.0, 1.0, 1.85]))
    # depth-dose table over water-equivalent depth
    dd_step: float = 1.0
    dd: np.ndarray = field(default_factory=lambda: synthetic_depth_dose())
    # kernel parameters A, a, B, b as cubic polynomials in depth z (mm); rows c0..c3
    kpoly: np.ndarray = field(default_factory=lambda: np.array([
        [1.0, 0.0, 0.0, 0.0],
        [0.50, -3e-4, 0.0, 0.0],
        [0.008, 2e-5, 0.0, 0.0],
        [0.030, -1e-5, 0.0, 0.0],
    ]))
    kz_max: float = 700.0
    # fluence corrections (§2.2.2 list), off unless fcorr
    fcorr: bool = False
    pen_fwhm_u: float = 0.0               # source penumbra FWHM along the leaf travel, mm
    pen_fwhm_v: float = 0.0               # ... across the leaves, mm
    hs_amp: float = 0.0                   # head-scatter amplitude
    hs_sigma: float = 0.0                 # head-scatter Gaussian sigma, mm
    oar: tuple = (0.0, 0.0)               # off-axis factor 1 + oar0 r + oar1 r^2 (r in mm)

    @property
    def leaf_edges(self) -> np.ndarray:
        L, w = self.n_leaf, self.leaf_width
        return (np.arange(L + 1, dtype=np.float64) - L / 2.0) * w


def with_fluence_corrections(m: "Machine") -> "Machine":
    """The synthetic machine with its fluence corrections switched on: penumbra FWHM
    3.5 mm (leaf travel) and 4.5 mm (across), 4 % head scatter with sigma 20 mm, and
    an off-axis rise of +4 % at 100 mm."""
    import dataclasses
    return dataclasses.replace(m, fcorr=True, pen_fwhm_u=3.5, pen_fwhm_v=4.5, hs_amp=0.04, hs_sigma=20.0,
                               oar=(0.0, 4e-6))


def synthetic_depth_dose(max_depth: float = 800.0, step: float = 1.0) -> np.ndarray:
    """A TPR-like depth-dose table: build-up to a maximum near 23 mm, then
    exponential fall-off; normalised to a maximum of one."""
    w = np.arange(0.0, max_depth + 0.5 * step, step)
    dd = (1.0 - 0.65 * np.exp(-w / 8.0)) * np.exp(-0.0045 * w)
    return dd / dd.max()


# --------------------------------------------------------------------------- case


@dataclass
class Case:
    """One dose-calculation problem: CT, geometry, plan and kernel choice."""

    name: str
    hu: np.ndarray                 # float32 [nz][ny][nx]
    spacing: tuple                 # (sx, sy, sz)
    origin: tuple                  # centre of voxel (0,0,0): (ox, oy, oz)
    iso: tuple                     # (px, py, pz)
    gantry: np.ndarray             # float [n_cp]
    leaves: np.ndarray             # float [n_cp][2][L]
    jaws: np.ndarray               # float [n_cp][4]  (x1, x2, y1, y2)
    mu: np.ndarray                 # float [n_cp]
    n_taps: int
    field_limit: tuple             # (F_u, F_v): largest |jaw| the fan grid must hold
    machine: Machine
    wepl_mode: int = WEPL_PER_RAY
    lat_step: Optional[float] = None
    depth_step: Optional[float] = None
    loss_w: Optional[np.ndarray] = None   # weights of L = sum w D
    collimator: Optional[np.ndarray] = None   # float [n_cp] collimator angles; None = no collimator rotation

    def __post_init__(self):
        s = min(self.spacing)
        if self.lat_step is None:
            self.lat_step = float(s)
        if self.depth_step is None:
            self.depth_step = float(s)

    @property
    def shape(self):
        return self.hu.shape

    @property
    def n_cp(self) -> int:
        return int(self.gantry.shape[0])


def _centred_origin(shape_zyx, spacing):
    nz, ny, nx = shape_zyx
    sx, sy, sz = spacing
    return (-(nx - 1) / 2.0 * sx, -(ny - 1) / 2.0 * sy, -(nz - 1) / 2.0 * sz)


def voxel_centres(shape_zyx, spacing, origin):
    nz, ny, nx = shape_zyx
    x = origin[0] + np.arange(nx) * spacing[0]
    y = origin[1] + np.arange(ny) * spacing[1]
    z = origin[2] + np.arange(nz) * spacing[2]
    return x, y, z


# --------------------------------------------------------------------------- phantoms


def water_phantom(n: int, spacing: float) -> tuple:
    hu = np.zeros((n, n, n), dtype=np.float32)
    sp = (spacing, spacing, spacing)
    return hu, sp, _centred_origin(hu.shape, sp)


def pelvis_phantom(shape_zyx, spacing: float, seed: int, randomise: bool = False) -> tuple:
    """Synthetic pelvis painted in order (voxels classified by their centre):
    background -1000 HU; elliptic water body along z (semi-axes 170 x 110 mm,
    HU ~ N(0, 20^2)); two femur cylinders (radius 25 mm at (+-95, +15) mm, HU
    ~ U(700, 1200) each); a gas pocket ellipsoid (15 x 12 x 20 mm at (0, 40, 0),
    -800 HU).  With randomise=True the recipe itself is drawn per plan."""
    rng = np.random.default_rng(seed)
    sp = (spacing, spacing, spacing)
    origin = _centred_origin(shape_zyx, sp)
    x, y, z = voxel_centres(shape_zyx, sp, origin)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    body_a, body_b = 170.0, 110.0
    fem_r, fem_x, fem_y = 25.0, (95.0, 95.0), 15.0
    air = True
    air_ax, air_c = (15.0, 12.0, 20.0), (0.0, 40.0, 0.0)
    if randomise:
        sc = rng.uniform(0.85, 1.15)
        body_a, body_b = body_a * sc, body_b * sc
        fem_r = rng.uniform(20.0, 30.0)
        fem_x = (rng.uniform(85.0, 105.0), rng.uniform(85.0, 105.0))
        fem_y = rng.uniform(0.0, 30.0)
        air = rng.uniform() < 0.8
        air_ax = tuple(rng.uniform(8.0, 20.0, size=3))
        air_c = (rng.uniform(-10, 10), rng.uniform(30, 50), rng.uniform(-30, 30))
    hu = np.full(shape_zyx, -1000.0, dtype=np.float32)
    body = (X / body_a) ** 2 + (Y / body_b) ** 2 <= 1.0
    hu[body] = rng.normal(0.0, 20.0, size=int(body.sum())).astype(np.float32)
    for sgn, fx in ((-1.0, fem_x[0]), (1.0, fem_x[1])):
        fem = (X - sgn * fx) ** 2 + (Y - fem_y) ** 2 <= fem_r ** 2
        hu[fem] = np.float32(rng.uniform(700.0, 1200.0))
    if air:
        pocket = (((X - air_c[0]) / air_ax[0]) ** 2 + ((Y - air_c[1]) / air_ax[1]) ** 2
                  + ((Z - air_c[2]) / air_ax[2]) ** 2) <= 1.0
        hu[pocket] = -800.0
    return hu, sp, origin


# --------------------------------------------------------------------------- plans


def arc_angles(n_cp: int, two_arcs: bool) -> np.ndarray:
    """Single arc: 0, d, ..., 360 - d clockwise.  Two arcs: the first clockwise
    0, 2d, ..., then the second counter-clockwise 360 - d, 360 - 3d, ..."""
    if not two_arcs:
        return np.arange(n_cp, dtype=np.float64) * (360.0 / n_cp)
    n1 = (n_cp + 1) // 2
    n2 = n_cp - n1
    step = 360.0 / n1
    a1 = np.arange(n1) * step
    a2 = 360.0 - step / 2.0 - np.arange(n2) * step
    return np.concatenate([a1, a2]).astype(np.float64)


def random_apertures(n_cp: int, n_leaf: int, jaw_half: float, seed: int, max_gap: float = 60.0):
    """Per leaf pair: gap ~ U(0, max_gap), centre ~ U(-J + g/2, J - g/2) inside the jaws."""
    rng = np.random.default_rng(seed)
    gap = rng.uniform(0.0, max_gap, size=(n_cp, n_leaf))
    gap = np.minimum(gap, 2.0 * jaw_half)
    lo = -jaw_half + gap / 2.0
    hi = jaw_half - gap / 2.0
    c = lo + (hi - lo) * rng.uniform(size=(n_cp, n_leaf))
    leaves = np.stack([c - gap / 2.0, c + gap / 2.0], axis=1)
    return leaves


def random_mu(n_cp: int, seed: int, lo: float = 1.0, hi: float = 5.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n_cp)


def jaws_square(n_cp: int, half_x: float, half_y: float) -> np.ndarray:
    j = np.empty((n_cp, 4))
    j[:, 0], j[:, 1], j[:, 2], j[:, 3] = -half_x, half_x, -half_y, half_y
    return j


# --------------------------------------------------------------------------- configs


def config_c0(variant: str = "base") -> Case:
    """Water phantom 32^3 at 5 mm, one static field at gantry 0, 10 x 10 cm jaws,
    40 leaf pairs of 10 mm with edges from seed 0, 100 MU, 7 x 7 kernel."""
    m = Machine(n_leaf=40, leaf_width=10.0)
    hu, sp, origin = water_phantom(32, 5.0)
    rng = np.random.default_rng(0)
    draws = rng.uniform(-50.0, 50.0, size=(40, 2))
    leaves = np.stack([draws.min(axis=1), draws.max(axis=1)])[None]   # [1][2][40]
    jaws = jaws_square(1, 50.0, 50.0)
    mu = np.array([100.0])
    if variant == "mirror":          # (l, r) -> (-r, -l)
        leaves = np.stack([-leaves[:, 1], -leaves[:, 0]], axis=1)
    elif variant == "jaws_closed":
        jaws = jaws.copy()
        jaws[:, 1] = jaws[:, 0]
    elif variant == "leaves_closed":
        leaves = np.zeros_like(leaves)
        m.tau = 0.0
    elif variant != "base":
        raise ValueError(variant)
    return Case("C0-" + variant, hu, sp, origin, (0.0, 0.0, 0.0), np.array([0.0]), leaves, jaws, mu,
                7, (50.0, 50.0), m)


def config_c1(n_cp: int = 90) -> Case:
    """Pelvis 128 x 128 x 96 at 3 mm, 90 control points over 360 degrees, 60 leaf pairs
    of 5 mm, jaws +-40 mm, MU ~ U(1, 5), 15 x 15 kernel."""
    m = Machine(n_leaf=60, leaf_width=5.0)
    hu, sp, origin = pelvis_phantom((96, 128, 128), 3.0, seed=1001)
    gantry = arc_angles(n_cp, two_arcs=False)
    leaves = random_apertures(n_cp, 60, 40.0, seed=1002)
    mu = random_mu(n_cp, seed=1003)
    w = np.random.default_rng(1004).uniform(0.0, 1.0, size=hu.shape)
    return Case("C1", hu, sp, origin, (0.0, 0.0, 0.0), gantry, leaves, jaws_square(n_cp, 40.0, 40.0),
                mu, 15, (40.0, 40.0), m, loss_w=w)


def config_c2(n_cp: int = 180) -> Case:
    """Pelvis 192 x 192 x 128 at 2.5 mm, two arcs of 180 control points in total, 60 leaf
    pairs of 5 mm, jaws +-40 mm, 31 x 31 kernel."""
    m = Machine(n_leaf=60, leaf_width=5.0)
    hu, sp, origin = pelvis_phantom((128, 192, 192), 2.5, seed=2001)
    gantry = arc_angles(n_cp, two_arcs=True)
    leaves = random_apertures(n_cp, 60, 40.0, seed=2002)
    mu = random_mu(n_cp, seed=2003)
    w = np.random.default_rng(2005).uniform(0.0, 1.0, size=hu.shape)
    return Case("C2", hu, sp, origin, (0.0, 0.0, 0.0), gantry, leaves, jaws_square(n_cp, 40.0, 40.0),
                mu, 31, (40.0, 40.0), m, loss_w=w)


def config_p0() -> Case:
    """The paper's timing shape (Table 6: a 105 x 224 x 224 dose grid, 180 control
    points, kernel 55; the voxel size is not printed and is taken as 2 mm): a pelvis
    224 x 224 x 105 at 2 mm, two arcs of 180 control points, 60 leaf pairs of 5 mm,
    jaws +-40 mm, 55 x 55 kernel."""
    m = Machine(n_leaf=60, leaf_width=5.0)
    hu, sp, origin = pelvis_phantom((105, 224, 224), 2.0, seed=5001)
    gantry = arc_angles(180, two_arcs=True)
    leaves = random_apertures(180, 60, 40.0, seed=5002)
    mu = random_mu(180, seed=5003)
    w = np.random.default_rng(5004).uniform(0.0, 1.0, size=hu.shape)
    return Case("P0", hu, sp, origin, (0.0, 0.0, 0.0), gantry, leaves, jaws_square(180, 40.0, 40.0),
                mu, 55, (40.0, 40.0), m, loss_w=w)


def config_c4_plan(p: int, n_taps: int = 61, bench: bool = False) -> Case:
    """Randomised pelvis 128^3 at 3 mm with a random VMAT plan (plan index p, seed
    4000 + p).  bench=True forces 180 control points on two arcs and jaws +-40 mm."""
    rng = np.random.default_rng(4000 + p)
    m = Machine(n_leaf=60, leaf_width=5.0)
    hu, sp, origin = pelvis_phantom((128, 128, 128), 3.0, seed=int(rng.integers(1 << 31)),
                                    randomise=True)
    if bench:
        n_cp, jx, jy = 180, 40.0, 40.0
    else:
        n_cp = int(rng.integers(60, 181))
        jx, jy = rng.uniform(20.0, 50.0, size=2)
    gantry = arc_angles(n_cp, two_arcs=n_cp > 120)
    leaves = random_apertures(n_cp, 60, float(jx), seed=int(rng.integers(1 << 31)))
    mu = random_mu(n_cp, seed=int(rng.integers(1 << 31)))
    name = "C4-bench" if bench else "C4-%d" % p
    limit = (40.0, 40.0) if bench else (50.0, 50.0)
    return Case(name, hu, sp, origin, (0.0, 0.0, 0.0), gantry, leaves, jaws_square(n_cp, jx, jy), mu,
                n_taps, limit, m)


C4_OOD_KINDS = ("bone_air_slabs", "lung_body", "bone_body", "water")


def config_c4_ood(kind: str, p: int = 2000) -> Case:
    """Held-out plan p of the randomised pelvis workload on an anatomy unlike any
    training phantom, for the learned correction's error estimate: "bone_air_slabs"
    (the whole grid alternates 24 mm slabs of 1500 HU and -1000 HU along z),
    "lung_body" / "bone_body" (soft tissue of the phantom set to -700 / 900 HU), or
    "water" (0 HU everywhere)."""
    base = config_c4_plan(p)
    c = copy.copy(base)
    h = base.hu
    if kind == "bone_air_slabs":
        z = np.arange(h.shape[0])[:, None, None]
        c.hu = (np.where((z // 8) % 2 == 0, 1500.0, -1000.0) * np.ones_like(h)).astype(np.float32)
    elif kind in ("lung_body", "bone_body"):
        h = h.copy()
        h[(h > -900) & (h < 500)] = -700.0 if kind == "lung_body" else 900.0
        c.hu = h
    elif kind == "water":
        c.hu = np.zeros_like(h)
    else:
        raise ValueError("unknown anatomy %r" % kind)
    c.name = "C4-%d-%s" % (p, kind)
    return c


def tiny_case(seed: int = 7, n_cp: int = 2, n_taps: int = 3, shape=(6, 6, 6), spacing: float = 10.0,
              field: float = 30.0, n_leaf: int = 6, leaf_width: float = 10.0,
              wepl_mode: int = WEPL_PER_RAY, gantry=None) -> Case:
    """A tiny heterogeneous problem for brute-force checks."""
    rng = np.random.default_rng(seed)
    m = Machine(n_leaf=n_leaf, leaf_width=leaf_width)
    hu = rng.uniform(-1000.0, 1500.0, size=shape).astype(np.float32)
    sp = (spacing, spacing, spacing)
    origin = _centred_origin(shape, sp)
    if gantry is None:
        gantry = rng.uniform(0.0, 360.0, size=n_cp)
    gantry = np.asarray(gantry, dtype=np.float64)
    leaves = random_apertures(n_cp, n_leaf, field, seed=seed + 1, max_gap=2 * field)
    jaws = jaws_square(n_cp, field * 0.9, field * 0.8)
    mu = rng.uniform(1.0, 5.0, size=n_cp)
    iso = tuple(rng.uniform(-5.0, 5.0, size=3))
    return Case("tiny", hu, sp, origin, iso, gantry, leaves, jaws, mu, n_taps, (field, field), m,
                wepl_mode=wepl_mode)


def structures_c3(case: Case) -> dict:
    """Masks for the optimisation workload: PTV ellipsoid (30 x 30 x 40 mm) at the
    isocentre; rectum cylinder r = 12 mm along z at (0, 42), |z| <= 50, minus the PTV;
    bladder ellipsoid (40 x 30 x 30 mm) at (0, -35, 35), minus the PTV; the two femur
    cylinders and the elliptic body outline ("external") of the default pelvis
    phantom.  Together the organs at risk of the paper's objective (§2.5)."""
    x, y, z = voxel_centres(case.shape, case.spacing, case.origin)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ptv = (X / 30.0) ** 2 + (Y / 30.0) ** 2 + (Z / 40.0) ** 2 <= 1.0
    rectum = (X ** 2 + (Y - 42.0) ** 2 <= 12.0 ** 2) & (np.abs(Z) <= 50.0) & ~ptv
    bladder = ((X / 40.0) ** 2 + ((Y + 35.0) / 30.0) ** 2 + ((Z - 35.0) / 30.0) ** 2 <= 1.0) & ~ptv
    femur_l = (X + 95.0) ** 2 + (Y - 15.0) ** 2 <= 25.0 ** 2
    femur_r = (X - 95.0) ** 2 + (Y - 15.0) ** 2 <= 25.0 ** 2
    external = (X / 170.0) ** 2 + (Y / 110.0) ** 2 <= 1.0
    return {"ptv": ptv, "rectum": rectum, "bladder": bladder, "femur_l": femur_l, "femur_r": femur_r,
            "external": external}


# --------------------------------------------------------------------------- reference conditions

def reference_case(machine: Machine, n_taps: int, spacing: float = 2.0, size_mm: float = 300.0,
                   field_mm: float = 100.0, depth_mm: float = 100.0, ssd_mm: float = 900.0):
    """A water cube for gantry 0 (source at y = -SAD, beam along +y) whose entrance
    face lies at y = -depth_mm, so the surface is at SSD = SAD - depth_mm and the
    isocentre at the reference depth; one control point, 1 MU, the field set by
    the jaws to field_mm x field_mm at the isocentre with the leaves retracted
    10 mm behind them.

    The density is sampled trilinearly with zero outside the grid, so the water
    edge seen by a ray lies half a voxel before the first voxel centre.  The
    lateral size is odd so that x = z = 0 are voxel centres; along y the reference
    point falls between voxels j_ref and j_ref + 1 when depth_mm / spacing is an
    integer, and its dose is their linear interpolation (weight `w`).
    Returns (case, (ix, j_ref, iz, w))."""
    if abs(machine.sad - (ssd_mm + depth_mm)) > 1e-9:
        raise ValueError("reference depth + SSD must equal the SAD")
    n = int(round(size_mm / spacing))
    n += (n + 1) % 2
    c = (n - 1) // 2
    hu = np.zeros((n, n, n), dtype=np.float32)
    oy = -depth_mm + 0.5 * spacing                   # first voxel centre, half a voxel inside the face
    t = (0.0 - oy) / spacing                         # continuous y index of the isocentre
    j_ref = int(np.floor(t))
    w = float(t - j_ref)
    if not (0 <= j_ref and j_ref + 1 < n):
        raise ValueError("reference point outside the phantom")
    origin = (-c * spacing, oy, -c * spacing)
    half = field_mm / 2.0
    m = machine
    leaves = np.stack([np.full(m.n_leaf, -half - 10.0), np.full(m.n_leaf, half + 10.0)])[None]
    jaws = jaws_square(1, half, half)
    case = Case("reference", hu, (spacing,) * 3, origin, (0.0, 0.0, 0.0), np.array([0.0]), leaves, jaws,
                np.array([1.0]), n_taps, (half, half), m)
    return case, (c, j_ref, c, w)
