/*
 * oracle.h — FP64 CPU oracle of the pencil-beam VMAT dose model of
 * arXiv:2512.18863 ("A physics-informed, plug-and-play dose engine for
 * gradient-based radiotherapy treatment planning"), §2.2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no header, source, table or helper
 * with the HIP library.
 *
 * Every routine is a plain, slow transcription of the model's definitions in
 * double precision.  Loops follow the order in which the paper describes the
 * layers (fluence -> depth -> primary -> kernel -> convolution -> rotation ->
 * sum), one control point at a time.  Where the paper is silent the reading
 * is stated next to the routine that takes it.
 *
 * Array layouts (row-major, last index fastest):
 *   CT / density / dose       [nz][ny][nx]
 *   leaves per control point  [2][L]  (bank A = left edges l_i, bank B = right edges r_i)
 *   jaws per control point    [4]     (x1, x2 along the leaf-travel axis; y1, y2 across)
 *   fluence map F             [Nv][Nu]
 *   fan-grid volumes          [Nk][Nv][Nu]
 *   kernel taps               [n][n]
 */
#ifndef PDRT_ORACLE_H
#define PDRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_WEPL_PER_RAY 0
#define OR_WEPL_CENTRAL_AXIS 1

typedef struct {
  /* CT grid: voxel (i,j,k) centre = (ox + i*sx, oy + j*sy, oz + k*sz), mm, patient LPS */
  int nx, ny, nz;
  double sx, sy, sz;
  double ox, oy, oz;
  /* beam geometry */
  double sad;              /* source-to-isocentre distance, mm */
  double iso[3];           /* isocentre, mm */
  int n_leaf;              /* leaf pairs L */
  const double* leaf_edges;/* L+1 ascending leaf boundaries along v at the isocentre plane, mm */
  double field_limit[2];   /* max |jaw| along u and v, mm: fixes the fan-grid extent */
  /* kernel / model spec */
  int n_taps;              /* odd lateral kernel size n */
  int wepl_mode;           /* OR_WEPL_PER_RAY or OR_WEPL_CENTRAL_AXIS */
  double lat_step;         /* lateral ray spacing Delta at the isocentre plane, mm */
  double depth_step;       /* plane spacing Delta_d along the central axis, mm */
  double tau;              /* MLC transmission */
  double calib;            /* dose per MU */
  int n_dd;                /* depth-dose table length */
  double dd_step;          /* depth-dose table spacing in water-equivalent depth, mm */
  const double* dd;        /* depth-dose table DD(m * dd_step), m = 0..n_dd-1 */
  double kpoly[4][4];      /* kernel parameters A, a, B, b as cubic polynomials in depth z (mm) */
  double kz_max;           /* depth clamp [0, kz_max] for the kernel parameters, mm */
  /* fluence corrections (§2.2.2 list), applied to the aperture fluence in this order;
   * all off when fcorr == 0 */
  int fcorr;
  double pen_fwhm_u;       /* source penumbra: Gaussian FWHM along u (leaf travel), mm at the isocentre plane */
  double pen_fwhm_v;       /* ... and along v (across the leaves, the y jaws), mm */
  double hs_amp;           /* head scatter: F + hs_amp (G * F), G an isotropic unit-sum Gaussian ... */
  double hs_sigma;         /* ... of standard deviation hs_sigma, mm */
  double oar[2];           /* off-axis factor 1 + oar[0] r + oar[1] r^2, r = distance from the central axis, mm */
  /* collimator rotation (§2.2.2, last paragraph): 0 = none (every control point at
   * collimator angle 0, fan grid as for the jaws); 1 = the plan carries collimator
   * angles, and the fan grid is square, large enough for any rotation of the jaw
   * rectangle (half-extent hypot(F_u, F_v) plus the kernel's reach) */
  int coll_rot;
} or_model;

/* Fan-grid sizes; returns 0 on success. dims = {Nu, Nv, Nk}. */
int or_fan_dims(const or_model* m, int dims[3], double* d0);

/* HU -> relative density, piecewise linear, clamped at both ends (§2.2). */
void or_hu_to_density(long n, const double* hu, double* rho, int n_pts, const double* hu_pts,
                      const double* rho_pts);

/* One control point: fluence map F [Nv][Nu] (§2.2.2, Eq. 4). */
void or_raster(const or_model* m, const double* leaves, const double* jaws, double* F);

/* Fluence corrections of §2.2.2 (source penumbra, head scatter, off-axis factor) on one
 * map [Nv][Nu], out of place; the identity copy when m->fcorr == 0.  transpose != 0
 * applies the adjoint (the same operators in reverse order). */
void or_fluence_correct(const or_model* m, const double* F, double* Fc, int transpose);

/* Collimator rotation (§2.2.2, last paragraph) of one map [Nv][Nu] about the central
 * axis: Fb(u, v) = bilinear sample of Fc at (c u + s v, -s u + c v), zero outside the
 * grid, with (s, c) = (sin, cos) of the collimator angle, so that a positive angle
 * turns the aperture from e_u towards e_v.  transpose != 0 applies the adjoint
 * (Fc <- R^T Fb).  Out of place. */
void or_rotate_fluence(const or_model* m, double coll_deg, const double* in, double* out, int transpose);

/* Density sample at a patient-frame point, trilinear with zero padding (§2.2.4). */
double or_rho_sample(const or_model* m, const double* rho, double x, double y, double z);

/* Central-axis water-equivalent depth z_k, k = 0..Nk-1 (§2.2.4, Eq. 7). */
void or_ca_depth(const or_model* m, const double* rho, double gantry_deg, double* z);

/* Water-equivalent path length W [Nk][Nv][Nu] along every divergent ray (§2.2.4, Eq. 7). */
void or_wepl(const or_model* m, const double* rho, double gantry_deg, double* W);

/* Kernel taps of one plane at distance d_k from the source and CA depth z_k (§2.2.5). */
void or_taps(const or_model* m, double d_k, double z_k, double* K);

/* Zero-padded 2-D convolution of one Nv x Nu plane with an n x n kernel (§2.2.6, Eq. 8). */
void or_conv_plane(int Nv, int Nu, int n, const double* K, const double* in, double* out);

/* Dose of one control point in the patient frame, trilinear fan-grid sampling (§2.2.7). */
void or_gather(const or_model* m, double gantry_deg, const double* Dfan, double* Db);

/* Transpose of or_gather: accumulates g into Ghat [Nk][Nv][Nu] (overwritten). */
void or_scatter(const or_model* m, double gantry_deg, const double* g, double* Ghat);

/* Intermediates of one control point; any output pointer may be NULL.  F is the fluence
 * in the beam frame (after the corrections and the collimator rotation). */
void or_forward_cp(const or_model* m, const double* rho, double gantry_deg, double coll_deg,
                   const double* leaves, const double* jaws, double* F, double* z, double* W, double* P,
                   double* Dfan, double* Db);

/* Whole plan: dose = calib * sum_b MU_b * D_b (§2.2.7, Eq. 9); dose [nz][ny][nx] overwritten.
 * coll_deg [n_cp] may be NULL (all collimator angles 0). */
void or_forward(const or_model* m, const double* rho, int n_cp, const double* gantry_deg,
                const double* coll_deg, const double* leaves, const double* jaws, const double* mu,
                double* dose);

/* Gradient of L with dL/dD = g w.r.t. leaves [n_cp][2][L], jaws [n_cp][4], mu [n_cp]. */
void or_backward(const or_model* m, const double* rho, int n_cp, const double* gantry_deg,
                 const double* coll_deg, const double* leaves, const double* jaws, const double* mu,
                 const double* g, double* gleaves, double* gjaws, double* gmu);

/* Backward of the fluence map of one control point: gF [Nv][Nu] -> gleaves [2][L], gjaws [4]. */
void or_raster_backward(const or_model* m, const double* leaves, const double* jaws, const double* gF,
                        double* gleaves, double* gjaws);

/* Hardware-constrained projection (§2.2.1, Eqs. 1-3) of n_cp control points, in place. */
void or_project(int n_cp, int n_leaf, double* leaves, double* jaws, double* mu, double leaf_limit,
                double jaw_limit_x, double jaw_limit_y, double w_min, double mu_min);

#ifdef __cplusplus
}
#endif
#endif
