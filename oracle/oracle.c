/*
 * oracle.c — FP64 CPU oracle of the pencil-beam VMAT dose model of
 * arXiv:2512.18863, §2.2 (layers 1-7 and the sum over control points).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops, double precision,
 * one control point at a time; OpenMP only splits independent outputs.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes of the repository):
 *  - frame: patient LPS, head-first supine; gantry angle phi puts the source
 *    at iso + SAD (sin phi, -cos phi, 0); beam direction (-sin phi, cos phi, 0);
 *    leaf-travel axis e_u = (cos phi, sin phi, 0); leaf-stacking axis e_v = z.
 *  - the fluence pixels are the rays: ray (i, j) passes through the isocentre
 *    plane at (u_i, v_j) = ((i - c_u) D, (j - c_v) D); the magnified bilinear
 *    sampling of §2.2.3 (Eq. 5) is then the identity.
 *  - "distance d from the source" is the distance of a plane along the central
 *    axis; planes d_k = d0 + k Dd.
 *  - depth dose enters as a separate table DD(W) of the per-ray water-equivalent
 *    path length W; the lateral kernel is normalised to unit plane integral.
 *  - kernel taps sit at the fan-plane spacing delta_k = D d_k / SAD.
 *  - all sampling (density, fan-grid dose) is trilinear with zero padding.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- helpers */

/* sin/cos of an angle in degrees, exact at multiples of 90 degrees. */
static void gantry_frame(double deg, double* sn, double* cs) {
  double r = fmod(deg, 360.0);
  if (r < 0) r += 360.0;
  if (r == 0.0) { *sn = 0.0; *cs = 1.0; }
  else if (r == 90.0) { *sn = 1.0; *cs = 0.0; }
  else if (r == 180.0) { *sn = 0.0; *cs = -1.0; }
  else if (r == 270.0) { *sn = -1.0; *cs = 0.0; }
  else { double a = r * (M_PI / 180.0); *sn = sin(a); *cs = cos(a); }
}

/* Fractional overlap of pixel [x - D/2, x + D/2] with the interval [a, b] (§2.2.2, Eq. 4). */
static double overlap(double x, double a, double b, double D) {
  double hi = fmin(b, x + 0.5 * D);
  double lo = fmax(a, x - 0.5 * D);
  double o = hi - lo;
  return o > 0.0 ? o / D : 0.0;
}

/* d overlap / d a and d overlap / d b (subgradient with strict inequalities). */
static double overlap_da(double x, double a, double b, double D) {
  double hi = fmin(b, x + 0.5 * D), lo = fmax(a, x - 0.5 * D);
  return (hi - lo > 0.0 && a > x - 0.5 * D) ? -1.0 / D : 0.0;
}
static double overlap_db(double x, double a, double b, double D) {
  double hi = fmin(b, x + 0.5 * D), lo = fmax(a, x - 0.5 * D);
  return (hi - lo > 0.0 && b < x + 0.5 * D) ? 1.0 / D : 0.0;
}

static double dd_lookup(const or_model* m, double W) {
  double x = W / m->dd_step;
  if (x <= 0.0) return m->dd[0];
  if (x >= (double)(m->n_dd - 1)) return m->dd[m->n_dd - 1];
  int i = (int)floor(x);
  double f = x - (double)i;
  return m->dd[i] * (1.0 - f) + m->dd[i + 1] * f;
}

static double poly3(const double c[4], double z) { return c[0] + z * (c[1] + z * (c[2] + z * c[3])); }

/* Trilinear sample of a [n2][n1][n0] array at continuous index (c0, c1, c2), zero padded. */
static double trilinear(const double* a, int n0, int n1, int n2, double c0, double c1, double c2) {
  double f0 = floor(c0), f1 = floor(c1), f2 = floor(c2);
  long i0 = (long)f0, i1 = (long)f1, i2 = (long)f2;
  double w0 = c0 - f0, w1 = c1 - f1, w2 = c2 - f2;
  double s = 0.0;
  for (int d2 = 0; d2 < 2; ++d2) {
    long k = i2 + d2;
    if (k < 0 || k >= n2) continue;
    double wk = d2 ? w2 : 1.0 - w2;
    for (int d1 = 0; d1 < 2; ++d1) {
      long j = i1 + d1;
      if (j < 0 || j >= n1) continue;
      double wj = d1 ? w1 : 1.0 - w1;
      for (int d0 = 0; d0 < 2; ++d0) {
        long i = i0 + d0;
        if (i < 0 || i >= n0) continue;
        double wi = d0 ? w0 : 1.0 - w0;
        s += wk * wj * wi * a[(k * n1 + j) * n0 + i];
      }
    }
  }
  return s;
}

/* Transpose of trilinear(): a[corner] += w * val. */
static void trilinear_t(double* a, int n0, int n1, int n2, double c0, double c1, double c2, double val) {
  double f0 = floor(c0), f1 = floor(c1), f2 = floor(c2);
  long i0 = (long)f0, i1 = (long)f1, i2 = (long)f2;
  double w0 = c0 - f0, w1 = c1 - f1, w2 = c2 - f2;
  for (int d2 = 0; d2 < 2; ++d2) {
    long k = i2 + d2;
    if (k < 0 || k >= n2) continue;
    double wk = d2 ? w2 : 1.0 - w2;
    for (int d1 = 0; d1 < 2; ++d1) {
      long j = i1 + d1;
      if (j < 0 || j >= n1) continue;
      double wj = d1 ? w1 : 1.0 - w1;
      for (int d0 = 0; d0 < 2; ++d0) {
        long i = i0 + d0;
        if (i < 0 || i >= n0) continue;
        double wi = d0 ? w0 : 1.0 - w0;
        a[(k * n1 + j) * n0 + i] += wk * wj * wi * val;
      }
    }
  }
}

/* ------------------------------------------------------------- fan grid */

/* Fan grid covering the CT for every gantry angle:
 *   Nu = 2 ceil((F_u + h D) / D) + 1 (likewise Nv), h = (n - 1) / 2, so that the
 *   kernel's reach beyond the field edge stays on the grid (with collimator rotation
 *   F_u and F_v are both replaced by hypot(F_u, F_v));
 *   R = largest in-plane distance from the isocentre to a corner of the CT's
 *   voxel-edge box; planes d_k = SAD - R + k Dd, Nk = ceil(2R / Dd) + 1. */
int or_fan_dims(const or_model* m, int dims[3], double* d0) {
  if (m->n_taps < 1 || (m->n_taps % 2) == 0 || m->lat_step <= 0 || m->depth_step <= 0) return -1;
  int h = (m->n_taps - 1) / 2;
  double D = m->lat_step;
  if (m->coll_rot) {
    /* any rotation of a jaw rectangle inside [-F_u, F_u] x [-F_v, F_v] stays within
     * the radius hypot(F_u, F_v) of the central axis */
    double F = hypot(m->field_limit[0], m->field_limit[1]);
    dims[0] = dims[1] = 2 * (int)ceil((F + h * D) / D - 1e-9) + 1;
  } else {
    dims[0] = 2 * (int)ceil((m->field_limit[0] + h * D) / D - 1e-9) + 1;
    dims[1] = 2 * (int)ceil((m->field_limit[1] + h * D) / D - 1e-9) + 1;
  }
  double xs[2] = {m->ox - 0.5 * m->sx, m->ox + (m->nx - 0.5) * m->sx};
  double ys[2] = {m->oy - 0.5 * m->sy, m->oy + (m->ny - 0.5) * m->sy};
  double R = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double r = hypot(xs[a] - m->iso[0], ys[b] - m->iso[1]);
      if (r > R) R = r;
    }
  dims[2] = (int)ceil(2.0 * R / m->depth_step - 1e-9) + 1;
  *d0 = m->sad - R;
  return 0;
}

/* ------------------------------------------------------------- layers */

/* HU -> relative electron density via a calibration curve (§2.2, CT
 * representation): piecewise-linear between table points, clamped outside. */
void or_hu_to_density(long n, const double* hu, double* rho, int n_pts, const double* hu_pts,
                      const double* rho_pts) {
  for (long q = 0; q < n; ++q) {
    double h = hu[q];
    double r;
    if (h <= hu_pts[0]) r = rho_pts[0];
    else if (h >= hu_pts[n_pts - 1]) r = rho_pts[n_pts - 1];
    else {
      int s = 0;
      while (h > hu_pts[s + 1]) ++s;
      double t = (h - hu_pts[s]) / (hu_pts[s + 1] - hu_pts[s]);
      r = rho_pts[s] + t * (rho_pts[s + 1] - rho_pts[s]);
    }
    rho[q] = r;
  }
}

/* FluenceMapLayer (§2.2.2): F_ji = f(u_i; x1, x2) f(v_j; y1, y2) [tau S_j + (1 - tau) O_ji],
 * with O_ji = sum_l w_jl f(u_i; l_l, r_l) the leaf-opening fraction (Eq. 4), w_jl the
 * fraction of pixel row j covered by leaf pair l and S_j = sum_l w_jl.  Jaws mask the
 * field "analogously" (a product of the same overlap fractions); tau is the MLC
 * transmission through closed leaves; area outside the leaf bank and behind the
 * jaws is opaque. */
void or_raster(const or_model* m, const double* leaves, const double* jaws, double* F) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  int Nu = dims[0], Nv = dims[1], L = m->n_leaf;
  double D = m->lat_step, cu = 0.5 * (Nu - 1), cv = 0.5 * (Nv - 1);
  for (int j = 0; j < Nv; ++j) {
    double v = (j - cv) * D;
    double fy = overlap(v, jaws[2], jaws[3], D);
    double S = 0.0;
    for (int l = 0; l < L; ++l) S += overlap(v, m->leaf_edges[l], m->leaf_edges[l + 1], D);
    for (int i = 0; i < Nu; ++i) {
      double u = (i - cu) * D;
      double fx = overlap(u, jaws[0], jaws[1], D);
      double O = 0.0;
      for (int l = 0; l < L; ++l) {
        double w = overlap(v, m->leaf_edges[l], m->leaf_edges[l + 1], D);
        if (w > 0.0) O += w * overlap(u, leaves[l], leaves[L + l], D);
      }
      F[(long)j * Nu + i] = fx * fy * (m->tau * S + (1.0 - m->tau) * O);
    }
  }
}

/* Unit-sum Gaussian taps g_m = exp(-(m D)^2 / (2 sigma^2)) / sum, m = -R..R with
 * R = ceil(3 sigma / D): the Gaussian sampled at the pixel centres of the fan grid
 * and truncated at three standard deviations.  sigma <= 0 gives the single tap 1. */
static int gauss_taps(double sigma, double D, double* g, int rmax) {
  if (!(sigma > 0.0)) {
    g[0] = 1.0;
    return 0;
  }
  int R = (int)ceil(3.0 * sigma / D - 1e-9);
  if (R > rmax) R = rmax;
  double s = 0.0;
  for (int m = -R; m <= R; ++m) {
    g[m + R] = exp(-(m * D) * (m * D) / (2.0 * sigma * sigma));
    s += g[m + R];
  }
  for (int m = 0; m <= 2 * R; ++m) g[m] /= s;
  return R;
}

/* out = 1-D correlation of `in` [Nv][Nu] with taps g (radius R) along u (axis 0) or v
 * (axis 1), zero outside the map.  The taps are even, so it is its own transpose. */
static void blur_axis(int Nu, int Nv, const double* g, int R, int axis, const double* in, double* out) {
  for (int j = 0; j < Nv; ++j)
    for (int i = 0; i < Nu; ++i) {
      double acc = 0.0;
      for (int m = -R; m <= R; ++m) {
        int ii = axis == 0 ? i + m : i, jj = axis == 0 ? j : j + m;
        if (ii < 0 || ii >= Nu || jj < 0 || jj >= Nv) continue;
        acc += g[m + R] * in[(long)jj * Nu + ii];
      }
      out[(long)j * Nu + i] = acc;
    }
}

/* Fluence corrections (§2.2.2 list), on the aperture fluence F (which already carries
 * the MLC transmission):
 *   source penumbra  F1 = G_v (G_u F), directional Gaussians of the given FWHM
 *                    (sigma = FWHM / (2 sqrt(2 ln 2)));
 *   head scatter     F2 = F1 + hs_amp G_hs F1, G_hs the isotropic Gaussian of hs_sigma;
 *   off-axis         Fc = F2 (1 + oar0 r + oar1 r^2), r = sqrt(u^2 + v^2) at the isocentre plane.
 * Every blur acts on the fan pixel grid with zero padding.  The adjoint applies the
 * transposes in reverse order (each blur and the pointwise factor is symmetric). */
void or_fluence_correct(const or_model* m, const double* F, double* Fc, int transpose) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  int Nu = dims[0], Nv = dims[1];
  long plane = (long)Nu * Nv;
  if (!m->fcorr) {
    memcpy(Fc, F, sizeof(double) * plane);
    return;
  }
  enum { RMAX = 512 };
  double* gu = (double*)malloc(sizeof(double) * (2 * RMAX + 1));
  double* gv = (double*)malloc(sizeof(double) * (2 * RMAX + 1));
  double* gh = (double*)malloc(sizeof(double) * (2 * RMAX + 1));
  const double k = 2.0 * sqrt(2.0 * log(2.0)), D = m->lat_step;
  int Ru = gauss_taps(m->pen_fwhm_u / k, D, gu, RMAX), Rv = gauss_taps(m->pen_fwhm_v / k, D, gv, RMAX);
  int Rh = gauss_taps(m->hs_sigma, D, gh, RMAX);
  double* a = (double*)malloc(sizeof(double) * plane);
  double* b = (double*)malloc(sizeof(double) * plane);
  double* c = (double*)malloc(sizeof(double) * plane);
  double cu = 0.5 * (Nu - 1), cv = 0.5 * (Nv - 1);
  if (!transpose) {
    blur_axis(Nu, Nv, gu, Ru, 0, F, a);
    blur_axis(Nu, Nv, gv, Rv, 1, a, b);   /* b = F1 */
    blur_axis(Nu, Nv, gh, Rh, 0, b, a);
    blur_axis(Nu, Nv, gh, Rh, 1, a, c);   /* c = G_hs F1 */
    for (int j = 0; j < Nv; ++j)
      for (int i = 0; i < Nu; ++i) {
        double u = (i - cu) * D, v = (j - cv) * D, r = sqrt(u * u + v * v);
        long q = (long)j * Nu + i;
        Fc[q] = (b[q] + m->hs_amp * c[q]) * (1.0 + m->oar[0] * r + m->oar[1] * r * r);
      }
  } else {
    for (int j = 0; j < Nv; ++j)
      for (int i = 0; i < Nu; ++i) {
        double u = (i - cu) * D, v = (j - cv) * D, r = sqrt(u * u + v * v);
        long q = (long)j * Nu + i;
        c[q] = F[q] * (1.0 + m->oar[0] * r + m->oar[1] * r * r);
      }
    blur_axis(Nu, Nv, gh, Rh, 1, c, a);
    blur_axis(Nu, Nv, gh, Rh, 0, a, b);
    for (long q = 0; q < plane; ++q) c[q] += m->hs_amp * b[q];
    blur_axis(Nu, Nv, gv, Rv, 1, c, a);
    blur_axis(Nu, Nv, gu, Ru, 0, a, Fc);
  }
  free(gu); free(gv); free(gh); free(a); free(b); free(c);
}

/* Bilinear sample of a [n1][n0] map at continuous index (c0, c1), zero padded. */
static double bilinear(const double* a, int n0, int n1, double c0, double c1) {
  return trilinear(a, n0, n1, 1, c0, c1, 0.0);
}

/* Collimator rotation of the fluence map (§2.2.2, last paragraph): the map rasterised
 * in the collimator frame is turned about the central axis by the collimator angle
 * before the rays are traced.  Beam-frame pixel (u, v) takes the collimator-frame map
 * at (u', v') = (c u + s v, -s u + c v), sampled bilinearly between pixel centres
 * (zero outside the grid); the transpose spreads each beam-frame value back onto the
 * same four pixels with the same weights. */
void or_rotate_fluence(const or_model* m, double coll_deg, const double* in, double* out, int transpose) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  int Nu = dims[0], Nv = dims[1];
  double D = m->lat_step, cu = 0.5 * (Nu - 1), cv = 0.5 * (Nv - 1);
  double sn, cs;
  gantry_frame(coll_deg, &sn, &cs);
  long plane = (long)Nu * Nv;
  if (transpose) memset(out, 0, sizeof(double) * plane);
  for (int j = 0; j < Nv; ++j)
    for (int i = 0; i < Nu; ++i) {
      double u = (i - cu) * D, v = (j - cv) * D;
      double ur = cs * u + sn * v, vr = -sn * u + cs * v;
      double ci = ur / D + cu, cj = vr / D + cv;
      long q = (long)j * Nu + i;
      if (!transpose) out[q] = bilinear(in, Nu, Nv, ci, cj);
      else if (in[q] != 0.0) trilinear_t(out, Nu, Nv, 1, ci, cj, 0.0, in[q]);
    }
}

double or_rho_sample(const or_model* m, const double* rho, double x, double y, double z) {
  return trilinear(rho, m->nx, m->ny, m->nz, (x - m->ox) / m->sx, (y - m->oy) / m->sy,
                   (z - m->oz) / m->sz);
}

/* RadiologicalDepthLayer on the central axis (§2.2.4, Eq. 7): the single ray from the
 * source through the isocentre, sampled at the plane distances d_k; the integral is an
 * inclusive cumulative sum z_k = sum_{k' <= k} rho(s + d_k' b) Dd. */
void or_ca_depth(const or_model* m, const double* rho, double gantry_deg, double* z) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  double sn, cs;
  gantry_frame(gantry_deg, &sn, &cs);
  double acc = 0.0;
  for (int k = 0; k < dims[2]; ++k) {
    double e = (d0 - m->sad) + k * m->depth_step; /* d_k - SAD */
    double x = m->iso[0] - e * sn, y = m->iso[1] + e * cs, zz = m->iso[2];
    acc += or_rho_sample(m, rho, x, y, zz) * m->depth_step;
    z[k] = acc;
  }
}

/* Water-equivalent path length along each divergent ray (§2.2.4, Eq. 7, evaluated per
 * ray): ray (i, j) meets plane k at q = s + d_k (b + (u_i e_u + v_j e_v) / SAD); the step
 * between consecutive planes along the ray is Dd sqrt(1 + (u_i^2 + v_j^2) / SAD^2).
 * In central-axis mode every ray takes the central-axis profile, as the paper does. */
void or_wepl(const or_model* m, const double* rho, double gantry_deg, double* W) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  int Nu = dims[0], Nv = dims[1], Nk = dims[2];
  long plane = (long)Nu * Nv;
  if (m->wepl_mode == OR_WEPL_CENTRAL_AXIS) {
    double* z = (double*)malloc(sizeof(double) * Nk);
    or_ca_depth(m, rho, gantry_deg, z);
    for (int k = 0; k < Nk; ++k)
      for (long r = 0; r < plane; ++r) W[k * plane + r] = z[k];
    free(z);
    return;
  }
  double sn, cs;
  gantry_frame(gantry_deg, &sn, &cs);
  double D = m->lat_step, cu = 0.5 * (Nu - 1), cv = 0.5 * (Nv - 1);
#pragma omp parallel for schedule(static)
  for (long r = 0; r < plane; ++r) {
    int j = (int)(r / Nu), i = (int)(r % Nu);
    double u = (i - cu) * D, v = (j - cv) * D;
    double ds = m->depth_step * sqrt(1.0 + (u * u + v * v) / (m->sad * m->sad));
    double acc = 0.0;
    for (int k = 0; k < Nk; ++k) {
      double e = (d0 - m->sad) + k * m->depth_step; /* d_k - SAD */
      double g = 1.0 + e / m->sad;                  /* d_k / SAD */
      /* q - iso = (d_k - SAD) b + (d_k / SAD)(u e_u + v e_v) */
      double x = m->iso[0] - e * sn + g * u * cs;
      double y = m->iso[1] + e * cs + g * u * sn;
      double zz = m->iso[2] + g * v;
      acc += or_rho_sample(m, rho, x, y, zz) * ds;
      W[k * plane + r] = acc;
    }
  }
}

/* PencilBeamKernelLayer (§2.2.5): a radially symmetric kernel of the double-exponential
 * pencil-beam form p(r; z) = (A e^{-a r} + B e^{-b r}) / (2 pi r (A/a + B/b)), whose plane
 * integral is one, with A, a, B, b polynomials in the depth z (clamped to [0, kz_max]).
 * Taps sit on the fan-plane grid, spacing delta = D d_k / SAD:
 *   K[p][q] = delta^2 p(delta sqrt(p^2 + q^2); z) off centre,
 *   K[0][0] = integral of p over the disc of area delta^2 (radius delta / sqrt(pi)).
 * The truncated kernel is not renormalised. */
void or_taps(const or_model* m, double d_k, double z_k, double* K) {
  int n = m->n_taps, h = (n - 1) / 2;
  double z = z_k < 0.0 ? 0.0 : (z_k > m->kz_max ? m->kz_max : z_k);
  double A = poly3(m->kpoly[0], z), a = poly3(m->kpoly[1], z);
  double B = poly3(m->kpoly[2], z), b = poly3(m->kpoly[3], z);
  double norm = A / a + B / b;
  double delta = m->lat_step * d_k / m->sad;
  for (int p = -h; p <= h; ++p)
    for (int q = -h; q <= h; ++q) {
      double val;
      if (p == 0 && q == 0) {
        double r0 = delta / sqrt(M_PI);
        val = (A / a * (1.0 - exp(-a * r0)) + B / b * (1.0 - exp(-b * r0))) / norm;
      } else {
        double r = delta * sqrt((double)(p * p + q * q));
        val = delta * delta * (A * exp(-a * r) + B * exp(-b * r)) / (2.0 * M_PI * r * norm);
      }
      K[(p + h) * n + (q + h)] = val;
    }
}

/* BeamWiseConvolutionLayer (§2.2.6, Eq. 8) for one depth plane, zero padded:
 *   out[j][i] = sum_{p,q = -h..h} K[p + h][q + h] in[j + p][i + q].
 * (A correlation; for the radially symmetric taps it equals the convolution.) */
void or_conv_plane(int Nv, int Nu, int n, const double* K, const double* in, double* out) {
  int h = (n - 1) / 2;
  for (int j = 0; j < Nv; ++j)
    for (int i = 0; i < Nu; ++i) {
      double s = 0.0;
      for (int p = -h; p <= h; ++p) {
        int jj = j + p;
        if (jj < 0 || jj >= Nv) continue;
        for (int q = -h; q <= h; ++q) {
          int ii = i + q;
          if (ii < 0 || ii >= Nu) continue;
          s += K[(p + h) * n + (q + h)] * in[(long)jj * Nu + ii];
        }
      }
      out[(long)j * Nu + i] = s;
    }
}

/* BeamRotationLayer (§2.2.7): every voxel centre x is mapped into the fan grid of the
 * control point (t = x - iso; d = t.b + SAD; u = SAD t.e_u / d; v = SAD t.e_v / d;
 * continuous indices ((d - d0)/Dd, v/D + c_v, u/D + c_u)) and the beam-frame dose is
 * sampled trilinearly, zero outside the fan grid. */
static void voxel_to_fan(const or_model* m, double sn, double cs, double d0, double cu, double cv,
                         long vox, double* ck, double* cj, double* ci) {
  long ix = vox % m->nx, iy = (vox / m->nx) % m->ny, iz = vox / ((long)m->nx * m->ny);
  double tx = m->ox + ix * m->sx - m->iso[0];
  double ty = m->oy + iy * m->sy - m->iso[1];
  double tz = m->oz + iz * m->sz - m->iso[2];
  double d = (-sn * tx + cs * ty) + m->sad;
  double u = m->sad * (cs * tx + sn * ty) / d;
  double v = m->sad * tz / d;
  *ck = (d - d0) / m->depth_step;
  *cj = v / m->lat_step + cv;
  *ci = u / m->lat_step + cu;
}

void or_gather(const or_model* m, double gantry_deg, const double* Dfan, double* Db) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  double sn, cs;
  gantry_frame(gantry_deg, &sn, &cs);
  double cu = 0.5 * (dims[0] - 1), cv = 0.5 * (dims[1] - 1);
  long nvox = (long)m->nx * m->ny * m->nz;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < nvox; ++x) {
    double ck, cj, ci;
    voxel_to_fan(m, sn, cs, d0, cu, cv, x, &ck, &cj, &ci);
    Db[x] = trilinear(Dfan, dims[0], dims[1], dims[2], ci, cj, ck);
  }
}

/* Transpose of or_gather (serial, so the summation order is fixed). */
void or_scatter(const or_model* m, double gantry_deg, const double* g, double* Ghat) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  double sn, cs;
  gantry_frame(gantry_deg, &sn, &cs);
  double cu = 0.5 * (dims[0] - 1), cv = 0.5 * (dims[1] - 1);
  long nfan = (long)dims[0] * dims[1] * dims[2];
  memset(Ghat, 0, sizeof(double) * nfan);
  long nvox = (long)m->nx * m->ny * m->nz;
  for (long x = 0; x < nvox; ++x) {
    if (g[x] == 0.0) continue;
    double ck, cj, ci;
    voxel_to_fan(m, sn, cs, d0, cu, cv, x, &ck, &cj, &ci);
    trilinear_t(Ghat, dims[0], dims[1], dims[2], ci, cj, ck, g[x]);
  }
}

/* ------------------------------------------------------------- pipeline */

/* Primary fluence volume (§2.2.3, Eq. 6, with the depth dose of the ray):
 * P_kji = F_ji (SAD / d_k)^2 DD(W_kji). */
static void primary(const or_model* m, const int dims[3], double d0, const double* F, const double* W,
                    double* P) {
  long plane = (long)dims[0] * dims[1];
  for (int k = 0; k < dims[2]; ++k) {
    double dk = d0 + k * m->depth_step;
    double c = (m->sad / dk) * (m->sad / dk);
    for (long r = 0; r < plane; ++r) P[k * plane + r] = F[r] * c * dd_lookup(m, W[k * plane + r]);
  }
}

static void conv_volume(const or_model* m, const int dims[3], double d0, const double* z, const double* in,
                        double* out) {
  int n = m->n_taps;
  long plane = (long)dims[0] * dims[1];
#pragma omp parallel
  {
    double* K = (double*)malloc(sizeof(double) * n * n);
#pragma omp for schedule(dynamic)
    for (int k = 0; k < dims[2]; ++k) {
      or_taps(m, d0 + k * m->depth_step, z[k], K);
      or_conv_plane(dims[1], dims[0], n, K, in + k * plane, out + k * plane);
    }
    free(K);
  }
}

void or_forward_cp(const or_model* m, const double* rho, double gantry_deg, double coll_deg,
                   const double* leaves, const double* jaws, double* F_out, double* z_out, double* W_out,
                   double* P_out, double* Dfan_out, double* Db_out) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  long plane = (long)dims[0] * dims[1], nfan = plane * dims[2];
  double* F = F_out ? F_out : (double*)malloc(sizeof(double) * plane);
  double* z = z_out ? z_out : (double*)malloc(sizeof(double) * dims[2]);
  double* W = W_out ? W_out : (double*)malloc(sizeof(double) * nfan);
  double* P = P_out ? P_out : (double*)malloc(sizeof(double) * nfan);
  double* Dfan = Dfan_out ? Dfan_out : (double*)malloc(sizeof(double) * nfan);
  or_raster(m, leaves, jaws, F);
  if (m->fcorr) {
    double* Fr = (double*)malloc(sizeof(double) * plane);
    memcpy(Fr, F, sizeof(double) * plane);
    or_fluence_correct(m, Fr, F, 0);
    free(Fr);
  }
  if (m->coll_rot) {
    double* Fr = (double*)malloc(sizeof(double) * plane);
    memcpy(Fr, F, sizeof(double) * plane);
    or_rotate_fluence(m, coll_deg, Fr, F, 0);
    free(Fr);
  }
  or_ca_depth(m, rho, gantry_deg, z);
  or_wepl(m, rho, gantry_deg, W);
  primary(m, dims, d0, F, W, P);
  conv_volume(m, dims, d0, z, P, Dfan);
  if (Db_out) or_gather(m, gantry_deg, Dfan, Db_out);
  if (!F_out) free(F);
  if (!z_out) free(z);
  if (!W_out) free(W);
  if (!P_out) free(P);
  if (!Dfan_out) free(Dfan);
}

/* Dose accumulation (§2.2.7, Eq. 9): D = calib sum_b MU_b D_b, summed in control-point order. */
void or_forward(const or_model* m, const double* rho, int n_cp, const double* gantry_deg,
                const double* coll_deg, const double* leaves, const double* jaws, const double* mu,
                double* dose) {
  long nvox = (long)m->nx * m->ny * m->nz;
  double* Db = (double*)malloc(sizeof(double) * nvox);
  memset(dose, 0, sizeof(double) * nvox);
  for (int b = 0; b < n_cp; ++b) {
    or_forward_cp(m, rho, gantry_deg[b], coll_deg ? coll_deg[b] : 0.0, leaves + (long)b * 2 * m->n_leaf,
                  jaws + (long)b * 4, NULL, NULL, NULL, NULL, NULL, Db);
    for (long x = 0; x < nvox; ++x) dose[x] += mu[b] * Db[x];
  }
  for (long x = 0; x < nvox; ++x) dose[x] *= m->calib;
  free(Db);
}

/* Chain rule through the fluence map: F_ji = fx_i fy_j [tau S_j + (1 - tau) O_ji]. */
void or_raster_backward(const or_model* m, const double* leaves, const double* jaws, const double* gF,
                        double* gleaves, double* gjaws) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  int Nu = dims[0], Nv = dims[1], L = m->n_leaf;
  double D = m->lat_step, cu = 0.5 * (Nu - 1), cv = 0.5 * (Nv - 1), tau = m->tau;
  memset(gleaves, 0, sizeof(double) * 2 * L);
  memset(gjaws, 0, sizeof(double) * 4);
  for (int j = 0; j < Nv; ++j) {
    double v = (j - cv) * D;
    double fy = overlap(v, jaws[2], jaws[3], D);
    double dfy1 = overlap_da(v, jaws[2], jaws[3], D), dfy2 = overlap_db(v, jaws[2], jaws[3], D);
    double S = 0.0;
    for (int l = 0; l < L; ++l) S += overlap(v, m->leaf_edges[l], m->leaf_edges[l + 1], D);
    for (int i = 0; i < Nu; ++i) {
      double g = gF[(long)j * Nu + i];
      if (g == 0.0) continue;
      double u = (i - cu) * D;
      double fx = overlap(u, jaws[0], jaws[1], D);
      double dfx1 = overlap_da(u, jaws[0], jaws[1], D), dfx2 = overlap_db(u, jaws[0], jaws[1], D);
      double O = 0.0;
      for (int l = 0; l < L; ++l) {
        double w = overlap(v, m->leaf_edges[l], m->leaf_edges[l + 1], D);
        if (w <= 0.0) continue;
        O += w * overlap(u, leaves[l], leaves[L + l], D);
        gleaves[l] += g * fx * fy * (1.0 - tau) * w * overlap_da(u, leaves[l], leaves[L + l], D);
        gleaves[L + l] += g * fx * fy * (1.0 - tau) * w * overlap_db(u, leaves[l], leaves[L + l], D);
      }
      double br = tau * S + (1.0 - tau) * O;
      gjaws[0] += g * dfx1 * fy * br;
      gjaws[1] += g * dfx2 * fy * br;
      gjaws[2] += g * fx * dfy1 * br;
      gjaws[3] += g * fx * dfy2 * br;
    }
  }
}

/* Reverse mode through the whole pipeline of every control point.  Density, depth and
 * kernel are outside the gradient graph (§2.1); per control point: Ghat = gather^T g,
 * H = K (*) Ghat (the taps are point symmetric, so the transposed convolution uses the
 * same taps), A_ji = sum_k H_kji (SAD/d_k)^2 DD(W_kji), dL/dMU_b = calib <A, F>,
 * dL/dF = calib MU_b A, then the fluence-map chain rule. */
void or_backward(const or_model* m, const double* rho, int n_cp, const double* gantry_deg,
                 const double* coll_deg, const double* leaves, const double* jaws, const double* mu,
                 const double* g, double* gleaves, double* gjaws, double* gmu) {
  int dims[3];
  double d0;
  or_fan_dims(m, dims, &d0);
  long plane = (long)dims[0] * dims[1], nfan = plane * dims[2];
  double* F = (double*)malloc(sizeof(double) * plane);
  double* z = (double*)malloc(sizeof(double) * dims[2]);
  double* W = (double*)malloc(sizeof(double) * nfan);
  double* Gh = (double*)malloc(sizeof(double) * nfan);
  double* H = (double*)malloc(sizeof(double) * nfan);
  double* A = (double*)malloc(sizeof(double) * plane);
  double* gF = (double*)malloc(sizeof(double) * plane);
  for (int b = 0; b < n_cp; ++b) {
    const double* lv = leaves + (long)b * 2 * m->n_leaf;
    const double* jw = jaws + (long)b * 4;
    or_raster(m, lv, jw, F);
    or_ca_depth(m, rho, gantry_deg[b], z);
    or_wepl(m, rho, gantry_deg[b], W);
    or_scatter(m, gantry_deg[b], g, Gh);
    conv_volume(m, dims, d0, z, Gh, H);
    for (long r = 0; r < plane; ++r) A[r] = 0.0;
    for (int k = 0; k < dims[2]; ++k) {
      double dk = d0 + k * m->depth_step;
      double c = (m->sad / dk) * (m->sad / dk);
      for (long r = 0; r < plane; ++r) A[r] += H[k * plane + r] * c * dd_lookup(m, W[k * plane + r]);
    }
    /* dL/dMU = calib <A, R Fc> (Fc the corrected map, R the collimator rotation);
     * dL/d(R Fc) = calib MU A, carried back through the rotation's transpose and the
     * corrections' adjoint to the aperture fluence, then to leaves and jaws */
    const double cb = coll_deg ? coll_deg[b] : 0.0;
    if (m->fcorr) {
      memcpy(gF, F, sizeof(double) * plane);
      or_fluence_correct(m, gF, F, 0);
    }
    if (m->coll_rot) {
      memcpy(gF, F, sizeof(double) * plane);
      or_rotate_fluence(m, cb, gF, F, 0);
    }
    double s = 0.0;
    for (long r = 0; r < plane; ++r) s += A[r] * F[r];
    gmu[b] = m->calib * s;
    for (long r = 0; r < plane; ++r) gF[r] = m->calib * mu[b] * A[r];
    if (m->coll_rot) {
      memcpy(A, gF, sizeof(double) * plane);
      or_rotate_fluence(m, cb, A, gF, 1);
    }
    if (m->fcorr) {
      memcpy(A, gF, sizeof(double) * plane);
      or_fluence_correct(m, A, gF, 1);
    }
    or_raster_backward(m, lv, jw, gF, gleaves + (long)b * 2 * m->n_leaf, gjaws + (long)b * 4);
  }
  free(F); free(z); free(W); free(Gh); free(H); free(A); free(gF);
}

/* BeamValidationLayer (§2.2.1): each opposing pair (a, b) goes to centre-width form
 * c = (a + b)/2, w = b - a (Eq. 1), w is raised to w_min, c is clamped to [-lim, lim],
 * and the pair is rebuilt as (c - w/2, c + w/2) (Eq. 2).  MU is raised to mu_min (the
 * floor of Eq. 3, computed by the caller). */
static void project_pair(double* a, double* b, double lim, double w_min) {
  double c = 0.5 * (*a + *b), w = *b - *a;
  if (w < w_min) w = w_min;
  if (c < -lim) c = -lim;
  if (c > lim) c = lim;
  *a = c - 0.5 * w;
  *b = c + 0.5 * w;
}

void or_project(int n_cp, int n_leaf, double* leaves, double* jaws, double* mu, double leaf_limit,
                double jaw_limit_x, double jaw_limit_y, double w_min, double mu_min) {
  for (int b = 0; b < n_cp; ++b) {
    double* lv = leaves + (long)b * 2 * n_leaf;
    for (int l = 0; l < n_leaf; ++l) project_pair(&lv[l], &lv[n_leaf + l], leaf_limit, w_min);
    double* jw = jaws + (long)b * 4;
    project_pair(&jw[0], &jw[1], jaw_limit_x, w_min);
    project_pair(&jw[2], &jw[3], jaw_limit_y, w_min);
    if (mu[b] < mu_min) mu[b] = mu_min;
  }
}
