/*
 * pdrt.h — C ABI of the MI355X (gfx950) differentiable pencil-beam VMAT dose
 * engine, after arXiv:2512.18863 §2.2 ("A physics-informed, plug-and-play dose
 * engine for gradient-based radiotherapy treatment planning").
 *
 * The engine maps per-control-point delivery parameters (MLC leaf positions,
 * jaw positions, monitor units) to a 3-D dose grid for a fixed CT and beam
 * geometry (§2.1-2.2), and returns the gradient of a scalar loss with respect
 * to those parameters only (§2.1: density, depth and kernels sit outside the
 * gradient graph).
 *
 * Conventions shared by every entry point
 *  - Units: lengths in mm, angles in degrees.  Patient frame LPS, head-first
 *    supine: gantry angle phi puts the source at iso + SAD (sin phi, -cos phi, 0);
 *    the leaves travel along e_u = (cos phi, sin phi, 0) and are stacked along z.
 *  - Arrays are row-major, last index fastest.  Volumes on the CT grid are
 *    [nz][ny][nx]; leaves [n_cp][2][L] (bank A = left edges, bank B = right
 *    edges); jaws [n_cp][4] = (x1, x2, y1, y2), x along e_u, y along z;
 *    mu [n_cp].
 *  - Pointers marked "device" must point to memory of the current HIP device;
 *    "host" pointers are read during the call only.  The caller allocates and
 *    owns every buffer, including the workspace; the library keeps no state
 *    between calls and never allocates or synchronises.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls only
 *    enqueue work on it and return; results are valid once the stream reaches
 *    that point.
 *  - Return value: PDRT_OK (0) or a negative PDRT_E_* code.  All arguments are
 *    validated on the host before anything is enqueued, so an invalid call
 *    enqueues nothing.  PDRT_E_HIP means a launch failed; the stream's state is
 *    then unspecified.
 *  - Outputs are overwritten, never accumulated.  NaN and Inf propagate.
 *  - Calls that share a workspace on different streams race.
 */
#ifndef PDRT_H
#define PDRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDRT_OK 0
#define PDRT_E_INVALID (-1)     /* NULL pointer, non-positive size, even kernel size, ... */
#define PDRT_E_WORKSPACE (-2)   /* workspace NULL or smaller than pdrt_workspace_bytes() */
#define PDRT_E_HIP (-3)         /* a HIP launch or API call failed */
#define PDRT_E_UNSUPPORTED (-4) /* valid request the library does not implement */
#define PDRT_E_SCRATCH (-5)     /* problem larger than pdrt_dose_forward_noalloc's static scratch */

#define PDRT_WEPL_PER_RAY 0      /* water-equivalent depth along every divergent ray */
#define PDRT_WEPL_CENTRAL_AXIS 1 /* every ray takes the central-axis depth profile (§2.2.4) */

#define PDRT_CONV_FP32 0 /* lateral convolution in FP32 */
#define PDRT_CONV_BF16 1 /* lateral convolution with BF16 operands, FP32 accumulation */

#define PDRT_CACHE_F32 0  /* geometry cache holds G in FP32: results identical to the uncached path */
#define PDRT_CACHE_BF16 1 /* geometry cache holds G in BF16 (half the bytes, G rounded to 8 bits) */

#define PDRT_MAX_LEAF_PAIRS 160
#define PDRT_MAX_TAPS 127
#define PDRT_MAX_BLUR_RADIUS 64
#define PDRT_MAX_STRUCTS 32

/* CT grid.  Voxel (i, j, k) has its centre at (ox + i sx, oy + j sy, oz + k sz).
 * At most 2^31 - 1 voxels (PDRT_E_INVALID otherwise). */
typedef struct {
  int32_t nx, ny, nz;
  double sx, sy, sz;
  double ox, oy, oz;
} pdrt_grid;

/* Beam geometry shared by all control points (§2.2, beam parameter vector).
 * Collimator rotation (§2.2.2, last paragraph): with collimator_deg == NULL every
 * control point has collimator angle 0, leaves travel along e_u and the beam-frame
 * grid spans the field limit along each axis.  With collimator_deg given, the
 * fluence map of control point b is rasterised (and corrected) in its collimator
 * frame and then turned about the central axis by collimator_deg[b]: beam-frame
 * pixel (u, v) takes the collimator-frame map at (c u + s v, -s u + c v), (s, c) =
 * (sin, cos) of the angle, sampled bilinearly between pixel centres with zero
 * outside the grid (a positive angle turns the aperture from e_u towards z); the
 * beam-frame grid is then square, with half-extent hypot(field_limit_mm[0],
 * field_limit_mm[1]) plus the kernel's reach, so any rotation of the jaw rectangle
 * stays on it.  The angles carry no gradient. */
typedef struct {
  double sad_mm;               /* source-to-isocentre distance */
  double iso_mm[3];            /* isocentre in the patient frame */
  int32_t n_leaf_pairs;        /* L, 1..PDRT_MAX_LEAF_PAIRS */
  const double* leaf_edges_mm; /* host [L+1], ascending leaf boundaries along z at the isocentre plane */
  int32_t n_cp;                /* number of control points, >= 1 */
  const void* gantry_deg;      /* device [n_cp]: float for the FP32 entry points, double for _f64 */
  double field_limit_mm[2];    /* largest |jaw| along e_u and z; fixes the beam-frame grid extent */
  const void* collimator_deg;  /* device [n_cp] (float / double like gantry_deg) or NULL: collimator angles */
} pdrt_beam;

/* Dose model: kernel size, depth mode, convolution precision and machine tables. */
typedef struct {
  int32_t n_taps;          /* odd lateral kernel size n, 1..PDRT_MAX_TAPS */
  int32_t wepl_mode;       /* PDRT_WEPL_* */
  int32_t conv_mode;       /* PDRT_CONV_*; the _f64 entry points accept PDRT_CONV_FP32 only */
  double lateral_step_mm;  /* ray spacing Delta at the isocentre plane (the fluence pixel size) */
  double depth_step_mm;    /* plane spacing Delta_d along the central axis */
  double transmission;     /* MLC transmission tau (§2.2.2) */
  double calib;            /* dose per MU */
  int32_t n_dd;            /* depth-dose table length, >= 2 */
  double dd_step_mm;       /* depth-dose table spacing in water-equivalent depth */
  const void* dd;          /* device [n_dd]: DD(m dd_step), float (FP32 entry points) or double (_f64) */
  double kpoly[4][4];      /* kernel parameters A, a, B, b as cubics in depth z: c0 + c1 z + c2 z^2 + c3 z^3 */
  double kz_max_mm;        /* depths are clamped to [0, kz_max] before the polynomials */
  int32_t max_cp_batch;    /* control points per internal batch; 0 = the whole plan */
  /* Fluence corrections (§2.2.2 list), applied in this order to the aperture fluence
   * (which already carries the transmission); all off when fluence_corr == 0:
   *   source penumbra  directional Gaussians of FWHM pen_fwhm_mm[0] along u (leaf
   *                    travel) and pen_fwhm_mm[1] along v;
   *   head scatter     F + hs_amp G F, G the isotropic Gaussian of hs_sigma_mm;
   *   off-axis factor  1 + oar[0] r + oar[1] r^2, r = distance (mm) from the central
   *                    axis at the isocentre plane.
   * Each Gaussian is sampled at the fan pixel centres, truncated at 3 sigma (at most
   * PDRT_MAX_BLUR_RADIUS pixels, else PDRT_E_UNSUPPORTED) and normalised to unit sum;
   * the maps are zero outside the beam-frame grid. */
  int32_t fluence_corr;
  double pen_fwhm_mm[2];
  double hs_amp, hs_sigma_mm;
  double oar[2];
  /* Form of the ray march that evaluates the depth integral of Eq. 7 (the same
   * arithmetic, a different order of the compensated sums, so results agree to
   * rounding): 0 = one thread per ray walks its planes in order (default, the
   * faster on the MI355X); 1 = the planes of 64 rays are split over the wavefronts
   * of a workgroup, each scanning its segment and adding the sums of the segments
   * before it, exchanged through LDS. */
  int32_t march_scan;
} pdrt_kernel_spec;

/* Beam-frame grid of a problem (§2.2.3): Nu x Nv rays, Nk planes, first plane at
 * distance d0 from the source.  dims = {Nu, Nv, Nk}.  Internal fan-grid arrays are
 * laid out [cp][Nk][Nu][Nv] (v fastest). */
int pdrt_fan_dims(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                  int32_t dims[3], double* d0_mm);

/* Bytes of device workspace that pdrt_dose_forward / pdrt_dose_backward need
 * (with_backward != 0 sizes for both).  elem_bytes is 4 for the FP32 entry points,
 * 8 for _f64.  Returns 0 for an invalid problem. */
size_t pdrt_workspace_bytes(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                            int32_t with_backward, int32_t elem_bytes);

/* Byte offsets of the intermediates inside the workspace after a forward call
 * (debugging and tests): frame, rho_t ([ny][nx][nz]), F ([B][Nu][Nv]), z ([B][Nk]),
 * P and Dfan ([B][Nk][Nu][Nv]), A ([B][Nu][Nv]), comp, the two fluence-correction
 * scratch maps fc_tmp (2 x [B][Nu][Nv], present only with fluence corrections) and
 * box (int32 [B][4]: each control point's aperture rectangle u0, u1, v0, v1 of fan
 * pixels outside which the beam-frame fluence and its derivatives vanish), and with
 * collimator angles cframe ([n_cp][2]: sin, cos of each angle) and rot ([B][Nu][Nv]:
 * the beam-frame fluence after the rotation in a forward call; F then holds the
 * collimator-frame map); B = control points per batch; the arrays hold the last
 * batch.  Offsets of absent arrays equal the next one's. */
typedef struct {
  size_t frame, rho_t, fluence, depth, vol0, vol1, adj, comp, fc_tmp, box, cframe, rot, total;
  int32_t batch;
} pdrt_ws_layout;
int pdrt_workspace_layout(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                          int32_t with_backward, int32_t elem_bytes, pdrt_ws_layout* out);

/* HU -> relative electron density (§2.2, CT representation): piecewise linear
 * through (hu_pts[i], rho_pts[i]), clamped outside.  hu, rho: device [nz][ny][nx]
 * float (may alias).  hu_pts, rho_pts: host [n_pts], hu_pts ascending, 2..16 points. */
int pdrt_hu_to_density(const pdrt_grid* grid, const float* hu, float* rho, int32_t n_pts,
                       const double* hu_pts, const double* rho_pts, void* stream);

/* Forward dose (§2.2.2-2.2.7): for every control point the fluence map of the
 * aperture (Eq. 4, jaw masks, transmission), the water-equivalent depth by ray
 * marching through rho (Eq. 7), the primary with inverse square (Eq. 6) and depth
 * dose, the per-plane lateral convolution with the depth-dependent kernel (Eq. 8),
 * then trilinear back-projection to the CT grid and dose = calib sum_b MU_b D_b
 * (Eq. 9, compensated summation).
 *   rho    device [nz][ny][nx] relative density
 *   leaves device [n_cp][2][L], jaws device [n_cp][4], mu device [n_cp]
 *   dose   device [nz][ny][nx], overwritten
 *   ws     device workspace of ws_bytes >= pdrt_workspace_bytes(..., 0, 4) */
int pdrt_dose_forward(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam, const float* leaves,
                      const float* jaws, const float* mu, const pdrt_kernel_spec* spec, float* dose, void* ws,
                      size_t ws_bytes, void* stream);

/* Reverse mode of pdrt_dose_forward: given grad_dose = dL/d dose (device
 * [nz][ny][nx]) writes dL/d leaves [n_cp][2][L], dL/d jaws [n_cp][4] and dL/d mu
 * [n_cp] (device, overwritten).  Beam-frame volumes are recomputed per control
 * point, nothing is kept from the forward call.  The fluence map is piecewise
 * linear; at its kinks the one-sided derivative with strict inequalities is used
 * (a leaf exactly on a pixel boundary contributes zero there).  Deterministic:
 * no atomics, every sum in a fixed order.  ws_bytes >= pdrt_workspace_bytes(..., 1, 4). */
int pdrt_dose_backward(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam, const float* leaves,
                       const float* jaws, const float* mu, const pdrt_kernel_spec* spec, const float* grad_dose,
                       float* grad_leaves, float* grad_jaws, float* grad_mu, void* ws, size_t ws_bytes,
                       void* stream);

/* ---------------------------------------------------------------- allocation-free forward
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): pdrt_dose_forward with
 * the workspace taken from a static device array of PDRT_NOALLOC_SCRATCH_BYTES
 * (128 MiB) inside the library, one copy per device, held from the library's
 * first use on that device until the process ends.  The control points are run
 * in the largest batches whose forward workspace fits that array (at most
 * spec->max_cp_batch when it is set); the dose is the same as pdrt_dose_forward's
 * up to the grouping of the batches (the compensated sum over control points is
 * carried across batches).  Arguments as for pdrt_dose_forward, without ws.
 * Nothing in the scratch needs to start at zero: every call writes each part
 * before it reads it.  The call allocates and frees nothing.
 * Returns PDRT_E_SCRATCH when even one control point's workspace exceeds the
 * scratch (for example a CT of more than about 16 M voxels), before anything is
 * enqueued.  All calls on one device share its scratch: calls that overlap on
 * one device (different streams or host threads without ordering) race. */
#define PDRT_NOALLOC_SCRATCH_BYTES (128u << 20)
int pdrt_dose_forward_noalloc(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam,
                              const float* leaves, const float* jaws, const float* mu,
                              const pdrt_kernel_spec* spec, float* dose, void* stream);

/* The forward in double precision throughout (for finite-difference checks):
 * every array argument is double, beam->gantry_deg and spec->dd point to
 * doubles, spec->conv_mode must be PDRT_CONV_FP32.
 * ws_bytes >= pdrt_workspace_bytes(..., 0, 8). */
int pdrt_dose_forward_f64(const pdrt_grid* grid, const double* rho, const pdrt_beam* beam,
                          const double* leaves, const double* jaws, const double* mu,
                          const pdrt_kernel_spec* spec, double* dose, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- geometry cache
 * In plan optimisation (§2.5) only leaves, jaws and MU change between calls.  The
 * primary of Eq. 6 factorises as P_k(u, v) = F(u, v) G_k(u, v) with the
 * aperture-free factor G_k = (SAD/d_k)^2 DD(W_k(u, v)) of Eqs. 6-7; G and the
 * central-axis depths z_k that set the kernel taps (§2.2.5) depend only on the
 * density, the gantry angles and the beam-frame grid.  The cache holds both for
 * every control point, so the cached forward / backward skip the ray march:
 *   layout (device, caller-owned, cache_bytes >= pdrt_geometry_cache_bytes):
 *   z float [n_cp][Nk] at byte 0, then G [n_cp][Nk][Nu][Nv] (float for
 *   PDRT_CACHE_F32, bf16 for PDRT_CACHE_BF16) at the next 256-byte boundary.
 * A cache is valid for the grid, density, beam (gantry angles, isocentre, SAD,
 * field limit) and the spec fields n_taps, wepl_mode, lateral/depth steps, the
 * depth-dose table and march_scan it was built with; the caller keeps those fixed (they are not
 * checked).  The spec's conv_mode, calib, transmission, kernel polynomials and
 * fluence corrections may change between builds and uses.  With PDRT_CACHE_F32
 * the cached calls return exactly what pdrt_dose_forward / _backward return.
 * Returns 0 for an invalid problem or cache type. */
size_t pdrt_geometry_cache_bytes(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                                 int32_t cache_type);

/* Fill a cache (one ray march over all control points).  ws as for
 * pdrt_dose_forward (pdrt_workspace_bytes(..., 0, 4)). */
int pdrt_geometry_cache_build(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam,
                              const pdrt_kernel_spec* spec, int32_t cache_type, void* cache, size_t cache_bytes,
                              void* ws, size_t ws_bytes, void* stream);

/* pdrt_dose_forward / pdrt_dose_backward with the march replaced by the cache
 * (rho is not needed).  Workspace requirements are those of the uncached calls. */
int pdrt_dose_forward_cached(const pdrt_grid* grid, const pdrt_beam* beam, const float* leaves,
                             const float* jaws, const float* mu, const pdrt_kernel_spec* spec,
                             int32_t cache_type, const void* cache, size_t cache_bytes, float* dose, void* ws,
                             size_t ws_bytes, void* stream);
int pdrt_dose_backward_cached(const pdrt_grid* grid, const pdrt_beam* beam, const float* leaves,
                              const float* jaws, const float* mu, const pdrt_kernel_spec* spec,
                              int32_t cache_type, const void* cache, size_t cache_bytes,
                              const float* grad_dose, float* grad_leaves, float* grad_jaws, float* grad_mu,
                              void* ws, size_t ws_bytes, void* stream);

/* Hardware-constrained projection (§2.2.1, Eqs. 1-3): every opposing pair
 * (leaf pair, x jaws, y jaws) goes to centre-width form, the width is raised to
 * w_min and the centre clamped to [-limit, limit]; MU is raised to mu_min.
 * In/out arrays as in pdrt_dose_forward (device, float); outputs may alias inputs. */
typedef struct {
  double leaf_limit_mm, jaw_limit_x_mm, jaw_limit_y_mm, w_min_mm, mu_min;
} pdrt_limits;
int pdrt_project_params(int32_t n_cp, int32_t n_leaf_pairs, const float* leaves_in, const float* jaws_in,
                        const float* mu_in, const pdrt_limits* limits, float* leaves_out, float* jaws_out,
                        float* mu_out, void* stream);

/* Backward of the projection.  straight_through != 0 passes the gradient
 * unchanged (the default: a clamped closed aperture could otherwise never
 * reopen); straight_through == 0 applies the projection's own Jacobian.
 * Inputs are the unprojected parameters and the gradients w.r.t. the projected
 * ones; outputs (may alias the gradients) are the gradients w.r.t. the inputs. */
int pdrt_project_params_backward(int32_t n_cp, int32_t n_leaf_pairs, const float* leaves_in,
                                 const float* jaws_in, const float* mu_in, const pdrt_limits* limits,
                                 int32_t straight_through, const float* g_leaves, const float* g_jaws,
                                 const float* g_mu, float* gi_leaves, float* gi_jaws, float* gi_mu, void* stream);

/* Per-launch timing, a profiling aid.  Between pdrt_profile_begin and
 * pdrt_profile_end every kernel that pdrt_dose_forward / _backward / _forward_f64
 * enqueue is bracketed by a pair of HIP events on the caller's stream (at most
 * max_launches launches are recorded; later ones run untimed).  pdrt_profile_end
 * waits for the recorded events, writes one entry per kernel name (summed
 * milliseconds and launch count) to out[0 .. *n_entries) and stops recording;
 * it returns PDRT_E_WORKSPACE if launches went unrecorded.  The recorder is
 * process-wide and not thread-safe; begin creates its HIP events once and keeps
 * them for the life of the process. */
typedef struct {
  char name[32];
  int32_t launches;
  double total_ms;
} pdrt_kernel_time;
int pdrt_profile_begin(int32_t max_launches);
int pdrt_profile_end(pdrt_kernel_time* out, int32_t max_entries, int32_t* n_entries);

/* ------------------------------------------------------------------------
 * Primitives of the small 3-D convolutional network that maps a small-kernel
 * dose plus the density to a large-kernel dose (a learned correction of the
 * kernel-size effect of Table 5; "smaller kernel sizes first", §4.1).
 * Tensors are channels-last [D][H][W][C].  "bf16" pointers are device arrays of
 * IEEE bfloat16 (2 bytes), 16-byte aligned; weights are FP32 masters
 * w[cout][27][cin] (tap = 9 kd + 3 kh + kw over offsets -1..1) converted by
 * pdrt_conv3d_prepare_weights into the two operand layouts wt (forward,
 * [cout][pdrt_conv3d_kpad(cin)]) and wd (data gradient, [cin][pdrt_conv3d_kpad(cout)]).
 * All 3 x 3 x 3 convolutions use "same" zero padding and stride 1, BF16
 * operands and FP32 accumulation.  Same error conventions as above. */
typedef struct {
  int32_t D, H, W;
} pdrt_vol;

/* K extent of the operand layouts: 27 cin rounded up to a multiple of 32. */
int32_t pdrt_conv3d_kpad(int32_t cin);
int pdrt_conv3d_prepare_weights(int32_t cout, int32_t cin, const float* w, void* wt, void* wd, void* stream);
/* y = act(bias + conv(x1 ++ x2, w)); x1 has c1 channels, x2 (may be NULL when
 * c2 == 0) c2 channels, read as their channel concatenation; act = ReLU if relu.
 * c1, c2 multiples of 8 with c1 + c2 a multiple of 16; cout 16, 32 or 64. */
int pdrt_conv3d_forward(const pdrt_vol* vol, int32_t c1, int32_t c2, const void* x1, const void* x2, int32_t cout,
                        const void* wt, const float* bias, int32_t relu, void* y, void* stream);
/* dx1 ++ dx2 = conv^T(dy * [y_act > 0], w) (y_act NULL: no activation); c1 + c2 in
 * {16, 32, 48, 64, 96}. */
int pdrt_conv3d_backward_data(const pdrt_vol* vol, int32_t cout, const void* dy, const void* y_act, int32_t c1,
                              int32_t c2, const void* wd, void* dx1, void* dx2, void* stream);
/* dw[cout][27][c1 + c2] and db[cout] = sums over positions of the masked dy (FP32),
 * split over nsplit position chunks whose partial sums (ws) are added in a fixed
 * order; cout <= 64. */
size_t pdrt_conv3d_wgrad_ws_bytes(int32_t cout, int32_t cin, int32_t nsplit);
int pdrt_conv3d_backward_weight(const pdrt_vol* vol, int32_t c1, int32_t c2, const void* x1, const void* x2,
                                int32_t cout, const void* dy, const void* y_act, int32_t nsplit, float* ws,
                                size_t ws_bytes, float* dw, float* db, void* stream);
/* x[p][16] = (dose[p] * scale[0], rho[p], 0, ..., 0) as bf16; n = D H W. */
int pdrt_net_input(int32_t n, const float* dose, const float* scale, const float* rho, void* x, void* stream);
/* Workspace bytes of the two-pass reductions of pdrt_net_scale,
 * pdrt_net_fallback_stats and the exact form of pdrt_net_input_backward. */
size_t pdrt_net_reduce_ws_bytes(int32_t n);
/* Gradient w.r.t. the dose fed to pdrt_net_scale, pdrt_net_input and pdrt_net_head,
 * given gp = dL/dpred (and dx0 = dL/dx from the first convolution's data gradient):
 * ddose[p] = scale[0] (gp[p] + dx0[p][0]) at fixed scale; with dose, pred and argmax
 * (all three, from the same forward, and a workspace of pdrt_net_reduce_ws_bytes) it
 * adds the dependence of scale = 1/max(dose) on the dose at the argmax m:
 *   ddose[m] -= scale[0] (sum_p dose[p] ddose[p] - sum_p gp[p] pred[p]).
 * dose, pred, argmax all NULL: the scale is treated as a constant (ws unused). */
int pdrt_net_input_backward(int32_t n, const void* dx0, const float* gp, const float* scale, const float* dose,
                            const float* pred, const int32_t* argmax, float* ddose, void* ws, size_t ws_bytes,
                            void* stream);
/* scale[0] = 1 / max(dose) (1 if no dose is positive); argmax (may be NULL) receives
 * the first index of the maximum, or -1 if no dose is positive.  ws: device, at
 * least pdrt_net_reduce_ws_bytes(n). */
int pdrt_net_scale(int32_t n, const float* dose, float* scale, int32_t* argmax, void* ws, size_t ws_bytes,
                   void* stream);
/* out = a * scale[0] (inverse == 0) or a / scale[0] (inverse != 0); out may alias a. */
int pdrt_scale_by(int32_t n, const float* a, const float* scale, int32_t inverse, float* out, void* stream);
/* out = a + b over n bf16 elements (out may alias a or b); a, b, out 16-byte
 * aligned, else PDRT_E_INVALID. */
int pdrt_add_bf16(size_t n, const void* a, const void* b, void* out, void* stream);
/* 2 x 2 x 2 average pooling of the fine volume `fine` (even dims) and its
 * backward (backward != 0: x = gradient w.r.t. the pooled output, y = gradient
 * w.r.t. the fine input).  c a multiple of 8, x and y 16-byte aligned and
 * D H W c < 2^31, else PDRT_E_INVALID. */
int pdrt_pool2(const pdrt_vol* fine, int32_t c, const void* x, void* y, int32_t backward, void* stream);
/* Nearest-neighbour x2 upsampling to `fine` and its backward (same requirements). */
int pdrt_upsample2(const pdrt_vol* fine, int32_t c, const void* x, void* y, int32_t backward, void* stream);
/* Output head (FP32): pred = dose * scale + hb[0] + hw[0] . x, resid = hb[1] + hw[1] . x. */
int pdrt_net_head(int32_t n, int32_t c, const void* x, const float* hw, const float* hb, const float* dose,
                  const float* scale, float* pred, float* resid, void* stream);
/* Backward of the head: dx (bf16) and dhead = (dhw[2][c], dhb[2]); gr may be NULL;
 * dhead may be NULL (no head-weight gradient; ws is then unused). */
size_t pdrt_net_head_ws_bytes(int32_t n, int32_t c);
int pdrt_net_head_backward(int32_t n, int32_t c, const void* x, const float* hw, const float* gp, const float* gr,
                           void* dx, float* ws, size_t ws_bytes, float* dhead, void* stream);
/* Training loss L = inv_count sum mask [(pred - t s)^2 + lam R] (t = target, s =
 * tscale[0], e = pred - t s) with R = (resid - |e|)^2 for quantile == 0, or, for
 * 0 < quantile < 1, the pinball loss R = u (quantile - [u < 0]), u = |e| - resid,
 * whose minimiser is the quantile of |e| (an upper bound of the local error for a
 * quantile near 1); its gradients gp (of the first term only) and gr; loss[0] = L. */
size_t pdrt_net_loss_ws_bytes(int32_t n);
int pdrt_net_train_loss(int32_t n, const float* pred, const float* resid, const float* target, const float* tscale,
                        const float* mask, float inv_count, float lam, float quantile, float* gp, float* gr,
                        float* ws, size_t ws_bytes, float* loss, void* stream);
/* stats[0] = max pred, stats[1] = max resid over pred >= frac * max pred (device);
 * ws: device, at least pdrt_net_reduce_ws_bytes(n). */
int pdrt_net_fallback_stats(int32_t n, const float* pred, const float* resid, float frac, float* stats, void* ws,
                            size_t ws_bytes, void* stream);
/* One Adam update of n FP32 parameters (step t >= 1, bias-corrected). */
int pdrt_adam_step(size_t n, float* w, const float* g, float* m, float* v, float lr, float beta1, float beta2,
                   float eps, int32_t t, void* stream);

/* ---------------------------------------------------------------- plan assessment
 * The dose objective of the gradient-based optimisation study (§2.5) and the plan
 * metrics it is judged by (DVH parameters, §3; Dice of the prescription isodose
 * volume with the PTV, §2.5).  Structures are given as one label per voxel of the
 * dose grid, device uint32 [n_vox]: bit s set = the voxel belongs to structure s,
 * 0 <= s < n_struct <= PDRT_MAX_STRUCTS; structures may overlap.  dose is device
 * float [n_vox], finite and non-negative; n_vox < 2^32.  All calls are
 * asynchronous on `stream` and deterministic (floating-point partial sums are
 * added in a fixed order; counts are exact integers).  ws: device scratch of at
 * least pdrt_eval_ws_bytes(n_struct) bytes, owned by the caller. */
size_t pdrt_eval_ws_bytes(int32_t n_struct);

/* Weighted L1 objective (§2.5): loss[0] = sum_s weight[s] sum_{v in s} |dose_v - target[s]|
 * (the PTV term has target = prescribed dose, an organ-at-risk term target 0), in
 * double precision; grad (device float [n_vox], may be NULL) = dL/d dose, i.e.
 * sum over the structures s containing v of weight[s] sign(dose_v - target[s]), with
 * sign(0) = 0.  weight, target: host double [n_struct]; loss: device double [1]. */
int pdrt_l1_objective(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct,
                      const double* weight, const double* target, double* loss, float* grad, void* ws,
                      size_t ws_bytes, void* stream);

/* Differential dose-volume histograms: hist (device uint32 [n_struct][n_bins],
 * overwritten) counts the voxels of each structure in bin floor(dose / bin_width)
 * (computed in double precision, clamped to [0, n_bins - 1]); stats (device double
 * [n_struct][3], overwritten) = voxel count, sum of dose and maximum dose (0 for an
 * empty structure).  1 <= n_bins <= 16384, bin_width > 0. */
int pdrt_dose_histogram(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct,
                        int32_t n_bins, double bin_width, uint32_t* hist, double* stats, void* ws,
                        size_t ws_bytes, void* stream);

/* Voxels at or above a dose level (comparison in double precision): counts (device
 * uint64 [n_struct + 1], overwritten) = per structure, then over the whole grid.
 * With threshold = the prescribed dose this gives the Dice coefficient of the
 * 100 % isodose volume with structure s, 2 counts[s] / (counts[n_struct] + |s|). */
int pdrt_threshold_counts(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct,
                          double threshold, uint64_t* counts, void* stream);

/* Human-readable text of a status code (static storage). */
const char* pdrt_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int pdrt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PDRT_H */
