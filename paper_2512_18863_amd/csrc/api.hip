// api.hip — the C ABI declared in include/pdrt.h: validation, beam-frame sizing,
// workspace layout and the launch sequence of the dose path.  Host code only; it
// never allocates, frees or synchronises.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <type_traits>
#include <vector>

#include "pdrt_internal.hpp"

using namespace pdrt;

namespace pdrt {

namespace {
struct ProfRec {
  const char* name;
  int a, b;  // indices into the event pool
};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> recs;
  bool overflow = false;
};
Profiler& prof() {
  static Profiler p;
  return p;
}
}  // namespace

bool prof_enabled() { return prof().on; }

int prof_mark(hipStream_t s) {
  Profiler& P = prof();
  if (P.used >= P.pool.size()) {
    P.overflow = true;
    return -1;
  }
  int i = (int)P.used++;
  if (hipEventRecord(P.pool[i], s) != hipSuccess) return -1;
  return i;
}

void prof_record(const char* name, int a, int b) { prof().recs.push_back(ProfRec{name, a, b}); }

hipError_t ensure_lds_limit(const void* kern, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> done;  // (device, kernel) -> limit set
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(dev, kern);
  auto it = done.find(key);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  done[key] = bytes;
  return hipSuccess;
}

}  // namespace pdrt

namespace {

struct Problem {
  int Nu, Nv, Nk;
  double R, d0;
  int batch;
  Layout lay;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

const double kFwhmPerSigma = 2.0 * std::sqrt(2.0 * std::log(2.0));

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int validate(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec) {
  if (!grid || !beam || !spec) return PDRT_E_INVALID;
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return PDRT_E_INVALID;
  if ((double)grid->nx * grid->ny * grid->nz >= 2147483648.0) return PDRT_E_INVALID;  // 32-bit voxel offsets
  if (!finite_pos(grid->sx) || !finite_pos(grid->sy) || !finite_pos(grid->sz)) return PDRT_E_INVALID;
  if (!std::isfinite(grid->ox) || !std::isfinite(grid->oy) || !std::isfinite(grid->oz)) return PDRT_E_INVALID;
  if (!finite_pos(beam->sad_mm)) return PDRT_E_INVALID;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(beam->iso_mm[a])) return PDRT_E_INVALID;
  if (beam->n_leaf_pairs < 1 || beam->n_leaf_pairs > PDRT_MAX_LEAF_PAIRS || !beam->leaf_edges_mm)
    return PDRT_E_INVALID;
  for (int l = 0; l <= beam->n_leaf_pairs; ++l)
    if (!std::isfinite(beam->leaf_edges_mm[l])) return PDRT_E_INVALID;
  for (int l = 0; l < beam->n_leaf_pairs; ++l)
    if (!(beam->leaf_edges_mm[l + 1] > beam->leaf_edges_mm[l])) return PDRT_E_INVALID;
  if (beam->n_cp < 1 || !beam->gantry_deg) return PDRT_E_INVALID;
  if (!(beam->field_limit_mm[0] >= 0.0) || !(beam->field_limit_mm[1] >= 0.0)) return PDRT_E_INVALID;
  if (!std::isfinite(beam->field_limit_mm[0]) || !std::isfinite(beam->field_limit_mm[1])) return PDRT_E_INVALID;
  if (spec->n_taps < 1 || spec->n_taps > PDRT_MAX_TAPS || (spec->n_taps % 2) == 0) return PDRT_E_INVALID;
  if (spec->wepl_mode != PDRT_WEPL_PER_RAY && spec->wepl_mode != PDRT_WEPL_CENTRAL_AXIS) return PDRT_E_INVALID;
  if (spec->conv_mode != PDRT_CONV_FP32 && spec->conv_mode != PDRT_CONV_BF16) return PDRT_E_INVALID;
  if (!finite_pos(spec->lateral_step_mm) || !finite_pos(spec->depth_step_mm)) return PDRT_E_INVALID;
  if (!(spec->transmission >= 0.0 && spec->transmission <= 1.0)) return PDRT_E_INVALID;
  if (!std::isfinite(spec->calib)) return PDRT_E_INVALID;
  if (spec->n_dd < 2 || spec->n_dd > 8192 || !spec->dd || !finite_pos(spec->dd_step_mm)) return PDRT_E_INVALID;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      if (!std::isfinite(spec->kpoly[a][b])) return PDRT_E_INVALID;
  if (!(spec->kz_max_mm >= 0.0) || !std::isfinite(spec->kz_max_mm)) return PDRT_E_INVALID;
  if (spec->max_cp_batch < 0) return PDRT_E_INVALID;
  if (spec->march_scan != 0 && spec->march_scan != 1) return PDRT_E_INVALID;
  if (spec->fluence_corr != 0 && spec->fluence_corr != 1) return PDRT_E_INVALID;
  if (spec->fluence_corr) {
    const double sig[3] = {spec->pen_fwhm_mm[0] / kFwhmPerSigma, spec->pen_fwhm_mm[1] / kFwhmPerSigma,
                           spec->hs_sigma_mm};
    for (double x : sig)
      if (!(x >= 0.0) || !std::isfinite(x)) return PDRT_E_INVALID;
    if (!std::isfinite(spec->hs_amp) || !std::isfinite(spec->oar[0]) || !std::isfinite(spec->oar[1]))
      return PDRT_E_INVALID;
    for (double x : sig)
      if (std::ceil(3.0 * x / spec->lateral_step_mm - 1e-9) > PDRT_MAX_BLUR_RADIUS) return PDRT_E_UNSUPPORTED;
  }
  return PDRT_OK;
}

// Unit-sum Gaussian taps sampled at the fan pixel centres, truncated at 3 sigma
// (one tap of 1 for sigma = 0); computed in double, stored in T.
template <typename T>
void gauss_taps(double sigma, double D, BlurTaps<T>* t) {
  if (!(sigma > 0.0)) {
    t->R = 0;
    t->g[0] = T(1);
    return;
  }
  int R = (int)std::ceil(3.0 * sigma / D - 1e-9);
  double w[2 * PDRT_MAX_BLUR_RADIUS + 1], sum = 0.0;
  for (int m = -R; m <= R; ++m) sum += (w[m + R] = std::exp(-(m * D) * (m * D) / (2.0 * sigma * sigma)));
  t->R = R;
  for (int m = 0; m <= 2 * R; ++m) t->g[m] = (T)(w[m] / sum);
}

// Beam-frame grid (one reading of §2.2.3, stated with the oracle's): Nu = 2
// ceil((F_u + h Delta)/Delta) + 1 (and Nv likewise) keeps the kernel's reach past
// the field edge on the grid; planes span [SAD - R, SAD + R] with R the largest
// in-plane distance from the isocentre to a corner of the CT box, so every voxel
// of every gantry angle falls inside.
int size_problem(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec, int with_bwd,
                 int elem, Problem* P) {
  int st = validate(grid, beam, spec);
  if (st != PDRT_OK) return st;
  if (elem != 4 && elem != 8) return PDRT_E_INVALID;
  int h = (spec->n_taps - 1) / 2;
  double D = spec->lateral_step_mm;
  double nu = 2.0 * std::ceil((beam->field_limit_mm[0] + h * D) / D - 1e-9) + 1.0;
  double nv = 2.0 * std::ceil((beam->field_limit_mm[1] + h * D) / D - 1e-9) + 1.0;
  const bool rot = beam->collimator_deg != nullptr;
  if (rot) {
    // any rotation of a jaw rectangle inside the field limits stays within the
    // radius hypot(F_u, F_v) of the central axis
    const double F = std::hypot(beam->field_limit_mm[0], beam->field_limit_mm[1]);
    nu = nv = 2.0 * std::ceil((F + h * D) / D - 1e-9) + 1.0;
  }
  double xs[2] = {grid->ox - 0.5 * grid->sx, grid->ox + (grid->nx - 0.5) * grid->sx};
  double ys[2] = {grid->oy - 0.5 * grid->sy, grid->oy + (grid->ny - 0.5) * grid->sy};
  double R = 0.0;
  for (double x : xs)
    for (double y : ys) R = std::fmax(R, std::hypot(x - beam->iso_mm[0], y - beam->iso_mm[1]));
  double nk = std::ceil(2.0 * R / spec->depth_step_mm - 1e-9) + 1.0;
  if (nu > 4095 || nv > 4095 || nk > 65535) return PDRT_E_INVALID;
  if (!(R < beam->sad_mm)) return PDRT_E_INVALID;  // the source must lie outside the CT box
  P->Nu = (int)nu;
  P->Nv = (int)nv;
  P->Nk = (int)nk;
  P->R = R;
  P->d0 = beam->sad_mm - R;
  int B = beam->n_cp;
  if (spec->max_cp_batch > 0 && spec->max_cp_batch < B) B = spec->max_cp_batch;
  if (B > 65535) B = 65535;  // grid z limit of the per-plane kernels
  P->batch = B;
  size_t nvox = (size_t)grid->nx * grid->ny * grid->nz;
  size_t plane = (size_t)P->Nu * P->Nv;
  size_t off = 0;
  Layout& L = P->lay;
  L.batch = B;
  L.frame = off;
  off += align256((size_t)2 * beam->n_cp * elem);
  L.rho_t = off;
  off += align256(nvox * elem);
  L.fluence = off;
  off += align256((size_t)B * plane * elem);
  L.depth = off;
  off += align256((size_t)B * P->Nk * elem);
  L.vol0 = off;
  off += align256((size_t)B * P->Nk * plane * elem);
  // (vol1 directly follows vol0: the register-resident forward convolution, whose
  // input is vol0, may read a few words past a row's end, i.e. past vol0's end
  // after the last row, which stays inside the workspace)
  L.vol1 = off;
  off += align256((size_t)B * P->Nk * plane * elem);
  L.adj = off;
  if (with_bwd) off += align256((size_t)B * plane * elem);
  L.comp = off;
  off += align256(nvox * elem);
  L.fc_tmp = off;
  if (spec->fluence_corr) off += align256((size_t)2 * B * plane * elem);
  L.box = off;
  off += align256((size_t)4 * B * sizeof(int));
  L.cframe = off;
  if (rot) off += align256((size_t)2 * beam->n_cp * elem);
  L.rot = off;
  if (rot) off += align256((size_t)B * plane * elem);
  L.total = off;
  return PDRT_OK;
}

template <typename T>
void make_geo(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec, const Problem& P,
              Geo<T>* g) {
  std::memset((void*)g, 0, sizeof(Geo<T>));
  g->nx = grid->nx;
  g->ny = grid->ny;
  g->nz = grid->nz;
  g->sx = (T)grid->sx;
  g->sy = (T)grid->sy;
  g->sz = (T)grid->sz;
  g->inv_sx = (T)(1.0 / grid->sx);
  g->inv_sy = (T)(1.0 / grid->sy);
  g->inv_sz = (T)(1.0 / grid->sz);
  g->rel_ox = (T)(grid->ox - beam->iso_mm[0]);
  g->rel_oy = (T)(grid->oy - beam->iso_mm[1]);
  g->rel_oz = (T)(grid->oz - beam->iso_mm[2]);
  g->iso_ix = (T)((beam->iso_mm[0] - grid->ox) / grid->sx);
  g->iso_iy = (T)((beam->iso_mm[1] - grid->oy) / grid->sy);
  g->iso_iz = (T)((beam->iso_mm[2] - grid->oz) / grid->sz);
  g->Nu = P.Nu;
  g->Nv = P.Nv;
  g->Nk = P.Nk;
  g->cu = (T)(0.5 * (P.Nu - 1));
  g->cv = (T)(0.5 * (P.Nv - 1));
  g->lat = (T)spec->lateral_step_mm;
  g->inv_lat = (T)(1.0 / spec->lateral_step_mm);
  g->dstep = (T)spec->depth_step_mm;
  g->inv_dstep = (T)(1.0 / spec->depth_step_mm);
  g->e0 = (T)(-P.R);
  g->sad = (T)beam->sad_mm;
  g->inv_sad = (T)(1.0 / beam->sad_mm);
  g->n_taps = spec->n_taps;
  g->h = (spec->n_taps - 1) / 2;
  g->wepl_mode = spec->wepl_mode;
  g->tau = (T)spec->transmission;
  g->calib = (T)spec->calib;
  g->n_dd = spec->n_dd;
  g->inv_dd_step = (T)(1.0 / spec->dd_step_mm);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) g->kpoly[a][b] = (T)spec->kpoly[a][b];
  g->kz_max = (T)spec->kz_max_mm;
  g->L = beam->n_leaf_pairs;
  for (int l = 0; l <= beam->n_leaf_pairs; ++l) g->leaf_edges[l] = (T)beam->leaf_edges_mm[l];
  g->fcorr = spec->fluence_corr;
  g->hs_amp = (T)spec->hs_amp;
  g->oar0 = (T)spec->oar[0];
  g->oar1 = (T)spec->oar[1];
  g->march_scan = spec->march_scan;
}

// The three Gaussians of the fluence corrections: penumbra along u and v, head scatter.
template <typename T>
struct FcTaps {
  BlurTaps<T> pu, pv, hs;
};

template <typename T>
void make_fc_taps(const pdrt_kernel_spec* spec, FcTaps<T>* t) {
  const double D = spec->lateral_step_mm;
  gauss_taps<T>(spec->pen_fwhm_mm[0] / kFwhmPerSigma, D, &t->pu);
  gauss_taps<T>(spec->pen_fwhm_mm[1] / kFwhmPerSigma, D, &t->pv);
  gauss_taps<T>(spec->hs_sigma_mm, D, &t->hs);
}

#define CHECK_HIP(x)                    \
  do {                                  \
    if ((x) != hipSuccess) return PDRT_E_HIP; \
  } while (0)

#define LAUNCH(name, x) PDRT_TIMED(name, s, x)

// Smallest kernel taken by the FP32 matrix-core convolution: below it the Toeplitz
// operand is mostly padding (a 9-tap row fills 9 of 32 columns) and the vector-ALU
// convolutions are faster.
constexpr int kMfmaMinTaps = 13;

// box / support: the aperture rectangles of the batch and how the convolution may
// use them (CONV_IN_BOX forward, CONV_OUT_BOX adjoint); kernels without support
// handling compute the dense convolution, which is a superset.
template <typename T>
hipError_t run_conv(const Geo<T>& g, int conv_mode, int nb, const T* z, const T* in, T* out, hipStream_t s,
                    const int* box, int support);

template <>
hipError_t run_conv<double>(const Geo<double>& g, int, int nb, const double* z, const double* in, double* out,
                            hipStream_t s, const int*, int) {
  return launch_conv_direct<double>(g, nb, z, in, out, s);
}

template <>
hipError_t run_conv<float>(const Geo<float>& g, int conv_mode, int nb, const float* z, const float* in, float* out,
                           hipStream_t s, const int* box, int support) {
  if (conv_mode == PDRT_CONV_BF16) return launch_conv_mfma_bf16(g, nb, z, in, out, s, box, support);
  if (g.n_taps >= kMfmaMinTaps) return launch_conv_mfma_f32(g, nb, z, in, out, s, box, support);
  if (conv_small_supported(g)) return launch_conv_small(g, nb, z, in, out, s);
  return launch_conv_direct<float>(g, nb, z, in, out, s);
}

template <typename T>
const char* conv_name(const Geo<T>& g, int conv_mode, int adjoint);

template <>
const char* conv_name<double>(const Geo<double>&, int, int adjoint) {
  return adjoint ? "conv_direct_f64_adj" : "conv_direct_f64";
}

// The matrix-core convolutions honour the aperture box (inputs read, outputs
// written only inside it); the vector-ALU ones are dense.
template <typename T>
bool conv_uses_box(const Geo<T>& g, int conv_mode) {
  return sizeof(T) == 4 && (conv_mode == PDRT_CONV_BF16 || g.n_taps >= kMfmaMinTaps);
}

template <>
const char* conv_name<float>(const Geo<float>& g, int conv_mode, int adjoint) {
  if (conv_mode == PDRT_CONV_BF16) return adjoint ? "conv_mfma_bf16_adj" : "conv_mfma_bf16";
  if (g.n_taps >= kMfmaMinTaps) return adjoint ? "conv_mfma_f32_adj" : "conv_mfma_f32";
  if (conv_small_supported(g)) return adjoint ? "conv_small_f32_adj" : "conv_small_f32";
  return adjoint ? "conv_direct_f32_adj" : "conv_direct_f32";
}

// Plan-level geometry cache: z [n_cp][Nk] float at offset 0, then G [n_cp][Nk][Nu][Nv]
// as float or bf16 at a 256-byte aligned offset.
struct GeoCache {
  int type;
  const float* z;
  const void* G;
};

bool cache_offsets(const Problem& P, int n_cp, int type, size_t* g_off, size_t* total) {
  if (type != PDRT_CACHE_F32 && type != PDRT_CACHE_BF16) return false;
  const size_t e = type == PDRT_CACHE_F32 ? sizeof(float) : sizeof(__bf16);
  *g_off = align256((size_t)n_cp * P.Nk * sizeof(float));
  *total = *g_off + (size_t)n_cp * P.Nk * P.Nu * P.Nv * e;
  return true;
}

// The cache as seen by the forward / backward, after checking its size.
int cache_view(const Problem& P, const pdrt_beam* beam, int type, const void* cache, size_t cache_bytes,
               GeoCache* gc) {
  size_t g_off = 0, total = 0;
  if (!cache || !cache_offsets(P, beam->n_cp, type, &g_off, &total)) return PDRT_E_INVALID;
  if (cache_bytes < total) return PDRT_E_WORKSPACE;
  gc->type = type;
  gc->z = (const float*)cache;
  gc->G = (const char*)cache + g_off;
  return PDRT_OK;
}

template <typename E>
hipError_t apply_geometry(const Geo<float>& g, int nb, int cp0, const GeoCache& gc, const float* F, float* P,
                          hipStream_t s, const int* box) {
  const E* G = (const E*)gc.G + (size_t)cp0 * g.Nk * g.Nu * g.Nv;
  return launch_apply_geometry<E>(g, nb, F, G, P, s, box);
}

template <typename E>
hipError_t geometry_adjoint(const Geo<float>& g, int nb, int cp0, const GeoCache& gc, const float* H, float* A,
                            hipStream_t s, const int* box) {
  const E* G = (const E*)gc.G + (size_t)cp0 * g.Nk * g.Nu * g.Nv;
  return launch_geometry_adjoint<E>(g, nb, H, G, A, s, box);
}

// With gc == nullptr the march computes the geometry from rho; with a cache (FP32
// only) rho is not read and the march is replaced by the cached factor.
template <typename T>
int forward_impl(const pdrt_grid* grid, const T* rho, const pdrt_beam* beam, const T* leaves, const T* jaws,
                 const T* mu, const pdrt_kernel_spec* spec, T* dose, void* ws, size_t ws_bytes, void* stream,
                 const GeoCache* gc = nullptr) {
  Problem P;
  int st = size_problem(grid, beam, spec, 0, (int)sizeof(T), &P);
  if (st != PDRT_OK) return st;
  if ((!rho && !gc) || !leaves || !jaws || !mu || !dose) return PDRT_E_INVALID;
  if (!ws || ws_bytes < P.lay.total) return PDRT_E_WORKSPACE;
  if (sizeof(T) == 8 && spec->conv_mode != PDRT_CONV_FP32) return PDRT_E_UNSUPPORTED;
  Geo<T> g;
  make_geo<T>(grid, beam, spec, P, &g);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  T* frame = (T*)(w + P.lay.frame);
  T* rho_t = (T*)(w + P.lay.rho_t);
  T* F = (T*)(w + P.lay.fluence);
  T* z = (T*)(w + P.lay.depth);
  T* vol0 = (T*)(w + P.lay.vol0);
  T* vol1 = (T*)(w + P.lay.vol1);
  T* comp = (T*)(w + P.lay.comp);
  T* t0 = (T*)(w + P.lay.fc_tmp);
  T* t1 = t0 + (size_t)P.batch * P.Nu * P.Nv;
  FcTaps<T> fct;
  if (g.fcorr) make_fc_taps<T>(spec, &fct);
  int* box = (int*)(w + P.lay.box);
  // collimator rotation: F holds the collimator-frame map, Fb the beam-frame one
  const bool rot = beam->collimator_deg != nullptr;
  T* cframe = (T*)(w + P.lay.cframe);
  T* Fb = rot ? (T*)(w + P.lay.rot) : F;
  // the corrections spread the aperture's fluence by their blur radii
  const int box_du = g.fcorr ? fct.pu.R + fct.hs.R : 0, box_dv = g.fcorr ? fct.pv.R + fct.hs.R : 0;
  // rays outside the box are skipped only when the convolution reads just the box
  const int* ray_box = conv_uses_box<T>(g, spec->conv_mode) ? box : nullptr;
  const T* dd = (const T*)spec->dd;
  const int L = beam->n_leaf_pairs, n_cp = beam->n_cp;
  LAUNCH("frame", launch_frame<T>(g, (const T*)beam->gantry_deg, n_cp, frame, s));
  if (rot) LAUNCH("frame", launch_frame<T>(g, (const T*)beam->collimator_deg, n_cp, cframe, s));
  if (!gc) LAUNCH("transpose_rho", launch_transpose_rho<T>(g, rho, rho_t, s));
  for (int cp0 = 0; cp0 < n_cp; cp0 += P.batch) {
    int nb = n_cp - cp0 < P.batch ? n_cp - cp0 : P.batch;
    const T* fr = frame + 2 * cp0;
    LAUNCH("raster", launch_raster<T>(g, nb, leaves + (size_t)2 * L * cp0, jaws + (size_t)4 * cp0, F, s));
    LAUNCH("aperture_box", launch_aperture_box<T>(g, nb, jaws + (size_t)4 * cp0, box_du, box_dv, box, s));
    if (g.fcorr) {
      // F1 = G_v G_u F; F <- O (F1 + a G_hv G_hu F1)
      LAUNCH("fluence_corr", launch_blur<T>(g, nb, 0, fct.pu, F, t0, s));
      LAUNCH("fluence_corr", launch_blur<T>(g, nb, 1, fct.pv, t0, t1, s));
      LAUNCH("fluence_corr", launch_blur<T>(g, nb, 0, fct.hs, t1, t0, s));
      LAUNCH("fluence_corr", launch_blur<T>(g, nb, 1, fct.hs, t0, F, s));
      LAUNCH("fluence_corr", launch_fcorr_combine<T>(g, nb, g.hs_amp, 1, t1, F, F, s));
    }
    if (rot) {
      LAUNCH("collimator", launch_rotate<T>(g, nb, cframe + 2 * cp0, F, Fb, 0, s));
      LAUNCH("collimator", launch_collimator_box<T>(g, nb, cframe + 2 * cp0, box, s));
    }
    const T* zb = z;
    if constexpr (std::is_same<T, float>::value) {
      if (gc) {
        zb = gc->z + (size_t)cp0 * g.Nk;
        LAUNCH("apply_geometry", gc->type == PDRT_CACHE_F32
                                     ? apply_geometry<float>(g, nb, cp0, *gc, Fb, vol0, s, ray_box)
                                     : apply_geometry<__bf16>(g, nb, cp0, *gc, Fb, vol0, s, ray_box));
      }
    }
    if (!gc) {
      LAUNCH("ca_depth", launch_ca_depth<T>(g, nb, fr, rho_t, z, s));
      LAUNCH("march", launch_march<T>(g, nb, fr, rho_t, Fb, z, dd, vol0, s, ray_box));
    }
    LAUNCH(conv_name<T>(g, spec->conv_mode, 0),
           run_conv<T>(g, spec->conv_mode, nb, zb, vol0, vol1, s, box, CONV_IN_BOX));
    LAUNCH("gather", launch_gather<T>(g, nb, cp0 == 0, cp0 + nb == n_cp, fr, mu + cp0, vol1, dose, comp, s));
  }
  return PDRT_OK;
}

template <typename T>
int backward_impl(const pdrt_grid* grid, const T* rho, const pdrt_beam* beam, const T* leaves, const T* jaws,
                  const T* mu, const pdrt_kernel_spec* spec, const T* grad, T* gleaves, T* gjaws, T* gmu, void* ws,
                  size_t ws_bytes, void* stream, const GeoCache* gc = nullptr) {
  Problem P;
  int st = size_problem(grid, beam, spec, 1, (int)sizeof(T), &P);
  if (st != PDRT_OK) return st;
  if ((!rho && !gc) || !leaves || !jaws || !mu || !grad || !gleaves || !gjaws || !gmu) return PDRT_E_INVALID;
  if (!ws || ws_bytes < P.lay.total) return PDRT_E_WORKSPACE;
  Geo<T> g;
  make_geo<T>(grid, beam, spec, P, &g);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  T* frame = (T*)(w + P.lay.frame);
  T* rho_t = (T*)(w + P.lay.rho_t);
  T* z = (T*)(w + P.lay.depth);
  T* vol0 = (T*)(w + P.lay.vol0);
  T* vol1 = (T*)(w + P.lay.vol1);
  T* A = (T*)(w + P.lay.adj);
  T* g_t = (T*)(w + P.lay.comp);  // dose gradient, z fastest
  T* t0 = (T*)(w + P.lay.fc_tmp);
  T* t1 = t0 + (size_t)P.batch * P.Nu * P.Nv;
  FcTaps<T> fct;
  if (g.fcorr) make_fc_taps<T>(spec, &fct);
  int* box = (int*)(w + P.lay.box);
  // collimator rotation: the march's adjoint gives dL/d(beam-frame map) in Ab, its
  // transpose through the rotation the collimator-frame A the rest reads
  const bool rot = beam->collimator_deg != nullptr;
  T* cframe = (T*)(w + P.lay.cframe);
  T* Ab = rot ? (T*)(w + P.lay.rot) : A;
  // the parameter gradients read A inside the aperture rectangle; the corrections'
  // adjoint gathers it from as far as their blur radii
  const int box_du = g.fcorr ? fct.pu.R + fct.hs.R : 0, box_dv = g.fcorr ? fct.pv.R + fct.hs.R : 0;
  // with a box-restricted convolution H is valid only inside the box
  const int* ray_box = conv_uses_box<T>(g, spec->conv_mode) ? box : nullptr;
  const T* dd = (const T*)spec->dd;
  const int L = beam->n_leaf_pairs, n_cp = beam->n_cp;
  LAUNCH("frame", launch_frame<T>(g, (const T*)beam->gantry_deg, n_cp, frame, s));
  if (rot) LAUNCH("frame", launch_frame<T>(g, (const T*)beam->collimator_deg, n_cp, cframe, s));
  if (!gc) LAUNCH("transpose_rho", launch_transpose_rho<T>(g, rho, rho_t, s));
  LAUNCH("transpose_grad", launch_transpose_rho<T>(g, grad, g_t, s));
  for (int cp0 = 0; cp0 < n_cp; cp0 += P.batch) {
    int nb = n_cp - cp0 < P.batch ? n_cp - cp0 : P.batch;
    const T* fr = frame + 2 * cp0;
    const T* zb = z;
    if constexpr (std::is_same<T, float>::value) {
      if (gc) zb = gc->z + (size_t)cp0 * g.Nk;
    }
    if (!gc) LAUNCH("ca_depth", launch_ca_depth<T>(g, nb, fr, rho_t, z, s));
    LAUNCH("aperture_box", launch_aperture_box<T>(g, nb, jaws + (size_t)4 * cp0, box_du, box_dv, box, s));
    if (rot) LAUNCH("collimator", launch_collimator_box<T>(g, nb, cframe + 2 * cp0, box, s));
    LAUNCH("backproject_adj", launch_backproject_adj<T>(g, nb, fr, g_t, vol0, s));
    LAUNCH(conv_name<T>(g, spec->conv_mode, 1),
           run_conv<T>(g, spec->conv_mode, nb, zb, vol0, vol1, s, box, CONV_OUT_BOX));
    if constexpr (std::is_same<T, float>::value) {
      if (gc)
        LAUNCH("geometry_adjoint", gc->type == PDRT_CACHE_F32
                                       ? geometry_adjoint<float>(g, nb, cp0, *gc, vol1, Ab, s, ray_box)
                                       : geometry_adjoint<__bf16>(g, nb, cp0, *gc, vol1, Ab, s, ray_box));
    }
    if (!gc) LAUNCH("march_adj", launch_march_adj<T>(g, nb, fr, rho_t, z, dd, vol1, Ab, s, ray_box));
    if (rot) LAUNCH("collimator", launch_rotate<T>(g, nb, cframe + 2 * cp0, Ab, A, 1, s));
    if (g.fcorr) {
      // A <- G_u G_v (X + a G_hu G_hv X), X = O A: the corrections' adjoint, so that
      // the parameter gradients see dL/d(aperture fluence)
      LAUNCH("fluence_corr_adj", launch_fcorr_combine<T>(g, nb, T(0), 1, A, A, t0, s));
      LAUNCH("fluence_corr_adj", launch_blur<T>(g, nb, 1, fct.hs, t0, t1, s));
      LAUNCH("fluence_corr_adj", launch_blur<T>(g, nb, 0, fct.hs, t1, A, s));
      LAUNCH("fluence_corr_adj", launch_fcorr_combine<T>(g, nb, g.hs_amp, 0, t0, A, t1, s));
      LAUNCH("fluence_corr_adj", launch_blur<T>(g, nb, 1, fct.pv, t1, t0, s));
      LAUNCH("fluence_corr_adj", launch_blur<T>(g, nb, 0, fct.pu, t0, A, s));
    }
    LAUNCH("param_grad", launch_param_grad<T>(g, nb, leaves + (size_t)2 * L * cp0, jaws + (size_t)4 * cp0, mu + cp0, A,
                                   gleaves + (size_t)2 * L * cp0, gjaws + (size_t)4 * cp0, gmu + cp0, s));
  }
  return PDRT_OK;
}

bool valid_limits(const pdrt_limits* lim) {
  return lim && std::isfinite(lim->leaf_limit_mm) && lim->leaf_limit_mm >= 0 && std::isfinite(lim->jaw_limit_x_mm) &&
         lim->jaw_limit_x_mm >= 0 && std::isfinite(lim->jaw_limit_y_mm) && lim->jaw_limit_y_mm >= 0 &&
         std::isfinite(lim->w_min_mm) && lim->w_min_mm >= 0 && std::isfinite(lim->mu_min);
}

// ------------------------------------------------------------------ allocation-free forward
// Device memory of pdrt_dose_forward_noalloc: one copy per device, held from the
// library's first use on that device until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it names a stand-in, not the
// device copy): it looks up each device's address once and uses that.
static __device__ __align__(256) unsigned char scratch[PDRT_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of that device's scratch

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PDRT_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PDRT_E_HIP;
    it = g_scratch_addr.emplace(dev, p).first;
  }
  *out = it->second;
  return PDRT_OK;
}

}  // namespace

extern "C" {

int pdrt_fan_dims(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec, int32_t dims[3],
                  double* d0_mm) {
  if (!dims || !d0_mm) return PDRT_E_INVALID;
  Problem P;
  int st = size_problem(grid, beam, spec, 0, 4, &P);
  if (st != PDRT_OK) return st;
  dims[0] = P.Nu;
  dims[1] = P.Nv;
  dims[2] = P.Nk;
  *d0_mm = P.d0;
  return PDRT_OK;
}

size_t pdrt_workspace_bytes(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                            int32_t with_backward, int32_t elem_bytes) {
  Problem P;
  if (size_problem(grid, beam, spec, with_backward != 0, elem_bytes, &P) != PDRT_OK) return 0;
  return P.lay.total;
}

int pdrt_workspace_layout(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                          int32_t with_backward, int32_t elem_bytes, pdrt_ws_layout* out) {
  if (!out) return PDRT_E_INVALID;
  Problem P;
  int st = size_problem(grid, beam, spec, with_backward != 0, elem_bytes, &P);
  if (st != PDRT_OK) return st;
  out->frame = P.lay.frame;
  out->rho_t = P.lay.rho_t;
  out->fluence = P.lay.fluence;
  out->depth = P.lay.depth;
  out->vol0 = P.lay.vol0;
  out->vol1 = P.lay.vol1;
  out->adj = P.lay.adj;
  out->comp = P.lay.comp;
  out->fc_tmp = P.lay.fc_tmp;
  out->box = P.lay.box;
  out->cframe = P.lay.cframe;
  out->rot = P.lay.rot;
  out->total = P.lay.total;
  out->batch = P.batch;
  return PDRT_OK;
}

int pdrt_hu_to_density(const pdrt_grid* grid, const float* hu, float* rho, int32_t n_pts, const double* hu_pts,
                       const double* rho_pts, void* stream) {
  if (!grid || !hu || !rho || !hu_pts || !rho_pts) return PDRT_E_INVALID;
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return PDRT_E_INVALID;
  if (n_pts < 2 || n_pts > 16) return PDRT_E_INVALID;
  float hp[16], rp[16];
  for (int i = 0; i < n_pts; ++i) {
    if (!std::isfinite(hu_pts[i]) || !std::isfinite(rho_pts[i])) return PDRT_E_INVALID;
    if (i > 0 && !(hu_pts[i] > hu_pts[i - 1])) return PDRT_E_INVALID;
    hp[i] = (float)hu_pts[i];
    rp[i] = (float)rho_pts[i];
  }
  long n = (long)grid->nx * grid->ny * grid->nz;
  CHECK_HIP(launch_hu_to_density(n, hu, rho, n_pts, hp, rp, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_dose_forward(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam, const float* leaves,
                      const float* jaws, const float* mu, const pdrt_kernel_spec* spec, float* dose, void* ws,
                      size_t ws_bytes, void* stream) {
  return forward_impl<float>(grid, rho, beam, leaves, jaws, mu, spec, dose, ws, ws_bytes, stream);
}

int pdrt_dose_backward(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam, const float* leaves,
                       const float* jaws, const float* mu, const pdrt_kernel_spec* spec, const float* grad_dose,
                       float* grad_leaves, float* grad_jaws, float* grad_mu, void* ws, size_t ws_bytes,
                       void* stream) {
  return backward_impl<float>(grid, rho, beam, leaves, jaws, mu, spec, grad_dose, grad_leaves, grad_jaws, grad_mu,
                              ws, ws_bytes, stream);
}

int pdrt_dose_forward_noalloc(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam, const float* leaves,
                              const float* jaws, const float* mu, const pdrt_kernel_spec* spec, float* dose,
                              void* stream) {
  if (!grid || !beam || !spec || !rho || !leaves || !jaws || !mu || !dose) return PDRT_E_INVALID;
  // the largest control-point batch whose forward workspace fits the scratch
  pdrt_kernel_spec sp = *spec;
  Problem P;
  sp.max_cp_batch = 1;
  int st = size_problem(grid, beam, &sp, 0, 4, &P);
  if (st != PDRT_OK) return st;
  if (P.lay.total > (size_t)PDRT_NOALLOC_SCRATCH_BYTES) return PDRT_E_SCRATCH;
  int lo = 1, hi = (spec->max_cp_batch > 0 && spec->max_cp_batch < beam->n_cp) ? spec->max_cp_batch : beam->n_cp;
  while (lo < hi) {
    int mid = lo + (hi - lo + 1) / 2;
    sp.max_cp_batch = mid;
    if (size_problem(grid, beam, &sp, 0, 4, &P) == PDRT_OK && P.lay.total <= (size_t)PDRT_NOALLOC_SCRATCH_BYTES)
      lo = mid;
    else
      hi = mid - 1;
  }
  sp.max_cp_batch = lo;
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != PDRT_OK) return st;
  return forward_impl<float>(grid, rho, beam, leaves, jaws, mu, &sp, dose, ws, (size_t)PDRT_NOALLOC_SCRATCH_BYTES,
                             stream);
}

int pdrt_dose_forward_f64(const pdrt_grid* grid, const double* rho, const pdrt_beam* beam, const double* leaves,
                          const double* jaws, const double* mu, const pdrt_kernel_spec* spec, double* dose, void* ws,
                          size_t ws_bytes, void* stream) {
  return forward_impl<double>(grid, rho, beam, leaves, jaws, mu, spec, dose, ws, ws_bytes, stream);
}

size_t pdrt_geometry_cache_bytes(const pdrt_grid* grid, const pdrt_beam* beam, const pdrt_kernel_spec* spec,
                                 int32_t cache_type) {
  Problem P;
  if (size_problem(grid, beam, spec, 0, 4, &P) != PDRT_OK) return 0;
  size_t g_off = 0, total = 0;
  if (!cache_offsets(P, beam->n_cp, cache_type, &g_off, &total)) return 0;
  return total;
}

int pdrt_geometry_cache_build(const pdrt_grid* grid, const float* rho, const pdrt_beam* beam,
                              const pdrt_kernel_spec* spec, int32_t cache_type, void* cache, size_t cache_bytes,
                              void* ws, size_t ws_bytes, void* stream) {
  Problem P;
  int st = size_problem(grid, beam, spec, 0, 4, &P);
  if (st != PDRT_OK) return st;
  if (!rho) return PDRT_E_INVALID;
  GeoCache gc;
  st = cache_view(P, beam, cache_type, cache, cache_bytes, &gc);
  if (st != PDRT_OK) return st;
  if (!ws || ws_bytes < P.lay.total) return PDRT_E_WORKSPACE;
  Geo<float> g;
  make_geo<float>(grid, beam, spec, P, &g);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  float* frame = (float*)(w + P.lay.frame);
  float* rho_t = (float*)(w + P.lay.rho_t);
  float* z = (float*)cache;
  const float* dd = (const float*)spec->dd;
  const int n_cp = beam->n_cp;
  const size_t node = (size_t)g.Nk * g.Nu * g.Nv;
  LAUNCH("frame", launch_frame<float>(g, (const float*)beam->gantry_deg, n_cp, frame, s));
  LAUNCH("transpose_rho", launch_transpose_rho<float>(g, rho, rho_t, s));
  LAUNCH("ca_depth", launch_ca_depth<float>(g, n_cp, frame, rho_t, z, s));
  for (int cp0 = 0; cp0 < n_cp; cp0 += P.batch) {
    const int nb = n_cp - cp0 < P.batch ? n_cp - cp0 : P.batch;
    const float* fr = frame + 2 * cp0;
    const float* zb = z + (size_t)cp0 * g.Nk;
    if (cache_type == PDRT_CACHE_F32)
      LAUNCH("march_geometry", launch_march_geometry<float>(g, nb, fr, rho_t, zb, dd,
                                                            (float*)gc.G + (size_t)cp0 * node, s));
    else
      LAUNCH("march_geometry", launch_march_geometry<__bf16>(g, nb, fr, rho_t, zb, dd,
                                                             (__bf16*)gc.G + (size_t)cp0 * node, s));
  }
  return PDRT_OK;
}

int pdrt_dose_forward_cached(const pdrt_grid* grid, const pdrt_beam* beam, const float* leaves, const float* jaws,
                             const float* mu, const pdrt_kernel_spec* spec, int32_t cache_type, const void* cache,
                             size_t cache_bytes, float* dose, void* ws, size_t ws_bytes, void* stream) {
  Problem P;
  int st = size_problem(grid, beam, spec, 0, 4, &P);
  if (st != PDRT_OK) return st;
  GeoCache gc;
  st = cache_view(P, beam, cache_type, cache, cache_bytes, &gc);
  if (st != PDRT_OK) return st;
  return forward_impl<float>(grid, nullptr, beam, leaves, jaws, mu, spec, dose, ws, ws_bytes, stream, &gc);
}

int pdrt_dose_backward_cached(const pdrt_grid* grid, const pdrt_beam* beam, const float* leaves, const float* jaws,
                              const float* mu, const pdrt_kernel_spec* spec, int32_t cache_type, const void* cache,
                              size_t cache_bytes, const float* grad_dose, float* grad_leaves, float* grad_jaws,
                              float* grad_mu, void* ws, size_t ws_bytes, void* stream) {
  Problem P;
  int st = size_problem(grid, beam, spec, 1, 4, &P);
  if (st != PDRT_OK) return st;
  GeoCache gc;
  st = cache_view(P, beam, cache_type, cache, cache_bytes, &gc);
  if (st != PDRT_OK) return st;
  return backward_impl<float>(grid, nullptr, beam, leaves, jaws, mu, spec, grad_dose, grad_leaves, grad_jaws,
                              grad_mu, ws, ws_bytes, stream, &gc);
}

int pdrt_project_params(int32_t n_cp, int32_t n_leaf_pairs, const float* leaves_in, const float* jaws_in,
                        const float* mu_in, const pdrt_limits* limits, float* leaves_out, float* jaws_out,
                        float* mu_out, void* stream) {
  if (n_cp < 1 || n_leaf_pairs < 1 || n_leaf_pairs > PDRT_MAX_LEAF_PAIRS) return PDRT_E_INVALID;
  if (!leaves_in || !jaws_in || !mu_in || !leaves_out || !jaws_out || !mu_out || !valid_limits(limits))
    return PDRT_E_INVALID;
  CHECK_HIP(launch_project(n_cp, n_leaf_pairs, leaves_in, jaws_in, mu_in, limits->leaf_limit_mm,
                           limits->jaw_limit_x_mm, limits->jaw_limit_y_mm, limits->w_min_mm, limits->mu_min,
                           leaves_out, jaws_out, mu_out, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_project_params_backward(int32_t n_cp, int32_t n_leaf_pairs, const float* leaves_in, const float* jaws_in,
                                 const float* mu_in, const pdrt_limits* limits, int32_t straight_through,
                                 const float* g_leaves, const float* g_jaws, const float* g_mu, float* gi_leaves,
                                 float* gi_jaws, float* gi_mu, void* stream) {
  if (n_cp < 1 || n_leaf_pairs < 1 || n_leaf_pairs > PDRT_MAX_LEAF_PAIRS) return PDRT_E_INVALID;
  if (!leaves_in || !jaws_in || !mu_in || !g_leaves || !g_jaws || !g_mu || !gi_leaves || !gi_jaws || !gi_mu ||
      !valid_limits(limits))
    return PDRT_E_INVALID;
  CHECK_HIP(launch_project_bwd(n_cp, n_leaf_pairs, leaves_in, jaws_in, mu_in, limits->leaf_limit_mm,
                               limits->jaw_limit_x_mm, limits->jaw_limit_y_mm, limits->w_min_mm, limits->mu_min,
                               straight_through != 0, g_leaves, g_jaws, g_mu, gi_leaves, gi_jaws, gi_mu,
                               (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_profile_begin(int32_t max_launches) {
  if (max_launches < 1) return PDRT_E_INVALID;
  auto& P = pdrt::prof();
  size_t need = 2 * (size_t)max_launches;
  while (P.pool.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return PDRT_E_HIP;
    P.pool.push_back(e);
  }
  P.used = 0;
  P.recs.clear();
  P.overflow = false;
  P.on = true;
  return PDRT_OK;
}

int pdrt_profile_end(pdrt_kernel_time* out, int32_t max_entries, int32_t* n_entries) {
  auto& P = pdrt::prof();
  if (!P.on) return PDRT_E_INVALID;
  P.on = false;
  if (!out || !n_entries || max_entries < 1) return PDRT_E_INVALID;
  int n = 0;
  for (const auto& r : P.recs) {
    if (hipEventSynchronize(P.pool[r.b]) != hipSuccess) return PDRT_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.pool[r.a], P.pool[r.b]) != hipSuccess) return PDRT_E_HIP;
    int q = 0;
    while (q < n && std::strcmp(out[q].name, r.name) != 0) ++q;
    if (q == n) {
      if (n == max_entries) continue;
      std::memset(&out[q], 0, sizeof(pdrt_kernel_time));
      std::strncpy(out[q].name, r.name, sizeof(out[q].name) - 1);
      ++n;
    }
    out[q].launches += 1;
    out[q].total_ms += ms;
  }
  *n_entries = n;
  return P.overflow ? PDRT_E_WORKSPACE : PDRT_OK;
}

const char* pdrt_status_string(int status) {
  switch (status) {
    case PDRT_OK: return "ok";
    case PDRT_E_INVALID: return "invalid argument";
    case PDRT_E_WORKSPACE: return "workspace missing or too small";
    case PDRT_E_HIP: return "HIP launch or runtime error";
    case PDRT_E_UNSUPPORTED: return "unsupported request";
    case PDRT_E_SCRATCH: return "problem too large for the allocation-free entry point's scratch";
    default: return "unknown status";
  }
}

int pdrt_version(void) { return 100; }

}  // extern "C"
