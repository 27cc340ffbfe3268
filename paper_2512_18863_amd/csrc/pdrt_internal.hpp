// pdrt_internal.hpp — shared definitions of the HIP dose library (not part of the ABI).
//
// Fan-grid ("beam frame") storage is [cp][Nk][Nu][Nv] with v (the leaf-stacking
// axis, parallel to patient z) fastest.  Because v is always patient z
// (collimator 0), consecutive v along a ray plane map to consecutive z in the CT,
// and the density copy the ray march reads is stored z-fastest ([ny][nx][nz]):
// lanes that walk along v then load neighbouring words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pdrt.h"

namespace pdrt {

// Geometry and model constants, passed to kernels by value.  Everything is
// stored relative to the isocentre so that FP32 never handles the 1000 mm source
// distance directly.
template <typename T>
struct Geo {
  // CT grid
  int nx, ny, nz;
  T sx, sy, sz;
  T inv_sx, inv_sy, inv_sz;
  T rel_ox, rel_oy, rel_oz;  // centre of voxel (0,0,0) minus the isocentre
  T iso_ix, iso_iy, iso_iz;  // continuous voxel index of the isocentre
  // beam frame
  int Nu, Nv, Nk;
  T cu, cv;           // (N - 1) / 2
  T lat, inv_lat;     // ray spacing at the isocentre plane
  T dstep, inv_dstep; // plane spacing along the central axis
  T e0;               // first plane distance minus SAD (= -R)
  T sad, inv_sad;
  // model
  int n_taps, h;
  int wepl_mode;
  T tau, calib;
  int n_dd;
  T inv_dd_step;
  T kpoly[4][4];
  T kz_max;
  int L;
  T leaf_edges[PDRT_MAX_LEAF_PAIRS + 1];
  // fluence corrections (off when fcorr == 0); the blur taps travel separately
  int fcorr;
  T hs_amp, oar0, oar1;
  // ray march: 0 = one thread per ray (serial), 1 = segmented scan across wavefronts
  int march_scan;
};

// Unit-sum taps of one Gaussian blur, radius R <= PDRT_MAX_BLUR_RADIUS.
template <typename T>
struct BlurTaps {
  int R;
  T g[2 * PDRT_MAX_BLUR_RADIUS + 1];
};

// Workspace layout (byte offsets) plus sizes, computed on the host.
struct Layout {
  size_t frame, rho_t, fluence, depth, vol0, vol1, adj, comp, fc_tmp, box, cframe, rot, total;
  int batch;
};

// The scan form of the ray march splits the Nk planes of a ray into segments
// scanned by separate wavefronts (segment w = planes [Nk w / n, Nk (w + 1) / n) of
// n = march_segments segments); its adjoint sums each segment in plane order and
// adds the segments' sums in segment order (the serial form: one segment).  The
// cached geometry adjoint follows the same order so that both give the same bits.
constexpr int kMarchSeg = 32;  // planes per segment and sampling pass
constexpr int kMarchMaxSegments = 8;
__host__ __device__ inline int march_segments(int Nk) {
  const int n = (Nk + kMarchSeg - 1) / kMarchSeg;
  return n < 1 ? 1 : (n > kMarchMaxSegments ? kMarchMaxSegments : n);
}

// Raises a kernel's dynamic-LDS limit to at least `bytes` on the current device.
// Each (device, kernel) pair is set once, or again when a larger limit is asked
// for; safe to call from several host threads.  Defined in api.hip.
hipError_t ensure_lds_limit(const void* kern, int bytes);

// --- launchers (defined in the kernel translation units) -------------------
template <typename T>
hipError_t launch_frame(const Geo<T>& g, const T* gantry_deg, int n_cp, T* frame, hipStream_t s);
hipError_t launch_hu_to_density(long n, const float* hu, float* rho, int n_pts, const float* hp, const float* rp,
                                hipStream_t s);
template <typename T>
hipError_t launch_transpose_rho(const Geo<T>& g, const T* rho, T* rho_t, hipStream_t s);
template <typename T>
hipError_t launch_raster(const Geo<T>& g, int nb, const T* leaves, const T* jaws, T* F, hipStream_t s);
template <typename T>
hipError_t launch_ca_depth(const Geo<T>& g, int nb, const T* frame, const T* rho_t, T* z, hipStream_t s);
template <typename T>
hipError_t launch_march(const Geo<T>& g, int nb, const T* frame, const T* rho_t, const T* F, const T* z,
                        const T* dd, T* P, hipStream_t s, const int* box = nullptr);
template <typename T>
hipError_t launch_march_adj(const Geo<T>& g, int nb, const T* frame, const T* rho_t, const T* z, const T* dd,
                            const T* H, T* A, hipStream_t s, const int* box = nullptr);
// Support of a lateral convolution: box[b] = {u0, u1, v0, v1} (int4 per control
// point) bounds the aperture; CONV_IN_BOX: inputs outside it are zero; CONV_OUT_BOX:
// only outputs inside it are needed (the rest are written as 0).
enum { CONV_DENSE = 0, CONV_IN_BOX = 1, CONV_OUT_BOX = 2 };
template <typename T>
hipError_t launch_aperture_box(const Geo<T>& g, int nb, const T* jaws, int du, int dv, int* box, hipStream_t s);
// Collimator rotation of the fluence maps (adjoint != 0: its transpose) and of the
// aperture rectangles; cframe = (sin, cos) of each control point's collimator angle.
template <typename T>
hipError_t launch_rotate(const Geo<T>& g, int nb, const T* cframe, const T* in, T* out, int adjoint, hipStream_t s);
template <typename T>
hipError_t launch_collimator_box(const Geo<T>& g, int nb, const T* cframe, int* box, hipStream_t s);

// Plan-level geometry cache: G = (SAD/d)^2 DD(W) per beam-frame node (E = float or
// __bf16), P = F G, and A = sum_k H_k G_k.
template <typename E>
hipError_t launch_march_geometry(const Geo<float>& g, int nb, const float* frame, const float* rho_t, const float* z,
                                 const float* dd, E* G, hipStream_t s);
template <typename E>
hipError_t launch_apply_geometry(const Geo<float>& g, int nb, const float* F, const E* G, float* P, hipStream_t s,
                                 const int* box = nullptr);
template <typename E>
hipError_t launch_geometry_adjoint(const Geo<float>& g, int nb, const float* H, const E* G, float* A,
                                   hipStream_t s, const int* box = nullptr);
template <typename T>
hipError_t launch_conv_direct(const Geo<T>& g, int nb, const T* z, const T* in, T* out, hipStream_t s);
// Small kernels (odd n <= 11) whose plane band fits the LDS budget.
bool conv_small_supported(const Geo<float>& g);
hipError_t launch_conv_small(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                             hipStream_t s);
hipError_t launch_conv_mfma_f32(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                hipStream_t s, const int* box = nullptr, int support = 0);
// forward convolution with the aperture rectangle in registers (FP32 or BF16
// operands, h <= 31)
bool conv_fwd_reg_supported(const Geo<float>& g, bool bf16);
hipError_t launch_conv_fwd_reg(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                               hipStream_t s, const int* box, bool bf16);
hipError_t launch_conv_mfma_bf16(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                 hipStream_t s, const int* box = nullptr, int support = 0);
template <typename T>
hipError_t launch_gather(const Geo<T>& g, int nb, int first, int last, const T* frame, const T* mu,
                         const T* Dfan, T* dose, T* comp, hipStream_t s);
template <typename T>
hipError_t launch_blur(const Geo<T>& g, int nb, int axis, const BlurTaps<T>& t, const T* in, T* out, hipStream_t s);
template <typename T>
hipError_t launch_fcorr_combine(const Geo<T>& g, int nb, T a, int use_oar, const T* x, const T* y, T* out,
                                hipStream_t s);
template <typename T>
hipError_t launch_backproject_adj(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s);
template <typename T>
hipError_t launch_param_grad(const Geo<T>& g, int nb, const T* leaves, const T* jaws, const T* mu, const T* A,
                             T* gleaves, T* gjaws, T* gmu, hipStream_t s);
hipError_t launch_project(int n_cp, int L, const float* lv, const float* jw, const float* mu, double leaf_lim,
                          double jx_lim, double jy_lim, double w_min, double mu_min, float* lo, float* jo,
                          float* mo, hipStream_t s);
hipError_t launch_project_bwd(int n_cp, int L, const float* lv, const float* jw, const float* mu, double leaf_lim,
                              double jx_lim, double jy_lim, double w_min, double mu_min, int ste,
                              const float* gl, const float* gj, const float* gm, float* ol, float* oj, float* om,
                              hipStream_t s);

// --- network primitives (net.hip) -------------------------------------------
struct Vol {
  int D, H, W;
};
hipError_t launch_conv3d_fwd(Vol v, int C1, int C2, const __bf16* X1, const __bf16* X2, int Cout, const __bf16* Wt,
                             int Kp, const float* bias, int relu, __bf16* Y, hipStream_t s);
hipError_t launch_conv3d_dgrad(Vol v, int Cout, const __bf16* dY, const __bf16* Yact, int Cin, const __bf16* Wd,
                               int Kp, int C1, __bf16* dX1, __bf16* dX2, hipStream_t s);
hipError_t launch_conv3d_wgrad(Vol v, int C1, int C2, const __bf16* X1, const __bf16* X2, int Cout, const __bf16* dY,
                               const __bf16* Yact, int nsplit, float* part, float* dW, float* db, hipStream_t s);
hipError_t launch_prep_weights(int Cout, int Cin, int Kpf, int Kpd, const float* W, __bf16* Wt, __bf16* Wd,
                               hipStream_t s);
hipError_t launch_net_input(int P, const float* dose, const float* scale, const float* rho, __bf16* X, hipStream_t s);
hipError_t launch_pool2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s);
hipError_t launch_up2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s);
hipError_t launch_head(int P, int C, const __bf16* X, const float* hw, const float* hb, const float* dose,
                       const float* scale, float* pred, float* resid, hipStream_t s);
hipError_t launch_head_bwd(int P, int C, const __bf16* X, const float* hw, const float* gp, const float* gr,
                           __bf16* dX, float* part, hipStream_t s);
hipError_t launch_train_loss(int P, const float* pred, const float* resid, const float* target, const float* tscale,
                             const float* mask, float inv_count, float lam, float tau, float* gp, float* gr,
                             float* part, hipStream_t s);
hipError_t launch_reduce_splits(int nsplit, size_t n, const float* part, float* out, hipStream_t s);
hipError_t launch_fallback_stats(int P, const float* pred, const float* resid, float frac, float* stats, void* ws,
                                 hipStream_t s);
size_t net_reduce_ws_bytes(int P);
hipError_t launch_inv_max(int P, const float* dose, float* scale, int* argmax, void* ws, hipStream_t s);
hipError_t launch_scale_adjoint(int P, const float* dose, const float* gp, const float* pred, const float* scale,
                                const int* argmax, float* ddose, void* ws, hipStream_t s);
hipError_t launch_scale_by(int P, const float* a, const float* scale, int inv, float* out, hipStream_t s);
hipError_t launch_add_bf16(size_t n, const __bf16* a, const __bf16* b, __bf16* out, hipStream_t s);
hipError_t launch_net_input_bwd(int P, const __bf16* dX0, const float* gp, const float* scale, float* ddose,
                                hipStream_t s);
hipError_t launch_adam(size_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s);

// Per-launch timing shared by every entry point (pdrt_profile_begin / _end): an
// event is recorded on the launch stream before and after each timed launch.
bool prof_enabled();
int prof_mark(hipStream_t s);                       // event index, or -1 (pool exhausted / error)
void prof_record(const char* name, int a, int b);

}  // namespace pdrt

// Enqueue `x` (a hipError_t expression) on stream `s`, timed under `name` when
// profiling is on; returns PDRT_E_HIP from the enclosing function on failure.
#define PDRT_TIMED(name, s, x)                                         \
  do {                                                                 \
    int pa_ = ::pdrt::prof_enabled() ? ::pdrt::prof_mark(s) : -1;      \
    if ((x) != hipSuccess) return PDRT_E_HIP;                          \
    if (pa_ >= 0) {                                                    \
      int pb_ = ::pdrt::prof_mark(s);                                  \
      if (pb_ >= 0) ::pdrt::prof_record(name, pa_, pb_);               \
    }                                                                  \
  } while (0)
