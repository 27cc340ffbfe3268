// net_api.hip — C ABI of the network primitives (declared in include/pdrt.h).
// Host-side validation, then one or two launches on the caller's stream.
#include <cmath>

#include "pdrt_internal.hpp"


using namespace pdrt;

namespace {

bool vol_ok(const pdrt_vol* v) {
  return v && v->D >= 1 && v->H >= 1 && v->W >= 1 && (double)v->D * v->H * v->W < 2.0e9;
}
bool even_vol(const pdrt_vol* v) { return vol_ok(v) && v->D % 2 == 0 && v->H % 2 == 0 && v->W % 2 == 0; }
Vol V(const pdrt_vol* v) { return Vol{v->D, v->H, v->W}; }
bool chan_ok(int c) { return c >= 8 && c <= 256 && c % 8 == 0; }
int kpad(int k) { return (k + 31) / 32 * 32; }

}  // namespace

extern "C" {

int32_t pdrt_conv3d_kpad(int32_t cin) { return cin >= 1 ? kpad(27 * cin) : 0; }

int pdrt_conv3d_prepare_weights(int32_t cout, int32_t cin, const float* w, void* wt, void* wd, void* stream) {
  if (!w || !wt || !wd || cout < 16 || cout % 16 || !chan_ok(cin)) return PDRT_E_INVALID;
  PDRT_TIMED("prep_weights", (hipStream_t)stream, launch_prep_weights(cout, cin, kpad(27 * cin), kpad(27 * cout), w, (__bf16*)wt, (__bf16*)wd,
                              (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_conv3d_forward(const pdrt_vol* vol, int32_t c1, int32_t c2, const void* x1, const void* x2, int32_t cout,
                        const void* wt, const float* bias, int32_t relu, void* y, void* stream) {
  if (!vol_ok(vol) || !chan_ok(c1) || c2 < 0 || (c2 && (!chan_ok(c2) || !x2)) || !x1 || !wt || !bias || !y)
    return PDRT_E_INVALID;
  if ((c1 + c2) % 16 || !(cout == 16 || cout == 32 || cout == 64)) return PDRT_E_UNSUPPORTED;
  PDRT_TIMED("conv3d_fwd", (hipStream_t)stream, launch_conv3d_fwd(V(vol), c1, c2, (const __bf16*)x1, (const __bf16*)x2, cout, (const __bf16*)wt,
                            kpad(27 * (c1 + c2)), bias, relu, (__bf16*)y, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_conv3d_backward_data(const pdrt_vol* vol, int32_t cout, const void* dy, const void* y_act, int32_t c1,
                              int32_t c2, const void* wd, void* dx1, void* dx2, void* stream) {
  int cin = c1 + c2;
  if (!vol_ok(vol) || !chan_ok(c1) || c2 < 0 || (c2 && (!chan_ok(c2) || !dx2)) || !dy || !wd || !dx1)
    return PDRT_E_INVALID;
  if (cout % 16 || cout < 16 || cout > 64) return PDRT_E_UNSUPPORTED;
  int nt = cin / 16;
  if (cin % 16 || !(nt == 1 || nt == 2 || nt == 3 || nt == 4 || nt == 6)) return PDRT_E_UNSUPPORTED;
  PDRT_TIMED("conv3d_dgrad", (hipStream_t)stream, launch_conv3d_dgrad(V(vol), cout, (const __bf16*)dy, (const __bf16*)y_act, cin, (const __bf16*)wd,
                              kpad(27 * cout), c1, (__bf16*)dx1, (__bf16*)dx2, (hipStream_t)stream));
  return PDRT_OK;
}

size_t pdrt_conv3d_wgrad_ws_bytes(int32_t cout, int32_t cin, int32_t nsplit) {
  if (cout < 1 || cin < 1 || nsplit < 1) return 0;
  return sizeof(float) * (size_t)nsplit * cout * 27 * cin;
}

int pdrt_conv3d_backward_weight(const pdrt_vol* vol, int32_t c1, int32_t c2, const void* x1, const void* x2,
                                int32_t cout, const void* dy, const void* y_act, int32_t nsplit, float* ws,
                                size_t ws_bytes, float* dw, float* db, void* stream) {
  if (!vol_ok(vol) || !chan_ok(c1) || c2 < 0 || (c2 && (!chan_ok(c2) || !x2)) || !x1 || !dy || !dw || !db ||
      cout < 1 || cout > 64 || nsplit < 1 || nsplit > 65535)
    return PDRT_E_INVALID;
  if (!ws || ws_bytes < pdrt_conv3d_wgrad_ws_bytes(cout, c1 + c2, nsplit)) return PDRT_E_WORKSPACE;
  PDRT_TIMED("conv3d_wgrad", (hipStream_t)stream, launch_conv3d_wgrad(V(vol), c1, c2, (const __bf16*)x1, (const __bf16*)x2, cout, (const __bf16*)dy,
                              (const __bf16*)y_act, nsplit, ws, dw, db, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_net_input(int32_t n, const float* dose, const float* scale, const float* rho, void* x, void* stream) {
  if (n < 1 || !dose || !scale || !rho || !x) return PDRT_E_INVALID;
  PDRT_TIMED("net_input", (hipStream_t)stream, launch_net_input(n, dose, scale, rho, (__bf16*)x, (hipStream_t)stream));
  return PDRT_OK;
}

size_t pdrt_net_reduce_ws_bytes(int32_t n) { return n < 1 ? 0 : net_reduce_ws_bytes(n); }

int pdrt_net_input_backward(int32_t n, const void* dx0, const float* gp, const float* scale, const float* dose,
                            const float* pred, const int32_t* argmax, float* ddose, void* ws, size_t ws_bytes,
                            void* stream) {
  if (n < 1 || !dx0 || !gp || !scale || !ddose) return PDRT_E_INVALID;
  const bool exact = dose || pred || argmax;
  if (exact && !(dose && pred && argmax)) return PDRT_E_INVALID;
  if (exact && (!ws || ws_bytes < net_reduce_ws_bytes(n))) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("net_input_bwd", s, launch_net_input_bwd(n, (const __bf16*)dx0, gp, scale, ddose, s));
  if (exact) PDRT_TIMED("scale_adjoint", s, launch_scale_adjoint(n, dose, gp, pred, scale, argmax, ddose, ws, s));
  return PDRT_OK;
}

int pdrt_net_scale(int32_t n, const float* dose, float* scale, int32_t* argmax, void* ws, size_t ws_bytes,
                   void* stream) {
  if (n < 1 || !dose || !scale) return PDRT_E_INVALID;
  if (!ws || ws_bytes < net_reduce_ws_bytes(n)) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("net_scale", s, launch_inv_max(n, dose, scale, argmax, ws, s));
  return PDRT_OK;
}

int pdrt_scale_by(int32_t n, const float* a, const float* scale, int32_t inverse, float* out, void* stream) {
  if (n < 1 || !a || !scale || !out) return PDRT_E_INVALID;
  PDRT_TIMED("scale_by", (hipStream_t)stream, launch_scale_by(n, a, scale, inverse != 0, out, (hipStream_t)stream));
  return PDRT_OK;
}

// 16-byte alignment of a device pointer (the pooling kernels move eight channels at a time)
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
static bool fits32(const pdrt_vol* v, int32_t c) { return (size_t)v->D * v->H * v->W * (size_t)c <= 0x7fffffffULL; }

int pdrt_add_bf16(size_t n, const void* a, const void* b, void* out, void* stream) {
  if (!n || !a || !b || !out || !aligned16(a) || !aligned16(b) || !aligned16(out)) return PDRT_E_INVALID;
  PDRT_TIMED("add_bf16", (hipStream_t)stream, launch_add_bf16(n, (const __bf16*)a, (const __bf16*)b, (__bf16*)out, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_pool2(const pdrt_vol* fine, int32_t c, const void* x, void* y, int32_t backward, void* stream) {
  if (!even_vol(fine) || c < 8 || c % 8 != 0 || !x || !y || !aligned16(x) || !aligned16(y) || !fits32(fine, c))
    return PDRT_E_INVALID;
  PDRT_TIMED("pool2", (hipStream_t)stream, launch_pool2(V(fine), c, (const __bf16*)x, (__bf16*)y, backward, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_upsample2(const pdrt_vol* fine, int32_t c, const void* x, void* y, int32_t backward, void* stream) {
  if (!even_vol(fine) || c < 8 || c % 8 != 0 || !x || !y || !aligned16(x) || !aligned16(y) || !fits32(fine, c))
    return PDRT_E_INVALID;
  PDRT_TIMED("upsample2", (hipStream_t)stream, launch_up2(V(fine), c, (const __bf16*)x, (__bf16*)y, backward, (hipStream_t)stream));
  return PDRT_OK;
}

int pdrt_net_head(int32_t n, int32_t c, const void* x, const float* hw, const float* hb, const float* dose,
                  const float* scale, float* pred, float* resid, void* stream) {
  if (n < 1 || c < 1 || !x || !hw || !hb || !dose || !scale || !pred || !resid) return PDRT_E_INVALID;
  PDRT_TIMED("net_head", (hipStream_t)stream, launch_head(n, c, (const __bf16*)x, hw, hb, dose, scale, pred, resid, (hipStream_t)stream));
  return PDRT_OK;
}

size_t pdrt_net_head_ws_bytes(int32_t n, int32_t c) {
  if (n < 1 || c < 1) return 0;
  return sizeof(float) * (size_t)((n + 255) / 256) * (2 * c + 2);
}

int pdrt_net_head_backward(int32_t n, int32_t c, const void* x, const float* hw, const float* gp, const float* gr,
                           void* dx, float* ws, size_t ws_bytes, float* dhead, void* stream) {
  if (n < 1 || c < 1 || !x || !hw || !gp || !dx) return PDRT_E_INVALID;
  if (dhead && (!ws || ws_bytes < pdrt_net_head_ws_bytes(n, c))) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("net_head_bwd", s, launch_head_bwd(n, c, (const __bf16*)x, hw, gp, gr, (__bf16*)dx, dhead ? ws : nullptr,
                                                s));
  if (dhead) PDRT_TIMED("reduce_splits", s, launch_reduce_splits((n + 255) / 256, (size_t)(2 * c + 2), ws, dhead, s));
  return PDRT_OK;
}

size_t pdrt_net_loss_ws_bytes(int32_t n) { return n < 1 ? 0 : sizeof(float) * (size_t)((n + 255) / 256); }

int pdrt_net_train_loss(int32_t n, const float* pred, const float* resid, const float* target, const float* tscale,
                        const float* mask, float inv_count, float lam, float quantile, float* gp, float* gr,
                        float* ws, size_t ws_bytes, float* loss, void* stream) {
  if (n < 1 || !pred || !resid || !target || !tscale || !mask || !gp || !gr || !loss) return PDRT_E_INVALID;
  if (!std::isfinite(inv_count) || !std::isfinite(lam)) return PDRT_E_INVALID;
  if (!(quantile >= 0.f && quantile < 1.f)) return PDRT_E_INVALID;
  if (!ws || ws_bytes < pdrt_net_loss_ws_bytes(n)) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("train_loss", s, launch_train_loss(n, pred, resid, target, tscale, mask, inv_count, lam, quantile, gp, gr, ws, s));
  PDRT_TIMED("reduce_splits", s, launch_reduce_splits((n + 255) / 256, 1, ws, loss, s));
  return PDRT_OK;
}

int pdrt_net_fallback_stats(int32_t n, const float* pred, const float* resid, float frac, float* stats, void* ws,
                            size_t ws_bytes, void* stream) {
  if (n < 1 || !pred || !resid || !stats || !std::isfinite(frac)) return PDRT_E_INVALID;
  if (!ws || ws_bytes < net_reduce_ws_bytes(n)) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("fallback_stats", s, launch_fallback_stats(n, pred, resid, frac, stats, ws, s));
  return PDRT_OK;
}

int pdrt_adam_step(size_t n, float* w, const float* g, float* m, float* v, float lr, float beta1, float beta2,
                   float eps, int32_t t, void* stream) {
  if (!n || !w || !g || !m || !v || t < 1 || !std::isfinite(lr) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return PDRT_E_INVALID;
  float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
  PDRT_TIMED("adam", (hipStream_t)stream, launch_adam(n, w, g, m, v, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
  return PDRT_OK;
}

}  // extern "C"
