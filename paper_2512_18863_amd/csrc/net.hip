// net.hip — kernels of the small 3-D convolutional network that maps a
// small-kernel dose plus density to a large-kernel dose (the learned correction
// of the lateral-kernel-size effect, cf. Table 5 and §4.1 "smaller kernel sizes
// first").
//
// Tensors are channels-last, [D][H][W][C], BF16 for activations and their
// gradients, FP32 for master weights, weight gradients and the dose channels.
// 3 x 3 x 3 convolutions ("same" zero padding, stride 1) are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   forward  Y[p][co]  = act(b[co] + sum_{tap,ci} X[p + o(tap)][ci] Wt[co][tap ci])
//   data     dX[p][ci] = sum_{tap,co} dY'[p - o(tap)][co] Wd[ci][tap co],  dY' = dY * [Y > 0]
//   weight   dW[co][tap ci] = sum_p dY'[p][co] X[p + o(tap)][ci]
// The K index (tap, channel) is flattened with the channel fastest, so a lane's
// eight consecutive K entries are eight channels of one neighbour: one 16-byte
// load.  The two operands of the forward may come from two tensors (a skip
// connection is a channel concatenation, read in place).
#include "pdrt_internal.hpp"

namespace pdrt {

typedef float nf32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 nbf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bool neighbour(const Vol& v, int p, int tap, int* q) {
  int w = p % v.W, t = p / v.W;
  int h = t % v.H, d = t / v.H;
  int dd = d + tap / 9 - 1, hh = h + (tap / 3) % 3 - 1, ww = w + tap % 3 - 1;
  if (dd < 0 || dd >= v.D || hh < 0 || hh >= v.H || ww < 0 || ww >= v.W) return false;
  *q = (dd * v.H + hh) * v.W + ww;
  return true;
}

__device__ __forceinline__ bool neighbour_back(const Vol& v, int p, int tap, int* q) {
  int w = p % v.W, t = p / v.W;
  int h = t % v.H, d = t / v.H;
  int dd = d - (tap / 9 - 1), hh = h - ((tap / 3) % 3 - 1), ww = w - (tap % 3 - 1);
  if (dd < 0 || dd >= v.D || hh < 0 || hh >= v.H || ww < 0 || ww >= v.W) return false;
  *q = (dd * v.H + hh) * v.W + ww;
  return true;
}

// ------------------------------------------------------------------ forward

// One wavefront: 16 consecutive positions x all NT*16 output channels.
template <int NT>
__global__ void __launch_bounds__(256) k_conv3d_fwd(Vol v, int C1, int C2, const __bf16* __restrict__ X1,
                                                    const __bf16* __restrict__ X2, const __bf16* __restrict__ Wt,
                                                    int Kp, const float* __restrict__ bias, int relu,
                                                    __bf16* __restrict__ Y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int P = v.D * v.H * v.W;
  const int p0 = (blockIdx.x * 4 + wave) * 16;
  if (p0 >= P) return;
  const int Cin = C1 + C2, Cout = NT * 16;
  const int m = lane & 15, kq = lane >> 4;
  const int p = p0 + m;
  const int K = 27 * Cin;
  nf32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = nf32x4{0.f, 0.f, 0.f, 0.f};
  const nbf16x8 zero8 = {};
  const int nsteps = Kp / 32;  // the same trip count for every lane
  for (int st = 0; st < nsteps; ++st) {
    const int k0 = 32 * st + 8 * kq;
    nbf16x8 a = zero8;
    if (k0 < K && p < P) {
      int tap = k0 / Cin, ci = k0 - tap * Cin, q;
      if (neighbour(v, p, tap, &q)) {
        const __bf16* src = ci < C1 ? X1 + (size_t)q * C1 + ci : X2 + (size_t)q * C2 + (ci - C1);
        a = *reinterpret_cast<const nbf16x8*>(src);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      nbf16x8 b = *reinterpret_cast<const nbf16x8*>(Wt + (size_t)(16 * t + m) * Kp + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = 16 * t + m;
    const float bb = bias[co];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pp = p0 + 4 * kq + r;
      if (pp < P) {
        float y = acc[t][r] + bb;
        if (relu) y = y > 0.f ? y : 0.f;
        Y[(size_t)pp * Cout + co] = (__bf16)y;
      }
    }
  }
}

// ------------------------------------------------------------------ data gradient

template <int NT>
__global__ void __launch_bounds__(256) k_conv3d_dgrad(Vol v, int Cout, const __bf16* __restrict__ dY,
                                                      const __bf16* __restrict__ Yact, const __bf16* __restrict__ Wd,
                                                      int Kp, int C1, __bf16* __restrict__ dX1,
                                                      __bf16* __restrict__ dX2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int P = v.D * v.H * v.W;
  const int p0 = (blockIdx.x * 4 + wave) * 16;
  if (p0 >= P) return;
  const int Cin = NT * 16, C2 = Cin - C1;
  const int m = lane & 15, kq = lane >> 4;
  const int p = p0 + m;
  const int K = 27 * Cout;
  nf32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = nf32x4{0.f, 0.f, 0.f, 0.f};
  const nbf16x8 zero8 = {};
  const int nsteps = Kp / 32;
  for (int st = 0; st < nsteps; ++st) {
    const int k0 = 32 * st + 8 * kq;
    nbf16x8 a = zero8;
    if (k0 < K && p < P) {
      int tap = k0 / Cout, co = k0 - tap * Cout, q;
      if (neighbour_back(v, p, tap, &q)) {
        a = *reinterpret_cast<const nbf16x8*>(dY + (size_t)q * Cout + co);
        if (Yact) {
          nbf16x8 y = *reinterpret_cast<const nbf16x8*>(Yact + (size_t)q * Cout + co);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (!((float)y[e] > 0.f)) a[e] = (__bf16)0.f;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      nbf16x8 b = *reinterpret_cast<const nbf16x8*>(Wd + (size_t)(16 * t + m) * Kp + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int ci = 16 * t + m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pp = p0 + 4 * kq + r;
      if (pp < P) {
        if (ci < C1)
          dX1[(size_t)pp * C1 + ci] = (__bf16)acc[t][r];
        else
          dX2[(size_t)pp * C2 + (ci - C1)] = (__bf16)acc[t][r];
      }
    }
  }
}

// ------------------------------------------------------------------ weight gradient

// Partial sums over a chunk of positions: part[split][co][tap][ci] (FP32).  A
// block owns one tap and 256 (co, ci) pairs; threads along ci read consecutive
// channels of the same neighbour, dY' is a broadcast within a channel group.
__global__ void __launch_bounds__(256) k_conv3d_wgrad_part(Vol v, int C1, int C2, const __bf16* __restrict__ X1,
                                                           const __bf16* __restrict__ X2, int Cout,
                                                           const __bf16* __restrict__ dY,
                                                           const __bf16* __restrict__ Yact, int chunk,
                                                           float* __restrict__ part) {
  const int Cin = C1 + C2;
  const int tap = blockIdx.x;
  const int pair = blockIdx.y * 256 + threadIdx.x;
  const int split = blockIdx.z;
  const int P = v.D * v.H * v.W;
  if (pair >= Cout * Cin) return;
  const int co = pair / Cin, ci = pair - co * Cin;
  const int pa = split * chunk, pb = min(P, pa + chunk);
  float s = 0.f;
  for (int p = pa; p < pb; ++p) {
    float g = (float)dY[(size_t)p * Cout + co];
    if (Yact && !((float)Yact[(size_t)p * Cout + co] > 0.f)) g = 0.f;
    if (g == 0.f) continue;
    int q;
    if (!neighbour(v, p, tap, &q)) continue;
    float x = ci < C1 ? (float)X1[(size_t)q * C1 + ci] : (float)X2[(size_t)q * C2 + (ci - C1)];
    s += g * x;
  }
  part[(((size_t)split * Cout + co) * 27 + tap) * Cin + ci] = s;
}

// Bias partial sums over the same position chunks: partb[split][co] = sum_p dY'[p][co].
__global__ void k_bias_part(Vol v, int Cout, const __bf16* __restrict__ dY, const __bf16* __restrict__ Yact,
                            int chunk, float* __restrict__ partb) {
  const int co = threadIdx.x, split = blockIdx.x;
  const int P = v.D * v.H * v.W;
  if (co >= Cout) return;
  const int pa = split * chunk, pb = min(P, pa + chunk);
  float s = 0.f;
  for (int p = pa; p < pb; ++p) {
    float g = (float)dY[(size_t)p * Cout + co];
    if (Yact && !((float)Yact[(size_t)p * Cout + co] > 0.f)) g = 0.f;
    s += g;
  }
  partb[(size_t)split * Cout + co] = s;
}

// dW[i] = sum over splits in order (deterministic).
// Few outputs, many splits: one block per output, each thread a strided partial
// sum, then a tree over the block (fixed order).
__global__ void __launch_bounds__(256) k_reduce_splits_tall(int nsplit, size_t n, const float* __restrict__ part,
                                                            float* __restrict__ out) {
  __shared__ float red[256];
  const size_t i = blockIdx.x;
  float s = 0.f;
  for (int k = threadIdx.x; k < nsplit; k += 256) s += part[(size_t)k * n + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

__global__ void k_reduce_splits(int nsplit, size_t n, const float* __restrict__ part, float* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * n + i];
  out[i] = s;
}

// ------------------------------------------------------------------ glue

// Weight layouts for the MFMA operands from FP32 master weights W[co][tap][ci]:
//   Wt[co][tap*Cin + ci] (forward), Wd[ci][tap*Cout + co] (data gradient), K padded to Kp.
__global__ void k_prep_weights(int Cout, int Cin, int Kpf, int Kpd, const float* __restrict__ W,
                               __bf16* __restrict__ Wt, __bf16* __restrict__ Wd) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int nf = Cout * Kpf, nd = Cin * Kpd;
  if (i < nf) {
    int co = i / Kpf, k = i - co * Kpf;
    float val = 0.f;
    if (k < 27 * Cin) val = W[(size_t)co * 27 * Cin + k];
    Wt[i] = (__bf16)val;
  } else if (i < nf + nd) {
    int j = i - nf;
    int ci = j / Kpd, k = j - ci * Kpd;
    float val = 0.f;
    if (k < 27 * Cout) {
      int tap = k / Cout, co = k - tap * Cout;
      val = W[((size_t)co * 27 + tap) * Cin + ci];
    }
    Wd[j] = (__bf16)val;
  }
}

// Network input: channel 0 = dose * scale, channel 1 = density, channels 2..15 = 0.
__global__ void k_net_input(int P, const float* __restrict__ dose, const float* __restrict__ scale,
                            const float* __restrict__ rho, __bf16* __restrict__ X) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  nbf16x8 a = {}, b = {};
  a[0] = (__bf16)(dose[p] * scale[0]);
  a[1] = (__bf16)rho[p];
  *reinterpret_cast<nbf16x8*>(X + (size_t)p * 16) = a;
  *reinterpret_cast<nbf16x8*>(X + (size_t)p * 16 + 8) = b;
}

// 2 x 2 x 2 average pooling (dims of the input; even).
__global__ void k_pool2(Vol v, int C, const __bf16* __restrict__ X, __bf16* __restrict__ Y) {
  int Do = v.D / 2, Ho = v.H / 2, Wo = v.W / 2;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)Do * Ho * Wo * C;
  if (i >= n) return;
  int c = i % C;
  size_t po = i / C;
  int w = po % Wo, t = po / Wo, h = t % Ho, d = t / Ho;
  float s = 0.f;
  for (int a = 0; a < 8; ++a) {
    int dd = 2 * d + (a >> 2), hh = 2 * h + ((a >> 1) & 1), ww = 2 * w + (a & 1);
    s += (float)X[(((size_t)dd * v.H + hh) * v.W + ww) * C + c];
  }
  Y[i] = (__bf16)(0.125f * s);
}

__global__ void k_pool2_bwd(Vol v, int C, const __bf16* __restrict__ dY, __bf16* __restrict__ dX) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)v.D * v.H * v.W * C;
  if (i >= n) return;
  int c = i % C;
  size_t p = i / C;
  int w = p % v.W, t = p / v.W, h = t % v.H, d = t / v.H;
  int Ho = v.H / 2, Wo = v.W / 2;
  dX[i] = (__bf16)(0.125f * (float)dY[(((size_t)(d / 2) * Ho + h / 2) * Wo + w / 2) * C + c]);
}

// Nearest-neighbour upsampling x2 (dims of the output).
__global__ void k_up2(Vol v, int C, const __bf16* __restrict__ X, __bf16* __restrict__ Y) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)v.D * v.H * v.W * C;
  if (i >= n) return;
  int c = i % C;
  size_t p = i / C;
  int w = p % v.W, t = p / v.W, h = t % v.H, d = t / v.H;
  int Hi = v.H / 2, Wi = v.W / 2;
  Y[i] = X[(((size_t)(d / 2) * Hi + h / 2) * Wi + w / 2) * C + c];
}

__global__ void k_up2_bwd(Vol v, int C, const __bf16* __restrict__ dY, __bf16* __restrict__ dX) {
  int Di = v.D / 2, Hi = v.H / 2, Wi = v.W / 2;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)Di * Hi * Wi * C;
  if (i >= n) return;
  int c = i % C;
  size_t po = i / C;
  int w = po % Wi, t = po / Wi, h = t % Hi, d = t / Hi;
  float s = 0.f;
  for (int a = 0; a < 8; ++a) {
    int dd = 2 * d + (a >> 2), hh = 2 * h + ((a >> 1) & 1), ww = 2 * w + (a & 1);
    s += (float)dY[(((size_t)dd * v.H + hh) * v.W + ww) * C + c];
  }
  dX[i] = (__bf16)s;
}

// Head: 1 x 1 x 1 convolution C -> 2 in FP32, output 0 added to the input dose
// channel (a residual on the small-kernel dose), output 1 the error estimate.
//   pred[p] = dose[p] * scale + hb[0] + sum_c hw[0][c] X[p][c]
//   resid[p] = hb[1] + sum_c hw[1][c] X[p][c]
__global__ void k_head(int P, int C, const __bf16* __restrict__ X, const float* __restrict__ hw,
                       const float* __restrict__ hb, const float* __restrict__ dose, const float* __restrict__ scale,
                       float* __restrict__ pred, float* __restrict__ resid) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float a = hb[0], r = hb[1];
  for (int c = 0; c < C; ++c) {
    float x = (float)X[(size_t)p * C + c];
    a += hw[c] * x;
    r += hw[C + c] * x;
  }
  pred[p] = dose[p] * scale[0] + a;
  resid[p] = r;
}

// Backward of the head for upstream gradients gp (pred) and gr (resid):
//   dX[p][c] = gp hw[0][c] + gr hw[1][c];  per-block partials of dhw, dhb.
__global__ void __launch_bounds__(256) k_head_bwd(int P, int C, const __bf16* __restrict__ X,
                                                  const float* __restrict__ hw, const float* __restrict__ gp,
                                                  const float* __restrict__ gr, __bf16* __restrict__ dX,
                                                  float* __restrict__ part) {
  __shared__ float red[256];
  int p = blockIdx.x * 256 + threadIdx.x;
  float g0 = 0.f, g1 = 0.f;
  if (p < P) {
    g0 = gp[p];
    g1 = gr ? gr[p] : 0.f;
  }
  const int np = part ? 2 * C + 2 : 0;  // no head-weight gradient wanted: skip the partial sums
  for (int j = 0; j < np; ++j) {
    float v = 0.f;
    if (p < P) {
      if (j < 2 * C) {
        int o = j / C, c = j - o * C;
        v = (o ? g1 : g0) * (float)X[(size_t)p * C + c];
      } else {
        v = (j == 2 * C) ? g0 : g1;
      }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * np + j] = red[0];
    __syncthreads();
  }
  if (p < P)
    for (int c = 0; c < C; ++c) dX[(size_t)p * C + c] = (__bf16)(g0 * hw[c] + g1 * hw[C + c]);
}

// Training loss over a mask: L = sum_p m [(pred - T)^2 + lam (resid - |pred - T|)^2] / sum m,
// gradients gp, gr (the residual target is not differentiated); per-block partial sums.
__global__ void __launch_bounds__(256) k_train_loss(int P, const float* __restrict__ pred,
                                                    const float* __restrict__ resid, const float* __restrict__ target,
                                                    const float* __restrict__ tscale, const float* __restrict__ mask,
                                                    float inv_count, float lam, float* __restrict__ gp,
                                                    float* __restrict__ gr, float* __restrict__ part) {
  __shared__ float red[256];
  int p = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (p < P) {
    float m = mask[p];
    float e = pred[p] - target[p] * tscale[0];
    float ae = fabsf(e);
    float er = resid[p] - ae;
    l = m * (e * e + lam * er * er) * inv_count;
    gp[p] = m * 2.f * e * inv_count;
    gr[p] = m * 2.f * lam * er * inv_count;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (FP32 master weights): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// w -= lr * mhat / (sqrt(vhat) + eps), bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(size_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// scale[0] = 1 / max(dose) (single block).
// Maximum with its first index (ties keep the smallest index), two passes with
// fixed order: blocks reduce strided slices into partials, one block reduces
// those.  Only positive values count (max <= 0 gives index -1).
constexpr int RED_BLOCKS = 512;

__device__ __forceinline__ void better(float& v, int& i, float v2, int i2) {
  if (v2 > v || (v2 == v && i2 >= 0 && (i < 0 || i2 < i))) v = v2, i = i2;
}

__global__ void __launch_bounds__(256) k_max_part(int P, const float* __restrict__ x, float init,
                                                  const float* __restrict__ gate, float gate_frac,
                                                  const float* __restrict__ gate_max, float* __restrict__ pv,
                                                  int* __restrict__ pi) {
  // values below init do not count; gate (optional): only p with
  // gate[p] >= gate_frac * gate_max[0] count
  __shared__ float rv[256];
  __shared__ int ri[256];
  const float thr = gate ? gate_frac * gate_max[0] : 0.f;
  float v = init;
  int im = -1;
  for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256) {
    if (gate && !(gate[p] >= thr)) continue;
    const float d = x[p];
    if (d > v) v = d, im = p;
  }
  rv[threadIdx.x] = v;
  ri[threadIdx.x] = im;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) better(rv[threadIdx.x], ri[threadIdx.x], rv[threadIdx.x + off], ri[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = rv[0];
    pi[blockIdx.x] = ri[0];
  }
}

// mode 0: scale[0] = 1 / max (1 if no positive value), argmax[0] (may be null);
// mode 1: out[0] = max (the raw maximum, for the fallback statistics)
__global__ void __launch_bounds__(256) k_max_final(int nb, const float* __restrict__ pv, const int* __restrict__ pi,
                                                   int mode, float* __restrict__ out, int* __restrict__ argmax) {
  __shared__ float rv[256];
  __shared__ int ri[256];
  float v = -3.4e38f;
  int im = -1;
  for (int b = threadIdx.x; b < nb; b += 256) better(v, im, pv[b], pi[b]);
  rv[threadIdx.x] = v;
  ri[threadIdx.x] = im;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) better(rv[threadIdx.x], ri[threadIdx.x], rv[threadIdx.x + off], ri[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (mode == 0) {
      const bool pos = rv[0] > 0.f;
      out[0] = pos ? 1.f / rv[0] : 1.f;
      if (argmax) argmax[0] = pos ? ri[0] : -1;
    } else {
      out[0] = rv[0];
    }
  }
}

// out[p] = a[p] * f, f = scale[0] (inv = 0) or 1 / scale[0] (inv = 1).
__global__ void k_scale_by(int P, const float* __restrict__ a, const float* __restrict__ scale, int inv,
                           float* __restrict__ out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float f = inv ? 1.f / scale[0] : scale[0];
  out[p] = a[p] * f;
}

// out = a + b (bf16), e.g. two gradient contributions of one activation.
__global__ void k_add_bf16(size_t n, const __bf16* __restrict__ a, const __bf16* __restrict__ b,
                           __bf16* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (__bf16)((float)a[i] + (float)b[i]);
}

// Gradient w.r.t. the input dose: d dose[p] = scale (gp[p] + dX0[p][0]) (the dose
// enters the head directly and the first convolution through channel 0).
__global__ void k_net_input_bwd(int P, const __bf16* __restrict__ dX0, const float* __restrict__ gp,
                                const float* __restrict__ scale, float* __restrict__ ddose) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  ddose[p] = scale[0] * (gp[p] + (float)dX0[(size_t)p * 16]);
}

// The normalisation s = 1 / max(dose) depends on the dose at its argmax m:
// ddose[m] -= s (sum_p dose[p] ddose[p] - sum_p gp[p] pred[p]), with ddose the
// gradient at fixed s.  FP64 partial sums per block, then one block adds them in
// a fixed order and updates ddose[m].
__global__ void __launch_bounds__(256) k_scale_adj_part(int P, const float* __restrict__ dose,
                                                        const float* __restrict__ gp, const float* __restrict__ pred,
                                                        const float* __restrict__ ddose, double* __restrict__ part) {
  __shared__ double red[256];
  double t = 0.0;
  for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256)
    t += (double)dose[p] * (double)ddose[p] - (double)gp[p] * (double)pred[p];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_scale_adj_final(int nb, const double* __restrict__ part,
                                                         const float* __restrict__ scale, const int* __restrict__ argmax,
                                                         float* __restrict__ ddose) {
  __shared__ double red[256];
  const int m = argmax[0];
  if (m < 0) return;  // zero dose: s is the constant 1 (uniform across the block)
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) t += part[b];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) ddose[m] = (float)((double)ddose[m] - (double)scale[0] * red[0]);
}

// Fallback statistics: stats[0] = max pred, stats[1] = max resid over voxels with
// pred >= frac * max pred; each a two-pass maximum (k_max_part / k_max_final).

// ------------------------------------------------------------------ launchers

static unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_conv3d_fwd(Vol v, int C1, int C2, const __bf16* X1, const __bf16* X2, int Cout,
                             const __bf16* Wt, int Kp, const float* bias, int relu, __bf16* Y, hipStream_t s) {
  size_t P = (size_t)v.D * v.H * v.W;
  dim3 grid(nblk(P, 64));
  switch (Cout / 16) {
    case 1: hipLaunchKernelGGL(k_conv3d_fwd<1>, grid, dim3(256), 0, s, v, C1, C2, X1, X2, Wt, Kp, bias, relu, Y); break;
    case 2: hipLaunchKernelGGL(k_conv3d_fwd<2>, grid, dim3(256), 0, s, v, C1, C2, X1, X2, Wt, Kp, bias, relu, Y); break;
    case 4: hipLaunchKernelGGL(k_conv3d_fwd<4>, grid, dim3(256), 0, s, v, C1, C2, X1, X2, Wt, Kp, bias, relu, Y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_conv3d_dgrad(Vol v, int Cout, const __bf16* dY, const __bf16* Yact, int Cin, const __bf16* Wd,
                               int Kp, int C1, __bf16* dX1, __bf16* dX2, hipStream_t s) {
  size_t P = (size_t)v.D * v.H * v.W;
  dim3 grid(nblk(P, 64));
  switch (Cin / 16) {
    case 1: hipLaunchKernelGGL(k_conv3d_dgrad<1>, grid, dim3(256), 0, s, v, Cout, dY, Yact, Wd, Kp, C1, dX1, dX2); break;
    case 2: hipLaunchKernelGGL(k_conv3d_dgrad<2>, grid, dim3(256), 0, s, v, Cout, dY, Yact, Wd, Kp, C1, dX1, dX2); break;
    case 3: hipLaunchKernelGGL(k_conv3d_dgrad<3>, grid, dim3(256), 0, s, v, Cout, dY, Yact, Wd, Kp, C1, dX1, dX2); break;
    case 4: hipLaunchKernelGGL(k_conv3d_dgrad<4>, grid, dim3(256), 0, s, v, Cout, dY, Yact, Wd, Kp, C1, dX1, dX2); break;
    case 6: hipLaunchKernelGGL(k_conv3d_dgrad<6>, grid, dim3(256), 0, s, v, Cout, dY, Yact, Wd, Kp, C1, dX1, dX2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_conv3d_wgrad(Vol v, int C1, int C2, const __bf16* X1, const __bf16* X2, int Cout, const __bf16* dY,
                               const __bf16* Yact, int nsplit, float* part, float* dW, float* db, hipStream_t s) {
  size_t P = (size_t)v.D * v.H * v.W;
  int chunk = (int)((P + nsplit - 1) / nsplit);
  int Cin = C1 + C2;
  dim3 grid(27, nblk((size_t)Cout * Cin), nsplit);
  hipLaunchKernelGGL(k_conv3d_wgrad_part, grid, dim3(256), 0, s, v, C1, C2, X1, X2, Cout, dY, Yact, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t n = (size_t)Cout * 27 * Cin;
  hipLaunchKernelGGL(k_reduce_splits, dim3(nblk(n)), dim3(256), 0, s, nsplit, n, part, dW);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // bias: reuse the start of the partial buffer (the weight partials are consumed)
  hipLaunchKernelGGL(k_bias_part, dim3(nsplit), dim3(64), 0, s, v, Cout, dY, Yact, chunk, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_splits, dim3(nblk(Cout)), dim3(256), 0, s, nsplit, (size_t)Cout, part, db);
  return hipGetLastError();
}

hipError_t launch_prep_weights(int Cout, int Cin, int Kpf, int Kpd, const float* W, __bf16* Wt, __bf16* Wd,
                               hipStream_t s) {
  size_t n = (size_t)Cout * Kpf + (size_t)Cin * Kpd;
  hipLaunchKernelGGL(k_prep_weights, dim3(nblk(n)), dim3(256), 0, s, Cout, Cin, Kpf, Kpd, W, Wt, Wd);
  return hipGetLastError();
}

hipError_t launch_net_input(int P, const float* dose, const float* scale, const float* rho, __bf16* X, hipStream_t s) {
  hipLaunchKernelGGL(k_net_input, dim3(nblk(P)), dim3(256), 0, s, P, dose, scale, rho, X);
  return hipGetLastError();
}

hipError_t launch_pool2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s) {
  size_t n = (size_t)v.D * v.H * v.W * C;
  if (!backward)
    hipLaunchKernelGGL(k_pool2, dim3(nblk(n / 8)), dim3(256), 0, s, v, C, X, Y);
  else
    hipLaunchKernelGGL(k_pool2_bwd, dim3(nblk(n)), dim3(256), 0, s, v, C, X, Y);
  return hipGetLastError();
}

hipError_t launch_up2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s) {
  size_t n = (size_t)v.D * v.H * v.W * C;
  if (!backward)
    hipLaunchKernelGGL(k_up2, dim3(nblk(n)), dim3(256), 0, s, v, C, X, Y);
  else
    hipLaunchKernelGGL(k_up2_bwd, dim3(nblk(n / 8)), dim3(256), 0, s, v, C, X, Y);
  return hipGetLastError();
}

hipError_t launch_head(int P, int C, const __bf16* X, const float* hw, const float* hb, const float* dose,
                       const float* scale, float* pred, float* resid, hipStream_t s) {
  hipLaunchKernelGGL(k_head, dim3(nblk(P)), dim3(256), 0, s, P, C, X, hw, hb, dose, scale, pred, resid);
  return hipGetLastError();
}

hipError_t launch_head_bwd(int P, int C, const __bf16* X, const float* hw, const float* gp, const float* gr,
                           __bf16* dX, float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nblk(P)), dim3(256), 0, s, P, C, X, hw, gp, gr, dX, part);
  return hipGetLastError();
}

hipError_t launch_train_loss(int P, const float* pred, const float* resid, const float* target, const float* tscale,
                             const float* mask, float inv_count, float lam, float* gp, float* gr, float* part,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_train_loss, dim3(nblk(P)), dim3(256), 0, s, P, pred, resid, target, tscale, mask, inv_count,
                     lam, gp, gr, part);
  return hipGetLastError();
}

hipError_t launch_reduce_splits(int nsplit, size_t n, const float* part, float* out, hipStream_t s) {
  if (n < 4096 && nsplit >= 64)
    hipLaunchKernelGGL(k_reduce_splits_tall, dim3((unsigned)n), dim3(256), 0, s, nsplit, n, part, out);
  else
    hipLaunchKernelGGL(k_reduce_splits, dim3(nblk(n)), dim3(256), 0, s, nsplit, n, part, out);
  return hipGetLastError();
}

static int red_blocks(int P) {
  int nb = (int)nblk((size_t)P, 1024);
  return nb < 1 ? 1 : (nb > RED_BLOCKS ? RED_BLOCKS : nb);
}

size_t net_reduce_ws_bytes(int P) {
  (void)P;
  return (size_t)RED_BLOCKS * (sizeof(double) + sizeof(int)) + 16;
}

hipError_t launch_fallback_stats(int P, const float* pred, const float* resid, float frac, float* stats, void* ws,
                                 hipStream_t s) {
  const int nb = red_blocks(P);
  float* pv = (float*)ws;
  int* pi = (int*)((char*)ws + RED_BLOCKS * sizeof(double));
  hipLaunchKernelGGL(k_max_part, dim3(nb), dim3(256), 0, s, P, pred, -3.4e38f, (const float*)nullptr, 0.f,
                     (const float*)nullptr, pv, pi);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, nb, pv, pi, 1, stats, (int*)nullptr);
  hipLaunchKernelGGL(k_max_part, dim3(nb), dim3(256), 0, s, P, resid, -3.4e38f, pred, frac, (const float*)stats, pv,
                     pi);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, nb, pv, pi, 1, stats + 1, (int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_inv_max(int P, const float* dose, float* scale, int* argmax, void* ws, hipStream_t s) {
  const int nb = red_blocks(P);
  float* pv = (float*)ws;
  int* pi = (int*)((char*)ws + RED_BLOCKS * sizeof(double));
  hipLaunchKernelGGL(k_max_part, dim3(nb), dim3(256), 0, s, P, dose, 0.f, (const float*)nullptr, 0.f,
                     (const float*)nullptr, pv, pi);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, nb, pv, pi, 0, scale, argmax);
  return hipGetLastError();
}

hipError_t launch_scale_by(int P, const float* a, const float* scale, int inv, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by, dim3(nblk(P)), dim3(256), 0, s, P, a, scale, inv, out);
  return hipGetLastError();
}

hipError_t launch_add_bf16(size_t n, const __bf16* a, const __bf16* b, __bf16* out, hipStream_t s) {
  hipLaunchKernelGGL(k_add_bf16, dim3(nblk(n)), dim3(256), 0, s, n, a, b, out);
  return hipGetLastError();
}

hipError_t launch_net_input_bwd(int P, const __bf16* dX0, const float* gp, const float* scale, float* ddose,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_net_input_bwd, dim3(nblk(P)), dim3(256), 0, s, P, dX0, gp, scale, ddose);
  return hipGetLastError();
}

hipError_t launch_scale_adjoint(int P, const float* dose, const float* gp, const float* pred, const float* scale,
                                const int* argmax, float* ddose, void* ws, hipStream_t s) {
  const int nb = red_blocks(P);
  double* part = (double*)ws;
  hipLaunchKernelGGL(k_scale_adj_part, dim3(nb), dim3(256), 0, s, P, dose, gp, pred, (const float*)ddose, part);
  hipLaunchKernelGGL(k_scale_adj_final, dim3(1), dim3(256), 0, s, nb, (const double*)part, scale, argmax, ddose);
  return hipGetLastError();
}

hipError_t launch_adam(size_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace pdrt
