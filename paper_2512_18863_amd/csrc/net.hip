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

// ------------------------------------------------------------------ forward and data gradient
//
// Implicit GEMM on v_mfma_f32_16x16x32_bf16 over a tile of 16 (w) x 8 (h) x
// 2 (d) output positions per workgroup: the input tile with its one-voxel halo
// is read from global memory once and kept in LDS (every position's 27
// neighbours are then LDS reads); the weights, shared by every workgroup, are
// read from global memory (cache resident) one K step ahead of their use.  M = 16 positions along w, N = 16 output channels per tile, K
// runs over (tap, input channel) in steps of 32, lane group kq holding 8
// consecutive channels of one tap; each lane tracks its (tap, channel)
// incrementally.  Each of the 4 wavefronts owns four position rows and all N,
// so each weight fragment it loads feeds four rows.
// The data gradient is the same GEMM with the taps mirrored, K over (tap,
// output channel), the ReLU mask applied while the tile is staged.

// A lane's position in K: tap (td, th, tw) in {0,1,2}^3 and channel ci < C.
struct KPos {
  int ci, tap, td, th, tw;
  __device__ void next_tap() {
    ++tap;
    if (++tw == 3) {
      tw = 0;
      if (++th == 3) {
        th = 0;
        ++td;
      }
    }
  }
  __device__ void advance(int add, int C) {  // ci += add (add <= 32, C >= 16: at most two taps)
    ci += add;
    if (ci >= C) {
      ci -= C;
      next_tap();
    }
    if (ci >= C) {
      ci -= C;
      next_tap();
    }
  }
};

constexpr int CT_W = 16, CT_H = 8, CT_D = 2;                          // output tile
constexpr int CT_RPW = CT_H * CT_D / 4;                              // position rows per wavefront
constexpr int CT_HW = CT_W + 2, CT_HH = CT_H + 2, CT_HD = CT_D + 2;   // with halo
constexpr int CT_POS = CT_HW * CT_HH * CT_HD;

struct ConvIO {
  const __bf16* a1;      // input, channels [0, c1)
  const __bf16* a2;      // input, channels [c1, c1 + c2) (may be null when c2 == 0)
  int c1, c2;
  const __bf16* mask;    // optional (c2 == 0): a1 counts only where mask > 0
  const __bf16* w;       // weights [N][Kp], K = 27 (c1 + c2)
  int Kp;
  const float* bias;     // optional
  int relu;
  __bf16* o1;            // output channels [0, n1)
  __bf16* o2;            // output channels [n1, N)
  int n1;
  int mirror;            // taps mirrored (data gradient)
};

__host__ __device__ static inline size_t conv_tile_lds(int cin) { return (size_t)CT_POS * (cin + 8) * 2; }

template <int NT>
__global__ void __launch_bounds__(256) k_conv3d_tiled(Vol v, ConvIO io) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int Cin = io.c1 + io.c2, N = NT * 16, CinP = Cin + 8;
  __bf16* tin = reinterpret_cast<__bf16*>(smem_raw);                  // [CT_POS][CinP]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_w = (v.W + CT_W - 1) / CT_W, tiles_h = (v.H + CT_H - 1) / CT_H;
  const int w0 = (blockIdx.x % tiles_w) * CT_W;
  const int h0 = ((blockIdx.x / tiles_w) % tiles_h) * CT_H;
  const int d0 = (blockIdx.x / (tiles_w * tiles_h)) * CT_D;
  // stage the input tile with halo (zero outside the volume), 8 channels per load
  const int CG = Cin / 8;
  for (int idx = tid; idx < CT_POS * CG; idx += 256) {
    const int pos = idx / CG, g = idx - pos * CG;
    const int pw = pos % CT_HW, ph = (pos / CT_HW) % CT_HH, pd = pos / (CT_HW * CT_HH);
    const int ww = w0 - 1 + pw, hh = h0 - 1 + ph, dd = d0 - 1 + pd;
    nbf16x8 val = nbf16x8{};
    if (ww >= 0 && ww < v.W && hh >= 0 && hh < v.H && dd >= 0 && dd < v.D) {
      const size_t q = ((size_t)dd * v.H + hh) * v.W + ww;
      const int c = 8 * g;
      if (c < io.c1) {
        val = *reinterpret_cast<const nbf16x8*>(io.a1 + q * io.c1 + c);
        if (io.mask) {
          const nbf16x8 mk = *reinterpret_cast<const nbf16x8*>(io.mask + q * io.c1 + c);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (!((float)mk[e] > 0.f)) val[e] = (__bf16)0.f;
        }
      } else {
        val = *reinterpret_cast<const nbf16x8*>(io.a2 + q * io.c2 + (c - io.c1));
      }
    }
    *reinterpret_cast<nbf16x8*>(tin + (size_t)pos * CinP + 8 * g) = val;
  }
  const int m = lane & 15, kq = lane >> 4;
  // this wavefront's CT_RPW position rows: (h, d) = (mt % CT_H, mt / CT_H), w = w0 + m
  int base[CT_RPW];
#pragma unroll
  for (int r = 0; r < CT_RPW; ++r) {
    const int mt = CT_RPW * wave + r;
    base[r] = ((mt / CT_H + 1) * CT_HH + (mt % CT_H + 1)) * CT_HW + (m + 1);
  }
  const int sgn = io.mirror ? -1 : 1;
  KPos kp{0, 0, 0, 0, 0};
  kp.advance(8 * kq, Cin);
  nf32x4 acc[CT_RPW][NT];
#pragma unroll
  for (int r = 0; r < CT_RPW; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = nf32x4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();  // the tile is staged
  // K loop: A from the LDS tile, B (weights, shared by every workgroup and so
  // cache resident) straight from global memory.  Both operands of step t + 1
  // are loaded while the matrix instructions of step t run (two operand sets,
  // alternating).  The loads are unconditional (past the last step they read
  // the last step's weights and a zero A), so the loop body is straight-line code
  // and each step waits only for its own operands, not for the next step's loads.
  const int nsteps = io.Kp / 32;
  const int last_kb = 32 * (nsteps - 1);
  const __bf16* wrow[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wrow[t] = io.w + (size_t)(16 * t + m) * io.Kp + 8 * kq;
  int kb = 0;
  auto load = [&](nbf16x8 (&b)[NT], nbf16x8 (&a)[CT_RPW]) {
    const int kbc = kb < last_kb ? kb : last_kb;
#pragma unroll
    for (int t = 0; t < NT; ++t) b[t] = *reinterpret_cast<const nbf16x8*>(wrow[t] + kbc);
    kb += 32;
    const bool kin = kp.tap < 27;  // K padding past the 27 taps reads as zero
    const int off = kin ? ((sgn * (kp.td - 1)) * CT_HH + sgn * (kp.th - 1)) * CT_HW + sgn * (kp.tw - 1) : 0;
    const int ci = kin ? kp.ci : 0;
#pragma unroll
    for (int r = 0; r < CT_RPW; ++r) {
      const nbf16x8 x = *reinterpret_cast<const nbf16x8*>(tin + (size_t)(base[r] + off) * CinP + ci);
      a[r] = kin ? x : nbf16x8{};
    }
    kp.advance(32, Cin);
  };
  auto compute = [&](const nbf16x8 (&b)[NT], const nbf16x8 (&a)[CT_RPW]) {
#pragma unroll
    for (int r = 0; r < CT_RPW; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], b[t], acc[r][t], 0, 0, 0);
  };
  nbf16x8 bx[NT], by[NT], ax[CT_RPW], ay[CT_RPW];
  load(bx, ax);
  int st = 0;
  for (; st + 1 < nsteps; st += 2) {
    load(by, ay);  // step st + 1
    __builtin_amdgcn_sched_barrier(0);
    compute(bx, ax);
    load(bx, ax);  // step st + 2 (a repeat of the last weights when st + 2 == nsteps)
    __builtin_amdgcn_sched_barrier(0);
    compute(by, ay);
  }
  if (st < nsteps) compute(bx, ax);
  // write: row r, lane (m = channel within the tile, kq) holds positions w0 + 4 kq + e
#pragma unroll
  for (int r = 0; r < CT_RPW; ++r) {
    const int mt = CT_RPW * wave + r;
    const int hh = h0 + mt % CT_H, dd = d0 + mt / CT_H;
    if (hh >= v.H || dd >= v.D) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = 16 * t + m;
      const float bb = io.bias ? io.bias[co] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ww = w0 + 4 * kq + e;
        if (ww >= v.W) continue;
        const size_t q = ((size_t)dd * v.H + hh) * v.W + ww;
        float y = acc[r][t][e] + bb;
        if (io.relu) y = y > 0.f ? y : 0.f;
        if (co < io.n1)
          io.o1[q * io.n1 + co] = (__bf16)y;
        else
          io.o2[q * (N - io.n1) + (co - io.n1)] = (__bf16)y;
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
// Pooling, upsampling and their transposes move eight channels (16 bytes) per
// thread with 32-bit index arithmetic; per channel the sums run in the same order
// (the eight children in a = 0..7 order) as a one-channel-per-thread loop.
__global__ void k_pool2(Vol v, int C, const __bf16* __restrict__ X, __bf16* __restrict__ Y) {
  const int Do = v.D / 2, Ho = v.H / 2, Wo = v.W / 2, CG = C / 8;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Do * Ho * Wo * CG) return;
  const int po = i / CG, c = 8 * (i - po * CG);
  const int w = po % Wo, t = po / Wo, h = t % Ho, d = t / Ho;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 8; ++a) {
    const int dd = 2 * d + (a >> 2), hh = 2 * h + ((a >> 1) & 1), ww = 2 * w + (a & 1);
    const nbf16x8 x = *reinterpret_cast<const nbf16x8*>(X + ((dd * v.H + hh) * v.W + ww) * C + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += (float)x[e];
  }
  nbf16x8 y;
#pragma unroll
  for (int e = 0; e < 8; ++e) y[e] = (__bf16)(0.125f * s[e]);
  *reinterpret_cast<nbf16x8*>(Y + po * C + c) = y;
}

__global__ void k_pool2_bwd(Vol v, int C, const __bf16* __restrict__ dY, __bf16* __restrict__ dX) {
  const int CG = C / 8, Ho = v.H / 2, Wo = v.W / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.D * v.H * v.W * CG) return;
  const int p = i / CG, c = 8 * (i - p * CG);
  const int w = p % v.W, t = p / v.W, h = t % v.H, d = t / v.H;
  const nbf16x8 g = *reinterpret_cast<const nbf16x8*>(dY + (((d / 2) * Ho + h / 2) * Wo + w / 2) * C + c);
  nbf16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = (__bf16)(0.125f * (float)g[e]);
  *reinterpret_cast<nbf16x8*>(dX + p * C + c) = o;
}

// Nearest-neighbour upsampling x2 (dims of the output).
__global__ void k_up2(Vol v, int C, const __bf16* __restrict__ X, __bf16* __restrict__ Y) {
  const int CG = C / 8, Hi = v.H / 2, Wi = v.W / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.D * v.H * v.W * CG) return;
  const int p = i / CG, c = 8 * (i - p * CG);
  const int w = p % v.W, t = p / v.W, h = t % v.H, d = t / v.H;
  *reinterpret_cast<nbf16x8*>(Y + p * C + c) =
      *reinterpret_cast<const nbf16x8*>(X + (((d / 2) * Hi + h / 2) * Wi + w / 2) * C + c);
}

__global__ void k_up2_bwd(Vol v, int C, const __bf16* __restrict__ dY, __bf16* __restrict__ dX) {
  const int Di = v.D / 2, Hi = v.H / 2, Wi = v.W / 2, CG = C / 8;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Di * Hi * Wi * CG) return;
  const int po = i / CG, c = 8 * (i - po * CG);
  const int w = po % Wi, t = po / Wi, h = t % Hi, d = t / Hi;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 8; ++a) {
    const int dd = 2 * d + (a >> 2), hh = 2 * h + ((a >> 1) & 1), ww = 2 * w + (a & 1);
    const nbf16x8 g = *reinterpret_cast<const nbf16x8*>(dY + ((dd * v.H + hh) * v.W + ww) * C + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += (float)g[e];
  }
  nbf16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = (__bf16)s[e];
  *reinterpret_cast<nbf16x8*>(dX + po * C + c) = o;
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
                                                    float inv_count, float lam, float tau, float* __restrict__ gp,
                                                    float* __restrict__ gr, float* __restrict__ part) {
  __shared__ float red[256];
  int p = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (p < P) {
    float m = mask[p];
    float e = pred[p] - target[p] * tscale[0];
    float ae = fabsf(e);
    float er = resid[p] - ae;
    if (tau > 0.f) {
      // pinball loss of the tau-quantile of |e|: u (tau - [u < 0]), u = |e| - resid
      const float below = er > 0.f ? 1.f : 0.f;  // u < 0
      l = m * (e * e - lam * er * (tau - below)) * inv_count;
      gr[p] = m * lam * (below - tau) * inv_count;
    } else {
      l = m * (e * e + lam * er * er) * inv_count;
      gr[p] = m * 2.f * lam * er * inv_count;
    }
    gp[p] = m * 2.f * e * inv_count;
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
// out = a + b in groups of eight (16 bytes), the tail one at a time.
__global__ void k_add_bf16(size_t n, const __bf16* __restrict__ a, const __bf16* __restrict__ b,
                           __bf16* __restrict__ out) {
  const size_t i = 8 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 8 <= n) {
    const nbf16x8 x = *reinterpret_cast<const nbf16x8*>(a + i), y = *reinterpret_cast<const nbf16x8*>(b + i);
    nbf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (__bf16)((float)x[e] + (float)y[e]);
    *reinterpret_cast<nbf16x8*>(out + i) = o;
  } else {
    for (size_t j = i; j < n; ++j) out[j] = (__bf16)((float)a[j] + (float)b[j]);
  }
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

template <int NT>
static hipError_t launch_tiled(Vol v, ConvIO io, hipStream_t s) {
  const size_t lds = conv_tile_lds(io.c1 + io.c2);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  {
    hipError_t e = ensure_lds_limit((const void*)k_conv3d_tiled<NT>, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  const unsigned tiles = (unsigned)(((v.W + CT_W - 1) / CT_W) * ((v.H + CT_H - 1) / CT_H) * ((v.D + CT_D - 1) / CT_D));
  hipLaunchKernelGGL(k_conv3d_tiled<NT>, dim3(tiles), dim3(256), lds, s, v, io);
  return hipGetLastError();
}

static hipError_t launch_tiled_n(Vol v, const ConvIO& io, int n, hipStream_t s) {
  switch (n / 16) {
    case 1: return launch_tiled<1>(v, io, s);
    case 2: return launch_tiled<2>(v, io, s);
    case 3: return launch_tiled<3>(v, io, s);
    case 4: return launch_tiled<4>(v, io, s);
    case 6: return launch_tiled<6>(v, io, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv3d_fwd(Vol v, int C1, int C2, const __bf16* X1, const __bf16* X2, int Cout,
                             const __bf16* Wt, int Kp, const float* bias, int relu, __bf16* Y, hipStream_t s) {
  ConvIO io{X1, X2, C1, C2, nullptr, Wt, Kp, bias, relu, Y, nullptr, Cout, 0};
  return launch_tiled_n(v, io, Cout, s);
}

hipError_t launch_conv3d_dgrad(Vol v, int Cout, const __bf16* dY, const __bf16* Yact, int Cin, const __bf16* Wd,
                               int Kp, int C1, __bf16* dX1, __bf16* dX2, hipStream_t s) {
  ConvIO io{dY, nullptr, Cout, 0, Yact, Wd, Kp, nullptr, 0, dX1, dX2, C1, 1};
  return launch_tiled_n(v, io, Cin, s);
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

// (v: the full-resolution volume; C a multiple of 8; the element count within 32 bits)
hipError_t launch_pool2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s) {
  const size_t n = (size_t)v.D * v.H * v.W * C;
  if (C % 8 != 0 || n > 0x7fffffffULL) return hipErrorInvalidValue;
  if (!backward)
    hipLaunchKernelGGL(k_pool2, dim3(nblk(n / 64)), dim3(256), 0, s, v, C, X, Y);
  else
    hipLaunchKernelGGL(k_pool2_bwd, dim3(nblk(n / 8)), dim3(256), 0, s, v, C, X, Y);
  return hipGetLastError();
}

hipError_t launch_up2(Vol v, int C, const __bf16* X, __bf16* Y, int backward, hipStream_t s) {
  const size_t n = (size_t)v.D * v.H * v.W * C;
  if (C % 8 != 0 || n > 0x7fffffffULL) return hipErrorInvalidValue;
  if (!backward)
    hipLaunchKernelGGL(k_up2, dim3(nblk(n / 8)), dim3(256), 0, s, v, C, X, Y);
  else
    hipLaunchKernelGGL(k_up2_bwd, dim3(nblk(n / 64)), dim3(256), 0, s, v, C, X, Y);
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
                             const float* mask, float inv_count, float lam, float tau, float* gp, float* gr,
                             float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_train_loss, dim3(nblk(P)), dim3(256), 0, s, P, pred, resid, target, tscale, mask, inv_count,
                     lam, tau, gp, gr, part);
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
  hipLaunchKernelGGL(k_add_bf16, dim3(nblk((n + 7) / 8)), dim3(256), 0, s, n, a, b, out);
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
