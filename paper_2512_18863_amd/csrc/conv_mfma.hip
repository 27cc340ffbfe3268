// conv_mfma.hip — the per-plane lateral convolution (arXiv:2512.18863 §2.2.6,
// Eq. 8) on the CDNA4 matrix cores.
//
// For one plane, out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q] (zero padded).  Fixing
// the tap row p, the sum over q is a product with a banded Toeplitz matrix:
//   out[i][j0..j0+15] += in[i+p][j0-h .. j0+15+h] * T_p,  T_p[c][n] = K[p][c - h - n],
// so a 16 x 16 output tile is a GEMM with K-dimension 16 + 2h over input columns.
// The Toeplitz operand depends only on (p, column step), never on the tile, so a
// wavefront keeps it in registers and streams the input rows of all its tiles past
// it.  A workgroup (4 wavefronts) owns a region of up to 6 x 6 tiles (96 x 96
// outputs) of one (control point, plane); the input region with its halo and the
// plane's taps are staged in LDS once.
//
//   FP32: v_mfma_f32_16x16x4_f32.  Tap rows p and -p are equal (the kernel is
//         radially symmetric), so rows i+p and i-p are added before the product
//         and only h+1 tap rows are multiplied (row 0 with halved taps).
//   BF16: v_mfma_f32_16x16x32_bf16, operands rounded to BF16 (round to nearest
//         even), FP32 accumulation; all n tap rows.
#include "taps.hpp"

namespace pdrt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MT = 16;      // MFMA output tile edge
constexpr int RMAX = 6;     // region edge in tiles

struct RegionShape {
  int TI, TJ;               // tiles per region along u (rows) and v (columns)
  int regions_i, regions_j;
};

static RegionShape region_shape(int Nu, int Nv, int rmax) {
  RegionShape r;
  int ti = (Nu + MT - 1) / MT, tj = (Nv + MT - 1) / MT;
  r.TI = ti < rmax ? ti : rmax;
  r.TJ = tj < rmax ? tj : rmax;
  r.regions_i = (ti + r.TI - 1) / r.TI;
  r.regions_j = (tj + r.TJ - 1) / r.TJ;
  return r;
}

// Row pitch (elements) congruent to 4 mod 32 so that the 16 rows x 4 columns an
// FP32 A-fragment touches fall in distinct LDS banks.
static int pitch_f32(int cols) { return ((cols + 27) / 32) * 32 + 4; }

// ------------------------------------------------------------------ FP32

struct F32Shape {
  int S;       // K-steps of 4 input columns: ceil((16 + 2h) / 4)
  int E;       // extended tap row length: 4 S + 16
  int rows, pitch;
};

static F32Shape f32_shape(int h, const RegionShape& r) {
  F32Shape s;
  s.S = (MT + 2 * h + 3) / 4;
  s.E = 4 * s.S + 16;
  s.rows = MT * r.TI + 2 * h;
  s.pitch = pitch_f32(MT * r.TJ + 2 * h + 4);
  return s;
}

static size_t f32_lds(const Geo<float>& g, const F32Shape& fs) {
  return sizeof(float) * ((size_t)fs.rows * fs.pitch + (size_t)(g.h + 1) * fs.E);
}

template <int TPW>
__global__ void __launch_bounds__(256) k_conv_mfma_f32(Geo<float> g, RegionShape rs, F32Shape fs,
                                                       const float* __restrict__ zca, const float* __restrict__ in,
                                                       float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  const int h = g.h;
  const int rows = fs.rows, pitch = fs.pitch, E = fs.E, S = fs.S;
  float* tile = lds;
  float* kx = lds + rows * pitch;  // (h + 1) x E, zero outside |q| <= h, row 0 halved
  const int k = blockIdx.y, b = blockIdx.z;
  const int I0 = (blockIdx.x / rs.regions_j) * rs.TI * MT;
  const int J0 = (blockIdx.x % rs.regions_j) * rs.TJ * MT;
  const int plane = g.Nu * g.Nv;
  const float* src = in + ((size_t)b * g.Nk + k) * plane;
  const int tid = threadIdx.x;

  for (int idx = tid; idx < rows * pitch; idx += 256) {
    int rr = idx / pitch, cc = idx - rr * pitch;
    int i = I0 - h + rr, j = J0 - h + cc;
    float v = 0.f;
    if (i >= 0 && i < g.Nu && j >= 0 && j < g.Nv && cc < MT * rs.TJ + 2 * h) v = src[(size_t)i * g.Nv + j];
    tile[idx] = v;
  }
  {
    TapParams<float> tp = tap_params(g, k, zca[(size_t)b * g.Nk + k]);
    const int off = h + 15;
    for (int idx = tid; idx < (h + 1) * E; idx += 256) {
      int p = idx / E, c = idx - p * E;
      int q = c - off;
      float v = 0.f;
      if (q >= -h && q <= h) {
        v = tap_value(tp, p, q);
        if (p == 0) v *= 0.5f;
      }
      kx[idx] = v;
    }
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kk = lane >> 4;
  int rowbase[TPW], colbase[TPW];
  bool active[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = wave + 4 * q;
    int ti = t / rs.TJ, tj = t - ti * rs.TJ;
    active[q] = t < rs.TI * rs.TJ && I0 + MT * ti < g.Nu && J0 + MT * tj < g.Nv;
    rowbase[q] = (MT * ti + m + h) * pitch;
    colbase[q] = MT * tj + kk;
  }
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int p = 0; p <= h; ++p) {
    const float* krow = kx + p * E + 15 + kk - m;
    const int up = p * pitch;
    for (int s = 0; s < S; ++s) {
      float bv = krow[4 * s];
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (active[q]) {
          const float* a0 = tile + rowbase[q] + colbase[q] + 4 * s;
          float av = a0[up] + a0[-up];
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
  }

  float* dst = out + ((size_t)b * g.Nk + k) * plane;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (!active[q]) continue;
    int t = wave + 4 * q;
    int ti = t / rs.TJ, tj = t - ti * rs.TJ;
    int j = J0 + MT * tj + m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i = I0 + MT * ti + 4 * kk + r;
      if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[q][r];
    }
  }
}

template <int TPW>
static hipError_t launch_f32_tpw(const Geo<float>& g, const RegionShape& rs, const F32Shape& fs, int nb,
                                 const float* z, const float* in, float* out, hipStream_t s) {
  size_t lds = f32_lds(g, fs);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_mfma_f32<TPW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  dim3 grid(rs.regions_i * rs.regions_j, g.Nk, nb);
  hipLaunchKernelGGL(k_conv_mfma_f32<TPW>, grid, dim3(256), lds, s, g, rs, fs, z, in, out);
  return hipGetLastError();
}

hipError_t launch_conv_mfma_f32(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                hipStream_t s) {
  // the largest region (in tiles) whose LDS image fits
  RegionShape rs;
  F32Shape fs;
  for (int rmax = RMAX; rmax >= 1; --rmax) {
    rs = region_shape(g.Nu, g.Nv, rmax);
    fs = f32_shape(g.h, rs);
    if (f32_lds(g, fs) <= 160 * 1024) break;
  }
  int tpw = (rs.TI * rs.TJ + 3) / 4;
  if (tpw <= 1) return launch_f32_tpw<1>(g, rs, fs, nb, z, in, out, s);
  if (tpw <= 2) return launch_f32_tpw<2>(g, rs, fs, nb, z, in, out, s);
  if (tpw <= 3) return launch_f32_tpw<3>(g, rs, fs, nb, z, in, out, s);
  if (tpw <= 4) return launch_f32_tpw<4>(g, rs, fs, nb, z, in, out, s);
  if (tpw <= 6) return launch_f32_tpw<6>(g, rs, fs, nb, z, in, out, s);
  return launch_f32_tpw<9>(g, rs, fs, nb, z, in, out, s);
}

// ------------------------------------------------------------------ BF16

struct BF16Shape {
  int S;       // K-steps of 32 input columns: ceil((16 + 2h) / 32)
  int E;       // extended tap row length: 32 S + 16
  int rows, pitch;
};

static BF16Shape bf16_shape(int h, const RegionShape& r) {
  BF16Shape s;
  s.S = (MT + 2 * h + 31) / 32;
  s.E = 32 * s.S + 16;
  s.rows = MT * r.TI + 2 * h;
  int cols = MT * r.TJ + 32 * s.S;  // covers the last K-step's overrun
  s.pitch = ((cols + 7) / 8) * 8 + 8;
  return s;
}

static size_t bf16_lds(const Geo<float>& g, const BF16Shape& bs) {
  size_t tile_bytes = ((size_t)bs.rows * bs.pitch * 2 + 15) & ~(size_t)15;
  return tile_bytes + sizeof(float) * (size_t)(g.h + 1) * bs.E;
}

template <int TPW>
__global__ void __launch_bounds__(256) k_conv_mfma_bf16(Geo<float> g, RegionShape rs, BF16Shape bs,
                                                        const float* __restrict__ zca, const float* __restrict__ in,
                                                        float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int h = g.h;
  const int rows = bs.rows, pitch = bs.pitch, E = bs.E, S = bs.S;
  __bf16* tile = reinterpret_cast<__bf16*>(smem_raw);
  size_t tile_bytes = ((size_t)rows * pitch * sizeof(__bf16) + 15) & ~(size_t)15;
  float* kx = reinterpret_cast<float*>(smem_raw + tile_bytes);  // (h + 1) x E taps, zero outside |q| <= h
  const int k = blockIdx.y, b = blockIdx.z;
  const int I0 = (blockIdx.x / rs.regions_j) * rs.TI * MT;
  const int J0 = (blockIdx.x % rs.regions_j) * rs.TJ * MT;
  const int plane = g.Nu * g.Nv;
  const float* src = in + ((size_t)b * g.Nk + k) * plane;
  const int tid = threadIdx.x;

  for (int idx = tid; idx < rows * pitch; idx += 256) {
    int rr = idx / pitch, cc = idx - rr * pitch;
    int i = I0 - h + rr, j = J0 - h + cc;
    float v = 0.f;
    if (i >= 0 && i < g.Nu && j >= 0 && j < g.Nv && cc < MT * rs.TJ + 2 * h) v = src[(size_t)i * g.Nv + j];
    tile[idx] = (__bf16)v;
  }
  {
    TapParams<float> tp = tap_params(g, k, zca[(size_t)b * g.Nk + k]);
    const int off = h + 15;
    for (int idx = tid; idx < (h + 1) * E; idx += 256) {
      int p = idx / E, c = idx - p * E;
      int q = c - off;
      kx[idx] = (q >= -h && q <= h) ? tap_value(tp, p, q) : 0.f;
    }
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kq = lane >> 4;  // A: row m, K-columns 8 kq .. 8 kq + 7
  int rowbase[TPW], colbase[TPW];
  bool active[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = wave + 4 * q;
    int ti = t / rs.TJ, tj = t - ti * rs.TJ;
    active[q] = t < rs.TI * rs.TJ && I0 + MT * ti < g.Nu && J0 + MT * tj < g.Nv;
    rowbase[q] = (MT * ti + m + h) * pitch;
    colbase[q] = MT * tj + 8 * kq;
  }
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int p = -h; p <= h; ++p) {
    const int ap = p < 0 ? -p : p;
    // B[kk][n] = T_p[c0 + kk][j0 + n] = K[p][c0 + kk - j0 - n], c0 - j0 = 32 s - h;
    // lane (n = m, kk = 8 kq + e) reads extended index 32 s + 8 kq + e - m + 15.
    const float* krow = kx + ap * E + 15 + 8 * kq - m;
    const int up = p * pitch;
    for (int s = 0; s < S; ++s) {
      bf16x8 bv;
#pragma unroll
      for (int e = 0; e < 8; ++e) bv[e] = (__bf16)krow[32 * s + e];
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (active[q]) {
          const bf16x8 av = *reinterpret_cast<const bf16x8*>(tile + rowbase[q] + up + colbase[q] + 32 * s);
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
  }

  float* dst = out + ((size_t)b * g.Nk + k) * plane;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (!active[q]) continue;
    int t = wave + 4 * q;
    int ti = t / rs.TJ, tj = t - ti * rs.TJ;
    int j = J0 + MT * tj + m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i = I0 + MT * ti + 4 * kq + r;
      if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[q][r];
    }
  }
}

template <int TPW>
static hipError_t launch_bf16_tpw(const Geo<float>& g, const RegionShape& rs, const BF16Shape& bs, int nb,
                                  const float* z, const float* in, float* out, hipStream_t s) {
  size_t lds = bf16_lds(g, bs);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_mfma_bf16<TPW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  dim3 grid(rs.regions_i * rs.regions_j, g.Nk, nb);
  hipLaunchKernelGGL(k_conv_mfma_bf16<TPW>, grid, dim3(256), lds, s, g, rs, bs, z, in, out);
  return hipGetLastError();
}

hipError_t launch_conv_mfma_bf16(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                 hipStream_t s) {
  RegionShape rs;
  BF16Shape bs;
  for (int rmax = RMAX; rmax >= 1; --rmax) {
    rs = region_shape(g.Nu, g.Nv, rmax);
    bs = bf16_shape(g.h, rs);
    if (bf16_lds(g, bs) <= 160 * 1024) break;
  }
  int tpw = (rs.TI * rs.TJ + 3) / 4;
  if (tpw <= 1) return launch_bf16_tpw<1>(g, rs, bs, nb, z, in, out, s);
  if (tpw <= 2) return launch_bf16_tpw<2>(g, rs, bs, nb, z, in, out, s);
  if (tpw <= 3) return launch_bf16_tpw<3>(g, rs, bs, nb, z, in, out, s);
  if (tpw <= 4) return launch_bf16_tpw<4>(g, rs, bs, nb, z, in, out, s);
  if (tpw <= 6) return launch_bf16_tpw<6>(g, rs, bs, nb, z, in, out, s);
  return launch_bf16_tpw<9>(g, rs, bs, nb, z, in, out, s);
}

}  // namespace pdrt
