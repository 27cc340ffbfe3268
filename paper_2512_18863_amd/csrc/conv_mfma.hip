// conv_mfma.hip — the per-plane lateral convolution (arXiv:2512.18863 §2.2.6,
// Eq. 8) on the CDNA4 matrix cores.
//
// For one plane, out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q] (zero padded).  Fixing
// the tap row p, the sum over q is a product with a banded Toeplitz matrix:
//   out[i][j0..j0+15] += in[i+p][j0-h .. j0+15+h] * T_p,  T_p[c][n] = K[p][c - h - n],
// so a 16 x 16 output tile is a GEMM with K-dimension 16 + 2h over input columns.
// The Toeplitz operand depends only on (p, column step), never on the tile, so a
// wavefront loads it once per step and streams the input rows of all its tiles
// past it.  A workgroup owns a region of up to 6 x 6 tiles (96 x 96 outputs) of
// one (control point, plane); the input region with its halo and the plane's
// taps are staged in LDS once, then NW wavefronts each run TPW tiles.  The inner
// loop is branch free and software pipelined: the operands of step t+1 are
// loaded from LDS before the matrix instructions of step t are issued.
//
//   FP32: v_mfma_f32_16x16x4_f32.  Tap rows p and -p are equal (the kernel is
//         radially symmetric), so rows i+p and i-p are added before the product
//         and only h+1 tap rows are multiplied (row 0 with halved taps).
//   BF16: v_mfma_f32_32x32x16_bf16, operands rounded to BF16 (round to nearest
//         even), FP32 accumulation; all n tap rows (see the BF16 section).  Each
//         lane's eight Toeplitz entries are one aligned 16-byte LDS read from one
//         of eight copies of the tap row, shifted so that every lane's run starts
//         on a 16-byte boundary.
#include "taps.hpp"

namespace pdrt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MT = 16;      // MFMA output tile edge
constexpr int RMAX = 6;     // region edge in tiles
constexpr size_t LDS_MAX = 160 * 1024;

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

// Unique taps K[p][q], 0 <= p, q <= h, of the plane into `kq` ((h+1) x (h+1)).
__device__ __forceinline__ void unique_taps(const Geo<float>& g, int k, float zk, float* kq, int tid, int nt) {
  TapParams<float> tp = tap_params(g, k, zk);
  const int h1 = g.h + 1;
  for (int idx = tid; idx < h1 * h1; idx += nt) kq[idx] = tap_value(tp, idx / h1, idx % h1);
}

// Stage the input region (rows I0-h .., columns J0-h ..) of one plane; zero
// outside the plane and beyond `cols_valid`.
template <typename E>
__device__ __forceinline__ void stage_tile(const Geo<float>& g, const float* __restrict__ src, int I0, int J0,
                                           int rows, int pitch, int cols_valid, E* tile, int tid, int nt) {
  const int h = g.h;
  for (int idx = tid; idx < rows * pitch; idx += nt) {
    int rr = idx / pitch, cc = idx - rr * pitch;
    int i = I0 - h + rr, j = J0 - h + cc;
    float v = 0.f;
    if (i >= 0 && i < g.Nu && j >= 0 && j < g.Nv && cc < cols_valid) v = src[(size_t)i * g.Nv + j];
    tile[idx] = (E)v;
  }
}

template <int TPW>
__device__ __forceinline__ void store_tiles(const Geo<float>& g, const RegionShape& rs, int NW, int wave, int I0,
                                            int J0, int lane, const f32x4 (&acc)[TPW], const bool (&active)[TPW],
                                            float* dst) {
  const int m = lane & 15, r4 = lane >> 4;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (!active[q]) continue;
    int t = wave + NW * q;
    int ti = t / rs.TJ, tj = t - ti * rs.TJ;
    int j = J0 + MT * tj + m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i = I0 + MT * ti + 4 * r4 + r;
      if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[q][r];
    }
  }
}

// ------------------------------------------------------------------ FP32
//
// v_mfma_f32_16x16x4_f32 on 16 x 16 tiles, tap rows folded (rows i+p and i-p
// added before the product).  The MFMA's K index may map to input columns in
// any order as long as both operands agree; here super-step u covers 16 input
// columns and its four instructions s = 0..3 use column 16 u + 4 k + s for K
// index k, so lane k's four A values of a super-step are one 16-byte LDS read.

typedef float f32x4v __attribute__((ext_vector_type(4)));

struct F32Shape {
  int SS;      // super-steps of 16 input columns: ceil((16 + 2h) / 16)
  int E;       // extended tap row length: 16 SS + 16
  int rows, pitch;
};

// Row pitch (elements) congruent to 4 mod 32.
static int pitch_f32(int cols) { return ((cols + 27) / 32) * 32 + 4; }

static F32Shape f32_shape(int h, const RegionShape& r) {
  F32Shape s;
  s.SS = (MT + 2 * h + 15) / 16;
  s.E = 16 * s.SS + 16;
  s.rows = MT * r.TI + 2 * h;
  s.pitch = pitch_f32(MT * r.TJ + 16 * s.SS);
  return s;
}

static size_t f32_lds(int h, const F32Shape& fs) {
  return sizeof(float) * ((size_t)fs.rows * fs.pitch + (size_t)(h + 1) * fs.E + (size_t)(h + 1) * (h + 1));
}

template <int NW, int TPW>
__global__ void __launch_bounds__(64 * NW) k_conv_mfma_f32(Geo<float> g, RegionShape rs, F32Shape fs,
                                                           const float* __restrict__ zca,
                                                           const float* __restrict__ in, float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int NT = 64 * NW;
  const int h = g.h;
  const int rows = fs.rows, pitch = fs.pitch, E = fs.E, SS = fs.SS;
  float* tile = lds;
  float* kx = lds + rows * pitch;  // (h + 1) x E, zero outside |q| <= h, row 0 halved
  float* kq = kx + (h + 1) * E;    // (h + 1) x (h + 1) unique taps
  const int k = blockIdx.y, b = blockIdx.z;
  const int I0 = (blockIdx.x / rs.regions_j) * rs.TI * MT;
  const int J0 = (blockIdx.x % rs.regions_j) * rs.TJ * MT;
  const int plane = g.Nu * g.Nv;
  const int tid = threadIdx.x;

  stage_tile(g, in + ((size_t)b * g.Nk + k) * plane, I0, J0, rows, pitch, MT * rs.TJ + 2 * h, tile, tid, NT);
  unique_taps(g, k, zca[(size_t)b * g.Nk + k], kq, tid, NT);
  __syncthreads();
  const int off = h + 15;
  for (int idx = tid; idx < (h + 1) * E; idx += NT) {
    int p = idx / E, c = idx - p * E;
    int q = c - off;
    float v = 0.f;
    if (q >= -h && q <= h) v = kq[p * (h + 1) + (q < 0 ? -q : q)] * (p == 0 ? 0.5f : 1.f);
    kx[idx] = v;
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kk = lane >> 4;
  const float* abase[TPW];
  bool active[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = wave + NW * q;
    bool valid = t < rs.TI * rs.TJ;
    int ti = valid ? t / rs.TJ : 0, tj = valid ? t - (t / rs.TJ) * rs.TJ : 0;
    active[q] = valid && I0 + MT * ti < g.Nu && J0 + MT * tj < g.Nv;
    abase[q] = tile + (MT * ti + m + h) * pitch + MT * tj + 4 * kk;
  }
  // B[k][n] of instruction s in super-step u = K[p][16 u + 4 k + s - h - n] = kx[p][16 u + 4 k + s + 15 - n]
  const float* bbase = kx + 4 * kk + 15 - m;
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int total = (h + 1) * SS;
  f32x4v an0[TPW], an1[TPW];
  float bn[4];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    an0[q] = *reinterpret_cast<const f32x4v*>(abase[q]);
    an1[q] = an0[q];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) bn[e] = bbase[e];
  int p = 0, u = 0;
  for (int it = 0; it < total; ++it) {
    f32x4v ac[TPW];
    float bc[4];
#pragma unroll
    for (int q = 0; q < TPW; ++q) ac[q] = an0[q] + an1[q];
#pragma unroll
    for (int e = 0; e < 4; ++e) bc[e] = bn[e];
    if (++u == SS) {
      u = 0;
      ++p;
    }
    if (it + 1 < total) {
      const int op = p * pitch + 16 * u, om = 16 * u - p * pitch;
      const float* br = bbase + p * E + 16 * u;
#pragma unroll
      for (int e = 0; e < 4; ++e) bn[e] = br[e];
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        an0[q] = *reinterpret_cast<const f32x4v*>(abase[q] + op);
        an1[q] = *reinterpret_cast<const f32x4v*>(abase[q] + om);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int q = 0; q < TPW; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[q][e], bc[e], acc[q], 0, 0, 0);
  }
  store_tiles<TPW>(g, rs, NW, wave, I0, J0, lane, acc, active, out + ((size_t)b * g.Nk + k) * plane);
}

// ------------------------------------------------------------------ BF16
//
// v_mfma_f32_32x32x16_bf16 on 32 x 32 output tiles.  A wavefront owns one strip
// of RJ tiles side by side (32 rows x 32 RJ columns) and a quarter of the tap
// rows p; its four partial sums are added in LDS at the end (fixed order).  For
// tile t at K-step s the input column block is a = 2 t + s (16 columns each), so
// per tap row the strip loads 2 RJ + S - 2 distinct A fragments and S Toeplitz
// fragments and issues RJ * S matrix instructions: each 1 KB A fragment feeds up
// to RJ instructions.

constexpr int BQ = 4;  // wavefronts sharing one strip (tap rows split in quarters)

struct BF16Shape {
  int S;       // K-steps of 16 input columns: ceil((32 + 2h) / 16)
  int CL;      // length of one shifted tap-row copy: 16 S + 40 (a multiple of 8)
  int rows, pitch;
  int RI, RJ;  // strips per region, 32-wide tiles per strip
  int regions_i, regions_j;
};

static BF16Shape bf16_shape(int Nu, int Nv, int h, int rmax) {
  BF16Shape s;
  int ti = (Nu + 31) / 32, tj = (Nv + 31) / 32;
  s.RI = ti < rmax ? ti : rmax;
  s.RJ = tj < 3 ? tj : 3;
  s.regions_i = (ti + s.RI - 1) / s.RI;
  s.regions_j = (tj + s.RJ - 1) / s.RJ;
  s.S = (32 + 2 * h + 15) / 16;
  s.CL = 16 * s.S + 40;
  s.rows = 32 * s.RI + 2 * h;
  s.pitch = 16 * (2 * s.RJ + s.S - 2) + 8;
  return s;
}

__host__ __device__ static size_t bf16_tile_bytes(const BF16Shape& bs) {
  return ((size_t)bs.rows * bs.pitch * 2 + 15) & ~(size_t)15;
}
__host__ __device__ static size_t bf16_copy_bytes(int h, const BF16Shape& bs) { return (size_t)(h + 1) * 8 * bs.CL * 2; }
static size_t bf16_lds(int h, const BF16Shape& bs) {
  size_t stage = bf16_tile_bytes(bs) + bf16_copy_bytes(h, bs) + sizeof(float) * (size_t)(h + 1) * (h + 1);
  size_t partial = sizeof(float) * (size_t)bs.RI * (BQ - 1) * bs.RJ * 1024;
  return stage > partial ? stage : partial;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int RJ, int SMAX>
__global__ void __launch_bounds__(256 * 3) k_conv_mfma_bf16(Geo<float> g, BF16Shape bs,
                                                            const float* __restrict__ zca,
                                                            const float* __restrict__ in, float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int NT = 64 * BQ * bs.RI;
  const int h = g.h;
  const int rows = bs.rows, pitch = bs.pitch, CL = bs.CL, S = bs.S;
  __bf16* tile = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* bcopy = reinterpret_cast<__bf16*>(smem_raw + bf16_tile_bytes(bs));  // [h+1][8][CL]
  float* kq = reinterpret_cast<float*>(smem_raw + bf16_tile_bytes(bs) + bf16_copy_bytes(h, bs));
  const int k = blockIdx.y, b = blockIdx.z;
  const int I0 = (blockIdx.x / bs.regions_j) * bs.RI * 32;
  const int J0 = (blockIdx.x % bs.regions_j) * RJ * 32;
  const int plane = g.Nu * g.Nv;
  const int tid = threadIdx.x;

  stage_tile(g, in + ((size_t)b * g.Nk + k) * plane, I0, J0, rows, pitch, 32 * RJ + 2 * h, tile, tid, NT);
  unique_taps(g, k, zca[(size_t)b * g.Nk + k], kq, tid, NT);
  __syncthreads();
  // Extended tap row x (x = q + h + 31) stored in copy r at position x + sigma_r,
  // sigma_r = (8 - r) % 8, so that a run starting at x with x % 8 == r is aligned.
  for (int idx = tid; idx < (h + 1) * 8 * CL; idx += NT) {
    int p = idx / (8 * CL), rem = idx - p * 8 * CL;
    int r = rem / CL, y = rem - r * CL;
    int x = y - ((8 - r) & 7);
    int q = x - (h + 31);
    float v = (x >= 0 && q >= -h && q <= h) ? kq[p * (h + 1) + (q < 0 ? -q : q)] : 0.f;
    bcopy[idx] = (__bf16)v;
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int strip = wave / BQ, quarter = wave - strip * BQ;
  const int m = lane & 31, hi = lane >> 5;  // A: row m, K 8 hi .. 8 hi + 7; B: column m
  const __bf16* abase = tile + (32 * strip + m + h) * pitch + 8 * hi;
  // B[kk][n] = K[p][16 s - h + kk - n]: lane (n = m, kk = 8 hi + e) needs extended
  // entries x0 + e, x0 = 16 s + 8 hi + 31 - m, residue r = (31 - m) % 8.
  const int rr = (31 - m) & 7;
  const __bf16* bbase = bcopy + rr * CL + 8 * hi + 31 - m + ((8 - rr) & 7);
  const int n_p = 2 * h + 1, per = (n_p + BQ - 1) / BQ;
  const int p_begin = -h + quarter * per, p_end = min(h + 1, p_begin + per);
  constexpr int NA = 2 * RJ + SMAX - 2;
  const int na = 2 * RJ + S - 2;
  f32x16 acc[RJ];
#pragma unroll
  for (int t = 0; t < RJ; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  for (int p = p_begin; p < p_end; ++p) {
    const int ap = p < 0 ? -p : p;
    const __bf16* brow = bbase + ap * 8 * CL;
    const __bf16* arow = abase + p * pitch;
    bf16x8 Bf[SMAX];
    bf16x8 Af[NA];
#pragma unroll
    for (int s = 0; s < SMAX; ++s)
      if (s < S) Bf[s] = *reinterpret_cast<const bf16x8*>(brow + 16 * s);
#pragma unroll
    for (int a = 0; a < NA; ++a)
      if (a < na) Af[a] = *reinterpret_cast<const bf16x8*>(arow + 16 * a);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < S) {
#pragma unroll
        for (int t = 0; t < RJ; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Af[2 * t + s], Bf[s], acc[t], 0, 0, 0);
      }
    }
  }
  // sum the quarters in LDS (the staged operands are dead after this barrier)
  __syncthreads();
  float* part = reinterpret_cast<float*>(smem_raw);
  if (quarter > 0) {
    float* dstp = part + ((size_t)(strip * (BQ - 1) + quarter - 1) * RJ) * 1024;
#pragma unroll
    for (int t = 0; t < RJ; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) dstp[t * 1024 + r * 64 + lane] = acc[t][r];
  }
  __syncthreads();
  if (quarter == 0) {
    float* dst = out + ((size_t)b * g.Nk + k) * plane;
#pragma unroll
    for (int t = 0; t < RJ; ++t) {
#pragma unroll
      for (int qd = 1; qd < BQ; ++qd) {
        const float* src = part + ((size_t)(strip * (BQ - 1) + qd - 1) * RJ + t) * 1024;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] += src[r * 64 + lane];
      }
      const int j = J0 + 32 * t + m;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = I0 + 32 * strip + 8 * (r >> 2) + 4 * hi + (r & 3);
        if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[t][r];
      }
    }
  }
}

// ------------------------------------------------------------------ launch

template <int NW, int TPW, typename Shape, typename Kern>
static hipError_t launch_cfg(Kern kern, const Geo<float>& g, const RegionShape& rs, const Shape& sh, size_t lds,
                             int nb, const float* z, const float* in, float* out, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > LDS_MAX) return hipErrorInvalidConfiguration;
  dim3 grid(rs.regions_i * rs.regions_j, g.Nk, nb);
  hipLaunchKernelGGL(kern, grid, dim3(64 * NW), lds, s, g, rs, sh, z, in, out);
  return hipGetLastError();
}

// Wavefronts x tiles per wavefront for a region of `tiles` tiles.
#define PDRT_CONV_DISPATCH(KERN, SHAPE)                                                          \
  int tiles = rs.TI * rs.TJ;                                                                     \
  if (tiles <= 4) return launch_cfg<4, 1>(KERN<4, 1>, g, rs, SHAPE, lds, nb, z, in, out, s);     \
  if (tiles <= 8) return launch_cfg<8, 1>(KERN<8, 1>, g, rs, SHAPE, lds, nb, z, in, out, s);     \
  if (tiles <= 16) return launch_cfg<8, 2>(KERN<8, 2>, g, rs, SHAPE, lds, nb, z, in, out, s);    \
  if (tiles <= 24) return launch_cfg<8, 3>(KERN<8, 3>, g, rs, SHAPE, lds, nb, z, in, out, s);    \
  return launch_cfg<12, 3>(KERN<12, 3>, g, rs, SHAPE, lds, nb, z, in, out, s);

hipError_t launch_conv_mfma_f32(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                hipStream_t s) {
  RegionShape rs;
  F32Shape fs;
  size_t lds = 0;
  for (int rmax = RMAX; rmax >= 1; --rmax) {  // the largest region whose LDS image fits
    rs = region_shape(g.Nu, g.Nv, rmax);
    fs = f32_shape(g.h, rs);
    lds = f32_lds(g.h, fs);
    if (lds <= LDS_MAX) break;
  }
  PDRT_CONV_DISPATCH(k_conv_mfma_f32, fs)
}

template <int RJ, int SMAX>
static hipError_t launch_bf16_cfg(const Geo<float>& g, const BF16Shape& bs, size_t lds, int nb, const float* z,
                                  const float* in, float* out, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_mfma_bf16<RJ, SMAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > LDS_MAX) return hipErrorInvalidConfiguration;
  dim3 grid(bs.regions_i * bs.regions_j, g.Nk, nb);
  hipLaunchKernelGGL((k_conv_mfma_bf16<RJ, SMAX>), grid, dim3(64 * BQ * bs.RI), lds, s, g, bs, z, in, out);
  return hipGetLastError();
}

template <int RJ>
static hipError_t launch_bf16_rj(const Geo<float>& g, const BF16Shape& bs, size_t lds, int nb, const float* z,
                                 const float* in, float* out, hipStream_t s) {
  if (bs.S <= 4) return launch_bf16_cfg<RJ, 4>(g, bs, lds, nb, z, in, out, s);
  if (bs.S <= 6) return launch_bf16_cfg<RJ, 6>(g, bs, lds, nb, z, in, out, s);
  if (bs.S <= 8) return launch_bf16_cfg<RJ, 8>(g, bs, lds, nb, z, in, out, s);
  return launch_bf16_cfg<RJ, 10>(g, bs, lds, nb, z, in, out, s);
}

hipError_t launch_conv_mfma_bf16(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                 hipStream_t s) {
  BF16Shape bs;
  size_t lds = 0;
  for (int rmax = 3; rmax >= 1; --rmax) {  // strips per region, while the LDS image fits
    bs = bf16_shape(g.Nu, g.Nv, g.h, rmax);
    lds = bf16_lds(g.h, bs);
    if (lds <= LDS_MAX) break;
  }
  if (bs.S > 10) return hipErrorInvalidConfiguration;
  if (bs.RJ == 1) return launch_bf16_rj<1>(g, bs, lds, nb, z, in, out, s);
  if (bs.RJ == 2) return launch_bf16_rj<2>(g, bs, lds, nb, z, in, out, s);
  return launch_bf16_rj<3>(g, bs, lds, nb, z, in, out, s);
}

}  // namespace pdrt
