// conv_fwd_reg.hip — the forward per-plane lateral convolution (arXiv:2512.18863
// §2.2.6, Eq. 8) in FP32 on the CDNA4 matrix cores, for an input that vanishes
// outside the aperture rectangle (the primary P = F G).
//
// out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q], with in zero outside the box
// [r0, r1) x [c0, c1).  Split by tap row p and by box row r:
//   Y_p[r][j] = sum_c K[p][c - j] in[r][c],   out[r - p][j] += Y_p[r][j],
// and since K[-p][.] = K[p][.] the same product also gives out[r + p][j] += Y_p[r][j].
// The input is small (the box) and the output large (the box and the kernel's
// reach around it), so the box stays in registers for the whole plane and only
// the Toeplitz band of tap row p is read from LDS:
//   v_mfma_f32_16x16x4_f32 with M = 16 output columns j, N = 16 box rows r and
//   K = 4 box columns c:  A[m][k] = K[p][c_k - j_m] (from the extended tap row),
//   B[k][n] = in[r_n][c_k] (registers, loaded once per plane).
// The product's box rows lie along the lanes of each 16-lane row of the result,
// so moving it by p rows is a DPP row shift within those 16 lanes: the part that
// stays in a 16-row output block is one shift, the part that crosses into the
// neighbouring block the complementary one; lanes shifted in from outside the row
// read zero.  Each wavefront owns one 16-column strip of the output and keeps its
// rows (the box rows and two blocks above and below, for h <= 31) in registers over
// all tap rows, then adds them into an LDS copy of the plane; the plane goes out
// with row-contiguous stores, zeros outside the reach included.
//
// Work skipped: groups of 16 box columns of which no column lies within h of the
// strip (one uniform branch per group and tap row; inside a group the band's zero
// taps are multiplied).  The products of skipped groups are exact zeros.  The sum of every output
// runs over p = 0, 1, ..., h in order, within a tap row over the box's row blocks,
// and within a product over the box columns in order (deterministic; the rounding
// differs from a direct sum only in order).
#include "conv_common.hpp"

namespace pdrt {

typedef float f32x4r __attribute__((ext_vector_type(4)));

constexpr int kRegNW = 8;    // wavefronts per workgroup (output strips in parallel)
constexpr int kRegQB = 2;    // output blocks of 16 rows above and below a row chunk
constexpr int kRegMaxH = 16 * (kRegQB - 1) + 15;  // largest half-width the blocks reach

// Extended tap row: kx[p][x] = K[p][|x - off|] for |x - off| <= h, else 0, with
// off = h + 34 and length 2h + 65: a column group in reach reads |c - j| <= h + 30
// (x in [4, 2h + 64]); a group out of reach reads x in [0, 30], all zero.
__host__ __device__ inline int reg_tap_len(int h) { return 2 * h + 65; }
__host__ __device__ inline int reg_tap_off(int h) { return h + 34; }

// Lane i takes lane i + S (LEFT) or i - S of its 16-lane row; 0 where that lane lies
// outside the row.  1 <= S <= 15.  (Each component is copied to a scalar before its
// bits are reinterpreted: this compiler turns __builtin_bit_cast of a vector element
// v[e] into a cast of v[0].)
template <int S, bool LEFT>
__device__ __forceinline__ f32x4r row_shift(const f32x4r& v) {
  constexpr int ctrl = LEFT ? 0x100 + S : 0x110 + S;  // row_shl:S / row_shr:S
  f32x4r r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float x = v[e];
    r[e] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, false));
  }
  return r;
}

// One tap row P: the products of the box's T row blocks with the band of tap row P
// and their shifted sums into the strip's output blocks O (block kRegQB + t holds
// the rows of box block t).  Column group u > 0 (K-steps 4u .. 4u + 3) is executed when
// bit u of umask (uniform) is set; group 0 always is.
template <int P, int T, int SU, int NB>
__device__ __forceinline__ void reg_tap_row(const float* const (&aaddr)[SU], int E, unsigned umask,
                                            const float (&B)[T][4 * SU], f32x4r (&O)[NB]) {
  constexpr int S = P & 15, Q = P >> 4;
  float A[4 * SU];
#pragma unroll
  for (int u = 0; u < SU; ++u)
#pragma unroll
    for (int s = 0; s < 4; ++s) A[4 * u + s] = aaddr[u][P * E + 4 * s];
  // the T products share each A and are independent chains, issued in turn; group 0
  // always runs and starts the chains from zero (out of reach its A is zero), the
  // others run when their bit of umask is set and accumulate in place
  f32x4r Y[T];
#pragma unroll
  for (int t = 0; t < T; ++t)
    Y[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0], B[t][0], f32x4r{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
  for (int s = 1; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < T; ++t) Y[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s], B[t][s], Y[t], 0, 0, 0);
#pragma unroll
  for (int u = 1; u < SU; ++u)
    if (umask & (1u << u)) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < T; ++t)
          Y[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[4 * u + s], B[t][4 * u + s], Y[t], 0, 0, 0);
    }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const f32x4r y = Y[t];
    constexpr int c = kRegQB;
    if constexpr (P == 0) {
      O[c + t] += y;
    } else if constexpr (S == 0) {
      O[c + t - Q] += y;  // rows r - P
      O[c + t + Q] += y;  // rows r + P
    } else {
      // rows r - P: box lanes n >= S land in block t - Q at lane n - S, the others in
      // block t - Q - 1 at lane n - S + 16
      O[c + t - Q] += row_shift<S, true>(y);
      O[c + t - Q - 1] += row_shift<16 - S, false>(y);
      // rows r + P: lanes n + S < 16 land in block t + Q at lane n + S, the others in
      // block t + Q + 1 at lane n + S - 16
      O[c + t + Q] += row_shift<S, false>(y);
      O[c + t + Q + 1] += row_shift<16 - S, true>(y);
    }
  }
}

template <int P, int T, int SU, int NB>
__device__ __forceinline__ void reg_tap_rows(int h, const float* const (&aaddr)[SU], int E, unsigned umask,
                                             const float (&B)[T][4 * SU], f32x4r (&O)[NB]) {
  if constexpr (P <= kRegMaxH) {
    if (P > h) return;
    reg_tap_row<P, T, SU, NB>(aaddr, E, umask, B, O);
    reg_tap_rows<P + 1, T, SU, NB>(h, aaddr, E, umask, B, O);
  }
}

// One workgroup per (control point, plane) item.  T: row blocks of 16 box rows per
// chunk; SU: 16-column groups of box columns per chunk (boxes larger than a chunk
// are taken chunk by chunk).  LDS: the extended tap rows, then the plane's rows x
// wpitch columns starting at the reach's first column (the unique taps alias it).
template <int T, int SU>
__global__ void __launch_bounds__(64 * kRegNW) k_conv_fwd_reg(Geo<float> g, int wpitch, const int4* __restrict__ box,
                                                              const float* __restrict__ zca,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int NT = 64 * kRegNW;
  constexpr int NKS = 4 * SU;
  constexpr int NB = T + 2 * kRegQB;
  const int h = g.h, E = reg_tap_len(h), off = reg_tap_off(h);
  float* kx = lds;
  float* win = lds + (((h + 1) * E + 3) & ~3);
  float* kq = win;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bk = blockIdx.x;
  const int b = bk / g.Nk, k = bk - b * g.Nk;
  const int Nu = g.Nu, Nv = g.Nv;
  const size_t plane = (size_t)Nu * Nv;
  float* dst = out + (size_t)bk * plane;
  const int4 bx = box[b];
  const int r0 = max(bx.x, 0), r1 = min(bx.y, Nu), c0 = max(bx.z, 0), c1 = min(bx.w, Nv);
  if (r1 <= r0 || c1 <= c0) {
    for (size_t i = tid; i < plane; i += NT) dst[i] = 0.f;
    return;
  }
  const float* src = in + (size_t)bk * plane;
  const int n = lane & 15, kk = lane >> 4;
  const int cw0 = max(0, c0 - h), cw1 = min(Nv, c1 + h);  // columns in reach
  const int njt = (cw1 - cw0 + 15) / 16;
  const int nrc = (r1 - r0 + 16 * T - 1) / (16 * T), ncc = (c1 - c0 + 16 * SU - 1) / (16 * SU);

  // B fragments of box chunk (rc, cc): lane (n, kk) holds in[R + 16 t + n][C + 4 ks + kk]
  float B[T][NKS];
  auto load_b = [&](int rc, int cc) {
    const int R = r0 + 16 * T * rc, C = c0 + 16 * SU * cc;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int r = R + 16 * t + n;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int c = C + 4 * ks + kk;
        B[t][ks] = (r < r1 && c < c1) ? src[(size_t)r * Nv + c] : 0.f;
      }
    }
  };
  const int jt0 = wave;  // this wavefront's first strip
  if (jt0 < njt) load_b(0, 0);  // in flight while the taps are built

  unique_taps(g, k, zca[bk], kq, tid, NT);
  __syncthreads();
  for (int p = wave; p <= h; p += kRegNW)
    for (int x = lane; x < E; x += 64) {
      const int q = x < off ? off - x : x - off;
      kx[p * E + x] = q <= h ? kq[p * (h + 1) + q] : 0.f;
    }
  // with one chunk each strip writes its rows of the plane copy once (rows it does
  // not cover are written as zeros at the end); with several chunks the strips add
  // into a cleared copy
  const bool single = nrc == 1 && ncc == 1;
  __syncthreads();
  if (!single) {
    for (int idx = 4 * tid; idx < Nu * wpitch; idx += 4 * NT) *reinterpret_cast<f32x4r*>(win + idx) = f32x4r{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
  }

  for (int jt = jt0; jt < njt; jt += kRegNW) {
    const int J = cw0 + 16 * jt;  // the strip's first output column
    for (int rc = 0; rc < nrc; ++rc) {
      const int R = r0 + 16 * T * rc;
      f32x4r O[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) O[q] = f32x4r{0.f, 0.f, 0.f, 0.f};
      for (int cc = 0; cc < ncc; ++cc) {
        if (jt != jt0 || rc != 0 || cc != 0) load_b(rc, cc);
        const int C = c0 + 16 * SU * cc;
        const int nsu = min(SU, (c1 - C + 15) / 16);
        // column groups with a column within h of the strip [J, J + 16)
        const int lo = J - h - C - 15, hi = J + 15 + h - C;
        const int ua = lo <= 0 ? 0 : (lo + 15) / 16;
        const int ub = min(nsu - 1, hi >= 0 ? hi / 16 : -1);
        if (ua > ub) continue;
        // A of K-step 4 u + s in tap row p: kx[p][C + 16 u + 4 s + kk - J - m + off];
        // groups outside [ua, ub] read the zeros at the start of the row (group 0
        // runs with them; the others are skipped)
        const float* aaddr[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u)
          aaddr[u] = kx + ((u >= ua && u <= ub) ? C + 16 * u + kk - J - n + off : 15 + kk - n);
        const unsigned umask = __builtin_amdgcn_readfirstlane((2u << ub) - (1u << ua));  // bits ua .. ub
        reg_tap_rows<0, T, SU, NB>(h, aaddr, E, umask, B, O);
      }
      // the strip's rows R - 16 kRegQB + 16 q + n (those in the plane), columns
      // J + 4 kk .. J + 4 kk + 3, into the LDS plane (written with one chunk, added
      // with several); only this wavefront writes them
      float* wcol = win + (J - cw0) + 4 * kk;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int row = R - 16 * kRegQB + 16 * q + n;
        if (row >= 0 && row < Nu) {
          f32x4r* w = reinterpret_cast<f32x4r*>(wcol + row * wpitch);
          if (single) *w = O[q];
          else *w += O[q];
        }
      }
    }
  }
  __syncthreads();
  // the plane, row by row: the LDS copy over the strips' rows and columns, zero elsewhere
  const int wr0 = single ? r0 - 16 * kRegQB : 0, wr1 = single ? r0 + 16 * (T + kRegQB) : Nu;
  RectWalk w(tid, NT, Nv);
  for (; w.r < Nu; w.next(Nv)) {
    const int j = w.c - cw0;
    dst[(size_t)w.r * Nv + w.c] = (j >= 0 && j < 16 * njt && w.r >= wr0 && w.r < wr1) ? win[w.r * wpitch + j] : 0.f;
  }
}

// LDS of the kernel: extended tap rows and the plane copy (wpitch columns).
static size_t reg_lds(int h, int Nu, int wpitch) {
  return sizeof(float) * ((((size_t)(h + 1) * reg_tap_len(h) + 3) & ~(size_t)3) + (size_t)Nu * wpitch);
}

static int reg_wpitch(int Nv) { return 16 * ((Nv + 15) / 16) + 4; }

bool conv_fwd_reg_supported(const Geo<float>& g) {
  return g.h >= 1 && g.h <= kRegMaxH && reg_lds(g.h, g.Nu, reg_wpitch(g.Nv)) <= 160 * 1024;
}

template <int T, int SU>
static hipError_t launch_reg_cfg(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                 float* out, hipStream_t s) {
  const int wpitch = reg_wpitch(g.Nv);
  const size_t lds = reg_lds(g.h, g.Nu, wpitch);
  const void* kern = (const void*)k_conv_fwd_reg<T, SU>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)nb * g.Nk;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_conv_fwd_reg<T, SU>), dim3((unsigned)n_items), dim3(64 * kRegNW), lds, s, g, wpitch, box, z,
                     in, out);
  return hipGetLastError();
}

// The chunk shape from the largest rectangle that jaws inside the field limits give
// (larger rectangles are taken in several chunks).
hipError_t launch_conv_fwd_reg(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                               hipStream_t s, const int* box) {
  if (!conv_fwd_reg_supported(g) || !box) return hipErrorInvalidConfiguration;
  const int4* bx = reinterpret_cast<const int4*>(box);
  const int half_u = (g.Nu - 1) / 2 - g.h, half_v = (g.Nv - 1) / 2 - g.h;  // field limit in pixels
  const int br = 2 * (half_u > 0 ? half_u : 0) + 4, bc = 2 * (half_v > 0 ? half_v : 0) + 4;
  int ch = (br > bc ? br : bc);
  ch = (ch + 15) / 16;
  if (ch <= 1) return launch_reg_cfg<1, 1>(g, nb, bx, z, in, out, s);
  if (ch == 2) return launch_reg_cfg<2, 2>(g, nb, bx, z, in, out, s);
  if (ch == 3) return launch_reg_cfg<3, 3>(g, nb, bx, z, in, out, s);
  return launch_reg_cfg<4, 4>(g, nb, bx, z, in, out, s);
}

}  // namespace pdrt
