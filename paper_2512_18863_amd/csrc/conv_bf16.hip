// conv_bf16.hip — the per-plane lateral convolution (arXiv:2512.18863 §2.2.6,
// Eq. 8) with BF16 operands and FP32 accumulation on v_mfma_f32_16x16x32_bf16
// (the optional mixed precision of §2.3).
//
// For one plane, out[i][n] = sum_{p,c} in[i+p][c] K[p][c-n] (zero padded), i.e.
// for each tap row p a GEMM of the input rows shifted by p with the banded
// Toeplitz matrix T_p[c][n] = K[p][c-n].  The inputs of the forward are zero
// outside the aperture rectangle ("box", a few tens of pixels), and the adjoint's
// outputs are needed only inside it, so the work is organised around the box:
//
//   forward  input support = the box, outputs = the box's reach (box +- h),
//   adjoint  outputs = the box, input support = its reach.
//
// One wavefront owns one (control point, plane) item: it evaluates the plane's
// taps, writes them as padded BF16 tap rows, stages the input support as a BF16
// image in LDS, and accumulates 16 x 16 output tiles, a block of up to BR x BC
// tiles at a time in registers.  For tap row p and K-step s (32 input columns
// starting at c0), a row tile at i0 reads the A fragment in[i0+p+m][c0+8kq ..]
// (one 16-byte LDS read per lane) only if its 16 input rows meet the support;
// a column tile at n0 reads the B fragment K[p][c0+8kq+e-n0-m], e = 0..7, only
// if the K-step lies within its reach; each A fragment feeds every column tile
// of the block and each B fragment every row tile.  The B fragment of a lane is
// eight consecutive entries of one padded tap row at an arbitrary offset: two
// copies of each row, the second shifted by one element, make every run start on
// a 4-byte boundary (four 4-byte LDS reads); lanes whose run lies wholly outside
// the band |c - n| <= h take zeros, so the rows need only 8 entries of padding.
//
// Rounding: inputs and taps are rounded to BF16 (nearest even), every product is
// exact in FP32 and accumulated in FP32 (matrix instructions, then tap rows and
// K-steps in a fixed order): deterministic.  Work items are independent, so
// several wavefronts share a compute unit and hide each other's set-up.
#include "conv_common.hpp"

namespace pdrt {

typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));
typedef float f32x4c __attribute__((ext_vector_type(4)));
typedef unsigned u32x4c __attribute__((ext_vector_type(4)));


struct Bf16Plan {
  int L, X0;      // padded tap row length and the position of tap q = 0 in it
  int img_rows;   // LDS image rows (bound on rows needed by one block and chunk)
  int pitch;      // LDS image row pitch, elements (= 8 mod 64: conflict-free 16-byte reads)
  int kq_floats;  // scratch for the unique FP32 taps (aliases the image)
};

__host__ __device__ inline size_t cb_tap_bytes(int h, const Bf16Plan& q) { return (size_t)2 * (h + 1) * q.L * 2; }
__host__ __device__ inline size_t cb_img_bytes(const Bf16Plan& q) {
  const size_t a = (size_t)q.img_rows * q.pitch * 2, b = (size_t)q.kq_floats * 4;
  return ((a > b ? a : b) + 15) & ~(size_t)15;
}

__device__ __forceinline__ unsigned bf16_pair(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (unsigned)(*reinterpret_cast<const unsigned short*>(&a)) |
         ((unsigned)(*reinterpret_cast<const unsigned short*>(&b)) << 16);
}

// NK: K-steps (32 input columns each) of one column chunk; BR x BC: output tiles
// of one register block; SUP: CONV_IN_BOX (forward) or CONV_OUT_BOX (adjoint).
template <int NK, int BR, int BC, int SUP>
__global__ void __launch_bounds__(64) k_conv_bf16(Geo<float> g, Bf16Plan q, const int4* __restrict__ box,
                                                  const float* __restrict__ zca, const float* __restrict__ in,
                                                  float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int h = g.h, L = q.L;
  unsigned* T0 = reinterpret_cast<unsigned*>(smem_raw);  // [h+1][L/2] dword pairs, run start even
  unsigned* T1 = T0 + (h + 1) * (L / 2);                 // the same rows shifted by one element
  (void)T1;                                              // (reached through T0 + (h+1) L/2)
  __bf16* img = reinterpret_cast<__bf16*>(smem_raw + cb_tap_bytes(h, q));
  float* kq = reinterpret_cast<float*>(img);             // unique taps, before the image is staged
  const int lane = threadIdx.x;
  const int item = blockIdx.x;
  const int b = item / g.Nk, k = item - b * g.Nk;
  const size_t plane = (size_t)g.Nu * g.Nv;
  const float* src = in + (size_t)item * plane;
  float* dst = out + (size_t)item * plane;

  int4 bx = box ? box[b] : make_int4(0, g.Nu, 0, g.Nv);
  const int u0 = max(bx.x, 0), u1 = min(bx.y, g.Nu), v0 = max(bx.z, 0), v1 = min(bx.w, g.Nv);
  const bool empty = u1 <= u0 || v1 <= v0;
  // input support [ir0, ir1) x [ic0, ic1), outputs [or0, or1) x [oc0, oc1)
  int ir0, ir1, ic0, ic1, or0, or1, oc0, oc1;
  if (SUP == CONV_IN_BOX) {
    ir0 = u0, ir1 = u1, ic0 = v0, ic1 = v1;
    or0 = max(0, u0 - h), or1 = min(g.Nu, u1 + h), oc0 = max(0, v0 - h), oc1 = min(g.Nv, v1 + h);
    // the forward's output plane is whole: zero everything outside the reach
    // (whole rows above and below it, the columns left and right of it between)
    if (empty) or0 = or1 = 0, oc0 = oc1 = 0;
    const int top = or0 * g.Nv, bottom = (g.Nu - or1) * g.Nv;
    for (int d = lane; d < top + bottom; d += 64) dst[d < top ? d : (size_t)or1 * g.Nv + (d - top)] = 0.f;
    const int side = oc0 + (g.Nv - oc1), mid = (or1 - or0) * side;
    for (int d = lane; d < mid; d += 64) {
      const int rr = d / side, cc = d - rr * side;
      dst[(size_t)(or0 + rr) * g.Nv + (cc < oc0 ? cc : oc1 + (cc - oc0))] = 0.f;
    }
    if (empty) return;
  } else {
    if (empty) return;  // the adjoint's outputs outside the box are not read
    or0 = u0, or1 = u1, oc0 = v0, oc1 = v1;
    ir0 = max(0, u0 - h), ir1 = min(g.Nu, u1 + h), ic0 = max(0, v0 - h), ic1 = min(g.Nv, v1 + h);
  }

  // ---- taps: unique FP32 values, then two padded BF16 copies of each row
  unique_taps(g, k, zca[item], kq, lane, 64);
  __syncthreads();
  {
    const int L2 = L / 2, n2 = (h + 1) * L2;
    for (int d = lane; d < n2; d += 64) {
      const int a = d / L2, j = d - a * L2;
      float v[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int qq = 2 * j + e - q.X0;
        const int aq = qq < 0 ? -qq : qq;
        v[e] = aq <= h ? kq[a * (h + 1) + aq] : 0.f;
      }
      T0[d] = bf16_pair(v[0], v[1]);
      T1[d] = bf16_pair(v[1], v[2]);
    }
  }
  __syncthreads();

  const int m = lane & 15, kqd = lane >> 4;  // A: row m, K entries 8 kqd ..; B: column m
  const int TR = (or1 - or0 + 15) / 16, TC = (oc1 - oc0 + 15) / 16;
  const int KCOLS = 32 * NK, L2 = L / 2;
  for (int rb = 0; rb < TR; rb += BR) {
    for (int cb = 0; cb < TC; cb += BC) {
      const int nr = min(BR, TR - rb), nc = min(BC, TC - cb);
      const int OI0 = or0 + 16 * rb, OJ0 = oc0 + 16 * cb;
      f32x4c acc[BR][BC];
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int t = 0; t < BC; ++t) acc[r][t] = f32x4c{0.f, 0.f, 0.f, 0.f};
      // input rows and columns this block can reach: i0 + p + m for |p| <= h
      const int br0 = max(ir0, OI0 - h), br1 = min(ir1, OI0 + 16 * nr + h);
      const int bc0 = max(ic0, OJ0 - h), bc1 = min(ic1, OJ0 + 16 * nc + h);
      if (br1 > br0 && bc1 > bc0) {
        // row chunks: the image holds chunk rows plus 15 zero rows above and below,
        // clipped to what the block's tap rows reach
        const int rows_all = min(br1 - br0 + 30, 16 * nr + 2 * h);
        const int rch = rows_all <= q.img_rows ? br1 - br0 : q.img_rows - 30;
        for (int cr0 = br0; cr0 < br1; cr0 += rch) {
          const int cr1 = min(br1, cr0 + rch);
          for (int cc0 = bc0; cc0 < bc1; cc0 += KCOLS) {
            const int cc1 = min(bc1, cc0 + KCOLS);
            const int IR0 = max(cr0 - 15, OI0 - h);
            const int nrows = min(cr1 + 15, OI0 + 16 * nr + h) - IR0;
            // stage rows [IR0, IR0 + nrows) x columns [cc0, cc0 + KCOLS): data in
            // [cr0, cr1) x [cc0, cc1), zero elsewhere; SB pairs per lane in flight
            __syncthreads();
            {
              constexpr int SB = 2;
              const int W2 = KCOLS / 2, total = nrows * W2;
              for (int d0 = 0; d0 < total; d0 += 64 * SB) {
                float x0[SB], x1[SB];
#pragma unroll
                for (int e = 0; e < SB; ++e) {
                  const int d = d0 + lane + 64 * e;
                  const int rr = d / W2, c2 = d - rr * W2;
                  const int i = IR0 + rr, j = cc0 + 2 * c2;
                  const bool rin = d < total && i >= cr0 && i < cr1;
                  const size_t o = (size_t)i * g.Nv + j;
                  x0[e] = rin && j < cc1 ? src[o] : 0.f;
                  x1[e] = rin && j + 1 < cc1 ? src[o + 1] : 0.f;
                }
#pragma unroll
                for (int e = 0; e < SB; ++e) {
                  const int d = d0 + lane + 64 * e;
                  if (d < total) {
                    const int rr = d / W2, c2 = d - rr * W2;
                    reinterpret_cast<unsigned*>(img + rr * q.pitch)[c2] = bf16_pair(x0[e], x1[e]);
                  }
                }
              }
            }
            __syncthreads();
            // per lane and (column tile, K-step): where its B run starts in a padded
            // tap row (copy by parity), and whether it meets the band at all
            int boff[BC][NK];
            unsigned bmask[BC][NK];
#pragma unroll
            for (int t = 0; t < BC; ++t) {
              const int n0 = OJ0 + 16 * t;
#pragma unroll
              for (int s2 = 0; s2 < NK; ++s2) {
                const int c0 = cc0 + 32 * s2;
                const int x = c0 + 8 * kqd - n0 - m + q.X0;
                const bool live = t < nc && c0 < cc1 && x + 7 >= q.X0 - h && x <= q.X0 + h;
                const int xs = live ? x : q.X0;
                boff[t][s2] = ((xs & 1) ? (h + 1) * L2 : 0) + (xs >> 1);
                bmask[t][s2] = live ? 0xffffffffu : 0u;
              }
            }
            const __bf16* abase = img + (m - IR0) * q.pitch + 8 * kqd;
            // tap rows reaching the chunk from any row tile of the block
            const int p_lo = max(-h, cr0 - (OI0 + 16 * nr - 1)), p_hi = min(h, cr1 - 1 - OI0);
            for (int p = p_lo; p <= p_hi; ++p) {
              const int ap = p < 0 ? -p : p;
              // all of this tap row's operands first (unconditional loads, kept as
              // 32-bit words until the matrix instructions), then the instructions
              u32x4c Bw[BC][NK];
#pragma unroll
              for (int t = 0; t < BC; ++t)
#pragma unroll
                for (int s2 = 0; s2 < NK; ++s2) {
                  const unsigned* row = T0 + ap * L2 + boff[t][s2];
                  const unsigned mk = bmask[t][s2];
                  Bw[t][s2] = u32x4c{row[0] & mk, row[1] & mk, row[2] & mk, row[3] & mk};
                }
              u32x4c Aw[BR][NK];
              bool rval[BR];
#pragma unroll
              for (int r = 0; r < BR; ++r) {
                const int i0 = OI0 + 16 * r;
                // the tile's 16 input rows [i0 + p, i0 + p + 16) must meet the chunk;
                // other tiles read image row 0 (in bounds) and skip their instructions
                rval[r] = r < nr && i0 + p + 15 >= cr0 && i0 + p < cr1;
                const int arow = rval[r] ? i0 + p : IR0;
#pragma unroll
                for (int s2 = 0; s2 < NK; ++s2)
                  Aw[r][s2] = *reinterpret_cast<const u32x4c*>(abase + arow * q.pitch + 32 * s2);
              }
#pragma unroll
              for (int r = 0; r < BR; ++r) {
                if (!rval[r]) continue;
#pragma unroll
                for (int s2 = 0; s2 < NK; ++s2)
#pragma unroll
                  for (int t = 0; t < BC; ++t)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8c, Aw[r][s2]),
                                                                         __builtin_bit_cast(bf16x8c, Bw[t][s2]),
                                                                         acc[r][t], 0, 0, 0);
              }
            }
          }
        }
      }
      // lane (m, kqd) holds rows 4 kqd + e, column m of each tile
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        if (r >= nr) break;
#pragma unroll
        for (int t = 0; t < BC; ++t) {
          if (t >= nc) break;
          const int j = OJ0 + 16 * t + m;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = OI0 + 16 * r + 4 * kqd + e;
            if (i < or1 && j < oc1) dst[(size_t)i * g.Nv + j] = acc[r][t][e];
          }
        }
      }
    }
  }
}

// Bounds of the aperture rectangle for jaws inside the field limits, as the
// aperture-box kernel computes it (one pixel of margin each side): the image is
// sized for it, and larger rectangles are processed in row and column chunks.
static int box_extent(double F, double D, double c, int N) {
  const double fa = -F / D + c - 0.5, fb = F / D + c + 0.5;
  int lo = (int)std::floor(fa) - 1, hi = (int)std::ceil(fb) + 1;
  lo = lo < 0 ? 0 : lo;
  hi = hi > N ? N : hi;
  return hi > lo ? hi - lo : 1;
}

// Row pitch with (pitch / 8) odd: eight consecutive rows' 16-byte reads fall in
// distinct 16-byte slots of a 128-byte window (no bank conflicts).
static int pitch_bf16(int cols) { return cols + 8; }

template <int NK, int BR, int BC, int SUP>
static hipError_t launch_bf16_nk(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                 float* out, hipStream_t s, int box_rows) {
  Bf16Plan q;
  q.X0 = g.h + 8;
  q.L = 2 * g.h + 16;
  const int out_rows = SUP == CONV_IN_BOX ? (box_rows + 2 * g.h < g.Nu ? box_rows + 2 * g.h : g.Nu) : box_rows;
  const int tr = (out_rows + 15) / 16;
  const int tr_blk = tr < BR ? tr : BR;
  const int in_rows = SUP == CONV_IN_BOX ? box_rows : (box_rows + 2 * g.h < g.Nu ? box_rows + 2 * g.h : g.Nu);
  int rows = in_rows + 30;
  if (rows > 16 * tr_blk + 2 * g.h) rows = 16 * tr_blk + 2 * g.h;
  if (rows < 31) rows = 31;  // at least one row of data per chunk
  q.img_rows = rows;
  q.pitch = pitch_bf16(32 * NK);
  q.kq_floats = (g.h + 1) * (g.h + 1);
  const size_t lds = cb_tap_bytes(g.h, q) + cb_img_bytes(q);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const void* kern = (const void*)k_conv_bf16<NK, BR, BC, SUP>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)nb * g.Nk;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_conv_bf16<NK, BR, BC, SUP>), dim3((unsigned)n_items), dim3(64), lds, s, g, q, box, z, in,
                     out);
  return hipGetLastError();
}

// Forward: one register block of up to 6 x 6 tiles covers the reach of a rectangle
// inside the field limits; adjoint: 2 x 2 tiles cover the rectangle itself.
template <int SUP>
static hipError_t launch_bf16_sup(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                  float* out, hipStream_t s) {
  // expected rectangle from the field limit: the grid is Nu = 2 ceil((F + h D)/D) + 1
  const double D = g.lat;
  const double Fu = ((g.Nu - 1) / 2 - g.h) * D, Fv = ((g.Nv - 1) / 2 - g.h) * D;
  const int br = box ? box_extent(Fu, D, 0.5 * (g.Nu - 1), g.Nu) : g.Nu;
  const int bc = box ? box_extent(Fv, D, 0.5 * (g.Nv - 1), g.Nv) : g.Nv;
  const int in_cols = SUP == CONV_IN_BOX ? bc : (bc + 2 * g.h < g.Nv ? bc + 2 * g.h : g.Nv);
  const int nk = (in_cols + 31) / 32;
  constexpr int BR = SUP == CONV_IN_BOX ? 6 : 2, BC = SUP == CONV_IN_BOX ? 3 : 2;
  if (nk <= 1) return launch_bf16_nk<1, BR, BC, SUP>(g, nb, box, z, in, out, s, br);
  if (nk == 2) return launch_bf16_nk<2, BR, BC, SUP>(g, nb, box, z, in, out, s, br);
  return launch_bf16_nk<3, BR, BC, SUP>(g, nb, box, z, in, out, s, br);
}

hipError_t launch_conv_mfma_bf16(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                 hipStream_t s, const int* box, int support) {
  const int4* bx = reinterpret_cast<const int4*>(box);
  if (support == CONV_OUT_BOX && bx) return launch_bf16_sup<CONV_OUT_BOX>(g, nb, bx, z, in, out, s);
  // forward, or no box: the input support is the box (the whole plane without one)
  return launch_bf16_sup<CONV_IN_BOX>(g, nb, support == CONV_DENSE ? nullptr : bx, z, in, out, s);
}

}  // namespace pdrt
