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
// One workgroup owns one (control point, plane) item: it evaluates the plane's
// taps, writes them as padded BF16 tap rows, stages the input support as a BF16
// image in LDS, and accumulates 16 x 16 output tiles in register blocks.  For tap
// row p and K-step s (32 input columns starting at c0), a row tile at i0 reads
// the A fragment in[i0+p+m][c0+8kq ..] (one 16-byte LDS read per lane) and runs
// its matrix instructions only if its 16 input rows meet the support; a column
// tile at n0 reads the B fragment K[p][c0+8kq+e-n0-m], e = 0..7; each A fragment
// feeds every column tile of the block and each B fragment every row tile.  The
// forward's two wavefronts take one block each (their columns split the reach);
// the adjoint's four share its one small block, each a quarter of the tap rows,
// and their sums are added in LDS in a fixed order.  The B fragment of a lane is
// eight consecutive entries of one padded tap row at an arbitrary offset: two
// copies of each row, the second shifted by one element, make every run start on
// a 4-byte boundary (four 4-byte LDS reads); lanes whose run lies wholly outside
// the band |c - n| <= h take zeros, so the rows need only 8 entries of padding.
//
// Rounding: inputs and taps are rounded to BF16 (nearest even), every product is
// exact in FP32 and accumulated in FP32 (matrix instructions, then tap rows and
// K-steps in a fixed order, the parts' sums in part order): deterministic.  Work
// items are independent, so several workgroups share a compute unit and hide
// each other's set-up; the first global loads of the input are issued before the
// taps are evaluated.
#include <type_traits>

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
// of one register block; NWB x NWP wavefronts: NWB blocks at a time, each block's
// tap rows split in NWP parts whose sums are added in LDS in a fixed order;
// SUP: CONV_IN_BOX (forward) or CONV_OUT_BOX (adjoint).
template <int NK, int BR, int BC, int NWB, int NWP, int SUP>
__global__ void __launch_bounds__(64 * NWB * NWP) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_conv_bf16(Geo<float> g, Bf16Plan q, const int4* __restrict__ box,
                                                              const float* __restrict__ zca,
                                                              const float* __restrict__ in, float* __restrict__ out) {
  constexpr int NT = 64 * NWB * NWP;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int h = g.h, L = q.L, L2 = L / 2;
  unsigned* T0 = reinterpret_cast<unsigned*>(smem_raw);  // [h+1][L/2] dword pairs, run start even
  unsigned* T1 = T0 + (h + 1) * L2;                      // the same rows shifted by one element
  __bf16* img = reinterpret_cast<__bf16*>(smem_raw + cb_tap_bytes(h, q));
  float* kq = reinterpret_cast<float*>(img);             // unique taps, before the image is staged
  f32x4c* red = reinterpret_cast<f32x4c*>(img);          // the parts' sums, after the last chunk
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wb = wave / NWP, wp = wave - wb * NWP;
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
    for (int d = tid; d < top + bottom; d += NT) dst[d < top ? d : (size_t)or1 * g.Nv + (d - top)] = 0.f;
    const int side = oc0 + (g.Nv - oc1), mid = (or1 - or0) * side;
    for (int d = tid; d < mid; d += NT) {
      const int rr = d / side, cc = d - rr * side;
      dst[(size_t)(or0 + rr) * g.Nv + (cc < oc0 ? cc : oc1 + (cc - oc0))] = 0.f;
    }
    if (empty) return;
  } else {
    if (empty) return;  // the adjoint's outputs outside the box are not read
    or0 = u0, or1 = u1, oc0 = v0, oc1 = v1;
    ir0 = max(0, u0 - h), ir1 = min(g.Nu, u1 + h), ic0 = max(0, v0 - h), ic1 = min(g.Nv, v1 + h);
  }

  const int m = lane & 15, kqd = lane >> 4;  // A: row m, K entries 8 kqd ..; B: column m
  const int TR = (or1 - or0 + 15) / 16, TC = (oc1 - oc0 + 15) / 16;
  const int KCOLS = 32 * NK, W2 = KCOLS / 2;
  // input chunks: rows [cr0, cr1) of at most rch rows, columns [cc0, cc0 + KCOLS);
  // the image holds rows [IR0, IR1): the chunk's rows with 15 zero rows above and
  // below, clipped to the rows that the output tiles' tap rows reach
  const int rows_all = min(ir1 - ir0 + 30, 16 * TR + 2 * h);
  const int rch = rows_all <= q.img_rows ? ir1 - ir0 : q.img_rows - 30;
  struct Chunk {
    int cr0, cr1, cc0, cc1, IR0, nrows;
  };
  auto chunk_at = [&](int cr0, int cc0) {
    Chunk c;
    c.cr0 = cr0, c.cr1 = min(ir1, cr0 + rch), c.cc0 = cc0, c.cc1 = min(ic1, cc0 + KCOLS);
    c.IR0 = max(cr0 - 15, or0 - h);
    c.nrows = min(c.cr1 + 15, or0 + 16 * TR + h) - c.IR0;
    return c;
  };
  auto load_pair = [&](const Chunk& c, int d, float& x0, float& x1) {
    const int rr = d / W2, c2 = d - rr * W2;
    const int i = c.IR0 + rr, j = c.cc0 + 2 * c2;
    const bool rin = d < c.nrows * W2 && i >= c.cr0 && i < c.cr1;
    const size_t o = (size_t)i * g.Nv + j;
    x0 = rin && j < c.cc1 ? src[o] : 0.f;
    x1 = rin && j + 1 < c.cc1 ? src[o + 1] : 0.f;
  };
  auto put_pair = [&](const Chunk& c, int d, float x0, float x1) {
    if (d < c.nrows * W2) {
      const int rr = d / W2, c2 = d - rr * W2;
      reinterpret_cast<unsigned*>(img + rr * q.pitch)[c2] = bf16_pair(x0, x1);
    }
  };

  // the first chunk (for an aperture inside the field limits, the only one): its
  // first PB pairs per thread are loaded before the taps are evaluated, so the
  // loads' latency overlaps that work
  constexpr int PB = 8, SB = 4;
  const Chunk first = chunk_at(ir0, ic0);
  float p0[PB], p1[PB];
#pragma unroll
  for (int e = 0; e < PB; ++e) load_pair(first, tid + NT * e, p0[e], p1[e]);

  // ---- taps: unique FP32 values, then two padded BF16 copies of each row
  unique_taps(g, k, zca[item], kq, tid, NT);
  __syncthreads();
  {
    const int n2 = (h + 1) * L2;
    for (int d = tid; d < n2; d += NT) {
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

  const int nbc = (TC + BC - 1) / BC, nblocks = ((TR + BR - 1) / BR) * nbc;
  for (int slot = 0; slot * NWB < nblocks; ++slot) {
    const int blk = slot * NWB + wb;
    const bool active = blk < nblocks;
    const int rb = active ? (blk / nbc) * BR : 0, cb = active ? (blk % nbc) * BC : 0;
    const int nr = active ? min(BR, TR - rb) : 0, nc = active ? min(BC, TC - cb) : 0;
    const int OI0 = or0 + 16 * rb, OJ0 = oc0 + 16 * cb;
    f32x4c acc[BR][BC];
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int t = 0; t < BC; ++t) acc[r][t] = f32x4c{0.f, 0.f, 0.f, 0.f};
    for (int cr0 = ir0; cr0 < ir1; cr0 += rch) {
      for (int cc0 = ic0; cc0 < ic1; cc0 += KCOLS) {
        const Chunk c = chunk_at(cr0, cc0);
        // stage the chunk's image (all threads; SB pairs per thread in flight)
        __syncthreads();
        int d0 = 0;
        if (slot == 0 && cr0 == ir0 && cc0 == ic0) {
#pragma unroll
          for (int e = 0; e < PB; ++e) put_pair(c, tid + NT * e, p0[e], p1[e]);
          d0 = NT * PB;
        }
        for (; d0 < c.nrows * W2; d0 += NT * SB) {
          float x0[SB], x1[SB];
#pragma unroll
          for (int e = 0; e < SB; ++e) load_pair(c, d0 + tid + NT * e, x0[e], x1[e]);
#pragma unroll
          for (int e = 0; e < SB; ++e) put_pair(c, d0 + tid + NT * e, x0[e], x1[e]);
        }
        __syncthreads();
        if (!active) continue;
        // tap rows reaching the chunk from any row tile of the block, this wave's part
        const int p_lo = max(-h, c.cr0 - (OI0 + 16 * nr - 1)), p_hi = min(h, c.cr1 - 1 - OI0);
        const int np = p_hi - p_lo + 1;
        if (np <= 0) continue;
        const int pa = p_lo + (np * wp) / NWP, pz = p_lo + (np * (wp + 1)) / NWP;
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
            const bool live = t < nc && c0 < c.cc1 && x + 7 >= q.X0 - h && x <= q.X0 + h;
            const int xs = live ? x : q.X0;
            boff[t][s2] = ((xs & 1) ? (h + 1) * L2 : 0) + (xs >> 1);
            bmask[t][s2] = live ? 0xffffffffu : 0u;
          }
        }
        const __bf16* abase = img + (m - c.IR0) * q.pitch + 8 * kqd;
        for (int p = pa; p < pz; ++p) {
          const int ap = p < 0 ? -p : p;
          // all of this tap row's operands first (unconditional loads, kept as
          // 32-bit words until the matrix instructions: branch-free code waits only
          // for the operands each instruction needs), then the instructions of the
          // row tiles whose 16 input rows [i0 + p, i0 + p + 16) meet the chunk
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
            rval[r] = r < nr && i0 + p + 15 >= c.cr0 && i0 + p < c.cr1;
            // other tiles read the chunk's first image row (in bounds), unused
            const int arow = rval[r] ? i0 + p : c.IR0;
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
    if (NWP > 1) {
      // parts 1 .. NWP-1 park their sums, part 0 adds them in that order
      __syncthreads();
      if (active && wp > 0) {
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
          for (int t = 0; t < BC; ++t)
            red[(((wb * (NWP - 1) + wp - 1) * BR + r) * BC + t) * 64 + lane] = acc[r][t];
      }
      __syncthreads();
      if (active && wp == 0) {
        for (int pp = 1; pp < NWP; ++pp)
#pragma unroll
          for (int r = 0; r < BR; ++r)
#pragma unroll
            for (int t = 0; t < BC; ++t)
              acc[r][t] += red[(((wb * (NWP - 1) + pp - 1) * BR + r) * BC + t) * 64 + lane];
      }
    }
    // lane (m, kqd) holds rows 4 kqd + e, column m of each tile
    if (active && wp == 0) {
      // (conditions rather than early exits: the loops stay fully unrolled and the
      // accumulators in registers)
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int t = 0; t < BC; ++t) {
          const int j = OJ0 + 16 * t + m;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = OI0 + 16 * r + 4 * kqd + e;
            if (r < nr && t < nc && i < or1 && j < oc1) dst[(size_t)i * g.Nv + j] = acc[r][t][e];
          }
        }
    }
  }
}

// ---------------------------------------------------------------- windowed adjoint
//
// The adjoint with persistent workgroups of eight wavefronts that stage, per item,
// only the window their output tiles read, as in the FP32 windowed adjoint: the
// rectangle (clipped to the plane) is covered by 16 x 16 output tiles at its
// corner, taken in pieces of at most 2 x 2 tiles; a piece's image holds plane
// rows [I - h, I + 16 nI + h) and the 32 NK columns from J - h that its K-steps
// read (zero outside the plane), staged in four-column groups (one four-word load,
// two BF16 pairs, one 8-byte LDS store) and prefetched into registers during the
// previous piece's matrix loop.  The tap rows are padded so that every B run of
// every lane lies inside them (no masks): two copies of each row of taps |p|, the
// second shifted by one element, so that a run is four aligned words at any
// offset.  The 2h + 1 tap rows are split over the eight wavefronts; their sums are
// added in LDS in wavefront order, one tile per wavefront.  The arithmetic of
// every output is that of the tiled kernel (BF16 operands, FP32 products and
// sums).
struct Bf16AdjWin {
  int rows, pitch;  // image rows (32 + 2h) and pitch in BF16 elements (32 NK + 16: 16 NK + 8 words, the
                    // 16-byte operand reads of a half-wavefront in distinct slots of a 512-byte line)
  int L2;           // words per padded tap row (each copy): 16 NK + 17 (odd, so that the
                    // taps' writes down a column of rows fall in distinct banks)
};

// Element x of a padded tap row holds K[p][|x - X0|] (zero beyond h), X0 = h + 32:
// the run of lane (m, kq) for column tile t and K-step s starts at
// x = 32 s + 8 kq - 16 t - m + 32, in [1, 32 NK + 24].
constexpr int kBwX0 = 32;

// Words from the first copy of the tap rows to the second: congruent to 16 mod 32,
// so that a half-wavefront's run read, whose lanes take words 8 to 20 of one copy
// and 8 to 19 of the other (plus a common offset), never asks one of the 32 banks
// that 4-byte reads see for two different words (measured: offsets congruent to
// 0 mod 32 cost twice the cycles per read).
__host__ __device__ inline int bw_t1_words(int h, int L2) { return (((h + 1) * L2 + 31) & ~31) + 16; }

// The taps of plane k written straight into both padded copies: tap K[p][q] sits
// at elements X0 + h +- q of row p and X0 + h +- p of row q; copy 0 holds element
// x at half-word x of its row, copy 1 at half-word x - 1.  Every other element of
// the rows is zero and is never written here (the rows are cleared once).
__device__ __forceinline__ void taps_to_bf16_rows(const Geo<float>& g, int k, float zk, unsigned* T0, unsigned* T1,
                                                  int L2, int tid, int nt) {
  TapParams<float> tp = tap_params(g, k, zk);
  const int h1 = g.h + 1, x0 = g.h + kBwX0;
  unsigned short* H0 = reinterpret_cast<unsigned short*>(T0);
  unsigned short* H1 = reinterpret_cast<unsigned short*>(T1);
  for (int t = tid; t < h1 * (h1 + 1) / 2; t += nt) {
    int q = (int)((sqrtf((float)(8 * t + 1)) - 1.f) * 0.5f);
    if ((q + 1) * (q + 2) / 2 <= t) ++q;
    if (q * (q + 1) / 2 > t) --q;
    const int p = t - q * (q + 1) / 2;
    const __bf16 b = (__bf16)tap_value(tp, p, q);
    const unsigned short v = *reinterpret_cast<const unsigned short*>(&b);
    const int rp = 2 * L2 * p + x0, rq = 2 * L2 * q + x0;
    H0[rp + q] = v;
    H0[rp - q] = v;
    H0[rq + p] = v;
    H0[rq - p] = v;
    H1[rp + q - 1] = v;
    H1[rp - q - 1] = v;
    H1[rq + p - 1] = v;
    H1[rq - p - 1] = v;
  }
}

template <int NK>
__global__ void __launch_bounds__(512) k_conv_bf16_adj_win(Geo<float> g, Bf16AdjWin bw, int n_items,
                                                           const int4* __restrict__ box,
                                                           const float* __restrict__ zca,
                                                           const float* __restrict__ in, float* __restrict__ out) {
  constexpr int NW = 8, NT = 64 * NW, BR = 2, BC = 2, PG = 5;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int h = g.h, L2 = bw.L2, pitch = bw.pitch;
  unsigned* T0 = reinterpret_cast<unsigned*>(smem_raw);  // [h + 1][L2]: elements (2i, 2i + 1)
  const int t1w = bw_t1_words(h, L2);
  unsigned* T1 = T0 + t1w;                               // elements (2i + 1, 2i + 2)
  // byte offsets from the (16-byte aligned) base, so that every access stays an
  // LDS access (an integer round trip of the address would make them generic)
  const int img_off = (4 * (t1w + (h + 1) * L2) + 15) & ~15;
  __bf16* img = reinterpret_cast<__bf16*>(smem_raw + img_off);
  f32x4c* red = reinterpret_cast<f32x4c*>(smem_raw + img_off + ((bw.rows * pitch * 2 + 15) & ~15));
  const size_t plane = (size_t)g.Nu * g.Nv;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, kqd = lane >> 4;

  struct Cov {
    int Iw, Jw, nI, nJ, npi, npj;
  };
  auto cov_of = [&](int item) {
    Cov c;
    const int4 bx = box[item / g.Nk];
    const int u0 = max(bx.x, 0), u1 = min(bx.y, g.Nu), v0 = max(bx.z, 0), v1 = min(bx.w, g.Nv);
    c.Iw = u0;
    c.Jw = v0;
    c.nI = u1 > u0 && v1 > v0 ? (u1 - u0 + 15) / 16 : 0;
    c.nJ = u1 > u0 && v1 > v0 ? (v1 - v0 + 15) / 16 : 0;
    c.npi = (c.nI + BR - 1) / BR;
    c.npj = (c.nJ + BC - 1) / BC;
    return c;
  };
  auto win_of = [&](const Cov& c, int pp, int* nIp, int* nJp) {
    const int pi = pp / c.npj, pj = pp - (pp / c.npj) * c.npj;
    *nIp = min(BR, c.nI - BR * pi);
    *nJp = min(BC, c.nJ - BC * pj);
    WinRect w;
    w.r0 = c.Iw + 16 * BR * pi - h;
    w.c0 = c.Jw + 16 * BC * pj - h;
    w.nr = 16 * *nIp + 2 * h;
    w.nc = 32 * NK;
    return w;
  };
  auto next_live = [&](int from, Cov* cv) {
    for (; from < n_items; from += gridDim.x) {
      *cv = cov_of(from);
      if (cv->nI > 0) break;
    }
    return from;
  };
  auto depth_of = [&](int item) { return zca[item + opaque(0)]; };
  // a piece's window groups into the BF16 image (masked, then rounded to BF16)
  auto put_bf16 = [&](const float* src, const WinRect& w, bool edge, const f32x4 (&buf)[PG]) {
    const WinStage st = win_stage(g, w, tid, NT);
    auto store = [&](int r, f32x4 v) {
      v = mask_group(g, w, st, r, v);
      *reinterpret_cast<uint2*>(img + r * pitch + 4 * st.cg) = make_uint2(bf16_pair(v[0], v[1]), bf16_pair(v[2], v[3]));
    };
#pragma unroll
    for (int e = 0; e < PG; ++e) {
      const int r = st.r0 + e * st.step;
      if (r < w.nr) store(r, buf[e]);
    }
    for (int r = st.r0 + PG * st.step; r < w.nr; r += st.step)
      store(r, edge ? load_group<true>(src, g, w, st, r) : load_group<false>(src, g, w, st, r));
  };

  f32x4 buf[PG];
  Cov c;
  int it = next_live(blockIdx.x, &c), pp = 0;
  float zk = 0.f;
  if (it < n_items) {
    int a, b;
    fetch_win<PG>(in + (size_t)it * plane, g, win_of(c, 0, &a, &b), it == 0 || it == n_items - 1, tid, NT, buf);
    zk = depth_of(it);
  }
  zero_lds(T0, t1w + (h + 1) * L2, tid, NT);  // both copies (and the gap between them)
  __syncthreads();
  while (it < n_items) {
    const float* src = in + (size_t)it * plane;
    float* dst = out + (size_t)it * plane;
    int nIp, nJp;
    const WinRect w = win_of(c, pp, &nIp, &nJp);
    put_bf16(src, w, it == 0 || it == n_items - 1, buf);
    if (pp == 0) taps_to_bf16_rows(g, it % g.Nk, zk, T0, T1, L2, tid, NT);
    int nit = it, npp = pp + 1;
    Cov cn = c;
    if (npp == c.npi * c.npj) {
      npp = 0;
      nit = next_live(it + gridDim.x, &cn);
    }
    __syncthreads();
    float zn = zk;
    if (nit < n_items) {
      int a, b;
      fetch_win<PG>(in + (size_t)nit * plane, g, win_of(cn, npp, &a, &b), nit == 0 || nit == n_items - 1, tid, NT,
                    buf);
      if (npp == 0) zn = depth_of(nit);
    }
    // this wavefront's tap rows p in [pa, pz)
    const int pa = -h + ((2 * h + 1) * wave) / NW, pz = -h + ((2 * h + 1) * (wave + 1)) / NW;
    // every B run of the lane has the parity of its first one (tile 0, K-step 0):
    // tile t, step s start 16 s - 8 t words further in the same copy
    const int x0 = 8 * kqd - m + kBwX0;
    const unsigned* bb = ((x0 & 1) ? T1 : T0) + (x0 >> 1);
    const __bf16* ab = img + (m + h) * pitch + 8 * kqd;
    const bool r1 = nIp > 1, t1 = nJp > 1;
    f32x4c acc[BR][BC];
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int t = 0; t < BC; ++t) acc[r][t] = f32x4c{0.f, 0.f, 0.f, 0.f};
    // the operands of tap row p: B runs of both column tiles, A fragments of both
    // row tiles (rows past the piece's tiles read the image's first rows, unused)
    struct Ops {
      u32x4c B[BC][NK], A[BR][NK];
    };
    auto load = [&](int p, Ops& o) {
      const unsigned* row = bb + (p < 0 ? -p : p) * L2;
      const __bf16* a0 = ab + p * pitch;
#pragma unroll
      for (int t = 0; t < BC; ++t)
#pragma unroll
        for (int s2 = 0; s2 < NK; ++s2) {
          const unsigned* w = row + 16 * s2 - 8 * t;
          o.B[t][s2] = u32x4c{w[0], w[1], w[2], w[3]};
        }
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int s2 = 0; s2 < NK; ++s2)
          o.A[r][s2] = *reinterpret_cast<const u32x4c*>(a0 + 16 * r * pitch + 32 * s2);
    };
    auto mfma = [&](const u32x4c& A, const u32x4c& B, f32x4c& c) {
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8c, A), __builtin_bit_cast(bf16x8c, B), c,
                                                  0, 0, 0);
    };
    // full: a piece of 2 x 2 tiles, no tests inside the loop
    auto rows_loop = [&](auto full) {
      auto compute = [&](const Ops& o) {
#pragma unroll
        for (int s2 = 0; s2 < NK; ++s2) {
          mfma(o.A[0][s2], o.B[0][s2], acc[0][0]);
          if (full || t1) mfma(o.A[0][s2], o.B[1][s2], acc[0][1]);
          if (full || r1) {
            mfma(o.A[1][s2], o.B[0][s2], acc[1][0]);
            if (full || t1) mfma(o.A[1][s2], o.B[1][s2], acc[1][1]);
          }
        }
      };
#pragma unroll 1
      for (int p = pa; p < pz; ++p) {
        Ops o;
        load(p, o);
        compute(o);
      }
    };
    if (r1 && t1)
      rows_loop(std::true_type{});
    else
      rows_loop(std::false_type{});
    // every wavefront parks its sums; wavefront t < 4 then adds tile t's eight
    // parts in wavefront order and stores the tile
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int t = 0; t < BC; ++t) red[((wave * BR + r) * BC + t) * 64 + lane] = acc[r][t];
    __syncthreads();
    if (wave < BR * BC) {
      const int r = wave / BC, t = wave % BC;
      if (r < nIp && t < nJp) {
        f32x4c sum = red[(r * BC + t) * 64 + lane];
#pragma unroll 1
        for (int v = 1; v < NW; ++v) sum += red[((v * BR + r) * BC + t) * 64 + lane];
        const int Ip = w.r0 + h, Jp = w.c0 + h;
        const int j = Jp + 16 * t + m;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = Ip + 16 * r + 4 * kqd + e;
          if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = sum[e];
        }
      }
    }
    __syncthreads();  // the image, the sums' area and (before a new item) the taps are rewritten next
    it = nit;
    pp = npp;
    c = cn;
    zk = zn;
  }
}

static size_t bf16_adj_win_lds(int h, const Bf16AdjWin& bw) {
  size_t b = (size_t)4 * (bw_t1_words(h, bw.L2) + (h + 1) * bw.L2);
  b = (b + 15) & ~(size_t)15;
  b += ((size_t)bw.rows * bw.pitch * 2 + 15) & ~(size_t)15;
  b += (size_t)8 * 4 * 64 * 16;  // the parts' sums
  return b + 16;
}

template <int NK>
static hipError_t launch_bf16_adj_win_nk(const Geo<float>& g, int nb, const int4* box, const float* z,
                                         const float* in, float* out, hipStream_t s) {
  Bf16AdjWin bw;
  bw.rows = 32 + 2 * g.h;
  bw.pitch = 32 * NK + 16;
  bw.L2 = 16 * NK + 17;
  const size_t lds = bf16_adj_win_lds(g.h, bw);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const void* kern = (const void*)k_conv_bf16_adj_win<NK>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)nb * g.Nk;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  const int grid = persistent_grid(kern, 512, lds, 1, n_items);
  hipLaunchKernelGGL((k_conv_bf16_adj_win<NK>), dim3(grid), dim3(512), lds, s, g, bw, (int)n_items, box, z, in, out);
  return hipGetLastError();
}

// The windowed adjoint for K-step counts up to 4 (h <= 48); false: not served.
static bool launch_bf16_adj_win(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                float* out, hipStream_t s, hipError_t* err) {
  const int nk = (32 + 2 * g.h + 31) / 32;
  switch (nk) {
    case 1: *err = launch_bf16_adj_win_nk<1>(g, nb, box, z, in, out, s); return true;
    case 2: *err = launch_bf16_adj_win_nk<2>(g, nb, box, z, in, out, s); return true;
    case 3: *err = launch_bf16_adj_win_nk<3>(g, nb, box, z, in, out, s); return true;
    case 4: *err = launch_bf16_adj_win_nk<4>(g, nb, box, z, in, out, s); return true;
    default: return false;
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

template <int NK, int BR, int BC, int NWB, int NWP, int SUP>
static hipError_t launch_bf16_nk(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                 float* out, hipStream_t s, int box_rows) {
  Bf16Plan q;
  q.X0 = g.h + 8;
  q.L = 2 * g.h + 16;
  const int out_rows = SUP == CONV_IN_BOX ? (box_rows + 2 * g.h < g.Nu ? box_rows + 2 * g.h : g.Nu) : box_rows;
  const int tr = (out_rows + 15) / 16;
  const int in_rows = SUP == CONV_IN_BOX ? box_rows : (box_rows + 2 * g.h < g.Nu ? box_rows + 2 * g.h : g.Nu);
  int rows = in_rows + 30;
  if (rows > 16 * tr + 2 * g.h) rows = 16 * tr + 2 * g.h;
  if (rows < 31) rows = 31;  // at least one row of data per chunk
  q.pitch = pitch_bf16(32 * NK);
  // the image area also holds the unique FP32 taps and the parts' sums
  const int red_rows = (NWB * (NWP - 1) * BR * BC * 1024 + 2 * q.pitch - 1) / (2 * q.pitch);
  q.img_rows = rows > red_rows ? rows : red_rows;
  q.kq_floats = (g.h + 1) * (g.h + 1);
  const size_t lds = cb_tap_bytes(g.h, q) + cb_img_bytes(q);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const void* kern = (const void*)k_conv_bf16<NK, BR, BC, NWB, NWP, SUP>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)nb * g.Nk;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_conv_bf16<NK, BR, BC, NWB, NWP, SUP>), dim3((unsigned)n_items), dim3(64 * NWB * NWP), lds, s,
                     g, q, box, z, in, out);
  return hipGetLastError();
}

// Forward: two wavefronts, each a block of 6 x 3 tiles (together the reach of a
// rectangle inside the field limits); adjoint: four wavefronts sharing one block
// of 2 x 2 tiles (the rectangle itself), each a quarter of the tap rows.
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
  constexpr bool F = SUP == CONV_IN_BOX;
  constexpr int BR = F ? 6 : 2, BC = F ? 3 : 2, NWB = F ? 2 : 1, NWP = F ? 1 : 4;
  if (nk <= 1) return launch_bf16_nk<1, BR, BC, NWB, NWP, SUP>(g, nb, box, z, in, out, s, br);
  if (nk == 2) return launch_bf16_nk<2, BR, BC, NWB, NWP, SUP>(g, nb, box, z, in, out, s, br);
  return launch_bf16_nk<3, BR, BC, NWB, NWP, SUP>(g, nb, box, z, in, out, s, br);
}

hipError_t launch_conv_mfma_bf16(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                 hipStream_t s, const int* box, int support) {
  const int4* bx = reinterpret_cast<const int4*>(box);
  if (support == CONV_OUT_BOX && bx) {
    // the windowed adjoint, unless the fluence corrections widen the rectangles (as
    // for FP32, the tiled kernel's chunks serve them)
    hipError_t e;
    if (!g.fcorr && launch_bf16_adj_win(g, nb, bx, z, in, out, s, &e)) return e;
    return launch_bf16_sup<CONV_OUT_BOX>(g, nb, bx, z, in, out, s);
  }
  // the forward with the rectangle in registers where its tap rows fit (not with
  // the fluence corrections' widened rectangles, as for FP32)
  if (support == CONV_IN_BOX && bx && !g.fcorr && conv_fwd_reg_supported(g, true))
    return launch_conv_fwd_reg(g, nb, z, in, out, s, box, true);
  // forward, or no box: the input support is the box (the whole plane without one)
  return launch_bf16_sup<CONV_IN_BOX>(g, nb, support == CONV_DENSE ? nullptr : bx, z, in, out, s);
}

}  // namespace pdrt
