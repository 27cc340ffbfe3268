// conv_fwd_reg.hip — the forward per-plane lateral convolution (arXiv:2512.18863
// §2.2.6, Eq. 8) on the CDNA4 matrix cores, in FP32 or with BF16 operands (FP32
// sums), for an input that vanishes outside the aperture rectangle (the primary
// P = F G).
//
// out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q], with in zero outside the box
// [r0, r1) x [c0, c1).  Split by tap row p and by box row r:
//   Y_p[r][j] = sum_c K[p][c - j] in[r][c],   out[r - p][j] += Y_p[r][j],
// and since K[-p][.] = K[p][.] the same product also gives out[r + p][j] += Y_p[r][j].
// The input is small (the box) and the output large (the box and the kernel's
// reach around it), so the box stays in registers for the whole plane and only
// the Toeplitz band of tap row p is read from LDS.  Matrix instructions with
// M = 16 output columns j, N = 16 box rows r and K = box columns c:
//   A[m][k] = K[p][c_k - j_m] (from the extended tap row),
//   B[k][n] = in[r_n][c_k] (registers, loaded once per plane);
// FP32: v_mfma_f32_16x16x4_f32, four per group of 16 box columns; BF16:
// v_mfma_f32_16x16x32_bf16, one per group of 32 box columns.  Both leave the
// product's box rows along the lanes of each 16-lane row of the result, so moving
// it by p rows is a DPP row shift within those 16 lanes: the part that stays in a
// 16-row output block is one shift, the part that crosses into the neighbouring
// block the complementary one; lanes shifted in from outside the row read zero.
// Each wavefront owns one 16-column strip of the output and keeps its rows (the
// box rows and two blocks above and below, for h <= 31) in registers over all tap
// rows, then stores them; the rest of the plane (outside the strips) is written
// with zeros.  A box larger than one chunk adds its chunks' strips into a cleared
// plane with atomic adds, each address by its own wavefront only, in chunk order
// (deterministic).
//
// Work skipped: column groups of which no column lies within h of the strip (one
// uniform branch per group and tap row; inside a group the band's zero taps are
// multiplied).  The products of skipped groups are exact zeros.  The sum of every
// output runs over p = 0, 1, ..., h in order, within a tap row over the box's row
// blocks, and within a product over the box columns (deterministic; the rounding
// differs from a direct sum only in order, and for BF16 in the operands' rounding).
#include "conv_common.hpp"

namespace pdrt {

typedef float f32x4r __attribute__((ext_vector_type(4)));
typedef unsigned u32x4r __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8r __attribute__((ext_vector_type(8)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));  // four floats at any word address

constexpr int kRegNW = 8;    // wavefronts per workgroup (output strips in parallel)
constexpr int kRegQB = 2;    // output blocks of 16 rows above and below a row chunk
constexpr int kRegMaxH = 16 * (kRegQB - 1) + 15;  // largest half-width the blocks reach

// Columns per group (one uniform branch each): FP32 16 (four K = 4 steps), BF16 32.
template <bool BF>
struct RegPrec {
  static constexpr int GW = BF ? 32 : 16;
};

// Extended tap row: kx[p][x] = K[p][|x - off|] for |x - off| <= h, else 0.  A group
// in reach has c - j in [-(h + GW + 14), h + GW + 14]; a group out of reach reads
// x in [0, GW + 14], which must be zero: off = h + GW + 15.  FP32 then reads x in
// [1, 2h + 61]; BF16 reads eight taps from each start, up to x = 2h + 93 (its rows
// are two copies of bf16 pairs, the second shifted by one tap).
__host__ __device__ inline int reg_tap_off(int h, bool bf) { return h + (bf ? 32 : 16) + 15; }
__host__ __device__ inline int reg_tap_len(int h, bool bf) { return bf ? 2 * h + 96 : 2 * h + 62; }

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

// Tap row P's products Y[t] of the box's row blocks t, added to the strip's output
// blocks O p rows up and down (block kRegQB + t holds the rows of box block t).
template <int P, int T, int NB>
__device__ __forceinline__ void reg_add_shifted(const f32x4r (&Y)[T], f32x4r (&O)[NB]) {
  constexpr int S = P & 15, Q = P >> 4, c = kRegQB;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const f32x4r y = Y[t];
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

// Operands of one precision.  FP32: A of group u and step s is one tap (aaddr[u] +
// P E + s), B[t][4 u + s] one input value.  BF16: A of group u is eight taps read
// as four words from the copy of the row whose pairs start at the lane's parity
// (aaddr[u] + P E / 2 words), B[t][u] eight inputs as four words.
template <bool BF, int T, int SU>
struct RegOps;

template <int T, int SU>
struct RegOps<false, T, SU> {
  typedef float BOp[T][4 * SU];
  typedef const float* Addr;
  template <int P>
  static __device__ __forceinline__ void tap_row(const Addr (&aaddr)[SU], int E, unsigned umask, const BOp& B,
                                                 f32x4r (&Y)[T]) {
    float A[4 * SU];
#pragma unroll
    for (int u = 0; u < SU; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) A[4 * u + s] = aaddr[u][P * E + s];
    // group 0 always runs and starts the chains from zero (out of reach its A is
    // zero); the others run when their bit of umask is set and accumulate in place
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
  }
};

template <int T, int SU>
struct RegOps<true, T, SU> {
  typedef u32x4r BOp[T][SU];
  typedef const unsigned* Addr;
  template <int P>
  static __device__ __forceinline__ void tap_row(const Addr (&aaddr)[SU], int E, unsigned umask, const BOp& B,
                                                 f32x4r (&Y)[T]) {
    u32x4r A[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const unsigned* a = aaddr[u] + P * (E / 2);
      A[u] = u32x4r{a[0], a[1], a[2], a[3]};
    }
#pragma unroll
    for (int t = 0; t < T; ++t)
      Y[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8r, A[0]),
                                                     __builtin_bit_cast(bf16x8r, B[t][0]), f32x4r{0.f, 0.f, 0.f, 0.f},
                                                     0, 0, 0);
#pragma unroll
    for (int u = 1; u < SU; ++u)
      if (umask & (1u << u)) {
#pragma unroll
        for (int t = 0; t < T; ++t)
          Y[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8r, A[u]),
                                                         __builtin_bit_cast(bf16x8r, B[t][u]), Y[t], 0, 0, 0);
      }
  }
};

template <bool BF, int P, int T, int SU, int NB>
__device__ __forceinline__ void reg_tap_rows(int h, const typename RegOps<BF, T, SU>::Addr (&aaddr)[SU], int E,
                                             unsigned umask, const typename RegOps<BF, T, SU>::BOp& B,
                                             f32x4r (&O)[NB]) {
  if constexpr (P <= kRegMaxH) {
    if (P > h) return;
    f32x4r Y[T];
    RegOps<BF, T, SU>::template tap_row<P>(aaddr, E, umask, B, Y);
    reg_add_shifted<P, T, NB>(Y, O);
    reg_tap_rows<BF, P + 1, T, SU, NB>(h, aaddr, E, umask, B, O);
  }
}

__device__ __forceinline__ unsigned reg_bf16_pair(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (unsigned)(*reinterpret_cast<const unsigned short*>(&a)) |
         ((unsigned)(*reinterpret_cast<const unsigned short*>(&b)) << 16);
}

// LDS words of the tap rows: FP32 (h + 1) E floats; BF16 two copies of (h + 1) E / 2
// pairs.  Rounded up to a multiple of four words (the plane copy is 16-byte aligned).
__host__ __device__ inline size_t reg_tap_words(int h, bool bf) {
  return ((size_t)(h + 1) * reg_tap_len(h, bf) + 3) & ~(size_t)3;
}

// One workgroup per (control point, plane) item.  T: row blocks of 16 box rows per
// chunk; SU: column groups per chunk (boxes larger than a chunk are taken chunk by
// chunk).  LDS: the tap rows.
template <bool BF, int T, int SU>
__global__ void __launch_bounds__(64 * kRegNW) k_conv_fwd_reg(Geo<float> g, const int4* __restrict__ box,
                                                              const float* __restrict__ zca,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  typedef RegOps<BF, T, SU> Ops;
  constexpr int NT = 64 * kRegNW;
  constexpr int GW = RegPrec<BF>::GW;
  constexpr int NB = T + 2 * kRegQB;
  const int h = g.h, E = reg_tap_len(h, BF), off = reg_tap_off(h, BF);
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
  const int nrc = (r1 - r0 + 16 * T - 1) / (16 * T), ncc = (c1 - c0 + GW * SU - 1) / (GW * SU);

  // B fragments of box chunk (rc, cc).  FP32: lane (n, kk) holds in[R + 16 t + n][C +
  // 16 u + 4 kk + s] for step s of group u (the K index of a matrix step may stand for
  // any column as long as A and B agree: here a lane's four columns of a group are
  // consecutive); BF16: in[R + 16 t + n][C + 32 u + 8 kk .. + 7] as bf16 pairs.  Each
  // run of four columns is one four-word load from a row inside the box (rows past it
  // and runs past its last column read the box's first row or column and are
  // cleared); a run that starts inside the box may read up to three words past its
  // last column, i.e. past the end of the row into the next one (or, after the
  // batch's last row, into the workspace that follows the convolution's input).
  typename Ops::BOp B;
  auto load_b = [&](int rc, int cc) {
    const int R = r0 + 16 * T * rc, C = c0 + GW * SU * cc;
    auto run4 = [&](int r, int c) {
      const f32x4u x = *reinterpret_cast<const f32x4u*>(src + (size_t)(r < r1 ? r : r0) * Nv + (c < c1 ? c : c0));
      f32x4r v;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (r < r1 && c + e < c1) ? x[e] : 0.f;
      return v;
    };
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int r = R + 16 * t + n;
      if constexpr (BF) {
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int c = C + 32 * u + 8 * kk;
          const f32x4r a = run4(r, c), b = run4(r, c + 4);
          B[t][u] = u32x4r{reg_bf16_pair(a[0], a[1]), reg_bf16_pair(a[2], a[3]), reg_bf16_pair(b[0], b[1]),
                           reg_bf16_pair(b[2], b[3])};
        }
      } else {
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const f32x4r v = run4(r, C + 16 * u + 4 * kk);
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) B[t][4 * u + s2] = v[s2];
        }
      }
    }
  };
  const int jt0 = wave;  // this wavefront's first strip
  if (jt0 < njt) load_b(0, 0);  // in flight while the taps are built

  if constexpr (BF) {
    // word i of copy c holds taps (2i + c, 2i + c + 1): element x of row p is half-word
    // x - c of the copy's row.  The taps go straight into both copies; the elements
    // farther than h from `off` are zero: the words made only of them are cleared
    // whole, and the two elements just outside the taps (off - h - 1, off + h + 1)
    // one by one.  Those entries are disjoint from the taps, so no barrier between.
    const int W2 = E / 2;
    unsigned* t0 = reinterpret_cast<unsigned*>(lds);
    unsigned* t1 = t0 + (size_t)(h + 1) * W2;
    unsigned short* H0 = reinterpret_cast<unsigned short*>(t0);
    unsigned short* H1 = reinterpret_cast<unsigned short*>(t1);
    {
      const TapParams<float> tp = tap_params(g, k, zca[bk]);
      const int h1 = h + 1;
      for (int t = tid; t < h1 * (h1 + 1) / 2; t += NT) {
        int q = (int)((sqrtf((float)(8 * t + 1)) - 1.f) * 0.5f);
        if ((q + 1) * (q + 2) / 2 <= t) ++q;
        if (q * (q + 1) / 2 > t) --q;
        const int p = t - q * (q + 1) / 2;
        const __bf16 bv = (__bf16)tap_value(tp, p, q);
        const unsigned short v = *reinterpret_cast<const unsigned short*>(&bv);
        const int rp = 2 * W2 * p + off, rq = 2 * W2 * q + off;
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
    const int xa = off - h, xb = off + h;             // the taps' elements
    const int nl0 = xa / 2, nl1 = (xa - 1) / 2;        // whole zero words left of them
    const int ir0 = xb / 2 + 1, ir1 = (xb - 1) / 2 + 1; // first whole zero word right of them
    const int n0 = nl0 + (W2 - ir0), n1 = nl1 + (W2 - ir1);
    for (int p = wave; p <= h; p += kRegNW) {
      for (int i = lane; i < n0 + n1; i += 64) {
        if (i < n0) {
          t0[p * W2 + (i < nl0 ? i : ir0 + (i - nl0))] = 0u;
        } else {
          const int j = i - n0;
          t1[p * W2 + (j < nl1 ? j : ir1 + (j - nl1))] = 0u;
        }
      }
      if (lane < 4) {
        const int c = lane & 1, x = lane < 2 ? xa - 1 : xb + 1;
        if (x - c >= 0 && x - c < 2 * W2) (c ? H1 : H0)[2 * W2 * p + x - c] = 0;
      }
    }
  } else {
    // the taps straight into the rows, and the rows' entries farther than h from
    // `off` (the ranges [0, off - h) and (off + h, E)) cleared: disjoint entries,
    // so no barrier between the two
    taps_to_kx(g, k, zca[bk], lds, E, off, tid, NT, 1.f);
    const int zl = off - h, zr = E - (off + h + 1);
    for (int p = wave; p <= h; p += kRegNW)
      for (int i = lane; i < zl + zr; i += 64) lds[p * E + (i < zl ? i : off + h + 1 + (i - zl))] = 0.f;
  }
  // With one chunk the strips are stored once and the plane outside them [wr0, wr1)
  // x [cw0, cw0 + 16 njt) is zero; with several the whole plane is cleared first
  // and the strips are added (the barrier below orders the clearing before them).
  const bool single = nrc == 1 && ncc == 1;
  const int wr0 = single ? r0 - 16 * kRegQB : 0, wr1 = single ? r0 + 16 * (T + kRegQB) : 0;
  {
    // whole rows above and below the window (two contiguous ranges), then the
    // columns left and right of it in the rows between
    const int zr0 = min(max(wr0, 0), Nu), zr1 = min(max(wr1, zr0), Nu);
    const int cz1 = min(Nv, cw0 + 16 * njt);
    const int top = zr0 * Nv, nfull = top + (Nu - zr1) * Nv;
    for (int d = tid; d < nfull; d += NT) dst[d < top ? d : zr1 * Nv + (d - top)] = 0.f;
    const int side = cw0 + (Nv - cz1), nside = (zr1 - zr0) * side;
    for (int d = tid; d < nside; d += NT) {
      const int rr = d / side, cc = d - rr * side;
      dst[(size_t)(zr0 + rr) * Nv + (cc < cw0 ? cc : cz1 + (cc - cw0))] = 0.f;
    }
  }
  __syncthreads();

  for (int jt = jt0; jt < njt; jt += kRegNW) {
    const int J = cw0 + 16 * jt;  // the strip's first output column
    for (int rc = 0; rc < nrc; ++rc) {
      const int R = r0 + 16 * T * rc;
      f32x4r O[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) O[q] = f32x4r{0.f, 0.f, 0.f, 0.f};
      for (int cc = 0; cc < ncc; ++cc) {
        if (jt != jt0 || rc != 0 || cc != 0) load_b(rc, cc);
        const int C = c0 + GW * SU * cc;
        const int nsu = min(SU, (c1 - C + GW - 1) / GW);
        // column groups with a column within h of the strip [J, J + 16)
        const int lo = J - h - C - (GW - 1), hi = J + 15 + h - C;
        const int ua = lo <= 0 ? 0 : (lo + GW - 1) / GW;
        const int ub = min(nsu - 1, hi >= 0 ? hi / GW : -1);
        if (ua > ub) continue;
        // A of group u in tap row p starts at x = C + GW u + KL kk - J - m + off (m the
        // lane's output column, KL its first box column's step: 4 for FP32, whose
        // steps s add s, 8 for BF16); groups outside [ua, ub] start at x = 15 +
        // KL kk - m, where the row is zero (group 0 runs with it, the others are
        // skipped)
        constexpr int KL = BF ? 8 : 4;
        typename Ops::Addr aaddr[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int x = (u >= ua && u <= ub) ? C + GW * u + KL * kk - J - n + off : 15 + KL * kk - n;
          if constexpr (BF) {
            const unsigned* t0 = reinterpret_cast<const unsigned*>(lds);
            aaddr[u] = (x & 1) ? t0 + (size_t)(h + 1) * (E / 2) + (x >> 1) : t0 + (x >> 1);
          } else {
            aaddr[u] = lds + x;
          }
        }
        const unsigned umask = __builtin_amdgcn_readfirstlane((2u << ub) - (1u << ua));  // bits ua .. ub
        reg_tap_rows<BF, 0, T, SU, NB>(h, aaddr, E, umask, B, O);
      }
      // the strip's rows R - 16 kRegQB + 16 q + n and columns J + 4 kk + e that lie in
      // the plane (stored with one chunk, added with several); only this wavefront
      // writes them
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int row = R - 16 * kRegQB + 16 * q + n;
        if (row >= 0 && row < Nu) {
          float* o = dst + (size_t)row * Nv + J + 4 * kk;
          if (single && J + 4 * kk + 3 < Nv) {
            *reinterpret_cast<f32x4u*>(o) = O[q];  // the lane's four consecutive columns
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float v = O[q][e];
              if (J + 4 * kk + e < Nv) {
                if (single) o[e] = v;
                else unsafeAtomicAdd(o + e, v);
              }
            }
          }
        }
      }
    }
  }
}

// LDS of the kernel: the tap rows.
static size_t reg_lds(int h, bool bf) { return sizeof(float) * reg_tap_words(h, bf); }

bool conv_fwd_reg_supported(const Geo<float>& g, bool bf16) {
  return g.h >= 1 && g.h <= kRegMaxH && reg_lds(g.h, bf16) <= 160 * 1024;
}

template <bool BF, int T, int SU>
static hipError_t launch_reg_cfg(const Geo<float>& g, int nb, const int4* box, const float* z, const float* in,
                                 float* out, hipStream_t s) {
  const size_t lds = reg_lds(g.h, BF);
  const void* kern = (const void*)k_conv_fwd_reg<BF, T, SU>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)nb * g.Nk;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_conv_fwd_reg<BF, T, SU>), dim3((unsigned)n_items), dim3(64 * kRegNW), lds, s, g, box, z, in,
                     out);
  return hipGetLastError();
}

// The chunk shape from the largest rectangle that jaws inside the field limits give
// (larger rectangles are taken in several chunks).
hipError_t launch_conv_fwd_reg(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                               hipStream_t s, const int* box, bool bf16) {
  if (!conv_fwd_reg_supported(g, bf16) || !box) return hipErrorInvalidConfiguration;
  const int4* bx = reinterpret_cast<const int4*>(box);
  const int half_u = (g.Nu - 1) / 2 - g.h, half_v = (g.Nv - 1) / 2 - g.h;  // field limit in pixels
  const int br = 2 * (half_u > 0 ? half_u : 0) + 4, bc = 2 * (half_v > 0 ? half_v : 0) + 4;
  int ch = (br > bc ? br : bc);
  ch = (ch + 15) / 16;
  if (bf16) {
    if (ch <= 1) return launch_reg_cfg<true, 1, 1>(g, nb, bx, z, in, out, s);
    if (ch == 2) return launch_reg_cfg<true, 2, 1>(g, nb, bx, z, in, out, s);
    if (ch == 3) return launch_reg_cfg<true, 3, 2>(g, nb, bx, z, in, out, s);
    return launch_reg_cfg<true, 4, 2>(g, nb, bx, z, in, out, s);
  }
  if (ch <= 1) return launch_reg_cfg<false, 1, 1>(g, nb, bx, z, in, out, s);
  if (ch == 2) return launch_reg_cfg<false, 2, 2>(g, nb, bx, z, in, out, s);
  if (ch == 3) return launch_reg_cfg<false, 3, 3>(g, nb, bx, z, in, out, s);
  return launch_reg_cfg<false, 4, 4>(g, nb, bx, z, in, out, s);
}

}  // namespace pdrt
