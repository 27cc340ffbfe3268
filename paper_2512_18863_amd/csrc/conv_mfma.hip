// conv_mfma.hip — the per-plane lateral convolution (arXiv:2512.18863 §2.2.6,
// Eq. 8) in FP32 on the CDNA4 matrix cores (the BF16 variant is conv_bf16.hip).
//
// For one plane, out[i][j] = sum_{p,q} K[p][q] in[i+p][j+q] (zero padded).  Fixing
// the tap row p, the sum over q is a product with a banded Toeplitz matrix:
//   out[i][j0..j0+15] += in[i+p][j0-h .. j0+15+h] * T_p,  T_p[c][n] = K[p][c - h - n],
// so a 16 x 16 output tile is a GEMM with K-dimension 16 + 2h over input columns.
// The Toeplitz operand depends only on (p, column step), never on the tile, so a
// wavefront loads it once per step and streams the input rows of all its tiles
// past it.  A workgroup owns a region of up to 6 x 6 tiles (96 x 96 outputs) and
// walks the (control point, plane) items of that region: workgroups are
// persistent (one per CU and LDS slot), the zero halo of the LDS image is written
// once, and each item's input is fetched into registers while the previous item's
// matrix instructions run, so staging costs an LDS write instead of a global-load
// round trip.  The inner loop is branch free and software pipelined: the operands
// of step t+1 are loaded from LDS before the matrix instructions of step t are
// issued.
//
// v_mfma_f32_16x16x4_f32.  Tap rows p and -p are equal (the kernel is radially
// symmetric), so rows i+p and i-p are added before the product and only h+1 tap
// rows are multiplied (row 0 with halved taps).
#include "conv_common.hpp"

namespace pdrt {

typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// One 16 x 16 output tile at plane position (i0, j0), clipped to the plane.
__device__ __forceinline__ void store_tile_at(const Geo<float>& g, int i0, int j0, int lane, const f32x4& acc,
                                              float* dst) {
  const int m = lane & 15, r4 = lane >> 4;
  const int j = j0 + m;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * r4 + r;
    if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[r];
  }
}

// The same, storing only rows >= ilo and columns >= jlo (tiles of a shifted grid).
__device__ __forceinline__ void store_tile_from(const Geo<float>& g, int i0, int j0, int ilo, int jlo, int lane,
                                                const f32x4& acc, float* dst) {
  const int m = lane & 15, r4 = lane >> 4;
  const int j = j0 + m;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * r4 + r;
    if (i >= ilo && j >= jlo && i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[r];
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

// Row pitch (elements): the smallest one not below `cols` that is congruent to 8
// mod 16.  A half-wavefront's 16-byte operand reads (16 rows, two four-column
// groups) then fall in 32 distinct 16-byte slots of a 512-byte LDS line, which
// gfx950 serves without bank conflicts; pitches congruent to 4 mod 16 (or 0 mod
// 16) were measured at twice the cycles per read.
static int pitch_f32(int cols) { return ((cols + 7) / 16) * 16 + 8; }

static F32Shape f32_shape(int h, const RegionShape& r) {
  F32Shape s;
  s.SS = (MT + 2 * h + 15) / 16;
  s.E = 16 * s.SS + 16;
  s.rows = MT * r.TI + 2 * h;
  s.pitch = pitch_f32(MT * r.TJ + 16 * s.SS);
  return s;
}

// CONV_IN_BOX image.  A tile reads only the tap rows and column super-steps that
// reach the input rectangle [r0, r1) x [c0, c1), so its reads stay inside rows
// [r0 - 15, r1 + 15) and columns [c0 - 18, c1 + 15) (the window start is rounded
// down to a multiple of 4 and may be moved left by less than 16 to keep the
// window inside the extended tap row).  The image is therefore placed at the
// rectangle, not at the region: its first row is R0 = max(I - h, r0 - 15) and its
// first column C0 the largest of J - h, J - h + 4, ... not above c0 - 18 (so the
// 16-byte reads stay aligned), with (I, J) the region's shifted origin.  The
// rectangle is clipped to the plane and to the region's reach, so the image needs
// at most min(Nu, rows of reach) + 30 rows and min(Nv, columns of reach) + 36
// columns, and never more than the region image.
static F32Shape f32_shape_in_box(int h, const RegionShape& r, int Nu, int Nv) {
  F32Shape s = f32_shape(h, r);
  auto lo = [](int a, int b) { return a < b ? a : b; };
  s.rows = lo(lo(Nu, MT * r.TI + 2 * h) + 30, s.rows);
  s.pitch = pitch_f32(lo(lo(Nv, MT * r.TJ + 2 * h) + 36, MT * r.TJ + 16 * s.SS));
  return s;
}

static size_t f32_lds(int h, const F32Shape& fs) {
  // image, extended taps, unique taps, and one counter
  return sizeof(float) * ((size_t)fs.rows * fs.pitch + (size_t)(h + 1) * fs.E + (size_t)(h + 1) * (h + 1)) + 16;
}

// CONV_IN_BOX: after the counter, per tile its step ranges (8 ints) and the tile
// order (one int), RMAX x RMAX tiles.
constexpr size_t kBoxTileLds = sizeof(int) * 9 * RMAX * RMAX;

constexpr int PF = 12;  // prefetched elements per thread

// The matrix loop over tap rows p in [pa, pb] and super-steps u in [ua, ub] for
// NA tiles that share the Toeplitz operand.  Two operand sets are loaded
// alternately one step ahead of their use: the loop body covers two steps and the
// last one or two steps are peeled, so every load is of a step that is computed
// and each matrix step waits only for its own operands, never for the loads in
// flight for the next step.  The LDS addresses advance by a running increment (16
// along a row of super-steps, a jump to the next tap row at its end), so a step
// costs a few scalar instructions besides its loads, adds and matrix work.
// B[k][n] of instruction s in super-step u = K[p][16 u + 4 k + s - h - n]
//                                           = kx[p][16 u + 4 k + s + 15 - n].
// MODE 0 adds the two folded rows i + p and i - p; MODE 1 uses row i + p only and
// MODE 2 row i - p only (tap rows whose other row lies outside the input's
// support, where it would add exact zeros): half the operand loads, no adds.
struct StepWalk {
  int lu, last;          // super-step of the next load within its row, and the row's last one
  int da, dm, db;        // address jumps at the end of a row (rows i + p, i - p, taps)
  __device__ __forceinline__ StepWalk(int nu, int pitch, int E) {
    lu = 0;
    last = nu - 1;
    const int span = 16 * (nu - 1);
    da = pitch - span;
    dm = -pitch - span;
    db = E - span;
  }
  // the increments of the addresses after a load, and the walk's advance
  __device__ __forceinline__ void next(int& ia, int& im, int& ib) {
    const bool wrap = lu == last;
    ia = wrap ? da : 16;
    im = wrap ? dm : 16;
    ib = wrap ? db : 16;
    lu = wrap ? 0 : lu + 1;
  }
};

template <int NA, int MODE = 0>
__device__ __forceinline__ void f32_steps(const float* const* abase, const float* bbase, int pitch, int E, int pa,
                                          int pb, int ua, int ub, f32x4* acc) {
  const int nu = ub - ua + 1;
  const int total = (pb >= pa && nu > 0) ? (pb - pa + 1) * nu : 0;
  if (total <= 0) return;
  const float* ap[NA];
  const float* am[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    ap[q] = abase[q] + pa * pitch + 16 * ua;
    am[q] = abase[q] - pa * pitch + 16 * ua;
  }
  const float* bp = bbase + pa * E + 16 * ua;
  StepWalk w(nu, pitch, E);
  f32x4 ac_[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) ac_[q] = acc[q];
  auto load = [&](f32x4v (&a0)[NA], f32x4v (&a1)[NA], float (&bb)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) bb[e] = bp[e];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      if (MODE != 2) a0[q] = *reinterpret_cast<const f32x4v*>(ap[q]);
      if (MODE != 1) a1[q] = *reinterpret_cast<const f32x4v*>(am[q]);
    }
    int ia, im, ib;
    w.next(ia, im, ib);
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      ap[q] += ia;
      am[q] += im;
    }
    bp += ib;
  };
  auto compute = [&](const f32x4v (&a0)[NA], const f32x4v (&a1)[NA], const float (&bb)[4]) {
    f32x4v ac[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) ac[q] = MODE == 0 ? a0[q] + a1[q] : (MODE == 1 ? a0[q] : a1[q]);
    // the step's adds before its matrix instructions: an add between two of them
    // costs more issue time than the adds grouped
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int q = 0; q < NA; ++q) ac_[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[q][e], bb[e], ac_[q], 0, 0, 0);
  };
  f32x4v x0[NA], x1[NA], y0[NA], y1[NA];
  float bx[4], by[4];
  load(x0, x1, bx);  // step 0
  int st = 0;
  for (; st + 2 < total; st += 2) {
    load(y0, y1, by);  // step st + 1
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the matrix work they overlap
    compute(x0, x1, bx);
    load(x0, x1, bx);  // step st + 2
    __builtin_amdgcn_sched_barrier(0);
    compute(y0, y1, by);
  }
  if (st + 1 < total) {  // steps st and st + 1 remain
    load(y0, y1, by);
    __builtin_amdgcn_sched_barrier(0);
    compute(x0, x1, bx);
    compute(y0, y1, by);
  } else {
    compute(x0, x1, bx);
  }
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = ac_[q];
}

// The same sums (tap rows p in [pa, pb], all SS super-steps, both folded rows) for
// a super-step count fixed at compile time: a tap row's steps are unrolled, so
// their LDS addresses are immediate offsets of three pointers that move once per
// row.  Two rows form one loop trip (with SS odd the second row's steps use the
// operand sets in the other order); the operands of each step are loaded one
// step ahead, across row ends as well; the order of every sum is that of
// f32_steps.
template <int NA, int SS>
__device__ __forceinline__ void f32_rows(const float* const* abase, const float* bbase, int pitch, int E, int pa,
                                         int pb, f32x4* acc) {
  if (pb < pa) return;
  const float* ap[NA];
  const float* am[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    ap[q] = abase[q] + pa * pitch;
    am[q] = abase[q] - pa * pitch;
  }
  const float* bp = bbase + pa * E;
  f32x4 ac_[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) ac_[q] = acc[q];
  f32x4v A0[2][NA], A1[2][NA];
  float B[2][4];
  auto load = [&](int set, int u) {
#pragma unroll
    for (int e = 0; e < 4; ++e) B[set][e] = bp[16 * u + e];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      A0[set][q] = *reinterpret_cast<const f32x4v*>(ap[q] + 16 * u);
      A1[set][q] = *reinterpret_cast<const f32x4v*>(am[q] + 16 * u);
    }
  };
  auto advance = [&](bool more) {  // to the next row, or (after the last) stay
    const int da = more ? pitch : 0, db = more ? E : 0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      ap[q] += da;
      am[q] -= da;
    }
    bp += db;
  };
  auto compute = [&](int set) {
    f32x4v ac[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) ac[q] = A0[set][q] + A1[set][q];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int q = 0; q < NA; ++q)
        ac_[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[q][e], B[set][e], ac_[q], 0, 0, 0);
    // the step's adds ahead of its matrix instructions, all together
    __builtin_amdgcn_sched_group_barrier(0x002, 4 * NA, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 4 * NA, 0);
  };
  // one row whose step u uses set (S0 + u) & 1; returns false after the last row
  auto row = [&](auto s0, int p) {
    constexpr int S0 = decltype(s0)::value;
#pragma unroll
    for (int u = 0; u < SS; ++u) {
      const int cur = (S0 + u) & 1, nxt = (S0 + u + 1) & 1;
      if (u + 1 < SS) {
        load(nxt, u + 1);
      } else {
        // the next row's first step (after the last row, the last row's again:
        // unconditional, so that each step waits for its own operands only)
        advance(p < pb);
        load(nxt, 0);
      }
      __builtin_amdgcn_sched_barrier(0);  // the loads ahead of the matrix work they overlap
      compute(cur);
    }
    return p < pb;
  };
  load(0, 0);
  for (int p = pa;; p += 2) {
    if (!row(std::integral_constant<int, 0>{}, p)) break;
    if (!row(std::integral_constant<int, SS & 1>{}, p + 1)) break;
  }
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = ac_[q];
}

// The same loop for two horizontally adjacent tiles whose column windows start at
// the same input column: they share the A operand (the same input rows and
// columns) and each multiplies it by its own Toeplitz operand, the right tile's
// starting 16 entries earlier in the extended tap row.  Four LDS reads feed eight
// matrix instructions instead of six; each tile's sum keeps the order of f32_steps.
template <int MODE>
__device__ __forceinline__ void f32_steps_hpair(const float* abase, const float* bbase0, const float* bbase1,
                                                int pitch, int E, int pa, int pb, int ua, int ub, f32x4& acc0,
                                                f32x4& acc1) {
  const int nu = ub - ua + 1;
  const int total = (pb >= pa && nu > 0) ? (pb - pa + 1) * nu : 0;
  if (total <= 0) return;
  f32x4 c0 = acc0, c1 = acc1;
  const float* ap = abase + pa * pitch + 16 * ua;
  const float* am = abase - pa * pitch + 16 * ua;
  const float* bp0 = bbase0 + pa * E + 16 * ua;
  const float* bp1 = bbase1 + pa * E + 16 * ua;
  StepWalk w(nu, pitch, E);
  auto load = [&](f32x4v& a0, f32x4v& a1, float (&b0)[4], float (&b1)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      b0[e] = bp0[e];
      b1[e] = bp1[e];
    }
    if (MODE != 2) a0 = *reinterpret_cast<const f32x4v*>(ap);
    if (MODE != 1) a1 = *reinterpret_cast<const f32x4v*>(am);
    int ia, im, ib;
    w.next(ia, im, ib);
    ap += ia;
    am += im;
    bp0 += ib;
    bp1 += ib;
  };
  auto compute = [&](const f32x4v& a0, const f32x4v& a1, const float (&b0)[4], const float (&b1)[4]) {
    const f32x4v a = MODE == 0 ? a0 + a1 : (MODE == 1 ? a0 : a1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b0[e], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b1[e], c1, 0, 0, 0);
    }
  };
  f32x4v x0, x1, y0, y1;
  float bx0[4], bx1[4], by0[4], by1[4];
  load(x0, x1, bx0, bx1);
  int st = 0;
  for (; st + 2 < total; st += 2) {
    load(y0, y1, by0, by1);  // step st + 1
    __builtin_amdgcn_sched_barrier(0);
    compute(x0, x1, bx0, bx1);
    load(x0, x1, bx0, bx1);  // step st + 2
    __builtin_amdgcn_sched_barrier(0);
    compute(y0, y1, by0, by1);
  }
  if (st + 1 < total) {
    load(y0, y1, by0, by1);
    __builtin_amdgcn_sched_barrier(0);
    compute(x0, x1, bx0, bx1);
    compute(y0, y1, by0, by1);
  } else {
    compute(x0, x1, bx0, bx1);
  }
  acc0 = c0;
  acc1 = c1;
}

// The part of a plane's data rectangle that lies inside the box [u0, u1) x [v0, v1).
__device__ __forceinline__ DataRect clip_rect(const DataRect& d, int4 bx) {
  DataRect c;
  const int r0 = max(d.r0, bx.x), r1 = min(d.r0 + d.nr, bx.y);
  const int c0 = max(d.c0, bx.z), c1 = min(d.c0 + d.nc, bx.w);
  c.r0 = r0;
  c.c0 = c0;
  c.nr = r1 > r0 && c1 > c0 ? r1 - r0 : 0;
  c.nc = r1 > r0 && c1 > c0 ? c1 - c0 : 1;
  c.lr0 = d.lr0 + (r0 - d.r0);
  c.lc0 = d.lc0 + (c0 - d.c0);
  return c;
}

__device__ __forceinline__ int floor_div16(int a) { return a >= 0 ? a / 16 : -((15 - a) / 16); }

// CONV_IN_BOX: the offset (gi, gj), each in [gmin, 0], of a region's tile grid that
// minimises its matrix steps for the box [u0, u1) x [v0, v1).  Only a region whose
// tiles reach past the plane has slack (the plane's last region along each
// axis): its grid may start up to 15 rows or columns early, the rows and columns
// before the region's first one being left to the previous region or lying
// outside the plane.  The step count is separable, (sum over tile rows of the tap
// rows in reach) x (sum over tile columns of the super-steps in reach), so each
// offset is chosen alone: lanes 0-15 try the row offsets 0, -1, ..., -15 and lanes
// 16-31 the column offsets; ties go to the offset nearest 0.
__device__ __forceinline__ int2 grid_offsets(const Geo<float>& g, const RegionShape& rs, int I0, int J0, int SS,
                                             int4 bx, int lane) {
  const int h = g.h;
  const bool col = lane >= 16;
  const int cand = lane & 15;
  const int N = col ? g.Nv : g.Nu, X0 = col ? J0 : I0, T = col ? rs.TJ : rs.TI;
  const int lo = max(col ? bx.z : bx.x, 0), hi = min(col ? bx.w : bx.y, N);
  const int gmin = max(-15, min(0, (N - X0) - MT * T));
  const int end = min(N, X0 + MT * T);
  int key = 0x7fffffff;
  if (lane < 32 && -cand >= gmin) {
    int cost = 0;
    for (int t = 0; t < RMAX; ++t) {
      const int X = X0 - cand + MT * t;
      if (t >= T || X >= end || hi <= lo) continue;
      if (col) {
        const int cb = X - h, ca = max(cb, lo), cz = min(cb + 16 * SS - 1, hi - 1);
        if (cz >= ca) {
          const int o = ((ca - cb) >> 2) << 2;
          cost += (cz - cb - o + 16) >> 4;
        }
      } else {
        const int a1 = max(0, lo - X - 15), b1 = min(h, hi - X - 1);
        const int a2 = max(0, X - hi + 1), b2 = min(h, X + 15 - lo);
        const int n1 = a1 <= b1 ? b1 - a1 + 1 : 0, n2 = a2 <= b2 ? b2 - a2 + 1 : 0;
        const int ov = n1 > 0 && n2 > 0 ? max(0, min(b1, b2) - max(a1, a2) + 1) : 0;
        cost += n1 + n2 - ov;
      }
    }
    key = (cost << 4) | cand;
  }
#pragma unroll
  for (int sh = 8; sh >= 1; sh >>= 1) key = min(key, __shfl_xor(key, sh));
  return int2{-(__builtin_amdgcn_readlane(key, 0) & 15), -(__builtin_amdgcn_readlane(key, 16) & 15)};
}

// The extended, folded tap rows of the FP32 kernels: kx[p][c] = K[p][|c - off|]
// where |c - off| <= h (halved for p = 0, whose row the fold counts twice), zero
// elsewhere.  Wavefronts walk the tap rows, lanes the columns.
__device__ __forceinline__ void build_kx(const float* kq, float* kx, int h, int E, int off, int wave, int lane,
                                         int nw) {
  for (int p = wave; p <= h; p += nw) {
    const float sc = p == 0 ? 0.5f : 1.f;
    for (int c = lane; c < E; c += 64) {
      const int q = c - off;
      float v = 0.f;
      if (q >= -h && q <= h) v = kq[p * (h + 1) + (q < 0 ? -q : q)] * sc;
      kx[p * E + c] = v;
    }
  }
}

// Support of the convolution (box: per control point [u0, u1) x [v0, v1), the
// aperture's rectangle outside which the fluence and its derivatives vanish):
//   CONV_DENSE    every input and output;
//   CONV_IN_BOX   the input is zero outside the box (forward: P = F G): only the
//                 box is staged, and each wavefront skips the tap rows and column
//                 super-steps whose inputs all lie outside it (exact zeros);
//   CONV_OUT_BOX  only outputs in the box are needed (adjoint: the parameter
//                 gradients read A only there): the region's tiles that meet the
//                 box are spread over the wavefronts, every other output is 0.
// The matrix arithmetic of every computed output is that of the dense kernel.

// Items it = blockIdx.x, blockIdx.x + gridDim.x, ... with region = it % regions
// and (control point, plane) = it / regions; gridDim.x is a multiple of the
// region count, so a workgroup keeps one region.
template <int NW, int TPW, int SUP>
__global__ void __launch_bounds__(64 * NW) k_conv_mfma_f32(Geo<float> g, RegionShape rs, F32Shape fs, int n_items,
                                                           const int4* __restrict__ box,
                                                           const float* __restrict__ zca,
                                                           const float* __restrict__ in, float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int NT = 64 * NW;
  const int h = g.h;
  const int rows = fs.rows, pitch = fs.pitch, E = fs.E, SS = fs.SS;
  float* tile = lds;
  float* kx = lds + rows * pitch;  // (h + 1) x E, zero outside |q| <= h, row 0 halved
  float* kq = kx + (h + 1) * E;    // (h + 1) x (h + 1) unique taps
  int* grab = reinterpret_cast<int*>(kq + (h + 1) * (h + 1));  // next tile to take (CONV_IN_BOX)
  // CONV_IN_BOX: per tile {a1, b1, a2, b2, column offset o, super-steps nu, steps, pair role}
  int* trange = grab + 4;
  int* order = trange + 8 * RMAX * RMAX;  // CONV_IN_BOX: tiles by decreasing step count
  const int nreg = rs.regions_i * rs.regions_j;
  const int region = blockIdx.x % nreg;
  const int I0 = (region / rs.regions_j) * rs.TI * MT;
  const int J0 = (region % rs.regions_j) * rs.TJ * MT;
  const size_t plane = (size_t)g.Nu * g.Nv;
  const int tid = threadIdx.x;
  const DataRect dr = data_rect(g, I0, J0, MT * rs.TI, MT * rs.TJ);
  const int n_tiles = rs.TI * rs.TJ;

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kk = lane >> 4;
  // this wavefront's fixed tiles t = wave + NW q (all of them stored every item)
  int tI[TPW], tJ[TPW];
  bool active[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = wave + NW * q;
    bool valid = t < rs.TI * rs.TJ;
    tI[q] = valid ? t / rs.TJ : 0;
    tJ[q] = valid ? t - (t / rs.TJ) * rs.TJ : 0;
    active[q] = valid && I0 + MT * tI[q] < g.Nu && J0 + MT * tJ[q] < g.Nv;
  }
  const float* bbase = kx + 4 * kk + 15 - m;
  const int off = h + 15;
  auto a_of = [&](int ti, int tj) { return tile + (MT * ti + m + h) * pitch + MT * tj + 4 * kk; };
  // with CONV_IN_BOX, an item's tile-grid offset (a whole wavefront's call) and its
  // data rectangle for a given offset
  auto offsets_of = [&](int item) {
    if (SUP == CONV_IN_BOX) return grid_offsets(g, rs, I0, J0, SS, box[(item / nreg) / g.Nk], lane);
    return int2{0, 0};
  };
  // (CONV_IN_BOX: the image sits at the rectangle, see f32_shape_in_box; an image
  // origin is always r0 - lr0, c0 - lc0 of the item's rectangle)
  auto rect_at = [&](int item, int2 go) {
    if (SUP == CONV_IN_BOX) {
      DataRect c = clip_rect(data_rect(g, I0 + go.x, J0 + go.y, MT * rs.TI, MT * rs.TJ), box[(item / nreg) / g.Nk]);
      const int Ilo = I0 + go.x - h, Clo = J0 + go.y - h;
      const int R0 = max(Ilo, c.r0 - 15);
      const int C0 = Clo + ((max(0, c.c0 - 18 - Clo) >> 2) << 2);
      c.lr0 = c.r0 - R0;
      c.lc0 = c.c0 - C0;
      return c;
    }
    return dr;
  };

  zero_lds(tile, rows * pitch, tid, NT);
  float buf[PF];
  int it = blockIdx.x;
  int2 cur_go = offsets_of(it < n_items ? it : 0), nxt_go;
  DataRect cur = rect_at(it < n_items ? it : 0, cur_go);
  DataRect prev = cur;
  prev.nr = 0;
  prev.nc = 1;
  if (it < n_items) fetch_rect<PF>(in + (size_t)(it / nreg) * plane, g.Nv, cur, tid, NT, buf);
  __syncthreads();
  for (; it < n_items; it += gridDim.x) {
    const int bk = it / nreg;  // b * Nk + k
    const int k = bk % g.Nk;
    const float* src = in + (size_t)bk * plane;
    put_rect<PF>(src, g.Nv, cur, pitch, tid, NT, buf, tile);
    if (SUP == CONV_IN_BOX) {
      if (tid == 0) *grab = 0;
      // the next item's grid offset, searched by one wavefront and read by all
      // after the barriers below
      if (wave == 0 && it + (int)gridDim.x < n_items) {
        const int2 go = offsets_of(it + gridDim.x);
        if (lane == 0) {
          grab[1] = go.x;
          grab[2] = go.y;
        }
      }
      if (tid < n_tiles) {
        // the steps of tile tid that meet the input rectangle: tap rows p whose row
        // I + p .. I + p + 15 (plus side, p in [a1, b1]) or I - p .. I - p + 15 (minus
        // side, p in [a2, b2]) meets [r0, r1), and nu super-steps of 16 input columns
        // starting at column J - h + o (o a multiple of 4, so the 16-byte reads stay
        // aligned) that cover the rectangle's columns in reach
        const int ti = tid / rs.TJ, tj = tid - (tid / rs.TJ) * rs.TJ;
        const int I = I0 + cur_go.x + MT * ti, J = J0 + cur_go.y + MT * tj;
        const int r0 = cur.r0, r1 = cur.r0 + cur.nr;
        const int a1 = max(0, r0 - I - 15), b1 = min(h, r1 - I - 1);
        const int a2 = max(0, I - r1 + 1), b2 = min(h, I + 15 - r0);
        const int cb = J - h;
        const int ca = max(cb, cur.c0), cz = min(cb + 16 * SS - 1, cur.c0 + cur.nc - 1);
        int o = 0, nu = 0;
        if (cur.nr > 0 && cz >= ca && I < g.Nu && J < g.Nv) {
          o = ((ca - cb) >> 2) << 2;
          nu = (cz - cb - o + 16) >> 4;
          o = min(o, 16 * (SS - nu));
        }
        // tap rows in the union of the two intervals
        const int n1 = a1 <= b1 ? b1 - a1 + 1 : 0, n2 = a2 <= b2 ? b2 - a2 + 1 : 0;
        const int lo = max(a1, a2), hi_ = min(b1, b2), both = n1 > 0 && n2 > 0 && lo <= hi_ ? hi_ - lo + 1 : 0;
        int* tr = trange + 8 * tid;
        tr[0] = a1;
        tr[1] = nu > 0 ? b1 : a1 - 1;
        tr[2] = a2;
        tr[3] = nu > 0 ? b2 : a2 - 1;
        tr[4] = o;
        tr[5] = nu;
        tr[6] = (n1 + n2 - both) * nu;
        // Horizontal pairs: scanning a tile row from the left, tiles j and j + 1 form
        // a pair when their column windows start at the same input column with the
        // same super-step count (the window depends on the tile column only, so
        // every row pairs alike).  Role: 1 left tile of a pair, -1 right tile, 0 alone.
        auto window = [&](int Jc, int& wo, int& wn) {
          const int wb = Jc - h;
          const int wa = max(wb, cur.c0), wz = min(wb + 16 * SS - 1, cur.c0 + cur.nc - 1);
          wo = 0;
          wn = 0;
          if (cur.nr > 0 && wz >= wa && Jc < g.Nv) {
            wo = ((wa - wb) >> 2) << 2;
            wn = (wz - wb - wo + 16) >> 4;
            wo = min(wo, 16 * (SS - wn));
          }
        };
        int role = 0;
        for (int jj = 0; jj < rs.TJ;) {
          int oa, na, ob = 0, nb_ = 0;
          window(J0 + cur_go.y + MT * jj, oa, na);
          if (jj + 1 < rs.TJ) window(J0 + cur_go.y + MT * (jj + 1), ob, nb_);
          if (jj + 1 < rs.TJ && na > 0 && nb_ == na && ob == oa - 16) {
            role = jj == tj ? 1 : (jj + 1 == tj ? -1 : role);
            jj += 2;
          } else {
            jj += 1;
          }
        }
        tr[7] = role;
      }
      // clear what the previous item wrote outside this item's rectangle
      for (RectWalk w(tid, NT, prev.nc); w.r < prev.nr; w.next(prev.nc)) {
        const int lr = prev.lr0 + w.r, lc = prev.lc0 + w.c;
        const bool in_cur = lr >= cur.lr0 && lr < cur.lr0 + cur.nr && lc >= cur.lc0 && lc < cur.lc0 + cur.nc;
        if (!in_cur) tile[lr * pitch + lc] = 0.f;
      }
    }
    unique_taps(g, k, zca[bk], kq, tid, NT);
    __syncthreads();
    if (SUP == CONV_IN_BOX && tid < n_tiles) {
      // the units (single tiles and left tiles of pairs) ranked by matrix
      // instructions, largest first (ties by index), so the last units taken are short
      auto work = [&](int t) { return trange[8 * t + 6] * (trange[8 * t + 7] == 1 ? 2 : 1); };
      const int w = work(tid);
      int rank = 0, units = 0;
      for (int t = 0; t < n_tiles; ++t) {
        if (trange[8 * t + 7] < 0) continue;
        const int v = work(t);
        rank += (v > w || (v == w && t < tid)) ? 1 : 0;
        ++units;
      }
      if (trange[8 * tid + 7] >= 0) order[rank] = tid;
      if (tid == 0) grab[3] = units;
    }
    build_kx(kq, kx, h, E, off, wave, lane, NW);
    __syncthreads();
    // next item's input, in flight while this item's matrix work runs
    const int nx = it + gridDim.x;
    DataRect nxt = cur;
    nxt_go = cur_go;
    if (nx < n_items) {
      if (SUP == CONV_IN_BOX) nxt_go = int2{__builtin_amdgcn_readfirstlane(grab[1]), __builtin_amdgcn_readfirstlane(grab[2])};
      nxt = rect_at(nx, nxt_go);
      fetch_rect<PF>(in + (size_t)(nx / nreg) * plane, g.Nv, nxt, tid, NT, buf);
    }
    float* dst = out + (size_t)bk * plane;

    if (SUP == CONV_IN_BOX) {
      // Tiles are taken one at a time from a shared counter, longest first, each with
      // only the tap rows and super-steps that reach the input rectangle, so
      // wavefronts whose tiles need little work take more tiles.  Every tile is
      // computed by one wavefront in a fixed step order.
      const int n_units = __builtin_amdgcn_readfirstlane(grab[3]);
      while (true) {
        int t = 0;
        if (lane == 0) t = atomicAdd(grab, 1);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= n_units) break;
        t = __builtin_amdgcn_readfirstlane(order[t]);
        const int ti = t / rs.TJ, tj = t - (t / rs.TJ) * rs.TJ;
        const int I = I0 + cur_go.x + MT * ti, J = J0 + cur_go.y + MT * tj;
        if (I >= g.Nu || J >= g.Nv) continue;
        const int* tr = trange + 8 * t;
        const int a1 = __builtin_amdgcn_readfirstlane(tr[0]), b1 = __builtin_amdgcn_readfirstlane(tr[1]);
        const int a2 = __builtin_amdgcn_readfirstlane(tr[2]), b2 = __builtin_amdgcn_readfirstlane(tr[3]);
        const int o = __builtin_amdgcn_readfirstlane(tr[4]), nu = __builtin_amdgcn_readfirstlane(tr[5]);
        const int R0 = cur.r0 - cur.lr0, C0 = cur.c0 - cur.lc0;
        const float* ab[1] = {tile + (I + m - R0) * pitch + (J - h - C0) + 4 * kk + o};
        const float* bb = bbase + o;
        f32x4 acc[1] = {f32x4{0.f, 0.f, 0.f, 0.f}};
        if (__builtin_amdgcn_readfirstlane(tr[7]) == 1) {
          // a pair: this tile and the one to its right (same tap rows, the same input
          // window, whose offset in the right tile's frame is o - 16)
          f32x4 acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
          int p = min(a1 <= b1 ? a1 : h + 1, a2 <= b2 ? a2 : h + 1);
          const int p_top = max(a1 <= b1 ? b1 : -1, a2 <= b2 ? b2 : -1);
          while (p <= p_top) {
            const bool plus = a1 <= p && p <= b1, minus = a2 <= p && p <= b2;
            int e = p_top;
            if (plus) e = min(e, b1);
            else if (a1 > p && a1 <= b1) e = min(e, a1 - 1);
            if (minus) e = min(e, b2);
            else if (a2 > p && a2 <= b2) e = min(e, a2 - 1);
            if (plus && minus) f32_steps_hpair<0>(ab[0], bb, bb - 16, pitch, E, p, e, 0, nu - 1, acc[0], acc1);
            else if (plus) f32_steps_hpair<1>(ab[0], bb, bb - 16, pitch, E, p, e, 0, nu - 1, acc[0], acc1);
            else if (minus) f32_steps_hpair<2>(ab[0], bb, bb - 16, pitch, E, p, e, 0, nu - 1, acc[0], acc1);
            p = e + 1;
          }
          store_tile_from(g, I, J, I0, J0, lane, acc[0], dst);
          store_tile_from(g, I, J + MT, I0, J0, lane, acc1, dst);
          continue;
        }
        // segments of p in increasing order, each loading only the fold sides it
        // needs (the image holds only the rows these clipped ranges reach)
        int p = min(a1 <= b1 ? a1 : h + 1, a2 <= b2 ? a2 : h + 1);
        const int p_top = max(a1 <= b1 ? b1 : -1, a2 <= b2 ? b2 : -1);
        while (p <= p_top) {
          const bool plus = a1 <= p && p <= b1, minus = a2 <= p && p <= b2;
          int e = p_top;  // the segment ends before the next interval boundary
          if (plus) e = min(e, b1);
          else if (a1 > p && a1 <= b1) e = min(e, a1 - 1);
          if (minus) e = min(e, b2);
          else if (a2 > p && a2 <= b2) e = min(e, a2 - 1);
          if (plus && minus) f32_steps<1, 0>(ab, bb, pitch, E, p, e, 0, nu - 1, acc);
          else if (plus) f32_steps<1, 1>(ab, bb, pitch, E, p, e, 0, nu - 1, acc);
          else if (minus) f32_steps<1, 2>(ab, bb, pitch, E, p, e, 0, nu - 1, acc);
          p = e + 1;
        }
        store_tile_from(g, I, J, I0, J0, lane, acc[0], dst);
      }
    } else {
      const float* ab[TPW];
#pragma unroll
      for (int q = 0; q < TPW; ++q) ab[q] = a_of(tI[q], tJ[q]);
      f32x4 acc[TPW];
#pragma unroll
      for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
      f32_steps<TPW>(ab, bbase, pitch, E, 0, h, 0, SS - 1, acc);
#pragma unroll
      for (int q = 0; q < TPW; ++q)
        if (active[q]) store_tile_at(g, I0 + MT * tI[q], J0 + MT * tJ[q], lane, acc[q], dst);
    }
    prev = cur;
    cur = nxt;
    cur_go = nxt_go;
    __syncthreads();  // the LDS image and taps are rewritten for the next item
  }
}

// The adjoint direction (CONV_OUT_BOX): only the outputs inside the box are
// needed.  Per item the box (clipped to the region) is covered by nI x nJ output
// tiles placed at the box corner (columns rounded down to a multiple of 4, so the
// 16-byte LDS reads stay aligned) instead of on the region's tile grid, and the
// work is split over the wavefronts by tile and by a range of tap rows: with nT
// tiles each tile's rows p = 0..h are cut into C = NW / nT chunks, whose partial
// sums are added in LDS in chunk order.  Outputs outside the covered rectangle are
// not written: the adjoint ray march reads this volume only inside the box.
template <int NW, int TPW>
__global__ void __launch_bounds__(64 * NW) k_conv_mfma_f32_adj(Geo<float> g, RegionShape rs, F32Shape fs,
                                                               int n_items, const int4* __restrict__ box,
                                                               const float* __restrict__ zca,
                                                               const float* __restrict__ in,
                                                               float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int NT = 64 * NW;
  const int h = g.h;
  const int rows = fs.rows, pitch = fs.pitch, E = fs.E, SS = fs.SS;
  float* tile = lds;
  float* kx = lds + rows * pitch;
  float* kq = kx + (h + 1) * E;
  // (NW - 1) x 256 partial sums, 16-byte aligned (see f32_adj_lds); an offset from
  // the base, so that the accesses stay LDS accesses
  float* part = lds + ((rows * pitch + (h + 1) * E + (h + 1) * (h + 1) + 3) & ~3);
  const int nreg = rs.regions_i * rs.regions_j;
  const size_t plane = (size_t)g.Nu * g.Nv;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kk = lane >> 4;
  const float* bbase = kx + 4 * kk + 15 - m;
  const int off = h + 15;

  // Item it is (control point, plane) it / nreg in region it % nreg.  The grid is
  // not a multiple of the region count, so a workgroup's items move over the
  // regions (a plane wider than one region, e.g. the square grid of a rotated
  // collimator, has its boxes in few regions: pinning workgroups to regions would
  // idle the others).  The image is cleared again when the region changes.  An item
  // whose box misses its region's outputs has nothing to compute or write and is
  // skipped without staging.
  struct Reg {
    int region, I0, J0, Ie, Je;  // first output row / column; outputs in the plane end at Ie, Je
    DataRect dr;
  };
  auto reg_of = [&](int item) {
    Reg r;
    r.region = item % nreg;
    r.I0 = (r.region / rs.regions_j) * rs.TI * MT;
    r.J0 = (r.region % rs.regions_j) * rs.TJ * MT;
    r.Ie = min(g.Nu, r.I0 + MT * rs.TI);
    r.Je = min(g.Nv, r.J0 + MT * rs.TJ);
    r.dr = data_rect(g, r.I0, r.J0, MT * rs.TI, MT * rs.TJ);
    return r;
  };
  auto live = [&](int item, const Reg& r) {
    const int4 b4 = box[(item / nreg) / g.Nk];
    return max(b4.x, r.I0) < min(b4.y, r.Ie) && max(b4.z, r.J0) < min(b4.w, r.Je);
  };
  zero_lds(tile, rows * pitch, tid, NT);
  float buf[PF];
  int it = blockIdx.x;
  int held = -1;  // the region whose data (and zero halo) the image holds
  if (it < n_items) {
    const Reg r = reg_of(it);
    if (live(it, r)) fetch_rect<PF>(in + (size_t)(it / nreg) * plane, g.Nv, r.dr, tid, NT, buf);
  }
  __syncthreads();
  for (; it < n_items; it += gridDim.x) {
    const int bk = it / nreg;
    const int k = bk % g.Nk;
    const float* src = in + (size_t)bk * plane;
    const Reg r = reg_of(it);
    const int I0 = r.I0, J0 = r.J0, Ie = r.Ie, Je = r.Je;
    const int nx = it + gridDim.x;
    const Reg rn = reg_of(nx);
    const bool next_live = nx < n_items && live(nx, rn);
    if (!live(it, r)) {  // uniform over the workgroup; the LDS is not touched
      if (next_live) fetch_rect<PF>(in + (size_t)(nx / nreg) * plane, g.Nv, rn.dr, tid, NT, buf);
      continue;
    }
    if (held >= 0 && held != r.region) {
      zero_lds(tile, rows * pitch, tid, NT);
      __syncthreads();
    }
    held = r.region;
    put_rect<PF>(src, g.Nv, r.dr, pitch, tid, NT, buf, tile);
    unique_taps(g, k, zca[bk], kq, tid, NT);
    __syncthreads();
    build_kx(kq, kx, h, E, off, wave, lane, NW);
    __syncthreads();
    if (next_live) fetch_rect<PF>(in + (size_t)(nx / nreg) * plane, g.Nv, rn.dr, tid, NT, buf);
    float* dst = out + (size_t)bk * plane;

    // the covered rectangle [Iw, Iw + 16 nI) x [Jw, Jw + 16 nJ)
    const int4 bx = box[bk / g.Nk];
    const int u0 = max(bx.x, I0), u1 = min(bx.y, Ie), v0 = max(bx.z, J0), v1 = min(bx.w, Je);
    int nI = 0, nJ = 0, Iw = I0, Jw = J0;
    if (u1 > u0 && v1 > v0) {
      nI = (u1 - u0 + MT - 1) / MT;
      Iw = min(u0, I0 + MT * rs.TI - MT * nI);
      const int ja = v0 - ((v0 - J0) & 3);
      nJ = (v1 - ja + MT - 1) / MT;
      Jw = min(ja, J0 + MT * rs.TJ - MT * nJ);
    }
    const int nT = nI * nJ;
    const int C = nT > 0 && nT < NW ? NW / nT : 1;  // tap-row chunks per tile
    const int chunk = wave % C, slot = wave / C, slots = NW / C;
    const int h1 = h + 1, pa = (h1 * chunk) / C, pb = (h1 * (chunk + 1)) / C - 1;
    int nact = 0;
    const float* ab[TPW];
    int oI[TPW], oJ[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = slot + slots * q;
      const bool use = t < nT;
      const int ti = use ? t / nJ : 0, tj = use ? t - (t / nJ) * nJ : 0;
      oI[q] = Iw + MT * ti;
      oJ[q] = Jw + MT * tj;
      ab[q] = tile + (oI[q] - I0 + m + h) * pitch + (oJ[q] - J0) + 4 * kk;
      nact += use ? 1 : 0;
    }
    f32x4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (nact == 1) f32_steps<1>(ab, bbase, pitch, E, pa, pb, 0, SS - 1, acc);
    if (TPW >= 2 && nact == 2) f32_steps<TPW >= 2 ? 2 : 1>(ab, bbase, pitch, E, pa, pb, 0, SS - 1, acc);
    if (TPW >= 3 && nact == 3) f32_steps<TPW >= 3 ? 3 : 1>(ab, bbase, pitch, E, pa, pb, 0, SS - 1, acc);
    if (C > 1) {
      // (C > 1 only with one tile per wavefront) chunks 1 .. C-1 park their sums, chunk 0 adds them in order
      __syncthreads();
      if (chunk > 0 && nact > 0)
        *reinterpret_cast<f32x4*>(part + ((slot * (C - 1) + chunk - 1) * 64 + lane) * 4) = acc[0];
      __syncthreads();
      if (chunk == 0 && nact > 0) {
        for (int c = 1; c < C; ++c) acc[0] += *reinterpret_cast<const f32x4*>(part + ((slot * (C - 1) + c - 1) * 64 + lane) * 4);
        store_tile_at(g, oI[0], oJ[0], lane, acc[0], dst);
      }
    } else {
#pragma unroll
      for (int q = 0; q < TPW; ++q)
        if (q < nact) store_tile_at(g, oI[q], oJ[q], lane, acc[q], dst);
    }
    __syncthreads();
  }
}


// One wavefront's partial sums into the LDS, as a call of its own: with the store
// inlined into the adjoint kernel below, the compiler's wait insertion makes the
// first matrix step of every loop iteration wait for all LDS loads in flight (the
// next step's included) instead of its own operands only.
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;
__device__ __attribute__((noinline)) void park_partial(lds_f32x4* p, f32x4 v) { *p = v; }

// The adjoint (CONV_OUT_BOX) with an image of its output tiles' read window only.
// Per item the box (clipped to the plane) is covered by nI x nJ output tiles at its
// corner; they are taken in pieces of at most WI x WJ tiles, and each piece's
// image holds rows [Ip - h, Ip + 16 nIp + h) and columns [Jp - h, Jp - h + 16 (nJp -
// 1) + 16 SS) of the plane (zero outside it), which is all its tiles read, so the
// image is a small fraction of a whole-plane one and two workgroups share a CU
// (one's setup, staging and barriers under the other's matrix loop).  The tap rows,
// the split of a tile's tap rows over wavefronts and the order of every sum are
// those of the tiled kernel; outputs outside the covered rectangle are not written
// (the adjoint ray march reads this volume only inside the box).
struct AdjWin {
  int WI, WJ;        // piece size in output tiles
  int rows, pitch;   // image rows (16 WI + 2h) and row pitch
  int E, SS;         // extended tap row length and column super-steps of a tile
};

// Column groups per thread prefetched by the windowed adjoint: the whole window of
// a piece of 2 x 2 tiles with 61 taps (92 rows of 24 groups, 21 rows a pass over
// 512 threads), so no group is loaded after the matrix loop that hides the latency.
constexpr int PGW = 5;

template <int NW, int TPW, int SSC>
__global__ void __launch_bounds__(64 * NW) k_conv_f32_adj_win(Geo<float> g, AdjWin aw, int n_items,
                                                              const int4* __restrict__ box,
                                                              const float* __restrict__ zca,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int NT = 64 * NW;
  const int h = g.h;
  const int pitch = aw.pitch, E = aw.E, SS = aw.SS;
  float* tile = lds;
  float* kx = lds + aw.rows * pitch;
  // (NW - 1) x 256 partial sums, 16-byte aligned; an offset from the base, so that
  // the accesses stay LDS accesses
  float* part = lds + ((aw.rows * pitch + (h + 1) * E + 3) & ~3);
  const size_t plane = (size_t)g.Nu * g.Nv;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = lane & 15, kk = lane >> 4;
  const float* bbase = kx + 4 * kk + 15 - m;
  const int off = h + 15;
  // the tap rows' entries farther than h from `off` stay zero; the taps of each item
  // overwrite the others
  zero_lds(kx, (h + 1) * E, tid, NT);
  __syncthreads();

  // the covered tiles of an item (nI = 0: nothing to compute) and a piece's window
  struct Cov {
    int Iw, Jw, nI, nJ, npi, npj;
  };
  auto cov_of = [&](int item) {
    Cov c;
    const int4 bx = box[item / g.Nk];
    const int u0 = max(bx.x, 0), u1 = min(bx.y, g.Nu), v0 = max(bx.z, 0), v1 = min(bx.w, g.Nv);
    c.Iw = u0;
    c.Jw = v0;
    c.nI = u1 > u0 && v1 > v0 ? (u1 - u0 + MT - 1) / MT : 0;
    c.nJ = u1 > u0 && v1 > v0 ? (v1 - v0 + MT - 1) / MT : 0;
    c.npi = (c.nI + aw.WI - 1) / aw.WI;
    c.npj = (c.nJ + aw.WJ - 1) / aw.WJ;
    return c;
  };
  auto win_of = [&](const Cov& c, int pp, int* nIp, int* nJp) {
    const int pi = pp / c.npj, pj = pp - (pp / c.npj) * c.npj;
    *nIp = min(aw.WI, c.nI - aw.WI * pi);
    *nJp = min(aw.WJ, c.nJ - aw.WJ * pj);
    WinRect w;
    w.r0 = c.Iw + MT * aw.WI * pi - h;
    w.c0 = c.Jw + MT * aw.WJ * pj - h;
    w.nr = MT * *nIp + 2 * h;
    w.nc = MT * (*nJp - 1) + 16 * SS;
    return w;
  };

  // One trip per piece: item it, piece pp.  Items whose box misses the plane are
  // skipped without staging; the next piece's input (of this item or of the next
  // live one) is in flight during each piece's matrix work.
  auto next_live = [&](int from, Cov* cv) {
    for (; from < n_items; from += gridDim.x) {
      *cv = cov_of(from);
      if (cv->nI > 0) break;
    }
    return from;
  };
  // the central-axis depth of an item, read with a vector load so that it can be in
  // flight during the matrix loop (an outstanding scalar load there would make
  // each LDS wait a full one)
  auto depth_of = [&](int item) { return zca[item + opaque(0)]; };
  f32x4 buf[PGW];
  Cov c;
  int it = next_live(blockIdx.x, &c), pp = 0;
  float zk = 0.f;
  if (it < n_items) {
    int a, b;
    fetch_win<PGW>(in + (size_t)it * plane, g, win_of(c, 0, &a, &b), it == 0 || it == n_items - 1, tid, NT, buf);
    zk = depth_of(it);
  }
  while (it < n_items) {
    const float* src = in + (size_t)it * plane;
    float* dst = out + (size_t)it * plane;
    int nIp, nJp;
    const WinRect w = win_of(c, pp, &nIp, &nJp);
    put_win<PGW>(src, g, w, it == 0 || it == n_items - 1, pitch, tid, NT, buf, tile);
    if (pp == 0) taps_to_kx(g, it % g.Nk, zk, kx, E, off, tid, NT);
    // the next piece: (it, pp + 1) or the first piece of the next live item
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
      fetch_win<PGW>(in + (size_t)nit * plane, g, win_of(cn, npp, &a, &b), nit == 0 || nit == n_items - 1, tid,
                     NT, buf);
      if (npp == 0) zn = depth_of(nit);
    }
    const int Ip = w.r0 + h, Jp = w.c0 + h;  // the piece's first output row and column
    const int nT = nIp * nJp;
    const int C = nT < NW ? NW / nT : 1;  // tap-row chunks per tile
    const int chunk = wave % C, slot = wave / C, slots = NW / C;
    const int h1 = h + 1, pa = (h1 * chunk) / C, pb = (h1 * (chunk + 1)) / C - 1;
    int nact = 0;
    const float* ab[TPW];
    int oI[TPW], oJ[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = slot + slots * q;
      const bool use = t < nT;
      const int ti = use ? t / nJp : 0, tj = use ? t - (t / nJp) * nJp : 0;
      oI[q] = Ip + MT * ti;
      oJ[q] = Jp + MT * tj;
      ab[q] = tile + (MT * ti + m + h) * pitch + MT * tj + 4 * kk;
      nact += use ? 1 : 0;
    }
    f32x4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    // (SSC: the super-step count when fixed at compile time, 0 when not)
    if (SSC > 0) {
      if (nact == 1) f32_rows<1, SSC>(ab, bbase, pitch, E, pa, pb, acc);
      if (TPW >= 2 && nact == 2) f32_rows<TPW >= 2 ? 2 : 1, SSC>(ab, bbase, pitch, E, pa, pb, acc);
    } else {
      if (nact == 1) f32_steps<1>(ab, bbase, pitch, E, pa, pb, 0, SS - 1, acc);
      if (TPW >= 2 && nact == 2) f32_steps<TPW >= 2 ? 2 : 1>(ab, bbase, pitch, E, pa, pb, 0, SS - 1, acc);
    }
    if (C > 1) {
      // (C > 1 only with one tile per wavefront) chunks 1 .. C-1 park their sums,
      // chunk 0 adds them in order
      __syncthreads();
      if (chunk > 0 && nact > 0)
        park_partial((lds_f32x4*)(part + ((slot * (C - 1) + chunk - 1) * 64 + lane) * 4), acc[0]);
      __syncthreads();
      if (chunk == 0 && nact > 0) {
        for (int cc = 1; cc < C; ++cc)
          acc[0] += *reinterpret_cast<const f32x4*>(part + ((slot * (C - 1) + cc - 1) * 64 + lane) * 4);
        store_tile_from(g, oI[0], oJ[0], 0, 0, lane, acc[0], dst);
      }
    } else {
#pragma unroll
      for (int q = 0; q < TPW; ++q)
        if (q < nact) store_tile_from(g, oI[q], oJ[q], 0, 0, lane, acc[q], dst);
    }
    __syncthreads();  // the image (and, before a new item, the taps) are rewritten next
    it = nit;
    pp = npp;
    c = cn;
    zk = zn;
  }
}

// ------------------------------------------------------------------ launch

// Persistent grid: as many workgroups as fit on the device at once (a multiple of
// the region count), never more than there are items.
template <int NW, int TPW, int SUP>
static hipError_t launch_f32_cfg(const Geo<float>& g, const RegionShape& rs, const F32Shape& fs, size_t lds, int nb,
                                 const int4* box, const float* z, const float* in, float* out, hipStream_t s) {
  const void* kern = (const void*)k_conv_mfma_f32<NW, TPW, SUP>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)LDS_MAX);
    if (e != hipSuccess) return e;
  }
  if (lds > LDS_MAX) return hipErrorInvalidConfiguration;
  const int nreg = rs.regions_i * rs.regions_j;
  const long n_items = (long)nreg * g.Nk * nb;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  const int grid = persistent_grid(kern, 64 * NW, lds, nreg, n_items);
  hipLaunchKernelGGL((k_conv_mfma_f32<NW, TPW, SUP>), dim3(grid), dim3(64 * NW), lds, s, g, rs, fs, (int)n_items,
                     box, z, in, out);
  return hipGetLastError();
}

template <int SUP>
static hipError_t launch_f32_sup(const Geo<float>& g, const RegionShape& rs, const F32Shape& fs, size_t lds, int nb,
                                 const int4* box, const float* z, const float* in, float* out, hipStream_t s) {
  const int tiles = rs.TI * rs.TJ;
  if (tiles <= 4) return launch_f32_cfg<4, 1, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
  if (tiles <= 8) return launch_f32_cfg<8, 1, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
  if (tiles <= 16) return launch_f32_cfg<8, 2, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
  if (tiles <= 24) return launch_f32_cfg<8, 3, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
  // CONV_IN_BOX: tiles are taken dynamically.  When two workgroups' images fit in
  // one CU's LDS, two workgroups of 8 wavefronts share each CU, so one's matrix loop
  // runs while the other stages its next plane, builds its taps or waits at a
  // barrier; otherwise one of 16 wavefronts.  CONV_DENSE: three fixed tiles per
  // wavefront.
  if (SUP == CONV_IN_BOX) {
    if (2 * lds <= LDS_MAX) return launch_f32_cfg<8, 3, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
    return launch_f32_cfg<16, 3, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
  }
  return launch_f32_cfg<12, 3, SUP>(g, rs, fs, lds, nb, box, z, in, out, s);
}

// Wavefronts of the adjoint kernel for regions of more than 24 tiles (four per
// SIMD, which hide the LDS latency of the matrix loop better than three).
constexpr int kAdjNW = 16;

// LDS of the adjoint kernel: the FP32 image and taps plus NW x 256 partial sums
// (16-byte aligned).
static size_t f32_adj_lds(int h, const F32Shape& fs, int nw) { return f32_lds(h, fs) + 16 + sizeof(float) * 256 * nw; }

template <int NW, int TPW>
static hipError_t launch_f32_adj_cfg(const Geo<float>& g, const RegionShape& rs, const F32Shape& fs, int nb,
                                     const int4* box, const float* z, const float* in, float* out, hipStream_t s) {
  const void* kern = (const void*)k_conv_mfma_f32_adj<NW, TPW>;
  {
    hipError_t e = ensure_lds_limit(kern, (int)LDS_MAX);
    if (e != hipSuccess) return e;
  }
  const size_t lds = f32_adj_lds(g.h, fs, NW);
  if (lds > LDS_MAX) return hipErrorInvalidConfiguration;
  const int nreg = rs.regions_i * rs.regions_j;
  const long n_items = (long)nreg * g.Nk * nb;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  // as many workgroups as fit, the count prime to the region count (a workgroup's
  // items then visit every region)
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * NW, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  long grid = (long)device_cus() * per_cu;
  if (grid < 1) grid = 1;
  auto gcd = [](long a, long b) { while (b) { const long t = a % b; a = b; b = t; } return a; };
  while (grid > 1 && gcd(grid, nreg) != 1) --grid;
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL((k_conv_mfma_f32_adj<NW, TPW>), dim3((unsigned)grid), dim3(64 * NW), lds, s, g, rs, fs,
                     (int)n_items, box, z, in, out);
  return hipGetLastError();
}

static hipError_t launch_f32_adj(const Geo<float>& g, const RegionShape& rs, const F32Shape& fs, int nb,
                                 const int4* box, const float* z, const float* in, float* out, hipStream_t s) {
  const int tiles = rs.TI * rs.TJ;
  if (tiles <= 4) return launch_f32_adj_cfg<4, 1>(g, rs, fs, nb, box, z, in, out, s);
  if (tiles <= 8) return launch_f32_adj_cfg<8, 1>(g, rs, fs, nb, box, z, in, out, s);
  if (tiles <= 16) return launch_f32_adj_cfg<8, 2>(g, rs, fs, nb, box, z, in, out, s);
  if (tiles <= 24) return launch_f32_adj_cfg<8, 3>(g, rs, fs, nb, box, z, in, out, s);
  return launch_f32_adj_cfg<kAdjNW, 3>(g, rs, fs, nb, box, z, in, out, s);
}


// Wavefronts of the windowed adjoint: 8, two workgroups per CU at the field sizes
// of the clinical planes (eight wavefronts, whose tiles' tap rows are split over
// them, measured faster than four with whole tiles each).
constexpr int kAdjWinNW = 8;

static size_t f32_adj_win_lds(int h, const AdjWin& aw, int nw) {
  return sizeof(float) * ((size_t)aw.rows * aw.pitch + (size_t)(h + 1) * aw.E) + 16 + sizeof(float) * 256 * (nw - 1);
}

template <int TPW, int SSC>
static hipError_t launch_f32_adj_win_cfg(const Geo<float>& g, const AdjWin& aw, int nb, const int4* box,
                                         const float* z, const float* in, float* out, hipStream_t s) {
  constexpr int NW = kAdjWinNW;
  const void* kern = (const void*)k_conv_f32_adj_win<NW, TPW, SSC>;
  const size_t lds = f32_adj_win_lds(g.h, aw, NW);
  if (lds > LDS_MAX) return hipErrorInvalidConfiguration;
  {
    hipError_t e = ensure_lds_limit(kern, (int)lds);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)g.Nk * nb;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  const int grid = persistent_grid(kern, 64 * NW, lds, 1, n_items);
  hipLaunchKernelGGL((k_conv_f32_adj_win<NW, TPW, SSC>), dim3(grid), dim3(64 * NW), lds, s, g, aw, (int)n_items, box, z,
                     in, out);
  return hipGetLastError();
}

// Pieces sized for the largest rectangle that jaws inside the field limits give
// (bigger rectangles take several pieces), at most 16 tiles (two per wavefront),
// made smaller while the image does not fit the LDS.  False: not even one tile's
// image fits.
static bool f32_adj_win_shape(const Geo<float>& g, AdjWin* out) {
  const int half_u = (g.Nu - 1) / 2 - g.h, half_v = (g.Nv - 1) / 2 - g.h;  // field limit in pixels
  const int bu = 2 * (half_u > 0 ? half_u : 0) + 4, bv = 2 * (half_v > 0 ? half_v : 0) + 4;
  AdjWin aw;
  aw.WI = (bu + MT - 1) / MT;
  aw.WJ = (bv + MT - 1) / MT;
  // (pieces of 2 x 2 tiles for 3 x 3 rectangles were measured slower: the overlap
  // of their windows and the per-piece barriers cost more than the one wavefront
  // with two tiles)
  aw.WI = aw.WI < 1 ? 1 : (aw.WI > 4 ? 4 : aw.WI);
  aw.WJ = aw.WJ < 1 ? 1 : (aw.WJ > 4 ? 4 : aw.WJ);
  aw.SS = (MT + 2 * g.h + 15) / 16;
  aw.E = 16 * aw.SS + 16;
  for (;;) {
    aw.rows = MT * aw.WI + 2 * g.h;
    aw.pitch = pitch_f32(MT * (aw.WJ - 1) + 16 * aw.SS);
    if (f32_adj_win_lds(g.h, aw, kAdjWinNW) <= LDS_MAX) break;
    if (aw.WI == 1 && aw.WJ == 1) return false;
    if (aw.WJ >= aw.WI) --aw.WJ;
    else --aw.WI;
  }
  *out = aw;
  return true;
}

static hipError_t launch_f32_adj_win(const Geo<float>& g, const AdjWin& aw, int nb, const int4* box,
                                     const float* z, const float* in, float* out, hipStream_t s) {
  // one or two tiles per wavefront; super-step counts 2 to 5 (h 1 to 32) unrolled,
  // others looped
  if (aw.WI * aw.WJ <= kAdjWinNW) {
    switch (aw.SS) {
      case 2: return launch_f32_adj_win_cfg<1, 2>(g, aw, nb, box, z, in, out, s);
      case 3: return launch_f32_adj_win_cfg<1, 3>(g, aw, nb, box, z, in, out, s);
      case 4: return launch_f32_adj_win_cfg<1, 4>(g, aw, nb, box, z, in, out, s);
      case 5: return launch_f32_adj_win_cfg<1, 5>(g, aw, nb, box, z, in, out, s);
      default: return launch_f32_adj_win_cfg<1, 0>(g, aw, nb, box, z, in, out, s);
    }
  }
  switch (aw.SS) {
    case 2: return launch_f32_adj_win_cfg<2, 2>(g, aw, nb, box, z, in, out, s);
    case 3: return launch_f32_adj_win_cfg<2, 3>(g, aw, nb, box, z, in, out, s);
    case 4: return launch_f32_adj_win_cfg<2, 4>(g, aw, nb, box, z, in, out, s);
    case 5: return launch_f32_adj_win_cfg<2, 5>(g, aw, nb, box, z, in, out, s);
    default: return launch_f32_adj_win_cfg<2, 0>(g, aw, nb, box, z, in, out, s);
  }
}

hipError_t launch_conv_mfma_f32(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                                hipStream_t s, const int* box, int support) {
  const int4* bx = reinterpret_cast<const int4*>(box);
  // the forward with the rectangle in registers, unless the fluence corrections
  // widen the rectangles by their blur radii (then several chunks per plane would
  // repeat the tap loop; the tiled kernel below is faster there)
  if (bx && support == CONV_IN_BOX && !g.fcorr && conv_fwd_reg_supported(g, false))
    return launch_conv_fwd_reg(g, nb, z, in, out, s, box, false);
  // the adjoint with a window image, unless the fluence corrections widen the
  // rectangles past the field limits its pieces are sized for (then each rectangle
  // takes several pieces whose windows overlap; the region kernel below stages its
  // data once)
  AdjWin aw;
  if (bx && support == CONV_OUT_BOX && !g.fcorr && f32_adj_win_shape(g, &aw))
    return launch_f32_adj_win(g, aw, nb, bx, z, in, out, s);
  const bool adj = bx && support == CONV_OUT_BOX;
  RegionShape rs;
  F32Shape fs;
  size_t lds = 0;
  for (int rmax = RMAX; rmax >= 1; --rmax) {  // the largest region whose LDS image fits
    rs = region_shape(g.Nu, g.Nv, rmax);
    const bool in_box = bx && support == CONV_IN_BOX;
    fs = in_box ? f32_shape_in_box(g.h, rs, g.Nu, g.Nv) : f32_shape(g.h, rs);
    lds = adj ? f32_adj_lds(g.h, fs, kAdjNW) : f32_lds(g.h, fs) + (in_box ? kBoxTileLds : 0);
    if (lds <= LDS_MAX) break;
  }
  if (adj) return launch_f32_adj(g, rs, fs, nb, bx, z, in, out, s);
  if (!bx || support == CONV_DENSE) return launch_f32_sup<CONV_DENSE>(g, rs, fs, lds, nb, bx, z, in, out, s);
  return launch_f32_sup<CONV_IN_BOX>(g, rs, fs, lds, nb, bx, z, in, out, s);
}

}  // namespace pdrt
