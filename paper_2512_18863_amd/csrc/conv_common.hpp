// conv_common.hpp — staging helpers shared by the per-plane lateral convolutions
// (arXiv:2512.18863 §2.2.6, Eq. 8): the unique taps of a plane, the rectangle of a
// plane that one workgroup's LDS image holds, register prefetch of the next
// plane, the windowed adjoints' staging in four-column groups, and the grid of a
// persistent launch.
#pragma once

#include "taps.hpp"

namespace pdrt {

// Unique taps K[p][q], 0 <= p, q <= h, of the plane into `kq` ((h+1) x (h+1)).
// The kernel is radial (K[p][q] = K[q][p], the same expression of p^2 + q^2), so
// only the pairs p <= q are evaluated, numbered column by column (pair t is
// q = floor((sqrt(8t + 1) - 1) / 2), p = t - q (q + 1) / 2), and each is written
// to both places.
__device__ __forceinline__ void unique_taps(const Geo<float>& g, int k, float zk, float* kq, int tid, int nt) {
  TapParams<float> tp = tap_params(g, k, zk);
  const int h1 = g.h + 1;
  for (int t = tid; t < h1 * (h1 + 1) / 2; t += nt) {
    int q = (int)((sqrtf((float)(8 * t + 1)) - 1.f) * 0.5f);
    if ((q + 1) * (q + 2) / 2 <= t) ++q;
    if (q * (q + 1) / 2 > t) --q;
    const int p = t - q * (q + 1) / 2;
    const float v = tap_value(tp, p, q);
    kq[p * h1 + q] = v;
    kq[q * h1 + p] = v;
  }
}

// The same taps written straight into extended tap rows: kx[p][off + q] =
// kx[p][off - q] = K[p][q] for 0 <= p, q <= h, row p = 0 scaled by s0 (0.5 for the
// folded rows of the FP32 adjoint, which count that row twice; 1 otherwise).  Pair
// (p, q), p <= q, fills the four places of K[p][q] and of K[q][p]; every entry
// within h of `off` is written, the rest of each row (zero) is not touched.
__device__ __forceinline__ void taps_to_kx(const Geo<float>& g, int k, float zk, float* kx, int E, int off, int tid,
                                           int nt, float s0 = 0.5f) {
  TapParams<float> tp = tap_params(g, k, zk);
  const int h1 = g.h + 1;
  for (int t = tid; t < h1 * (h1 + 1) / 2; t += nt) {
    int q = (int)((sqrtf((float)(8 * t + 1)) - 1.f) * 0.5f);
    if ((q + 1) * (q + 2) / 2 <= t) ++q;
    if (q * (q + 1) / 2 > t) --q;
    const int p = t - q * (q + 1) / 2;
    const float v = tap_value(tp, p, q);
    const float vp = p == 0 ? s0 * v : v;  // row p
    const float vq = q == 0 ? s0 * v : v;  // row q
    kx[p * E + off + q] = vp;
    kx[p * E + off - q] = vp;
    kx[q * E + off + p] = vq;
    kx[q * E + off - p] = vq;
  }
}

// The part of the plane that a region's LDS image holds: rows [r0, r0 + nr) and
// columns [c0, c0 + nc) of the plane, stored at LDS row r - (I0 - h), column
// c - (J0 - h).  Everything else in the image is zero and stays zero.
struct DataRect {
  int r0, nr, c0, nc;
  int lr0, lc0;  // LDS row / column of (r0, c0)
};

__device__ __forceinline__ DataRect data_rect(const Geo<float>& g, int I0, int J0, int out_rows, int out_cols) {
  const int h = g.h;
  DataRect d;
  d.r0 = max(0, I0 - h);
  d.c0 = max(0, J0 - h);
  d.nr = max(0, min(g.Nu, I0 + out_rows + h) - d.r0);
  d.nc = max(0, min(g.Nv, J0 + out_cols + h) - d.c0);
  d.lr0 = d.r0 - (I0 - h);
  d.lc0 = d.c0 - (J0 - h);
  return d;
}

// Issue the global loads of the first PF * nt elements of one plane's data
// rectangle into registers (the caller consumes them after other work).
// (The element index goes through an empty asm statement so that the compiler
// recomputes the index arithmetic per item instead of keeping PF offsets live
// across the matrix loop.)
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Row and column of the elements tid, tid + nt, tid + 2 nt, ... of a rectangle nc
// wide (element idx at row idx / nc, column idx % nc), advanced by one addition
// and a carry instead of a division per element.
struct RectWalk {
  int r, c, dr, dc;
  __device__ __forceinline__ RectWalk(int tid, int nt, int nc) {
    r = opaque(tid) / nc;
    c = tid - r * nc;
    dr = nt / nc;
    dc = nt - dr * nc;
  }
  __device__ __forceinline__ void next(int nc) {
    r += dr;
    c += dc;
    if (c >= nc) {
      c -= nc;
      ++r;
    }
  }
};

template <int PF>
__device__ __forceinline__ void fetch_rect(const float* __restrict__ src, int Nv, const DataRect& d, int tid, int nt,
                                           float (&buf)[PF]) {
  RectWalk w(tid, nt, d.nc);
  const float* s0 = src + (size_t)d.r0 * Nv + d.c0;
#pragma unroll
  for (int e = 0; e < PF; ++e) {
    float v = 0.f;
    if (w.r < d.nr) v = s0[w.r * Nv + w.c];
    buf[e] = v;
    w.next(d.nc);
  }
}

// Write the fetched elements into the LDS image, then load and write whatever
// lies beyond PF * nt directly.
template <int PF, typename E>
__device__ __forceinline__ void put_rect(const float* __restrict__ src, int Nv, const DataRect& d, int pitch,
                                         int tid, int nt, const float (&buf)[PF], E* tile) {
  RectWalk w(tid, nt, d.nc);
  E* t0 = tile + d.lr0 * pitch + d.lc0;
#pragma unroll
  for (int e = 0; e < PF; ++e) {
    if (w.r < d.nr) t0[w.r * pitch + w.c] = (E)buf[e];
    w.next(d.nc);
  }
  const float* s0 = src + (size_t)d.r0 * Nv + d.c0;
  for (; w.r < d.nr; w.next(d.nc)) t0[w.r * pitch + w.c] = (E)s0[w.r * Nv + w.c];
}

template <typename E>
__device__ __forceinline__ void zero_lds(E* p, int n, int tid, int nt) {
  for (int idx = tid; idx < n; idx += nt) p[idx] = (E)0.f;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// A piece's window: plane rows [r0, r0 + nr) and columns [c0, c0 + nc) go to image
// rows and columns [0, nr) x [0, nc); plane positions outside the plane read zero.
struct WinRect {
  int r0, c0, nr, nc;
};

// Staging of a window in groups of four columns.  A thread keeps one column group
// and walks rows with a stride of NT / (groups per row): its column tests are made
// once per piece, and each group is one four-word load (any word address) and one
// 16-byte LDS store.  Positions outside the plane read as zero.  A group partly
// outside the plane's columns reads the words before column 0 or after column
// Nv - 1 from the neighbouring row and clears them; only in the batch's first and
// last planes could that leave the batch's data (before its first row, after its
// last), so those planes are loaded word by word, the columns inside only.
typedef float f32x4u_w __attribute__((ext_vector_type(4), aligned(4)));

struct WinStage {
  int cg, r0, step;  // the thread's column group and first window row; rows per pass
  int pc;            // plane column of the group's first element
  int cmask;         // bit e: column pc + e lies in the plane
};

__device__ __forceinline__ WinStage win_stage(const Geo<float>& g, const WinRect& w, int tid, int nt) {
  WinStage st;
  const int gw = w.nc >> 2;
  st.r0 = opaque(tid) / gw;
  st.cg = tid - st.r0 * gw;
  st.step = nt / gw;
  if (st.r0 >= st.step) st.r0 = w.nr;  // threads past the last whole row of groups stay idle
  st.pc = w.c0 + 4 * st.cg;
  st.cmask = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) st.cmask |= (st.pc + e >= 0 && st.pc + e < g.Nv) ? 1 << e : 0;
  return st;
}

// Group r (window row) of the stage as loaded: positions outside the plane hold
// whatever lies there (or zero) until mask_group clears them, so that a prefetch
// does not wait for its loads.  SAFE (the batch's first and last planes) loads word
// by word only the columns inside the plane; it is a uniform choice per plane, so
// both forms keep every load of a thread in registers of its own.
__device__ __forceinline__ bool group_row_ok(const Geo<float>& g, const WinRect& w, const WinStage& st, int r) {
  const int pr = w.r0 + r;
  return pr >= 0 && pr < g.Nu && st.cmask != 0;
}

template <bool SAFE>
__device__ __forceinline__ f32x4 load_group(const float* __restrict__ src, const Geo<float>& g, const WinRect& w,
                                            const WinStage& st, int r) {
  const int pr = w.r0 + r;
  const bool rok = group_row_ok(g, w, st, r);
  const float* p = src + (rok ? pr * g.Nv + st.pc : 0);
  f32x4 v;
  if (SAFE) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = rok && ((st.cmask >> e) & 1) ? p[e] : 0.f;
  } else {
    const f32x4u_w x = *reinterpret_cast<const f32x4u_w*>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = x[e];
  }
  return v;
}

__device__ __forceinline__ f32x4 mask_group(const Geo<float>& g, const WinRect& w, const WinStage& st, int r,
                                            f32x4 v) {
  const bool rok = group_row_ok(g, w, st, r);
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = rok && ((st.cmask >> e) & 1) ? v[e] : 0.f;
  return v;
}

template <int PG, bool SAFE>
__device__ __forceinline__ void fetch_win_as(const float* __restrict__ src, const Geo<float>& g, const WinRect& w,
                                             int tid, int nt, f32x4 (&buf)[PG]) {
  const WinStage st = win_stage(g, w, tid, nt);
  // every group is loaded (rows past the window read in-plane data or nothing and
  // are not stored), so that no register keeps an older value beside the load
#pragma unroll
  for (int e = 0; e < PG; ++e) buf[e] = load_group<SAFE>(src, g, w, st, st.r0 + e * st.step);
}

template <int PG>
__device__ __forceinline__ void fetch_win(const float* __restrict__ src, const Geo<float>& g, const WinRect& w,
                                          bool edge, int tid, int nt, f32x4 (&buf)[PG]) {
  if (edge) fetch_win_as<PG, true>(src, g, w, tid, nt, buf);
  else fetch_win_as<PG, false>(src, g, w, tid, nt, buf);
}

template <int PG>
__device__ __forceinline__ void put_win(const float* __restrict__ src, const Geo<float>& g, const WinRect& w,
                                        bool edge, int pitch, int tid, int nt, const f32x4 (&buf)[PG],
                                        float* tile) {
  const WinStage st = win_stage(g, w, tid, nt);
  float* t = tile + st.r0 * pitch + 4 * st.cg;
#pragma unroll
  for (int e = 0; e < PG; ++e) {
    const int r = st.r0 + e * st.step;
    if (r < w.nr) *reinterpret_cast<f32x4*>(t + e * st.step * pitch) = mask_group(g, w, st, r, buf[e]);
  }
  for (int r = st.r0 + PG * st.step; r < w.nr; r += st.step) {
    const f32x4 v = edge ? load_group<true>(src, g, w, st, r) : load_group<false>(src, g, w, st, r);
    *reinterpret_cast<f32x4*>(tile + r * pitch + 4 * st.cg) = mask_group(g, w, st, r, v);
  }
}

inline int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cached[dev] = n;
  }
  return cached[dev];
}

inline int persistent_grid(const void* kern, int threads, size_t lds, int nreg, long n_items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  long want = (long)device_cus() * per_cu;
  if (want < nreg) want = nreg;
  want -= want % nreg;
  return (int)(n_items < want ? n_items : want);
}

}  // namespace pdrt
