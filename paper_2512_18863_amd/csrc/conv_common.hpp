// conv_common.hpp — staging helpers shared by the per-plane lateral convolutions
// (arXiv:2512.18863 §2.2.6, Eq. 8): the unique taps of a plane, the rectangle of a
// plane that one workgroup's LDS image holds, register prefetch of the next
// plane, and the grid of a persistent launch.
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

// The same taps written straight into the extended, folded tap rows of the FP32
// matrix kernels: kx[p][off + q] = kx[p][off - q] = K[p][q] for 0 <= p, q <= h,
// row p = 0 halved (the fold counts it twice).  Pair (p, q), p <= q, fills the
// four places of K[p][q] and of K[q][p]; every entry within h of `off` is written,
// the rest of each row (zero) is not touched.
__device__ __forceinline__ void taps_to_kx(const Geo<float>& g, int k, float zk, float* kx, int E, int off, int tid,
                                           int nt) {
  TapParams<float> tp = tap_params(g, k, zk);
  const int h1 = g.h + 1;
  for (int t = tid; t < h1 * (h1 + 1) / 2; t += nt) {
    int q = (int)((sqrtf((float)(8 * t + 1)) - 1.f) * 0.5f);
    if ((q + 1) * (q + 2) / 2 <= t) ++q;
    if (q * (q + 1) / 2 > t) --q;
    const int p = t - q * (q + 1) / 2;
    const float v = tap_value(tp, p, q);
    const float vp = p == 0 ? 0.5f * v : v;  // row p
    const float vq = q == 0 ? 0.5f * v : v;  // row q
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
