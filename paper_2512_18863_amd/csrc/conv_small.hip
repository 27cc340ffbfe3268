// conv_small.hip — the per-plane lateral convolution (arXiv:2512.18863 §2.2.6,
// Eq. 8) for small kernels (n <= 11) on the vector ALUs.
//
// With few taps a plane costs little arithmetic (81 FMAs per output at n = 9), so
// what has to be avoided is per-plane overhead: the whole width of the plane (a
// band of its rows when it is tall) is one workgroup's LDS image, workgroups are
// persistent over the (control point, plane) items of their band, the zero halo
// is written once, the next item's input is fetched into registers while the
// current item is convolved, and the n x n taps are evaluated straight into LDS.
//
// A thread owns R = 8 consecutive outputs of one row i.  For each tap row p it
// reads the R + n - 1 image values of row i + p that they need (16-byte LDS
// reads at fixed offsets) and the n taps of row p (broadcast reads), then does
// R n FMAs from registers.  Lanes run along i; the image pitch is 4 mod 32
// floats, so the 16-byte reads of eight neighbouring lanes hit distinct banks.
#include "conv_common.hpp"

namespace pdrt {

namespace {

constexpr int SR = 8;               // outputs per thread along v
constexpr int SPF = 8;              // prefetched elements per thread
constexpr size_t SMALL_LDS_MAX = 48 * 1024;

typedef float f32x4s __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int round4(int x) { return (x + 3) & ~3; }

struct SmallShape {
  int band_rows;                    // output rows per band
  int bands;                        // ceil(Nu / band_rows)
  int jblocks;                      // ceil(Nv / SR)
  int pitch;                        // LDS image row pitch (floats), 4 mod 32
  int rows;                         // LDS image rows: band_rows + n - 1
};

size_t small_lds(int n, const SmallShape& ss) {
  return sizeof(float) * ((size_t)ss.rows * ss.pitch + (size_t)n * round4(n));
}

bool small_shape(const Geo<float>& g, SmallShape* ss) {
  const int n = g.n_taps;
  ss->jblocks = (g.Nv + SR - 1) / SR;
  // the last column block reads round4(SR + n - 1) values from column SR (jblocks - 1)
  const int cols = SR * (ss->jblocks - 1) + round4(SR + n - 1);
  ss->pitch = ((cols + 27) / 32) * 32 + 4;
  int band_rows = g.Nu;
  while (true) {
    ss->band_rows = band_rows;
    ss->bands = (g.Nu + band_rows - 1) / band_rows;
    ss->rows = band_rows + n - 1;
    if (small_lds(n, *ss) <= SMALL_LDS_MAX) return true;
    if (band_rows <= 8) return false;
    band_rows = (band_rows + 1) / 2;
  }
}

// Items it = blockIdx.x, blockIdx.x + gridDim.x, ... with band = it % bands and
// (control point, plane) = it / bands; gridDim.x is a multiple of the band count,
// so a workgroup keeps one band: its data rectangle, and with it the zero border
// of the image and every thread's load and store offsets, are fixed.
template <int N>
__global__ void __launch_bounds__(256) k_conv_small(Geo<float> g, SmallShape ss, int n_items,
                                                    const float* __restrict__ zca, const float* __restrict__ in,
                                                    float* __restrict__ out) {
  extern __shared__ __align__(16) float lds[];
  constexpr int H = N / 2, WR = round4(SR + N - 1), KP = round4(N);
  const int nt = blockDim.x, tid = threadIdx.x;
  const int pitch = ss.pitch;
  float* img = lds;                      // image row r, column c = plane row I0 - H + r, column c - H
  float* K = lds + ss.rows * pitch;      // N rows of KP taps
  const int band = blockIdx.x % ss.bands;
  const int I0 = band * ss.band_rows;
  const int out_rows = min(ss.band_rows, g.Nu - I0);
  const DataRect dr = data_rect(g, I0, 0, out_rows, g.Nv);
  const size_t plane = (size_t)g.Nu * g.Nv;
  const int tasks = out_rows * ss.jblocks;
  const int area = dr.nr * dr.nc;

  // this thread's first SPF elements of the data rectangle: plane and image offsets
  int goff[SPF], loff[SPF];
#pragma unroll
  for (int e = 0; e < SPF; ++e) {
    const int idx = tid + e * nt;
    const int r = idx / dr.nc, c = idx - r * dr.nc;
    goff[e] = idx < area ? (dr.r0 + r) * g.Nv + dr.c0 + c : -1;
    loff[e] = (dr.lr0 + r) * pitch + dr.lc0 + c;
  }
  auto fetch = [&](int item, float (&buf)[SPF], float& zk) {
    const float* src = in + (size_t)(item / ss.bands) * plane;
#pragma unroll
    for (int e = 0; e < SPF; ++e) buf[e] = goff[e] >= 0 ? src[goff[e]] : 0.f;
    zk = zca[item / ss.bands];
  };

  for (int idx = tid; idx < ss.rows * pitch + N * KP; idx += nt) lds[idx] = 0.f;
  float buf[SPF], zk = 0.f;
  int it = blockIdx.x;
  if (it < n_items) fetch(it, buf, zk);
  __syncthreads();
  for (; it < n_items; it += gridDim.x) {
    const int bk = it / ss.bands;  // b * Nk + k
    const int k = bk % g.Nk;
    const float* src = in + (size_t)bk * plane;
#pragma unroll
    for (int e = 0; e < SPF; ++e)
      if (goff[e] >= 0) img[loff[e]] = buf[e];
    for (int idx = tid + SPF * nt; idx < area; idx += nt) {  // planes larger than SPF elements per thread
      const int r = idx / dr.nc, c = idx - r * dr.nc;
      img[(dr.lr0 + r) * pitch + dr.lc0 + c] = src[(size_t)(dr.r0 + r) * g.Nv + dr.c0 + c];
    }
    if (tid < N * N) {
      const TapParams<float> tp = tap_params(g, k, zk);
      const int p = tid / N, q = tid - (tid / N) * N;
      const int dp = p - H, dq = q - H;
      K[p * KP + q] = tap_value(tp, dp < 0 ? -dp : dp, dq < 0 ? -dq : dq);
    }
    __syncthreads();
    const int nx = it + gridDim.x;
    if (nx < n_items) fetch(nx, buf, zk);

    float* dst = out + (size_t)bk * plane;
    for (int t = tid; t < tasks; t += nt) {
      const int jb = t / out_rows, i = t - jb * out_rows;
      const float* row = img + i * pitch + SR * jb;
      float acc[SR];
#pragma unroll
      for (int r = 0; r < SR; ++r) acc[r] = 0.f;
#pragma unroll 1
      for (int p = 0; p < N; ++p) {
        float w[WR], kq[KP];
#pragma unroll
        for (int e = 0; e < WR; e += 4) {
          const f32x4s v = *reinterpret_cast<const f32x4s*>(row + p * pitch + e);
          w[e] = v[0];
          w[e + 1] = v[1];
          w[e + 2] = v[2];
          w[e + 3] = v[3];
        }
#pragma unroll
        for (int e = 0; e < KP; e += 4) {
          const f32x4s v = *reinterpret_cast<const f32x4s*>(K + p * KP + e);
          kq[e] = v[0];
          kq[e + 1] = v[1];
          kq[e + 2] = v[2];
          kq[e + 3] = v[3];
        }
#pragma unroll
        for (int q = 0; q < N; ++q)
#pragma unroll
          for (int r = 0; r < SR; ++r) acc[r] = fmaf(kq[q], w[r + q], acc[r]);
      }
      const int j0 = SR * jb;
      float* o = dst + (size_t)(I0 + i) * g.Nv + j0;
#pragma unroll
      for (int r = 0; r < SR; ++r)
        if (j0 + r < g.Nv) o[r] = acc[r];
    }
    __syncthreads();  // the image and taps are rewritten for the next item
  }
}

template <int N>
hipError_t launch_small_n(const Geo<float>& g, const SmallShape& ss, int nb, const float* z, const float* in,
                          float* out, hipStream_t s) {
  const void* kern = (const void*)k_conv_small<N>;
  const size_t lds = small_lds(N, ss);
  {
    hipError_t e = ensure_lds_limit(kern, (int)SMALL_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  const long n_items = (long)ss.bands * g.Nk * nb;
  if (n_items > 0x7fffffffL) return hipErrorInvalidConfiguration;
  // whole wavefronts that cover one band's tasks in as few rounds as possible
  const int tasks = ss.band_rows * ss.jblocks;
  const int rounds = (tasks + 255) / 256;
  int threads = ((tasks + rounds - 1) / rounds + 63) / 64 * 64;
  if (threads < N * N) threads = (N * N + 63) / 64 * 64;
  const int grid = persistent_grid(kern, threads, lds, ss.bands, n_items);
  hipLaunchKernelGGL((k_conv_small<N>), dim3(grid), dim3(threads), lds, s, g, ss, (int)n_items, z, in, out);
  return hipGetLastError();
}

}  // namespace

bool conv_small_supported(const Geo<float>& g) {
  SmallShape ss;
  return g.n_taps <= 11 && (g.n_taps & 1) && small_shape(g, &ss);
}

hipError_t launch_conv_small(const Geo<float>& g, int nb, const float* z, const float* in, float* out,
                             hipStream_t s) {
  SmallShape ss;
  if (!conv_small_supported(g) || !small_shape(g, &ss)) return hipErrorInvalidConfiguration;
  switch (g.n_taps) {
    case 1: return launch_small_n<1>(g, ss, nb, z, in, out, s);
    case 3: return launch_small_n<3>(g, ss, nb, z, in, out, s);
    case 5: return launch_small_n<5>(g, ss, nb, z, in, out, s);
    case 7: return launch_small_n<7>(g, ss, nb, z, in, out, s);
    case 9: return launch_small_n<9>(g, ss, nb, z, in, out, s);
    case 11: return launch_small_n<11>(g, ss, nb, z, in, out, s);
    default: return hipErrorInvalidConfiguration;
  }
}

}  // namespace pdrt
