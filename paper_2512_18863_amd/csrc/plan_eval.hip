// plan_eval.hip — plan assessment on the GPU (arXiv:2512.18863 §2.5 and §3): the
// weighted L1 dose objective of the optimisation study with its gradient with
// respect to the dose, differential dose-volume histograms with per-structure
// count / sum / maximum, and the number of voxels at or above a dose level (for
// the isodose Dice coefficient and V_d).
//
// Structures are one uint32 label per voxel, bit s = member of structure s.
// Every floating-point sum is formed per block in a fixed order and the block
// partials are added in a fixed order by one more block, so results do not
// depend on scheduling; counts are integers and may use atomics.
#include <cmath>

#include "pdrt_internal.hpp"

namespace pdrt {

namespace {

constexpr int EV_BLOCKS = 1024;
constexpr int EV_THREADS = 256;
constexpr int HIST_LDS_BINS = 16384;  // u32 counters per block (64 KB)

struct ObjTerms {
  int n;
  double weight[PDRT_MAX_STRUCTS], target[PDRT_MAX_STRUCTS];
};

// Sum over the block in a fixed order; the result is valid in thread 0.
__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

__device__ float block_max(float v, float* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  float s = v;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmaxf(s, sh[w]);
  __syncthreads();
  return s;
}

__global__ void __launch_bounds__(EV_THREADS) k_l1_objective(long n, const float* __restrict__ dose,
                                                             const uint32_t* __restrict__ labels, ObjTerms ot,
                                                             float* __restrict__ grad, double* __restrict__ part) {
  __shared__ double sh[EV_THREADS / 64];
  double acc = 0.0;
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    const double d = dose[v];
    const uint32_t m = labels[v];
    double gv = 0.0;
    for (int s = 0; s < ot.n; ++s) {
      if ((m >> s) & 1u) {
        const double x = d - ot.target[s];
        acc += ot.weight[s] * fabs(x);
        gv += x > 0.0 ? ot.weight[s] : (x < 0.0 ? -ot.weight[s] : 0.0);
      }
    }
    if (grad) grad[v] = (float)gv;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[i] = sum over j of part[i * n + j], j ascending per thread, then the block sum.
__global__ void __launch_bounds__(EV_THREADS) k_sum_rows(int n, const double* __restrict__ part,
                                                         double* __restrict__ out, int out_stride) {
  __shared__ double sh[EV_THREADS / 64];
  const double* row = part + (size_t)blockIdx.x * n;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) acc += row[j];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(size_t)blockIdx.x * out_stride] = s;
}

// stats[s] = (count, sum, max) from the partial rows part[s][0..2][0..n).
__global__ void __launch_bounds__(EV_THREADS) k_stats_final(int n, const double* __restrict__ part,
                                                            double* __restrict__ stats) {
  __shared__ double sh[EV_THREADS / 64];
  __shared__ float shm[EV_THREADS / 64];
  const double* row = part + (size_t)blockIdx.x * 3 * n;
  double c = 0.0, t = 0.0;
  float mx = 0.f;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    c += row[j];
    t += row[n + j];
    mx = fmaxf(mx, (float)row[2 * n + j]);
  }
  const double sc = block_sum(c, sh);
  const double st = block_sum(t, sh);
  const float sm = block_max(mx, shm);
  if (threadIdx.x == 0) {
    stats[3 * blockIdx.x] = sc;
    stats[3 * blockIdx.x + 1] = st;
    stats[3 * blockIdx.x + 2] = (double)sm;
  }
}

__device__ __forceinline__ int dose_bin(float d, int n_bins, double width) {
  const double q = floor((double)d / width);
  if (!(q >= 0.0)) return 0;
  return q >= (double)(n_bins - 1) ? n_bins - 1 : (int)q;
}

// Structures s0 .. s0 + ns - 1 with block-private LDS counters.
__global__ void __launch_bounds__(EV_THREADS) k_histogram(long n, const float* __restrict__ dose,
                                                          const uint32_t* __restrict__ labels, int s0, int ns,
                                                          int n_bins, double width, uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t lh[];
  const int cells = ns * n_bins;
  for (int i = threadIdx.x; i < cells; i += blockDim.x) lh[i] = 0u;
  __syncthreads();
  const uint32_t sel = ns >= 32 ? 0xffffffffu : ((1u << ns) - 1u);
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    uint32_t m = (labels[v] >> s0) & sel;
    if (!m) continue;
    const int b = dose_bin(dose[v], n_bins, width);
    while (m) {
      const int s = __builtin_ctz(m);
      atomicAdd(&lh[s * n_bins + b], 1u);
      m &= m - 1u;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cells; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[(size_t)s0 * n_bins + i], lh[i]);
}

// Per block and structure s = blockIdx.y: count, sum and maximum of the dose.
__global__ void __launch_bounds__(EV_THREADS) k_struct_stats(long n, const float* __restrict__ dose,
                                                             const uint32_t* __restrict__ labels,
                                                             double* __restrict__ part) {
  __shared__ double sh[EV_THREADS / 64];
  __shared__ float shm[EV_THREADS / 64];
  const int s = blockIdx.y;
  double sum = 0.0, cnt = 0.0;
  float mx = 0.f;
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    if ((labels[v] >> s) & 1u) {
      const float d = dose[v];
      sum += (double)d;
      cnt += 1.0;
      mx = fmaxf(mx, d);
    }
  }
  const double ssum = block_sum(sum, sh);
  const double scnt = block_sum(cnt, sh);
  const float smax = block_max(mx, shm);
  if (threadIdx.x == 0) {
    const size_t base = (size_t)s * 3 * gridDim.x;
    part[base + blockIdx.x] = scnt;
    part[base + gridDim.x + blockIdx.x] = ssum;
    part[base + 2 * gridDim.x + blockIdx.x] = (double)smax;
  }
}

// counts[s] += voxels of structure s with dose >= thr; counts[n_struct] += all such voxels.
__global__ void __launch_bounds__(EV_THREADS) k_threshold_counts(long n, const float* __restrict__ dose,
                                                                 const uint32_t* __restrict__ labels, int n_struct,
                                                                 double thr, unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long wc[EV_THREADS / 64][PDRT_MAX_STRUCTS + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane <= n_struct) wc[wave][lane] = 0ull;
  const long stride = (long)gridDim.x * blockDim.x;
  const long v0 = (long)blockIdx.x * blockDim.x + threadIdx.x - lane;  // first voxel of this wavefront
  for (long base = v0; base < n; base += stride) {
    const long v = base + lane;
    const bool in = v < n;
    const bool hot = in && (double)dose[v] >= thr;
    const uint32_t m = hot ? labels[v] : 0u;
    const unsigned long long all = __ballot(hot);
    if (lane == 0) wc[wave][n_struct] += __popcll(all);
    for (int s = 0; s < n_struct; ++s) {
      const unsigned long long b = __ballot((m >> s) & 1u);
      if (lane == 0) wc[wave][s] += __popcll(b);
    }
  }
  __syncthreads();
  if (threadIdx.x <= n_struct) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wc[w][threadIdx.x];
    if (t) atomicAdd(&counts[threadIdx.x], t);
  }
}

__global__ void k_fill_u32(size_t n, uint32_t* p) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_fill_u64(size_t n, unsigned long long* p) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}


bool eval_args_ok(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct) {
  return n_vox >= 0 && n_vox < (int64_t)0xffffffffLL && (n_vox == 0 || (dose && labels)) && n_struct >= 1 &&
         n_struct <= PDRT_MAX_STRUCTS;
}

int ev_grid(int64_t n_vox) {
  const int64_t want = (n_vox + EV_THREADS - 1) / EV_THREADS;
  return (int)(want < 1 ? 1 : (want > EV_BLOCKS ? EV_BLOCKS : want));
}

}  // namespace

}  // namespace pdrt

using namespace pdrt;

extern "C" {

size_t pdrt_eval_ws_bytes(int32_t n_struct) {
  if (n_struct < 1 || n_struct > PDRT_MAX_STRUCTS) return 0;
  return sizeof(double) * (size_t)EV_BLOCKS * 3 * n_struct;
}

int pdrt_l1_objective(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct,
                      const double* weight, const double* target, double* loss, float* grad, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!eval_args_ok(n_vox, dose, labels, n_struct) || !weight || !target || !loss) return PDRT_E_INVALID;
  if (!ws || ws_bytes < pdrt_eval_ws_bytes(n_struct)) return PDRT_E_WORKSPACE;
  ObjTerms ot;
  ot.n = n_struct;
  for (int s = 0; s < PDRT_MAX_STRUCTS; ++s) {
    ot.weight[s] = s < n_struct ? weight[s] : 0.0;
    ot.target[s] = s < n_struct ? target[s] : 0.0;
    if (!std::isfinite(ot.weight[s]) || !std::isfinite(ot.target[s])) return PDRT_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)ws;
  const int grid = ev_grid(n_vox);
  PDRT_TIMED("l1_objective", s,
             [&]() {
               hipLaunchKernelGGL(k_l1_objective, dim3(grid), dim3(EV_THREADS), 0, s, (long)n_vox, dose, labels, ot,
                                 grad, part);
               return hipGetLastError();
             }());
  PDRT_TIMED("l1_objective", s,
             [&]() {
               hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(EV_THREADS), 0, s, grid, (const double*)part, loss, 1);
               return hipGetLastError();
             }());
  return PDRT_OK;
}

int pdrt_dose_histogram(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct, int32_t n_bins,
                        double bin_width, uint32_t* hist, double* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!eval_args_ok(n_vox, dose, labels, n_struct) || !hist || !stats) return PDRT_E_INVALID;
  if (n_bins < 1 || n_bins > HIST_LDS_BINS || !std::isfinite(bin_width) || !(bin_width > 0.0))
    return PDRT_E_INVALID;
  if (!ws || ws_bytes < pdrt_eval_ws_bytes(n_struct)) return PDRT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const size_t cells = (size_t)n_struct * n_bins;
  PDRT_TIMED("dose_histogram", s,
             [&]() {
               hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((cells + 255) / 256 < 1024 ? (cells + 255) / 256 : 1024)),
                                 dim3(256), 0, s, cells, hist);
               return hipGetLastError();
             }());
  if (ensure_lds_limit((const void*)k_histogram, (int)(HIST_LDS_BINS * sizeof(uint32_t))) != hipSuccess)
    return PDRT_E_HIP;
  const int grid = ev_grid(n_vox);
  const int per_pass = HIST_LDS_BINS / n_bins;
  for (int s0 = 0; s0 < n_struct; s0 += per_pass) {
    const int ns = n_struct - s0 < per_pass ? n_struct - s0 : per_pass;
    const size_t lds = sizeof(uint32_t) * (size_t)ns * n_bins;
    PDRT_TIMED("dose_histogram", s,
               [&]() {
               hipLaunchKernelGGL(k_histogram, dim3(grid), dim3(EV_THREADS), lds, s, (long)n_vox, dose, labels, s0,
                                   ns, (int)n_bins, bin_width, hist);
               return hipGetLastError();
             }());
  }
  double* part = (double*)ws;
  PDRT_TIMED("dose_histogram", s,
             [&]() {
               hipLaunchKernelGGL(k_struct_stats, dim3(grid, n_struct), dim3(EV_THREADS), 0, s, (long)n_vox, dose,
                                 labels, part);
               return hipGetLastError();
             }());
  // part = [s][count | sum | max][grid]: rows of `grid` partials, one output per row
  PDRT_TIMED("dose_histogram", s,
             [&]() {
               hipLaunchKernelGGL(k_stats_final, dim3(n_struct), dim3(EV_THREADS), 0, s, grid, (const double*)part,
                                 stats);
               return hipGetLastError();
             }());
  return PDRT_OK;
}

int pdrt_threshold_counts(int64_t n_vox, const float* dose, const uint32_t* labels, int32_t n_struct,
                          double threshold, uint64_t* counts, void* stream) {
  if (!eval_args_ok(n_vox, dose, labels, n_struct) || !counts || std::isnan(threshold)) return PDRT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  PDRT_TIMED("threshold_counts", s,
             [&]() {
               hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (size_t)n_struct + 1,
                                 (unsigned long long*)counts);
               return hipGetLastError();
             }());
  PDRT_TIMED("threshold_counts", s,
             [&]() {
               hipLaunchKernelGGL(k_threshold_counts, dim3(ev_grid(n_vox)), dim3(EV_THREADS), 0, s, (long)n_vox,
                                 dose, labels, (int)n_struct, threshold, (unsigned long long*)counts);
               return hipGetLastError();
             }());
  return PDRT_OK;
}

}  // extern "C"
