// Mutual-information scores of the feature rows against the noisy pixel values, used to rank
// the features before they are cut into windows of at most three (paper Sec. 5, generation of
// the windows).  Plug-in estimate from a joint histogram of uniformly binned values.
//
// Three launches: the minimum and maximum of every row (one block per row), the joint
// histograms (LDS counters per block, one global add per non-empty counter), and the scores
// (one block per feature, fixed reduction order).  All binning arithmetic is IEEE double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>

#include "nld_internal.h"

namespace nld {
namespace {

constexpr int kMisThreads = 256;
constexpr int kMisLds = 32 * 1024;   // bytes of LDS counters per histogram block

// Bin of value x: min(B - 1, floor((x - lo) * s)), s = B / (hi - lo), or 0 when hi = lo.
// Always in [0, B - 1] (a NaN goes to bin 0), so the counter index never leaves the table.
__device__ __forceinline__ int mis_bin(double x, double lo, double s, int B) {
  const double q = floor((x - lo) * s);
  return q >= 0.0 ? (q < (double)(B - 1) ? (int)q : B - 1) : 0;
}

struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpAdd { __device__ double operator()(double a, double b) const { return a + b; } };

// Fixed-tree reduction over the block (kMisThreads threads); every thread gets the result.
template <typename Op>
__device__ double block_reduce(double v, Op op, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kMisThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = op(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Row r < d is feature r, row d is the target.  Writes lo, hi and the bin scale of the row.
template <typename T>
__global__ void __launch_bounds__(kMisThreads)
k_mis_range(const T* __restrict__ F, const T* __restrict__ y, long long N, int d, int B,
            double* __restrict__ par) {
  __shared__ double sh[kMisThreads];
  const int r = blockIdx.x;
  const T* x = r < d ? F + (size_t)r * N : y;
  double lo = INFINITY, hi = -INFINITY;
  for (long long i = threadIdx.x; i < N; i += kMisThreads) {
    const double v = (double)x[i];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  lo = block_reduce(lo, OpMin(), sh);
  hi = block_reduce(hi, OpMax(), sh);
  if (threadIdx.x == 0) {
    par[2 * r] = lo;
    par[2 * r + 1] = hi > lo ? (double)B / (hi - lo) : 0.0;
  }
}

__global__ void k_mis_zero(unsigned* __restrict__ c, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

// Block (x, y): rows [x * chunk, (x + 1) * chunk) of the features [y * G, y * G + G).
// counts[j][a][b] += #{i : bin(F[j][i]) = a, bin(y[i]) = b}.
template <typename T>
__global__ void __launch_bounds__(kMisThreads)
k_mis_joint(const T* __restrict__ F, const T* __restrict__ y, long long N, int d, int B, int G,
            long long chunk, const double* __restrict__ par, unsigned* __restrict__ counts) {
  extern __shared__ unsigned h[];
  const int j0 = blockIdx.y * G;
  const int g = min(G, d - j0);
  const int BB = B * B;
  for (int k = threadIdx.x; k < g * BB; k += kMisThreads) h[k] = 0u;
  __syncthreads();
  const long long i0 = (long long)blockIdx.x * chunk;
  const long long i1 = min(N, i0 + chunk);
  const double ylo = par[2 * d], ys = par[2 * d + 1];
  for (long long i = i0 + threadIdx.x; i < i1; i += kMisThreads) {
    const int b = mis_bin((double)y[i], ylo, ys, B);
    for (int c = 0; c < g; ++c) {
      const int j = j0 + c;
      const int a = mis_bin((double)F[(size_t)j * N + i], par[2 * j], par[2 * j + 1], B);
      atomicAdd(&h[c * BB + a * B + b], 1u);
    }
  }
  __syncthreads();
  unsigned* out = counts + (size_t)j0 * BB;
  for (int k = threadIdx.x; k < g * BB; k += kMisThreads)
    if (h[k]) atomicAdd(&out[k], h[k]);
}

// One block per feature: marginals, then sum over the non-empty cells of
// (n_ab / N) log(N n_ab / (n_a n_b)) in a fixed order.
__global__ void __launch_bounds__(kMisThreads)
k_mis_score(const unsigned* __restrict__ counts, int B, long long N, double* __restrict__ score) {
  __shared__ double na[64], nb[64], sh[kMisThreads];
  const int j = blockIdx.x, t = threadIdx.x, BB = B * B;
  const unsigned* c = counts + (size_t)j * BB;
  if (t < B) {
    unsigned long long ra = 0, cb = 0;
    for (int k = 0; k < B; ++k) {
      ra += c[t * B + k];
      cb += c[k * B + t];
    }
    na[t] = (double)ra;
    nb[t] = (double)cb;
  }
  __syncthreads();
  const double n = (double)N;
  double acc = 0.0;
  for (int k = t; k < BB; k += kMisThreads) {
    const unsigned v = c[k];
    if (v) {
      const double x = (double)v;
      acc += x / n * log(n * x / (na[k / B] * nb[k % B]));
    }
  }
  acc = block_reduce(acc, OpAdd(), sh);
  if (t == 0) score[j] = acc;
}

// The three stages on caller-provided scratch: par [2 (d + 1)] doubles, counts [d B^2].
template <typename T>
void mis_launch(const T* F, long long N, int d, const T* y, int B, double* scores, double* par,
                unsigned* counts, hipStream_t s) {
  const int BB = B * B;
  const int G = std::max(1, std::min(d, kMisLds / (4 * BB)));
  const int ngroups = (d + G - 1) / G;
  const long long max_rb = std::max(1LL, (N + 1023) / 1024);
  const long long nrb = std::min<long long>(max_rb, std::max(1, 2048 / ngroups));
  const long long chunk = (N + nrb - 1) / nrb;
  const long long ncount = (long long)d * BB;
  hipLaunchKernelGGL(k_mis_range<T>, dim3(d + 1), dim3(kMisThreads), 0, s, F, y, N, d, B, par);
  hipLaunchKernelGGL(k_mis_zero, dim3((unsigned)((ncount + 255) / 256)), dim3(256), 0, s,
                     counts, ncount);
  hipLaunchKernelGGL(k_mis_joint<T>, dim3((unsigned)((N + chunk - 1) / chunk), ngroups),
                     dim3(kMisThreads), (size_t)G * BB * sizeof(unsigned), s, F, y, N, d, B, G,
                     chunk, par, counts);
  hipLaunchKernelGGL(k_mis_score, dim3(d), dim3(kMisThreads), 0, s, counts, B, N, scores);
  NLD_HIP(hipGetLastError());
}

template <typename T>
void mis_t(const T* F, long long N, int d, const T* y, int B, double* scores, hipStream_t s) {
  double* par = nullptr;
  unsigned* counts = nullptr;
  NLD_HIP(hipMallocAsync((void**)&par, sizeof(double) * 2 * (d + 1), s));
  NLD_HIP(hipMallocAsync((void**)&counts, sizeof(unsigned) * (size_t)d * B * B, s));
  mis_launch<T>(F, N, d, y, B, scores, par, counts, s);
  NLD_HIP(hipFreeAsync(counts, s));
  NLD_HIP(hipFreeAsync(par, s));
}

// ---------------------------------------------------------------------------- no allocation
// Scratch of mis_scores_noalloc: the range table (4 (d + 1) words) followed by the joint
// histograms (d B^2 words) in one file-scope device array, which every device the library runs
// on holds until the process ends.  In host code `scratch` names a host-side stand-in, not the
// device copy: its device address is looked up once per device (scratch_on_device) and only
// that address is handed to kernels.
constexpr long long kMisScratchWords = 1LL << 20;   // 4 MiB
static __device__ __align__(256) unsigned scratch[kMisScratchWords];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned* g_scratch_dev[kMaxScratchDevices] = {};

unsigned* scratch_on_device() {
  int dev = 0;
  NLD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) throw HipError{e, "hipGetSymbolAddress(scratch)"};
    g_scratch_dev[dev] = static_cast<unsigned*>(p);
  }
  return g_scratch_dev[dev];
}

}  // namespace

long long mis_noalloc_words(int d, int bins) {
  return 4LL * (d + 1) + (long long)d * bins * bins;
}

long long mis_noalloc_capacity() { return kMisScratchWords; }

void launch_mis_noalloc(const void* F, long long N, int d, const void* y, nld_prec prec, int bins,
                        double* scores, hipStream_t s) {
  if (bins < 2 || bins > 64) throw std::invalid_argument("bins out of range");
  if (mis_noalloc_words(d, bins) > kMisScratchWords)
    throw std::invalid_argument("4 (d + 1) + d bins^2 exceeds the static scratch of 1048576 words");
  unsigned* base = scratch_on_device();
  double* par = reinterpret_cast<double*>(base);                 // 256-byte aligned
  unsigned* counts = base + 4LL * (d + 1);
  if (prec == NLD_FP32)
    mis_launch<float>((const float*)F, N, d, (const float*)y, bins, scores, par, counts, s);
  else
    mis_launch<double>((const double*)F, N, d, (const double*)y, bins, scores, par, counts, s);
}

int mis_default_bins(long long N) {
  int B = 1;
  while ((long long)(B + 1) * (B + 1) * (B + 1) <= N / 4) ++B;
  return std::min(64, std::max(4, B));
}

void launch_mis(const void* F, long long N, int d, const void* y, nld_prec prec, int bins,
                double* scores, hipStream_t s) {
  if (bins < 2 || bins > 64) throw std::invalid_argument("bins out of range");
  if (prec == NLD_FP32)
    mis_t<float>((const float*)F, N, d, (const float*)y, bins, scores, s);
  else
    mis_t<double>((const double*)F, N, d, (const double*)y, bins, scores, s);
}

}  // namespace nld
