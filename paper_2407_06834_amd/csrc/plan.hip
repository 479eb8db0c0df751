// Plan construction: features, per-window torus scaling, grid coordinates, stable radix sort
// of the nodes by grid tile, work schedules.  (Paper Sec. 3: NFFT fast Gauss summation; the
// parameter choices follow the NFFT literature the paper cites and are listed in the design
// notes of the repository.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>

#include "nld_internal.h"

namespace nld {

namespace {

constexpr int kTileChunk = kMaxChunk;   // nodes per spreading / gathering workgroup (default)
int tile_chunk() {
  const char* e = std::getenv("NLD_TILE_CHUNK");
  return e ? std::max(64, std::min(kMaxChunk, std::atoi(e))) : kTileChunk;
}
constexpr int kMaxCellBits = 16;     // sort key = global tile << cell_bits | cell within the tile

template <typename T>
__global__ void k_features(const T* __restrict__ img, int n1, int n2, int rho, int with_pos,
                           T* __restrict__ F) {
  // One pixel per lane, all its features: x covers a row's columns, y strides over the rows;
  // each feature row's stores are contiguous across the wavefront.
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n2) return;
  const long long N = (long long)n1 * n2;
  const int P = 2 * rho + 1;
  for (int row = blockIdx.y; row < n1; row += gridDim.y) {
    T* out = F + (long long)row * n2 + col;
    if (with_pos) {
      out[0] = (T)((double)col / (double)n2);
      out[N] = (T)((double)row / (double)n1);
      out += 2 * N;
    }
    for (int a = 0; a < P; ++a) {
      const int r = row + a - rho;
      const bool rin = r >= 0 && r < n1;
      for (int b = 0; b < P; ++b) {
        const int c = col + b - rho;
        *out = (rin && c >= 0 && c < n2) ? img[(long long)r * n2 + c] : (T)0;
        out += N;
      }
    }
  }
}

// Per-block min / max of selected feature rows; partials [ncol][nblk][2].
template <typename T>
__global__ void k_minmax(const T* __restrict__ F, long long N, const int* __restrict__ cols,
                         double* __restrict__ part) {
  const int c = blockIdx.y;
  const T* x = F + (long long)cols[c] * N;
  // Min and max are taken in T (exact; the conversion to double is monotonic), eight
  // independent loads in flight per lane.
  T lo = (T)INFINITY, hi = (T)-INFINITY;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i + 7 * stride < N; i += 8 * stride) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[i + u * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      lo = fmin(lo, v[u]);
      hi = fmax(hi, v[u]);
    }
  }
  for (; i < N; i += stride) {
    lo = fmin(lo, x[i]);
    hi = fmax(hi, x[i]);
  }
  __shared__ double slo[256], shi[256];
  slo[threadIdx.x] = (double)lo;
  shi[threadIdx.x] = (double)hi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((long long)c * gridDim.x + blockIdx.x) * 2 + 0] = slo[0];
    part[((long long)c * gridDim.x + blockIdx.x) * 2 + 1] = shi[0];
  }
}

struct CoordParams {
  int feat[3];        // feature row per internal dimension (-1: unused)
  double centre[3], scale[3];
  int n[3], m;
  int ts[3], nts[3];
  unsigned tile_off;
  int cell_bits;      // bits of the cell-within-tile part of the sort key (same for all windows)
};

__device__ inline int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Grid coordinates of every (window, node): packed base cell and fractional offsets in one
// entry (16 bytes in FP32, 32 in FP64, so that the permutation into sorted order reads one
// cache line per entry), and the sort key within the window: tile << cell_bits | cell.
template <typename T> struct CoordEntry;
template <> struct __attribute__((aligned(16))) CoordEntry<float> { unsigned base; float f[3]; };
template <> struct __attribute__((aligned(16))) CoordEntry<double> { unsigned base, pad; double f[3]; };

// Grid: y is the window (its parameters are wave-uniform), x strides over the nodes.  Also
// writes the identity permutation that the sort carries along (val = flat entry index).
template <typename T>
__global__ void k_coords(const T* __restrict__ F, long long N,
                         const CoordParams* __restrict__ cp, CoordEntry<T>* __restrict__ ent,
                         unsigned* __restrict__ key, unsigned* __restrict__ val) {
  const int l = blockIdx.y;
  const CoordParams p = cp[l];
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < N;
       j += (long long)gridDim.x * blockDim.x) {
    const long long idx = (long long)l * N + j;
    int b[3];
    CoordEntry<T> e{};
    for (int dd = 0; dd < 3; ++dd) {
      T fr = (T)0;
      int bi = 0;
      if (p.feat[dd] >= 0) {
        const double x = (double)F[(long long)p.feat[dd] * N + j];
        const double xt = __dmul_rn(x - p.centre[dd], p.scale[dd]);
        const double u = __dadd_rn(__dmul_rn((double)p.n[dd], xt), 0.5 * p.n[dd]);
        const double fl = floor(u);
        bi = (int)fl;
        fr = (T)(u - fl);
        if (fr >= (T)1) { fr = (T)0; bi += 1; }
        bi &= p.n[dd] - 1;                       // periodic wrap (n is a power of two)
      }
      b[dd] = bi;
      e.f[dd] = fr;
    }
    e.base = (unsigned)b[0] | ((unsigned)b[1] << 8) | ((unsigned)b[2] << 16);
    ent[idx] = e;
    // tile and cell within the tile (tile extents are powers of two)
    const int l0 = __builtin_ctz(p.ts[0]), l1 = __builtin_ctz(p.ts[1]), l2 = __builtin_ctz(p.ts[2]);
    const int g = ((b[0] >> l0) * p.nts[1] + (b[1] >> l1)) * p.nts[2] + (b[2] >> l2);
    const int lc = ((b[0] & (p.ts[0] - 1)) * p.ts[1] + (b[1] & (p.ts[1] - 1))) * p.ts[2] +
                   (b[2] & (p.ts[2] - 1));
    key[idx] = ((unsigned)g << p.cell_bits) | (unsigned)lc;   // key within the window
    val[idx] = (unsigned)idx;
  }
}

// First position of every global tile (0..ntiles) in the sorted entries: window l's entries
// occupy [l N, (l + 1) N), sorted by their key within the window (tile << cell_bits | cell), so
// tile k of window l starts at the lower bound of (k - tile_off) << cell_bits in that segment.
__global__ void k_key_offsets(const unsigned* __restrict__ keys, long long N, int L,
                              const CoordParams* __restrict__ cp, int ntiles, int cell_bits,
                              unsigned* __restrict__ off) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > ntiles) return;
  if (k == ntiles) {
    off[k] = (unsigned)(N * L);
    return;
  }
  int l = 0;
  while (l + 1 < L && (int)cp[l + 1].tile_off <= k) ++l;
  const unsigned long long target = (unsigned long long)(k - (int)cp[l].tile_off) << cell_bits;
  long long lo = (long long)l * N, hi = (long long)(l + 1) * N;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if ((unsigned long long)keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  off[k] = (unsigned)lo;
}

// ---------------------------------------------------------------- exclusive scan (uint32)
constexpr int kScanThreads = 256, kScanPer = 8, kScanBlock = kScanThreads * kScanPer;

__global__ void k_scan_local(unsigned* __restrict__ data, long long n, unsigned* __restrict__ sums) {
  __shared__ unsigned s[kScanThreads];
  const long long b0 = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanPer;
  unsigned v[kScanPer];
  unsigned tsum = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (b0 + k < n) ? data[b0 + k] : 0u;
    tsum += v[k];
  }
  s[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const unsigned add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  unsigned run = s[threadIdx.x] - tsum;   // exclusive prefix of this thread
  for (int k = 0; k < kScanPer; ++k) {
    if (b0 + k < n) data[b0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[kScanThreads - 1];
}

__global__ void k_scan_add(unsigned* __restrict__ data, long long n, const unsigned* __restrict__ sums) {
  const unsigned add = sums[blockIdx.x];
  const long long b0 = (long long)blockIdx.x * kScanBlock;
  for (int k = threadIdx.x; k < kScanBlock; k += kScanThreads)
    if (b0 + k < n) data[b0 + k] += add;
}

// Device buffers of plans come from a per-device cache.  Plans are built and released once per
// kernel width on the solver's path, a plan holds about 45 buffers and its build some 20
// temporaries, and hipMallocAsync / hipFreeAsync cost tens of microseconds of host time each.
// A released buffer enters the cache once its stream has been synchronised (dev_synced); a
// request takes the smallest cached buffer of at least its size and at most 5/4 of it plus
// 64 KiB.  Beyond kDevCacheCap bytes per device, released buffers are freed instead.
namespace {
constexpr size_t kDevCacheCap = 8ULL << 30;
constexpr int kMaxDevices = 64;
std::mutex g_dev_mu;
std::multimap<size_t, void*> g_dev_free[kMaxDevices];            // bytes -> cached buffer
std::map<void*, std::pair<int, size_t>> g_dev_owner;              // buffer -> (device, bytes)
std::map<hipStream_t, std::vector<void*>> g_dev_pending;          // released, not yet synced
size_t g_dev_cached[kMaxDevices] = {};

int current_device() {
  int dev = 0;
  NLD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device index out of range");
  return dev;
}

void* dev_get(size_t bytes, hipStream_t s) {
  const int dev = current_device();
  {
    std::lock_guard<std::mutex> lock(g_dev_mu);
    auto& fl = g_dev_free[dev];
    auto it = fl.lower_bound(bytes);
    if (it != fl.end() && it->first <= bytes + bytes / 4 + (64 << 10)) {
      void* p = it->second;
      g_dev_cached[dev] -= it->first;
      fl.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, s);
  if (e != hipSuccess) throw HipError{e, "hipMallocAsync"};
  std::lock_guard<std::mutex> lock(g_dev_mu);
  g_dev_owner[p] = {dev, bytes};
  return p;
}

// p is idle (its stream has been synchronised): keep it for a later request, or free it
void dev_release_idle(void* p) {
  if (!p) return;
  std::unique_lock<std::mutex> lock(g_dev_mu);
  auto it = g_dev_owner.find(p);
  if (it == g_dev_owner.end()) return;
  const int dev = it->second.first;
  const size_t bytes = it->second.second;
  if (g_dev_cached[dev] + bytes <= kDevCacheCap) {
    g_dev_free[dev].emplace(bytes, p);
    g_dev_cached[dev] += bytes;
    return;
  }
  g_dev_owner.erase(it);
  lock.unlock();
  (void)hipFree(p);
}
}  // namespace

// the buffers released on stream s since its last synchronisation enter the cache
void dev_synced(hipStream_t s) {
  std::vector<void*> done;
  {
    std::lock_guard<std::mutex> lock(g_dev_mu);
    auto it = g_dev_pending.find(s);
    if (it == g_dev_pending.end()) return;
    done.swap(it->second);
    g_dev_pending.erase(it);
  }
  for (void* p : done) dev_release_idle(p);
}

template <typename P>
P* dalloc(long long count, hipStream_t s) {
  if (count <= 0) count = 1;
  return (P*)dev_get((size_t)count * sizeof(P), s);
}
// released in stream order: reusable after the stream's next synchronisation (dev_synced)
inline void dfree(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_dev_mu);
  g_dev_pending[s].push_back(p);
}

// Segment i of a staged blob: bytes at blob + off go to dst.
struct UploadSeg {
  unsigned long long dst, off, bytes;
};

// Copies every segment of the blob to its buffer (grid x: segment, y: strided part of it);
// 16-byte words where the destination, offset and length allow, bytes otherwise.
__global__ void k_scatter_copy(const unsigned char* __restrict__ blob,
                               const UploadSeg* __restrict__ segs) {
  const UploadSeg g = segs[blockIdx.x];
  unsigned char* dst = reinterpret_cast<unsigned char*>(g.dst);
  const unsigned char* src = blob + g.off;
  const unsigned long long step = (unsigned long long)gridDim.y * blockDim.x;
  const unsigned long long t0 = (unsigned long long)blockIdx.y * blockDim.x + threadIdx.x;
  if (((g.dst | g.off) & 15ull) == 0) {
    const unsigned long long nw = g.bytes / 16;
    for (unsigned long long i = t0; i < nw; i += step)
      reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (unsigned long long i = nw * 16 + t0; i < g.bytes; i += step) dst[i] = src[i];
  } else {
    for (unsigned long long i = t0; i < g.bytes; i += step) dst[i] = src[i];
  }
}

// Host tables reach the device through pinned staging blocks: a copy from pageable memory holds
// the host until it has finished, tens of microseconds each.  The blocks return to the pool at
// the plan's next stream synchronisation (staging_done).
static void upload(Plan& P, void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (P.defer_uploads) {
    const size_t off = (P.pending_blob.size() + 15) & ~(size_t)15;
    P.pending_blob.resize(off + bytes);
    std::memcpy(P.pending_blob.data() + off, src, bytes);
    P.pending_dst.push_back(dst);
    P.pending_off.push_back(off);
    P.pending_bytes.push_back(bytes);
    return;
  }
  void* p = pinned_get(bytes, false);
  P.staging.push_back(p);
  std::memcpy(p, src, bytes);
  NLD_HIP(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s));
}
static void staging_done(Plan& P, hipStream_t s) {   // call only after synchronising s
  for (void* p : P.staging) pinned_put(p);
  P.staging.clear();
  dev_synced(s);
}

// The deferred tables: one host-to-device copy of the blob and its segment table, then one
// kernel that copies every segment to its buffer.
static void flush_uploads(Plan& P, hipStream_t s) {
  P.defer_uploads = false;
  const size_t nseg = P.pending_dst.size();
  if (nseg > 0) {
    std::vector<UploadSeg> seg(nseg);
    for (size_t i = 0; i < nseg; ++i)
      seg[i] = UploadSeg{(unsigned long long)(uintptr_t)P.pending_dst[i], P.pending_off[i],
                         P.pending_bytes[i]};
    const size_t toff = (P.pending_blob.size() + 15) & ~(size_t)15;
    const size_t total = toff + nseg * sizeof(UploadSeg);
    P.pending_blob.resize(total);
    std::memcpy(P.pending_blob.data() + toff, seg.data(), nseg * sizeof(UploadSeg));
    unsigned char* dblob = dalloc<unsigned char>((long long)total, s);
    upload(P, dblob, P.pending_blob.data(), total, s);
    hipLaunchKernelGGL(k_scatter_copy, dim3((unsigned)nseg, 16), dim3(256), 0, s,
                       (const unsigned char*)dblob, (const UploadSeg*)(dblob + toff));
    NLD_HIP(hipGetLastError());
    dfree(dblob, s);
  }
  P.pending_blob.clear();
  P.pending_dst.clear();
  P.pending_off.clear();
  P.pending_bytes.clear();
}

void exclusive_scan(unsigned* data, long long n, hipStream_t s) {
  if (n <= 0) return;
  const long long nb = (n + kScanBlock - 1) / kScanBlock;
  unsigned* sums = dalloc<unsigned>(nb, s);
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
  NLD_HIP(hipGetLastError());
  if (nb > 1) {
    exclusive_scan(sums, nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    NLD_HIP(hipGetLastError());
  }
  dfree(sums, s);
}

// ---------------------------------------------------------------- stable LSD radix sort
// Segments of equal length (one per window) sorted separately, 7-bit digits, blocks of 4
// wavefronts and 4096 items that never straddle a segment.  A wavefront ranks its 1024 items in
// order with ballots (equal keys keep their input order), the block places its items in digit
// order in LDS and writes every digit's run to its global position with consecutive threads on
// consecutive positions.  The block offsets come from one exclusive scan over (segment, digit,
// block), so every segment stays in place.
constexpr int kSortThreads = 256, kSortPer = 16, kSortItems = kSortThreads * kSortPer;
constexpr int kSortWaveItems = kSortItems / (kSortThreads / 64);
constexpr int kSortBits = 7, kSortBuckets = 1 << kSortBits;

__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const unsigned* __restrict__ keys, long long seglen, int bps, int shift,
             unsigned* __restrict__ hist) {
  __shared__ unsigned h[kSortBuckets];
  if (threadIdx.x < kSortBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const int seg = blockIdx.x / bps, lb = blockIdx.x - seg * bps;
  const long long b0 = (long long)seg * seglen + (long long)lb * kSortItems;
  const long long e = (long long)seg * seglen + min(seglen, (long long)(lb + 1) * kSortItems);
  for (int r = 0; r < kSortPer; ++r) {
    const long long i = b0 + r * kSortThreads + threadIdx.x;
    if (i < e) atomicAdd(&h[(keys[i] >> shift) & (kSortBuckets - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kSortBuckets)
    hist[((long long)seg * kSortBuckets + threadIdx.x) * bps + lb] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const unsigned* __restrict__ kin, const unsigned* __restrict__ vin,
                unsigned* __restrict__ kout, unsigned* __restrict__ vout, long long seglen,
                int bps, int shift, const unsigned* __restrict__ offs) {
  constexpr int kWaves = kSortThreads / 64;
  static_assert(kSortBuckets % 64 == 0 && kSortBuckets <= kSortThreads, "whole wavefronts of digits");
  __shared__ unsigned wcnt[kWaves][kSortBuckets];   // per-wavefront counts, then their prefixes
  __shared__ unsigned lstart[kSortBuckets];         // first block-local position of every digit
  __shared__ unsigned goff[kSortBuckets];           // first global position of every digit
  __shared__ unsigned wsum[kWaves];
  __shared__ unsigned skey[kSortItems], sval[kSortItems];
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int seg = blockIdx.x / bps, lb = blockIdx.x - seg * bps;
  const long long s0 = (long long)seg * seglen;
  const long long e = s0 + min(seglen, (long long)(lb + 1) * kSortItems);
  for (int d = t; d < kWaves * kSortBuckets; d += kSortThreads) (&wcnt[0][0])[d] = 0u;
  if (t < kSortBuckets) goff[t] = offs[((long long)seg * kSortBuckets + t) * bps + lb];
  __syncthreads();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const long long b0 = s0 + (long long)lb * kSortItems + (long long)wv * kSortWaveItems;
  unsigned key[kSortPer], val[kSortPer], pos[kSortPer];   // pos: digit << 16 | rank in wavefront
  for (int r = 0; r < kSortPer; ++r) {
    const long long i = b0 + r * 64 + lane;
    const bool valid = i < e;
    const unsigned k = valid ? kin[i] : 0u;
    const unsigned dg = (k >> shift) & (kSortBuckets - 1);
    unsigned long long mask = __ballot(valid);
    for (int bit = 0; bit < kSortBits; ++bit) {
      const bool set = (dg >> bit) & 1u;
      const unsigned long long bal = __ballot(set);
      mask &= set ? bal : ~bal;
    }
    const unsigned rank = (unsigned)__popcll(mask & below);
    const unsigned group = (unsigned)__popcll(mask);
    // every lane reads its digit's count before the last lane of each group stores the new one
    // (LDS operations of a wavefront execute in order)
    const unsigned base = wcnt[wv][dg];
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == group - 1) wcnt[wv][dg] = base + group;
    __builtin_amdgcn_wave_barrier();
    key[r] = k;
    val[r] = valid ? vin[i] : 0u;
    pos[r] = valid ? ((dg << 16) | (base + rank)) : 0xffffffffu;
  }
  __syncthreads();
  // digit t: prefixes over the wavefronts and the block-local start (exclusive scan of totals)
  // (the digits are whole wavefronts, so the branches below are uniform per wavefront)
  unsigned c[kWaves], tot = 0, inc = 0;
  if (t < kSortBuckets) {
    for (int w = 0; w < kWaves; ++w) {
      c[w] = tot;
      tot += wcnt[w][t];
    }
    inc = tot;
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
  }
  __syncthreads();
  if (t < kSortBuckets) {
    unsigned before = 0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    lstart[t] = before + inc - tot;
    for (int w = 0; w < kWaves; ++w) wcnt[w][t] = c[w];
  }
  __syncthreads();
  for (int r = 0; r < kSortPer; ++r) {
    if (pos[r] == 0xffffffffu) continue;
    const unsigned dg = pos[r] >> 16;
    const unsigned q = lstart[dg] + wcnt[wv][dg] + (pos[r] & 0xffffu);
    skey[q] = key[r];
    sval[q] = val[r];
  }
  __syncthreads();
  const int nvalid = (int)(e - (s0 + (long long)lb * kSortItems));
  for (int r = 0; r < kSortPer; ++r) {
    const int q = r * kSortThreads + t;
    if (q >= nvalid) break;
    const unsigned k = skey[q];
    const unsigned dg = (k >> shift) & (kSortBuckets - 1);
    const unsigned dst = goff[dg] + (unsigned)q - lstart[dg];
    kout[dst] = k;
    vout[dst] = sval[q];
  }
}

// Sorts each of nseg consecutive segments of seglen (key, value) pairs by the low key_bits bits
// of the keys, stably.  keys / vals are replaced by the buffers that hold the result (the other
// pair is returned to the buffer cache).
void radix_sort_segments(unsigned*& keys, unsigned*& vals, int nseg, long long seglen,
                         int key_bits, hipStream_t s) {
  if ((long long)nseg * seglen <= 1) return;
  const int bps = (int)((seglen + kSortItems - 1) / kSortItems);
  const int nblk = nseg * bps;
  unsigned* k2 = dalloc<unsigned>((long long)nseg * seglen, s);
  unsigned* v2 = dalloc<unsigned>((long long)nseg * seglen, s);
  unsigned* hist = dalloc<unsigned>((long long)kSortBuckets * nblk, s);
  unsigned *ka = keys, *va = vals, *kb = k2, *vb = v2;
  const int passes = std::max(1, (key_bits + kSortBits - 1) / kSortBits);
  for (int pss = 0; pss < passes; ++pss) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, s, ka, seglen, bps,
                       kSortBits * pss, hist);
    NLD_HIP(hipGetLastError());
    exclusive_scan(hist, (long long)kSortBuckets * nblk, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, s, ka, va, kb, vb,
                       seglen, bps, kSortBits * pss, hist);
    NLD_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // ka / va hold the result; kb / vb the other pair
  keys = ka;
  vals = va;
  dfree(kb, s);
  dfree(vb, s);
  dfree(hist, s);
}

// Copy the coordinates of sorted entries: out[e] = in[(window of e, node of e)].  Every
// window's entries are sorted within their own segment [l N, (l + 1) N), so the window of a
// sorted entry is its segment: grid y is the window, x strides over the segment.
template <typename T>
__global__ void k_gather_entries(const unsigned* __restrict__ vals, long long N,
                                 const CoordEntry<T>* __restrict__ ent, int* __restrict__ out_idx,
                                 unsigned* __restrict__ out_base, T* __restrict__ out_frac,
                                 long long out_stride) {
  const long long seg = (long long)blockIdx.y * N;
  for (long long e = seg + blockIdx.x * (long long)blockDim.x + threadIdx.x; e < seg + N;
       e += (long long)gridDim.x * blockDim.x) {
    const unsigned flat = vals[e];
    const long long j = (long long)flat - seg;
    const CoordEntry<T> c = ent[flat];
    out_idx[e] = (int)j;
    out_base[e] = c.base;
    for (int dd = 0; dd < 3; ++dd) out_frac[dd * out_stride + e] = c.f[dd];
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, long long n, T val) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = val;
}

inline unsigned grid_for(long long n, int threads = 256) {
  long long b = (n + threads - 1) / threads;
  return (unsigned)std::max<long long>(1, std::min<long long>(b, 65536));
}

// ---------------------------------------------------------------- host math for the plan
double compression(double sigma, double R, int M) {
  const double q = 2.0 * M_PI * M * sigma * sigma / (R * R);
  return (std::sqrt(1.0 + q) - 1.0) / q;
}

// Fourier factor carried by the spreading grid for frequency k (scaled Kaiser-Bessel window:
// pi m I0(m sqrt(b^2 - (2 pi k / n)^2)) / sinh(b m)).
double kb_fourier(double k, int n, int m, double b) {
  const double x = m * std::sqrt(b * b - std::pow(2.0 * M_PI * k / n, 2));
  return M_PI * m * std::cyl_bessel_i(0.0, x) / std::sinh(b * m);
}

// Scaled Kaiser-Bessel window psi(delta) = m sinh(b z) / (z sinh(b m)), z = sqrt(m^2 - delta^2).
double kb_psi_host(double delta, int m, double b) {
  const double z = std::sqrt(std::max(m * (double)m - delta * delta, 0.0));
  const double den = -std::expm1(-2.0 * b * m);
  if (z > 0.0) return (m / z) * std::exp(b * (z - m)) * (-std::expm1(-2.0 * b * z)) / den;
  return 2.0 * b * m * std::exp(-b * m) / den;
}

// Per-tap polynomial in x = 2 fr - 1 (fr in [0, 1)) for tap i at distance fr + m - 1 - i:
// Chebyshev interpolation at deg + 1 nodes, converted to monomial coefficients.
// Returns the coefficients [2m][deg + 1] and the max abs error on a fine test grid.
std::vector<double> fit_window(int m, double b, int deg, double* max_err) {
  const int W = 2 * m, K = deg + 1;
  std::vector<double> out((size_t)W * K, 0.0);
  double err = 0.0;
  for (int i = 0; i < W; ++i) {
    std::vector<double> y(K), c(K, 0.0);
    for (int j = 0; j < K; ++j) {
      const double x = std::cos(M_PI * (j + 0.5) / K);
      y[j] = kb_psi_host(0.5 * (x + 1.0) + m - 1 - i, m, b);
    }
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int j = 0; j < K; ++j) acc += y[j] * std::cos(M_PI * k * (j + 0.5) / K);
      c[k] = acc * 2.0 / K;
    }
    c[0] *= 0.5;
    std::vector<double> tprev(K, 0.0), tcur(K, 0.0), mono(K, 0.0);
    tprev[0] = 1.0;                       // T_0
    if (K > 1) tcur[1] = 1.0;             // T_1
    for (int q = 0; q < K; ++q) mono[q] += c[0] * tprev[q];
    if (K > 1)
      for (int q = 0; q < K; ++q) mono[q] += c[1] * tcur[q];
    for (int k = 2; k < K; ++k) {
      std::vector<double> tn(K, 0.0);
      for (int q = 0; q < K; ++q) {
        if (q > 0) tn[q] += 2.0 * tcur[q - 1];
        tn[q] -= tprev[q];
      }
      for (int q = 0; q < K; ++q) mono[q] += c[k] * tn[q];
      tprev = tcur;
      tcur = tn;
    }
    for (int q = 0; q < K; ++q) out[(size_t)i * K + q] = mono[q];
    for (int s = 0; s <= 256; ++s) {
      const double fr = s / 256.0, x = 2.0 * fr - 1.0;
      double v = 0.0;
      for (int q = K - 1; q >= 0; --q) v = v * x + mono[q];
      err = std::max(err, std::abs(v - kb_psi_host(fr + m - 1 - i, m, b)));
    }
  }
  *max_err = err;
  return out;
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Per-entry error estimate of the band-limited periodic kernel in one dimension.
double dim_error(double sigma, double R, int M) {
  const double a = compression(sigma, R, M);
  const double st = 2.0 * a * sigma / R;
  return std::exp(-std::pow(M_PI * st * M / 2.0, 2));
}

}  // namespace

void* plan_buffer(size_t bytes, hipStream_t s) { return dev_get(std::max<size_t>(1, bytes), s); }

void launch_features(const void* img, int n1, int n2, int rho, int with_pos, nld_prec prec,
                     void* F, hipStream_t s) {
  const dim3 grid((unsigned)((n2 + 255) / 256), (unsigned)std::min(n1, 1024));
  if (prec == NLD_FP32)
    hipLaunchKernelGGL(k_features<float>, grid, dim3(256), 0, s, (const float*)img, n1, n2, rho,
                       with_pos, (float*)F);
  else
    hipLaunchKernelGGL(k_features<double>, grid, dim3(256), 0, s, (const double*)img, n1, n2,
                       rho, with_pos, (double*)F);
  NLD_HIP(hipGetLastError());
}

// Smallest bandwidth from a fixed ladder whose per-entry error estimate is below 1e-2 * tol in
// every dimension of the window (the largest candidate if none is).
static int auto_bandwidth(double sigma, const std::vector<double>& R, double tol) {
  static const int cand[] = {16, 24, 32, 48, 64, 96, 128};
  for (int c : cand) {
    double e = 0.0;
    for (double r : R) e = std::max(e, dim_error(sigma, r, c));
    if (e <= 1e-2 * tol) return c;
  }
  return 128;
}

// Fourier multipliers of every window from the scaled widths P.sig_t: per internal dimension
// d the periodic Gaussian coefficients over the squared Kaiser-Bessel factor on |k| <= M/2 - 1
// (zero elsewhere), and for the sigma derivative the same tables with dimension d's factor
// multiplied by (1 - 2 pi^2 st_d^2 k^2), so that the sum over d of the three products gives
// the coefficients b_k (t - 2 pi^2 sum_d st_d^2 k_d^2) of sigma dK/dsigma.
template <typename T>
static void upload_tables(Plan& P, std::vector<T>& coef_all, std::vector<T>& coef_dv_all,
                          hipStream_t s) {
  const int L = P.L, n_max = P.n_max;
  P.coef_host.assign(L, {});
  // the window's Fourier factor depends on (n, m, b) only (b fixes M / n): evaluated once per
  // distinct triple
  std::vector<double> ph_tab;
  int ph_n = -1, ph_m = -1;
  double ph_b = 0.0;
  for (int l = 0; l < L; ++l) {
    const WinDev& w = P.wins[l];
    const int n = P.info[l].grid, M = P.info[l].bandwidth;
    if (n != ph_n || w.m != ph_m || w.b != ph_b) {
      ph_n = n;
      ph_m = w.m;
      ph_b = w.b;
      ph_tab.assign(n, 0.0);
      for (int q = 0; q < n; ++q) {
        const int kf = (q < n / 2) ? q : q - n;
        if (std::abs(kf) <= M / 2 - 1) ph_tab[q] = kb_fourier(kf, n, w.m, w.b);
      }
    }
    std::vector<double> coef(3LL * n, 0.0);
    for (int dd = 0; dd < 3; ++dd) {
      if (w.n[dd] == 1) continue;
      const double st = P.sig_t[3 * (size_t)l + dd];
      for (int q = 0; q < n; ++q) {
        const int kf = (q < n / 2) ? q : q - n;
        if (std::abs(kf) <= M / 2 - 1) {
          const double bh = std::sqrt(M_PI) * st * std::exp(-std::pow(M_PI * st * kf, 2));
          const double ph = ph_tab[q];
          coef[(long long)dd * n + q] = bh / (ph * ph);
        }
      }
    }
    P.coef_host[l] = std::move(coef);
  }
  coef_all.assign(3LL * n_max * L, (T)0);
  for (int l = 0; l < L; ++l) {
    const int n = P.info[l].grid;
    for (int dd = 0; dd < 3; ++dd)
      for (int q = 0; q < n; ++q)
        coef_all[((long long)l * 3 + dd) * n_max + q] = (T)P.coef_host[l][(long long)dd * n + q];
  }
  if (!P.coef) P.coef = dalloc<T>((long long)coef_all.size(), s);
  upload(P, P.coef, coef_all.data(), coef_all.size() * sizeof(T), s);
  for (int l = 0; l < L; ++l) {
    P.wins[l].coef = (const T*)P.coef + (long long)l * 3 * n_max;
    P.wins[l].n_max = n_max;
  }
  coef_dv_all.assign(3 * coef_all.size(), (T)0);
  for (int d = 0; d < 3; ++d) {
    P.dv_used[d] = false;
    for (int l = 0; l < L; ++l) {
      const int n = P.info[l].grid;
      if (P.wins[l].n[d] == 1 || P.wins[l].t == 0) continue;   // no dimension d: zero tables
      P.dv_used[d] = true;
      const double st = P.sig_t[3 * (size_t)l + d];
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < n; ++q) {
          double c = P.coef_host[l][(long long)a * n + q];
          if (a == d) {
            const int kf = (q < n / 2) ? q : q - n;
            c *= 1.0 - 2.0 * M_PI * M_PI * st * st * (double)kf * kf;
          }
          coef_dv_all[(size_t)d * coef_all.size() + ((size_t)l * 3 + a) * n_max + q] = (T)c;
        }
    }
  }
  if (!P.coef_dv) P.coef_dv = dalloc<T>((long long)coef_dv_all.size(), s);
  upload(P, P.coef_dv, coef_dv_all.data(), coef_dv_all.size() * sizeof(T), s);
}

// Device copies of the window descriptors: one with the kernel multipliers, and one per
// internal dimension with the sigma-derivative multipliers of that dimension.
template <typename T>
static void upload_windows(Plan& P, std::vector<WinDev> (&wins_dv)[3], hipStream_t s) {
  const int L = P.L;
  const size_t table = 3ULL * P.n_max * L;
  if (!P.d_wins) P.d_wins = dalloc<WinDev>(L, s);
  upload(P, P.d_wins, P.wins.data(), L * sizeof(WinDev), s);
  for (int d = 0; d < 3; ++d) {
    wins_dv[d] = P.wins;
    for (int l = 0; l < L; ++l)
      wins_dv[d][l].coef = (const T*)P.coef_dv + (size_t)d * table + (size_t)l * 3 * P.n_max;
    if (!P.d_wins_dv[d]) P.d_wins_dv[d] = dalloc<WinDev>(L, s);
    upload(P, P.d_wins_dv[d], wins_dv[d].data(), L * sizeof(WinDev), s);
  }
}

template <typename T>
static void build_plan_t(Plan& P, const void* features, hipStream_t s) {
  const long long N = P.N;
  const int L = P.L;
  // ---- 1. data range of every feature row used by a window
  std::vector<int> cols(P.win_feat);
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  const int ncol = (int)cols.size();
  const int nblk = (int)std::min<long long>(256, (N + 255) / 256);
  int* d_cols = dalloc<int>(ncol, s);
  double* d_part = dalloc<double>(2LL * ncol * nblk, s);
  upload(P, d_cols, cols.data(), ncol * sizeof(int), s);
  hipLaunchKernelGGL(k_minmax<T>, dim3(nblk, ncol), dim3(256), 0, s, (const T*)features, N, d_cols,
                     d_part);
  NLD_HIP(hipGetLastError());
  std::vector<double> part(2LL * ncol * nblk);
  NLD_HIP(hipMemcpyAsync(part.data(), d_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  NLD_HIP(hipStreamSynchronize(s));
  staging_done(P, s);
  dfree(d_cols, s);
  dfree(d_part, s);
  std::vector<double> lo(P.d, 0.0), hi(P.d, 0.0);
  for (int c = 0; c < ncol; ++c) {
    double a = INFINITY, b = -INFINITY;
    for (int k = 0; k < nblk; ++k) {
      a = std::min(a, part[(c * nblk + k) * 2]);
      b = std::max(b, part[(c * nblk + k) * 2 + 1]);
    }
    if (!std::isfinite(a) || !std::isfinite(b))
      throw std::invalid_argument("features contain non-finite values");
    lo[cols[c]] = a;
    hi[cols[c]] = b;
  }

  // ---- 2. per-window parameters
  const bool fp32 = (P.prec == NLD_FP32);
  std::vector<CoordParams> cp(L);
  P.wins.assign(L, WinDev{});
  P.info.assign(L, nld_window_info{});
  P.coef_host.assign(L, {});
  P.sig_t.assign(3 * (size_t)L, 0.0);
  P.scale_t.assign(3 * (size_t)L, 0.0);
  unsigned tile_total = 0;
  long long max_padded = 1;
  long long grid_total = 0;
  int n_max = 1;
  int off = 0;
  for (int l = 0; l < L; ++l) {
    const int dl = P.win_dim[l];
    std::vector<int> kept;
    std::vector<double> R;
    for (int k = 0; k < dl; ++k) {
      const int c = P.win_feat[off + k];
      const double r = hi[c] - lo[c];
      if (r > 0.0) {
        kept.push_back(c);
        R.push_back(r);
      }
    }
    off += dl;
    const int t = (int)kept.size();
    const double sigma = P.sigma[l];
    // bandwidth M
    int M = P.bw[l];
    if (M == 0) M = auto_bandwidth(sigma, R, P.tol);
    int m = P.cutoff;
    if (m == 0) m = fp32 ? 4 : (P.tol >= 1e-9 ? 6 : 8);
    int n = next_pow2((int)std::ceil(P.oversampling * M - 1e-9));
    n = std::max(n, 32);
    if (n <= M) n = next_pow2(M + 1);
    // a grid cap: the largest allowed grid if it still oversamples the band by 1.25
    if (P.max_grid > 0 && n > P.max_grid && 4 * P.max_grid >= 5 * M) n = P.max_grid;
    if (n > 256) throw std::invalid_argument("grid larger than 256 points per dimension");
    if (2 * m > n / 2) throw std::invalid_argument("cutoff too large for the grid");
    const double b = M_PI * (2.0 - (double)M / n);
    WinDev& w = P.wins[l];
    w.t = t;
    w.m = m;
    w.b = b;
    w.kb_den = 1.0 / (-std::expm1(-2.0 * b * m));
    w.weight = P.weight[l];
    CoordParams& p = cp[l];
    p.m = m;
    nld_window_info& inf = P.info[l];
    inf.dims_kept = t;
    inf.bandwidth = M;
    inf.grid = n;
    inf.cutoff = m;
    for (int dd = 0; dd < 3; ++dd) {
      const int k = dd - (3 - t);   // kept-dimension index of internal dim dd
      if (k >= 0) {
        const int c = kept[k];
        const double a = compression(sigma, R[k], M);
        const double sc = 2.0 * a / R[k];
        p.feat[dd] = c;
        P.scale_t[3 * (size_t)l + dd] = sc;
        P.sig_t[3 * (size_t)l + dd] = sigma * sc;
        p.centre[dd] = 0.5 * (lo[c] + hi[c]);
        p.scale[dd] = sc;
        p.n[dd] = n;
        w.n[dd] = n;
        w.taps[dd] = 2 * m;
        inf.compression[k] = a;
        inf.lo[k] = lo[c];
        inf.hi[k] = hi[c];
      } else {
        p.feat[dd] = -1;
        p.centre[dd] = 0.0;
        p.scale[dd] = 0.0;
        p.n[dd] = 1;
        w.n[dd] = 1;
        w.taps[dd] = 1;
      }
    }
    // tiles: the padded tile (tile + 2m - 1 halo cells per dimension) must fit in LDS
    int tsz;
    if (t == 3) {
      // the spreading accumulates the padded tile in 8 bytes of fixed point per cell
      // 8^3 tiles: smaller padded tiles in LDS give more resident workgroups, which measured
      // faster than 16^3 tiles on the 512^2 workload despite the larger halo overhead
      tsz = P.tile3 ? P.tile3 : 8;
      if (P.tile3 == 0)
        if (const char* e = std::getenv("NLD_TILE3")) tsz = std::atoi(e);
      if (tsz != 8 && tsz != 16) tsz = 8;
      if ((long long)std::pow(tsz + 2 * m - 1, 3) * 8LL > P.lds_limit) tsz = 8;
    } else if (t == 2) {
      tsz = std::min(64, n);
    } else {
      tsz = n;
    }
    if (t > 0 && (tsz < m || n % tsz != 0)) throw std::invalid_argument("no tile size fits the cutoff");
    long long padded = 1;
    for (int dd = 0; dd < 3; ++dd) {
      const int ts = (w.n[dd] == 1) ? 1 : std::min(tsz, w.n[dd]);
      w.ts[dd] = p.ts[dd] = ts;
      w.nts[dd] = p.nts[dd] = w.n[dd] / ts;
      w.pe[dd] = ts + w.taps[dd] - 1;
      w.lts[dd] = 0;
      while ((1 << w.lts[dd]) < ts) ++w.lts[dd];
      w.lnts[dd] = 0;
      while ((1 << w.lnts[dd]) < w.nts[dd]) ++w.lnts[dd];
      if ((1 << w.lts[dd]) != ts || (1 << w.lnts[dd]) != w.nts[dd])
        throw std::invalid_argument("tile sizes must be powers of two");
      padded *= w.pe[dd];
    }
    if (padded * 8LL > P.lds_limit)
      throw std::invalid_argument("padded tile does not fit in LDS");
    if ((long long)w.ts[0] * w.ts[1] * w.ts[2] > (1LL << kMaxCellBits))
      throw std::invalid_argument("tile too large for the sort key");
    max_padded = std::max<long long>(max_padded, padded);
    p.tile_off = tile_total;
    w.tile_off = (int)tile_total;
    tile_total += (unsigned)(w.nts[0] * w.nts[1] * w.nts[2]);
    w.grid_off = grid_total;
    w.grid_size = (long long)w.n[0] * w.n[1] * w.n[2];
    grid_total += w.grid_size;
    n_max = std::max(n_max, n);
  }
  P.n_max = n_max;
  // bits of the cell-within-tile part of the sort key: enough for the largest tile
  int cell_bits = 1;
  for (int l = 0; l < L; ++l) {
    const long long cells = (long long)P.wins[l].ts[0] * P.wins[l].ts[1] * P.wins[l].ts[2];
    while ((1LL << cell_bits) < cells) ++cell_bits;
  }
  for (int l = 0; l < L; ++l) cp[l].cell_bits = cell_bits;
  // ---- 3. coordinates of every (window, node)
  const long long LN = N * L;
  CoordParams* d_cp = dalloc<CoordParams>(L, s);
  upload(P, d_cp, cp.data(), L * sizeof(CoordParams), s);
  CoordEntry<T>* ent = dalloc<CoordEntry<T>>(LN, s);
  unsigned* key = dalloc<unsigned>(LN, s);
  unsigned* val = dalloc<unsigned>(LN, s);
  const dim3 win_grid(std::min<unsigned>(grid_for(N), (unsigned)((65536 + L - 1) / L)), (unsigned)L);
  hipLaunchKernelGGL(k_coords<T>, win_grid, dim3(256), 0, s, (const T*)features, N, d_cp, ent, key,
                     val);
  NLD_HIP(hipGetLastError());

  // ---- 4. nodes of every window sorted (stably) by tile; tile offsets by binary search
  // bits of the key within a window: its tile count and the cell bits
  int kbits = 1;
  for (int l = 0; l < L; ++l) {
    const unsigned nt = (unsigned)(P.wins[l].nts[0] * P.wins[l].nts[1] * P.wins[l].nts[2]);
    while ((1u << kbits) < nt) ++kbits;
  }
  if (kbits + cell_bits > 32) throw std::invalid_argument("too many tiles");
  radix_sort_segments(key, val, L, N, kbits + cell_bits, s);
  // tile offsets first: the host builds the schedules from them while the device permutes the
  // node entries into sorted order
  unsigned* toff = dalloc<unsigned>(tile_total + 1, s);
  hipLaunchKernelGGL(k_key_offsets, dim3((tile_total + 256) / 256), dim3(256), 0, s, key, N, L,
                     (const CoordParams*)d_cp, (int)tile_total, cell_bits, toff);
  NLD_HIP(hipGetLastError());
  unsigned* ht_pin = (unsigned*)pinned_get((tile_total + 1) * sizeof(unsigned), false);
  NLD_HIP(hipMemcpyAsync(ht_pin, toff, (tile_total + 1) * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  hipEvent_t ev_off;
  NLD_HIP(hipEventCreateWithFlags(&ev_off, hipEventDisableTiming));
  NLD_HIP(hipEventRecord(ev_off, s));
  P.g_idx = dalloc<int>(LN, s);
  P.g_base = dalloc<unsigned>(LN, s);
  P.g_frac = dalloc<T>(3 * LN, s);
  hipLaunchKernelGGL(k_gather_entries<T>, win_grid, dim3(256), 0, s, val, N,
                     (const CoordEntry<T>*)ent, P.g_idx, P.g_base, (T*)P.g_frac, LN);
  NLD_HIP(hipGetLastError());
  // the remaining host tables reach the device together at the end of the build
  P.defer_uploads = true;
  // Fourier multipliers and window polynomials: host work that only the products need, done
  // while the device sorts and permutes
  std::vector<T> coef_all, coef_dv_all;   // host staging, alive until the final synchronisation
  upload_tables<T>(P, coef_all, coef_dv_all, s);

  // window polynomials (same cutoff for every window; the shape b depends on M / n)
  std::vector<T> psi_all;   // host staging buffers live until the final synchronisation
  {
    const int deg = PsiDeg<T>::value;
    const int W = 2 * P.wins[0].m;
    psi_all.assign((size_t)L * W * (deg + 1), (T)0);
    P.psi_err = 0.0;
    std::vector<double> c;                    // fitted once per distinct window shape (m, b)
    int c_m = -1;
    double c_b = 0.0;
    for (int l = 0; l < L; ++l) {
      double err = 0.0;
      if (P.wins[l].m != c_m || P.wins[l].b != c_b) {
        c = fit_window(P.wins[l].m, P.wins[l].b, deg, &err);
        c_m = P.wins[l].m;
        c_b = P.wins[l].b;
        P.psi_err = std::max(P.psi_err, err);
      }
      for (size_t q = 0; q < c.size(); ++q) psi_all[(size_t)l * W * (deg + 1) + q] = (T)c[q];
    }
    P.psi = dalloc<T>((long long)psi_all.size(), s);
    upload(P, P.psi, psi_all.data(), psi_all.size() * sizeof(T), s);
    for (int l = 0; l < L; ++l) P.wins[l].psi = (const T*)P.psi + (size_t)l * W * (deg + 1);
  }
  // ---- 5. fold, plane and convolution jobs (they depend on the windows only)
  // fold jobs: per tile for 3-D windows (uniform tile size), 256 grid cells each otherwise
  std::vector<FoldJob> fj;
  std::vector<Fold3Job> f3;
  P.f3_ts = 0;
  P.f3_quad = true;
  for (int l = 0; l < L; ++l) {
    const WinDev& w = P.wins[l];
    if (w.t == 3) {
      if (P.f3_ts != 0 && P.f3_ts != w.ts[0]) throw std::runtime_error("internal: mixed 3-D tile sizes");
      if (w.ts[0] != w.ts[1] || w.ts[1] != w.ts[2]) throw std::runtime_error("internal: non-cubic tile");
      P.f3_ts = w.ts[0];
      P.f3_quad = P.f3_quad && w.nts[2] % 4 == 0;
      const int nt = w.nts[0] * w.nts[1] * w.nts[2];
      for (int tl = 0; tl < nt; ++tl) f3.push_back(Fold3Job{l, tl});
    } else if (w.t > 0) {
      for (long long c = 0; c < w.grid_size; c += 256)
        fj.push_back(FoldJob{l, (int)std::min<long long>(256, w.grid_size - c), c});
    }
  }
  P.h_fjobs = fj;
  P.n_fjobs = (int)fj.size();
  P.d_fjobs = dalloc<FoldJob>(std::max<size_t>(1, fj.size()), s);
  upload(P, P.d_fjobs, fj.data(), fj.size() * sizeof(FoldJob), s);
  // windows whose convolutions along the last two dimensions run fused per grid plane: FP32,
  // three kept dimensions of n = 64 or 128 points (plane, exchange buffer and twiddles in LDS)
  std::vector<char> fused(L, 0);
  const bool no_plane = std::getenv("NLD_NO_PLANE") != nullptr;
  for (int l = 0; l < L; ++l) {
    const WinDev& w = P.wins[l];
    const int n = w.n[0];
    fused[l] = !no_plane && P.prec == NLD_FP32 && w.t == 3 && n == w.n[1] && n == w.n[2] &&
               (n == 64 || n == 128) && (long long)plane_lds_bytes(n) <= P.lds_limit;
  }
  std::vector<PlaneJob> pj;
  for (int gi = 0; gi < 2; ++gi) {
    P.pjob_begin[gi] = (int)pj.size();
    const int ng = 64 << gi;
    for (int l = 0; l < L; ++l)
      if (fused[l] && P.wins[l].n[0] == ng)
        for (int i0 = 0; i0 < ng; ++i0) pj.push_back(PlaneJob{l, i0});
  }
  P.pjob_begin[2] = (int)pj.size();
  P.h_pjobs = pj;
  P.d_pjobs = dalloc<PlaneJob>(std::max<size_t>(1, pj.size()), s);
  upload(P, P.d_pjobs, pj.data(), pj.size() * sizeof(PlaneJob), s);
  std::vector<Fold3Job> f3f(f3);                // the fold still runs for every window
  P.h_f3jobs = f3f;
  P.n_f3jobs = (int)f3f.size();
  P.d_f3jobs = dalloc<Fold3Job>(std::max<size_t>(1, f3f.size()), s);
  upload(P, P.d_f3jobs, f3f.data(), f3f.size() * sizeof(Fold3Job), s);
  P.n_f3jobs_u = (int)f3.size();
  P.d_f3jobs_u = dalloc<Fold3Job>(std::max<size_t>(1, f3.size()), s);
  upload(P, P.d_f3jobs_u, f3.data(), f3.size() * sizeof(Fold3Job), s);

  // convolution jobs: for each axis, lines of every window that has that axis, grouped by the
  // grid size n; each job holds the real lines one workgroup transforms (64 for n = 64 and 128,
  // 32 for n = 32 and 256), adjacent in memory along the contiguous dimension.  The fused
  // schedule drops the last two axes of the fused windows.
  std::vector<ConvJob> cjobs_all[3], cjobs_f[3];
  for (int ax = 0; ax < 3; ++ax) {
    for (int gi = 0; gi < 4; ++gi) {
      P.conv_begin_u[ax][gi] = (int)cjobs_all[ax].size();
      P.conv_begin[ax][gi] = (int)cjobs_f[ax].size();
      const int ng = 32 << gi;
      const int lines_per = (ng == 64 || ng == 128) ? 64 : 32;
      for (int l = 0; l < L; ++l) {
        const WinDev& w = P.wins[l];
        if (w.n[ax] == 1 || w.n[ax] != ng) continue;
        const int n0 = w.n[0], n1 = w.n[1], n2 = w.n[2];
        std::vector<ConvJob> jl;
        if (ax == 2) {
          const long long lines = (long long)n0 * n1;
          for (long long q = 0; q < lines; q += lines_per)
            jl.push_back(ConvJob{l, (int)std::min<long long>(lines_per, lines - q), q * n2});
        } else if (ax == 1) {
          for (int i0 = 0; i0 < n0; ++i0)
            for (int i2 = 0; i2 < n2; i2 += lines_per)
              jl.push_back(ConvJob{l, std::min(lines_per, n2 - i2), (long long)i0 * n1 * n2 + i2});
        } else {
          for (int i1 = 0; i1 < n1; ++i1)
            for (int i2 = 0; i2 < n2; i2 += lines_per)
              jl.push_back(ConvJob{l, std::min(lines_per, n2 - i2), (long long)i1 * n2 + i2});
        }
        cjobs_all[ax].insert(cjobs_all[ax].end(), jl.begin(), jl.end());
        if (!(fused[l] && ax != 0)) cjobs_f[ax].insert(cjobs_f[ax].end(), jl.begin(), jl.end());
      }
    }
    P.conv_begin_u[ax][4] = (int)cjobs_all[ax].size();
    P.conv_begin[ax][4] = (int)cjobs_f[ax].size();
    P.h_conv[ax] = cjobs_f[ax];
    if (!cjobs_f[ax].empty()) {
      P.d_conv[ax] = dalloc<ConvJob>(cjobs_f[ax].size(), s);
      upload(P, P.d_conv[ax], cjobs_f[ax].data(), cjobs_f[ax].size() * sizeof(ConvJob), s);
    }
    if (!cjobs_all[ax].empty()) {
      P.d_conv_u[ax] = dalloc<ConvJob>(cjobs_all[ax].size(), s);
      upload(P, P.d_conv_u[ax], cjobs_all[ax].data(), cjobs_all[ax].size() * sizeof(ConvJob), s);
    }
  }
  const hipError_t ev_err = hipEventSynchronize(ev_off);
  (void)hipEventDestroy(ev_off);
  NLD_HIP(ev_err);
  std::vector<unsigned> ht(ht_pin, ht_pin + tile_total + 1);
  pinned_put(ht_pin);
  if (ht[tile_total] != (unsigned)LN) throw std::runtime_error("internal: tile offsets do not add up");

  // ---- 6. schedules (host): chunks of the nodes of every non-empty tile, grouped by t;
  // every chunk owns one padded-tile slot; the fold sums a tile's slots in order.
  std::vector<TileJob> jobs;
  std::vector<int> slot0(tile_total, 0), nslot(tile_total, 0);
  int slots = 0;
  const long long chunk = tile_chunk();
  for (int g = 0; g < 3; ++g) {
    P.tjob_begin[g] = (int)jobs.size();
    for (int l = 0; l < L; ++l) {
      const WinDev& w = P.wins[l];
      if (w.t != g + 1) continue;      // windows without kept dimensions need no grid
      const int nt = w.nts[0] * w.nts[1] * w.nts[2];
      for (int tl = 0; tl < nt; ++tl) {
        const unsigned gt = (unsigned)w.tile_off + tl;
        const long long b0 = ht[gt], b1 = ht[gt + 1];
        if (b1 == b0) continue;
        slot0[gt] = slots;
        for (long long c = b0; c < b1; c += chunk) {
          jobs.push_back(TileJob{l, tl, (int)c, (int)std::min(b1, c + chunk), slots});
          ++slots;
          ++nslot[gt];
        }
      }
    }
  }
  P.tjob_begin[3] = (int)jobs.size();
  // the gathering: tile order (neighbouring tiles stage overlapping grid cells), largest chunks
  // first within each XCD's range
  P.h_gjobs = jobs;
  {
    std::vector<TileJob> gj(jobs);
    for (int g = 0; g < 3; ++g) gather_order(gj, P.tjob_begin[g], P.tjob_begin[g + 1]);
    P.d_gjobs = dalloc<TileJob>(std::max<size_t>(1, gj.size()), s);
    upload(P, P.d_gjobs, gj.data(), gj.size() * sizeof(TileJob), s);
  }
  // largest chunks first within each group, so the long workgroups start early
  for (int g = 0; g < 3; ++g) sort_by_size_desc(jobs, P.tjob_begin[g], P.tjob_begin[g + 1]);
  if (std::getenv("NLD_PLAN_STATS")) {
    long long ne = 0, maxc = 0;
    for (unsigned gt = 0; gt < tile_total; ++gt) {
      const long long c = (long long)ht[gt + 1] - ht[gt];
      ne += (c > 0);
      maxc = std::max(maxc, c);
    }
    std::fprintf(stderr, "plan: N=%lld L=%d tiles=%u nonempty=%lld jobs=%zu slots=%d max_tile_nodes=%lld "
                 "max_padded=%lld psi_err=%.2e\n", (long long)N, L, tile_total, ne, jobs.size(), slots,
                 maxc, max_padded, P.psi_err);
  }
  P.h_tjobs = jobs;
  P.d_tjobs = dalloc<TileJob>(std::max<size_t>(1, jobs.size()), s);
  upload(P, P.d_tjobs, jobs.data(), jobs.size() * sizeof(TileJob), s);
  P.n_tiles_total = (int)tile_total;
  P.tile_slot0 = dalloc<int>(tile_total, s);
  P.tile_nslot = dalloc<int>(tile_total, s);
  upload(P, P.tile_slot0, slot0.data(), tile_total * sizeof(int), s);
  upload(P, P.tile_nslot, nslot.data(), tile_total * sizeof(int), s);
  P.max_padded = (int)max_padded;
  P.slot_stride = max_padded;
  P.padded = dalloc<T>((long long)std::max(1, slots) * max_padded, s);

  // ---- 7. work buffers
  P.grid_total = grid_total;
  P.grid = dalloc<T>(grid_total, s);
  P.ylocal = dalloc<T>(LN, s);
  P.D = dalloc<double>(N, s);
  P.sumv = dalloc<double>(1, s);
  P.has_flat = false;
  for (const auto& w : P.wins) P.has_flat = P.has_flat || (w.t == 0);
  P.ones = dalloc<T>(N, s);
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(N)), dim3(256), 0, s, (T*)P.ones, N, (T)1);
  NLD_HIP(hipGetLastError());
  P.z = dalloc<T>(N, s);
  P.r = dalloc<T>(N, s);
  P.p = dalloc<T>(N, s);
  P.q = dalloc<T>(N, s);
  P.red = dalloc<double>((long long)kRedBlocks * 8, s);
  P.st = dalloc<CgState>(1, s);
  hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(256), 0, s, (unsigned char*)P.st,
                     (long long)sizeof(CgState), (unsigned char)0);
  NLD_HIP(hipGetLastError());
  // every window points at the plan's buffers
  for (int l = 0; l < L; ++l) {
    WinDev& w = P.wins[l];
    w.img = 0;
    w.wl = l;
    w.N = N;
    w.LN = LN;
    w.g_idx = P.g_idx;
    w.g_base = P.g_base;
    w.g_frac = P.g_frac;
    w.grid = P.grid;
    w.padded = P.padded;
    w.slot_stride = P.slot_stride;
    w.tile_slot0 = P.tile_slot0;
    w.tile_nslot = P.tile_nslot;
    w.ylocal = static_cast<T*>(P.ylocal) + (long long)l * N;
  }
  std::vector<WinDev> wins_dv[3];
  upload_windows<T>(P, wins_dv, s);
  // the plan's own image table (f and u are set by each solve)
  // blocks of the FP64 reductions: at least 8 entries per thread, since every block adds one
  // ticket to the last-block count and those same-address atomics serialise
  const int nred = (int)std::max<long long>(
      1, std::min<long long>(kRedBlocks, (N + 8 * kRedThreads - 1) / (8 * kRedThreads)));
  P.img_host = (ImgDev*)pinned_get(sizeof(ImgDev));
  ImgDev& im = *P.img_host;
  im = ImgDev{};
  im.N = N;
  im.win0 = 0;
  im.L = L;
  im.nred = nred;
  im.vec[V_Z] = P.z;
  im.vec[V_R] = P.r;
  im.vec[V_P] = P.p;
  im.vec[V_Q] = P.q;
  im.vec[V_F] = nullptr;
  im.vec[V_U] = nullptr;
  im.vec[V_ONES] = P.ones;
  im.D = P.D;
  im.D2 = nullptr;
  im.sumv = P.sumv;
  im.st = P.st;
  im.red = P.red;
  P.d_img = dalloc<ImgDev>(1, s);
  upload(P, P.d_img, P.img_host, sizeof(ImgDev), s);
  LaunchSet& ls = P.ls;
  ls = LaunchSet{};
  ls.prec = P.prec;
  ls.m = P.wins[0].m;
  ls.d_wins = P.d_wins;
  ls.d_tjobs = P.d_tjobs;
  ls.d_gjobs = P.d_gjobs;
  for (int g = 0; g < 4; ++g) ls.tjob_begin[g] = P.tjob_begin[g];
  ls.max_padded = P.max_padded;
  ls.ts3 = (P.f3_ts == 8) ? 8 : 0;
  ls.f3_quad = P.f3_quad;
  ls.d_f3jobs = P.d_f3jobs;
  ls.f3_begin[0] = 0;
  ls.f3_begin[1] = (P.f3_ts == 16) ? 0 : P.n_f3jobs;
  ls.f3_begin[2] = P.n_f3jobs;
  ls.d_fjobs = P.d_fjobs;
  ls.n_fjobs = P.n_fjobs;
  for (int ax = 0; ax < 3; ++ax) {
    ls.d_conv[ax] = P.d_conv[ax];
    for (int g = 0; g < 5; ++g) ls.conv_begin[ax][g] = P.conv_begin[ax][g];
  }
  ls.d_pjobs = P.d_pjobs;
  for (int g = 0; g < 3; ++g) ls.pjob_begin[g] = P.pjob_begin[g];
  ls.d_imgs = P.d_img;
  ls.n_imgs = 1;
  ls.max_N = N;
  ls.max_nred = nred;
  ls.has_flat = P.has_flat;
  LaunchSet& lu = P.ls_unfused;
  lu = ls;
  lu.d_f3jobs = P.d_f3jobs_u;
  lu.f3_begin[1] = (P.f3_ts == 16) ? 0 : P.n_f3jobs_u;
  lu.f3_begin[2] = P.n_f3jobs_u;
  for (int ax = 0; ax < 3; ++ax) {
    lu.d_conv[ax] = P.d_conv_u[ax];
    for (int g = 0; g < 5; ++g) lu.conv_begin[ax][g] = P.conv_begin_u[ax][g];
  }
  lu.d_pjobs = nullptr;
  for (int g = 0; g < 3; ++g) lu.pjob_begin[g] = 0;
  flush_uploads(P, s);

  dfree(d_cp, s);
  dfree(ent, s);
  dfree(key, s);
  dfree(val, s);
  dfree(toff, s);
  NLD_HIP(hipStreamSynchronize(s));
  staging_done(P, s);
  P.have_D = false;
}

// Plans take their buffers from the device's stream-ordered pool (hipMallocAsync).  The pool's
// default release threshold of zero hands freed memory back at every synchronisation, so a
// new plan (with slot buffers of up to a few hundred MB) would map it again; the library keeps
// it in the pool instead, for the life of the process, once per device.
static void keep_pool_memory() {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  NLD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  NLD_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = ~0ULL;
  NLD_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done[dev] = true;
}

// Small pinned host blocks (CG state mirrors, image tables) are reused across plans and solves:
// hipHostMalloc and hipHostFree of even a few hundred bytes take on the order of a millisecond,
// more than the rest of a plan's release.  Blocks are kept by size class (powers of two from
// 4 KiB) for the life of the process and handed out zeroed.
namespace {
std::mutex g_pinned_mu;
std::map<size_t, std::vector<void*>> g_pinned_free;     // size class -> free blocks
std::map<void*, size_t> g_pinned_class;                 // block -> its size class
}  // namespace

void* pinned_get(size_t bytes, bool zero) {
  size_t cls = 4096;
  while (cls < bytes) cls <<= 1;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    auto& fl = g_pinned_free[cls];
    if (!fl.empty()) {
      p = fl.back();
      fl.pop_back();
    }
  }
  if (!p) {
    NLD_HIP(hipHostMalloc(&p, cls, hipHostMallocDefault));
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_pinned_class[p] = cls;
  }
  if (zero) std::memset(p, 0, bytes);
  return p;
}

void pinned_put(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_pinned_mu);
  auto it = g_pinned_class.find(p);
  if (it == g_pinned_class.end()) return;                // not from pinned_get: leave it alone
  g_pinned_free[it->second].push_back(p);
}

// Stable sort of jobs [b, e) by node count, largest first: a counting sort over the chunk sizes
// (at most kMaxChunk), the same order as a comparison-based stable sort in a fraction of the time.
void sort_by_size_desc(std::vector<TileJob>& jobs, size_t b, size_t e) {
  if (e - b < 2) return;
  auto key = [](const TileJob& j) { return std::min(kMaxChunk + 1, std::max(0, j.pend - j.pbeg)); };
  std::vector<unsigned> pos(kMaxChunk + 2, 0u);
  for (size_t i = b; i < e; ++i) ++pos[key(jobs[i])];
  unsigned acc = 0;
  for (int sz = kMaxChunk + 1; sz >= 0; --sz) {
    const unsigned c = pos[sz];
    pos[sz] = acc;
    acc += c;
  }
  std::vector<TileJob> tmp(e - b);
  for (size_t i = b; i < e; ++i) tmp[pos[key(jobs[i])]++] = jobs[i];
  std::copy(tmp.begin(), tmp.end(), jobs.begin() + b);
}

void gather_order(std::vector<TileJob>& jobs, size_t begin, size_t end) {
  const size_t nj = end - begin;
  for (size_t x = 0; x < 8; ++x) {
    const size_t b = begin + x * (nj / 8) + std::min(x, nj % 8);
    const size_t e = b + nj / 8 + (x < nj % 8 ? 1 : 0);
    sort_by_size_desc(jobs, b, e);
  }
}

void build_plan(Plan& P, const void* features, hipStream_t s) {
  keep_pool_memory();
  P.features = const_cast<void*>(features);
  P.stream = s;
  if (P.prec == NLD_FP32) build_plan_t<float>(P, features, s);
  else build_plan_t<double>(P, features, s);
}

// Per-entry error estimate of one dimension with the node compression a kept fixed: the
// truncation of the Fourier series and the nearest periodic image at distance 1 - 2a.
static double dim_error_fixed(double st, double a, int M) {
  const double trunc = std::exp(-std::pow(M_PI * st * M / 2.0, 2));
  const double wrap = std::exp(-std::pow((1.0 - 2.0 * a) / st, 2));
  return std::max(trunc, wrap);
}

template <typename T>
static void update_kernel_t(Plan& P, const double* sigma, const double* weight, hipStream_t s) {
  const int L = P.L;
  // the scaled node coordinates (and with them the sort and every schedule) stay; only the
  // widths on the torus change, so check that the kept compression and bandwidth still fit
  std::vector<double> sig_new(P.sig_t);
  for (int l = 0; l < L; ++l) {
    const WinDev& w = P.wins[l];
    const int M = P.info[l].bandwidth;
    if (P.bw[l] == 0 && w.t > 0) {
      // an autotuned bandwidth must still be the one the autotuner picks for the new width
      std::vector<double> R;
      for (int k = 0; k < w.t; ++k) R.push_back(P.info[l].hi[k] - P.info[l].lo[k]);
      if (auto_bandwidth(sigma[l], R, P.tol) != M)
        throw std::runtime_error("nfft_plan_update_kernel: window " + std::to_string(l) +
                                 " needs another bandwidth for the new sigma");
    }
    for (int dd = 0; dd < 3; ++dd) {
      if (w.n[dd] == 1) continue;
      const int k = dd - (3 - w.t);
      const double a = P.info[l].compression[k];
      const double st_old = P.sig_t[3 * (size_t)l + dd];
      const double st = sigma[l] * P.scale_t[3 * (size_t)l + dd];
      const double R = P.info[l].hi[k] - P.info[l].lo[k];
      const double e_new = dim_error_fixed(st, a, M);
      const double e_ref = std::max(dim_error_fixed(st_old, a, M), dim_error(sigma[l], R, M));
      if (e_new > std::max(1e-2 * P.tol, 10.0 * e_ref))
        throw std::runtime_error("nfft_plan_update_kernel: window " + std::to_string(l) +
                         " needs a new bandwidth or node scaling for the new sigma");
      sig_new[3 * (size_t)l + dd] = st;
    }
  }
  P.sig_t = sig_new;
  for (int l = 0; l < L; ++l) {
    P.sigma[l] = sigma[l];
    P.weight[l] = weight[l];
    P.wins[l].weight = weight[l];
  }
  std::vector<T> coef_all, coef_dv_all;
  upload_tables<T>(P, coef_all, coef_dv_all, s);
  std::vector<WinDev> wins_dv[3];
  upload_windows<T>(P, wins_dv, s);
  NLD_HIP(hipStreamSynchronize(s));
  staging_done(P, s);
  P.have_D = false;
  P.have_D2 = false;
  P.have_dl = false;
}

// Multiplier tables of exp(-r^2 / (sigma_l^2 / 2)) on the plan's grids (the squared kernels:
// widths on the torus divided by sqrt 2, same bandwidth and window), descriptors with weights
// w_l^2, and D2 = sum_l w_l^2 K_l(sigma_l / sqrt 2) 1 for the l2 preconditioner.  The coarser
// truncation at the same bandwidth only affects the preconditioner, never the solution.
template <typename T>
static void ensure_l2_t(Plan& P, hipStream_t s) {
  const int L = P.L, n_max = P.n_max;
  std::vector<T> cb(3LL * n_max * L, (T)0);
  for (int l = 0; l < L; ++l) {
    const WinDev& w = P.wins[l];
    const int n = P.info[l].grid, M = P.info[l].bandwidth;
    for (int dd = 0; dd < 3; ++dd) {
      if (w.n[dd] == 1) continue;
      const double st = P.sig_t[3 * (size_t)l + dd] / std::sqrt(2.0);
      for (int q = 0; q < n; ++q) {
        const int kf = (q < n / 2) ? q : q - n;
        if (std::abs(kf) <= M / 2 - 1) {
          const double bh = std::sqrt(M_PI) * st * std::exp(-std::pow(M_PI * st * kf, 2));
          const double ph = kb_fourier(kf, n, w.m, w.b);
          cb[((size_t)l * 3 + dd) * n_max + q] = (T)(bh / (ph * ph));
        }
      }
    }
  }
  if (!P.coef_b) P.coef_b = dalloc<T>((long long)cb.size(), s);
  upload(P, P.coef_b, cb.data(), cb.size() * sizeof(T), s);
  std::vector<WinDev> wb(P.wins);
  for (int l = 0; l < L; ++l) {
    wb[l].coef = (const T*)P.coef_b + (size_t)l * 3 * n_max;
    wb[l].weight = P.weight[l] * P.weight[l];
  }
  if (!P.d_wins_b) P.d_wins_b = dalloc<WinDev>(L, s);
  upload(P, P.d_wins_b, wb.data(), L * sizeof(WinDev), s);
  if (!P.D2) P.D2 = dalloc<double>(P.N, s);
  LaunchSet lb = P.ls_unfused;
  lb.d_wins = P.d_wins_b;
  matvec_set(lb, VecArg{P.ones, V_ONES}, VecArg{nullptr, V_Q}, P.D2, EPI_DEGREE, s);
  P.img_host->D2 = P.D2;
  NLD_HIP(hipMemcpyAsync(P.d_img, P.img_host, sizeof(ImgDev), hipMemcpyHostToDevice, s));
  NLD_HIP(hipStreamSynchronize(s));   // host staging above is released on return
  staging_done(P, s);
  P.have_D2 = true;
}

void ensure_l2_degree(Plan& P, hipStream_t s) {
  if (P.have_D2) return;
  if (P.prec == NLD_FP32) ensure_l2_t<float>(P, s);
  else ensure_l2_t<double>(P, s);
}

void update_kernel(Plan& P, const double* sigma, const double* weight, hipStream_t s) {
  if (P.prec == NLD_FP32) update_kernel_t<float>(P, sigma, weight, s);
  else update_kernel_t<double>(P, sigma, weight, s);
}

void release_plan(Plan& P) {
  hipStream_t s = P.stream;
  void* bufs[] = {P.d_wins, P.g_idx, P.g_base, P.g_frac, P.coef, P.grid, P.padded, P.tile_slot0,
                  P.tile_nslot, P.ylocal, P.D, P.sumv, P.ones, P.psi, P.d_tjobs, P.d_gjobs, P.d_fjobs, P.d_f3jobs, P.d_conv[0], P.d_conv[1],
                  P.d_conv[2], P.z, P.r, P.p, P.q, P.red, P.st, P.coef_dv, P.d_wins_dv[0],
                  P.d_wins_dv[1], P.d_wins_dv[2], P.grid_save, P.yk, P.yks, P.dl, P.dls,
                  P.adj_part, P.d_img, P.d_pjobs, P.d_f3jobs_u, P.d_conv_u[0], P.d_conv_u[1],
                  P.d_conv_u[2], P.coef_b, P.d_wins_b, P.D2};
  (void)hipStreamSynchronize(s);
  staging_done(P, s);
  for (void* b : bufs) dev_release_idle(b);
  pinned_put(P.img_host);
  P.img_host = nullptr;
}

}  // namespace nld
