// NFFT fast Gauss summation of every window in batched launches (paper Sec. 3), the window
// reduction W~ v = sum_l w_l K~_l v (Sec. 3, ANOVA summation) and the Laplacian / system
// epilogues (Sec. 2.6).
//
//   spreading    output-tiled: one wavefront per grid tile accumulates, in LDS, the taps of
//                every node whose 2m^t support touches the tile (lists built at plan time),
//                then writes the tile once; no global atomics, deterministic order.
//   convolution  per dimension, a real circulant convolution of every grid line: two real
//                lines packed as one complex line, radix-2 Stockham FFT in LDS, multiplication
//                by the window's real even Fourier multiplier, inverse FFT, unpack.
//   gathering    one thread per node (nodes sorted by tile) sums its 2m^t taps.
//   reduction    FP64 sum over windows fused with the epilogue of the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "nld_device.h"

namespace nld {

namespace {

constexpr int kSpreadWaves = 4;
constexpr int kSpreadThreads = 64 * kSpreadWaves;
constexpr int kConvThreads = 256;
constexpr int kGatherThreads = 256;

__device__ __forceinline__ int wrap(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

__device__ __forceinline__ int tile_origin(const WinDev& w, int tile, int dd) {
  int tt;
  if (dd == 2) tt = tile % w.nts[2];
  else if (dd == 1) tt = (tile / w.nts[2]) % w.nts[1];
  else tt = tile / (w.nts[2] * w.nts[1]);
  return tt * w.ts[dd];
}

// Weights of the W = 2m taps of one node in one dimension: tap i sits at cell b - m + 1 + i,
// at distance fr + m - 1 - i from the node.
template <typename T, int W>
__device__ __forceinline__ void tap_row(T fr, T b, T den, T* wt) {
  constexpr int m = W / 2;
#pragma unroll
  for (int i = 0; i < W; ++i) wt[i] = kb_psi(fr + (T)(m - 1 - i), (T)m, b, den);
}

// ---------------------------------------------------------------------------- spreading
// One workgroup of kSpreadWaves wavefronts per chunk of a tile's nodes.  The chunk's taps are
// accumulated in LDS over the padded tile (tile plus the 2m - 1 halo cells its nodes' taps
// reach) and written to the chunk's slot; the fold kernel adds the slots covering each grid
// cell.  Every wavefront visits all nodes of the chunk but only adds the taps that fall in its
// own slab of the padded tile along the first kept dimension, so no two wavefronts touch the
// same LDS cell and the accumulation order is fixed: results are reproducible.  Within a
// wavefront, lane l walks the taps of its node in an order rotated by l, so lanes whose nodes
// share a grid cell (common: neighbouring pixels with equal features) hit different cells.
template <typename T, int W>
__device__ __forceinline__ void rotated_taps(T fr, T b, T den, int rot, T* wt, int* off) {
  constexpr int m = W / 2;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    int i = k + rot;
    i = (i >= W) ? i - W : i;
    off[k] = i;
    wt[k] = kb_psi(fr + (T)(m - 1 - i), (T)m, b, den);
  }
}

template <typename T, int W, int TD>
__global__ void __launch_bounds__(kSpreadThreads)
k_spread(const WinDev* __restrict__ wins, const TileJob* __restrict__ jobs, int job0,
         const int* __restrict__ g_idx, const unsigned* __restrict__ g_base,
         const T* __restrict__ g_frac, long long LN, const T* __restrict__ v,
         T* __restrict__ padded, long long slot_stride, const CgState* __restrict__ st) {
  if (st && st->done) return;
  extern __shared__ unsigned char smem_raw[];
  // FP64 accumulators in both precisions: LDS float atomics are far slower than double ones
  double* acc = reinterpret_cast<double*>(smem_raw);
  const TileJob job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  const int pe0 = w.pe[0], pe1 = w.pe[1], pe2 = w.pe[2];
  const int cells = pe0 * pe1 * pe2;
  for (int c = threadIdx.x; c < cells; c += kSpreadThreads) acc[c] = 0.0;
  __syncthreads();
  constexpr int m = W / 2;
  constexpr int OD = 3 - TD;                       // first kept (outer) dimension
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pe_out = w.pe[OD];
  const int own_lo = (wave * pe_out) / kSpreadWaves, own_hi = ((wave + 1) * pe_out) / kSpreadWaves;
  const int o_out = tile_origin(w, job.tile, OD);
  const int o1 = tile_origin(w, job.tile, 1), o2 = tile_origin(w, job.tile, 2);
  const T b = (T)w.b, den = (T)w.kb_den;
  const int r2 = lane % W, r1 = (lane / W) % W, r0 = lane % W;
  for (int p = job.pbeg + lane; p < job.pend; p += 64) {
    const unsigned bb = g_base[p];
    const int l_out = (int)((bb >> (8 * OD)) & 255u) - o_out;
    // taps along the outer dimension that land in this wave's slab: local l_out + i
    const int i_lo = max(0, own_lo - l_out), i_hi = min(W, own_hi - l_out);
    if (i_lo >= i_hi) continue;
    const T vj = v[g_idx[p]];
    if (vj == (T)0) continue;
    const T fr_out = g_frac[(long long)OD * LN + p];
    const int span = i_hi - i_lo;
    if constexpr (TD == 1) {
      for (int k = 0; k < span; ++k) {
        int i = i_lo + (k + r0) % span;
        atomicAdd(&acc[l_out + i], (double)(vj * kb_psi(fr_out + (T)(m - 1 - i), (T)m, b, den)));
      }
    } else {
      const int l2 = (int)((bb >> 16) & 255u) - o2;
      T w2[W];
      int c2[W];
      rotated_taps<T, W>(g_frac[2 * LN + p], b, den, r2, w2, c2);
      if constexpr (TD == 2) {
        for (int k = 0; k < span; ++k) {
          const int i = i_lo + (k + r1) % span;
          const T c1 = vj * kb_psi(fr_out + (T)(m - 1 - i), (T)m, b, den);
          double* row = acc + (l_out + i) * pe2 + l2;
#pragma unroll
          for (int k2 = 0; k2 < W; ++k2) atomicAdd(&row[c2[k2]], (double)(c1 * w2[k2]));
        }
      } else {
        const int l1 = (int)((bb >> 8) & 255u) - o1;
        T w1[W];
        int c1i[W];
        rotated_taps<T, W>(g_frac[LN + p], b, den, r1, w1, c1i);
        for (int k = 0; k < span; ++k) {
          const int i = i_lo + (k + r0) % span;
          const T c0 = vj * kb_psi(fr_out + (T)(m - 1 - i), (T)m, b, den);
          double* plane = acc + ((l_out + i) * pe1 + l1) * pe2 + l2;
#pragma unroll
          for (int k1 = 0; k1 < W; ++k1) {
            const T cc1 = c0 * w1[k1];
            double* row = plane + c1i[k1] * pe2;
#pragma unroll
            for (int k2 = 0; k2 < W; ++k2) atomicAdd(&row[c2[k2]], (double)(cc1 * w2[k2]));
          }
        }
      }
    }
  }
  __syncthreads();
  T* out = padded + (long long)job.slot * slot_stride;
  for (int c = threadIdx.x; c < cells; c += kSpreadThreads) out[c] = (T)acc[c];
}

// Grid cell value = sum of the padded-tile slots that cover the cell, in fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
k_fold(const WinDev* __restrict__ wins, const FoldJob* __restrict__ jobs,
       const T* __restrict__ padded, long long slot_stride, const int* __restrict__ tile_slot0,
       const int* __restrict__ tile_nslot, T* __restrict__ grid, const CgState* __restrict__ st) {
  if (st && st->done) return;
  const FoldJob job = jobs[blockIdx.x];
  if ((int)threadIdx.x >= job.ncell) return;
  const WinDev& w = wins[job.win];
  const long long c = job.cell0 + threadIdx.x;
  int cc[3];
  cc[2] = (int)(c % w.n[2]);
  cc[1] = (int)((c / w.n[2]) % w.n[1]);
  cc[0] = (int)(c / ((long long)w.n[2] * w.n[1]));
  // up to three (tile, local index) candidates per dimension, in the order left, home, right
  int ct[3][3], cl[3][3];
  bool ok[3][3];
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    const int ts = w.ts[dd];
    // taps reach m - 1 cells to the left of a tile and m cells to the right
    const int left = (w.taps[dd] > 1) ? w.m - 1 : 0;
    const int home = cc[dd] / ts;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int tu = home + k - 1;
      const int li = cc[dd] - tu * ts + left;
      ok[dd][k] = (li >= 0 && li < w.pe[dd]);
      ct[dd][k] = ((tu % w.nts[dd]) + w.nts[dd]) % w.nts[dd];
      cl[dd][k] = li;
    }
  }
  T sum = (T)0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int bq = 0; bq < 3; ++bq)
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        if (!(ok[0][a] && ok[1][bq] && ok[2][e])) continue;
        const int gt = w.tile_off + (ct[0][a] * w.nts[1] + ct[1][bq]) * w.nts[2] + ct[2][e];
        const int ns = tile_nslot[gt];
        if (ns == 0) continue;
        const long long pidx = ((long long)cl[0][a] * w.pe[1] + cl[1][bq]) * w.pe[2] + cl[2][e];
        const T* src = padded + (long long)tile_slot0[gt] * slot_stride + pidx;
        for (int q = 0; q < ns; ++q) sum += src[(long long)q * slot_stride];
      }
  grid[w.grid_off + c] = sum;
}

// ---------------------------------------------------------------------------- convolution
template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ void fft_lines(Cx<T>* a, Cx<T>* b, const Cx<T>* tw, int nlines, int n,
                                          bool inverse, Cx<T>** out) {
  // radix-2 Stockham autosort; tw[q] = exp(-2 pi i q / n), q < n/2
  const int half = n >> 1;
  const int total = nlines * half;
  for (int p = 1; p < n; p <<= 1) {
    const int stride = n / (2 * p);
    for (int idx = threadIdx.x; idx < total; idx += kConvThreads) {
      const int ln = idx / half, i = idx - ln * half;
      const Cx<T>* x = a + ln * n;
      Cx<T>* y = b + ln * n;
      const int k = i & (p - 1);
      const Cx<T> u0 = x[i];
      const Cx<T> v1 = x[i + half];
      Cx<T> t = tw[k * stride];
      if (inverse) t.y = -t.y;
      const Cx<T> u1 = {v1.x * t.x - v1.y * t.y, v1.x * t.y + v1.y * t.x};
      const int j = (i << 1) - k;
      y[j] = {u0.x + u1.x, u0.y + u1.y};
      y[j + p] = {u0.x - u1.x, u0.y - u1.y};
    }
    __syncthreads();
    Cx<T>* tmp = a;
    a = b;
    b = tmp;
  }
  *out = a;
}

template <typename T>
__global__ void __launch_bounds__(kConvThreads)
k_conv(const WinDev* __restrict__ wins, const ConvJob* __restrict__ jobs, int axis, int lb,
       T* __restrict__ grid, const CgState* __restrict__ st) {
  if (st && st->done) return;
  extern __shared__ unsigned char smem_raw[];
  const ConvJob job = jobs[blockIdx.x];
  const WinDev& w = wins[job.win];
  const int n = w.n[axis];
  const int nc = lb / 2;                        // complex lines
  Cx<T>* buf0 = reinterpret_cast<Cx<T>*>(smem_raw);
  Cx<T>* buf1 = buf0 + nc * w.n_max;
  Cx<T>* tw = buf1 + nc * w.n_max;
  for (int q = threadIdx.x; q < n / 2; q += kConvThreads) {
    T sn, cs;
    if constexpr (sizeof(T) == 4) sincospif(-2.0f * (float)q / (float)n, &sn, &cs);
    else sincospi(-2.0 * (double)q / (double)n, &sn, &cs);
    tw[q] = {cs, sn};
  }
  long long es, ls;   // element stride along the line, stride between adjacent lines
  if (axis == 2) { es = 1; ls = n; }
  else if (axis == 1) { es = w.n[2]; ls = 1; }
  else { es = (long long)w.n[1] * w.n[2]; ls = 1; }
  T* g = grid + w.grid_off + job.off;
  const int total = lb * n;
  for (int idx = threadIdx.x; idx < total; idx += kConvThreads) {
    int ln, c;
    if (axis == 2) { ln = idx / n; c = idx - ln * n; }
    else { c = idx / lb; ln = idx - c * lb; }
    const T val = (ln < job.nl) ? g[c * es + ln * ls] : (T)0;
    T* slot = reinterpret_cast<T*>(&buf0[(ln >> 1) * n + c]);
    slot[ln & 1] = val;
  }
  __syncthreads();
  Cx<T>* res;
  fft_lines<T>(buf0, buf1, tw, nc, n, false, &res);
  const T* coef = reinterpret_cast<const T*>(w.coef) + (long long)axis * w.n_max;
  for (int idx = threadIdx.x; idx < nc * n; idx += kConvThreads) {
    const int k = idx % n;
    const T c = coef[k];
    res[idx].x *= c;
    res[idx].y *= c;
  }
  __syncthreads();
  Cx<T>* other = (res == buf0) ? buf1 : buf0;
  fft_lines<T>(res, other, tw, nc, n, true, &res);
  for (int idx = threadIdx.x; idx < total; idx += kConvThreads) {
    int ln, c;
    if (axis == 2) { ln = idx / n; c = idx - ln * n; }
    else { c = idx / lb; ln = idx - c * lb; }
    if (ln < job.nl) {
      const T* slot = reinterpret_cast<const T*>(&res[(ln >> 1) * n + c]);
      g[c * es + ln * ls] = slot[ln & 1];
    }
  }
}

// ---------------------------------------------------------------------------- gathering
// One thread per node.  Chunks with many nodes first stage the padded tile of the convolved
// grid in LDS; small chunks read the grid directly.
constexpr int kStageMin = 192;

template <typename T, int W, int TD>
__global__ void __launch_bounds__(kGatherThreads)
k_gather(const WinDev* __restrict__ wins, const TileJob* __restrict__ jobs, int job0,
         const int* __restrict__ g_idx, const unsigned* __restrict__ g_base,
         const T* __restrict__ g_frac, long long N, long long LN, const T* __restrict__ grid,
         T* __restrict__ ylocal, const CgState* __restrict__ st) {
  if (st && st->done) return;
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const TileJob job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  const T* h = grid + w.grid_off;
  const int n0 = w.n[0], n1 = w.n[1], n2 = w.n[2];
  const int pe0 = w.pe[0], pe1 = w.pe[1], pe2 = w.pe[2];
  const int o0 = tile_origin(w, job.tile, 0), o1 = tile_origin(w, job.tile, 1),
            o2 = tile_origin(w, job.tile, 2);
  constexpr int m = W / 2;
  // first grid cell covered by the padded tile, per dimension
  const int s0 = (TD == 3) ? o0 - m + 1 : o0;
  const int s1 = (TD >= 2) ? o1 - m + 1 : o1;
  const int s2 = o2 - m + 1;
  const bool staged = (job.pend - job.pbeg) >= kStageMin;
  if (staged) {
    const int cells = pe0 * pe1 * pe2;
    for (int c = threadIdx.x; c < cells; c += kGatherThreads) {
      const int a2 = c % pe2, a1 = (c / pe2) % pe1, a0 = c / (pe2 * pe1);
      const int g0 = wrap(s0 + a0, n0), g1 = wrap(s1 + a1, n1), g2 = wrap(s2 + a2, n2);
      tile[c] = h[((long long)g0 * n1 + g1) * n2 + g2];
    }
    __syncthreads();
  }
  const T b = (T)w.b, den = (T)w.kb_den;
  const long long ybase = (long long)job.win * N;
  for (int p = job.pbeg + threadIdx.x; p < job.pend; p += kGatherThreads) {
    const unsigned bb = g_base[p];
    const int b2 = (int)((bb >> 16) & 255u), b1 = (int)((bb >> 8) & 255u), b0 = (int)(bb & 255u);
    T w2[W];
    tap_row<T, W>(g_frac[2 * LN + p], b, den, w2);
    T w1[W];
    if constexpr (TD >= 2) tap_row<T, W>(g_frac[LN + p], b, den, w1);
    T acc = (T)0;
    if (staged) {
      const int l2 = b2 - o2, l1 = b1 - o1, l0 = b0 - o0;
      auto line = [&](const T* row) {
        T sacc = (T)0;
#pragma unroll
        for (int i2 = 0; i2 < W; ++i2) sacc += row[i2] * w2[i2];
        return sacc;
      };
      if constexpr (TD == 1) {
        acc = line(tile + l2);
      } else if constexpr (TD == 2) {
#pragma unroll
        for (int i1 = 0; i1 < W; ++i1) acc += w1[i1] * line(tile + (l1 + i1) * pe2 + l2);
      } else {
        const T fr0 = g_frac[p];
        for (int i0 = 0; i0 < W; ++i0) {
          const T* plane = tile + ((l0 + i0) * pe1 + l1) * pe2 + l2;
          T pacc = (T)0;
#pragma unroll
          for (int i1 = 0; i1 < W; ++i1) pacc += w1[i1] * line(plane + i1 * pe2);
          acc += kb_psi(fr0 + (T)(m - 1 - i0), (T)m, b, den) * pacc;
        }
      }
    } else {
      int c2[W];
#pragma unroll
      for (int i2 = 0; i2 < W; ++i2) c2[i2] = wrap(b2 - m + 1 + i2, n2);
      auto line = [&](const T* row) {
        T sacc = (T)0;
#pragma unroll
        for (int i2 = 0; i2 < W; ++i2) sacc += row[c2[i2]] * w2[i2];
        return sacc;
      };
      if constexpr (TD == 1) {
        acc = line(h);
      } else if constexpr (TD == 2) {
#pragma unroll
        for (int i1 = 0; i1 < W; ++i1) acc += w1[i1] * line(h + (long long)wrap(b1 - m + 1 + i1, n1) * n2);
      } else {
        const T fr0 = g_frac[p];
        for (int i0 = 0; i0 < W; ++i0) {
          const T* plane = h + (long long)wrap(b0 - m + 1 + i0, n0) * n1 * n2;
          T pacc = (T)0;
#pragma unroll
          for (int i1 = 0; i1 < W; ++i1) pacc += w1[i1] * line(plane + (long long)wrap(b1 - m + 1 + i1, n1) * n2);
          acc += kb_psi(fr0 + (T)(m - 1 - i0), (T)m, b, den) * pacc;
        }
      }
    }
    ylocal[ybase + g_idx[p]] = acc;
  }
}

// ---------------------------------------------------------------------------- reduction
struct ReduceArgs {
  const void* yl;
  const double* wts;   // [L] window weights (device)
  int L;
  long long N;
  const void* v;
  void* out;
  double* Dout;
  const double* D;
  const void* f;
  CgState* st;
  double* red;
  const double* sumv;
  int mode;
};

// sum of v (FP64), for windows whose kernel is the constant 1 1^T
template <typename T>
__global__ void __launch_bounds__(1024) k_sum(const T* __restrict__ v, long long N,
                                              double* __restrict__ out, const CgState* __restrict__ st) {
  if (st && st->done) return;
  __shared__ double sh[1024];
  double a = 0.0;
  for (long long i = threadIdx.x; i < N; i += 1024) a += (double)v[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_reduce(const WinDev* __restrict__ wins, ReduceArgs a) {
  CgState* st = a.st;
  if (st && a.mode == EPI_CG_Q && st->done) return;
  const T* yl = (const T*)a.yl;
  const T* v = (const T*)a.v;
  T* out = (T*)a.out;
  const long long N = a.N;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const double alpha = st ? st->alpha : 0.0;
  const double mean_f = st ? st->mean_f : 0.0;
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kRedThreads) {
    double y = 0.0;
    for (int l = 0; l < a.L; ++l)
      y += wins[l].weight * (wins[l].t > 0 ? (double)yl[(long long)l * N + i] : *a.sumv);
    switch (a.mode) {
      case EPI_ANOVA:
        out[i] = (T)y;
        break;
      case EPI_LAPLACIAN:
        out[i] = (T)(a.D[i] * (double)v[i] - y);
        break;
      case EPI_DEGREE:
        a.Dout[i] = y;
        break;
      case EPI_CG_Q: {
        const double vi = (double)v[i];
        const double q = vi + alpha * (a.D[i] * vi - y);
        out[i] = (T)q;
        s0 += vi * q;
        s1 += q;
        s2 += vi;
        break;
      }
      case EPI_CG_INIT:
      case EPI_CG_TRUE: {
        const double vi = (double)v[i];
        const double b = (double)((const T*)a.f)[i] - mean_f;
        const double r = b - (vi + alpha * (a.D[i] * vi - y));
        if (a.mode == EPI_CG_INIT) out[i] = (T)r;
        s0 += r;
        s1 += (a.mode == EPI_CG_INIT) ? b * b : r * r;
        break;
      }
    }
  }
  if (a.mode < EPI_CG_Q) return;
  const double vals[3] = {s0, s1, s2};
  double tot[3];
  if (!grid_reduce<3>(vals, a.red, &st->ticket[0], tot)) return;
  if (threadIdx.x != 0) return;
  const double dN = (double)N;
  if (a.mode == EPI_CG_Q) {
    const double mean_q = st->deflate ? tot[1] / dN : 0.0;
    const double pq = tot[0] - mean_q * tot[2];
    st->mean_q = mean_q;
    st->last_pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      st->status = NLD_E_BREAKDOWN;
      st->done = 1;
    } else {
      st->a = st->rho / pq;
    }
  } else if (a.mode == EPI_CG_INIT) {
    st->mean_r = st->deflate ? tot[0] / dN : 0.0;
    st->bnorm2 = tot[1];
    st->tol2_b2 = st->tol * st->tol * tot[1];
  } else {
    const double mr = st->deflate ? tot[0] / dN : 0.0;
    st->rr_true = tot[1] - mr * mr * dN;
  }
}

inline unsigned grid_for(long long n, int threads = 256) {
  long long b = (n + threads - 1) / threads;
  return (unsigned)std::max<long long>(1, std::min<long long>(b, 65536));
}

template <typename T, int W>
void launch_tiles(Plan& P, const void* v, const CgState* st, hipStream_t s, bool gather) {
  const size_t lds = (size_t)P.max_padded * (gather ? sizeof(T) : sizeof(double));
  const long long LN = (long long)P.N * P.L;
  for (int g = 0; g < 3; ++g) {
    const int j0 = P.tjob_begin[g], nj = P.tjob_begin[g + 1] - j0;
    if (nj == 0) continue;
    if (!gather) {
      auto k = (g == 0) ? k_spread<T, W, 1> : (g == 1) ? k_spread<T, W, 2> : k_spread<T, W, 3>;
      if (lds > 65536) NLD_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(k, dim3(nj), dim3(kSpreadThreads), lds, s, P.d_wins, P.d_tjobs, j0, P.g_idx,
                         P.g_base, (const T*)P.g_frac, LN, (const T*)v, (T*)P.padded, P.slot_stride, st);
    } else {
      auto k = (g == 0) ? k_gather<T, W, 1> : (g == 1) ? k_gather<T, W, 2> : k_gather<T, W, 3>;
      if (lds > 65536) NLD_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(k, dim3(nj), dim3(kGatherThreads), lds, s, P.d_wins, P.d_tjobs, j0, P.g_idx,
                         P.g_base, (const T*)P.g_frac, (long long)P.N, LN, (const T*)P.grid,
                         (T*)P.ylocal, st);
    }
    NLD_HIP(hipGetLastError());
  }
}

template <typename T>
void tiles_dispatch(Plan& P, const void* v, const CgState* st, hipStream_t s, bool gather) {
  switch (P.wins[0].m) {
    case 1: launch_tiles<T, 2>(P, v, st, s, gather); break;
    case 2: launch_tiles<T, 4>(P, v, st, s, gather); break;
    case 3: launch_tiles<T, 6>(P, v, st, s, gather); break;
    case 4: launch_tiles<T, 8>(P, v, st, s, gather); break;
    case 5: launch_tiles<T, 10>(P, v, st, s, gather); break;
    case 6: launch_tiles<T, 12>(P, v, st, s, gather); break;
    case 7: launch_tiles<T, 14>(P, v, st, s, gather); break;
    case 8: launch_tiles<T, 16>(P, v, st, s, gather); break;
    default: throw std::invalid_argument("cutoff out of range");
  }
}

template <typename T>
void matvec_t(Plan& P, const void* v, void* out, Epilogue epi, const void* f, hipStream_t s) {
  const bool cg = (epi == EPI_CG_Q || epi == EPI_CG_INIT || epi == EPI_CG_TRUE);
  // only the iteration's product stops early once the solve has finished
  const CgState* st = (epi == EPI_CG_Q) ? P.st : nullptr;
  if (P.has_flat) {
    hipLaunchKernelGGL(k_sum<T>, dim3(1), dim3(1024), 0, s, (const T*)v, (long long)P.N, P.sumv, st);
    NLD_HIP(hipGetLastError());
  }
  tiles_dispatch<T>(P, v, st, s, false);
  if (P.n_fjobs > 0) {
    hipLaunchKernelGGL(k_fold<T>, dim3(P.n_fjobs), dim3(256), 0, s, P.d_wins, P.d_fjobs,
                       (const T*)P.padded, P.slot_stride, P.tile_slot0, P.tile_nslot, (T*)P.grid, st);
    NLD_HIP(hipGetLastError());
  }
  int n_max = 1;
  for (const auto& w : P.wins) n_max = std::max(n_max, w.n_max);
  for (int ax = 2; ax >= 0; --ax) {
    if (P.n_conv[ax] == 0) continue;
    const int lb = P.conv_lines[ax];
    const size_t lds = (size_t)(2 * (lb / 2) * n_max + n_max / 2 + 1) * 2 * sizeof(T);
    hipLaunchKernelGGL(k_conv<T>, dim3(P.n_conv[ax]), dim3(kConvThreads), lds, s, P.d_wins,
                       P.d_conv[ax], ax, lb, (T*)P.grid, st);
    NLD_HIP(hipGetLastError());
  }
  tiles_dispatch<T>(P, v, st, s, true);
  ReduceArgs a;
  a.yl = P.ylocal;
  a.wts = nullptr;
  a.L = P.L;
  a.N = P.N;
  a.v = v;
  a.out = out;
  a.Dout = (epi == EPI_DEGREE) ? (double*)out : nullptr;
  a.D = P.D;
  a.f = f;
  a.st = cg ? P.st : nullptr;
  a.red = P.red;
  a.sumv = P.sumv;
  a.mode = (int)epi;
  const unsigned nb = (epi >= EPI_CG_Q) ? red_blocks(P.N) : grid_for(P.N, kRedThreads);
  hipLaunchKernelGGL(k_reduce<T>, dim3(nb), dim3(kRedThreads), 0, s, P.d_wins, a);
  NLD_HIP(hipGetLastError());
}

}  // namespace

void matvec(Plan& P, const void* v, void* out, Epilogue epi, const void* f, hipStream_t s) {
  if (P.prec == NLD_FP32) matvec_t<float>(P, v, out, epi, f, s);
  else matvec_t<double>(P, v, out, epi, f, s);
}

}  // namespace nld
