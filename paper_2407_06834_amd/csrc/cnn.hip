// Warm-start network on the matrix cores: five 3x3 convolutions (in -> 32 -> 32 -> 32 -> 32 -> 1,
// ReLU between), BF16 activations and weights, FP32 accumulation, FP32 master weights, MSE
// loss and Adam.  The network predicts u0 = f + residual from (f, log alpha, log sigma_l); the
// paper's PCG then starts from u0.
//
// Layout: activations NHWC with 32 BF16 channels per pixel (64 bytes; unused channels are
// zero), so a pixel's channels are one contiguous vector.  A convolution is an implicit GEMM
// per 8 x 32 pixel tile: for each of the 9 taps, D^T[cout][pixels] += W_tap^T[cout][cin] *
// X_shift^T[cin][pixels] with v_mfma_f32_16x16x32_bf16 (16 output channels x 16 pixels x 32
// input channels per instruction; with the weights as the left operand a lane's accumulators
// are four consecutive channels of one pixel, one 8-byte store).  The input tile with its
// one-pixel halo is staged in LDS (80-byte pixel stride against bank conflicts); every wave
// keeps the 18 weight fragments of the layer in registers.  The backward pass to the input is the same kernel with the transposed, flipped
// weights and a ReLU-mask epilogue; the weight gradient contracts over pixels with both
// operands staged channel-major in LDS (three copies of the input tile shifted by -1, 0, +1
// columns keep every fragment read 16-byte aligned) and writes per-block partials that a
// second kernel sums in fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nld_cnn.h"
#include "nld_internal.h"

namespace nld {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int C = 32;          // channels of every stored activation
constexpr int TH = 8, TW = 32; // pixel tile
constexpr int HP = 40;         // LDS pixel stride of the forward tile (u16), 80 bytes
constexpr int kLayers = 5;

__device__ __forceinline__ unsigned short f2bf(float x) {
  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

enum Epi { EPI_RELU = 0, EPI_OUT = 1, EPI_MASK = 2 };

// Input channels (f, cond[0..nc-1], zeros) of every pixel; grid y is the image.
__global__ void k_cnn_input(const float* __restrict__ f, const float* __restrict__ cond, int nc,
                            long long hw, unsigned short* __restrict__ x) {
  const long long img = blockIdx.y;
  // every channel but f's is the same for all pixels of the image
  unsigned short v[C];
  for (int c = 1; c < C; ++c) v[c] = (c - 1 < nc) ? f2bf(cond[img * nc + c - 1]) : (unsigned short)0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < hw;
       i += (long long)gridDim.x * blockDim.x) {
    const long long p = img * hw + i;
    v[0] = f2bf(f[p]);
    u32x4* dst = reinterpret_cast<u32x4*>(x + p * C);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u32x4 w;
      w.x = v[8 * q] | ((unsigned)v[8 * q + 1] << 16);
      w.y = v[8 * q + 2] | ((unsigned)v[8 * q + 3] << 16);
      w.z = v[8 * q + 4] | ((unsigned)v[8 * q + 5] << 16);
      w.w = v[8 * q + 6] | ((unsigned)v[8 * q + 7] << 16);
      dst[q] = w;
    }
  }
}

// 3x3 convolution of one 8 x 32 tile of one image.  wt: [9][32 cout][32 cin] BF16.  COUT 32, or
// 16 with only channel 0 meaningful (last layer).  Epilogues: ReLU(acc + b) -> BF16; f + acc +
// b (channel 0) -> FP32 out; acc * (mask > 0) -> BF16.  FROM_IMG: the input channels are built
// while staging, from the image f and the nc conditioning values of each image (the channels
// k_cnn_input stores), so inference of the first layer reads 4 bytes per pixel instead of 64.
// Four waves per SIMD: the compiler then keeps the weight fragments and the accumulators in 123
// VGPRs (no AGPRs, no scratch) instead of 139 registers at three waves; five would spill.
template <int COUT, int EPI, bool FROM_IMG = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_conv(const unsigned short* __restrict__ x, const unsigned short* __restrict__ wt,
       const float* __restrict__ bias, int h, int w, unsigned short* __restrict__ y,
       float* __restrict__ yout, const float* __restrict__ f,
       const unsigned short* __restrict__ mask, const float* __restrict__ cond = nullptr,
       int nc = 0) {
  constexpr int NH = COUT / 16;
  __shared__ __attribute__((aligned(16))) unsigned short xs[(TH + 2) * (TW + 2) * HP];
  const int img = blockIdx.z;
  const int y0 = blockIdx.y * TH, x0 = blockIdx.x * TW;
  const long long ibase = (long long)img * h * w;
  // FROM_IMG: the image's four 16-byte channel chunks with f = 0 (channel 0 is set per pixel)
  __shared__ u32x4 cpat[4];
  if constexpr (FROM_IMG) {
    if (threadIdx.x < 4) {
      unsigned short ch[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = 8 * (int)threadIdx.x + i;
        ch[i] = (k >= 1 && k - 1 < nc) ? f2bf(cond[(long long)img * nc + k - 1]) : (unsigned short)0;
      }
      u32x4 v;
      v.x = ch[0] | ((unsigned)ch[1] << 16);
      v.y = ch[2] | ((unsigned)ch[3] << 16);
      v.z = ch[4] | ((unsigned)ch[5] << 16);
      v.w = ch[6] | ((unsigned)ch[7] << 16);
      cpat[threadIdx.x] = v;
    }
    __syncthreads();
  }
  // stage the halo tile: 10 x 34 pixels, 4 chunks of 16 bytes each
  for (int idx = threadIdx.x; idx < (TH + 2) * (TW + 2) * 4; idx += 256) {
    const int pl = idx >> 2, part = idx & 3;
    const int r = pl / (TW + 2), c = pl - r * (TW + 2);
    const int gy = y0 - 1 + r, gx = x0 - 1 + c;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (gy >= 0 && gy < h && gx >= 0 && gx < w) {
      if constexpr (FROM_IMG) {
        v = cpat[part];
        if (part == 0) v.x = (v.x & 0xffff0000u) | f2bf(f[ibase + (long long)gy * w + gx]);
      } else {
        v = *reinterpret_cast<const u32x4*>(x + (ibase + (long long)gy * w + gx) * C + part * 8);
      }
    }
    *reinterpret_cast<u32x4*>(xs + pl * HP + part * 8) = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, lr = lane & 15;
  // weight fragments: lane holds cout = 16 hh + lr, cin = 8 kq .. 8 kq + 7
  bf16x8 b[9][NH];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int hh = 0; hh < NH; ++hh)
      b[t][hh] = *reinterpret_cast<const bf16x8*>(wt + ((t * 32 + 16 * hh + lr) * 32 + 8 * kq));
  __syncthreads();
  f32x4 acc[4][NH];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int hh = 0; hh < NH; ++hh) acc[q][hh] = f32x4{0.f, 0.f, 0.f, 0.f};
  // wave: rows 2 wave and 2 wave + 1; fragment q = (row q / 2, 16 columns from 16 (q % 2))
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3, dx = t % 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 2 * wave + (q >> 1) + dy, c = 16 * (q & 1) + lr + dx;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(xs + (r * (TW + 2) + c) * HP + 8 * kq);
#pragma unroll
      for (int hh = 0; hh < NH; ++hh)
        acc[q][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[t][hh], a, acc[q][hh], 0, 0, 0);
    }
  }
  // the weights are the left operand, so lane holds D^T[cout 16 hh + 4 kq + j][pixel lr] of
  // each fragment: four consecutive output channels of one pixel, stored as 8 bytes
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gy = y0 + 2 * wave + (q >> 1);
    const int gx = x0 + 16 * (q & 1) + lr;
    if (gy >= h || gx >= w) continue;
    const long long p = ibase + (long long)gy * w + gx;
#pragma unroll
    for (int hh = 0; hh < NH; ++hh) {
      const int co = 16 * hh + 4 * kq;
      const f32x4 v = acc[q][hh];
      if constexpr (EPI == EPI_OUT) {
        if (co == 0) yout[p] = f[p] + v[0] + bias[0];
      } else {
        unsigned short o[4];
        if constexpr (EPI == EPI_RELU) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float z = v[j] + bias[co + j];
            o[j] = f2bf(z > 0.f ? z : 0.f);
          }
        } else {
          const uint2 mk = *reinterpret_cast<const uint2*>(mask + p * C + co);
          const unsigned short mv[4] = {(unsigned short)(mk.x & 0xffffu), (unsigned short)(mk.x >> 16),
                                        (unsigned short)(mk.y & 0xffffu), (unsigned short)(mk.y >> 16)};
#pragma unroll
          for (int j = 0; j < 4; ++j) o[j] = bf2f(mv[j]) > 0.f ? f2bf(v[j]) : (unsigned short)0;
        }
        uint2 st;
        st.x = o[0] | ((unsigned)o[1] << 16);
        st.y = o[2] | ((unsigned)o[3] << 16);
        *reinterpret_cast<uint2*>(y + p * C + co) = st;
      }
    }
  }
}

// Weight gradient of one tile: dW[t][cout][cin] += sum_px dZ[px][cout] X[px + off_t][cin]
// (per-block partial), and db[cout] += sum_px dZ[px][cout].
constexpr int ZS = TH * TW + 8;            // cout stride of the staged dZ^T (u16)
constexpr int XSR = (TH + 2) * TW;         // one shifted copy: 10 rows x 32 px per channel
constexpr int XS = XSR + 8;                // cin stride (u16)
constexpr int kPart = 9 * C * C + C;       // floats per block partial
static_assert(C * TH == 256, "bias gradient assumes one thread per (channel, row)");

__global__ void __launch_bounds__(256)
k_conv_dw(const unsigned short* __restrict__ x, const unsigned short* __restrict__ dz, int h,
          int w, float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned short sm[];
  unsigned short* zt = sm;                       // [32 cout][ZS]
  unsigned short* xt = sm + C * ZS;              // [3 shifts][32 cin][XS]
  const int img = blockIdx.z;
  const int y0 = blockIdx.y * TH, x0 = blockIdx.x * TW;
  const long long ibase = (long long)img * h * w;
  const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  // dZ^T: one pixel's 32 channels per thread
  {
    const int pl = threadIdx.x;                  // 256 pixels of the tile
    const int r = pl / TW, c = pl % TW;
    const int gy = y0 + r, gx = x0 + c;
    unsigned short v[C];
    if (gy < h && gx < w) {
      const u32x4* src = reinterpret_cast<const u32x4*>(dz + (ibase + (long long)gy * w + gx) * C);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u32x4 u = src[q];
        v[8 * q] = u.x & 0xffff; v[8 * q + 1] = u.x >> 16;
        v[8 * q + 2] = u.y & 0xffff; v[8 * q + 3] = u.y >> 16;
        v[8 * q + 4] = u.z & 0xffff; v[8 * q + 5] = u.z >> 16;
        v[8 * q + 6] = u.w & 0xffff; v[8 * q + 7] = u.w >> 16;
      }
    } else {
#pragma unroll
      for (int k = 0; k < C; ++k) v[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) zt[k * ZS + pl] = v[k];
  }
  // X^T shifted by s - 1 columns: xt[s][ci][hr * 32 + c] = X[y0 - 1 + hr][x0 + c + s - 1][ci]
  for (int idx = threadIdx.x; idx < (TH + 2) * (TW + 2); idx += 256) {
    const int hr = idx / (TW + 2), hc = idx % (TW + 2);   // halo column hc <-> x0 - 1 + hc
    const int gy = y0 - 1 + hr, gx = x0 - 1 + hc;
    unsigned short v[C];
    if (gy >= 0 && gy < h && gx >= 0 && gx < w) {
      const u32x4* src = reinterpret_cast<const u32x4*>(x + (ibase + (long long)gy * w + gx) * C);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u32x4 u = src[q];
        v[8 * q] = u.x & 0xffff; v[8 * q + 1] = u.x >> 16;
        v[8 * q + 2] = u.y & 0xffff; v[8 * q + 3] = u.y >> 16;
        v[8 * q + 4] = u.z & 0xffff; v[8 * q + 5] = u.z >> 16;
        v[8 * q + 6] = u.w & 0xffff; v[8 * q + 7] = u.w >> 16;
      }
    } else {
#pragma unroll
      for (int k = 0; k < C; ++k) v[k] = 0;
    }
    // column c of shift s reads halo column c + s
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int c = hc - s;
      if (c < 0 || c >= TW) continue;
#pragma unroll
      for (int k = 0; k < C; ++k) xt[(s * C + k) * XS + hr * TW + c] = v[k];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, lr = lane & 15;
  // 36 output fragments (tap, cout half, cin half); wave takes q = wave + 4 i
  f32x4 acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int q = wave + 4 * i;
    const int t = q >> 2, hco = (q >> 1) & 1, hci = q & 1;
    const int dy = t / 3, dx = t % 3;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(zt + (16 * hco + lr) * ZS + r * TW + 8 * kq);
      const bf16x8 bb = *reinterpret_cast<const bf16x8*>(
          xt + (dx * C + 16 * hci + lr) * XS + (r + dy) * TW + 8 * kq);
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[i], 0, 0, 0);
    }
  }
  float* out = part + blk * kPart;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int q = wave + 4 * i;
    const int t = q >> 2, hco = (q >> 1) & 1, hci = q & 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = 16 * hco + 4 * kq + j, ci = 16 * hci + lr;
      out[(t * C + co) * C + ci] = acc[i][j];
    }
  }
  // bias gradient: thread (cout, row) sums one row of the tile, then row sums in order
  __shared__ float sb[C * TH];
  {
    const int co = threadIdx.x / TH, r = threadIdx.x % TH;   // C * TH == 256 threads
    float sacc = 0.f;
    for (int c = 0; c < TW; ++c) sacc += bf2f(zt[co * ZS + r * TW + c]);
    sb[threadIdx.x] = sacc;
  }
  __syncthreads();
  if (threadIdx.x < C) {
    float tsum = 0.f;
    for (int k = 0; k < TH; ++k) tsum += sb[threadIdx.x * TH + k];
    out[9 * C * C + threadIdx.x] = tsum;
  }
}

// Sum of the per-block partials in block order, then the layer's gradient in the flat order
// (W[cout][cin][3][3], b[cout]) for the real channel counts.
__global__ void k_dw_reduce(const float* __restrict__ part, long long nblk, int cout, int cin,
                            float* __restrict__ grad) {
  const int nw = cout * cin * 9;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nw + cout; k += gridDim.x * blockDim.x) {
    int src;
    if (k < nw) {
      const int co = k / (cin * 9), rem = k % (cin * 9), ci = rem / 9, t = rem % 9;
      src = (t * C + co) * C + ci;
    } else {
      src = 9 * C * C + (k - nw);
    }
    float s = 0.f;
    for (long long b = 0; b < nblk; ++b) s += part[b * kPart + src];
    grad[k] = s;
  }
}

// MSE: per-block FP64 partial sums of (u0 - t)^2 and the gradient 2 (u0 - t) / count packed as
// channel 0 of a 32-channel BF16 tensor.
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ u0, const float* __restrict__ tgt, long long total, double inv_count,
      unsigned short* __restrict__ dz, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long p = blockIdx.x * 256LL + threadIdx.x; p < total; p += (long long)gridDim.x * 256) {
    const double e = (double)u0[p] - (double)tgt[p];
    s += e * e;
    u32x4* dst = reinterpret_cast<u32x4*>(dz + p * C);
    u32x4 z = {0u, 0u, 0u, 0u};
    u32x4 first = z;
    first.x = f2bf((float)(2.0 * e * inv_count));
    dst[0] = first;
    dst[1] = z;
    dst[2] = z;
    dst[3] = z;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// BF16 kernel weights of every layer from the FP32 master parameters: forward [9][co][ci] and
// transposed-flipped [9][ci][co] (zero outside the real channels).
__global__ void k_pack_weights(const float* __restrict__ theta, int off, int cout, int cin,
                               unsigned short* __restrict__ wf, unsigned short* __restrict__ wb) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 9 * C * C; k += gridDim.x * blockDim.x) {
    const int t = k / (C * C), a = (k / C) % C, bq = k % C;
    // forward: a = cout, bq = cin
    float vf = 0.f;
    if (a < cout && bq < cin) vf = theta[off + (a * cin + bq) * 9 + t];
    wf[k] = f2bf(vf);
    // transposed: output channel a = original cin, input channel bq = original cout, tap 8 - t
    float vb = 0.f;
    if (bq < cout && a < cin) vb = theta[off + (bq * cin + a) * 9 + (8 - t)];
    wb[k] = f2bf(vb);
  }
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace

// ---------------------------------------------------------------------------- network object
struct Cnn {
  int cin = 0;                  // real input channels (1 + conditioning)
  int cout[kLayers], cinl[kLayers], off[kLayers];
  long long nparam = 0;
  float* theta = nullptr;       // FP32 master parameters (flat, oracle order)
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  long long step = 0;
  unsigned short* wf = nullptr; // [5][9][32][32] forward BF16 weights
  unsigned short* wb = nullptr; // [5][9][32][32] transposed-flipped
  float* bias = nullptr;        // [5][32] (layer-padded copy of the biases)
  bool packed = false;
  // activation buffers, grown on demand (pixels)
  long long cap = 0;
  unsigned short* act[kLayers] = {};   // act[0] input, act[k] output of layer k (k = 1..4)
  unsigned short* dzA = nullptr;
  unsigned short* dzB = nullptr;
  float* u0 = nullptr;
  float* cond = nullptr;
  int cond_cap = 0;
  float* part = nullptr;
  long long part_cap = 0;
  double* lpart = nullptr;
};

namespace {

template <typename X>
void grow(X*& p, long long& cap, long long need) {
  if (need <= cap) return;
  if (p) (void)hipFree(p);
  p = nullptr;
  NLD_HIP(hipMalloc((void**)&p, (size_t)need * sizeof(X)));
  cap = need;
}

void ensure(Cnn& net, long long px, int n, long long tiles) {
  if (px > net.cap) {
    for (auto& a : net.act) {
      if (a) (void)hipFree(a);
      a = nullptr;
    }
    for (unsigned short** a : {&net.dzA, &net.dzB}) {
      if (*a) (void)hipFree(*a);
      *a = nullptr;
    }
    if (net.u0) (void)hipFree(net.u0);
    for (auto& a : net.act) NLD_HIP(hipMalloc((void**)&a, (size_t)px * C * 2));
    NLD_HIP(hipMalloc((void**)&net.dzA, (size_t)px * C * 2));
    NLD_HIP(hipMalloc((void**)&net.dzB, (size_t)px * C * 2));
    NLD_HIP(hipMalloc((void**)&net.u0, (size_t)px * sizeof(float)));
    net.cap = px;
  }
  if (n * (net.cin - 1) > net.cond_cap) {
    if (net.cond) (void)hipFree(net.cond);
    net.cond_cap = n * (net.cin - 1);
    NLD_HIP(hipMalloc((void**)&net.cond, (size_t)std::max(1, net.cond_cap) * sizeof(float)));
  }
  grow(net.part, net.part_cap, tiles * kPart);
}

void pack(Cnn& net, hipStream_t s) {
  if (net.packed) return;
  for (int k = 0; k < kLayers; ++k) {
    hipLaunchKernelGGL(k_pack_weights, dim3(36), dim3(256), 0, s, net.theta, net.off[k], net.cout[k],
                       net.cinl[k], net.wf + (size_t)k * 9 * C * C, net.wb + (size_t)k * 9 * C * C);
    // biases: padded copy
    NLD_HIP(hipMemsetAsync(net.bias + k * C, 0, C * sizeof(float), s));
    NLD_HIP(hipMemcpyAsync(net.bias + k * C, net.theta + net.off[k] + net.cout[k] * net.cinl[k] * 9,
                           net.cout[k] * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  NLD_HIP(hipGetLastError());
  net.packed = true;
}

dim3 tiles_of(int n, int h, int w) { return dim3((w + TW - 1) / TW, (h + TH - 1) / TH, n); }

void forward(Cnn& net, const float* f, const float* cond_host, int n, int h, int w, hipStream_t s,
             bool keep_input) {
  const long long px = (long long)n * h * w;
  const dim3 g = tiles_of(n, h, w);
  ensure(net, px, n, (long long)g.x * g.y * g.z);
  pack(net, s);
  const int nc = net.cin - 1;
  if (nc > 0)
    NLD_HIP(hipMemcpyAsync(net.cond, cond_host, (size_t)n * nc * sizeof(float), hipMemcpyHostToDevice, s));
  const long long hw = (long long)h * w;
  const unsigned nb = (unsigned)std::max<long long>(1, std::min<long long>(65536 / n, (hw + 255) / 256));
  // the weight gradient of the first layer needs its stored input; inference builds it on the fly
  if (keep_input)
    hipLaunchKernelGGL(k_cnn_input, dim3(nb, n), dim3(256), 0, s, f, net.cond, nc, hw, net.act[0]);
  else
    hipLaunchKernelGGL((k_conv<32, EPI_RELU, true>), g, dim3(256), 0, s, nullptr, net.wf,
                       net.bias, h, w, net.act[1], nullptr, f, nullptr, (const float*)net.cond, nc);
  for (int k = keep_input ? 0 : 1; k < kLayers - 1; ++k)
    hipLaunchKernelGGL((k_conv<32, EPI_RELU>), g, dim3(256), 0, s, net.act[k],
                       net.wf + (size_t)k * 9 * C * C, net.bias + k * C, h, w, net.act[k + 1],
                       nullptr, nullptr, nullptr);
  hipLaunchKernelGGL((k_conv<16, EPI_OUT>), g, dim3(256), 0, s, net.act[kLayers - 1],
                     net.wf + (size_t)(kLayers - 1) * 9 * C * C, net.bias + (kLayers - 1) * C, h, w,
                     nullptr, net.u0, f, nullptr);
  NLD_HIP(hipGetLastError());
}

}  // namespace

void cnn_backward(Cnn& net, const float* target, int n, int h, int w, double* loss, hipStream_t s) {
  const long long px = (long long)n * h * w;
  const dim3 g = tiles_of(n, h, w);
  const long long nblk = (long long)g.x * g.y * g.z;
  const unsigned nb = (unsigned)std::min<long long>(1024, (px + 255) / 256);
  if (!net.lpart) NLD_HIP(hipMalloc((void**)&net.lpart, 1024 * sizeof(double)));
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, net.u0, target, px, 1.0 / (double)px, net.dzA,
                     net.lpart);
  NLD_HIP(hipGetLastError());
  const size_t dw_lds = (size_t)(C * ZS + 3 * C * XS) * sizeof(unsigned short);
  NLD_HIP(hipFuncSetAttribute((const void*)k_conv_dw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dw_lds));
  unsigned short* dz = net.dzA;
  unsigned short* other = net.dzB;
  for (int k = kLayers - 1; k >= 0; --k) {
    hipLaunchKernelGGL(k_conv_dw, g, dim3(256), dw_lds, s, net.act[k], dz, h, w, net.part);
    hipLaunchKernelGGL(k_dw_reduce, dim3(64), dim3(256), 0, s, net.part, nblk, net.cout[k], net.cinl[k],
                       net.grad + net.off[k]);
    if (k > 0) {
      // gradient to the previous layer's output, masked by its ReLU
      hipLaunchKernelGGL((k_conv<32, EPI_MASK>), g, dim3(256), 0, s, dz, net.wb + (size_t)k * 9 * C * C,
                         net.bias, h, w, other, nullptr, nullptr, net.act[k]);
      std::swap(dz, other);
    }
    NLD_HIP(hipGetLastError());
  }
  std::vector<double> lp(nb);
  NLD_HIP(hipMemcpyAsync(lp.data(), net.lpart, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  NLD_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (double v : lp) acc += v;
  *loss = acc / (double)px;
}

}  // namespace nld

// ---------------------------------------------------------------------------- C ABI
struct nld_cnn_s {
  nld::Cnn net;
};

namespace {
nld_status cnn_fail(nld_status st, const std::string& msg) {
  nld::set_error(msg);
  return st;
}
template <typename F>
nld_status cnn_guard(const char* name, F&& body) {
  try {
    body();
    return NLD_OK;
  } catch (const nld::HipError& e) {
    return cnn_fail(NLD_E_HIP, std::string(name) + ": " + e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    return cnn_fail(NLD_E_NOMEM, std::string(name) + ": host allocation failed");
  } catch (const std::exception& e) {
    return cnn_fail(NLD_E_STATE, std::string(name) + ": " + e.what());
  }
}
bool shape_ok(int n, int h, int w) {
  return n >= 1 && h >= 1 && w >= 1 && (long long)n * h * w <= (1LL << 31) && n <= 65535;
}
}  // namespace

extern "C" {

nld_status cnn_create(nld_cnn_t* out, int32_t n_cond, uint64_t seed) {
  if (!out) return cnn_fail(NLD_E_INVAL, "cnn_create: null pointer");
  *out = nullptr;
  if (n_cond < 0 || n_cond > 31) return cnn_fail(NLD_E_INVAL, "cnn_create: n_cond must be in [0, 31]");
  nld_cnn_s* h = new nld_cnn_s();
  nld::Cnn& net = h->net;
  nld_status st = cnn_guard("cnn_create", [&] {
    net.cin = 1 + n_cond;
    int c = net.cin;
    long long o = 0;
    for (int k = 0; k < nld::kLayers; ++k) {
      net.cinl[k] = c;
      net.cout[k] = (k == nld::kLayers - 1) ? 1 : nld::C;
      net.off[k] = (int)o;
      o += (long long)net.cout[k] * c * 9 + net.cout[k];
      c = net.cout[k];
    }
    net.nparam = o;
    // He initialisation (normal, std sqrt(2 / (9 cin))), zero biases, last layer scaled by 0.1
    std::vector<float> th((size_t)o, 0.f);
    std::mt19937_64 rng(seed);
    for (int k = 0; k < nld::kLayers; ++k) {
      std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (9.0 * net.cinl[k])));
      const double sc = (k == nld::kLayers - 1) ? 0.1 : 1.0;
      for (long long i = 0; i < (long long)net.cout[k] * net.cinl[k] * 9; ++i)
        th[(size_t)(net.off[k] + i)] = (float)(sc * nd(rng));
    }
    NLD_HIP(hipMalloc((void**)&net.theta, o * sizeof(float)));
    NLD_HIP(hipMalloc((void**)&net.grad, o * sizeof(float)));
    NLD_HIP(hipMalloc((void**)&net.adam_m, o * sizeof(float)));
    NLD_HIP(hipMalloc((void**)&net.adam_v, o * sizeof(float)));
    NLD_HIP(hipMalloc((void**)&net.wf, (size_t)nld::kLayers * 9 * nld::C * nld::C * 2));
    NLD_HIP(hipMalloc((void**)&net.wb, (size_t)nld::kLayers * 9 * nld::C * nld::C * 2));
    NLD_HIP(hipMalloc((void**)&net.bias, (size_t)nld::kLayers * nld::C * sizeof(float)));
    NLD_HIP(hipMemcpy(net.theta, th.data(), o * sizeof(float), hipMemcpyHostToDevice));
    NLD_HIP(hipMemset(net.grad, 0, o * sizeof(float)));
    NLD_HIP(hipMemset(net.adam_m, 0, o * sizeof(float)));
    NLD_HIP(hipMemset(net.adam_v, 0, o * sizeof(float)));
  });
  if (st != NLD_OK) {
    cnn_destroy(h);
    return st;
  }
  *out = h;
  return NLD_OK;
}

nld_status cnn_destroy(nld_cnn_t h) {
  if (!h) return cnn_fail(NLD_E_INVAL, "cnn_destroy: null network");
  nld::Cnn& n = h->net;
  (void)hipDeviceSynchronize();
  void* bufs[] = {n.theta, n.grad, n.adam_m, n.adam_v, n.wf, n.wb, n.bias, n.dzA, n.dzB, n.u0,
                  n.cond, n.part, n.lpart, n.act[0], n.act[1], n.act[2], n.act[3], n.act[4]};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete h;
  return NLD_OK;
}

int64_t cnn_param_count(nld_cnn_t h) { return h ? h->net.nparam : -1; }

nld_status cnn_get_params(nld_cnn_t h, float* theta, float* grad) {
  if (!h || (!theta && !grad)) return cnn_fail(NLD_E_INVAL, "cnn_get_params: null pointer");
  return cnn_guard("cnn_get_params", [&] {
    NLD_HIP(hipDeviceSynchronize());
    if (theta) NLD_HIP(hipMemcpy(theta, h->net.theta, h->net.nparam * sizeof(float), hipMemcpyDeviceToHost));
    if (grad) NLD_HIP(hipMemcpy(grad, h->net.grad, h->net.nparam * sizeof(float), hipMemcpyDeviceToHost));
  });
}

nld_status cnn_set_params(nld_cnn_t h, const float* theta) {
  if (!h || !theta) return cnn_fail(NLD_E_INVAL, "cnn_set_params: null pointer");
  for (long long i = 0; i < h->net.nparam; ++i)
    if (!std::isfinite(theta[i])) return cnn_fail(NLD_E_INVAL, "cnn_set_params: non-finite parameter");
  return cnn_guard("cnn_set_params", [&] {
    NLD_HIP(hipDeviceSynchronize());
    NLD_HIP(hipMemcpy(h->net.theta, theta, h->net.nparam * sizeof(float), hipMemcpyHostToDevice));
    h->net.packed = false;
  });
}

nld_status cnn_predict(nld_cnn_t h, const float* f, const float* cond, int32_t n, int32_t hh,
                       int32_t w, float* u0, hipStream_t s) {
  if (!h || !f || !u0 || (!cond && h->net.cin > 1)) return cnn_fail(NLD_E_INVAL, "cnn_predict: null pointer");
  if (!shape_ok(n, hh, w)) return cnn_fail(NLD_E_INVAL, "cnn_predict: bad shape");
  return cnn_guard("cnn_predict", [&] {
    nld::forward(h->net, f, cond, n, hh, w, s, false);
    NLD_HIP(hipMemcpyAsync(u0, h->net.u0, (size_t)n * hh * w * sizeof(float), hipMemcpyDeviceToDevice, s));
    NLD_HIP(hipStreamSynchronize(s));
  });
}

nld_status cnn_loss_grad(nld_cnn_t h, const float* f, const float* cond, const float* target,
                         int32_t n, int32_t hh, int32_t w, double* loss, hipStream_t s) {
  if (!h || !f || !target || !loss || (!cond && h->net.cin > 1))
    return cnn_fail(NLD_E_INVAL, "cnn_loss_grad: null pointer");
  if (!shape_ok(n, hh, w)) return cnn_fail(NLD_E_INVAL, "cnn_loss_grad: bad shape");
  return cnn_guard("cnn_loss_grad", [&] {
    nld::forward(h->net, f, cond, n, hh, w, s, true);
    nld::cnn_backward(h->net, target, n, hh, w, loss, s);
  });
}

nld_status cnn_adam_step(nld_cnn_t h, const nld_adam* opt, hipStream_t s) {
  if (!h || !opt) return cnn_fail(NLD_E_INVAL, "cnn_adam_step: null pointer");
  if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) ||
      !(opt->beta2 >= 0.f && opt->beta2 < 1.f) || !(opt->eps >= 0.f))
    return cnn_fail(NLD_E_INVAL, "cnn_adam_step: bad hyper-parameters");
  return cnn_guard("cnn_adam_step", [&] {
    nld::Cnn& net = h->net;
    net.step += 1;
    const float c1 = 1.f - std::pow(opt->beta1, (float)net.step);
    const float c2 = 1.f - std::pow(opt->beta2, (float)net.step);
    hipLaunchKernelGGL(nld::k_adam, dim3(128), dim3(256), 0, s, net.theta, net.grad, net.adam_m,
                       net.adam_v, net.nparam, opt->lr, opt->beta1, opt->beta2, opt->eps, c1, c2);
    NLD_HIP(hipGetLastError());
    net.packed = false;
  });
}

}  // extern "C"
