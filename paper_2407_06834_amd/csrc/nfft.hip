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
#include <cstdlib>
#include <type_traits>
#include <utility>
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

// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{})
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// Slot layout.  Along each dimension a padded tile of pe = ts + 2m - 1 cells splits into the
// m - 1 cells that fold into the left neighbour tile, the ts cells of the tile itself and the
// m cells that fold into the right neighbour (an unused dimension: one cell, one part).  A slot
// stores the 27 blocks these parts form one after the other (lexicographic order of the parts,
// cells row-major inside a block), so that the fold reads each block it needs as one
// contiguous range instead of short pieces of many padded rows.
struct SlotPart {
  int pre, sz;   // first padded index and extent of the part that holds padded index x
};
__device__ __forceinline__ SlotPart slot_part(int x, int a, int b, int pe) {
  return x < a ? SlotPart{0, a} : (x < a + b ? SlotPart{a, b} : SlotPart{a + b, pe - a - b});
}
__device__ __forceinline__ int slot_index(const WinDev& w, int x0, int x1, int x2) {
  const int a0 = w.taps[0] > 1 ? w.m - 1 : 0, a1 = w.taps[1] > 1 ? w.m - 1 : 0,
            a2 = w.taps[2] > 1 ? w.m - 1 : 0;
  const SlotPart q0 = slot_part(x0, a0, w.ts[0], w.pe[0]);
  const SlotPart q1 = slot_part(x1, a1, w.ts[1], w.pe[1]);
  const SlotPart q2 = slot_part(x2, a2, w.ts[2], w.pe[2]);
  const int pe1 = w.pe[1], pe2 = w.pe[2];
  return q0.pre * pe1 * pe2 + q0.sz * (q1.pre * pe2 + q1.sz * q2.pre) +
         ((x0 - q0.pre) * q1.sz + (x1 - q1.pre)) * q2.sz + (x2 - q2.pre);
}


// ---------------------------------------------------------------------------- window polynomial
// Pointers with an explicit address space: global (vector loads without the flat-address
// check) and constant (uniform data the compiler may read with scalar loads).
template <typename T> using GlobalPtr = const T __attribute__((address_space(1)))*;
template <typename T> using ConstPtr = const T __attribute__((address_space(4)))*;
template <typename T> using LdsPtr = const T __attribute__((address_space(3)))*;

template <typename T, int K, typename P>
__device__ __forceinline__ T horner(P c, T x) {
  T r = c[K - 1];
#pragma unroll
  for (int k = K - 2; k >= 0; --k) r = r * x + c[k];
  return r;
}

__device__ __forceinline__ unsigned lane_bcast(unsigned v, int q) {
  return (unsigned)__builtin_amdgcn_readlane((int)v, q);
}
__device__ __forceinline__ float lane_bcast(float v, int q) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
}
__device__ __forceinline__ double lane_bcast(double v, int q) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), q);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), q);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Value of v in the lane whose index is byte_addr / 4 (ds_bpermute; no LDS storage is used)
__device__ __forceinline__ float lane_fetch(float v, int byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(double v, int byte_addr) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(bits & 0xffffffffLL));
  const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// acc[i] += w(lane i of this lane's row of 16) * b for i < W (W = 6 or 8): the row broadcast
// (DPP row_newbcast) is part of each FMA, so no readlane or separate move is issued.  The
// leading s_nop covers the two wait states a DPP read needs after a VALU write of its source.
// Same single-rounding FMA as fmaf(b, w_i, acc[i]).
template <int W>
__device__ __forceinline__ void fmac_row_bcast(float (&acc)[W], float w, float b) {
  static_assert(W == 6 || W == 8, "row broadcast FMAs for 6 or 8 taps");
  if constexpr (W == 8) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %8, %9 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %8, %9 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %8, %9 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %8, %9 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %8, %9 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, %8, %9 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %8, %9 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, %8, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
          "+v"(acc[6]), "+v"(acc[7])
        : "v"(w), "v"(b));
  } else {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %6, %7 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %7 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %6, %7 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %6, %7 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %6, %7 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, %6, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5])
        : "v"(w), "v"(b));
  }
}

// Weights of the W = 2m taps of one node in one dimension (tap i at cell floor(u) - m + 1 + i,
// distance fr + m - 1 - i): the per-tap window polynomials evaluated at x = 2 fr - 1.
template <typename T, int W, typename P>
__device__ __forceinline__ void poly_row(P psi, T fr, T* wt) {
  constexpr int K = PsiDeg<T>::value + 1;
  const T x = (T)2 * fr - (T)1;
#pragma unroll
  for (int i = 0; i < W; ++i) wt[i] = horner<T, K>(psi + i * K, x);
}

// ---------------------------------------------------------------------------- spreading
// One workgroup (4 wavefronts) per chunk (<= 4096) of a tile's nodes, which the plan sorted by
// tile and then by cell, so nodes sharing a grid cell are consecutive ("runs").  A wavefront
// walks its quarter of the chunk one node at a time; lane l owns the tap pair (i1, i2) of the
// last two kept dimensions and keeps the 2m taps of the first kept dimension in registers, so a
// run of r nodes costs one set of LDS additions instead of r.  When the cell changes the
// registers are added into the padded tile (tile plus the 2m - 1 halo cells the taps reach) as
// fixed-point integers (2^e <= sum |v| over the chunk; FP32 data: a 32-bit word scaled by
// 2^(29 - e) plus a 32-bit remainder word 2^20 finer, FP64 data: one 64-bit word scaled by
// 2^(61 - e)): integer addition is exact and associative, so the result does not depend on the
// order in which the wavefronts add (reproducible), and ds_add_u32 / ds_add_u64 are fast where
// LDS float atomics are not.  (Packing the two FP32 words into one 64-bit add measured slower:
// the lanes' 8-byte addresses meet in fewer LDS banks.)
// The slot is then written back in the working precision, in the slot layout above; the fold
// kernel sums the slots that cover each grid cell.
// TSC = 8: every 3-D window of the launch has 8^3 tiles, so the padded extents and strides are
// compile-time constants (LDS offsets fold into the instructions); TSC = 0 reads them from the
// window descriptor.
template <typename T, int W, int TD, int TSC>
__global__ void __launch_bounds__(kSpreadThreads)
k_spread(const WinDev* __restrict__ wins, const TileJob* __restrict__ jobs, int job0,
         const ImgDev* __restrict__ imgs, VecArg in, int check) {
  const TileJob job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  const ImgDev& im = imgs[w.img];
  if (check && im.st->done) return;
  GlobalPtr<T> v = (GlobalPtr<T>)vin<T>(im, in);
  GlobalPtr<int> g_idx = (GlobalPtr<int>)w.g_idx;
  GlobalPtr<unsigned> g_base = (GlobalPtr<unsigned>)w.g_base;
  GlobalPtr<T> g_frac = (GlobalPtr<T>)w.g_frac;
  const long long LN = w.LN;
  T __attribute__((address_space(1)))* padded = (T __attribute__((address_space(1)))*)w.padded;
  const long long slot_stride = w.slot_stride;
  constexpr int K = PsiDeg<T>::value + 1;
  constexpr int PAIRS = (TD == 1) ? W : W * W;
  constexpr int NP = (PAIRS + 63) / 64;
  constexpr int NI0 = (TD == 3) ? W : 1;
  // Fixed-point accumulators with scale 2^(kFix - e), 2^e <= sum |v| over the chunk.  FP64
  // data: one 64-bit word (resolution 2^-61 of sum |v|).  FP32 data: two 32-bit words per
  // cell, the rounded value and its remainder in units of 2^-20 (resolution 2^-49 of sum |v|),
  // so that the spreading stays far more accurate than FP32 rounding of the result (the
  // product then stays symmetric to working precision, which CG in FP32 needs).
  using Acc = typename std::conditional<sizeof(T) == 4, unsigned int, unsigned long long>::type;
  using SAcc = typename std::conditional<sizeof(T) == 4, int, long long>::type;
  constexpr int kFix = sizeof(T) == 4 ? 29 : 61;
  constexpr bool kTwo = sizeof(T) == 4;
  constexpr float kLoScale = 1048576.0f;                 // 2^20
  extern __shared__ unsigned char smem_raw[];
  Acc* acc = reinterpret_cast<Acc*>(smem_raw);
  Acc* acc_lo = acc + (kTwo ? w.pe[0] * w.pe[1] * w.pe[2] : 0);
  __shared__ double s_part[kSpreadWaves];
  constexpr int PEC = (TD == 3 && TSC > 0) ? TSC + W - 1 : 0;
  const int pe1 = PEC ? PEC : w.pe[1], pe2 = PEC ? PEC : w.pe[2];
  const int cells = PEC ? PEC * PEC * PEC : w.pe[0] * pe1 * pe2;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
  GlobalPtr<T> psi = (GlobalPtr<T>)w.psi;
  for (int c = threadIdx.x; c < cells; c += kSpreadThreads) {
    acc[c] = (Acc)0;
    if constexpr (kTwo) acc_lo[c] = (Acc)0;
  }
  // fixed-point scale of this chunk: 2^e <= sum |v| over its nodes.  The row-broadcast path
  // (kDpp below) loads the values of all of a wavefront's rounds here, all loads in flight, and
  // keeps them in registers for its node loop; the generic path sums them in a separate pass.
  const int npts = job.pend - job.pbeg;
  const int per = (npts + kSpreadWaves - 1) / kSpreadWaves;
  const int q0 = job.pbeg + wave * per, q1 = min(job.pend, q0 + per);
  constexpr bool kDppV = TD == 3 && (W == 6 || W == 8) && sizeof(T) == 4;
  constexpr int kRounds = kMaxChunk / (64 * kSpreadWaves);
  static_assert(kMaxChunk % (64 * kSpreadWaves) == 0, "whole rounds per wavefront");
  float vreg[kDppV ? kRounds : 1];
  double sa = 0.0;
  if constexpr (kDppV) {
    int ireg[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int p = q0 + 64 * r + lane;
      ireg[r] = p < q1 ? g_idx[p] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) vreg[r] = (q0 + 64 * r + lane < q1) ? (float)v[ireg[r]] : 0.0f;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) sa += fabs((double)vreg[r]);
  } else {
    for (int p = job.pbeg + threadIdx.x; p < job.pend; p += kSpreadThreads)
      sa += fabs((double)v[g_idx[p]]);
  }
  for (int off = 32; off > 0; off >>= 1) sa += __shfl_xor(sa, off);
  if (lane == 0) s_part[wave] = sa;
  __syncthreads();
  double tot = 0.0;
  for (int k = 0; k < kSpreadWaves; ++k) tot += s_part[k];
  auto out = padded + (long long)job.slot * slot_stride;
  if (!(tot > 0.0)) {
    for (int c = threadIdx.x; c < cells; c += kSpreadThreads) out[c] = (T)0;
    return;
  }
  // |cell| <= sum |v| < 2^(e + 1): scaled values stay below 2^(kFix + 1)
  const int e = max(ilogb(tot), -90);
  const double scale = ldexp(1.0, kFix - e);
  const T scale_t = (T)scale;
  // Tap weights: lanes [0, W) evaluate the window polynomial of the first kept dimension's taps,
  // [W, 2W) the second's, [2W, 3W) the third's (one polynomial per lane and node); the lane that
  // owns tap pair (i1, i2) of the last two dimensions fetches its two factors with ds_bpermute,
  // and the first dimension's W weights are broadcast to every lane.
  // FP32, 3 kept dimensions, W = 6 or 8 taps (m = 3 or 4): every row of 16 lanes holds the
  // first dimension's weights in its lanes 0..W-1 (the row broadcast of fmac_row_bcast reads
  // them there); lanes 8..8+W-1 hold the second dimension's in rows 0 and 2 and the third's in
  // rows 1 and 3 (lanes of a row past W evaluate the last tap's polynomial, unused).  A node's
  // x = 2 f - 1 per dimension and its scaled value are staged per wavefront in LDS.  The
  // polynomials of two consecutive nodes are evaluated in one pass (one per half wavefront).
  constexpr bool kDpp = TD == 3 && (W == 6 || W == 8) && sizeof(T) == 4;
  __shared__ float4 s_stage[kDpp ? kSpreadWaves * 64 : 1];
  static_assert(TD * W <= 64, "one lane per tap and dimension");
  const int my_tap = kDpp ? min(lane & 7, W - 1) : lane % W;
  const int my_dim = kDpp ? ((lane & 8) ? 1 + ((lane >> 4) & 1) : 0)
                          : lane / W;               // lanes with my_dim >= TD idle here
  // x = 2 f - 1 of this lane's dimension as three FMAs with per-lane factors 2 or 0 (a node's
  // fractions are wave-uniform scalars): the same rounding as 2 f - 1, no selects
  const T sel0 = my_dim == 0 ? (T)2 : (T)0, sel1 = my_dim == 1 ? (T)2 : (T)0,
          sel2 = my_dim == 2 ? (T)2 : (T)0;
  T cf[K];
#pragma unroll
  for (int q = 0; q < K; ++q) cf[q] = psi[my_tap * K + q];
  int i1[NP], i2[NP], src1[NP], src2[NP];
  bool pv[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int t = lane + 64 * k;
    pv[k] = t < PAIRS;
    const int tt = pv[k] ? t : 0;
    i1[k] = (TD == 1) ? 0 : tt / W;
    i2[k] = (TD == 1) ? tt : tt % W;
    src2[k] = (kDpp ? 24 + i2[k] : (TD - 1) * W + i2[k]) * 4;   // byte addresses of the source
    src1[k] = kDpp ? (8 + i1[k]) * 4 : (TD >= 2) ? ((TD - 2) * W + i1[k]) * 4 : 0;   // lanes
  }
  const int o0 = tile_origin(w, job.tile, 0), o1 = tile_origin(w, job.tile, 1),
            o2 = tile_origin(w, job.tile, 2);
  T accr[NP][NI0];
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int i = 0; i < NI0; ++i) accr[k][i] = (T)0;
  // padded-tile offset of this lane's tap pair relative to a node's first tap, and the stride of
  // the first dimension's taps
  int loff[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) loff[k] = (TD >= 2 ? i1[k] * pe2 : 0) + i2[k];
  const int s01 = pe1 * pe2;
  constexpr unsigned kNone = 0xffffffffu;
  unsigned cur = kNone;
  // the register accumulators hold fixed-point units already (the node values are pre-scaled)
  auto flush = [&]() {
    const int l0 = (int)(cur & 255u) - o0, l1 = (int)((cur >> 8) & 255u) - o1,
              l2 = (int)((cur >> 16) & 255u) - o2;
    int cbase;
    if constexpr (TD == 3) cbase = (l0 * pe1 + l1) * pe2 + l2;
    else if constexpr (TD == 2) cbase = l1 * pe2 + l2;
    else cbase = l2;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      if (!pv[k]) continue;
      const int b = cbase + loff[k];
#pragma unroll
      for (int i = 0; i < NI0; ++i) {
        if constexpr (kTwo) {
          const float x = accr[k][i];
          const float hf = rintf(x);
          const int lo = __float2int_rn((x - hf) * kLoScale);   // x - hf is exact, |.| <= 1/2
          atomicAdd(&acc[b + i * s01], (Acc)(int)hf);
          atomicAdd(&acc_lo[b + i * s01], (Acc)lo);
        } else {
          atomicAdd(&acc[b + i * s01], (Acc)__double2ll_rn(accr[k][i]));
        }
        accr[k][i] = (T)0;
      }
    }
  };
  if constexpr (kDpp) {
    // the wavefront's own 64 entries of s_stage; LDS operations of one wavefront execute in
    // order, so the stores are visible to the loads of the node loop below and the next
    // round's stores follow them
    float4* stg = s_stage + wave * 64;
    float (&aw)[W] = accr[0];
    // the next round's entries are loaded while this round's nodes are spread; the input
    // values are in vreg (round r of the wavefront in vreg[0] at round r)
    unsigned n_mb = 0u;
    float n_f0 = 0.0f, n_f1 = 0.0f, n_f2 = 0.0f;
    auto load_round = [&](int bp) {
      const int pp = bp + lane;
      if (pp < q1) {
        n_mb = g_base[pp];
        n_f0 = g_frac[pp];
        n_f1 = g_frac[LN + pp];
        n_f2 = g_frac[2 * LN + pp];
      }
    };
    if (q0 < q1) load_round(q0);
    for (int base_p = q0; base_p < q1; base_p += 64) {
      const int p = base_p + lane;
      const bool ok = p < q1;
      const unsigned mb = ok ? n_mb : 0u;
      float4 nd;
      nd.x = ok ? fmaf(n_f0, 2.0f, -1.0f) : 0.0f;
      nd.y = ok ? fmaf(n_f1, 2.0f, -1.0f) : 0.0f;
      nd.z = ok ? fmaf(n_f2, 2.0f, -1.0f) : 0.0f;
      nd.w = ok ? vreg[0] * scale_t : 0.0f;
#pragma unroll
      for (int r = 0; r + 1 < kRounds; ++r) vreg[r] = vreg[r + 1];
      const bool more = base_p + 64 < q1;
      if (more) load_round(base_p + 64);
      __builtin_amdgcn_wave_barrier();
      stg[lane] = nd;
      __builtin_amdgcn_wave_barrier();
      const LdsPtr<float> sf = (LdsPtr<float>)stg;
      const int cnt = __builtin_amdgcn_readfirstlane(min(64, q1 - base_p));
      // two nodes per polynomial pass: lanes 0-31 evaluate node q's weights and lanes 32-63
      // node q + 1's (same layout within each half); v_permlane32_swap of the result with
      // itself gives each half's values replicated in both halves, the layout one node uses
      const int half = lane >> 5;
      // nodes that start a run (their cell differs from the previous node's): one ballot per
      // round, so the per-node test is a scalar bit test and the cell is read only at a run start
      const unsigned prev_mb = (unsigned)__builtin_amdgcn_ds_bpermute(((lane + 63) & 63) * 4, (int)mb);
      const unsigned long long starts = __ballot(ok && mb != (lane == 0 ? cur : prev_mb));
      auto node = [&](int q, float wv) {
        if ((starts >> q) & 1ull) {
          if (cur != kNone) flush();
          cur = __builtin_amdgcn_readfirstlane(lane_bcast(mb, q));
        }
        const float vq = sf[4 * q + 3];
        const float a2 = lane_fetch(wv, src2[0]);
        const float a1 = lane_fetch(wv, src1[0]);
        fmac_row_bcast<W>(aw, wv, vq * a1 * a2);
      };
      for (int q = 0; q < cnt; q += 2) {
        const float x = sf[4 * (q + half) + my_dim];     // q + half <= 63
        const float wv = horner<float, K>(cf, x);
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(wv), __float_as_uint(wv),
                                                         false, false);
        node(q, __uint_as_float(sw[0]));
        if (q + 1 < cnt) node(q + 1, __uint_as_float(sw[1]));
      }
      __builtin_amdgcn_wave_barrier();
    }
  } else
  for (int base_p = q0; base_p < q1; base_p += 64) {
    const int p = base_p + lane;
    const bool ok = p < q1;
    const unsigned mb = ok ? g_base[p] : 0u;
    const T f0 = (ok && TD == 3) ? g_frac[p] : (T)0;
    const T f1 = (ok && TD >= 2) ? g_frac[LN + p] : (T)0;
    const T f2 = ok ? g_frac[2 * LN + p] : (T)0;
    const T vv = ok ? v[g_idx[p]] * scale_t : (T)0;
    const int cnt = min(64, q1 - base_p);
    for (int q = 0; q < cnt; ++q) {
      const unsigned bq = __builtin_amdgcn_readfirstlane(lane_bcast(mb, q));
      if (bq != cur) {
        if (cur != kNone) flush();
        cur = bq;
      }
      const T vq = lane_bcast(vv, q);
      T xsel;
      if constexpr (TD == 3) {
        xsel = fma(lane_bcast(f0, q), sel0, (T)-1);
        xsel = fma(lane_bcast(f1, q), sel1, xsel);
        xsel = fma(lane_bcast(f2, q), sel2, xsel);
      } else if constexpr (TD == 2) {
        xsel = fma(lane_bcast(f1, q), sel0, (T)-1);
        xsel = fma(lane_bcast(f2, q), sel1, xsel);
      } else {
        xsel = fma(lane_bcast(f2, q), sel0, (T)-1);
      }
      const T wv = horner<T, K>(cf, xsel);
      T w12[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const T a2 = lane_fetch(wv, src2[k]);
        const T a1 = (TD >= 2) ? lane_fetch(wv, src1[k]) : (T)1;
        w12[k] = vq * a1 * a2;
      }
      if constexpr (TD == 3) {
        T s0[W];                                      // lanes [0, W) hold the first dimension's taps
#pragma unroll
        for (int i = 0; i < W; ++i) s0[i] = lane_bcast(wv, i);
#pragma unroll
        for (int i = 0; i < W; ++i)
#pragma unroll
          for (int k = 0; k < NP; ++k) accr[k][i] += w12[k] * s0[i];
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) accr[k][0] += w12[k];
      }
    }
  }
  if (cur != kNone) flush();
  __syncthreads();
  // the two FP32 words combine exactly in double (at most 50 significant bits)
  const double inv = kTwo ? 1.0 / (scale * (double)kLoScale) : 1.0 / scale;
  // a thread owns columns (x1, x2) of the padded tile and walks them along the first dimension
  const int pe0 = PEC ? PEC : w.pe[0], a0 = w.taps[0] > 1 ? w.m - 1 : 0;
  const int a1 = w.taps[1] > 1 ? w.m - 1 : 0, a2 = w.taps[2] > 1 ? w.m - 1 : 0;
  for (int col = threadIdx.x; col < s01; col += kSpreadThreads) {
    const int x1 = col / pe2, x2 = col - x1 * pe2;
    const SlotPart q1 = slot_part(x1, a1, w.ts[1], pe1), q2 = slot_part(x2, a2, w.ts[2], pe2);
    const int in_block = (x1 - q1.pre) * q2.sz + (x2 - q2.pre);
    for (int x0 = 0; x0 < pe0; ++x0) {
      const SlotPart q0 = slot_part(x0, a0, w.ts[0], pe0);
      const int o = q0.pre * s01 + q0.sz * (q1.pre * pe2 + q1.sz * q2.pre) +
                    (x0 - q0.pre) * q1.sz * q2.sz + in_block;
      const int c = x0 * s01 + col;
      double val = (double)(SAcc)acc[c];
      if constexpr (kTwo) val = val * (double)kLoScale + (double)(SAcc)acc_lo[c];
      out[o] = (T)(val * inv);
    }
  }
}

// Fold: every grid cell sums, in fixed order, the padded-tile slots that cover it.  Along each
// dimension a cell at local offset x of its tile is covered by the left neighbour if x < m
// (padded index x + ts + m - 1), by its own tile (index x + m - 1) and by the right neighbour if
// x > ts - m (index x - ts + m - 1); tile sizes are powers of two, so only shifts and masks.
template <typename T>
__global__ void __launch_bounds__(256)
k_fold(const WinDev* __restrict__ wins, const FoldJob* __restrict__ jobs,
       const ImgDev* __restrict__ imgs, int check) {
  const FoldJob job = jobs[blockIdx.x];
  const WinDev& w = wins[job.win];
  if (check && imgs[w.img].st->done) return;
  if ((int)threadIdx.x >= job.ncell) return;
  GlobalPtr<T> padded = (GlobalPtr<T>)w.padded;
  const long long slot_stride = w.slot_stride;
  ConstPtr<int> tile_slot0 = (ConstPtr<int>)w.tile_slot0;
  ConstPtr<int> tile_nslot = (ConstPtr<int>)w.tile_nslot;
  T __attribute__((address_space(1)))* grid = (T __attribute__((address_space(1)))*)w.grid;
  const long long c = job.cell0 + threadIdx.x;
  int ct[3][3], cl[3][3], cn[3];
  {
    const int n12 = w.n[1] * w.n[2];
    int cc[3];
    cc[0] = (int)(c / n12);
    const int r = (int)(c - (long long)cc[0] * n12);
    cc[1] = r / w.n[2];
    cc[2] = r - cc[1] * w.n[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int ts = w.ts[k], lts = w.lts[k], mask = w.nts[k] - 1;
      const int left = (w.taps[k] > 1) ? w.m - 1 : 0;
      const int x = cc[k] & (ts - 1), home = cc[k] >> lts;
      int q = 0;
      if (w.taps[k] > 1 && x < w.m) {             // left neighbour's halo
        ct[k][q] = (home - 1) & mask;
        cl[k][q] = x + ts + left;
        ++q;
      }
      ct[k][q] = home;
      cl[k][q] = x + left;
      ++q;
      if (w.taps[k] > 1 && x > ts - w.m) {        // right neighbour's halo
        ct[k][q] = (home + 1) & mask;
        cl[k][q] = x - ts + left;
        ++q;
      }
      cn[k] = q;
    }
  }
  T sum = (T)0;
  for (int a = 0; a < cn[0]; ++a)
    for (int bq = 0; bq < cn[1]; ++bq)
      for (int e = 0; e < cn[2]; ++e) {
        const int gt = w.tile_off + (((ct[0][a] << w.lnts[1]) + ct[1][bq]) << w.lnts[2]) + ct[2][e];
        const int ns = tile_nslot[gt];
        if (ns == 0) continue;
        const int pidx = slot_index(w, cl[0][a], cl[1][bq], cl[2][e]);
        const auto src = padded + (long long)tile_slot0[gt] * slot_stride + pidx;
        for (int k = 0; k < ns; ++k) sum += src[(long long)k * slot_stride];
      }
  grid[w.grid_off + c] = sum;
}

// Fold of a 3-D window, one workgroup per tile of TS^3 cells: thread (x1, x2) owns a column of
// TS cells along the first dimension in registers and adds, neighbour by neighbour (fixed
// order) and slot by slot, the padded-tile values that fall on its column.  Consecutive threads
// read consecutive padded cells; no barriers, no LDS.
template <typename T, int TS>
__global__ void __launch_bounds__(TS * TS)
k_fold3(const WinDev* __restrict__ wins, const Fold3Job* __restrict__ jobs, int job0,
        const ImgDev* __restrict__ imgs, int check) {
  const Fold3Job job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  if (check && imgs[w.img].st->done) return;
  GlobalPtr<T> padded = (GlobalPtr<T>)w.padded;
  const long long slot_stride = w.slot_stride;
  ConstPtr<int> tile_slot0 = (ConstPtr<int>)w.tile_slot0;
  ConstPtr<int> tile_nslot = (ConstPtr<int>)w.tile_nslot;
  T __attribute__((address_space(1)))* grid = (T __attribute__((address_space(1)))*)w.grid;
  const int x2 = threadIdx.x % TS, x1 = threadIdx.x / TS;
  const int tc2 = job.tile & (w.nts[2] - 1);
  const int tc1 = (job.tile >> w.lnts[2]) & (w.nts[1] - 1);
  const int tc0 = job.tile >> (w.lnts[2] + w.lnts[1]);
  const int left = w.m - 1, pe = w.pe[0];
  T acc[TS];
#pragma unroll
  for (int k = 0; k < TS; ++k) acc[k] = (T)0;
  for (int d0 = -1; d0 <= 1; ++d0) {
    const int s0 = d0 * TS - left;                 // neighbour's padded origin, local coords
    const int lo0 = max(0, s0), hi0 = min(TS, s0 + pe);
    if (lo0 >= hi0) continue;
    const int t0 = (tc0 + d0) & (w.nts[0] - 1);
    for (int d1 = -1; d1 <= 1; ++d1) {
      const int s1 = d1 * TS - left;
      if (max(0, s1) >= min(TS, s1 + pe)) continue;
      const int t1 = (tc1 + d1) & (w.nts[1] - 1);
      for (int d2 = -1; d2 <= 1; ++d2) {
        const int s2 = d2 * TS - left;
        if (max(0, s2) >= min(TS, s2 + pe)) continue;
        const int t2 = (tc2 + d2) & (w.nts[2] - 1);
        const int gt = w.tile_off + (((t0 << w.lnts[1]) + t1) << w.lnts[2]) + t2;
        const int ns = tile_nslot[gt];
        if (ns == 0) continue;
        const int p1 = x1 - s1, p2 = x2 - s2;        // padded indices of this column
        if (p1 < 0 || p1 >= pe || p2 < 0 || p2 >= pe) continue;
        const auto src = padded + (long long)tile_slot0[gt] * slot_stride;
#pragma unroll
        for (int x0 = 0; x0 < TS; ++x0) {
          if (x0 < lo0 || x0 >= hi0) continue;
          const auto q = src + slot_index(w, x0 - s0, p1, p2);
          T sum = (T)0;
          for (int k = 0; k < ns; ++k) sum += q[(long long)k * slot_stride];
          acc[x0] += sum;
        }
      }
    }
  }
  auto g = grid + w.grid_off;
  const int o0 = tc0 * TS, o1 = tc1 * TS, o2 = tc2 * TS;
#pragma unroll
  for (int x0 = 0; x0 < TS; ++x0)
    g[((long long)(o0 + x0) * w.n[1] + (o1 + x1)) * w.n[2] + (o2 + x2)] = acc[x0];
}

// Fold of a 3-D window with 8^3 tiles and cutoff M known at compile time.  A workgroup of Q
// wavefronts (Q = 1 or 4) takes Q consecutive jobs; with Q = 4 they are the same window's tiles
// t2 = 4g .. 4g + 3 (jobs list every tile of a window in order, and Q = 4 is used only when
// every window has a multiple of four tiles along the last dimension).  Each wavefront folds
// one tile.  Each of the 27 neighbours contributes one
// block of its slot (the slot layout stores it contiguously): the wavefront reads the block
// with consecutive lanes on consecutive cells and adds it into its tile in LDS, neighbour after
// neighbour and slot after slot, the order of k_fold3 (so the same sums bit for bit).  Block
// shapes and positions are compile-time constants; the lanes of one block hit distinct cells,
// and one wavefront keeps its LDS updates in order.  When every neighbour has at most one slot,
// the loads of a group of blocks (all 27, or the 9 of one offset d0 for large M) are issued
// before any of their additions, so a wavefront waits on memory once per group rather than once
// per block.  The Q tiles are then written together, rows of 8 Q cells along the contiguous
// dimension (128 bytes for Q = 4 in FP32).
template <int M>
struct Fold8Geo {
  static constexpr int TS = 8, LEFT = M - 1, PE = TS + 2 * M - 1;
  // Neighbour offset d along a dimension selects the block of its slot that folds into this
  // tile: d = -1 its right part (M cells, padded start LEFT + TS) onto cells [0, M), d = 0 the
  // tile part (TS cells, start LEFT) onto [0, TS), d = +1 its left part (M - 1 cells, start 0)
  // onto [TS - LEFT, TS).
  static constexpr int pre(int d) { return d < 0 ? LEFT + TS : (d == 0 ? LEFT : 0); }
  static constexpr int sz(int d) { return d < 0 ? M : (d == 0 ? TS : LEFT); }
  static constexpr int off(int d) { return d > 0 ? TS - LEFT : 0; }
  static constexpr int d0(int n) { return n / 9 - 1; }
  static constexpr int d1(int n) { return (n / 3) % 3 - 1; }
  static constexpr int d2(int n) { return n % 3 - 1; }
  static constexpr int bs(int n) { return sz(d0(n)) * sz(d1(n)) * sz(d2(n)); }
  static constexpr int nit(int n) { return (bs(n) + 63) / 64; }       // loads per lane
  static constexpr int first(int n) {                                 // registers before block n
    int s = 0;
    for (int k = 0; k < n; ++k) s += nit(k);
    return s;
  }
  static constexpr int group = first(27) <= 96 ? 27 : 9;              // blocks loaded together
  static constexpr int base(int n) {                                  // block start in the slot
    return pre(d0(n)) * PE * PE + sz(d0(n)) * (pre(d1(n)) * PE + sz(d1(n)) * pre(d2(n)));
  }
};

template <typename T, int M, int Q>
__global__ void __launch_bounds__(64 * Q)
k_fold3m(const WinDev* __restrict__ wins, const Fold3Job* __restrict__ jobs, int job0,
         const ImgDev* __restrict__ imgs, int check) {
  constexpr int TS = 8;
  __shared__ T tiles[Q][TS * TS * TS];
  const int wave = Q == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Fold3Job job = jobs[job0 + Q * blockIdx.x + wave];
  const WinDev& w = wins[job.win];
  // The image's finished flag is read after the block loads are issued (the same image for the
  // Q jobs), so its two dependent loads overlap the slot tables and the slot data; a finished
  // image's slots are read but never used.
  const CgState* st = imgs[w.img].st;
  T* tile = tiles[wave];
  GlobalPtr<T> padded = (GlobalPtr<T>)w.padded;
  const long long slot_stride = w.slot_stride;
  ConstPtr<int> tile_slot0 = (ConstPtr<int>)w.tile_slot0;
  ConstPtr<int> tile_nslot = (ConstPtr<int>)w.tile_nslot;
  const int lane = threadIdx.x & 63;
  const int tc2 = job.tile & (w.nts[2] - 1);
  const int tc1 = (job.tile >> w.lnts[2]) & (w.nts[1] - 1);
  const int tc0 = job.tile >> (w.lnts[2] + w.lnts[1]);
  // slot tables of the 27 neighbours: lane n < 27 loads neighbour n's entries (one round trip
  // of vector loads rather than a chain of scalar ones), then every lane reads them (uniform)
  int my_ns = 0, my_s0 = 0;
  if (lane < 27) {
    const int d0 = lane / 9 - 1, d1 = (lane / 3) % 3 - 1, d2 = lane % 3 - 1;
    const int t0 = (tc0 + d0) & (w.nts[0] - 1), t1 = (tc1 + d1) & (w.nts[1] - 1),
              t2 = (tc2 + d2) & (w.nts[2] - 1);
    const int gt = w.tile_off + (((t0 << w.lnts[1]) + t1) << w.lnts[2]) + t2;
    my_ns = tile_nslot[gt];
    my_s0 = tile_slot0[gt];
  }
  int ns[27], s0t[27];
#pragma unroll
  for (int n = 0; n < 27; ++n) {
    ns[n] = __builtin_amdgcn_readlane(my_ns, n);
    s0t[n] = __builtin_amdgcn_readlane(my_s0, n);
  }
#pragma unroll
  for (int k = 0; k < TS * TS * TS / 64; ++k) tile[lane + 64 * k] = (T)0;
  bool multi = false;
#pragma unroll
  for (int n = 0; n < 27; ++n) multi = multi || ns[n] > 1;
  using G = Fold8Geo<M>;
  // one neighbour's block (lanes past the block reread cell 0), added into the tile
  auto add_block = [&](auto n_c, const T* val) {
    constexpr int n = decltype(n_c)::value;
    constexpr int sz1 = G::sz(G::d1(n)), sz2 = G::sz(G::d2(n));
#pragma unroll
    for (int it = 0; it < G::nit(n); ++it) {
      const int e = lane + 64 * it;
      if (e >= G::bs(n)) continue;
      const int r2 = e % sz2, r1 = (e / sz2) % sz1, r0 = e / (sz1 * sz2);
      tile[((r0 + G::off(G::d0(n))) * TS + (r1 + G::off(G::d1(n)))) * TS + (r2 + G::off(G::d2(n)))] +=
          val[it];
    }
  };
  bool finished = false;
  if (!multi) {
    // groups of blocks: every load of the group, then the additions in neighbour order
    static_for<27 / G::group>([&](auto g_c) {
      if (finished) return;
      constexpr int n0 = decltype(g_c)::value * G::group, v0 = G::first(n0);
      T val[G::first(n0 + G::group) - v0];
      static_for<G::group>([&](auto k_c) {
        constexpr int n = n0 + decltype(k_c)::value;
        if constexpr (G::bs(n) > 0) {
          if (ns[n] != 0) {                                   // uniform: empty neighbour tile
            const long long src = (long long)s0t[n] * slot_stride + G::base(n);
#pragma unroll
            for (int it = 0; it < G::nit(n); ++it) {
              const int e = lane + 64 * it;
              val[G::first(n) - v0 + it] = padded[src + (e < G::bs(n) ? e : 0)];
            }
          }
        }
      });
      if (decltype(g_c)::value == 0 && check && st->done) {
        finished = true;
        return;
      }
      static_for<G::group>([&](auto k_c) {
        constexpr int n = n0 + decltype(k_c)::value;
        if constexpr (G::bs(n) > 0)
          if (ns[n] != 0) add_block(std::integral_constant<int, n>{}, val + (G::first(n) - v0));
      });
    });
  } else {
    finished = check && st->done;
    // some neighbour has several slots: each block is the sum of its slots in order
    if (!finished) static_for<27>([&](auto n_c) {
      constexpr int n = decltype(n_c)::value;
      if constexpr (G::bs(n) > 0) {
        if (ns[n] == 0) return;                               // uniform: empty neighbour tile
        const long long src = (long long)s0t[n] * slot_stride + G::base(n);
        constexpr int NI = G::nit(n);
        // KB slots per round: their NI * KB loads are issued together (the last slot is
        // reloaded past the end), then added in slot order, as a one-at-a-time sum would
        constexpr int KB = NI <= 2 ? 8 : (NI <= 4 ? 4 : 2);
        T val[NI];
#pragma unroll
        for (int it = 0; it < NI; ++it) val[it] = (T)0;
        for (int k = 0; k < ns[n]; k += KB) {
          T ld[KB][NI];
#pragma unroll
          for (int j = 0; j < KB; ++j) {
            const long long so = src + (long long)min(k + j, ns[n] - 1) * slot_stride;
#pragma unroll
            for (int it = 0; it < NI; ++it) {
              const int e = lane + 64 * it;
              ld[j][it] = padded[so + (e < G::bs(n) ? e : 0)];
            }
          }
#pragma unroll
          for (int j = 0; j < KB; ++j)
            if (k + j < ns[n])
#pragma unroll
              for (int it = 0; it < NI; ++it) val[it] += ld[j][it];
        }
        add_block(n_c, val);
      }
    });
  }
  if (finished) return;                                   // uniform over the workgroup
  __syncthreads();
  // rows (x0, x1) of the Q tiles: 8 Q consecutive cells from the first tile's origin
  T __attribute__((address_space(1)))* g = (T __attribute__((address_space(1)))*)w.grid + w.grid_off;
  const int o0 = tc0 * TS, o1 = tc1 * TS, o2 = (tc2 & ~(Q - 1)) * TS;
#pragma unroll
  for (int it = 0; it < TS; ++it) {
    const int idx = threadIdx.x + 64 * Q * it;
    const int col = idx % (Q * TS), row = idx / (Q * TS);   // row = x0 * TS + x1
    const int x0 = row / TS, x1 = row % TS;
    g[((long long)(o0 + x0) * w.n[1] + (o1 + x1)) * w.n[2] + (o2 + col)] =
        tiles[col / TS][(x0 * TS + x1) * TS + (col % TS)];
  }
}

// ---------------------------------------------------------------------------- convolution
// Per dimension, every grid line is circularly convolved with the window's real even kernel
// (multiplication of its DFT by the Fourier multiplier).  Two real lines are packed as one
// complex line.  A complex line of length N = A * B is held by B threads with A values each and
// transformed with the four-step method: length-A DFTs in registers, twiddles, an LDS
// exchange, length-B DFTs in registers; the multiplier is applied in that (transposed) order
// and the inverse runs the same steps backwards, so a line visits LDS twice per transform pair.
template <typename T>
struct Cx {
  T x, y;
};
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {   // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

__host__ __device__ constexpr int bit_reverse(int i, int bits) {
  int r = 0;
  for (int k = 0; k < bits; ++k) r |= ((i >> k) & 1) << (bits - 1 - k);
  return r;
}
__host__ __device__ constexpr int ilog2c(int p) { return p <= 1 ? 0 : 1 + ilog2c(p / 2); }

// cos and sin of 2 pi q / 16, q = 0..7
__device__ __constant__ const double kCos16[8] = {1.0, 0.92387953251128674, 0.70710678118654752,
                                                  0.38268343236508977, 0.0, -0.38268343236508977,
                                                  -0.70710678118654752, -0.92387953251128674};
__device__ __constant__ const double kSin16[8] = {0.0, 0.38268343236508977, 0.70710678118654752,
                                                  0.92387953251128674, 1.0, 0.92387953251128674,
                                                  0.70710678118654752, 0.38268343236508977};

// In-register DFT of length P (power of two, P <= 16), natural order in and out; forward uses
// exp(-2 pi i jk / P), inverse exp(+2 pi i jk / P), no normalisation.
template <typename T, int P, bool INV>
__device__ __forceinline__ void dft_reg(Cx<T>* v) {
  constexpr int LB = ilog2c(P);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int r = bit_reverse(i, LB);
    if (r > i) {
      const Cx<T> t = v[i];
      v[i] = v[r];
      v[r] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= P; len <<= 1) {
#pragma unroll
    for (int i = 0; i < P; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const int q = k * (16 / len);
        const Cx<T> wv = {(T)kCos16[q], INV ? (T)kSin16[q] : -(T)kSin16[q]};
        const Cx<T> a = v[i + k];
        const Cx<T> bb = cmul(v[i + k + len / 2], wv);
        v[i + k] = {a.x + bb.x, a.y + bb.y};
        v[i + k + len / 2] = {a.x - bb.x, a.y - bb.y};
      }
    }
  }
}

// Exchange-buffer layout of the four-step transform.  Line ql holds element (k2, k) (k2 < A,
// k < B) at ql * XS + k2 * B + (k XOR ((k2 / R) mod B)) when B >= 8: the XOR spreads the lanes
// that hold consecutive k2 over different banks, and XS = N + 8 (an odd multiple of 8 complex
// values) puts neighbouring lines in opposite halves of the banks, so that both exchange
// patterns (lane j1 writing column j1, lane j1 reading rows j1 R .. j1 R + R - 1) hit every bank
// equally often.  (With XS = N + 1 and no XOR the rows pattern put all eight lanes of a line in
// one bank.)  Narrow lines (B = 4) keep the plain layout, which measured no worse there.
template <int B, int R, bool SWZ>
__device__ __forceinline__ int xpos(int k2, int k) {
  return k2 * B + (SWZ ? (k ^ ((k2 / R) & (B - 1))) : k);
}

template <int N> struct FftShape {
  static constexpr int A = (N >= 128) ? 16 : 8;   // values per thread
  static constexpr int B = N / A;                 // threads per complex line
  static constexpr int R = A / B > 0 ? A / B : 1; // length-B DFTs per thread
  static constexpr int CL = (256 / B < N / 2) ? 256 / B : N / 2;   // complex lines per workgroup
  static constexpr int RL = 2 * CL;               // real lines per workgroup
  static constexpr int SP = N + 1;                // padded LDS line stride of the real lines
  static constexpr bool SWZ = B >= 8;
  static constexpr int XS = SWZ ? N + 8 : N + 1;  // exchange line stride (complex values)
  template <typename T>
  static constexpr size_t main_bytes() {          // real lines and exchange buffer share bytes
    const size_t a = (size_t)RL * SP * sizeof(T), b = (size_t)CL * XS * 2 * sizeof(T);
    return a > b ? a : b;
  }
};

template <typename T, int N>
__global__ void __launch_bounds__(256)
k_conv(const WinDev* __restrict__ wins, const ConvJob* __restrict__ jobs, int job0, int axis,
       const ImgDev* __restrict__ imgs, int check) {
  const ConvJob job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  if (check && imgs[w.img].st->done) return;
  T __attribute__((address_space(1)))* grid = (T __attribute__((address_space(1)))*)w.grid;
  using S = FftShape<N>;
  constexpr int A = S::A, B = S::B, CL = S::CL, RL = S::RL, SP = S::SP, XS = S::XS;
  extern __shared__ unsigned char smem_raw[];
  T* stage = reinterpret_cast<T*>(smem_raw);                      // RL * SP reals
  Cx<T>* ex = reinterpret_cast<Cx<T>*>(smem_raw);                 // CL * XS complex (same bytes)
  Cx<T>* tw = reinterpret_cast<Cx<T>*>(smem_raw + S::template main_bytes<T>());  // N twiddles
  for (int q = threadIdx.x; q < N; q += 256) {
    T sn, cs;
    if constexpr (sizeof(T) == 4) sincospif(-2.0f * (float)q / (float)N, &sn, &cs);
    else sincospi(-2.0 * (double)q / (double)N, &sn, &cs);
    tw[q] = {cs, sn};
  }
  long long es, ls;   // element stride along a line, stride between adjacent lines
  if (axis == 2) { es = 1; ls = N; }
  else if (axis == 1) { es = w.n[2]; ls = 1; }
  else { es = (long long)w.n[1] * w.n[2]; ls = 1; }
  auto g = grid + w.grid_off + job.off;
  const int nl = job.nl;
  for (int idx = threadIdx.x; idx < RL * N; idx += 256) {
    int ln, c;
    if (axis == 2) { ln = idx / N; c = idx - ln * N; }
    else { c = idx / RL; ln = idx - c * RL; }
    stage[ln * SP + c] = (ln < nl) ? g[c * es + ln * ls] : (T)0;
  }
  __syncthreads();
  const int ql = threadIdx.x / B, j1 = threadIdx.x % B;
  const bool act = ql < CL;
  GlobalPtr<T> coef = (GlobalPtr<T>)w.coef + (long long)axis * w.n_max;
  Cx<T> v[A];
  if (act) {
#pragma unroll
    for (int j2 = 0; j2 < A; ++j2) {
      const int c = j1 + B * j2;
      v[j2] = {stage[(2 * ql) * SP + c], stage[(2 * ql + 1) * SP + c]};
    }
    dft_reg<T, A, false>(v);
#pragma unroll
    for (int k2 = 0; k2 < A; ++k2) v[k2] = cmul(v[k2], tw[(j1 * k2) & (N - 1)]);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k2 = 0; k2 < A; ++k2) ex[ql * XS + xpos<B, S::R, S::SWZ>(k2, j1)] = v[k2];
  }
  __syncthreads();
  constexpr int R = S::R;
  if (act) {
    Cx<T> u[R][B];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k2 = j1 * R + r;
#pragma unroll
      for (int k1 = 0; k1 < B; ++k1) u[r][k1] = ex[ql * XS + xpos<B, R, S::SWZ>(k2, k1)];
      dft_reg<T, B, false>(u[r]);                 // u[r][k1] = X[k2 + A k1]
#pragma unroll
      for (int k1 = 0; k1 < B; ++k1) {
        const T cm = coef[k2 + A * k1];
        u[r][k1].x *= cm;
        u[r][k1].y *= cm;
      }
      dft_reg<T, B, true>(u[r]);                  // u[r][j1'] = Z[k2][j1']
#pragma unroll
      for (int j = 0; j < B; ++j) u[r][j] = cmulc(u[r][j], tw[(j * k2) & (N - 1)]);
#pragma unroll
      for (int j = 0; j < B; ++j) ex[ql * XS + xpos<B, R, S::SWZ>(k2, j)] = u[r][j];
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k2 = 0; k2 < A; ++k2) v[k2] = ex[ql * XS + xpos<B, R, S::SWZ>(k2, j1)];
    dft_reg<T, A, true>(v);                       // v[j2] = x'[j1 + B j2]
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j2 = 0; j2 < A; ++j2) {
      const int c = j1 + B * j2;
      stage[(2 * ql) * SP + c] = v[j2].x;
      stage[(2 * ql + 1) * SP + c] = v[j2].y;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < RL * N; idx += 256) {
    int ln, c;
    if (axis == 2) { ln = idx / N; c = idx - ln * N; }
    else { c = idx / RL; ln = idx - c * RL; }
    if (ln < nl) g[c * es + ln * ls] = stage[ln * SP + c];
  }
}

// ---------------------------------------------------------------------------- plane kernel
// The convolutions along the last two dimensions of a 3-D window (FP32, n = N <= 128), one
// workgroup per grid plane i0: the plane is read into LDS once, its lines are convolved along
// the last and then the middle dimension in LDS (same four-step arithmetic as k_conv, so the
// result is bitwise that of two convolution passes), and the plane is written once.  Saves one
// read/write pass over the grid.  (Folding the padded-tile slots straight into the plane was
// measured slower than the separate per-tile fold, which shares its neighbour lookups across a
// tile's planes.)
template <int N> struct PlaneShape {
  static constexpr int A = (N >= 128) ? 16 : 8;
  static constexpr int B = N / A;
  static constexpr int R = A / B > 0 ? A / B : 1;
  static constexpr int CL = N / 2;                // complex lines: every line of the plane
  static constexpr int THREADS = 512;
  // plane row stride (floats): N + 5 spreads both the row and the column accesses of a
  // wavefront over the banks better than N + 1 (which put every other lane pair in one bank)
  static constexpr int PS = N + 5;
  static constexpr bool SWZ = B >= 8;
  static constexpr int XS = SWZ ? N + 8 : N + 1;  // exchange line stride (complex), aliasing the plane
  static constexpr size_t lds() {
    const size_t plane = (size_t)N * PS * sizeof(float), exch = (size_t)CL * XS * 2 * sizeof(float);
    return (plane > exch ? plane : exch) + (size_t)N * 2 * sizeof(float);
  }
  static_assert(CL * B <= THREADS, "plane lines exceed the workgroup");
};

template <int N>
__global__ void __launch_bounds__(512)
k_plane(const WinDev* __restrict__ wins, const PlaneJob* __restrict__ jobs, int job0,
        const ImgDev* __restrict__ imgs, int check) {
  using T = float;
  using S = PlaneShape<N>;
  constexpr int A = S::A, B = S::B, CL = S::CL, PS = S::PS, XS = S::XS;
  const PlaneJob job = jobs[job0 + blockIdx.x];
  const WinDev& w = wins[job.win];
  if (check && imgs[w.img].st->done) return;
  extern __shared__ unsigned char smem_raw[];
  T* plane = reinterpret_cast<T*>(smem_raw);
  Cx<T>* ex = reinterpret_cast<Cx<T>*>(smem_raw);   // the same bytes, used while lines are in registers
  constexpr size_t kMain = (size_t)N * PS * sizeof(T) > (size_t)CL * XS * 2 * sizeof(T)
                               ? (size_t)N * PS * sizeof(T) : (size_t)CL * XS * 2 * sizeof(T);
  Cx<T>* tw = reinterpret_cast<Cx<T>*>(smem_raw + kMain);
  const int tid = threadIdx.x;
  for (int q = tid; q < N; q += S::THREADS) {
    T sn, cs;
    sincospif(-2.0f * (float)q / (float)N, &sn, &cs);
    tw[q] = {cs, sn};
  }
  // ---- the folded plane into LDS
  T __attribute__((address_space(1)))* g =
      (T __attribute__((address_space(1)))*)w.grid + w.grid_off + (long long)job.i0 * N * N;
  for (int idx = tid; idx < N * N; idx += S::THREADS) {
    const int i1 = idx / N, i2 = idx - i1 * N;
    plane[i1 * PS + i2] = g[idx];
  }
  __syncthreads();
  // ---- convolution of every line along the last (rows) and then the middle (columns) dimension
  const int ql = tid / B, j1 = tid % B;
  const bool act = ql < CL;
  GlobalPtr<T> coef_all = (GlobalPtr<T>)w.coef;
  for (int axis = 2; axis >= 1; --axis) {
    const int ls = (axis == 2) ? PS : 1, es = (axis == 2) ? 1 : PS;
    GlobalPtr<T> coef = coef_all + (long long)axis * w.n_max;
    Cx<T> v[A];
    if (act) {
#pragma unroll
      for (int j2 = 0; j2 < A; ++j2) {
        const int c = j1 + B * j2;
        v[j2] = {plane[(2 * ql) * ls + c * es], plane[(2 * ql + 1) * ls + c * es]};
      }
      dft_reg<T, A, false>(v);
#pragma unroll
      for (int k2 = 0; k2 < A; ++k2) v[k2] = cmul(v[k2], tw[(j1 * k2) & (N - 1)]);
    }
    __syncthreads();   // every line is in registers: the plane's bytes become the exchange buffer
    if (act) {
#pragma unroll
      for (int k2 = 0; k2 < A; ++k2) ex[ql * XS + xpos<B, S::R, S::SWZ>(k2, j1)] = v[k2];
    }
    __syncthreads();
    constexpr int R = S::R;
    if (act) {
      Cx<T> u[R][B];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k2 = j1 * R + r;
#pragma unroll
        for (int k1 = 0; k1 < B; ++k1) u[r][k1] = ex[ql * XS + xpos<B, R, S::SWZ>(k2, k1)];
        dft_reg<T, B, false>(u[r]);
#pragma unroll
        for (int k1 = 0; k1 < B; ++k1) {
          const T cm = coef[k2 + A * k1];
          u[r][k1].x *= cm;
          u[r][k1].y *= cm;
        }
        dft_reg<T, B, true>(u[r]);
#pragma unroll
        for (int j = 0; j < B; ++j) u[r][j] = cmulc(u[r][j], tw[(j * k2) & (N - 1)]);
#pragma unroll
        for (int j = 0; j < B; ++j) ex[ql * XS + xpos<B, R, S::SWZ>(k2, j)] = u[r][j];
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k2 = 0; k2 < A; ++k2) v[k2] = ex[ql * XS + xpos<B, R, S::SWZ>(k2, j1)];
      dft_reg<T, A, true>(v);
    }
    __syncthreads();   // the exchange buffer is read: its bytes hold the plane again
    if (act) {
#pragma unroll
      for (int j2 = 0; j2 < A; ++j2) {
        const int c = j1 + B * j2;
        plane[(2 * ql) * ls + c * es] = v[j2].x;
        plane[(2 * ql + 1) * ls + c * es] = v[j2].y;
      }
    }
    __syncthreads();
  }
  // ---- write the plane
  for (int idx = tid; idx < N * N; idx += S::THREADS) {
    const int i1 = idx / N, i2 = idx - i1 * N;
    g[idx] = plane[i1 * PS + i2];
  }
}

// ---------------------------------------------------------------------------- gathering
// One thread per node.  Chunks with enough nodes first stage the padded tile of the convolved
// grid in LDS; small chunks read the grid directly.  The two cases are separate instantiations
// of the node loop, so the staged one reads through an LDS pointer (ds_read) rather than a
// generic one (flat loads).

template <typename T, int W, int TD, bool STAGED, int TSC, typename PP>
__device__ __forceinline__ void gather_nodes(const TileJob& job, const WinDev& w,
                                             const T* __restrict__ tile, const T* __restrict__ h,
                                             PP psi, int o0, int o1, int o2) {
  constexpr int m = W / 2;
  constexpr int K = PsiDeg<T>::value + 1;
  // large rows (FP64, m >= 6): evaluate the middle dimension's weights inside the loop instead of
  // keeping a second register row, to stay within the register file
  constexpr bool BIG = W * (int)sizeof(T) > 64;
  GlobalPtr<int> g_idx = (GlobalPtr<int>)w.g_idx;
  GlobalPtr<unsigned> g_base = (GlobalPtr<unsigned>)w.g_base;
  GlobalPtr<T> g_frac = (GlobalPtr<T>)w.g_frac;
  const long long LN = w.LN;
  T* __restrict__ ylocal = reinterpret_cast<T*>(w.ylocal);
  const int n0 = w.n[0], n1 = w.n[1], n2 = w.n[2];
  constexpr int PEC = (TD == 3 && TSC > 0) ? TSC + W - 1 : 0;
  const int pe1 = PEC ? PEC : w.pe[1], pe2 = PEC ? PEC : w.pe[2];
  // explicit address spaces: LDS reads for the staged tile, global loads otherwise
  LdsPtr<T> tile_l = (LdsPtr<T>)tile;
  GlobalPtr<T> h_g = (GlobalPtr<T>)h;
  // a node's entries are loaded one iteration ahead, so their latency overlaps the previous
  // node's arithmetic
  unsigned nb_ = 0u;
  T nf0 = (T)0, nf1 = (T)0, nf2 = (T)0;
  int nidx = 0;
  auto load_node = [&](int q) {
    nb_ = g_base[q];
    if constexpr (TD == 3) nf0 = g_frac[q];
    if constexpr (TD >= 2) nf1 = g_frac[LN + q];
    nf2 = g_frac[2 * LN + q];
    nidx = g_idx[q];
  };
  if (job.pbeg + (int)threadIdx.x < job.pend) load_node(job.pbeg + threadIdx.x);
  for (int p = job.pbeg + threadIdx.x; p < job.pend; p += kGatherThreads) {
    const unsigned bb = nb_;
    const T fr0 = nf0, fr1 = nf1, fr2 = nf2;
    const int out_idx = nidx;
    if (p + kGatherThreads < job.pend) load_node(p + kGatherThreads);
    const int b2 = (int)((bb >> 16) & 255u), b1 = (int)((bb >> 8) & 255u), b0 = (int)(bb & 255u);
    T w2[W];
    poly_row<T, W>(psi, fr2, w2);
    const T x1 = (TD >= 2) ? (T)2 * fr1 - (T)1 : (T)0;
    T w1[BIG ? 1 : W];
    if constexpr (TD >= 2 && !BIG) poly_row<T, W>(psi, fr1, w1);
    const T x0 = (TD == 3) ? (T)2 * fr0 - (T)1 : (T)0;
    int c2[W];
#pragma unroll
    for (int i2 = 0; i2 < W; ++i2) c2[i2] = STAGED ? b2 - o2 + i2 : wrap(b2 - m + 1 + i2, n2);
    // row start of (i0, i1) in the staged tile or in the grid
    auto row_of = [&](int i0, int i1) {
      if constexpr (STAGED) {
        return tile_l + ((b0 - o0 + i0) * pe1 + (b1 - o1 + i1)) * pe2;
      } else {
        const int g0 = (TD == 3) ? wrap(b0 - m + 1 + i0, n0) : 0;
        const int g1 = (TD >= 2) ? wrap(b1 - m + 1 + i1, n1) : 0;
        return h_g + ((long long)g0 * n1 + g1) * n2;
      }
    };
    auto line = [&](auto row) {
      T sacc = (T)0;
#pragma unroll
      for (int i2 = 0; i2 < W; ++i2) sacc += row[c2[i2]] * w2[i2];
      return sacc;
    };
    auto plane = [&](int i0) {
      T pacc = (T)0;
      if constexpr (TD == 1) {
        pacc = line(row_of(0, 0));
      } else if constexpr (BIG) {
        for (int i1 = 0; i1 < W; ++i1) pacc += horner<T, K>(psi + i1 * K, x1) * line(row_of(i0, i1));
      } else {
#pragma unroll
        for (int i1 = 0; i1 < W; ++i1) pacc += w1[i1] * line(row_of(i0, i1));
      }
      return pacc;
    };
    T acc = (T)0;
    if constexpr (TD == 3) {
      for (int i0 = 0; i0 < W; ++i0) acc += horner<T, K>(psi + i0 * K, x0) * plane(i0);
    } else {
      acc = plane(0);
    }
    ylocal[out_idx] = acc;
  }
}

template <typename T, int W, int TD, int TSC>
__global__ void __launch_bounds__(kGatherThreads)
k_gather(const WinDev* __restrict__ wins, const TileJob* __restrict__ jobs, int job0,
         const ImgDev* __restrict__ imgs, int check, int stage_min) {
  // Workgroups are dealt round-robin to the 8 XCDs in launch order.  XCD x takes the x-th of
  // eight contiguous ranges of the jobs (tile order between ranges, largest chunks first within
  // one), so neighbouring tiles, whose padded tiles share grid cells, are staged through one L2.
  const int nj = gridDim.x, x = blockIdx.x % 8, k = blockIdx.x / 8;
  const int jx = x * (nj / 8) + min(x, nj % 8) + k;
  const TileJob job = jobs[job0 + jx];
  const WinDev& w = wins[job.win];
  if (check && imgs[w.img].st->done) return;
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const T* h = reinterpret_cast<const T*>(w.grid) + w.grid_off;
  const int n0 = w.n[0], n1 = w.n[1], n2 = w.n[2];
  constexpr int PEC = (TD == 3 && TSC > 0) ? TSC + W - 1 : 0;
  const int pe0 = PEC ? PEC : w.pe[0], pe1 = PEC ? PEC : w.pe[1], pe2 = PEC ? PEC : w.pe[2];
  const int o0 = tile_origin(w, job.tile, 0), o1 = tile_origin(w, job.tile, 1),
            o2 = tile_origin(w, job.tile, 2);
  constexpr int m = W / 2;
  // window polynomials: from global (scalar loads) when small, else staged in LDS
  constexpr int KP = PsiDeg<T>::value + 1;
  constexpr bool PSI_LDS = (W * KP * (int)sizeof(T) / 4) > 96;
  __shared__ T s_psi[PSI_LDS ? W * KP : 1];
  const T* psi_g = reinterpret_cast<const T*>(w.psi);
  if constexpr (PSI_LDS) {
    for (int c = threadIdx.x; c < W * KP; c += kGatherThreads) s_psi[c] = psi_g[c];
  }
  const bool staged = (job.pend - job.pbeg) >= stage_min;
  if (staged) {
    // first grid cell covered by the padded tile, per dimension
    const int s0 = (TD == 3) ? o0 - m + 1 : o0;
    const int s1 = (TD >= 2) ? o1 - m + 1 : o1;
    const int s2 = o2 - m + 1;
    // grid sizes are powers of two: periodic wrap by masking; a thread owns columns (a1, a2)
    // of the padded tile and walks them along the first dimension
    const int s01 = pe1 * pe2;
    for (int col = threadIdx.x; col < s01; col += kGatherThreads) {
      const int a1 = col / pe2, a2 = col - a1 * pe2;
      const long long row = (long long)((s1 + a1) & (n1 - 1)) * n2 + ((s2 + a2) & (n2 - 1));
      for (int a0 = 0; a0 < pe0; ++a0)
        tile[a0 * s01 + col] = h[(long long)((s0 + a0) & (n0 - 1)) * n1 * n2 + row];
    }
    __syncthreads();
    if constexpr (PSI_LDS) gather_nodes<T, W, TD, true, TSC>(job, w, tile, h, (LdsPtr<T>)s_psi, o0, o1, o2);
    else gather_nodes<T, W, TD, true, TSC>(job, w, tile, h, (ConstPtr<T>)psi_g, o0, o1, o2);
  } else {
    if constexpr (PSI_LDS) {
      __syncthreads();
      gather_nodes<T, W, TD, false, TSC>(job, w, tile, h, (LdsPtr<T>)s_psi, o0, o1, o2);
    } else {
      gather_nodes<T, W, TD, false, TSC>(job, w, tile, h, (ConstPtr<T>)psi_g, o0, o1, o2);
    }
  }
}

// ---------------------------------------------------------------------------- reduction
struct ReduceArgs {
  VecArg in;           // the product's input v
  VecArg out;          // result vector (unused for EPI_DEGREE and EPI_CG_TRUE)
  double* Dout;        // EPI_DEGREE: destination if non-null, else the image's D
  int mode;
};

// sum of v (FP64) per image, for windows whose kernel is the constant 1 1^T
template <typename T>
__global__ void __launch_bounds__(1024) k_sum(const ImgDev* __restrict__ imgs, VecArg in, int check) {
  const ImgDev& im = imgs[blockIdx.y];
  if (check && im.st->done) return;
  const T* v = vin<T>(im, in);
  __shared__ double sh[1024];
  double a = 0.0;
  for (long long i = threadIdx.x; i < im.N; i += 1024) a += (double)v[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *im.sumv = sh[0];
}

// One row of blocks per image (blockIdx.y): the FP64 sum over the image's windows fused with
// the epilogue; the CG epilogues reduce their sums over the image's nred blocks.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_reduce(const WinDev* __restrict__ wins, const ImgDev* __restrict__ imgs, ReduceArgs a) {
  const ImgDev& im = imgs[blockIdx.y];
  const bool cg = a.mode >= EPI_CG_Q;
  CgState* st = im.st;
  if (a.mode == EPI_CG_Q && st->done) return;
  if (cg && blockIdx.x >= (unsigned)im.nred) return;
  const unsigned nb = cg ? (unsigned)im.nred : gridDim.x;
  const T* v = vin<T>(im, a.in);
  const long long N = im.N;
  const int l0 = im.win0, l1 = im.win0 + im.L;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const double alpha = cg ? st->alpha : 0.0;
  const double mean_f = cg ? st->mean_f : 0.0;
  const T* f = cg ? reinterpret_cast<const T*>(im.vec[V_F]) : nullptr;
  // the image's window weights and per-window results, read once per block (the output
  // stores below could alias the descriptors, so the compiler would reload them per element);
  // windows of kernel 1 1^T contribute the sum of v
  constexpr int kWinCache = 64;
  __shared__ const T* s_y[kWinCache];
  __shared__ double s_w[kWinCache];
  const int nw = l1 - l0;
  const bool cached = nw <= kWinCache;
  if (cached && (int)threadIdx.x < nw) {
    const WinDev& wl = wins[l0 + threadIdx.x];
    s_w[threadIdx.x] = wl.weight;
    s_y[threadIdx.x] = wl.t > 0 ? reinterpret_cast<const T*>(wl.ylocal) : nullptr;
  }
  __syncthreads();
  const double sumv = *im.sumv;
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)nb * kRedThreads) {
    double y = 0.0;
    if (cached) {
      // eight windows' loads in flight at a time, summed in window order; a window of kernel
      // 1 1^T loads from the input (any valid address) and takes the sum of v instead
      int l = 0;
      for (; l + 8 <= nw; l += 8) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const T* yl = s_y[l + k];
          const GlobalPtr<T> src = (GlobalPtr<T>)(yl ? yl : v);
          const double ld = (double)src[i];
          t[k] = yl ? ld : sumv;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) y += s_w[l + k] * t[k];
      }
      for (; l < nw; ++l) {
        const T* yl = s_y[l];
        y += s_w[l] * (yl ? (double)yl[i] : sumv);
      }
    } else {
      for (int l = l0; l < l1; ++l)
        y += wins[l].weight *
             (wins[l].t > 0 ? (double)reinterpret_cast<const T*>(wins[l].ylocal)[i] : sumv);
    }
    switch (a.mode) {
      case EPI_ANOVA:
        vout<T>(im, a.out)[i] = (T)y;
        break;
      case EPI_LAPLACIAN:
        vout<T>(im, a.out)[i] = (T)(im.D[i] * (double)v[i] - y);
        break;
      case EPI_DEGREE:
        (a.Dout ? a.Dout : im.D)[i] = y;
        break;
      case EPI_CG_Q: {
        const double vi = (double)v[i];
        const double q = vi + alpha * (im.D[i] * vi - y);
        vout<T>(im, a.out)[i] = (T)q;
        s0 += vi * q;
        s1 += q;
        s2 += vi;
        break;
      }
      case EPI_CG_INIT:
      case EPI_CG_TRUE: {
        const double vi = (double)v[i];
        const double b = (double)f[i] - mean_f;
        const double r = b - (vi + alpha * (im.D[i] * vi - y));
        if (a.mode == EPI_CG_INIT) vout<T>(im, a.out)[i] = (T)r;
        s0 += r;
        s1 += (a.mode == EPI_CG_INIT) ? b * b : r * r;
        break;
      }
    }
  }
  if (!cg) return;
  const double vals[3] = {s0, s1, s2};
  double tot[3];
  if (!grid_reduce<3>(vals, im.red, &st->ticket[0], tot, nb)) return;
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

template <typename K>
void allow_lds(K k, size_t lds) {
  if (lds > 65536)
    NLD_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

// Chunks with at least this many nodes stage the padded tile of the convolved grid in LDS for
// the gathering (a tile is read once instead of 8^t scattered reads per node).
int gather_stage_min() {
  static const int v = [] {
    const char* e = std::getenv("NLD_GATHER_STAGE_MIN");
    return e ? std::max(1, std::atoi(e)) : 1;
  }();
  return v;
}

template <typename T, int W>
void launch_tiles(const LaunchSet& ls, VecArg in, int check, hipStream_t s, bool gather) {
  // spreading accumulates in fixed point: two 32-bit words (FP32) or one 64-bit word (FP64) per
  // cell; gathering stages the tile in T
  const size_t lds = (size_t)ls.max_padded * (gather ? sizeof(T) : 8);
  for (int g = 0; g < 3; ++g) {
    const int j0 = ls.tjob_begin[g], nj = ls.tjob_begin[g + 1] - j0;
    if (nj == 0) continue;
    const bool c8 = ls.ts3 == 8;
    if (!gather) {
      auto k = (g == 0) ? k_spread<T, W, 1, 0> : (g == 1) ? k_spread<T, W, 2, 0>
             : c8 ? k_spread<T, W, 3, 8> : k_spread<T, W, 3, 0>;
      allow_lds(k, lds);
      hipLaunchKernelGGL(k, dim3(nj), dim3(kSpreadThreads), lds, s, ls.d_wins, ls.d_tjobs, j0,
                         ls.d_imgs, in, check);
    } else {
      auto k = (g == 0) ? k_gather<T, W, 1, 0> : (g == 1) ? k_gather<T, W, 2, 0>
             : c8 ? k_gather<T, W, 3, 8> : k_gather<T, W, 3, 0>;
      allow_lds(k, lds);
      hipLaunchKernelGGL(k, dim3(nj), dim3(kGatherThreads), lds, s, ls.d_wins,
                         ls.d_gjobs ? ls.d_gjobs : ls.d_tjobs, j0, ls.d_imgs, check,
                         gather_stage_min());
    }
    NLD_HIP(hipGetLastError());
  }
}

template <typename T>
void tiles_dispatch(const LaunchSet& ls, VecArg in, int check, hipStream_t s, bool gather) {
  switch (ls.m) {
    case 1: launch_tiles<T, 2>(ls, in, check, s, gather); break;
    case 2: launch_tiles<T, 4>(ls, in, check, s, gather); break;
    case 3: launch_tiles<T, 6>(ls, in, check, s, gather); break;
    case 4: launch_tiles<T, 8>(ls, in, check, s, gather); break;
    case 5: launch_tiles<T, 10>(ls, in, check, s, gather); break;
    case 6: launch_tiles<T, 12>(ls, in, check, s, gather); break;
    case 7: launch_tiles<T, 14>(ls, in, check, s, gather); break;
    case 8: launch_tiles<T, 16>(ls, in, check, s, gather); break;
    default: throw std::invalid_argument("cutoff out of range");
  }
}

template <typename T, int N>
void launch_conv(const LaunchSet& ls, int ax, int j0, int nj, int check, hipStream_t s) {
  using S = FftShape<N>;
  const size_t lds = S::template main_bytes<T>() + (size_t)N * 2 * sizeof(T);
  allow_lds(k_conv<T, N>, lds);
  hipLaunchKernelGGL((k_conv<T, N>), dim3(nj), dim3(256), lds, s, ls.d_wins, ls.d_conv[ax], j0, ax,
                     ls.d_imgs, check);
  NLD_HIP(hipGetLastError());
}

template <int N>
void launch_plane(const LaunchSet& ls, int j0, int nj, int check, hipStream_t s) {
  const size_t lds = PlaneShape<N>::lds();
  allow_lds(k_plane<N>, lds);
  hipLaunchKernelGGL(k_plane<N>, dim3(nj), dim3(PlaneShape<N>::THREADS), lds, s, ls.d_wins,
                     ls.d_pjobs, j0, ls.d_imgs, check);
  NLD_HIP(hipGetLastError());
}

// fused convolution of the last two dimensions, per grid plane (FP32 3-D windows)
void planes_all(const LaunchSet& ls, int check, hipStream_t s) {
  const int n64 = ls.pjob_begin[1] - ls.pjob_begin[0], n128 = ls.pjob_begin[2] - ls.pjob_begin[1];
  if (n64 > 0) launch_plane<64>(ls, ls.pjob_begin[0], n64, check, s);
  if (n128 > 0) launch_plane<128>(ls, ls.pjob_begin[1], n128, check, s);
}

template <typename T>
void conv_all(const LaunchSet& ls, int check, hipStream_t s) {
  for (int ax = 2; ax >= 0; --ax) {
    for (int gi = 0; gi < 4; ++gi) {
      const int j0 = ls.conv_begin[ax][gi], nj = ls.conv_begin[ax][gi + 1] - j0;
      if (nj == 0) continue;
      switch (gi) {
        case 0: launch_conv<T, 32>(ls, ax, j0, nj, check, s); break;
        case 1: launch_conv<T, 64>(ls, ax, j0, nj, check, s); break;
        case 2: launch_conv<T, 128>(ls, ax, j0, nj, check, s); break;
        default: launch_conv<T, 256>(ls, ax, j0, nj, check, s); break;
      }
    }
  }
}

template <typename T>
void spread_fold(const LaunchSet& ls, VecArg in, int check, hipStream_t s) {
  if (ls.has_flat) {
    hipLaunchKernelGGL(k_sum<T>, dim3(1, ls.n_imgs), dim3(1024), 0, s, ls.d_imgs, in, check);
    NLD_HIP(hipGetLastError());
  }
  tiles_dispatch<T>(ls, in, check, s, false);
  const int n8 = ls.f3_begin[1] - ls.f3_begin[0], n16 = ls.f3_begin[2] - ls.f3_begin[1];
  if (n8 > 0) {
    auto pick = [&](auto q) {
      constexpr int Q = decltype(q)::value;
      return (ls.m == 1) ? k_fold3m<T, 1, Q> : (ls.m == 2) ? k_fold3m<T, 2, Q>
           : (ls.m == 3) ? k_fold3m<T, 3, Q> : (ls.m == 4) ? k_fold3m<T, 4, Q>
           : (ls.m == 5) ? k_fold3m<T, 5, Q> : (ls.m == 6) ? k_fold3m<T, 6, Q>
           : (ls.m == 7) ? k_fold3m<T, 7, Q> : k_fold3m<T, 8, Q>;
    };
    if (ls.f3_quad) {
      if (n8 % 4 != 0) throw std::runtime_error("internal: 8^3 fold jobs not in groups of four");
      hipLaunchKernelGGL(pick(std::integral_constant<int, 4>{}), dim3(n8 / 4), dim3(256), 0, s,
                         ls.d_wins, ls.d_f3jobs, ls.f3_begin[0], ls.d_imgs, check);
    } else {
      hipLaunchKernelGGL(pick(std::integral_constant<int, 1>{}), dim3(n8), dim3(64), 0, s,
                         ls.d_wins, ls.d_f3jobs, ls.f3_begin[0], ls.d_imgs, check);
    }
  }
  if (n16 > 0)
    hipLaunchKernelGGL((k_fold3<T, 16>), dim3(n16), dim3(256), 0, s, ls.d_wins, ls.d_f3jobs,
                       ls.f3_begin[1], ls.d_imgs, check);
  NLD_HIP(hipGetLastError());
  if (ls.n_fjobs > 0) {
    hipLaunchKernelGGL(k_fold<T>, dim3(ls.n_fjobs), dim3(256), 0, s, ls.d_wins, ls.d_fjobs,
                       ls.d_imgs, check);
    NLD_HIP(hipGetLastError());
  }
}

// per-window results of the flat windows (no kept dimension): K = 1 1^T, sigma dK/dsigma = 0
template <typename T>
__global__ void k_flat_parts(const WinDev* __restrict__ wins, int L, long long N,
                             const double* __restrict__ sumv, T* __restrict__ yk, T* __restrict__ yks) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    for (int l = 0; l < L; ++l)
      if (wins[l].t == 0) {
        yk[(long long)l * N + i] = (T)*sumv;
        yks[(long long)l * N + i] = (T)0;
      }
}

template <typename T>
__global__ void k_axpy_windows(const T* __restrict__ src, T* __restrict__ dst, long long n, int first) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = first ? src[i] : dst[i] + src[i];
}

template <typename T>
void matvec_parts_t(Plan& P, const void* v, void* yk, void* yks, hipStream_t s) {
  const long long LN = (long long)P.N * P.L;
  const size_t gbytes = (size_t)P.grid_total * sizeof(T);
  const VecArg in{v, 0};
  spread_fold<T>(P.ls_unfused, in, 0, s);
  NLD_HIP(hipMemcpyAsync(P.grid_save, P.grid, gbytes, hipMemcpyDeviceToDevice, s));
  conv_all<T>(P.ls_unfused, 0, s);
  tiles_dispatch<T>(P.ls_unfused, in, 0, s, true);
  NLD_HIP(hipMemcpyAsync(yk, P.ylocal, LN * sizeof(T), hipMemcpyDeviceToDevice, s));
  bool first = true;
  for (int d = 0; d < 3; ++d) {
    if (!P.dv_used[d]) continue;
    LaunchSet lsd = P.ls_unfused;
    lsd.d_wins = P.d_wins_dv[d];
    NLD_HIP(hipMemcpyAsync(P.grid, P.grid_save, gbytes, hipMemcpyDeviceToDevice, s));
    conv_all<T>(lsd, 0, s);
    tiles_dispatch<T>(lsd, in, 0, s, true);
    hipLaunchKernelGGL(k_axpy_windows<T>, dim3(grid_for(LN)), dim3(256), 0, s, (const T*)P.ylocal,
                       (T*)yks, LN, first ? 1 : 0);
    NLD_HIP(hipGetLastError());
    first = false;
  }
  if (first) NLD_HIP(hipMemsetAsync(yks, 0, LN * sizeof(T), s));
  if (P.has_flat) {
    hipLaunchKernelGGL(k_flat_parts<T>, dim3(grid_for(P.N)), dim3(256), 0, s, P.d_wins, P.L,
                       (long long)P.N, (const double*)P.sumv, (T*)yk, (T*)yks);
    NLD_HIP(hipGetLastError());
  }
}

// Per-block partial sums for the gradient: for each window l (NS = 4 L + 3 values)
//   p u D_l,  p K_l u,  p u Ds_l,  p Ks_l u   and then  p,  u,  p u.
template <typename T>
__global__ void __launch_bounds__(256)
k_grad_sums(const T* __restrict__ p, const T* __restrict__ u, const T* __restrict__ dl,
            const T* __restrict__ ku, const T* __restrict__ dls, const T* __restrict__ ksu, int L,
            long long N, double* __restrict__ part) {
  const int NS = 4 * L + 3;
  __shared__ double sh[256];
  for (int k = 0; k < NS; ++k) {
    const int l = k / 4, kind = k % 4;
    double a = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < N; i += (long long)gridDim.x * 256) {
      const double pi = (double)p[i], ui = (double)u[i];
      if (k < 4 * L) {
        const long long o = (long long)l * N + i;
        if (kind == 0) a += pi * ui * (double)dl[o];
        else if (kind == 1) a += pi * (double)ku[o];
        else if (kind == 2) a += pi * ui * (double)dls[o];
        else a += pi * (double)ksu[o];
      } else if (k == 4 * L) {
        a += pi;
      } else if (k == 4 * L + 1) {
        a += ui;
      } else {
        a += pi * ui;
      }
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if ((int)threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)blockIdx.x * NS + k] = sh[0];
    __syncthreads();
  }
}

__global__ void k_grad_final(const double* __restrict__ part, int nblk, int NS, double* __restrict__ out) {
  for (int k = threadIdx.x; k < NS; k += blockDim.x) {
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[(long long)b * NS + k];
    out[k] = a;
  }
}

template <typename T>
void gradient_sums_t(Plan& P, const void* p, const void* u, std::vector<double>& out, hipStream_t s) {
  const int NS = 4 * P.L + 3;
  const int nblk = (int)std::min<long long>(256, (P.N + 255) / 256);
  double* part = P.adj_part;
  hipLaunchKernelGGL(k_grad_sums<T>, dim3(nblk), dim3(256), 0, s, (const T*)p, (const T*)u,
                     (const T*)P.dl, (const T*)P.yk, (const T*)P.dls, (const T*)P.yks, P.L,
                     (long long)P.N, part);
  double* fin = part + (long long)nblk * NS;
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), 0, s, (const double*)part, nblk, NS, fin);
  NLD_HIP(hipGetLastError());
  out.assign(NS, 0.0);
  NLD_HIP(hipMemcpyAsync(out.data(), fin, NS * sizeof(double), hipMemcpyDeviceToHost, s));
  NLD_HIP(hipStreamSynchronize(s));
}

template <typename T>
void matvec_set_t(const LaunchSet& ls, VecArg in, VecArg out, double* Dout, Epilogue epi,
                  hipStream_t s) {
  // only the iteration's product stops early once a solve has finished
  const int check = (epi == EPI_CG_Q) ? 1 : 0;
  spread_fold<T>(ls, in, check, s);
  planes_all(ls, check, s);
  conv_all<T>(ls, check, s);
  tiles_dispatch<T>(ls, in, check, s, true);
  ReduceArgs a;
  a.in = in;
  a.out = out;
  a.Dout = Dout;
  a.mode = (int)epi;
  const unsigned nb = (epi >= EPI_CG_Q) ? (unsigned)ls.max_nred : grid_for(ls.max_N, kRedThreads);
  hipLaunchKernelGGL(k_reduce<T>, dim3(nb, ls.n_imgs), dim3(kRedThreads), 0, s, ls.d_wins,
                     ls.d_imgs, a);
  NLD_HIP(hipGetLastError());
}

}  // namespace

size_t plane_lds_bytes(int n) {
  return n == 64 ? PlaneShape<64>::lds() : n == 128 ? PlaneShape<128>::lds() : (size_t)1 << 40;
}

void matvec_parts(Plan& P, const void* v, void* yk, void* yks, hipStream_t s) {
  if (P.prec == NLD_FP32) matvec_parts_t<float>(P, v, yk, yks, s);
  else matvec_parts_t<double>(P, v, yk, yks, s);
}

void gradient_sums(Plan& P, const void* p, const void* u, std::vector<double>& out, hipStream_t s) {
  if (P.prec == NLD_FP32) gradient_sums_t<float>(P, p, u, out, s);
  else gradient_sums_t<double>(P, p, u, out, s);
}

void matvec_set(const LaunchSet& ls, VecArg in, VecArg out, double* Dout, Epilogue epi,
                hipStream_t s) {
  if (ls.prec == NLD_FP32) matvec_set_t<float>(ls, in, out, Dout, epi, s);
  else matvec_set_t<double>(ls, in, out, Dout, epi, s);
}

void matvec(Plan& P, const void* v, void* out, Epilogue epi, hipStream_t s) {
  VecArg in{v, V_P}, o{out, V_Q};
  double* Dout = nullptr;
  if (epi == EPI_CG_INIT || epi == EPI_CG_TRUE) {
    in.sel = V_Z;
    o.sel = V_R;
  }
  if (epi == EPI_DEGREE) {
    Dout = static_cast<double*>(out);
    o.ext = nullptr;
  }
  matvec_set(P.ls, in, o, Dout, epi, s);
}

}  // namespace nld
