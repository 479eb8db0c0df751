// Deflated Jacobi-preconditioned CG for (I + alpha L~) u = f (paper Sec. 4.2-4.3, 5.3-5.4).
//
// The paper changes basis with the orthonormal U whose first column is 1/sqrt(N), solves the
// decoupled first component exactly and runs CG on the remaining (N-1) block with the
// preconditioner pi_2(U^T P^-1 U), P = I + alpha diag(eta).  Because U_2 U_2^T is the
// orthogonal projector Pi = I - 1 1^T / N, the same iteration is run here in the original
// coordinates: u = mean(f) 1 + z with z in the complement of 1, residuals projected with Pi
// and the preconditioner applied as s = Pi (r / P).  All scalars and inner products are FP64
// and stay on the device; kernels after convergence return immediately, so the host only
// polls the state every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "nld_device.h"

namespace nld {

namespace {

// Inverse diagonal preconditioner: none (precond 0), Jacobi P_a = 1 + alpha eta (1), or the l2
// diagonal P_b' = (alpha^2 (D2 - sum w_l^2) + P_a^2)^(1/2) of Sec. 4.3.1 (2).
template <typename T>
__device__ __forceinline__ double pinv(const CgState* st, const ImgDev& im, long long i) {
  if (st->precond == 0) return 1.0;
  const double pa = 1.0 + st->alpha * (im.D[i] - st->wsum);
  if (st->precond == 1) return 1.0 / pa;
  const double d2 = fmax(im.D2[i] - st->w2sum, 0.0);   // the off-diagonal sum, never negative
  return 1.0 / sqrt(st->alpha * st->alpha * d2 + pa * pa);
}

// Every CG kernel runs one row of blocks per image (blockIdx.y); the reductions of an image use
// its first nred blocks, so an image's sums do not depend on the other images of the launch.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_cg_stats(const ImgDev* __restrict__ imgs, int u0sel) {
  const ImgDev& im = imgs[blockIdx.y];
  if (blockIdx.x >= (unsigned)im.nred) return;
  CgState* st = im.st;
  const T* f = reinterpret_cast<const T*>(im.vec[V_F]);
  const T* u0 = reinterpret_cast<const T*>(im.vec[u0sel]);
  const long long N = im.N;
  const T f0 = f[0];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)im.nred * kRedThreads) {
    s0 += (double)f[i];
    s1 += (double)u0[i];
    s2 += (f[i] != f0) ? 1.0 : 0.0;
    s3 += pinv<T>(st, im, i);
  }
  const double vals[4] = {s0, s1, s2, s3};
  double tot[4];
  if (!grid_reduce<4>(vals, im.red, &st->ticket[1], tot, im.nred)) return;
  if (threadIdx.x != 0) return;
  st->sum_pinv = tot[3];
  st->mean_f = st->deflate ? tot[0] / (double)N : 0.0;
  st->mean_u0 = st->deflate ? tot[1] / (double)N : 0.0;
  st->const_f = tot[2];
  if (tot[2] == 0.0 && st->deflate) {   // f_perp = 0: u = f, no iteration
    st->done = 1;
    st->status = NLD_OK;
  }
}

template <typename T>
__global__ void k_cg_z0(const ImgDev* __restrict__ imgs, int u0sel) {
  const ImgDev& im = imgs[blockIdx.y];
  const CgState* st = im.st;
  if (st->done) return;
  const T* u0 = reinterpret_cast<const T*>(im.vec[u0sel]);
  T* z = reinterpret_cast<T*>(im.vec[V_Z]);
  const double mu = st->mean_u0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < im.N;
       i += (long long)gridDim.x * blockDim.x)
    z[i] = (T)((double)u0[i] - mu);
}

__device__ __forceinline__ void finish_residual(CgState* st, const double (&tot)[4], long long N,
                                                bool count_iteration) {
  if (count_iteration) st->iters += 1;
  // a non-finite sum (e.g. from a non-finite initial guess) is a breakdown; tested first, since
  // the clamp below would turn a NaN residual into 0
  if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2]) || !isfinite(tot[3])) {
    st->rr = tot[0];
    st->done = 1;
    st->status = NLD_E_BREAKDOWN;
    return;
  }
  const double dN = (double)N;
  const double c = st->deflate ? tot[3] / dN : 0.0;
  const double rr = fmax(tot[0] - c * c * dN, 0.0);
  const double sum_t = tot[1] - c * st->sum_pinv;               // sum r~ / P
  const double rt = tot[2] - 2.0 * c * tot[1] + c * c * st->sum_pinv;   // <r~, r~ / P>
  st->rr = rr;
  st->mean_r = c;
  if (rr <= st->tol2_b2) {
    st->done = 1;
    st->status = NLD_OK;
    return;
  }
  const double mean_t = st->deflate ? sum_t / dN : 0.0;
  const double rho_new = rt;                                    // <r~, r~/P - mean_t>, sum r~ = 0
  st->last_rho = rho_new;
  if (!(rho_new > 0.0) || !isfinite(rho_new) || !isfinite(tot[0])) {
    st->done = 1;
    st->status = NLD_E_BREAKDOWN;
    return;
  }
  st->mean_t = mean_t;
  st->beta = count_iteration ? rho_new / st->rho : 0.0;
  st->rho = rho_new;
  if (st->iters >= st->maxit) {
    st->done = 1;
    st->status = NLD_E_NOCONV;
  }
}

// residual sums of the initial residual
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_cg_init2(const ImgDev* __restrict__ imgs) {
  const ImgDev& im = imgs[blockIdx.y];
  CgState* st = im.st;
  if (st->done || blockIdx.x >= (unsigned)im.nred) return;
  const T* r = reinterpret_cast<const T*>(im.vec[V_R]);
  const long long N = im.N;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)im.nred * kRedThreads) {
    const double rv = (double)r[i];
    const double t = rv * pinv<T>(st, im, i);
    s[0] += rv * rv;
    s[1] += t;
    s[2] += rv * t;
    s[3] += rv;
  }
  double tot[4];
  if (!grid_reduce<4>(s, im.red, &st->ticket[2], tot, im.nred)) return;
  if (threadIdx.x == 0) finish_residual(st, tot, N, false);
}

// z += a p, r -= a Pi q, then the residual sums
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_cg_update(const ImgDev* __restrict__ imgs) {
  const ImgDev& im = imgs[blockIdx.y];
  CgState* st = im.st;
  if (st->done || blockIdx.x >= (unsigned)im.nred) return;
  T* __restrict__ z = reinterpret_cast<T*>(im.vec[V_Z]);
  T* __restrict__ r = reinterpret_cast<T*>(im.vec[V_R]);
  const T* __restrict__ p = reinterpret_cast<const T*>(im.vec[V_P]);
  const T* __restrict__ q = reinterpret_cast<const T*>(im.vec[V_Q]);
  const long long N = im.N;
  const double a = st->a, mq = st->mean_q;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  // a thread's entries i, i + S, i + 2S, ... in that order (the sums' order); the loads of four
  // of them are issued before any of their stores, one memory round trip per four entries
  constexpr int U = 4;
  const long long S = (long long)im.nred * kRedThreads;
  for (long long i0 = blockIdx.x * (long long)kRedThreads + threadIdx.x; i0 < N; i0 += U * S) {
    double zv[U], pv[U], rv0[U], qv[U], pi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * S < N ? i0 + u * S : i0;     // past the end: a valid entry
      zv[u] = (double)z[i];
      pv[u] = (double)p[i];
      rv0[u] = (double)r[i];
      qv[u] = (double)q[i];
      pi[u] = pinv<T>(st, im, i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * S;
      if (i >= N) break;
      z[i] = (T)(zv[u] + a * pv[u]);
      const T rt = (T)(rv0[u] - a * (qv[u] - mq));
      r[i] = rt;
      const double rv = (double)rt;
      const double t = rv * pi[u];
      s[0] += rv * rv;
      s[1] += t;
      s[2] += rv * t;
      s[3] += rv;
    }
  }
  double tot[4];
  if (!grid_reduce<4>(s, im.red, &st->ticket[3], tot, im.nred)) return;
  if (threadIdx.x == 0) finish_residual(st, tot, N, true);
}

// r <- r - mean(r) (stored residual back into the complement of 1), p <- Pi(r / P) + beta p
template <typename T>
__global__ void k_cg_direction(const ImgDev* __restrict__ imgs, int first) {
  const ImgDev& im = imgs[blockIdx.y];
  const CgState* st = im.st;
  if (st->done) return;
  T* __restrict__ r = reinterpret_cast<T*>(im.vec[V_R]);
  T* __restrict__ p = reinterpret_cast<T*>(im.vec[V_P]);
  const double mt = st->mean_t, beta = st->beta, c = st->mean_r;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < im.N;
       i += (long long)gridDim.x * blockDim.x) {
    const double rv = (double)r[i] - c;
    r[i] = (T)rv;
    const double s = rv * pinv<T>(st, im, i) - mt;
    p[i] = (T)(first ? s : s + beta * (double)p[i]);
  }
}

// Energy-optimal multiple of a warm start: with z = Pi u0 and r = f_perp - A z (the initial
// residual just formed), <z, A z> = <z, f_perp> - <z, r>, and b = <z, f_perp> / <z, A z>
// minimises ||b z - z*||_A over b (A z* = f_perp), so the scaled start is never farther from
// the solution in the energy norm than the zero start u = mean(f) 1.  b = 0 when <z, A z> is not
// positive and finite (a constant guess).
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_cg_scale_sums(const ImgDev* __restrict__ imgs) {
  const ImgDev& im = imgs[blockIdx.y];
  CgState* st = im.st;
  if (st->done || blockIdx.x >= (unsigned)im.nred) return;
  const T* z = reinterpret_cast<const T*>(im.vec[V_Z]);
  const T* r = reinterpret_cast<const T*>(im.vec[V_R]);
  const T* f = reinterpret_cast<const T*>(im.vec[V_F]);
  const double mf = st->mean_f;
  double s[2] = {0.0, 0.0};
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < im.N;
       i += (long long)im.nred * kRedThreads) {
    const double zi = (double)z[i];
    s[0] += zi * ((double)f[i] - mf);
    s[1] += zi * (double)r[i];
  }
  double tot[2];
  if (!grid_reduce<2>(s, im.red, &st->ticket[4], tot, im.nred)) return;
  if (threadIdx.x != 0) return;
  const double zaz = tot[0] - tot[1];
  st->scale_b = (zaz > 0.0 && isfinite(zaz) && isfinite(tot[0])) ? tot[0] / zaz : 0.0;
}

// z <- b z, r <- f_perp - A (b z) = (1 - b) f_perp + b r
template <typename T>
__global__ void k_cg_scale_apply(const ImgDev* __restrict__ imgs) {
  const ImgDev& im = imgs[blockIdx.y];
  const CgState* st = im.st;
  if (st->done) return;
  T* __restrict__ z = reinterpret_cast<T*>(im.vec[V_Z]);
  T* __restrict__ r = reinterpret_cast<T*>(im.vec[V_R]);
  const T* __restrict__ f = reinterpret_cast<const T*>(im.vec[V_F]);
  const double b = st->scale_b, mf = st->mean_f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < im.N;
       i += (long long)gridDim.x * blockDim.x) {
    z[i] = (T)(b * (double)z[i]);
    r[i] = (T)((1.0 - b) * ((double)f[i] - mf) + b * (double)r[i]);
  }
}

template <typename T>
__global__ void k_cg_finish(const ImgDev* __restrict__ imgs) {
  const ImgDev& im = imgs[blockIdx.y];
  const CgState* st = im.st;
  const T* z = reinterpret_cast<const T*>(im.vec[V_Z]);
  const T* f = reinterpret_cast<const T*>(im.vec[V_F]);
  T* u = reinterpret_cast<T*>(im.vec[V_U]);
  const bool constant = st->const_f == 0.0 && st->deflate;
  const double mf = st->mean_f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < im.N;
       i += (long long)gridDim.x * blockDim.x)
    u[i] = constant ? f[i] : (T)(mf + (double)z[i]);
}

// per-block maxima of x (grid-stride), the first stage of max_eta
__global__ void k_max_part(const double* __restrict__ x, long long N, double* __restrict__ part) {
  __shared__ double sh[256];
  double m = -INFINITY;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < N; i += (long long)gridDim.x * 256)
    m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_max(const double* __restrict__ x, long long N, double* __restrict__ out) {
  __shared__ double sh[1024];
  double m = -INFINITY;
  for (long long i = threadIdx.x; i < N; i += 1024) m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// max of every image's degree vector, one block per image
__global__ void k_max_imgs(const ImgDev* __restrict__ imgs, double* __restrict__ out) {
  const ImgDev& im = imgs[blockIdx.x];
  __shared__ double sh[1024];
  double m = -INFINITY;
  for (long long i = threadIdx.x; i < im.N; i += 1024) m = fmax(m, im.D[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

inline unsigned grid_for(long long n, int threads = 256) {
  long long b = (n + threads - 1) / threads;
  return (unsigned)std::max<long long>(1, std::min<long long>(b, 16384));
}

template <typename T>
nld_status run_pcg_t(Plan& P, double alpha, const void* f, void* u, const nld_pcg_opts& o,
                     nld_pcg_info& info, hipStream_t s) {
  const long long N = P.N;
  const auto t0 = std::chrono::steady_clock::now();
  double wsum = 0.0;
  for (double w : P.weight) wsum += w;
  CgState* h = P.st_host;
  *h = CgState{};
  h->alpha = alpha;
  h->tol = o.tol;
  h->wsum = wsum;
  h->maxit = o.maxit;
  h->precond = o.precond;
  h->deflate = o.deflate;
  for (double w : P.weight) h->w2sum += w * w;
  h->status = NLD_OK;
  NLD_HIP(hipMemcpyAsync(P.st, h, sizeof(CgState), hipMemcpyHostToDevice, s));
  P.img_host->vec[V_F] = const_cast<void*>(f);
  P.img_host->vec[V_U] = u;
  NLD_HIP(hipMemcpyAsync(P.d_img, P.img_host, sizeof(ImgDev), hipMemcpyHostToDevice, s));
  const dim3 rb(P.ls.max_nred, 1);
  const dim3 gb(grid_for(N), 1);
  const ImgDev* im = P.d_img;
  const CgState fresh = *h;
  // initial state and residual r0 = Pi (f_perp - A z0) of the start u0 = vec[sel]
  auto init_from = [&](int sel, bool reset) {
    if (reset) {
      *h = fresh;
      NLD_HIP(hipMemcpyAsync(P.st, h, sizeof(CgState), hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_cg_stats<T>, rb, dim3(kRedThreads), 0, s, im, sel);
    hipLaunchKernelGGL(k_cg_z0<T>, gb, dim3(256), 0, s, im, sel);
    NLD_HIP(hipGetLastError());
    matvec(P, nullptr, nullptr, EPI_CG_INIT, s);
    hipLaunchKernelGGL(k_cg_init2<T>, rb, dim3(kRedThreads), 0, s, im);
    NLD_HIP(hipGetLastError());
  };
  auto read_state = [&]() {
    NLD_HIP(hipMemcpyAsync(h, P.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    NLD_HIP(hipStreamSynchronize(s));
  };
  info.u0_rejected = 0;
  if (!o.use_u0) {
    init_from(V_F, false);
  } else {
    // warm start with plain PCG as the fallback: a guess whose initial residual is not finite
    // (use_u0 = 1, 3), or also exceeds the residual of the plain start u0 = f (use_u0 = 2), is
    // replaced by f; use_u0 = 3 starts from the energy-optimal multiple of the guess
    double rr_f = INFINITY;
    bool plain_done = false;
    if (o.use_u0 == 2) {
      init_from(V_F, false);
      read_state();
      rr_f = h->rr;
      plain_done = h->done != 0;          // constant f, or f already within the tolerance
    }
    if (!plain_done) {
      init_from(V_U, o.use_u0 == 2);
      read_state();
      const bool bad = h->status == NLD_E_BREAKDOWN || !std::isfinite(h->rr) ||
                       (o.use_u0 == 2 && h->rr > rr_f);
      if (bad) {
        info.u0_rejected = 1;
        init_from(V_F, true);
      } else if (o.use_u0 == 3) {
        // start from the energy-optimal multiple of the guess, then the residual sums again
        h->done = 0;
        h->status = NLD_OK;
        NLD_HIP(hipMemcpyAsync(P.st, h, sizeof(CgState), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_cg_scale_sums<T>, rb, dim3(kRedThreads), 0, s, im);
        hipLaunchKernelGGL(k_cg_scale_apply<T>, gb, dim3(256), 0, s, im);
        hipLaunchKernelGGL(k_cg_init2<T>, rb, dim3(kRedThreads), 0, s, im);
        NLD_HIP(hipGetLastError());
      }
    }
  }
  hipLaunchKernelGGL(k_cg_direction<T>, gb, dim3(256), 0, s, im, 1);
  NLD_HIP(hipGetLastError());
  const bool trace = std::getenv("NLD_TRACE_CG") != nullptr;
  const int chunk = trace ? 1 : 4;
  int launched = 0;
  // optional event pairs around every operator application of the loop
  std::vector<hipEvent_t> ev;
  auto new_event = [&]() {
    hipEvent_t e;
    NLD_HIP(hipEventCreate(&e));
    ev.push_back(e);
    return e;
  };
  while (true) {
    NLD_HIP(hipMemcpyAsync(h, P.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    NLD_HIP(hipStreamSynchronize(s));
    if (trace)
      std::fprintf(stderr, "cg it=%d done=%d st=%d rr=%.6e rho=%.6e a=%.6e beta=%.6e mean_t=%.3e "
                   "mean_q=%.3e mean_r=%.3e b2=%.6e pq=%.6e rho_new=%.6e\n", h->iters, h->done, h->status,
                   h->rr, h->rho, h->a, h->beta, h->mean_t, h->mean_q, h->mean_r, h->bnorm2,
                   h->last_pq, h->last_rho);
    if (h->done || launched >= o.maxit) break;
    for (int k = 0; k < chunk; ++k) {
      if (o.timing) NLD_HIP(hipEventRecord(new_event(), s));
      matvec(P, nullptr, nullptr, EPI_CG_Q, s);
      if (o.timing) NLD_HIP(hipEventRecord(new_event(), s));
      hipLaunchKernelGGL(k_cg_update<T>, rb, dim3(kRedThreads), 0, s, im);
      hipLaunchKernelGGL(k_cg_direction<T>, gb, dim3(256), 0, s, im, 0);
      NLD_HIP(hipGetLastError());
      ++launched;
    }
  }
  hipLaunchKernelGGL(k_cg_finish<T>, gb, dim3(256), 0, s, im);
  NLD_HIP(hipGetLastError());
  double rr_true = -1.0;
  if (o.true_residual && !(h->const_f == 0.0 && o.deflate)) {
    // true residual of the final iterate: || Pi (f_perp - A z) ||
    matvec(P, nullptr, nullptr, EPI_CG_TRUE, s);
  }
  NLD_HIP(hipMemcpyAsync(h, P.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  NLD_HIP(hipStreamSynchronize(s));
  if (o.true_residual && !(h->const_f == 0.0 && o.deflate)) rr_true = h->rr_true;
  const auto t1 = std::chrono::steady_clock::now();
  info.iters = h->iters;
  info.ms_matvec = 0.0;
  info.matvecs_timed = 0;
  if (o.timing) {
    // operator applications after convergence return at once: count only the executed ones
    const int used = std::min<int>((int)ev.size() / 2, h->iters);
    double tot = 0.0;
    for (int k = 0; k < used; ++k) {
      float ms = 0.f;
      NLD_HIP(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
      tot += ms;
    }
    info.ms_matvec = used > 0 ? tot / used : 0.0;
    info.matvecs_timed = used;
  }
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  const double b2 = h->bnorm2;
  info.relres_rec = (h->const_f == 0.0 && o.deflate) ? 0.0 : (b2 > 0 ? std::sqrt(h->rr / b2) : 0.0);
  info.relres_true = rr_true >= 0 ? (b2 > 0 ? std::sqrt(std::max(rr_true, 0.0) / b2) : 0.0) : -1.0;
  info.kappa_est = 2.0 * alpha * (P.max_eta) + 1.0;
  info.ms_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
  nld_status stt = (nld_status)h->status;
  if (stt == NLD_OK && !h->done) stt = NLD_E_NOCONV;
  info.status = stt;
  return stt;
}

}  // namespace

void compute_max_eta(Plan& P, hipStream_t s) {
  // per-block maxima over 1024 blocks, then their maximum (max is exact in any order)
  constexpr int kParts = 1024;
  double* d = nullptr;
  NLD_HIP(hipMallocAsync((void**)&d, (kParts + 1) * sizeof(double), s));
  const long long nb = std::max<long long>(1, std::min<long long>(kParts, (P.N + 255) / 256));
  hipLaunchKernelGGL(k_max_part, dim3((unsigned)nb), dim3(256), 0, s, P.D, (long long)P.N, d + 1);
  NLD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, (const double*)(d + 1), nb, d);
  NLD_HIP(hipGetLastError());
  double mx = 0.0;
  NLD_HIP(hipMemcpyAsync(&mx, d, sizeof(double), hipMemcpyDeviceToHost, s));
  NLD_HIP(hipStreamSynchronize(s));
  (void)hipFreeAsync(d, s);
  double wsum = 0.0;
  for (double w : P.weight) wsum += w;
  P.max_eta = mx - wsum;
}

nld_status run_adjoint(Plan& P, double alpha, const void* u, const void* g, void* p, double* grad,
                       const nld_pcg_opts& o, nld_pcg_info& info, hipStream_t s) {
  // adjoint state: A p = g with the same symmetric operator
  const nld_status st = run_pcg(P, alpha, g, p, o, info, s);
  const long long LN = (long long)P.N * P.L;
  auto alloc = [&](void** b, size_t bytes) {   // owned by the plan, returned on release
    if (!*b) *b = plan_buffer(bytes, s);
  };
  alloc(&P.yk, LN * P.elem);
  alloc(&P.yks, LN * P.elem);
  alloc(&P.grid_save, (size_t)P.grid_total * P.elem);
  alloc((void**)&P.adj_part, (size_t)257 * (4 * P.L + 3) * sizeof(double));
  alloc(&P.dl, LN * P.elem);
  alloc(&P.dls, LN * P.elem);
  if (!P.have_dl) {
    matvec_parts(P, P.ones, P.dl, P.dls, s);     // per-window degrees K_l 1 and K^s_l 1
    P.have_dl = true;
  }
  matvec_parts(P, u, P.yk, P.yks, s);
  std::vector<double> sums;
  gradient_sums(P, p, u, sums, s);
  const int L = P.L;
  const double sp = sums[4 * L], su = sums[4 * L + 1], spu = sums[4 * L + 2];
  double g_la = 0.0;
  for (int l = 0; l < L; ++l) {
    double pLu, pLsu;
    if (P.wins[l].t > 0) {
      pLu = sums[4 * l] - sums[4 * l + 1];            // p^T (diag(K_l 1) - K_l) u
      pLsu = sums[4 * l + 2] - sums[4 * l + 3];
    } else {                                          // K_l = 1 1^T, sigma derivative 0
      pLu = (double)P.N * spu - sp * su;
      pLsu = 0.0;
    }
    const double gw = -alpha * pLu;
    grad[1 + L + l] = gw;                             // d J / d w_l
    grad[1 + l] = -alpha * P.weight[l] * pLsu;        // d J / d log sigma_l
    g_la += P.weight[l] * gw;                         // alpha scales every weight
  }
  grad[0] = g_la;                                     // d J / d log alpha
  return st;
}

nld_status run_pcg(Plan& P, double alpha, const void* f, void* u, const nld_pcg_opts& o,
                   nld_pcg_info& info, hipStream_t s) {
  if (o.precond == 2) ensure_l2_degree(P, s);
  if (!P.have_D) {
    matvec(P, P.ones, P.D, EPI_DEGREE, s);
    P.have_D = true;
    compute_max_eta(P, s);
  }
  if (P.prec == NLD_FP32) return run_pcg_t<float>(P, alpha, f, u, o, info, s);
  return run_pcg_t<double>(P, alpha, f, u, o, info, s);
}

// ---------------------------------------------------------------------------- batched solves
// Independent solves of several plans advance together: the window tables, schedules and image
// tables of the plans are concatenated, so every stage of an iteration (spreading, fold, the
// convolution passes, gathering, the epilogue and the CG updates) is one launch for the whole
// batch, and a finished solve only costs the early exit of its workgroups.  Each image keeps
// its own reduction blocks, so its iterates are bit-identical to a solve of its plan alone.
// A chunk of iterations is captured once as a HIP graph and replayed until every solve has
// finished (polled on the host between chunks).

namespace {

template <typename X>
X* dev_copy(const std::vector<X>& h, hipStream_t s, std::vector<void*>& owned) {
  X* d = nullptr;
  NLD_HIP(hipMallocAsync((void**)&d, std::max<size_t>(1, h.size()) * sizeof(X), s));
  owned.push_back(d);
  if (!h.empty()) NLD_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice, s));
  return d;
}

hipStream_t batch_stream() {
  // one non-blocking stream (default priority) per device for the captured iteration chunks
  static hipStream_t streams[64] = {};
  int dev = 0;
  NLD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw std::runtime_error("device index out of range");
  if (!streams[dev]) NLD_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

template <typename T>
nld_status run_pcg_batched_t(Plan* const* plans, const double* alpha, const void* const* f,
                             void* const* u, int count, const nld_pcg_opts& o, nld_pcg_info* infos,
                             hipStream_t s) {
  if (o.precond == 2)
    for (int b = 0; b < count; ++b) ensure_l2_degree(*plans[b], s);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t cs = batch_stream();
  hipEvent_t ev_in, ev_out;
  NLD_HIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
  NLD_HIP(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  NLD_HIP(hipEventRecord(ev_in, s));
  NLD_HIP(hipStreamWaitEvent(cs, ev_in, 0));
  std::vector<void*> owned;
  CgState* sth = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* b : owned) (void)hipFreeAsync(b, cs);
    (void)hipStreamSynchronize(cs);
    pinned_put(sth);
    (void)hipEventDestroy(ev_in);
    (void)hipEventDestroy(ev_out);
  };
  try {
    // ---- concatenated tables
    std::vector<WinDev> wins;
    std::vector<TileJob> tj[3], gj[3];
    std::vector<Fold3Job> f3[2];
    std::vector<FoldJob> fj;
    std::vector<ConvJob> cj[3][4];
    std::vector<PlaneJob> pj[2];
    std::vector<ImgDev> imgs(count);
    LaunchSet ls;
    ls.prec = plans[0]->prec;
    ls.m = plans[0]->wins[0].m;
    ls.n_imgs = count;
    ls.ts3 = 8;                                   // unless a plan's 3-D windows use 16^3 tiles
    ls.f3_quad = true;                            // unless a plan's 3-D windows break the groups
    CgState* d_st = nullptr;
    NLD_HIP(hipMallocAsync((void**)&d_st, (size_t)count * sizeof(CgState), cs));
    owned.push_back(d_st);
    double* d_red = nullptr;
    NLD_HIP(hipMallocAsync((void**)&d_red, (size_t)count * kRedBlocks * 8 * sizeof(double), cs));
    owned.push_back(d_red);
    for (int b = 0; b < count; ++b) {
      Plan& P = *plans[b];
      const int wo = (int)wins.size();
      for (const WinDev& w0 : P.wins) {
        WinDev w = w0;
        w.img = b;
        wins.push_back(w);
      }
      for (int g = 0; g < 3; ++g)
        for (int j = P.tjob_begin[g]; j < P.tjob_begin[g + 1]; ++j) {
          TileJob t = P.h_tjobs[j];
          t.win += wo;
          tj[g].push_back(t);
          TileJob u = P.h_gjobs[j];
          u.win += wo;
          gj[g].push_back(u);
        }
      for (Fold3Job j : P.h_f3jobs) {
        j.win += wo;
        f3[P.f3_ts == 16 ? 1 : 0].push_back(j);
      }
      for (FoldJob j : P.h_fjobs) {
        j.win += wo;
        fj.push_back(j);
      }
      for (int gi = 0; gi < 2; ++gi)
        for (int j = P.pjob_begin[gi]; j < P.pjob_begin[gi + 1]; ++j) {
          PlaneJob q = P.h_pjobs[j];
          q.win += wo;
          pj[gi].push_back(q);
        }
      for (int ax = 0; ax < 3; ++ax)
        for (int gi = 0; gi < 4; ++gi)
          for (int j = P.conv_begin[ax][gi]; j < P.conv_begin[ax][gi + 1]; ++j) {
            ConvJob c = P.h_conv[ax][j];
            c.win += wo;
            cj[ax][gi].push_back(c);
          }
      ImgDev& im = imgs[b];
      im = *P.img_host;
      im.win0 = wo;
      im.vec[V_F] = const_cast<void*>(f[b]);
      im.vec[V_U] = u[b];
      im.st = d_st + b;
      im.red = d_red + (size_t)b * kRedBlocks * 8;
      ls.max_padded = std::max(ls.max_padded, P.max_padded);
      if (P.f3_ts == 16) ls.ts3 = 0;
      ls.f3_quad = ls.f3_quad && P.f3_quad;
      ls.max_N = std::max<long long>(ls.max_N, P.N);
      ls.max_nred = std::max(ls.max_nred, im.nred);
      ls.has_flat = ls.has_flat || P.has_flat;
    }
    std::vector<TileJob> tjobs, gjobs;
    for (int g = 0; g < 3; ++g) {
      // largest chunks first, across the whole batch; the gathering's order per XCD range
      sort_by_size_desc(tj[g], 0, tj[g].size());
      ls.tjob_begin[g] = (int)tjobs.size();
      tjobs.insert(tjobs.end(), tj[g].begin(), tj[g].end());
      gjobs.insert(gjobs.end(), gj[g].begin(), gj[g].end());
      gather_order(gjobs, ls.tjob_begin[g], gjobs.size());
    }
    ls.tjob_begin[3] = (int)tjobs.size();
    std::vector<Fold3Job> f3all(f3[0]);
    f3all.insert(f3all.end(), f3[1].begin(), f3[1].end());
    ls.f3_begin[0] = 0;
    ls.f3_begin[1] = (int)f3[0].size();
    ls.f3_begin[2] = (int)f3all.size();
    ls.n_fjobs = (int)fj.size();
    ls.d_wins = dev_copy(wins, cs, owned);
    ls.d_tjobs = dev_copy(tjobs, cs, owned);
    ls.d_gjobs = dev_copy(gjobs, cs, owned);
    ls.d_f3jobs = dev_copy(f3all, cs, owned);
    ls.d_fjobs = dev_copy(fj, cs, owned);
    for (int ax = 0; ax < 3; ++ax) {
      std::vector<ConvJob> all;
      for (int gi = 0; gi < 4; ++gi) {
        ls.conv_begin[ax][gi] = (int)all.size();
        all.insert(all.end(), cj[ax][gi].begin(), cj[ax][gi].end());
      }
      ls.conv_begin[ax][4] = (int)all.size();
      ls.d_conv[ax] = dev_copy(all, cs, owned);
    }
    {
      std::vector<PlaneJob> all(pj[0]);
      all.insert(all.end(), pj[1].begin(), pj[1].end());
      ls.pjob_begin[0] = 0;
      ls.pjob_begin[1] = (int)pj[0].size();
      ls.pjob_begin[2] = (int)all.size();
      ls.d_pjobs = dev_copy(all, cs, owned);
    }
    ls.d_imgs = dev_copy(imgs, cs, owned);

    // ---- degree vectors (every image, if any plan still lacks its own) and max eta
    bool need_D = false;
    for (int b = 0; b < count; ++b) need_D = need_D || !plans[b]->have_D;
    sth = (CgState*)pinned_get((size_t)count * sizeof(CgState));
    if (need_D) {
      matvec_set(ls, VecArg{nullptr, V_ONES}, VecArg{nullptr, V_Q}, nullptr, EPI_DEGREE, cs);
      double* d_max = nullptr;
      NLD_HIP(hipMallocAsync((void**)&d_max, (size_t)count * sizeof(double), cs));
      owned.push_back(d_max);
      hipLaunchKernelGGL(k_max_imgs, dim3(count), dim3(1024), 0, cs, ls.d_imgs, d_max);
      NLD_HIP(hipGetLastError());
      std::vector<double> mx(count);
      NLD_HIP(hipMemcpyAsync(mx.data(), d_max, count * sizeof(double), hipMemcpyDeviceToHost, cs));
      NLD_HIP(hipStreamSynchronize(cs));
      for (int b = 0; b < count; ++b) {
        double wsum = 0.0;
        for (double w : plans[b]->weight) wsum += w;
        plans[b]->max_eta = mx[b] - wsum;
        plans[b]->have_D = true;
      }
    }

    // ---- CG set-up
    for (int b = 0; b < count; ++b) {
      double wsum = 0.0;
      for (double w : plans[b]->weight) wsum += w;
      CgState& h = sth[b];
      h = CgState{};
      h.alpha = alpha[b];
      h.tol = o.tol;
      h.wsum = wsum;
      h.maxit = o.maxit;
      h.precond = o.precond;
      h.deflate = o.deflate;
      for (double w : plans[b]->weight) h.w2sum += w * w;
      h.status = NLD_OK;
    }
    NLD_HIP(hipMemcpyAsync(d_st, sth, (size_t)count * sizeof(CgState), hipMemcpyHostToDevice, cs));
    const int u0sel = o.use_u0 ? V_U : V_F;
    const dim3 rb(ls.max_nred, count);
    const dim3 gb(grid_for(ls.max_N), count);
    const ImgDev* dimg = ls.d_imgs;
    hipLaunchKernelGGL(k_cg_stats<T>, rb, dim3(kRedThreads), 0, cs, dimg, u0sel);
    hipLaunchKernelGGL(k_cg_z0<T>, gb, dim3(256), 0, cs, dimg, u0sel);
    NLD_HIP(hipGetLastError());
    matvec_set(ls, VecArg{nullptr, V_Z}, VecArg{nullptr, V_R}, nullptr, EPI_CG_INIT, cs);
    hipLaunchKernelGGL(k_cg_init2<T>, rb, dim3(kRedThreads), 0, cs, dimg);
    hipLaunchKernelGGL(k_cg_direction<T>, gb, dim3(256), 0, cs, dimg, 1);
    NLD_HIP(hipGetLastError());

    // ---- iterations: chunks of 4, captured once as a graph
    const int chunk = 4;
    auto body = [&]() {
      for (int k = 0; k < chunk; ++k) {
        matvec_set(ls, VecArg{nullptr, V_P}, VecArg{nullptr, V_Q}, nullptr, EPI_CG_Q, cs);
        hipLaunchKernelGGL(k_cg_update<T>, rb, dim3(kRedThreads), 0, cs, dimg);
        hipLaunchKernelGGL(k_cg_direction<T>, gb, dim3(256), 0, cs, dimg, 0);
        NLD_HIP(hipGetLastError());
      }
    };
    const bool use_graph = std::getenv("NLD_NO_GRAPH") == nullptr;
    std::vector<double> done_ms(count, -1.0);
    int launched = 0;
    bool captured = false;
    while (true) {
      NLD_HIP(hipMemcpyAsync(sth, d_st, (size_t)count * sizeof(CgState), hipMemcpyDeviceToHost, cs));
      NLD_HIP(hipStreamSynchronize(cs));
      const double now = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      int open = 0;
      for (int b = 0; b < count; ++b) {
        if (sth[b].done && done_ms[b] < 0) done_ms[b] = now;
        open += !sth[b].done;
      }
      if (open == 0 || launched >= o.maxit) break;
      if (use_graph && launched > 0 && !captured) {
        // the first chunk ran eagerly (kernel attributes are set); capture the next one
        captured = true;
        NLD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        body();
        NLD_HIP(hipStreamEndCapture(cs, &graph));
        NLD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      }
      if (exec) NLD_HIP(hipGraphLaunch(exec, cs));
      else body();
      launched += chunk;
    }

    // ---- solutions, true residuals, reports
    hipLaunchKernelGGL(k_cg_finish<T>, gb, dim3(256), 0, cs, dimg);
    NLD_HIP(hipGetLastError());
    if (o.true_residual) matvec_set(ls, VecArg{nullptr, V_Z}, VecArg{nullptr, V_R}, nullptr, EPI_CG_TRUE, cs);
    NLD_HIP(hipMemcpyAsync(sth, d_st, (size_t)count * sizeof(CgState), hipMemcpyDeviceToHost, cs));
    NLD_HIP(hipStreamSynchronize(cs));
    const double end_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    nld_status worst = NLD_OK;
    for (int b = 0; b < count; ++b) {
      const CgState& h = sth[b];
      nld_pcg_info& info = infos[b];
      const bool cst = h.const_f == 0.0 && o.deflate;
      info.iters = h.iters;
      const double b2 = h.bnorm2;
      info.relres_rec = cst ? 0.0 : (b2 > 0 ? std::sqrt(h.rr / b2) : 0.0);
      info.relres_true = (o.true_residual && !cst) ? (b2 > 0 ? std::sqrt(std::max(h.rr_true, 0.0) / b2) : 0.0) : -1.0;
      info.kappa_est = 2.0 * alpha[b] * plans[b]->max_eta + 1.0;
      info.ms_solve = done_ms[b] >= 0 ? done_ms[b] : end_ms;
      info.ms_matvec = 0.0;
      info.matvecs_timed = 0;
      nld_status stt = (nld_status)h.status;
      if (stt == NLD_OK && !h.done) stt = NLD_E_NOCONV;
      info.status = stt;
      if (stt != NLD_OK && worst == NLD_OK) worst = stt;
    }
    NLD_HIP(hipEventRecord(ev_out, cs));
    NLD_HIP(hipStreamWaitEvent(s, ev_out, 0));
    cleanup();
    return worst;
  } catch (...) {
    (void)hipStreamEndCapture(cs, &graph);
    cleanup();
    throw;
  }
}

}  // namespace

nld_status run_pcg_batched(Plan* const* plans, const double* alpha, const void* const* f,
                           void* const* u, int count, const nld_pcg_opts& o, nld_pcg_info* infos,
                           hipStream_t s) {
  if (plans[0]->prec == NLD_FP32) return run_pcg_batched_t<float>(plans, alpha, f, u, count, o, infos, s);
  return run_pcg_batched_t<double>(plans, alpha, f, u, count, o, infos, s);
}

}  // namespace nld
