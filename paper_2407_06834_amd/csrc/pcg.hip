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

template <typename T>
__device__ __forceinline__ double pinv(const CgState* st, const double* D, long long i) {
  return st->precond ? 1.0 / (1.0 + st->alpha * (D[i] - st->wsum)) : 1.0;
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_cg_stats(const T* __restrict__ f, const T* __restrict__ u0, const double* __restrict__ D,
           long long N, CgState* st, double* red) {
  const T f0 = f[0];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kRedThreads) {
    s0 += (double)f[i];
    s1 += (double)u0[i];
    s2 += (f[i] != f0) ? 1.0 : 0.0;
    s3 += pinv<T>(st, D, i);
  }
  const double vals[4] = {s0, s1, s2, s3};
  double tot[4];
  if (!grid_reduce<4>(vals, red, &st->ticket[1], tot)) return;
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
__global__ void k_cg_z0(const T* __restrict__ u0, T* __restrict__ z, long long N,
                        const CgState* __restrict__ st) {
  if (st->done) return;
  const double mu = st->mean_u0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    z[i] = (T)((double)u0[i] - mu);
}

// Residual bookkeeping from sums over the stored residual r (precision T):
//   tot = {sum r^2, sum t, sum r t, sum r},  t = r / P.
// The stored r may carry a rounding-level component along 1; it is removed here analytically
// (c = mean(r), r~ = r - c) and from the stored vector by the next direction kernel, so the
// residual norm, rho = <r~, Pi(r~ / P)> and the projected preconditioned residual all refer
// to r~ in the complement of 1.  (Without this the constant component, which the updates
// never reduce, puts a floor under the residual in FP32.)
__device__ __forceinline__ void finish_residual(CgState* st, const double (&tot)[4], long long N,
                                                bool count_iteration) {
  if (count_iteration) st->iters += 1;
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
__global__ void __launch_bounds__(kRedThreads)
k_cg_init2(const T* __restrict__ r, const double* __restrict__ D, long long N, CgState* st,
           double* red) {
  if (st->done) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kRedThreads) {
    const double rv = (double)r[i];
    const double t = rv * pinv<T>(st, D, i);
    s[0] += rv * rv;
    s[1] += t;
    s[2] += rv * t;
    s[3] += rv;
  }
  double tot[4];
  if (!grid_reduce<4>(s, red, &st->ticket[2], tot)) return;
  if (threadIdx.x == 0) finish_residual(st, tot, N, false);
}

// z += a p, r -= a Pi q, then the residual sums
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_cg_update(T* __restrict__ z, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
            const double* __restrict__ D, long long N, CgState* st, double* red) {
  if (st->done) return;
  const double a = st->a, mq = st->mean_q;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kRedThreads) {
    z[i] = (T)((double)z[i] + a * (double)p[i]);
    const T rt = (T)((double)r[i] - a * ((double)q[i] - mq));
    r[i] = rt;
    const double rv = (double)rt;
    const double t = rv * pinv<T>(st, D, i);
    s[0] += rv * rv;
    s[1] += t;
    s[2] += rv * t;
    s[3] += rv;
  }
  double tot[4];
  if (!grid_reduce<4>(s, red, &st->ticket[3], tot)) return;
  if (threadIdx.x == 0) finish_residual(st, tot, N, true);
}

// r <- r - mean(r) (stored residual back into the complement of 1), p <- Pi(r / P) + beta p
template <typename T>
__global__ void k_cg_direction(T* __restrict__ r, T* __restrict__ p, const double* __restrict__ D,
                               long long N, const CgState* __restrict__ st, int first) {
  if (st->done) return;
  const double mt = st->mean_t, beta = st->beta, c = st->mean_r;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const double rv = (double)r[i] - c;
    r[i] = (T)rv;
    const double s = rv * pinv<T>(st, D, i) - mt;
    p[i] = (T)(first ? s : s + beta * (double)p[i]);
  }
}

template <typename T>
__global__ void k_cg_finish(const T* __restrict__ z, const T* __restrict__ f, T* __restrict__ u,
                            long long N, const CgState* __restrict__ st) {
  const bool constant = st->const_f == 0.0 && st->deflate;
  const double mf = st->mean_f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    u[i] = constant ? f[i] : (T)(mf + (double)z[i]);
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
  h->status = NLD_OK;
  NLD_HIP(hipMemcpyAsync(P.st, h, sizeof(CgState), hipMemcpyHostToDevice, s));
  const T* u0 = (const T*)(o.use_u0 ? u : f);
  const unsigned rb = red_blocks(N);
  const unsigned gb = grid_for(N);
  hipLaunchKernelGGL(k_cg_stats<T>, dim3(rb), dim3(kRedThreads), 0, s, (const T*)f, u0, P.D, N, P.st,
                     P.red);
  hipLaunchKernelGGL(k_cg_z0<T>, dim3(gb), dim3(256), 0, s, u0, (T*)P.z, N, P.st);
  NLD_HIP(hipGetLastError());
  matvec(P, P.z, P.r, EPI_CG_INIT, f, s);
  hipLaunchKernelGGL(k_cg_init2<T>, dim3(rb), dim3(kRedThreads), 0, s, (const T*)P.r, P.D, N, P.st,
                     P.red);
  hipLaunchKernelGGL(k_cg_direction<T>, dim3(gb), dim3(256), 0, s, (T*)P.r, (T*)P.p, P.D, N, P.st, 1);
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
      matvec(P, P.p, P.q, EPI_CG_Q, nullptr, s);
      if (o.timing) NLD_HIP(hipEventRecord(new_event(), s));
      hipLaunchKernelGGL(k_cg_update<T>, dim3(rb), dim3(kRedThreads), 0, s, (T*)P.z, (T*)P.r,
                         (const T*)P.p, (const T*)P.q, P.D, N, P.st, P.red);
      hipLaunchKernelGGL(k_cg_direction<T>, dim3(gb), dim3(256), 0, s, (T*)P.r, (T*)P.p, P.D, N,
                         P.st, 0);
      NLD_HIP(hipGetLastError());
      ++launched;
    }
  }
  hipLaunchKernelGGL(k_cg_finish<T>, dim3(gb), dim3(256), 0, s, (const T*)P.z, (const T*)f, (T*)u, N,
                     P.st);
  NLD_HIP(hipGetLastError());
  double rr_true = -1.0;
  if (o.true_residual && !(h->const_f == 0.0 && o.deflate)) {
    // true residual of the final iterate: || Pi (f_perp - A z) ||
    matvec(P, P.z, nullptr, EPI_CG_TRUE, f, s);
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
  double* d = nullptr;
  NLD_HIP(hipMallocAsync((void**)&d, sizeof(double), s));
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, P.D, (long long)P.N, d);
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
  auto alloc = [&](void** b, size_t bytes) {
    if (!*b) NLD_HIP(hipMallocAsync(b, bytes, s));
  };
  alloc(&P.yk, LN * P.elem);
  alloc(&P.yks, LN * P.elem);
  alloc(&P.grid_save, (size_t)P.grid_total * P.elem);
  alloc((void**)&P.adj_part, (size_t)257 * (4 * P.L + 3) * sizeof(double));
  if (!P.dl) {
    alloc(&P.dl, LN * P.elem);
    alloc(&P.dls, LN * P.elem);
    matvec_parts(P, P.ones, P.dl, P.dls, s);     // per-window degrees K_l 1 and K^s_l 1
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
  if (!P.have_D) {
    matvec(P, P.ones, P.D, EPI_DEGREE, nullptr, s);
    P.have_D = true;
    compute_max_eta(P, s);
  }
  if (P.prec == NLD_FP32) return run_pcg_t<float>(P, alpha, f, u, o, info, s);
  return run_pcg_t<double>(P, alpha, f, u, o, info, s);
}

}  // namespace nld
