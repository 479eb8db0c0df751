// extern "C" entry points of libnld: argument validation, error reporting, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>
#include <algorithm>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>

#include "nld_internal.h"

struct nld_plan_s {
  nld::Plan P;
};

namespace nld {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace nld

namespace {

nld_status fail(nld_status st, const std::string& msg) {
  nld::set_error(msg);
  return st;
}

template <typename F>
nld_status guarded(const char* name, F&& body) {
  try {
    return body();
  } catch (const nld::HipError& e) {
    return fail(NLD_E_HIP, std::string(name) + ": " + e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    return fail(NLD_E_NOMEM, std::string(name) + ": host allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(NLD_E_INVAL, std::string(name) + ": " + e.what());
  } catch (const std::exception& e) {
    return fail(NLD_E_STATE, std::string(name) + ": " + e.what());
  }
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

const char* nld_last_error(void) { return nld::g_last_error.c_str(); }

nld_status features_from_image(const void* img, int32_t n1, int32_t n2, int32_t rho,
                               int32_t with_pos, nld_prec prec, void* features, hipStream_t s) {
  if (!img || !features) return fail(NLD_E_INVAL, "features_from_image: null pointer");
  if (n1 < 1 || n2 < 1) return fail(NLD_E_INVAL, "features_from_image: image sides must be >= 1");
  if (rho < 0 || rho > 15) return fail(NLD_E_INVAL, "features_from_image: rho must be in [0, 15]");
  if (with_pos != 0 && with_pos != 1) return fail(NLD_E_INVAL, "features_from_image: with_pos must be 0 or 1");
  if (prec != NLD_FP32 && prec != NLD_FP64) return fail(NLD_E_INVAL, "features_from_image: bad precision");
  if ((long long)n1 * n2 > (1LL << 31) - 1) return fail(NLD_E_INVAL, "features_from_image: image too large");
  return guarded("features_from_image", [&] {
    nld::launch_features(img, n1, n2, rho, with_pos, prec, features, s);
    return NLD_OK;
  });
}

nld_status mis_scores(const void* features, int64_t N, int32_t d, const void* target,
                      nld_prec prec, int32_t bins, double* scores, hipStream_t s) {
  if (!features || !target || !scores) return fail(NLD_E_INVAL, "mis_scores: null pointer");
  if (N < 1 || N > 0x7fffffffLL) return fail(NLD_E_INVAL, "mis_scores: N must be in [1, 2^31 - 1]");
  if (d < 1 || d > 4096) return fail(NLD_E_INVAL, "mis_scores: d must be in [1, 4096]");
  if (prec != NLD_FP32 && prec != NLD_FP64) return fail(NLD_E_INVAL, "mis_scores: bad precision");
  if (bins != 0 && (bins < 2 || bins > 64)) return fail(NLD_E_INVAL, "mis_scores: bins must be 0 or in [2, 64]");
  return guarded("mis_scores", [&] {
    nld::launch_mis(features, N, d, target, prec, bins ? bins : nld::mis_default_bins(N), scores, s);
    return NLD_OK;
  });
}

nld_status mis_scores_noalloc(const void* features, int64_t N, int32_t d, const void* target,
                              nld_prec prec, int32_t bins, double* scores, hipStream_t s) {
  if (!features || !target || !scores) return fail(NLD_E_INVAL, "mis_scores_noalloc: null pointer");
  if (N < 1 || N > 0x7fffffffLL) return fail(NLD_E_INVAL, "mis_scores_noalloc: N must be in [1, 2^31 - 1]");
  if (d < 1 || d > 4096) return fail(NLD_E_INVAL, "mis_scores_noalloc: d must be in [1, 4096]");
  if (prec != NLD_FP32 && prec != NLD_FP64) return fail(NLD_E_INVAL, "mis_scores_noalloc: bad precision");
  if (bins != 0 && (bins < 2 || bins > 64))
    return fail(NLD_E_INVAL, "mis_scores_noalloc: bins must be 0 or in [2, 64]");
  const int B = bins ? bins : nld::mis_default_bins(N);
  if (nld::mis_noalloc_words(d, B) > nld::mis_noalloc_capacity())
    return fail(NLD_E_INVAL, "mis_scores_noalloc: 4 (d + 1) + d bins^2 exceeds the static scratch "
                             "of 1048576 words");
  return guarded("mis_scores_noalloc", [&] {
    nld::launch_mis_noalloc(features, N, d, target, prec, B, scores, s);
    return NLD_OK;
  });
}

nld_status nfft_plan(nfft_plan_t* out, const void* features, int64_t N, int32_t d,
                     const nld_kernel_desc* desc, hipStream_t s) {
  if (!out || !features || !desc) return fail(NLD_E_INVAL, "nfft_plan: null pointer");
  *out = nullptr;
  if (N < 1) return fail(NLD_E_INVAL, "nfft_plan: N must be >= 1");
  if (d < 1) return fail(NLD_E_INVAL, "nfft_plan: d must be >= 1");
  const int L = desc->n_windows;
  if (L < 1 || L > 1024) return fail(NLD_E_INVAL, "nfft_plan: n_windows must be in [1, 1024]");
  if (!desc->win_dim || !desc->win_feat || !desc->sigma || !desc->weight)
    return fail(NLD_E_INVAL, "nfft_plan: null window table");
  if ((long long)N * L > 0x7fffffffLL) return fail(NLD_E_INVAL, "nfft_plan: N * n_windows too large");
  if (desc->prec != NLD_FP32 && desc->prec != NLD_FP64) return fail(NLD_E_INVAL, "nfft_plan: bad precision");
  int nf = 0;
  for (int l = 0; l < L; ++l) {
    if (desc->win_dim[l] < 1 || desc->win_dim[l] > 3)
      return fail(NLD_E_INVAL, "nfft_plan: window dimension must be 1, 2 or 3");
    nf += desc->win_dim[l];
    if (!finite_pos(desc->sigma[l])) return fail(NLD_E_INVAL, "nfft_plan: sigma must be finite and > 0");
    if (!std::isfinite(desc->weight[l]) || desc->weight[l] < 0.0)
      return fail(NLD_E_INVAL, "nfft_plan: weights must be finite and >= 0");
  }
  for (int k = 0; k < nf; ++k)
    if (desc->win_feat[k] < 0 || desc->win_feat[k] >= d)
      return fail(NLD_E_INVAL, "nfft_plan: window feature index out of range");
  auto bw_ok = [](int M) { return M == 0 || (M >= 8 && M <= 256 && M % 2 == 0); };
  if (!bw_ok(desc->bandwidth)) return fail(NLD_E_INVAL, "nfft_plan: bandwidth must be 0 or even in [8, 256]");
  if (desc->win_bandwidth)
    for (int l = 0; l < L; ++l)
      if (!bw_ok(desc->win_bandwidth[l]))
        return fail(NLD_E_INVAL, "nfft_plan: window bandwidth must be 0 or even in [8, 256]");
  if (desc->cutoff < 0 || desc->cutoff > 8) return fail(NLD_E_INVAL, "nfft_plan: cutoff must be in [0, 8]");
  if (desc->max_grid != 0 && desc->max_grid != 32 && desc->max_grid != 64 &&
      desc->max_grid != 128 && desc->max_grid != 256)
    return fail(NLD_E_INVAL, "nfft_plan: max_grid must be 0, 32, 64, 128 or 256");
  const double os = desc->oversampling == 0.0 ? 2.0 : desc->oversampling;
  if (!std::isfinite(os) || os < 1.25 || os > 8.0)
    return fail(NLD_E_INVAL, "nfft_plan: oversampling must be in [1.25, 8]");
  const double tol = desc->matvec_tol == 0.0 ? 1e-6 : desc->matvec_tol;
  if (!finite_pos(tol) || tol >= 1.0) return fail(NLD_E_INVAL, "nfft_plan: matvec_tol must be in (0, 1)");
  if (desc->tile != 0 && desc->tile != 8 && desc->tile != 16)
    return fail(NLD_E_INVAL, "nfft_plan: tile must be 0, 8 or 16");
  nld_plan_s* h = nullptr;
  nld_status st = guarded("nfft_plan", [&] {
    h = new nld_plan_s();
    nld::Plan& P = h->P;
    P.prec = desc->prec;
    P.N = N;
    P.d = d;
    P.L = L;
    P.elem = desc->prec == NLD_FP32 ? 4 : 8;
    P.win_dim.assign(desc->win_dim, desc->win_dim + L);
    P.win_feat.assign(desc->win_feat, desc->win_feat + nf);
    P.sigma.assign(desc->sigma, desc->sigma + L);
    P.weight.assign(desc->weight, desc->weight + L);
    P.bw.assign(L, desc->bandwidth);
    if (desc->win_bandwidth)
      for (int l = 0; l < L; ++l)
        if (desc->win_bandwidth[l]) P.bw[l] = desc->win_bandwidth[l];
    P.cutoff = desc->cutoff;
    P.oversampling = os;
    P.tol = tol;
    P.tile3 = desc->tile;
    P.max_grid = desc->max_grid;
    P.st_host = (nld::CgState*)nld::pinned_get(sizeof(nld::CgState));
    int dev = 0, lds = 65536;
    NLD_HIP(hipGetDevice(&dev));
    NLD_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    P.lds_limit = std::min<long long>(lds, 160 * 1024);
    nld::build_plan(P, features, s);
    return NLD_OK;
  });
  if (st != NLD_OK) {
    if (h) {
      nld::release_plan(h->P);
      nld::pinned_put(h->P.st_host);
      delete h;
    }
    return st;
  }
  *out = h;
  return NLD_OK;
}

nld_status nfft_plan_update_kernel(nfft_plan_t plan, const double* sigma, const double* weight,
                                   hipStream_t s) {
  if (!plan || !sigma || !weight) return fail(NLD_E_INVAL, "nfft_plan_update_kernel: null pointer");
  nld::Plan& P = plan->P;
  for (int l = 0; l < P.L; ++l) {
    if (!finite_pos(sigma[l])) return fail(NLD_E_INVAL, "nfft_plan_update_kernel: sigma must be finite and > 0");
    if (!std::isfinite(weight[l]) || weight[l] < 0.0)
      return fail(NLD_E_INVAL, "nfft_plan_update_kernel: weights must be finite and >= 0");
  }
  return guarded("nfft_plan_update_kernel", [&] {
    nld::update_kernel(P, sigma, weight, s);
    return NLD_OK;
  });
}

nld_status nfft_plan_destroy(nfft_plan_t plan) {
  if (!plan) return fail(NLD_E_INVAL, "nfft_plan_destroy: null plan");
  nld::release_plan(plan->P);
  nld::pinned_put(plan->P.st_host);
  delete plan;
  return NLD_OK;
}

nld_status nfft_plan_window_info(nfft_plan_t plan, int32_t l, nld_window_info* info) {
  if (!plan || !info) return fail(NLD_E_INVAL, "nfft_plan_window_info: null pointer");
  if (l < 0 || l >= plan->P.L) return fail(NLD_E_INVAL, "nfft_plan_window_info: window out of range");
  *info = plan->P.info[l];
  return NLD_OK;
}

nld_status nfft_plan_size(nfft_plan_t plan, int64_t* N, int32_t* L, nld_prec* prec) {
  if (!plan) return fail(NLD_E_INVAL, "nfft_plan_size: null plan");
  if (N) *N = plan->P.N;
  if (L) *L = plan->P.L;
  if (prec) *prec = plan->P.prec;
  return NLD_OK;
}

nld_status degree_vector(nfft_plan_t plan, double* D, hipStream_t s) {
  if (!plan || !D) return fail(NLD_E_INVAL, "degree_vector: null pointer");
  return guarded("degree_vector", [&] {
    nld::Plan& P = plan->P;
    P.stream = s;
    if (!P.have_D) {
      nld::matvec(P, P.ones, P.D, nld::EPI_DEGREE, s);
      P.have_D = true;
      nld::compute_max_eta(P, s);
    }
    NLD_HIP(hipMemcpyAsync(D, P.D, P.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    return NLD_OK;
  });
}

nld_status anova_matvec(nfft_plan_t plan, const void* v, void* y, hipStream_t s) {
  if (!plan || !v || !y) return fail(NLD_E_INVAL, "anova_matvec: null pointer");
  return guarded("anova_matvec", [&] {
    plan->P.stream = s;
    nld::matvec(plan->P, v, y, nld::EPI_ANOVA, s);
    return NLD_OK;
  });
}

nld_status laplacian_matvec(nfft_plan_t plan, const void* v, void* y, hipStream_t s) {
  if (!plan || !v || !y) return fail(NLD_E_INVAL, "laplacian_matvec: null pointer");
  return guarded("laplacian_matvec", [&] {
    nld::Plan& P = plan->P;
    P.stream = s;
    if (!P.have_D) {
      nld::matvec(P, P.ones, P.D, nld::EPI_DEGREE, s);
      P.have_D = true;
      nld::compute_max_eta(P, s);
    }
    nld::matvec(P, v, y, nld::EPI_LAPLACIAN, s);
    return NLD_OK;
  });
}

nld_status pcg_solve(nfft_plan_t plan, double alpha, const void* f, void* u,
                     const nld_pcg_opts* opts, nld_pcg_info* info, hipStream_t s) {
  if (!plan || !f || !u || !opts || !info) return fail(NLD_E_INVAL, "pcg_solve: null pointer");
  if (!finite_pos(alpha)) return fail(NLD_E_INVAL, "pcg_solve: alpha must be finite and > 0");
  if (!finite_pos(opts->tol) || opts->tol >= 1.0) return fail(NLD_E_INVAL, "pcg_solve: tol must be in (0, 1)");
  if (opts->maxit < 0) return fail(NLD_E_INVAL, "pcg_solve: maxit must be >= 0");
  if (opts->precond < 0 || opts->precond > 2)
    return fail(NLD_E_INVAL, "pcg_solve: precond must be 0, 1 or 2");
  if (opts->deflate != 0 && opts->deflate != 1) return fail(NLD_E_INVAL, "pcg_solve: deflate must be 0 or 1");
  if (opts->use_u0 < 0 || opts->use_u0 > 3) return fail(NLD_E_INVAL, "pcg_solve: use_u0 must be 0, 1, 2 or 3");
  std::memset(info, 0, sizeof(*info));
  info->relres_true = -1.0;
  nld_status result = NLD_OK;
  nld_status st = guarded("pcg_solve", [&] {
    plan->P.stream = s;
    result = nld::run_pcg(plan->P, alpha, f, u, *opts, *info, s);
    return NLD_OK;
  });
  if (st != NLD_OK) {
    info->status = st;
    return st;
  }
  if (result == NLD_E_NOCONV) nld::set_error("pcg_solve: maximum number of iterations reached");
  if (result == NLD_E_BREAKDOWN) nld::set_error("pcg_solve: CG breakdown (non-finite or non-positive scalar)");
  return result;
}

nld_status pcg_solve_batched(const nfft_plan_t* plans, const double* alpha, const void* const* f,
                             void* const* u, int32_t count, const nld_pcg_opts* opts,
                             nld_pcg_info* infos, hipStream_t s) {
  if (!plans || !alpha || !f || !u || !opts || !infos)
    return fail(NLD_E_INVAL, "pcg_solve_batched: null pointer");
  if (count < 1 || count > 65536) return fail(NLD_E_INVAL, "pcg_solve_batched: count must be in [1, 65536]");
  if (!finite_pos(opts->tol) || opts->tol >= 1.0) return fail(NLD_E_INVAL, "pcg_solve_batched: tol must be in (0, 1)");
  if (opts->maxit < 0) return fail(NLD_E_INVAL, "pcg_solve_batched: maxit must be >= 0");
  if (opts->precond < 0 || opts->precond > 2)
    return fail(NLD_E_INVAL, "pcg_solve_batched: precond must be 0, 1 or 2");
  if ((opts->deflate != 0 && opts->deflate != 1) || (opts->use_u0 != 0 && opts->use_u0 != 1))
    return fail(NLD_E_INVAL, "pcg_solve_batched: deflate and use_u0 must be 0 or 1");
  std::vector<nld::Plan*> P(count);
  for (int b = 0; b < count; ++b) {
    if (!plans[b] || !f[b] || !u[b]) return fail(NLD_E_INVAL, "pcg_solve_batched: null plan or vector");
    if (!finite_pos(alpha[b])) return fail(NLD_E_INVAL, "pcg_solve_batched: alpha must be finite and > 0");
    P[b] = &plans[b]->P;
    if (P[b]->prec != P[0]->prec) return fail(NLD_E_INVAL, "pcg_solve_batched: plans of different precision");
    if (P[b]->wins[0].m != P[0]->wins[0].m) return fail(NLD_E_INVAL, "pcg_solve_batched: plans of different cutoff");
  }
  {
    std::vector<nld::Plan*> sorted(P);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(NLD_E_INVAL, "pcg_solve_batched: a plan appears twice");
  }
  for (int b = 0; b < count; ++b) {
    std::memset(&infos[b], 0, sizeof(nld_pcg_info));
    infos[b].relres_true = -1.0;
  }
  nld_status result = NLD_OK;
  nld_status st = guarded("pcg_solve_batched", [&] {
    result = nld::run_pcg_batched(P.data(), alpha, f, u, count, *opts, infos, s);
    return NLD_OK;
  });
  if (st != NLD_OK) {
    for (int b = 0; b < count; ++b) infos[b].status = st;
    return st;
  }
  if (result == NLD_E_NOCONV) nld::set_error("pcg_solve_batched: some solve reached the maximum number of iterations");
  if (result == NLD_E_BREAKDOWN) nld::set_error("pcg_solve_batched: CG breakdown in some solve");
  return result;
}

nld_status adjoint_solve(nfft_plan_t plan, double alpha, const void* f, const void* u,
                         const void* g, void* p, double* grad, const nld_pcg_opts* opts,
                         nld_pcg_info* info, hipStream_t s) {
  if (!plan || !f || !u || !g || !p || !grad || !opts || !info)
    return fail(NLD_E_INVAL, "adjoint_solve: null pointer");
  if (!finite_pos(alpha)) return fail(NLD_E_INVAL, "adjoint_solve: alpha must be finite and > 0");
  if (!finite_pos(opts->tol) || opts->tol >= 1.0) return fail(NLD_E_INVAL, "adjoint_solve: tol must be in (0, 1)");
  if (opts->maxit < 0) return fail(NLD_E_INVAL, "adjoint_solve: maxit must be >= 0");
  if (opts->precond < 0 || opts->precond > 2)
    return fail(NLD_E_INVAL, "adjoint_solve: precond must be 0, 1 or 2");
  if (opts->deflate != 0 && opts->deflate != 1) return fail(NLD_E_INVAL, "adjoint_solve: deflate must be 0 or 1");
  if (opts->use_u0 < 0 || opts->use_u0 > 3) return fail(NLD_E_INVAL, "adjoint_solve: use_u0 must be 0, 1, 2 or 3");
  std::memset(info, 0, sizeof(*info));
  info->relres_true = -1.0;
  nld_status result = NLD_OK;
  nld_status st = guarded("adjoint_solve", [&] {
    plan->P.stream = s;
    result = nld::run_adjoint(plan->P, alpha, u, g, p, grad, *opts, *info, s);
    return NLD_OK;
  });
  if (st != NLD_OK) {
    info->status = st;
    return st;
  }
  if (result == NLD_E_NOCONV) nld::set_error("adjoint_solve: maximum number of iterations reached");
  if (result == NLD_E_BREAKDOWN) nld::set_error("adjoint_solve: CG breakdown");
  return result;
}

}  // extern "C"
