// Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: every
// call below fails argument validation on the host, before any HIP call, so the driver runs
// without a GPU.  Exit status 0 when each call returns the expected status and a message.
#include <cstdio>
#include <cstring>

#include "../../include/nld.h"
#include "../../include/nld_cnn.h"

static int failures = 0;

static void expect(const char* what, nld_status got, nld_status want) {
  const char* msg = nld_last_error();
  if (got != want || msg == nullptr || (want != NLD_OK && std::strlen(msg) == 0)) {
    std::fprintf(stderr, "%s: status %d (want %d), message '%s'\n", what, (int)got, (int)want,
                 msg ? msg : "(null)");
    ++failures;
  }
}

int main() {
  void* fake = reinterpret_cast<void*>(0x1000);   // never dereferenced: validation fails first
  double* dfake = static_cast<double*>(fake);
  int32_t wd[2] = {3, 2}, wf[5] = {0, 1, 2, 0, 1};
  double sg[2] = {0.1, 0.2}, wt[2] = {1.0, 1.0};
  nld_kernel_desc d{};
  d.n_windows = 2; d.win_dim = wd; d.win_feat = wf; d.sigma = sg; d.weight = wt;
  d.bandwidth = 64; d.cutoff = 4; d.oversampling = 2.0; d.matvec_tol = 1e-6; d.prec = NLD_FP32;
  nfft_plan_t plan = nullptr;
  expect("plan null out", nfft_plan(nullptr, fake, 100, 3, &d, nullptr), NLD_E_INVAL);
  expect("plan N=0", nfft_plan(&plan, fake, 0, 3, &d, nullptr), NLD_E_INVAL);
  expect("plan feature index", nfft_plan(&plan, fake, 100, 2, &d, nullptr), NLD_E_INVAL);
  nld_kernel_desc bad = d;
  bad.bandwidth = 63;
  expect("plan odd bandwidth", nfft_plan(&plan, fake, 100, 3, &bad, nullptr), NLD_E_INVAL);
  bad = d; bad.cutoff = 9;
  expect("plan cutoff", nfft_plan(&plan, fake, 100, 3, &bad, nullptr), NLD_E_INVAL);
  bad = d; bad.max_grid = 100;
  expect("plan max_grid", nfft_plan(&plan, fake, 100, 3, &bad, nullptr), NLD_E_INVAL);
  bad = d; bad.n_windows = 0;
  expect("plan no windows", nfft_plan(&plan, fake, 100, 3, &bad, nullptr), NLD_E_INVAL);
  double sneg[2] = {-1.0, 0.1};
  bad = d; bad.sigma = sneg;
  expect("plan sigma", nfft_plan(&plan, fake, 100, 3, &bad, nullptr), NLD_E_INVAL);
  if (plan != nullptr) { std::fprintf(stderr, "plan written on failure\n"); ++failures; }
  nld_pcg_opts o{};
  o.tol = 1e-6; o.maxit = 10; o.precond = 1; o.deflate = 1;
  nld_pcg_info info{};
  expect("pcg null plan", pcg_solve(nullptr, 1.0, fake, fake, &o, &info, nullptr), NLD_E_INVAL);
  expect("adjoint null plan",
         adjoint_solve(nullptr, 1.0, fake, fake, fake, fake, nullptr, &o, &info, nullptr),
         NLD_E_INVAL);
  expect("batched null", pcg_solve_batched(nullptr, nullptr, nullptr, nullptr, 1, &o, &info, nullptr),
         NLD_E_INVAL);
  expect("features rho", features_from_image(fake, 8, 8, 16, 1, NLD_FP32, fake, nullptr), NLD_E_INVAL);
  expect("features sides", features_from_image(fake, 0, 8, 1, 1, NLD_FP32, fake, nullptr), NLD_E_INVAL);
  expect("mis bins", mis_scores(fake, 100, 3, fake, NLD_FP32, 65, dfake, nullptr), NLD_E_INVAL);
  expect("mis d", mis_scores(fake, 100, 0, fake, NLD_FP32, 8, dfake, nullptr), NLD_E_INVAL);
  expect("mis noalloc size",
         mis_scores_noalloc(fake, 100, 300, fake, NLD_FP32, 64, dfake, nullptr), NLD_E_INVAL);
  expect("degree null", degree_vector(nullptr, nullptr, nullptr), NLD_E_INVAL);
  expect("anova null", anova_matvec(nullptr, fake, fake, nullptr), NLD_E_INVAL);
  expect("laplacian null", laplacian_matvec(nullptr, fake, fake, nullptr), NLD_E_INVAL);
  expect("destroy null", nfft_plan_destroy(nullptr), NLD_E_INVAL);
  expect("cnn destroy null", cnn_destroy(nullptr), NLD_E_INVAL);
  std::printf("%d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
