/* nld.h — C ABI of libnld: NFFT-accelerated nonlocal image denoising on MI355X (gfx950).
 *
 * Method: arXiv 2407.06834, "Efficient nonlocal linear image denoising: bilevel
 * optimization with Nonequispaced Fast Fourier Transform and matrix-free preconditioning".
 *
 * The library solves the nonlocal system of the paper's Sec. 2.6 (discretised state
 * equation), written with alpha = mu / lambda as
 *
 *     (I + alpha L) u = f,      L = diag(D) - W,   D = W 1,
 *
 * where W = sum_l w_l K_l is the extended Gaussian ANOVA kernel of Sec. 2.5/2.6 over
 * per-pixel features split into windows of at most three dimensions,
 *     K_l(i, j) = exp(-||F_i[W_l] - F_j[W_l]||^2 / sigma_l^2),
 * each K_l v evaluated by the NFFT fast Gauss summation of Sec. 3 (spreading, FFT,
 * multiplication by the kernel's Fourier coefficients, inverse FFT, gathering), inside the
 * deflated Jacobi-preconditioned CG of Sec. 4.3 / 5.4.
 *
 * Conventions for every entry point
 *   - Vector and feature pointers are DEVICE pointers to contiguous arrays allocated and
 *     owned by the caller (e.g. torch tensors' data_ptr()).  Their element type is the
 *     plan's precision: float for NLD_FP32, double for NLD_FP64.  D is always double.
 *   - Work is enqueued on the caller's stream `s` (0 = the null stream).
 *   - Arguments are validated on the host before any launch; on NLD_E_INVAL nothing is
 *     written.  nld_last_error() returns a thread-local message for the last failure.
 *   - One plan is used from one stream at a time; plans are not thread-safe.
 *   - Results are deterministic: the same inputs give bitwise-identical outputs.
 */
#ifndef NLD_H
#define NLD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nld_plan_s* nfft_plan_t;

typedef enum {
  NLD_OK = 0,
  NLD_E_INVAL = 1,     /* invalid argument; nothing launched, outputs untouched        */
  NLD_E_NOMEM = 2,     /* device allocation failed                                      */
  NLD_E_HIP = 3,       /* a HIP runtime call failed (message names it)                  */
  NLD_E_NOCONV = 4,    /* CG hit maxit; u holds the last iterate, info is filled        */
  NLD_E_BREAKDOWN = 5, /* non-finite or non-positive CG scalar; u holds the last iterate */
  NLD_E_STATE = 6      /* request incompatible with the plan's state                    */
} nld_status;

typedef enum { NLD_FP32 = 0, NLD_FP64 = 1 } nld_prec;

/* Kernel descriptor (host memory, copied at plan time).
 *   n_windows   L >= 1 windows; win_dim[l] in {1,2,3}; win_feat lists the feature rows of
 *               each window back to back (sum of win_dim entries, each in [0, d)).
 *   sigma       [L], > 0: Gaussian width of window l (kernel exp(-r^2 / sigma^2), Sec. 2.6).
 *   weight      [L], >= 0: window weight w_l (the paper uses 1/L).
 *   bandwidth   M, the number of Fourier coefficients per dimension (even, 8..256), used for
 *               every window; 0 selects M per window from sigma_l, the data range and
 *               matvec_tol.  win_bandwidth (optional, may be NULL) overrides per window.
 *   cutoff      m, window half-width in grid cells (1..8); 0 selects it from matvec_tol.
 *   oversampling  sigma_os >= 1.25; the grid has n = next power of two >= sigma_os * M
 *               points per dimension (n <= 256).
 *   matvec_tol  target relative error of K_l v when M or m are selected automatically.
 *   prec        arithmetic of features, grids and vectors.  CG inner products, the
 *               deflation means, D and the Laplacian epilogue are FP64 in both modes.
 *   tile        grid tile extent of 3-dimensional windows for the spreading and gathering
 *               schedules: 8 or 16 (0 selects 8).  Results do not depend on it beyond
 *               rounding; it trades halo work against workgroup count.
 *   max_grid    largest grid side n (0 for no limit, else 32, 64, 128 or 256): a window whose
 *               oversampled grid would exceed it uses n = max_grid instead, provided that still
 *               oversamples its band by at least 1.25 (n >= 1.25 M); the window function's
 *               shape follows the ratio n / M, so the same cutoff stays accurate (about 1e-6
 *               relative at m = 4 for n / M = 4/3, against 1e-7 at n / M = 2).
 */
typedef struct {
  int32_t n_windows;
  const int32_t* win_dim;
  const int32_t* win_feat;
  const double* sigma;
  const double* weight;
  int32_t bandwidth;
  const int32_t* win_bandwidth;
  int32_t cutoff;
  double oversampling;
  double matvec_tol;
  nld_prec prec;
  int32_t tile;
  int32_t max_grid;
} nld_kernel_desc;

/* Per-window parameters chosen by the plan (for reports and tests). */
typedef struct {
  int32_t dims_kept;       /* window dimensions with a nonzero data range               */
  int32_t bandwidth;       /* M                                                          */
  int32_t grid;            /* n                                                          */
  int32_t cutoff;          /* m                                                          */
  double compression[3];   /* torus compression a per kept dimension                    */
  double lo[3], hi[3];     /* data range per kept dimension                             */
} nld_window_info;

/* Build a plan over N nodes with d features stored SoA ([d][N], element type of prec):
 * per-window torus scaling (data range reduction), Fourier multipliers, tile keys and the
 * stable counting sort of the nodes by grid tile.  Blocks until the plan is ready.
 * Paper Sec. 3 (fast Gauss summation) and Sec. 5 (windows of at most three features). */
nld_status nfft_plan(nfft_plan_t* out, const void* features, int64_t N, int32_t d,
                     const nld_kernel_desc* desc, hipStream_t s);

/* New kernel widths sigma[L] (> 0) and weights weight[L] (>= 0), host arrays, for an existing
 * plan: the Fourier multipliers of Sec. 3 (periodic Gaussian coefficients of every window)
 * and of the width derivative are rewritten, the degree vector is recomputed on next use;
 * node coordinates, the sort and all schedules are kept, so this costs a few table uploads.
 * The node compression a and bandwidth M of every window stay as built: if the per-entry
 * error estimate at the new width, max(exp(-(pi st M / 2)^2), exp(-((1 - 2a) / st)^2)) with
 * st the width on the torus, exceeds both 1e-2 * matvec_tol and ten times the larger of its
 * value at the old width and the estimate a new plan with the same M would reach (optimal a),
 * the call returns NLD_E_STATE and leaves the plan unchanged (build a new plan instead); so
 * does a window whose bandwidth was autotuned (0 in the descriptor) when the autotuner would
 * pick another M for the new width.
 * Blocks until the tables are on the device.  The bilevel learning of Sec. 5.5 changes
 * (sigma_l, w_l) once per outer step. */
nld_status nfft_plan_update_kernel(nfft_plan_t plan, const double* sigma, const double* weight,
                                   hipStream_t s);

/* Release the plan.  Waits for the plan's last stream, then hands the plan's device buffers to
 * the library's per-device cache, from which later plans take theirs (at most 8 GiB cached per
 * device; beyond that buffers are freed).  No work using the plan may still be in flight on
 * another stream. */
nld_status nfft_plan_destroy(nfft_plan_t plan);

/* Copy the chosen parameters of window l into *info (host). */
nld_status nfft_plan_window_info(nfft_plan_t plan, int32_t l, nld_window_info* info);

/* Number of nodes N and windows L of the plan. */
nld_status nfft_plan_size(nfft_plan_t plan, int64_t* N, int32_t* L, nld_prec* prec);

/* D = W~ 1 (FP64, device [N]): the degree vector of the approximated kernel, self term
 * included (Sec. 2.6: eta = D - sum_l w_l is the zero-diagonal degree). */
nld_status degree_vector(nfft_plan_t plan, double* D, hipStream_t s);

/* y = W~ v = sum_l w_l K~_l v (self term included).  Asynchronous.  Sec. 3. */
nld_status anova_matvec(nfft_plan_t plan, const void* v, void* y, hipStream_t s);

/* y = L~ v = D o v - W~ v with the plan's own D, evaluated in FP64 before the final
 * rounding to the plan's precision (L~ 1 = 0 exactly).  Asynchronous.  Sec. 2.6. */
nld_status laplacian_matvec(nfft_plan_t plan, const void* v, void* y, hipStream_t s);

typedef struct {
  double tol;        /* stop when ||r_k||_2 <= tol * ||f - mean(f)||_2 (recursive residual) */
  int32_t maxit;     /* maximum number of iterations (operator applications)              */
  int32_t use_u0;    /* 0: start from f (Sec. 5.3).  1: u holds an initial guess u0 on     */
                     /* entry; a u0 whose initial residual is not finite is replaced by f.  */
                     /* 2: as 1, and u0 is also replaced by f when its initial residual     */
                     /* ||Pi (f - A u0)|| exceeds that of u0 = f (costs one more operator   */
                     /* application).  3: as 1, and CG starts from b Pi u0 with          */
                     /* b = <Pi u0, f_perp> / <Pi u0, A Pi u0>, the multiple of the guess    */
                     /* nearest to the solution in the energy norm (never farther than the   */
                     /* start u = mean(f) 1; no extra operator application).  Plain PCG from */
                     /* f is the fallback of a warm start.                                   */
  int32_t precond;   /* 0: none; 1: Jacobi P_a = I + alpha diag(eta); 2: the l2 diagonal   */
                     /* P_b' = (alpha^2 sum_l w_l^2 diag(Gamma_l o Gamma_l 1) + P_a^2)^(1/2) */
                     /* of Sec. 4.3.1 (squared kernels = Gaussians of width sigma_l / sqrt 2, */
                     /* summed once per plan on the plan's grids; Gamma_l: K_l, zero diagonal) */
  int32_t deflate;   /* 1: change of basis removing the eigenvector 1 (Sec. 4.2, 5.4)      */
  int32_t true_residual; /* 1: also compute the true residual at exit (one more matvec)     */
  int32_t timing;    /* 1: time every operator application with HIP events on the stream s   */
} nld_pcg_opts;

typedef struct {
  int32_t iters;        /* CG iterations (operator applications after the initial residual) */
  double relres_rec;    /* recursive residual / ||f_perp||                                   */
  double relres_true;   /* true residual / ||f_perp|| (if requested, else -1)                */
  double kappa_est;     /* 2 alpha max(eta) + 1 (paper Sec. 5.3 condition estimate)          */
  double ms_solve;      /* wall time of the solve, ms                                        */
  double ms_matvec;     /* mean duration of one operator application (if timing), ms         */
  int32_t matvecs_timed;/* operator applications that entered the mean                       */
  nld_status status;
  int32_t u0_rejected;  /* 1 if the initial guess was replaced by f (use_u0 = 1 or 2)        */
} nld_pcg_info;

/* Solve (I + alpha L~) u = f with deflated Jacobi PCG (Sec. 4.3.2, 5.4), projector form:
 * mean(f) is kept exactly and CG runs on the complement of the constant vector with the
 * preconditioner s = Pi (r / P), P = 1 + alpha eta, Pi = I - 1 1^T / N.  A constant f is
 * returned unchanged with 0 iterations.  Blocks until done; fills *info (host). */
nld_status pcg_solve(nfft_plan_t plan, double alpha, const void* f, void* u,
                     const nld_pcg_opts* opts, nld_pcg_info* info, hipStream_t s);

/* Independent solves of `count` plans (distinct handles, equal precision and cutoff), each
 * (I + alpha[b] L~_b) u_b = f_b with the deflated Jacobi PCG of pcg_solve and the same opts;
 * f[b] and u[b] are device vectors of plan b's N and precision (u[b] holds u0 if use_u0, which
 * must be 0 or 1 here; a non-finite u0 ends that solve with NLD_E_BREAKDOWN instead of the
 * fallback of pcg_solve).
 * All solves advance together: every stage of an iteration is one launch over all plans, a
 * chunk of iterations is captured once as a HIP graph and replayed until every solve has
 * finished, and solves that finish early stop costing work.  Each solve's iterates are
 * bit-identical to pcg_solve on its plan.  infos[b] (host, count entries) gets each solve's
 * report; ms_solve is the time from the call until that solve was seen finished.  Computes
 * the degree vectors of plans that lack them.  Uses each plan's CG work vectors, so a plan
 * must not be solved elsewhere concurrently.  Blocks until all solves are done; the work runs
 * on an internal stream ordered after s, and s is ordered after it on return.  Returns
 * NLD_OK if every solve converged, else the first failing status (infos tell which).
 * Paper Sec. 4.2-4.3 and 5.3-5.4 (the solver), applied to a batch of images. */
nld_status pcg_solve_batched(const nfft_plan_t* plans, const double* alpha, const void* const* f,
                             void* const* u, int32_t count, const nld_pcg_opts* opts,
                             nld_pcg_info* infos, hipStream_t s);

/* Bilevel gradient by the adjoint method (paper Sec. 2.4 optimality system, Sec. 5.5):
 * given the state u of (I + alpha L~) u = f and g = dJ/du (device, precision of the plan),
 * solves A p = g with the same operator and options as pcg_solve (p: device, out; if
 * opts->use_u0, p holds the initial guess on entry), then writes to grad (host, 1 + 2L doubles)
 *   grad[0]         = dJ/dlog(alpha)   = sum_l w_l dJ/dw_l
 *   grad[1 + l]     = dJ/dlog(sigma_l) = -alpha w_l p^T L^s_l u
 *   grad[1 + L + l] = dJ/dw_l          = -alpha p^T L_l u
 * where L_l is the Laplacian of window l's kernel and L^s_l that of sigma_l dK_l/dsigma_l =
 * (2 r^2 / sigma_l^2) exp(-r^2 / sigma_l^2), both evaluated by NFFT fast summation (the
 * derivative kernel's Fourier coefficients are the Gaussian's times t - 2 pi^2 sum_d
 * st_d^2 k_d^2).  Features are treated as data; dJ/df is p.  f is accepted for the interface
 * and validated but not read (the state enters through u).  Blocks; fills *info for the adjoint
 * solve.  */
nld_status adjoint_solve(nfft_plan_t plan, double alpha, const void* f, const void* u, const void* g,
                         void* p, double* grad, const nld_pcg_opts* opts, nld_pcg_info* info,
                         hipStream_t s);

/* Features of an n1 x n2 image (device, row-major, element type of prec) into the SoA
 * matrix features [d][N] (device), d = 2*with_pos + (2 rho + 1)^2, N = n1 n2: position
 * (col/n2, row/n1) then the patch intensities of radius rho in raster order of the offsets,
 * zero outside the image (paper Sec. 5, patches).  Asynchronous. */
nld_status features_from_image(const void* img, int32_t n1, int32_t n2, int32_t rho,
                               int32_t with_pos, nld_prec prec, void* features, hipStream_t s);

/* Mutual information score of every feature row against a target (paper Sec. 5: the features
 * are ranked by this score against the noisy pixel values and the ranking is cut into windows
 * of at most three).  The paper does not name its estimator; this is the plug-in estimate of a
 * joint histogram.  A row x with minimum lo and maximum hi puts value v into bin
 * min(bins - 1, floor((v - lo) * s)), s = bins / (hi - lo) (s = 0 when hi = lo), all in IEEE
 * double; with counts n_ab of the N pairs (bin of the feature, bin of the target) and their
 * marginals n_a, n_b,
 *     scores[j] = sum over n_ab > 0 of (n_ab / N) log(N n_ab / (n_a n_b))   (natural log).
 * features [d][N] and target [N]: device, element type of prec, finite values; scores [d]:
 * device doubles written by the call.  bins: 2..64, or 0 for the largest B with
 * B^3 <= N / 4 clamped to [4, 64].  N in [1, 2^31 - 1], d in [1, 4096].  Allocates and frees
 * its counters stream-ordered on s; asynchronous. */
nld_status mis_scores(const void* features, int64_t N, int32_t d, const void* target,
                      nld_prec prec, int32_t bins, double* scores, hipStream_t s);

/* mis_scores without any device allocation, for callers that cannot allocate: code under HIP
 * graph capture, allocation-free serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, validation and results (bit for bit) as mis_scores.  Its range table and joint
 * histograms live in a static device array of 1048576 32-bit words (4 MiB) that each device the
 * library runs on holds until the process ends; a call with 4 (d + 1) + d * B^2 > 1048576
 * (B = bins, or the default bin count for bins = 0) returns NLD_E_INVAL with nothing launched.
 * Every call on one device shares that array and leaves its last contents there (the
 * histograms are cleared by a fill kernel at the start of each call): calls that overlap on one
 * device (different streams or threads without ordering) race; calls on one stream are
 * ordered.  Asynchronous. */
nld_status mis_scores_noalloc(const void* features, int64_t N, int32_t d, const void* target,
                              nld_prec prec, int32_t bins, double* scores, hipStream_t s);

/* Message describing the last non-OK status returned on this thread. */
const char* nld_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NLD_H */
