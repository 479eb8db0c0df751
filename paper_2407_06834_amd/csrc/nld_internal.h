// Internal declarations of libnld (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nld.h"

namespace nld {

constexpr int kMaxTap = 16;        // 2m for m <= 8
constexpr int kRedBlocks = 512;    // blocks of the FP64 reductions
constexpr int kMaxChunk = 4096;    // most nodes of one spreading / gathering workgroup
constexpr int kRedThreads = 256;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct HipError {
  hipError_t err;
  std::string where;
};
#define NLD_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) throw ::nld::HipError{e_, std::string(#call)};           \
  } while (0)

// ------------------------------------------------------------------ per-window data
// Every window is stored with three internal dimensions; a window with t kept dimensions
// uses the last t of them and the leading ones have n = 1, a single tap of weight 1.
struct WinDev {
  int t;               // kept dimensions
  int n[3];            // grid points per internal dimension
  int taps[3];         // 2m, or 1 for an unused dimension
  int m;
  double b;            // Kaiser-Bessel shape
  double kb_den;       // 1 / (1 - exp(-2 b m))
  double weight;       // w_l
  int ts[3], nts[3];   // tiles: extent and count per dimension
  int pe[3];           // padded tile extent: ts + taps - 1
  int lts[3], lnts[3]; // log2 of ts and nts (all powers of two)
  int tile_off;        // first global tile id of this window
  long long grid_off;  // offset of this window's grid in the concatenated grid buffer
  long long grid_size; // n0 n1 n2
  const void* coef;    // [3][n_max] per-dimension Fourier multipliers (precision T)
  int n_max;
  const void* psi;     // [2m][deg + 1] window polynomial per tap (precision T), see psi_deg
  // buffers of the plan that owns the window, so that windows of several plans share launches
  int img;             // index of the window's image in the launch's image table
  int wl;              // index of the window in its plan
  long long N;         // nodes of the plan
  long long LN;        // N L of the plan: stride of the coordinate planes of g_frac
  const int* g_idx;    // the plan's sorted node lists (positions are plan-global)
  const unsigned* g_base;
  const void* g_frac;
  void* grid;          // the plan's concatenated grids (this window at grid_off)
  void* padded;        // the plan's padded-tile slots
  long long slot_stride;
  const int* tile_slot0;   // indexed by the plan's global tile id (tile_off + tile)
  const int* tile_nslot;
  void* ylocal;        // [N] this window's result
};

// Per-image (per-solve) data of a launch: vectors, degree, CG state and reduction scratch.
enum VecSel { V_Z = 0, V_R = 1, V_P = 2, V_Q = 3, V_F = 4, V_U = 5, V_ONES = 6, kNumVec = 7 };
struct CgState;
struct ImgDev {
  long long N;
  int win0, L;         // the image's windows in the launch's window table
  int nred;            // blocks of the image's FP64 reductions
  void* vec[kNumVec];  // CG vectors z, r, p, q, right-hand side f, solution u, ones
  double* D;           // degree vector
  double* D2;          // sum_l w_l^2 K_l(sigma_l / sqrt 2) 1 (l2 preconditioner), or null
  double* sumv;        // sum of the input (windows without kept dimensions)
  CgState* st;
  double* red;         // reduction partials [nred][8]
};
// A vector operand: ext if non-null (launches over a single image), else the image's vec[sel].
struct VecArg {
  const void* ext;
  int sel;
};

// Degree of the per-tap polynomial that replaces the window evaluation: the scaled
// Kaiser-Bessel window is an entire function of the distance, so a Chebyshev interpolant on each
// unit interval converges fast (max error ~4e-8 at degree 7, below FP32 rounding, and ~3e-15 at
// degree 14 for m = 3..8).
template <typename T> struct PsiDeg { static constexpr int value = sizeof(T) == 4 ? 7 : 14; };

struct TileJob {       // a chunk of the nodes of one tile (spreading and gathering)
  int win, tile, pbeg, pend, slot;   // pbeg/pend: positions in the sorted node list
};
struct FoldJob {       // 256 consecutive cells of one window's grid
  int win, ncell;
  long long cell0;
};
struct Fold3Job {      // one tile of a 3-D window
  int win, tile;
};
struct PlaneJob {     // one grid plane of a 3-D window (two fused convolution passes)
  int win, i0;
};
struct ConvJob {
  int win;
  int nl;              // lines in this job (<= lines per workgroup)
  long long off;       // offset of the first element of the first line in the window grid
};

// FP64 state of one CG solve (device)
struct CgState {
  double alpha;        // system parameter alpha
  double tol;          // relative tolerance
  double wsum;         // sum_l w_l (eta = D - wsum)
  double tol2_b2;      // tol^2 ||f_perp||^2
  double bnorm2;       // ||f_perp||^2
  double mean_f, mean_u0;
  double rho, a, beta, mean_t, mean_q, mean_r;
  double rr;           // ||r||^2 of the last update
  double rr_true;      // true residual norm^2 (diagnostic)
  double const_f;      // 0 if f is constant
  double last_pq, last_rho;  // last <p, A p> and <r, s> (diagnostics)
  double sum_pinv;     // sum_i 1 / P_i
  double w2sum;        // sum_l w_l^2 (self terms of D2)
  double scale_b;      // energy-optimal multiple of a warm start (use_u0 = 3)
  int iters, maxit, done, status, precond, deflate;
  unsigned int ticket[8];
};

// Everything one set of launches needs: the window table, the schedules and the image table.
// A plan has one over its own windows (one image); a batch concatenates those of its plans.
struct LaunchSet {
  nld_prec prec = NLD_FP32;
  int m = 4;                                    // cutoff (equal for every window of the set)
  const WinDev* d_wins = nullptr;
  const TileJob* d_tjobs = nullptr;
  const TileJob* d_gjobs = nullptr;             // the gathering's order of the same jobs
  int tjob_begin[4] = {0, 0, 0, 0};             // group g: windows with t = g + 1
  int max_padded = 1;                           // largest padded tile (cells)
  int ts3 = 0;                                  // 8 if every 3-D window has 8^3 tiles, else 0
  bool f3_quad = false;                         // every 8^3-tiled window: 4 | tiles along dim 2
  const Fold3Job* d_f3jobs = nullptr;
  int f3_begin[3] = {0, 0, 0};                  // tile extent 8: [0], [1]); 16: [1], [2])
  const FoldJob* d_fjobs = nullptr;
  int n_fjobs = 0;
  const ConvJob* d_conv[3] = {nullptr, nullptr, nullptr};
  int conv_begin[3][5] = {{0}};                 // per axis, grid size n = 32 << g
  const PlaneJob* d_pjobs = nullptr;
  int pjob_begin[3] = {0, 0, 0};                // n = 64: [0], [1]); n = 128: [1], [2])
  ImgDev* d_imgs = nullptr;
  int n_imgs = 0;
  long long max_N = 0;
  int max_nred = 1;
  bool has_flat = false;
};

// Host-side plan
struct Plan {
  nld_prec prec;
  int64_t N;
  int d;
  int L;
  int elem;                        // sizeof(T)
  std::vector<int> win_dim, win_feat;
  std::vector<double> sigma, weight;
  std::vector<int> bw;             // requested bandwidth per window (0 = automatic)
  int cutoff = 0;
  double oversampling = 2.0;
  double tol = 1e-6;
  long long lds_limit = 65536;      // bytes of LDS a workgroup may use
  std::vector<WinDev> wins;        // host copy
  std::vector<nld_window_info> info;
  std::vector<std::vector<double>> coef_host;  // per window [3][n_max]
  hipStream_t stream = nullptr;

  // device buffers
  WinDev* d_wins = nullptr;
  void* features = nullptr;        // not owned
  int* g_idx = nullptr;            // nodes of every window sorted by tile: node index,
  unsigned* g_base = nullptr;      // packed base cell and fractional offsets [3][L N]
  void* g_frac = nullptr;
  void* coef = nullptr;            // all windows' multipliers
  void* psi = nullptr;             // all windows' window polynomials
  // sigma-derivative kernel: for pass d, multiplier tables with dimension d's factor multiplied
  // by (1 - 2 pi^2 st_d^2 k^2) (zero for windows without dimension d), and window descriptors
  // pointing at them; buffers for the per-window products of the adjoint gradient
  void* coef_dv = nullptr;
  WinDev* d_wins_dv[3] = {nullptr, nullptr, nullptr};
  bool dv_used[3] = {false, false, false};
  void* grid_save = nullptr;
  void* yk = nullptr;              // [L][N] K_l v
  void* yks = nullptr;             // [L][N] K^s_l v
  void* dl = nullptr;              // [L][N] K_l 1
  void* dls = nullptr;             // [L][N] K^s_l 1
  double* adj_part = nullptr;      // reduction partials of the gradient sums
  std::vector<double> sig_t;       // [L][3] scaled widths per internal dimension
  std::vector<double> scale_t;     // [L][3] node scaling per internal dimension (0: dropped)
  int n_max = 1;                   // largest grid side over the windows (table stride)
  double psi_err = 0.0;            // max abs error of the window polynomial (plan time check)
  void* grid = nullptr;            // concatenated grids
  long long grid_total = 0;
  void* padded = nullptr;          // padded tile accumulators, one slot per spreading job
  long long slot_stride = 0;       // cells per slot
  int* tile_slot0 = nullptr;       // first slot of each global tile, and slot count
  int* tile_nslot = nullptr;
  int n_tiles_total = 0;
  void* ylocal = nullptr;          // [L][N] per-window results
  double* D = nullptr;             // degree vector
  double* sumv = nullptr;          // sum of the vector (windows without kept dimensions)
  bool has_flat = false;           // some window has no kept dimension: K_l = 1 1^T
  bool have_D = false;
  bool have_dl = false;            // dl / dls hold the per-window degrees of the current widths
  // l2 preconditioner (Sec. 4.3.1): multiplier tables of the kernels exp(-r^2 / (sigma_l^2 / 2))
  // on the same grids, window descriptors with weights w_l^2, and D2 (built on first use)
  void* coef_b = nullptr;
  WinDev* d_wins_b = nullptr;
  double* D2 = nullptr;
  bool have_D2 = false;
  double max_eta = 0.0;            // max(D) - sum_l w_l
  void* ones = nullptr;            // vector of ones (precision T)
  // schedules: tile jobs grouped by window dimension t (group g holds the jobs of t = g + 1)
  TileJob* d_tjobs = nullptr;
  int tjob_begin[4] = {0, 0, 0, 0};  // jobs of group g are [tjob_begin[g], tjob_begin[g + 1])
  int max_padded = 1;              // largest padded tile (cells)
  int max_tile_cells = 1;          // largest tile (cells)
  FoldJob* d_fjobs = nullptr; int n_fjobs = 0;     // per-cell fold (windows with t <= 2)
  Fold3Job* d_f3jobs = nullptr; int n_f3jobs = 0;   // per-tile fold (windows with t = 3)
  int f3_ts = 0;                                   // tile extent of the 3-D windows (8 or 16)
  bool f3_quad = false;                            // 4 | tiles along dim 2 in every 3-D window
  // convolution jobs per axis, grouped by grid size n = 32, 64, 128, 256 (group g: n = 32 << g)
  ConvJob* d_conv[3] = {nullptr, nullptr, nullptr};
  int conv_begin[3][5] = {{0}};
  // CG work vectors (precision T) and FP64 scratch
  void* z = nullptr; void* r = nullptr; void* p = nullptr; void* q = nullptr;
  double* red = nullptr;           // reduction partials [kRedBlocks][8]
  CgState* st = nullptr;           // device CG state
  CgState* st_host = nullptr;      // pinned mirror
  std::vector<void*> staging;      // pinned blocks of host-to-device copies in flight
  // while set, host tables collect in pending_blob (16-byte aligned) and reach the device in one
  // copy and one scatter kernel (each separate copy costs about 10 us of stream time)
  bool defer_uploads = false;
  std::vector<unsigned char> pending_blob;
  std::vector<void*> pending_dst;
  std::vector<size_t> pending_off, pending_bytes;
  // launch description of this plan alone, its image table and a pinned host mirror of it; the
  // fused schedule (plane kernels) and the unfused one (three convolution passes), which the
  // per-window products of the gradient use
  LaunchSet ls;
  LaunchSet ls_unfused;
  ImgDev* d_img = nullptr;
  ImgDev* img_host = nullptr;
  // host copies of the schedules (a batch concatenates them)
  std::vector<TileJob> h_tjobs;
  std::vector<TileJob> h_gjobs;                  // tile order, same groups (gathering)
  TileJob* d_gjobs = nullptr;
  std::vector<Fold3Job> h_f3jobs;
  std::vector<FoldJob> h_fjobs;
  std::vector<ConvJob> h_conv[3];
  std::vector<PlaneJob> h_pjobs;
  int pjob_begin[3] = {0, 0, 0};
  PlaneJob* d_pjobs = nullptr;
  Fold3Job* d_f3jobs_u = nullptr;               // unfused schedule (device only)
  int n_f3jobs_u = 0;
  ConvJob* d_conv_u[3] = {nullptr, nullptr, nullptr};
  int conv_begin_u[3][5] = {{0}};
  int tile3 = 0;                   // requested tile extent of 3-D windows (0: default)
  int max_grid = 0;                // largest grid side (0: no limit beyond 256)
};

// ------------------------------------------------------------------ launchers
// plan construction (plan.hip)
void build_plan(Plan& P, const void* features, hipStream_t s);
void release_plan(Plan& P);
// the gathering's order of the tile-ordered jobs [begin, end): eight contiguous ranges, one per
// XCD, each with its largest chunks first
void gather_order(std::vector<TileJob>& jobs, size_t begin, size_t end);
// stable sort of the jobs [b, e) by node count, largest first
void sort_by_size_desc(std::vector<TileJob>& jobs, size_t b, size_t e);
// device buffer of at least `bytes` from the library's per-device cache; a plan that stores it
// in one of its buffer fields returns it to the cache on release
void* plan_buffer(size_t bytes, hipStream_t s);
// pinned host block of at least `bytes` (zeroed unless zero = false), reused across calls;
// pinned_put returns it
void* pinned_get(size_t bytes, bool zero = true);
void pinned_put(void* p);
void launch_features(const void* img, int n1, int n2, int rho, int with_pos, nld_prec prec,
                     void* F, hipStream_t s);
// feature ranking (mis.hip)
int mis_default_bins(long long N);
void launch_mis(const void* F, long long N, int d, const void* y, nld_prec prec, int bins,
                double* scores, hipStream_t s);
// the same scores on the library's static device scratch (no allocation); words needed and held
long long mis_noalloc_words(int d, int bins);
long long mis_noalloc_capacity();
void launch_mis_noalloc(const void* F, long long N, int d, const void* y, nld_prec prec, int bins,
                        double* scores, hipStream_t s);

// fast summation (nfft.hip)
size_t plane_lds_bytes(int n);   // LDS of the fused plane convolution for n = 64 or 128
enum Epilogue { EPI_ANOVA = 0, EPI_LAPLACIAN = 1, EPI_DEGREE = 2, EPI_CG_Q = 3, EPI_CG_INIT = 4,
                EPI_CG_TRUE = 5 };
// Runs the per-window fast summations on the input of every image of the set and the window
// reduction with the epilogue (EPI_DEGREE writes Dout if given, else each image's D).  The
// iteration product (EPI_CG_Q) skips images whose solve has finished.
void matvec_set(const LaunchSet& ls, VecArg in, VecArg out, double* Dout, Epilogue epi,
                hipStream_t s);
// Single-plan form with external vectors (v, out may be null to use the plan's CG vectors
// through the selectors of the epilogue).
void matvec(Plan& P, const void* v, void* out, Epilogue epi, hipStream_t s);

// Per-window products K_l v -> yk and (sigma dK_l/dsigma) v -> yks (nfft.hip)
void matvec_parts(Plan& P, const void* v, void* yk, void* yks, hipStream_t s);
// FP64 sums for the gradient: per window {p.u.D_l, p.K_l u, p.u.Ds_l, p.Ks_l u}, then sum p,
// sum u, sum p u; result on the host (nfft.hip)
void gradient_sums(Plan& P, const void* p, const void* u, std::vector<double>& out, hipStream_t s);

// CG (pcg.hip)
void compute_max_eta(Plan& P, hipStream_t s);
void update_kernel(Plan& P, const double* sigma, const double* weight, hipStream_t s);
// D2 = sum_l w_l^2 K_l(sigma_l / sqrt 2) 1 for the l2 preconditioner (plan.hip, lazily)
void ensure_l2_degree(Plan& P, hipStream_t s);
nld_status run_pcg(Plan& P, double alpha, const void* f, void* u, const nld_pcg_opts& o,
                   nld_pcg_info& info, hipStream_t s);
nld_status run_adjoint(Plan& P, double alpha, const void* u, const void* g, void* p, double* grad,
                       const nld_pcg_opts& o, nld_pcg_info& info, hipStream_t s);
// Independent solves of several plans with one launch per stage (batch.hip)
nld_status run_pcg_batched(Plan* const* plans, const double* alpha, const void* const* f,
                           void* const* u, int count, const nld_pcg_opts& o, nld_pcg_info* infos,
                           hipStream_t s);

}  // namespace nld
