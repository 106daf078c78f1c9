// Host side of the MI355X Bloch-Maxwell eigensolver: multigrid hierarchy, V-cycles,
// null-space projection, Ritz step, preconditioned block inverse iteration and
// Rayleigh-quotient extrapolation across Bloch parameters, behind the C ABI of bloch.h.
// Every numerical step runs in the gfx950 kernels of stencils.hip and dense.hip; the host
// only sequences launches on the caller's stream and reads back the per-iteration
// residual norms that decide convergence.
#include "bloch.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace bl;

void axpy_inplace_d(double* y, const double* x, int64_t n, hipStream_t st);
void axpy_inplace_f(float* y, const float* x, int64_t n, hipStream_t st);
void split_gram(const double* GH, int q, double* G, double* H, hipStream_t st);

namespace {

constexpr int kMaxLevels = 16;
constexpr int64_t kMaxCoarse = 2048;
// Ritz step: basis directions whose squared M-distance from the previously kept ones is
// below this fraction of their squared M-norm are dropped as numerically dependent.
constexpr double kDropRel = 1e-10;   // largest coarsest-level edge count solved densely

struct Level {
  Geo g{};
  double* kappa64 = nullptr;
  float* kappa32 = nullptr;
  double* sinv64 = nullptr;
  float* sinv32 = nullptr;
  PatchT T4{};
  double Q[16]{};
  // V-cycle work blocks per precision (0 = FP64, 1 = FP32)
  void* ex[2] = {nullptr, nullptr};
  void* eb[2] = {nullptr, nullptr};
  void* er[2] = {nullptr, nullptr};
  int ecap[2] = {0, 0};
  void* nx[2] = {nullptr, nullptr};
  void* nb[2] = {nullptr, nullptr};
  void* nr[2] = {nullptr, nullptr};
  int ncap[2] = {0, 0};
};

Geo make_geo(int n, int m, double a, double b) {
  Geo g;
  g.n = n;
  g.m = m;
  g.h1 = a / n;
  g.h2 = b / m;
  g.s = 1.0 / (g.h1 * g.h2);
  g.mx = g.h2 / g.h1;
  g.my = g.h1 / g.h2;
  g.nm = (int64_t)n * m;
  g.ne = 2 * g.nm;
  return g;
}

bool is_gamma(double k1, double k2, double a, double b) {
  const double tp = 2.0 * M_PI;
  const double t1 = k1 * a - tp * std::nearbyint(k1 * a / tp);
  const double t2 = k2 * b - tp * std::nearbyint(k2 * b / tp);
  return std::fabs(t1) <= 1e-14 && std::fabs(t2) <= 1e-14;
}

// Smallest non-zero eigenvalues of the homogeneous cell (eps = eps0) at k = 0: the discrete
// plane-wave spectrum (4/h1^2) s1/(1 - 2/3 s1) + (4/h2^2) s2/(1 - 2/3 s2), used to scale mu.
double homogeneous_lambda(int n, int m, double a, double b, double eps0, int p) {
  std::vector<double> v;
  const double h1 = a / n, h2 = b / m;
  const int span1 = std::min(n, 2 * p + 4), span2 = std::min(m, 2 * p + 4);
  for (int r = -span2; r <= span2; ++r)
    for (int q = -span1; q <= span1; ++q) {
      const double s1 = std::pow(std::sin(M_PI * q / n), 2), s2 = std::pow(std::sin(M_PI * r / m), 2);
      const double l = (4 / (h1 * h1)) * s1 / (1 - 2.0 / 3.0 * s1) + (4 / (h2 * h2)) * s2 / (1 - 2.0 / 3.0 * s2);
      if (l > 1e-12) v.push_back(l / eps0);
    }
  std::sort(v.begin(), v.end());
  if (v.empty()) return 1.0;
  return v[std::min<size_t>(v.size() - 1, (size_t)std::max(0, p - 1))];
}

thread_local char g_errbuf[512];

}  // namespace

struct bl_solver {
  bl_grid grid{};
  bl_opts opts{};
  hipStream_t st = nullptr;
  int device = 0;
  int p = 0, qmax = 0;
  double mu = 1.0;
  std::vector<Level> lv;
  NodalStencil ns{};
  Phase ph{};
  bool gamma = false;
  bool kset = false;
  double k1 = 0, k2 = 0;
  int64_t nce = 0, ncn = 0;
  double* kc_inv64 = nullptr;
  float* kc_inv32 = nullptr;
  double* pc_inv64 = nullptr;
  float* pc_inv32 = nullptr;
  double* probe_in = nullptr;
  double* probe_out = nullptr;
  // iteration state
  double* E = nullptr;
  double* Enew = nullptr;
  double* S = nullptr;
  double* W = nullptr;
  double* hist[3] = {nullptr, nullptr, nullptr};
  int hist_count = 0;
  double hist_lam1 = 0.0;
  double* lam_d = nullptr;
  double* theta_d = nullptr;
  int* count_d = nullptr;
  double* partial = nullptr;
  int64_t partial_cap = 0;
  double* norms = nullptr;
  double* gram_partial = nullptr;
  int64_t gram_cap = 0;
  double* GH = nullptr;
  double* Gm = nullptr;
  double* Hm = nullptr;
  double* Yd = nullptr;
  double* ritz_work = nullptr;
  double* mean_scratch = nullptr;
  void* nodal_extra[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [prec][residual, correction]
  int nodal_extra_cap[2] = {0, 0};
  std::vector<void*> allocs;
  size_t dev_bytes = 0;
  int64_t launches = 0;
  std::vector<double> res_hist;
  int res_rows = 0;
  // opt-in HIP-event timing of the finest-level smoother launches
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  double timed_ms = 0.0;
  int64_t timed_count = 0;
  int64_t timed_cols = 0;
  bool debug = false;
};

namespace {

int set_error(int code, const char* fmt, const char* detail = "") {
  std::snprintf(g_errbuf, sizeof(g_errbuf), fmt, detail);
  return code;
}

#define HIP_OK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e_)); \
  } while (0)

int dalloc(bl_solver* s, void** out, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return set_error(BL_ENOMEM, "device allocation failed%s");
  s->allocs.push_back(p);
  s->dev_bytes += bytes;
  *out = p;
  return BL_OK;
}
template <typename T>
int dalloc_t(bl_solver* s, T** out, size_t count) {
  return dalloc(s, reinterpret_cast<void**>(out), count * sizeof(T));
}

size_t edge_block_bytes(const Geo& g, int cols, int prec) { return (size_t)cols * 2 * g.ne * (prec ? 4 : 8); }
size_t nodal_block_bytes(const Geo& g, int cols, int prec) { return (size_t)cols * 2 * g.nm * (prec ? 4 : 8); }

int ensure_level_buffers(bl_solver* s, int prec, int ecols, int ncols) {
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    if (L.ecap[prec] < ecols) {
      int rc;
      if (l > 0 && (rc = dalloc(s, &L.ex[prec], edge_block_bytes(L.g, ecols, prec)))) return rc;
      if (l > 0 && (rc = dalloc(s, &L.eb[prec], edge_block_bytes(L.g, ecols, prec)))) return rc;
      if ((rc = dalloc(s, &L.er[prec], edge_block_bytes(L.g, ecols, prec)))) return rc;
      L.ecap[prec] = ecols;
    }
    if (L.ncap[prec] < ncols) {
      int rc;
      if ((rc = dalloc(s, &L.nx[prec], nodal_block_bytes(L.g, ncols, prec)))) return rc;
      if ((rc = dalloc(s, &L.nb[prec], nodal_block_bytes(L.g, ncols, prec)))) return rc;
      if ((rc = dalloc(s, &L.nr[prec], nodal_block_bytes(L.g, ncols, prec)))) return rc;
      L.ncap[prec] = ncols;
    }
  }
  if (s->nodal_extra_cap[prec] < ncols) {
    int rc;
    for (int k = 0; k < 2; ++k)
      if ((rc = dalloc(s, &s->nodal_extra[prec][k], nodal_block_bytes(s->lv[0].g, ncols, prec)))) return rc;
    s->nodal_extra_cap[prec] = ncols;
  }
  return BL_OK;
}

template <typename T> struct PrecOf;
template <> struct PrecOf<double> { static constexpr int v = 0; };
template <> struct PrecOf<float> { static constexpr int v = 1; };

template <typename T>
const void* kc_inv(const bl_solver* s) { return PrecOf<T>::v ? (const void*)s->kc_inv32 : (const void*)s->kc_inv64; }
template <typename T>
const void* pc_inv(const bl_solver* s) { return PrecOf<T>::v ? (const void*)s->pc_inv32 : (const void*)s->pc_inv64; }

// ---- edge V-cycle for K = A + mu M with zero initial guess: x = V(b) ---------------------
// Event pairs around the finest-level smoother launches (opt-in, see bl_set_timing).
void timing_begin(bl_solver* s, int l) {
  if (!s->timing || l != 0) return;
  if (s->ev_used + 2 > (int)s->ev_pool.size()) return;
  (void)hipEventRecord(s->ev_pool[s->ev_used], s->st);
}
void timing_end(bl_solver* s, int l, int ncols) {
  if (!s->timing || l != 0) return;
  if (s->ev_used + 2 > (int)s->ev_pool.size()) return;
  (void)hipEventRecord(s->ev_pool[s->ev_used + 1], s->st);
  s->ev_used += 2;
  s->timed_cols += ncols;
}
void timing_collect(bl_solver* s) {
  if (!s->timing) return;
  for (int i = 0; i + 1 < s->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventSynchronize(s->ev_pool[i + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, s->ev_pool[i], s->ev_pool[i + 1]) == hipSuccess) {
      s->timed_ms += ms;
      s->timed_count += 1;
    }
  }
  s->ev_used = 0;
}

template <typename T>
void vcycle_edge(bl_solver* s, int l, const T* b, T* x, int ncols) {
  const int pr = PrecOf<T>::v;
  Level& L = s->lv[l];
  const int nl = (int)s->lv.size();
  if (l == nl - 1) {
    dense_apply<T>(kc_inv<T>(s), s->nce, b, x, ncols, s->st);
    s->launches += 1;
    return;
  }
  fill_zero<T>(x, (int64_t)ncols * 2 * L.g.ne, s->st);
  for (int it = 0; it < s->opts.nu_pre; ++it)
    for (int c = 0; c < 4; ++c) {
      timing_begin(s, l);
      edge_gs<T>(x, b, L.kappa64, L.kappa32, L.sinv64, L.sinv32, L.g, s->ph, s->mu, L.T4, c, ncols, s->st);
      timing_end(s, l, ncols);
    }
  T* r = static_cast<T*>(L.er[pr]);
  edge_apply<T, T>(EM_RESID_K, x, b, r, L.kappa64, L.kappa32, nullptr, L.g, s->ph, s->mu, ncols, nullptr, nullptr, s->st);
  Level& C = s->lv[l + 1];
  T* bc = static_cast<T*>(C.eb[pr]);
  T* xc = static_cast<T*>(C.ex[pr]);
  edge_restrict<T>(r, L.g, bc, C.g, s->ph, ncols, s->st);
  vcycle_edge<T>(s, l + 1, bc, xc, ncols);
  edge_prolong_add<T>(xc, C.g, x, L.g, s->ph, ncols, s->st);
  for (int it = 0; it < s->opts.nu_post; ++it)
    for (int c = 3; c >= 0; --c) {
      timing_begin(s, l);
      edge_gs<T>(x, b, L.kappa64, L.kappa32, L.sinv64, L.sinv32, L.g, s->ph, s->mu, L.T4, c, ncols, s->st);
      timing_end(s, l, ncols);
    }
  s->launches += 4 + 4 * (s->opts.nu_post + s->opts.nu_pre);
}

// ---- nodal V-cycle for P = L^* M L ----------------------------------------------------------
template <typename T>
void vcycle_nodal(bl_solver* s, int l, const T* b, T* x, int ncols) {
  const int pr = PrecOf<T>::v;
  Level& L = s->lv[l];
  const int nl = (int)s->lv.size();
  if (l == nl - 1) {
    dense_apply<T>(pc_inv<T>(s), s->ncn, b, x, ncols, s->st);
    s->launches += 1;
    return;
  }
  fill_zero<T>(x, (int64_t)ncols * 2 * L.g.nm, s->st);
  for (int it = 0; it < s->opts.nu_pre; ++it)
    for (int c = 0; c < 4; ++c) nodal_gs<T>(x, b, L.g, s->ph, s->ns, c, ncols, s->st);
  T* r = static_cast<T*>(L.nr[pr]);
  nodal_apply<T>(x, b, r, L.g, s->ph, s->ns, true, ncols, s->st);
  Level& C = s->lv[l + 1];
  T* bc = static_cast<T*>(C.nb[pr]);
  T* xc = static_cast<T*>(C.nx[pr]);
  nodal_restrict<T>(r, L.g, bc, C.g, s->ph, ncols, s->st);
  vcycle_nodal<T>(s, l + 1, bc, xc, ncols);
  nodal_prolong_add<T>(xc, C.g, x, L.g, s->ph, ncols, s->st);
  for (int it = 0; it < s->opts.nu_post; ++it)
    for (int c = 3; c >= 0; --c) nodal_gs<T>(x, b, L.g, s->ph, s->ns, c, ncols, s->st);
  s->launches += 4 + 4 * (s->opts.nu_pre + s->opts.nu_post);
}

// phi ~ P^{-1} b by `cycles` V-cycles (level-0 blocks b and phi must differ from the
// level-0 work blocks).
template <typename T>
void nodal_solve(bl_solver* s, const T* b, T* phi, int ncols, int cycles) {
  const int pr = PrecOf<T>::v;
  vcycle_nodal<T>(s, 0, b, phi, ncols);
  T* res = static_cast<T*>(s->nodal_extra[pr][0]);
  T* cor = static_cast<T*>(s->nodal_extra[pr][1]);
  const Geo& g = s->lv[0].g;
  for (int c = 1; c < cycles; ++c) {
    nodal_apply<T>(phi, b, res, g, s->ph, s->ns, true, ncols, s->st);
    vcycle_nodal<T>(s, 0, res, cor, ncols);
    const int64_t cnt = (int64_t)ncols * 2 * g.nm;
    if (pr) axpy_inplace_f(reinterpret_cast<float*>(phi), reinterpret_cast<const float*>(cor), cnt, s->st);
    else axpy_inplace_d(reinterpret_cast<double*>(phi), reinterpret_cast<const double*>(cor), cnt, s->st);
    s->launches += 3;
  }
}

struct Group {
  const void* ptr;
  int prec;
  int cols;
};

// Null-space elimination (Section 4) of the column groups into S (FP64, contiguous):
// S = U - L Phi with Phi from nodal V-cycles for P Phi = L^* M U; at k = 0 also the
// constant edge fields are removed.  Nodal arithmetic in the inner precision `ip`.
template <typename TN>
int project_groups(bl_solver* s, const std::vector<Group>& groups, double* Sout) {
  const int pr = PrecOf<TN>::v;
  int total = 0;
  for (auto& g : groups) total += g.cols;
  int rc = ensure_level_buffers(s, pr, s->lv[0].ecap[pr] > 0 ? s->lv[0].ecap[pr] : s->p, std::max(total, s->qmax));
  if (rc) return rc;
  const Geo& g0 = s->lv[0].g;
  // right-hand side and solution of the nodal solve: the level-0 nodal blocks nb and nx,
  // which the level-0 V-cycle itself does not use (it works in nr and the coarser levels)
  TN* b0 = static_cast<TN*>(s->lv[0].nb[pr]);
  TN* phi = static_cast<TN*>(s->lv[0].nx[pr]);
  int off = 0;
  for (auto& gr : groups) {
    TN* dst = b0 + (int64_t)off * 2 * g0.nm;
    if (gr.prec == 0) lhm<double, TN>(static_cast<const double*>(gr.ptr), dst, g0, s->ph, gr.cols, s->st);
    else lhm<float, TN>(static_cast<const float*>(gr.ptr), dst, g0, s->ph, gr.cols, s->st);
    off += gr.cols;
    s->launches += 1;
  }
  // the V-cycle at level 0 writes its own x into the buffer passed; keep b0 and phi apart
  // from the level-0 work blocks used inside vcycle_nodal (nr) and nodal_solve (extra).
  nodal_solve<TN>(s, b0, phi, total, std::max(1, s->opts.nodal_cycles));
  off = 0;
  for (auto& gr : groups) {
    const TN* ph_ = phi + (int64_t)off * 2 * g0.nm;
    double* dst = Sout + (int64_t)off * 2 * g0.ne;
    if (gr.prec == 0) lift_sub<double, TN, double>(static_cast<const double*>(gr.ptr), ph_, dst, g0, s->ph, gr.cols, s->st);
    else lift_sub<float, TN, double>(static_cast<const float*>(gr.ptr), ph_, dst, g0, s->ph, gr.cols, s->st);
    off += gr.cols;
    s->launches += 1;
  }
  if (s->gamma) {
    gamma_deflate(Sout, g0, total, s->mean_scratch, s->st);
    s->launches += 2;
  }
  return BL_OK;
}

int project(bl_solver* s, const std::vector<Group>& groups, double* Sout) {
  if (s->opts.precision) return project_groups<float>(s, groups, Sout);
  return project_groups<double>(s, groups, Sout);
}

// Ritz step on the q columns of S (FP64): G = S^* M S, H = S^* A S, generalised eigen-
// problem, E <- S Y for the `want` smallest Ritz values above zero_thr.  Returns the count.
int ritz_step(bl_solver* s, int q, int nfix, int want, double zero_thr, int* found) {
  const Level& L = s->lv[0];
  const Geo& g = L.g;
  double* WM = s->W;
  double* WA = s->W + (int64_t)q * 2 * g.ne;
  edge_apply<double, double>(EM_M, s->S, nullptr, WM, L.kappa64, L.kappa32, nullptr, g, s->ph, s->mu, q, nullptr, nullptr, s->st);
  edge_apply<double, double>(EM_A, s->S, nullptr, WA, L.kappa64, L.kappa32, nullptr, g, s->ph, s->mu, q, nullptr, nullptr, s->st);
  gram(s->S, q, s->W, 2 * q, g.ne, s->gram_partial, s->gram_cap, s->GH, s->st);
  split_gram(s->GH, q, s->Gm, s->Hm, s->st);
  ritz_small(s->Gm, s->Hm, q, nfix, want, zero_thr, kDropRel, s->ritz_work, s->Yd, s->theta_d, s->count_d, s->st);
  block_combine(s->S, q, s->Yd, want, g.ne, s->Enew, s->st);
  s->launches += 7;
  if (s->debug) {
    double sw[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    (void)hipMemcpyAsync(sw, s->ritz_work + 10 * q * q + 8 * q, 10 * 8, hipMemcpyDeviceToHost, s->st);
    (void)hipStreamSynchronize(s->st);
    std::fprintf(stderr, "bloch: ritz q=%d want=%d rank %.0f  shader MHz %.0f  phase us: chol %.1f basis %.1f hprime %.1f tridiag %.1f eig %.1f back %.1f\n",
                 q, want, sw[0], (sw[9] - sw[8]) / ((sw[7] - sw[1]) * 0.01), (sw[2] - sw[1]) * 0.01, (sw[3] - sw[2]) * 0.01, (sw[4] - sw[3]) * 0.01,
                 (sw[5] - sw[4]) * 0.01, (sw[6] - sw[5]) * 0.01, (sw[7] - sw[6]) * 0.01);
  }
  std::swap(s->E, s->Enew);
  std::swap(s->lam_d, s->theta_d);
  int cnt = 0;
  HIP_OK(hipMemcpyAsync(&cnt, s->count_d, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  *found = cnt;
  return BL_OK;
}

int setup_k(bl_solver* s, double k1, double k2) {
  if (!std::isfinite(k1) || !std::isfinite(k2)) return set_error(BL_EINVAL, "non-finite Bloch parameter%s");
  s->gamma = is_gamma(k1, k2, s->grid.a, s->grid.b);
  if (s->gamma) {
    s->ph = {1.0, 0.0, 1.0, 0.0};
  } else {
    s->ph = {std::cos(k1 * s->grid.a), std::sin(k1 * s->grid.a), std::cos(k2 * s->grid.b), std::sin(k2 * s->grid.b)};
  }
  s->k1 = k1;
  s->k2 = k2;
  // coarsest-level direct solvers for this k
  Level& C = s->lv.back();
  identity_block(s->probe_in, s->nce, s->st);
  edge_apply<double, double>(EM_K, s->probe_in, nullptr, s->probe_out, C.kappa64, C.kappa32, nullptr, C.g, s->ph, s->mu, (int)s->nce, nullptr, nullptr, s->st);
  planar_to_matrix(s->probe_out, s->nce, s->kc_inv64, s->st);
  invert_hpd(s->kc_inv64, s->nce, s->st);
  matrix_to_float(s->kc_inv64, s->kc_inv32, 2 * s->nce * s->nce, s->st);
  identity_block(s->probe_in, s->ncn, s->st);
  nodal_apply<double>(s->probe_in, nullptr, s->probe_out, C.g, s->ph, s->ns, false, (int)s->ncn, s->st);
  planar_to_matrix(s->probe_out, s->ncn, s->pc_inv64, s->st);
  if (s->gamma) add_constant_rank_one(s->pc_inv64, s->ncn, s->ns.c0, s->st);
  invert_hpd(s->pc_inv64, s->ncn, s->st);
  matrix_to_float(s->pc_inv64, s->pc_inv32, 2 * s->ncn * s->ncn, s->st);
  s->launches += 10;
  s->kset = true;
  return BL_OK;
}

int validate(const bl_grid* grid, const double* eps, const bl_opts* o) {
  if (!grid) return set_error(BL_EINVAL, "grid is NULL%s");
  if (grid->n < 2 || grid->m < 2) return set_error(BL_EINVAL, "n and m must be >= 2%s");
  if (!(grid->a > 0) || !(grid->b > 0) || !std::isfinite(grid->a) || !std::isfinite(grid->b))
    return set_error(BL_EINVAL, "a and b must be positive and finite%s");
  if (!eps) return set_error(BL_EINVAL, "eps is NULL%s");
  const int64_t nm = (int64_t)grid->n * grid->m;
  for (int64_t i = 0; i < nm; ++i)
    if (!(eps[i] > 0) || !std::isfinite(eps[i])) return set_error(BL_EINVAL, "eps must be positive and finite%s");
  if (o->nev < 1 || o->nthrow < 0) return set_error(BL_EINVAL, "nev >= 1 and nthrow >= 0 required%s");
  const int p = o->nev + o->nthrow;
  if (p > 80) return set_error(BL_EINVAL, "nev + nthrow must be <= 80%s");
  if ((int64_t)p > nm - 1) return set_error(BL_EINVAL, "nev + nthrow must be <= n*m - 1%s");
  if (o->max_iter < 0 || o->nu_pre < 0 || o->nu_post < 0 || o->nodal_cycles < 1)
    return set_error(BL_EINVAL, "invalid iteration options%s");
  if (o->variant != 0) return set_error(BL_EINVAL, "only the gradient variant is available%s");
  if (o->precision != 0 && o->precision != 1) return set_error(BL_EINVAL, "precision must be 0 or 1%s");
  if (o->extrap_depth < 1 || o->extrap_depth > 3) return set_error(BL_EINVAL, "extrap_depth must be 1..3%s");
  if (!(o->tol > 0)) return set_error(BL_EINVAL, "tol must be positive%s");
  return BL_OK;
}

void fill_defaults(bl_opts* o) {
  if (o->max_iter == 0) o->max_iter = 200;
  if (o->coarsest_min <= 0) o->coarsest_min = 8;
  if (o->nodal_cycles <= 0) o->nodal_cycles = 2;
  if (o->extrap_depth <= 0) o->extrap_depth = 3;
  if (!(o->tol > 0)) o->tol = 1e-8;
  if (!(o->zero_rel > 0)) o->zero_rel = 1e-2;
}

std::vector<std::pair<int, int>> hierarchy(int n, int m, int max_levels, int cmin) {
  std::vector<std::pair<int, int>> v{{n, m}};
  while (true) {
    auto [cn, cm] = v.back();
    if (max_levels && (int)v.size() >= max_levels) break;
    if ((int)v.size() >= kMaxLevels) break;
    if (cn % 2 || cm % 2 || cn / 2 < cmin || cm / 2 < cmin) break;
    v.push_back({cn / 2, cm / 2});
  }
  return v;
}

size_t footprint(const bl_grid* grid, const bl_opts* o) {
  const int p = o->nev + o->nthrow;
  const int q = 3 * p;
  auto lv = hierarchy(grid->n, grid->m, o->levels, o->coarsest_min > 0 ? o->coarsest_min : 8);
  const int pr = o->precision ? 1 : 0;
  size_t bytes = 0;
  for (size_t l = 0; l < lv.size(); ++l) {
    Geo g = make_geo(lv[l].first, lv[l].second, grid->a, grid->b);
    bytes += g.nm * (8 + 4) + (l + 1 < lv.size() ? g.nm * 6 * 12 : 0);
    bytes += edge_block_bytes(g, p, pr) * (l ? 3 : 1) + nodal_block_bytes(g, q, pr) * 3;
  }
  Geo g0 = make_geo(grid->n, grid->m, grid->a, grid->b);
  const size_t col = (size_t)2 * g0.ne * 8;
  bytes += col * (2 * p + q + 2 * q + 3 * p);   // E, Enew, S, W, history
  bytes += edge_block_bytes(g0, p, pr) * 2;      // R and C
  bytes += nodal_block_bytes(g0, q, pr) * 2;     // nodal multi-cycle work
  Geo gc = make_geo(lv.back().first, lv.back().second, grid->a, grid->b);
  bytes += (size_t)gc.ne * gc.ne * 16 * 3 + (size_t)gc.nm * gc.nm * 16 * 3;
  bytes += (size_t)256 * q * 2 * q * 16 + (size_t)12 * q * q * 16;
  return bytes;
}

int alloc_all(bl_solver* s, const double* eps) {
  const bl_grid& gr = s->grid;
  auto sizes = hierarchy(gr.n, gr.m, s->opts.levels, s->opts.coarsest_min);
  s->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) s->lv[l].g = make_geo(sizes[l].first, sizes[l].second, gr.a, gr.b);
  const Geo& c = s->lv.back().g;
  s->nce = c.ne;
  s->ncn = c.nm;
  if (s->nce > kMaxCoarse) return set_error(BL_EINVAL, "grid cannot be coarsened to a small enough level%s");
  // nodal stencil (same on every level: depends on h2/h1 only)
  {
    const double r = s->lv[0].g.mx, q = s->lv[0].g.my;
    s->ns = {(4.0 / 3.0) * (r + q), -(2.0 / 3.0) * r + (1.0 / 3.0) * q, (1.0 / 3.0) * r - (2.0 / 3.0) * q, -(1.0 / 6.0) * (r + q)};
  }
  int rc;
  // kappa per level
  std::vector<double> kap((size_t)gr.n * gr.m);
  for (size_t i = 0; i < kap.size(); ++i) kap[i] = 1.0 / eps[i];
  double eps_min = eps[0];
  for (size_t i = 0; i < kap.size(); ++i) eps_min = std::min(eps_min, eps[i]);
  if (!(s->opts.mu > 0)) s->mu = homogeneous_lambda(gr.n, gr.m, gr.a, gr.b, eps_min, s->p) / 10.0;
  else s->mu = s->opts.mu;
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    if ((rc = dalloc_t(s, &L.kappa64, L.g.nm))) return rc;
    if ((rc = dalloc_t(s, &L.kappa32, L.g.nm))) return rc;
    if (l == 0) HIP_OK(hipMemcpyAsync(L.kappa64, kap.data(), kap.size() * 8, hipMemcpyHostToDevice, s->st));
    else coarsen_kappa(s->lv[l - 1].kappa64, s->lv[l - 1].g, L.kappa64, s->st);
    to_float(L.kappa64, L.kappa32, L.g.nm, s->st);
    if (l + 1 < s->lv.size()) {
      // stabilised patch transform: Q e1 = D^{1/2} g / |D^{1/2} g|, g = (-1, 1, -1, 1)
      const double dx = L.g.mx * 2.0 / 3.0, dy = L.g.my * 2.0 / 3.0;
      double z[4] = {-std::sqrt(dx), std::sqrt(dx), -std::sqrt(dy), std::sqrt(dy)};
      const double nz = std::sqrt(2 * dx + 2 * dy);
      for (double& v : z) v /= nz;
      double w[4] = {1.0 - z[0], -z[1], -z[2], -z[3]};
      double ww = 0;
      for (double v : w) ww += v * v;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) L.Q[i * 4 + j] = (i == j ? 1.0 : 0.0) - 2.0 * w[i] * w[j] / ww;
      const double dd[4] = {dx, dx, dy, dy};
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) L.T4.t[i * 4 + j] = L.Q[i * 4 + j] / std::sqrt(dd[i]);
      if ((rc = dalloc_t(s, &L.sinv64, L.g.nm * 6))) return rc;
      if ((rc = dalloc_t(s, &L.sinv32, L.g.nm * 6))) return rc;
      patch_setup(L.kappa64, L.g, L.T4, L.Q, s->mu, L.sinv64, L.sinv32, s->st);
    }
  }
  const Geo& g0 = s->lv[0].g;
  const int p = s->p, q = s->qmax;
  const size_t col = (size_t)2 * g0.ne;
  if ((rc = dalloc_t(s, &s->E, col * p))) return rc;
  if ((rc = dalloc_t(s, &s->Enew, col * p))) return rc;
  if ((rc = dalloc_t(s, &s->S, col * q))) return rc;
  if ((rc = dalloc_t(s, &s->W, col * 2 * q))) return rc;
  for (int h = 0; h < 3; ++h)
    if ((rc = dalloc_t(s, &s->hist[h], col * p))) return rc;
  if ((rc = dalloc_t(s, &s->lam_d, q))) return rc;
  if ((rc = dalloc_t(s, &s->theta_d, q))) return rc;
  if ((rc = dalloc_t(s, &s->count_d, 4))) return rc;
  s->partial_cap = (int64_t)p * ((g0.ne + 255) / 256) * 2;
  if ((rc = dalloc_t(s, &s->partial, s->partial_cap))) return rc;
  if ((rc = dalloc_t(s, &s->norms, (size_t)2 * q))) return rc;
  s->gram_cap = (int64_t)gram_blocks(g0.ne) * q * 2 * q * 2;
  if ((rc = dalloc_t(s, &s->gram_partial, s->gram_cap))) return rc;
  if ((rc = dalloc_t(s, &s->GH, (size_t)q * 2 * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->Gm, (size_t)q * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->Hm, (size_t)q * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->Yd, (size_t)q * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->ritz_work, ritz_small_work_doubles(q)))) return rc;
  if ((rc = dalloc_t(s, &s->mean_scratch, (size_t)4 * q))) return rc;
  const int64_t pc = std::max(s->nce, s->ncn);
  if ((rc = dalloc_t(s, &s->probe_in, (size_t)2 * pc * pc))) return rc;
  if ((rc = dalloc_t(s, &s->probe_out, (size_t)2 * pc * pc))) return rc;
  if ((rc = dalloc_t(s, &s->kc_inv64, (size_t)2 * s->nce * s->nce))) return rc;
  if ((rc = dalloc_t(s, &s->kc_inv32, (size_t)2 * s->nce * s->nce))) return rc;
  if ((rc = dalloc_t(s, &s->pc_inv64, (size_t)2 * s->ncn * s->ncn))) return rc;
  if ((rc = dalloc_t(s, &s->pc_inv32, (size_t)2 * s->ncn * s->ncn))) return rc;
  const int ip = s->opts.precision;
  if ((rc = ensure_level_buffers(s, ip, p, q))) return rc;
  // level-0 edge x / b blocks of the V-cycle are the correction C and the residual R
  if ((rc = dalloc(s, &s->lv[0].ex[ip], edge_block_bytes(g0, p, ip)))) return rc;
  if ((rc = dalloc(s, &s->lv[0].eb[ip], edge_block_bytes(g0, p, ip)))) return rc;
  HIP_OK(hipStreamSynchronize(s->st));
  return BL_OK;
}

int check_hip(bl_solver* s) {
  (void)s;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BL_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return BL_OK;
}

// Residuals of the current Ritz block; returns relres (host, p) and copies lam to host.
int residuals(bl_solver* s, void* Rbuf, int inner_prec, std::vector<double>& lam, std::vector<double>& rel) {
  const Level& L = s->lv[0];
  int nblk = 0;
  if (inner_prec)
    edge_apply<double, float>(EM_EIGRES, s->E, nullptr, static_cast<float*>(Rbuf), L.kappa64, L.kappa32, s->lam_d, L.g, s->ph, s->mu, s->p, s->partial, &nblk, s->st);
  else
    edge_apply<double, double>(EM_EIGRES, s->E, nullptr, static_cast<double*>(Rbuf), L.kappa64, L.kappa32, s->lam_d, L.g, s->ph, s->mu, s->p, s->partial, &nblk, s->st);
  reduce_partials(s->partial, nblk, s->p, 2, s->norms, s->st);
  s->launches += 2;
  std::vector<double> nr((size_t)2 * s->p);
  lam.resize(s->p);
  HIP_OK(hipMemcpyAsync(nr.data(), s->norms, nr.size() * 8, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipMemcpyAsync(lam.data(), s->lam_d, lam.size() * 8, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  timing_collect(s);
  int rc = check_hip(s);
  if (rc) return rc;
  rel.resize(s->p);
  for (int j = 0; j < s->p; ++j) {
    const double den = std::fabs(lam[j]) * std::sqrt(nr[2 * j + 1]);
    rel[j] = den > 0 ? std::sqrt(nr[2 * j]) / den : INFINITY;
  }
  return BL_OK;
}

int solve_one(bl_solver* s, double k1, double k2, const void* start_dev, double* evals,
              double* relres, int32_t* iters, void* evecs_dev) {
  const int p = s->p, nev = s->opts.nev;
  const int ip = s->opts.precision;
  const Geo& g0 = s->lv[0].g;
  if (!start_dev && s->hist_count == 0) return set_error(BL_ESTATE, "no start block and no history to extrapolate from%s");
  int rc = setup_k(s, k1, k2);
  if (rc) return rc;
  int found = 0;
  if (start_dev) {
    rc = project(s, {{start_dev, 0, p}}, s->S);
    if (rc) return rc;
    rc = ritz_step(s, p, 0, p, -INFINITY, &found);
  } else {
    std::vector<Group> gs;
    const int depth = std::min(s->hist_count, s->opts.extrap_depth);
    for (int h = 0; h < depth; ++h) gs.push_back({s->hist[h], 0, p});
    rc = project(s, gs, s->S);
    if (rc) return rc;
    rc = ritz_step(s, depth * p, 0, p, s->opts.zero_rel * s->hist_lam1, &found);
  }
  if (rc) return rc;
  if (found < p) return set_error(BL_ENOCONV, "start block spans fewer than p non-null directions%s");
  void* R = s->lv[0].eb[ip];
  void* C = s->lv[0].ex[ip];
  std::vector<double> lam, rel;
  s->res_hist.clear();
  s->res_rows = 0;
  int it = 0;
  bool conv = false;
  while (true) {
    rc = residuals(s, R, ip, lam, rel);
    if (rc) return rc;
    for (int j = 0; j < nev; ++j) s->res_hist.push_back(rel[j]);
    ++s->res_rows;
    conv = true;
    for (int j = 0; j < nev; ++j) conv = conv && (rel[j] <= s->opts.tol);
    if (conv || it >= s->opts.max_iter) break;
    if (ip) vcycle_edge<float>(s, 0, static_cast<float*>(R), static_cast<float*>(C), p);
    else vcycle_edge<double>(s, 0, static_cast<double*>(R), static_cast<double*>(C), p);
    rc = project(s, {{s->E, 0, p}, {C, ip, p}}, s->S);
    if (rc) return rc;
    rc = ritz_step(s, 2 * p, p, p, -INFINITY, &found);
    if (rc) return rc;
    ++it;
  }
  // history: most recent first
  double* last = s->hist[2];
  s->hist[2] = s->hist[1];
  s->hist[1] = s->hist[0];
  s->hist[0] = last;
  HIP_OK(hipMemcpyAsync(s->hist[0], s->E, (size_t)p * 2 * g0.ne * 8, hipMemcpyDeviceToDevice, s->st));
  s->hist_count = std::min(3, s->hist_count + 1);
  s->hist_lam1 = lam[0];
  if (evals) std::memcpy(evals, lam.data(), (size_t)nev * 8);
  if (relres) std::memcpy(relres, rel.data(), (size_t)nev * 8);
  if (iters) *iters = it;
  if (evecs_dev) HIP_OK(hipMemcpyAsync(evecs_dev, s->E, (size_t)nev * 2 * g0.ne * 8, hipMemcpyDeviceToDevice, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  rc = check_hip(s);
  if (rc) return rc;
  return conv ? BL_OK : set_error(BL_ENOCONV, "max_iter reached%s");
}

}  // namespace

// small helper kernels used above (defined here to keep them next to their only users)
namespace {
__global__ void k_axpy_d(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}
__global__ void k_axpy_f(float* __restrict__ y, const float* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}
__global__ void k_split_gram(const double* __restrict__ GH, int q, double* __restrict__ G, double* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)q * q) return;
  const int i = (int)(e / q), j = (int)(e % q);
  G[2 * e] = GH[2 * ((int64_t)i * 2 * q + j)];
  G[2 * e + 1] = GH[2 * ((int64_t)i * 2 * q + j) + 1];
  H[2 * e] = GH[2 * ((int64_t)i * 2 * q + q + j)];
  H[2 * e + 1] = GH[2 * ((int64_t)i * 2 * q + q + j) + 1];
}
}  // namespace
void axpy_inplace_d(double* y, const double* x, int64_t n, hipStream_t st) {
  k_axpy_d<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(y, x, n);
}
void axpy_inplace_f(float* y, const float* x, int64_t n, hipStream_t st) {
  k_axpy_f<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(y, x, n);
}
void split_gram(const double* GH, int q, double* G, double* H, hipStream_t st) {
  k_split_gram<<<(unsigned)(((int64_t)q * q + 255) / 256), 256, 0, st>>>(GH, q, G, H);
}

namespace {
template <typename T>
int apply_t(bl_solver* s, int op, int level, int ncols, const void* xv, const void* yv, void* outv) {
  const int pr = PrecOf<T>::v;
  const int nl = (int)s->lv.size();
  if (level < 0 || level >= nl) return set_error(BL_EINVAL, "level out of range%s");
  Level& L = s->lv[level];
  const T* x = static_cast<const T*>(xv);
  const T* y = static_cast<const T*>(yv);
  T* out = static_cast<T*>(outv);
  const bool smoothed = level < nl - 1;
  int rc;
  switch (op) {
    case BL_OP_A: edge_apply<T, T>(EM_A, x, nullptr, out, L.kappa64, L.kappa32, nullptr, L.g, s->ph, s->mu, ncols, nullptr, nullptr, s->st); break;
    case BL_OP_M: edge_apply<T, T>(EM_M, x, nullptr, out, L.kappa64, L.kappa32, nullptr, L.g, s->ph, s->mu, ncols, nullptr, nullptr, s->st); break;
    case BL_OP_K: edge_apply<T, T>(EM_K, x, nullptr, out, L.kappa64, L.kappa32, nullptr, L.g, s->ph, s->mu, ncols, nullptr, nullptr, s->st); break;
    case BL_OP_LIFT: lift<T, T>(x, out, L.g, s->ph, ncols, s->st); break;
    case BL_OP_LHM: lhm<T, T>(x, out, L.g, s->ph, ncols, s->st); break;
    case BL_OP_P: nodal_apply<T>(x, nullptr, out, L.g, s->ph, s->ns, false, ncols, s->st); break;
    case BL_OP_EDGE_SMOOTH:
    case BL_OP_EDGE_SMOOTH_BACK:
      if (!smoothed || !y) return set_error(BL_EINVAL, "no smoother on this level / rhs missing%s");
      for (int c = 0; c < 4; ++c)
        edge_gs<T>(out, y, L.kappa64, L.kappa32, L.sinv64, L.sinv32, L.g, s->ph, s->mu, L.T4,
                   op == BL_OP_EDGE_SMOOTH ? c : 3 - c, ncols, s->st);
      break;
    case BL_OP_NODAL_SMOOTH:
      if (!smoothed || !y) return set_error(BL_EINVAL, "no smoother on this level / rhs missing%s");
      for (int c = 0; c < 4; ++c) nodal_gs<T>(out, y, L.g, s->ph, s->ns, c, ncols, s->st);
      break;
    case BL_OP_EDGE_VCYCLE:
    case BL_OP_NODAL_VCYCLE: {
      if ((rc = ensure_level_buffers(s, pr, ncols, ncols))) return rc;
      if (op == BL_OP_EDGE_VCYCLE) vcycle_edge<T>(s, level, x, out, ncols);
      else vcycle_nodal<T>(s, level, x, out, ncols);
      break;
    }
    case BL_OP_EDGE_PROLONG:
    case BL_OP_EDGE_RESTRICT:
    case BL_OP_NODAL_PROLONG:
    case BL_OP_NODAL_RESTRICT: {
      if (!smoothed) return set_error(BL_EINVAL, "no coarser level%s");
      Level& C = s->lv[level + 1];
      if (op == BL_OP_EDGE_PROLONG) {
        fill_zero<T>(out, (int64_t)ncols * 2 * L.g.ne, s->st);
        edge_prolong_add<T>(x, C.g, out, L.g, s->ph, ncols, s->st);
      } else if (op == BL_OP_EDGE_RESTRICT) {
        edge_restrict<T>(x, L.g, out, C.g, s->ph, ncols, s->st);
      } else if (op == BL_OP_NODAL_PROLONG) {
        fill_zero<T>(out, (int64_t)ncols * 2 * L.g.nm, s->st);
        nodal_prolong_add<T>(x, C.g, out, L.g, s->ph, ncols, s->st);
      } else {
        nodal_restrict<T>(x, L.g, out, C.g, s->ph, ncols, s->st);
      }
      break;
    }
    case BL_OP_PROJECT: {
      if (level != 0 || pr != 0) return set_error(BL_EINVAL, "projection runs on FP64 level-0 blocks%s");
      if (ncols > s->qmax) return set_error(BL_EINVAL, "too many columns%s");
      rc = project(s, {{x, 0, ncols}}, reinterpret_cast<double*>(out));
      if (rc) return rc;
      break;
    }
    case BL_OP_COARSE_EDGE:
      if (level != nl - 1) return set_error(BL_EINVAL, "coarse solve only on the coarsest level%s");
      dense_apply<T>(kc_inv<T>(s), s->nce, x, out, ncols, s->st);
      break;
    case BL_OP_COARSE_NODAL:
      if (level != nl - 1) return set_error(BL_EINVAL, "coarse solve only on the coarsest level%s");
      dense_apply<T>(pc_inv<T>(s), s->ncn, x, out, ncols, s->st);
      break;
    default: return set_error(BL_EINVAL, "unknown operator%s");
  }
  return BL_OK;
}
}  // namespace

// =========================================================================================
// C ABI
extern "C" {

void bl_default_opts(bl_opts* o, int32_t nev) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nev = nev > 0 ? nev : 8;
  o->nthrow = o->nev / 2;
  o->max_iter = 200;
  o->levels = 0;
  o->coarsest_min = 8;
  o->nu_pre = 1;
  o->nu_post = 1;
  o->nodal_cycles = 2;
  o->variant = 0;
  o->precision = 0;
  o->extrap_depth = 3;
  o->tol = 1e-8;
  o->mu = 0.0;
  o->zero_rel = 1e-2;
}

const char* bl_strerror(int code) {
  switch (code) {
    case BL_OK: return "ok";
    case BL_EINVAL: return "invalid argument";
    case BL_ENOMEM: return "out of memory";
    case BL_EHIP: return "HIP runtime error";
    case BL_ENOCONV: return "not converged";
    case BL_EAGAIN: return "not ready";
    case BL_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* bl_last_error(void) { return g_errbuf; }

size_t bl_footprint_bytes(const bl_grid* grid, const bl_opts* opts) {
  if (!grid) return 0;
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  return footprint(grid, &o);
}

int bl_create(const bl_grid* grid, const double* eps_cells, const bl_opts* opts, void* stream,
              bl_solver** out) {
  if (!out) return set_error(BL_EINVAL, "out is NULL%s");
  *out = nullptr;
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  int rc = validate(grid, eps_cells, &o);
  if (rc) return rc;
  bl_solver* s = new (std::nothrow) bl_solver();
  if (!s) return set_error(BL_ENOMEM, "host allocation failed%s");
  s->grid = *grid;
  s->opts = o;
  s->st = static_cast<hipStream_t>(stream);
  s->p = o.nev + o.nthrow;
  s->qmax = 3 * s->p;
  s->debug = std::getenv("BL_DEBUG") != nullptr;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return set_error(BL_EHIP, "no HIP device%s");
  }
  rc = alloc_all(s, eps_cells);
  if (rc == BL_OK) rc = check_hip(s);
  if (rc) {
    bl_destroy(s);
    return rc;
  }
  *out = s;
  return BL_OK;
}

void bl_destroy(bl_solver* s) {
  if (!s) return;
  if (s->st) (void)hipStreamSynchronize(s->st);
  else (void)hipDeviceSynchronize();
  for (void* p : s->allocs) (void)hipFree(p);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  delete s;
}

int bl_get_info(const bl_solver* s, bl_info* out) {
  if (!s || !out) return set_error(BL_EINVAL, "NULL argument%s");
  std::memset(out, 0, sizeof(*out));
  out->n = s->grid.n;
  out->m = s->grid.m;
  out->p = s->p;
  out->nev = s->opts.nev;
  out->levels = (int)s->lv.size();
  out->precision = s->opts.precision;
  for (size_t l = 0; l < s->lv.size() && l < 16; ++l) {
    out->level_n[l] = s->lv[l].g.n;
    out->level_m[l] = s->lv[l].g.m;
  }
  out->mu = s->mu;
  out->device_bytes = s->dev_bytes;
  out->kernel_launches = s->launches;
  return BL_OK;
}

int bl_solve_k(bl_solver* s, double k1, double k2, const void* start_dev, double* evals,
               double* relres, int32_t* iters, void* evecs_dev) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  return solve_one(s, k1, k2, start_dev, evals, relres, iters, evecs_dev);
}

int bl_solve_path(bl_solver* s, const double* ks, int32_t nk, const void* start_dev,
                  double* evals, double* relres, int32_t* iters, void* evecs_last_dev) {
  if (!s || !ks || nk < 1) return set_error(BL_EINVAL, "invalid path arguments%s");
  const int nev = s->opts.nev;
  int status = BL_OK;
  for (int t = 0; t < nk; ++t) {
    const void* st = (t == 0) ? start_dev : nullptr;
    int it = 0;
    int rc = solve_one(s, ks[2 * t], ks[2 * t + 1], st, evals ? evals + (size_t)t * nev : nullptr,
                       relres ? relres + (size_t)t * nev : nullptr, &it,
                       (t == nk - 1) ? evecs_last_dev : nullptr);
    if (iters) iters[t] = it;
    if (rc != BL_OK && rc != BL_ENOCONV) return rc;
    if (rc != BL_OK && status == BL_OK) status = rc;
  }
  return status;
}

int bl_reset_history(bl_solver* s) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  s->hist_count = 0;
  return BL_OK;
}

int bl_last_residual_history(const bl_solver* s, double* relres, int32_t cap) {
  if (!s || !relres) return set_error(BL_EINVAL, "NULL argument%s");
  const int nev = s->opts.nev;
  const int rows = std::min(cap, s->res_rows);
  std::memcpy(relres, s->res_hist.data(), (size_t)rows * nev * 8);
  return rows;
}

int bl_set_timing(bl_solver* s, int32_t enable) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  if (enable && s->ev_pool.empty()) {
    s->ev_pool.resize(4096);
    for (auto& e : s->ev_pool) HIP_OK(hipEventCreate(&e));
  }
  s->timing = enable != 0;
  s->timed_ms = 0.0;
  s->timed_count = 0;
  s->timed_cols = 0;
  s->ev_used = 0;
  return BL_OK;
}

int bl_get_timing(const bl_solver* s, double* total_ms, int64_t* launches, int64_t* columns) {
  if (!s || !total_ms || !launches || !columns) return set_error(BL_EINVAL, "NULL argument%s");
  *total_ms = s->timed_ms;
  *launches = s->timed_count;
  *columns = s->timed_cols;
  return BL_OK;
}

int bl_set_k(bl_solver* s, double k1, double k2) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  int rc = setup_k(s, k1, k2);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(s->st));
  return check_hip(s);
}


int bl_apply(bl_solver* s, int32_t op, int32_t level, int32_t prec, int32_t ncols, const void* x,
             const void* y, void* out) {
  if (!s || !x || !out || ncols < 1) return set_error(BL_EINVAL, "invalid apply arguments%s");
  if (!s->kset) return set_error(BL_ESTATE, "call bl_set_k first%s");
  if (prec != 0 && prec != 1) return set_error(BL_EINVAL, "prec must be 0 or 1%s");
  int rc = prec ? apply_t<float>(s, op, level, ncols, x, y, out) : apply_t<double>(s, op, level, ncols, x, y, out);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(s->st));
  return check_hip(s);
}

int bl_gram(bl_solver* s, const void* X, int32_t q, const void* W, int32_t r, int64_t len,
            double* out) {
  if (!s || !X || !W || !out || q < 1 || r < 1 || len < 1) return set_error(BL_EINVAL, "invalid gram arguments%s");
  double *part = nullptr, *res = nullptr;
  const int nb = gram_blocks(len);
  const int64_t cap = (int64_t)nb * q * r * 2;
  HIP_OK(hipMalloc(&part, cap * 8));
  HIP_OK(hipMalloc(&res, (size_t)q * r * 2 * 8));
  gram(static_cast<const double*>(X), q, static_cast<const double*>(W), r, len, part, cap, res, s->st);
  hipError_t e = hipMemcpyAsync(out, res, (size_t)q * r * 2 * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  (void)hipFree(part);
  (void)hipFree(res);
  if (e != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e));
  return check_hip(s);
}

int bl_ritz_small(bl_solver* s, const double* G, const double* H, int32_t q, int32_t want,
                  double zero_thr, double* theta, double* Y) {
  if (!s || !G || !H || !theta || !Y || q < 1 || q > 255 || want < 1 || want > q)
    return set_error(BL_EINVAL, "invalid ritz arguments%s");
  double *dG, *dH, *dW, *dY, *dT;
  int* dc;
  const size_t m2 = (size_t)q * q * 2 * 8;
  HIP_OK(hipMalloc(&dG, m2));
  HIP_OK(hipMalloc(&dH, m2));
  HIP_OK(hipMalloc(&dW, ritz_small_work_doubles(q) * 8));
  HIP_OK(hipMalloc(&dY, (size_t)q * want * 2 * 8));
  HIP_OK(hipMalloc(&dT, (size_t)want * 8));
  HIP_OK(hipMalloc(&dc, sizeof(int)));
  HIP_OK(hipMemcpyAsync(dG, G, m2, hipMemcpyHostToDevice, s->st));
  HIP_OK(hipMemcpyAsync(dH, H, m2, hipMemcpyHostToDevice, s->st));
  ritz_small(dG, dH, q, 0, want, zero_thr, kDropRel, dW, dY, dT, dc, s->st);
  int cnt = 0;
  hipError_t e = hipMemcpyAsync(Y, dY, (size_t)q * want * 2 * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(theta, dT, (size_t)want * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(&cnt, dc, sizeof(int), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  (void)hipFree(dG);
  (void)hipFree(dH);
  (void)hipFree(dW);
  (void)hipFree(dY);
  (void)hipFree(dT);
  (void)hipFree(dc);
  if (e != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e));
  int rc = check_hip(s);
  return rc ? rc : cnt;
}

}  // extern "C"
