// Host side of the MI355X Bloch-Maxwell eigensolver engine: multigrid hierarchy, V-cycles,
// null-space projection, Ritz step, preconditioned block inverse iteration and
// Rayleigh-quotient extrapolation across Bloch parameters, for a batch of problem slots.
// Every numerical step runs in the gfx950 kernels of stencils.hip, dense.hip and ritz.hip;
// the host sequences launches on the engine's stream and reads back, once per round, the
// residual norms that decide convergence.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

namespace bl {

namespace {

// Ritz step: basis directions whose squared M-distance from the previously kept ones is
// below this fraction of their squared M-norm are dropped as numerically dependent.
constexpr double kDropRel = 1e-10;

thread_local char g_errbuf[512];

#define HIP_OK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e_)); \
  } while (0)

template <typename T> struct PrecOf;
template <> struct PrecOf<double> { static constexpr int v = 0; };
template <> struct PrecOf<float> { static constexpr int v = 1; };

template <typename T>
View<const T> cv(View<T> v) { return View<const T>{v.p, v.cps, v.off}; }

}  // namespace

const char* last_error_message() { return g_errbuf; }

int set_error(int code, const char* fmt, const char* detail) {
  std::snprintf(g_errbuf, sizeof(g_errbuf), fmt, detail);
  return code;
}

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

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

void fill_defaults(bl_opts* o) {
  if (o->max_iter == 0) o->max_iter = 200;
  if (o->coarsest_min <= 0) o->coarsest_min = 8;
  if (o->nodal_cycles <= 0) o->nodal_cycles = 2;
  if (o->extrap_depth <= 0) o->extrap_depth = 3;
  if (!(o->tol > 0)) o->tol = 1e-8;
  if (!(o->zero_rel > 0)) o->zero_rel = 1e-2;
  if (o->engine_streams == 0) o->engine_streams = 3;
}

int validate_opts(const bl_opts* o) {
  if (o->nev < 1 || o->nthrow < 0) return set_error(BL_EINVAL, "nev >= 1 and nthrow >= 0 required%s");
  const int p = o->nev + o->nthrow;
  if (p > 80) return set_error(BL_EINVAL, "nev + nthrow must be <= 80%s");
  if (o->max_iter < 0 || o->nu_pre < 0 || o->nu_post < 0 || o->nodal_cycles < 1)
    return set_error(BL_EINVAL, "invalid iteration options%s");
  if (o->variant != 0 && o->variant != 1) return set_error(BL_EINVAL, "variant must be 0 (gradient) or 1 (LOBPCG)%s");
  if (o->precision != 0 && o->precision != 1) return set_error(BL_EINVAL, "precision must be 0 or 1%s");
  if (o->extrap_depth < 1 || o->extrap_depth > 3) return set_error(BL_EINVAL, "extrap_depth must be 1..3%s");
  if (o->autotune != 0 && o->autotune != 1) return set_error(BL_EINVAL, "autotune must be 0 or 1%s");
  if (o->coarse_fuse != 0 && o->coarse_fuse != 1) return set_error(BL_EINVAL, "coarse_fuse must be 0 or 1%s");
  if (o->tiled_sweeps < 0 || o->tiled_sweeps > 2) return set_error(BL_EINVAL, "tiled_sweeps must be 0, 1 or 2%s");
  if (o->engine_streams < 1 || o->engine_streams > 16) return set_error(BL_EINVAL, "engine_streams must be 1..16%s");
  if (!(o->tol > 0)) return set_error(BL_EINVAL, "tol must be positive%s");
  if (o->tol_abs != 0 && o->tol_abs != 1) return set_error(BL_EINVAL, "tol_abs must be 0 or 1%s");
  if (o->tol_floor != 0 && o->tol_floor != 1) return set_error(BL_EINVAL, "tol_floor must be 0 or 1%s");
  if (o->nested_start != 0 && o->nested_start != 1) return set_error(BL_EINVAL, "nested_start must be 0 or 1%s");
  if (!(o->nested_tol >= 0) || o->nested_tol >= 1) return set_error(BL_EINVAL, "nested_tol must be in [0, 1)%s");
  if (!(o->lock_rel >= 0) || o->lock_rel > 1) return set_error(BL_EINVAL, "lock_rel must be in [0, 1]%s");
  if (o->throw_precond < 0 || o->reserved_opts != 0) return set_error(BL_EINVAL, "throw_precond must be >= 0%s");
  return BL_OK;
}

int validate_grid(const bl_grid* grid, int p) {
  if (!grid) return set_error(BL_EINVAL, "grid is NULL%s");
  if (grid->n < 2 || grid->m < 2) return set_error(BL_EINVAL, "n and m must be >= 2%s");
  if (!(grid->a > 0) || !(grid->b > 0) || !std::isfinite(grid->a) || !std::isfinite(grid->b))
    return set_error(BL_EINVAL, "a and b must be positive and finite%s");
  if ((int64_t)p > (int64_t)grid->n * grid->m - 1) return set_error(BL_EINVAL, "nev + nthrow must be <= n*m - 1%s");
  return BL_OK;
}

int validate_eps(const double* eps, int64_t count) {
  if (!eps) return set_error(BL_EINVAL, "eps is NULL%s");
  for (int64_t i = 0; i < count; ++i)
    if (!(eps[i] > 0) || !std::isfinite(eps[i])) return set_error(BL_EINVAL, "eps must be positive and finite%s");
  return BL_OK;
}

namespace {

int dalloc(bl_solver* s, void** out, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(BL_ENOMEM, "device allocation failed%s");
  }
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

// Work blocks of the V-cycles (levels below the finest for the edge cycle; the finest
// level's x and b blocks are the correction C and residual R of the iteration).
int ensure_level_buffers(bl_solver* s, int prec, int ecols, int ncols) {
  const int S = s->nslots;
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    if (L.ecap[prec] < ecols) {
      int rc;
      if ((rc = dalloc(s, &L.ex[prec], edge_block_bytes(L.g, ecols * S, prec)))) return rc;
      if ((rc = dalloc(s, &L.eb[prec], edge_block_bytes(L.g, ecols * S, prec)))) return rc;
      if ((rc = dalloc(s, &L.er[prec], edge_block_bytes(L.g, ecols * S, prec)))) return rc;
      L.ecap[prec] = ecols;
    }
    if (L.ncap[prec] < ncols) {
      int rc;
      if ((rc = dalloc(s, &L.nx[prec], nodal_block_bytes(L.g, ncols * S, prec)))) return rc;
      if ((rc = dalloc(s, &L.nb[prec], nodal_block_bytes(L.g, ncols * S, prec)))) return rc;
      if ((rc = dalloc(s, &L.nr[prec], nodal_block_bytes(L.g, ncols * S, prec)))) return rc;
      L.ncap[prec] = ncols;
    }
  }
  if (s->nodal_extra_cap[prec] < ncols) {
    int rc;
    for (int k = 0; k < 2; ++k)
      if ((rc = dalloc(s, &s->nodal_extra[prec][k], nodal_block_bytes(s->lv[0].g, ncols * S, prec)))) return rc;
    s->nodal_extra_cap[prec] = ncols;
  }
  return BL_OK;
}

// Partials and coefficients of the plane-wave deflation for projections of up to `cols`
// columns per slot.
int ensure_pw(bl_solver* s, int cols) {
  if (cols <= s->pw_cap) return BL_OK;
  const size_t nb = (size_t)pw_blocks(s->lv[0].g);
  int rc;
  if ((rc = dalloc_t(s, &s->pw_part, nb * 2 * cols * s->nslots))) return rc;
  if ((rc = dalloc_t(s, &s->pw_coef, (size_t)6 * cols * s->nslots))) return rc;
  s->pw_cap = cols;
  return BL_OK;
}

template <typename T>
const void* kc_inv(const bl_solver* s) { return PrecOf<T>::v ? (const void*)s->kc_inv32 : (const void*)s->kc_inv64; }
template <typename T>
const void* pc_inv(const bl_solver* s) { return PrecOf<T>::v ? (const void*)s->pc_inv32 : (const void*)s->pc_inv64; }

// Blocks of a coarser level inside the slot-major blocks E (p columns per slot) and S (qmax
// per slot): with the column stride per slot scaled by N_0 / N_l (= 4^l) the level-l columns of
// a slot start where its finest-level block starts and stay inside it.
int level_scale(const bl_solver* s, int lev) { return (int)(s->lv[0].g.ne / s->lv[lev].g.ne); }

// ---- slot lists -------------------------------------------------------------------------
// Device list for a launch over `v`; null when v is 0, 1, ..., |v|-1 (the kernels then use
// the launch index itself).
const int* slot_list(bl_solver* s, const std::vector<int>& v) {
  bool ident = true;
  for (size_t i = 0; i < v.size(); ++i) ident = ident && v[i] == (int)i;
  if (ident) return nullptr;
  if (s->lists_used >= kMaxLists) {
    // every list in the ring may still be read by queued kernels: drain the stream first
    (void)hipStreamSynchronize(s->st);
    s->lists_used = 0;
  }
  int* h = s->lists_h + (size_t)s->lists_used * s->nslots;
  int* d = s->lists_d + (size_t)s->lists_used * s->nslots;
  ++s->lists_used;
  std::memcpy(h, v.data(), v.size() * sizeof(int));
  (void)hipMemcpyAsync(d, h, v.size() * sizeof(int), hipMemcpyHostToDevice, s->st);
  return d;
}
Launch make_launch(bl_solver* s, const std::vector<int>& v, int ncps) {
  return Launch{slot_list(s, v), (int)v.size(), ncps, s->st};
}

// ---- timing of the finest-level smoother (opt-in) ----------------------------------------
void timing_begin(bl_solver* s, int l) {
  if (!s->timing || l != 0) return;
  if (s->ev_used + 2 > (int)s->ev_pool.size()) return;
  (void)hipEventRecord(s->ev_pool[s->ev_used], s->st);
}
void timing_end(bl_solver* s, int l, int ncols, double bytes) {
  if (!s->timing || l != 0) return;
  if (s->ev_used + 2 > (int)s->ev_pool.size()) return;
  (void)hipEventRecord(s->ev_pool[s->ev_used + 1], s->st);
  s->ev_used += 2;
  s->timed_cols += ncols;
  s->timed_bytes += bytes;
}
// Algorithmic HBM bytes of one smoother launch over `ncols` columns of `nact` slots: a tiled
// sweep reads b (and x unless it starts from zero) and writes x once; a colour pass reads x
// and half of b and writes half of x.  Per slot: the cell coefficients and the patch
// inverses (kPatchW per node) once per sweep, a quarter of the inverses per colour pass.
// extra: further vectors per column, in units of one fine edge vector (a folded restriction
// writes and a folded prolongation reads a coarse vector, a quarter of one)
double smooth_bytes(const Geo& g, size_t elem, bool sweep, bool zero_start, int ncols, int nact,
                    double extra = 0.0) {
  const double vec = 2.0 * (double)g.ne * (double)elem;
  if (sweep) return ncols * vec * ((zero_start ? 2.0 : 3.0) + extra) + nact * (double)g.nm * elem * (1.0 + kPatchW);
  return ncols * vec * 2.0 + nact * (double)g.nm * elem * (1.0 + kPatchW / 4.0);
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

// ---- fused coarse levels --------------------------------------------------------------------
CoarseCycle coarse_cycle(const bl_solver* s, int first, const void* inv, int64_t nc) {
  CoarseCycle C{};
  C.nlev = (int)s->lv.size() - first;
  C.nu_pre = s->opts.nu_pre;
  C.nu_post = s->opts.nu_post;
  C.nc = nc;
  C.inv = inv;
  C.ns = s->ns;
  for (int i = 0; i < C.nlev; ++i) {
    const Level& L = s->lv[first + i];
    C.L[i] = CoarseLevel{L.g, L.T4, L.kappa64, L.kappa32, L.sinv64, L.sinv32};
  }
  return C;
}

// First level from which the rest of a V-cycle fits one workgroup's LDS (at least two
// levels, at most 64 x 64 nodes on the first, at most kMaxFused levels), or -1.
int plan_fusion(const bl_solver* s, bool edge, size_t elem) {
  if (!s->opts.coarse_fuse) return -1;
  const int nl = (int)s->lv.size();
  const size_t cap = std::min<size_t>(fused_lds_limit(), 144 * 1024);
  int best = -1;
  for (int f = nl - 2; f >= 0 && nl - f <= kMaxFused; --f) {
    if (s->lv[f].g.nm > 4096) break;
    const CoarseCycle C = coarse_cycle(s, f, nullptr, edge ? s->nce : s->ncn);
    if (fused_lds_bytes(C, edge, elem) > cap) break;
    best = f;
  }
  return best;
}

// ---- edge V-cycle for K = A + mu M with zero initial guess: x = V(b) ---------------------
template <typename T>
void vcycle_edge(bl_solver* s, int l, View<const T> b, View<T> x, const Launch& L) {
  const int pr = PrecOf<T>::v;
  Level& lv = s->lv[l];
  const int nl = (int)s->lv.size();
  if (l == nl - 1) {
    dense_apply<T>(kc_inv<T>(s), s->nce, b, x, L);
    s->launches += 1;
    return;
  }
  if (l == s->fuse_edge[pr]) {
    edge_vcycle_fused<T>(b, x, coarse_cycle(s, l, kc_inv<T>(s), s->nce), s->ph_d, s->mu_d, L);
    s->launches += 1;
    return;
  }
  // Tiled sweeps never update in place: they alternate between x and the level's residual
  // block r (free outside the residual/restriction step), arranged so that the last sweep
  // of each smoothing phase writes x; the prolongation then writes x + Pr xc into the first
  // post-sweep's input.
  const bool tiled = s->opts.tiled_sweeps != 0;
  const int ncols = L.nact * L.ncps;
  const int npre = s->opts.nu_pre, npost = s->opts.nu_post;
  View<T> r = view(static_cast<T*>(lv.er[pr]), lv.ecap[pr]);
  if (s->opts.tiled_sweeps == 2 && npre > 0 && npost > 0 && edge_sweep_restricts(sizeof(T))) {
    // transfers folded into the sweeps, as in the nodal cycle (x and r alternate as sweep
    // buffers; the pre-smoothed iterate lands in E so that the last post-sweep writes x)
    Level& C = s->lv[l + 1];
    View<T> bc = view(static_cast<T*>(C.eb[pr]), C.ecap[pr]);
    View<T> xc = view(static_cast<T*>(C.ex[pr]), C.ecap[pr]);
    const View<T> E = (npost % 2 == 1) ? r : x, F = (npost % 2 == 1) ? x : r;
    View<T> prev = E;
    for (int it = 0; it < npre; ++it) {
      const View<T> dst = ((npre - 1 - it) % 2 == 0) ? E : F;
      SweepFuse<T> fz;
      if (it == npre - 1) {
        fz.bc = bc;
        fz.gc = C.g;
      }
      timing_begin(s, l);
      edge_sweep<T>(cv(prev), dst, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4,
                    false, it == 0, s->tune_sweep[0], L, fz);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), true, it == 0, ncols, L.nact, fz.bc.p ? 0.25 : 0.0));
      prev = dst;
    }
    vcycle_edge<T>(s, l + 1, cv(bc), xc, L);
    for (int it = 0; it < npost; ++it) {
      const View<T> dst = ((npost - 1 - it) % 2 == 0) ? x : r;
      SweepFuse<T> fz;
      if (it == 0) {
        fz.xc = cv(xc);
        fz.gc = C.g;
      }
      timing_begin(s, l);
      edge_sweep<T>(cv(prev), dst, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4,
                    true, false, s->tune_sweep[0], L, fz);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), true, false, ncols, L.nact, it == 0 ? 0.25 : 0.0));
      prev = dst;
    }
    s->launches += npre + npost;
    return;
  }
  int nl_launch = 0;
  if (!tiled || npre == 0) {
    zero_cols<T>(x, lv.g.ne, L);
    nl_launch += 1;
  }
  for (int it = 0; it < npre; ++it) {
    if (tiled) {
      View<T> src = ((npre - it) % 2 == 0) ? x : r;   // the previous sweep's output
      View<T> dst = ((npre - 1 - it) % 2 == 0) ? x : r;
      timing_begin(s, l);
      edge_sweep<T>(cv(src), dst, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4,
                    false, it == 0, s->tune_sweep[0], L);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), true, it == 0, ncols, L.nact));
      nl_launch += 1;
      continue;
    }
    for (int c = 0; c < 4; ++c) {
      timing_begin(s, l);
      edge_gs<T>(x, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4, c, s->tune_edge, L);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), false, false, ncols, L.nact));
    }
    nl_launch += 4;
  }
  edge_apply<T, T>(EM_RESID_K, cv(x), b, r, lv.kappa64, lv.kappa32, nullptr, 0, lv.g, s->ph_d, s->mu_d, L, nullptr, nullptr);
  Level& C = s->lv[l + 1];
  View<T> bc = view(static_cast<T*>(C.eb[pr]), C.ecap[pr]);
  View<T> xc = view(static_cast<T*>(C.ex[pr]), C.ecap[pr]);
  edge_restrict<T>(cv(r), lv.g, bc, C.g, s->ph_d, L);
  vcycle_edge<T>(s, l + 1, cv(bc), xc, L);
  if (tiled && npost > 0) {
    View<T> cur = (npost % 2 == 1) ? r : x;
    edge_prolong_to<T>(cv(xc), C.g, cv(x), cur, lv.g, s->ph_d, L);
    for (int it = 0; it < npost; ++it) {
      View<T> dst = (cur.p == x.p && cur.off == x.off && cur.cps == x.cps) ? r : x;
      timing_begin(s, l);
      edge_sweep<T>(cv(cur), dst, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4,
                    true, false, s->tune_sweep[0], L);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), true, false, ncols, L.nact));
      cur = dst;
      nl_launch += 1;
    }
    s->launches += 3 + nl_launch;
    return;
  }
  edge_prolong_add<T>(cv(xc), C.g, x, lv.g, s->ph_d, L);
  for (int it = 0; it < npost; ++it) {
    for (int c = 3; c >= 0; --c) {
      timing_begin(s, l);
      edge_gs<T>(x, b, lv.kappa64, lv.kappa32, lv.sinv64, lv.sinv32, lv.g, s->ph_d, s->mu_d, lv.T4, c, s->tune_edge, L);
      timing_end(s, l, ncols, smooth_bytes(lv.g, sizeof(T), false, false, ncols, L.nact));
    }
    nl_launch += 4;
  }
  s->launches += 3 + nl_launch;
}

// ---- nodal V-cycle for P = L^* M L ----------------------------------------------------------
// x = V(b); with add_to, a cycle that can fold the update into its last sweep writes
// *add_to + V(b) to *add_to instead (x is then not written) and returns true.
template <typename T>
bool vcycle_nodal(bl_solver* s, int l, View<const T> b, View<T> x, const Launch& L, const View<T>* add_to = nullptr,
                  const View<T>* res_out = nullptr, bool* res_done = nullptr) {
  if (res_done) *res_done = false;
  const int pr = PrecOf<T>::v;
  Level& lv = s->lv[l];
  const int nl = (int)s->lv.size();
  if (l == nl - 1) {
    dense_apply<T>(pc_inv<T>(s), s->ncn, b, x, L);
    s->launches += 1;
    return false;
  }
  if (l == s->fuse_nodal[pr]) {
    nodal_vcycle_fused<T>(b, x, coarse_cycle(s, l, pc_inv<T>(s), s->ncn), s->ph_d, L);
    s->launches += 1;
    return false;
  }
  // tiled sweeps alternate between x and the residual block r, as in the edge cycle
  const bool tiled = s->opts.tiled_sweeps != 0;
  const int npre = s->opts.nu_pre, npost = s->opts.nu_post;
  View<T> r = view(static_cast<T*>(lv.nr[pr]), lv.ncap[pr]);
  if (s->opts.tiled_sweeps == 2 && npre > 0 && npost > 0) {
    // Transfers folded into the sweeps: the last pre-sweep also restricts its residual to the
    // coarse right-hand side, the first post-sweep starts from its input plus the prolongated
    // coarse correction.  No residual block is stored: x and r only alternate as sweep
    // buffers, the pre-smoothed iterate landing in E so that the last post-sweep writes x.
    Level& C = s->lv[l + 1];
    View<T> bc = view(static_cast<T*>(C.nb[pr]), C.ncap[pr]);
    View<T> xc = view(static_cast<T*>(C.nx[pr]), C.ncap[pr]);
    const View<T> E = (npost % 2 == 1) ? r : x, F = (npost % 2 == 1) ? x : r;
    View<T> prev = E;
    for (int it = 0; it < npre; ++it) {
      const View<T> dst = ((npre - 1 - it) % 2 == 0) ? E : F;
      SweepFuse<T> fz;
      if (it == npre - 1) {
        fz.bc = bc;
        fz.gc = C.g;
      }
      nodal_sweep<T>(cv(prev), dst, b, lv.g, s->ph_d, s->ns, false, it == 0, s->tune_sweep[1], L, fz);
      prev = dst;
    }
    vcycle_nodal<T>(s, l + 1, cv(bc), xc, L);
    for (int it = 0; it < npost; ++it) {
      View<T> dst = ((npost - 1 - it) % 2 == 0) ? x : r;
      SweepFuse<T> fz;
      if (it == 0) {
        fz.xc = cv(xc);
        fz.gc = C.g;
      }
      if (it == npost - 1 && add_to) {
        dst = *add_to;
        fz.base = cv(*add_to);
      }
      if (it == npost - 1 && res_out && !add_to) {   // the residual b - P x of the result
        fz.res = *res_out;
        if (res_done) *res_done = true;
      }
      nodal_sweep<T>(cv(prev), dst, b, lv.g, s->ph_d, s->ns, true, false, s->tune_sweep[1], L, fz);
      prev = dst;
    }
    s->launches += npre + npost;
    return add_to != nullptr;
  }
  int nl_launch = 0;
  if (!tiled || npre == 0) {
    zero_cols<T>(x, lv.g.nm, L);
    nl_launch += 1;
  }
  for (int it = 0; it < npre; ++it) {
    if (tiled) {
      View<T> src = ((npre - it) % 2 == 0) ? x : r;
      View<T> dst = ((npre - 1 - it) % 2 == 0) ? x : r;
      nodal_sweep<T>(cv(src), dst, b, lv.g, s->ph_d, s->ns, false, it == 0, s->tune_sweep[1], L);
      nl_launch += 1;
    } else {
      for (int c = 0; c < 4; ++c) nodal_gs<T>(x, b, lv.g, s->ph_d, s->ns, c, s->tune_nodal, L);
      nl_launch += 4;
    }
  }
  nodal_apply<T>(cv(x), b, r, lv.g, s->ph_d, s->ns, true, L);
  Level& C = s->lv[l + 1];
  View<T> bc = view(static_cast<T*>(C.nb[pr]), C.ncap[pr]);
  View<T> xc = view(static_cast<T*>(C.nx[pr]), C.ncap[pr]);
  nodal_restrict<T>(cv(r), lv.g, bc, C.g, s->ph_d, L);
  vcycle_nodal<T>(s, l + 1, cv(bc), xc, L);
  if (tiled && npost > 0) {
    View<T> cur = (npost % 2 == 1) ? r : x;
    nodal_prolong_to<T>(cv(xc), C.g, cv(x), cur, lv.g, s->ph_d, L);
    for (int it = 0; it < npost; ++it) {
      View<T> dst = (cur.p == x.p && cur.off == x.off && cur.cps == x.cps) ? r : x;
      nodal_sweep<T>(cv(cur), dst, b, lv.g, s->ph_d, s->ns, true, false, s->tune_sweep[1], L);
      cur = dst;
      nl_launch += 1;
    }
  } else {
    nodal_prolong_add<T>(cv(xc), C.g, x, lv.g, s->ph_d, L);
    for (int it = 0; it < npost; ++it) {
      for (int c = 3; c >= 0; --c) nodal_gs<T>(x, b, lv.g, s->ph_d, s->ns, c, s->tune_nodal, L);
      nl_launch += 4;
    }
  }
  s->launches += 3 + nl_launch;
  return false;
}

// phi ~ P^{-1} b by `cycles` V-cycles; b and phi must not be level-0 work blocks of the
// nodal cycle (nr) or the multi-cycle work blocks.
template <typename T>
void nodal_solve(bl_solver* s, View<const T> b, View<T> phi, const Launch& L, int cycles, int lev = 0) {
  const int pr = PrecOf<T>::v;
  View<T> res = view(static_cast<T*>(s->nodal_extra[pr][0]), s->nodal_extra_cap[pr]);
  View<T> cor = view(static_cast<T*>(s->nodal_extra[pr][1]), s->nodal_extra_cap[pr]);
  // the first cycle's last sweep also forms the residual the second cycle starts from
  bool have_res = false;
  vcycle_nodal<T>(s, lev, b, phi, L, nullptr, cycles > 1 ? &res : nullptr, &have_res);
  const Geo& g = s->lv[lev].g;
  for (int c = 1; c < cycles; ++c) {
    if (!have_res) {
      nodal_apply<T>(cv(phi), b, res, g, s->ph_d, s->ns, true, L);
      s->launches += 1;
    }
    have_res = false;
    if (!vcycle_nodal<T>(s, lev, cv(res), cor, L, &phi)) {
      axpy<T>(phi, cv(cor), g.nm, L);
      s->launches += 1;
    }
  }
}

struct Group {
  const void* ptr;
  int cps;
  int off;
  int prec;
  int cols;
};

// Null-space elimination (Section 4) of the column groups into `out` (FP64 edge view):
// out = U - L Phi with Phi from nodal V-cycles for P Phi = L^* M U; at k = 0 also the
// constant edge fields are removed (the slots of Lg).  Nodal arithmetic in TN.
template <typename TN>
int project_groups(bl_solver* s, const std::vector<Group>& groups, View<double> out,
                   const std::vector<int>& slots, const std::vector<int>& gslots, int lev) {
  const int pr = PrecOf<TN>::v;
  int total = 0;
  for (auto& g : groups) total += g.cols;
  int rc = ensure_level_buffers(s, pr, std::max(s->lv[0].ecap[pr], s->p), std::max(total, s->qmax));
  if (rc) return rc;
  if ((rc = ensure_pw(s, total))) return rc;
  const Geo& g0 = s->lv[lev].g;
  Launch L = make_launch(s, slots, 0);
  const int nc = s->lv[lev].ncap[pr];
  // right-hand side and solution of the nodal solve: the level's nodal blocks nb and nx,
  // which the V-cycle from that level does not use (it works in nr and the coarser levels)
  TN* b0 = static_cast<TN*>(s->lv[lev].nb[pr]);
  TN* phi = static_cast<TN*>(s->lv[lev].nx[pr]);
  const PWDefl pw{s->pw_tab, s->pw_d, s->pw_part, s->pw_coef, 2 * (int64_t)(g0.n + g0.m), total, 0, pw_blocks(g0)};
  int off = 0;
  for (auto& gr : groups) {
    Launch Lg = L;
    Lg.ncps = gr.cols;
    PWDefl pg = pw;
    pg.off = off;
    if (gr.prec == 0) lhm<double, TN>(View<const double>{static_cast<const double*>(gr.ptr), gr.cps, gr.off}, view(b0, nc, off), g0, s->ph_d, Lg, &pg);
    else lhm<float, TN>(View<const float>{static_cast<const float*>(gr.ptr), gr.cps, gr.off}, view(b0, nc, off), g0, s->ph_d, Lg, &pg);
    off += gr.cols;
    s->launches += 1;
  }
  Launch Lt = L;
  Lt.ncps = total;
  // plane-wave deflation: b <- b - w (w^* b)/nm, the cycles on the complement, then the
  // exact plane-wave coefficient added back through the lift
  pw_reduce(pw, 0, apply_blocks(g0), Lt);   // k_lhm: one partial per point tile
  pw_rhs<TN>(view(b0, nc), g0, pw, Lt);
  nodal_solve<TN>(s, cview(b0, nc), view(phi, nc), Lt, std::max(1, s->opts.nodal_cycles), lev);
  const int nd = pw_dot<TN>(cview(phi, nc), g0, pw, Lt);
  pw_reduce(pw, 1, nd, Lt);
  s->launches += 4;
  off = 0;
  for (auto& gr : groups) {
    Launch Lg = L;
    Lg.ncps = gr.cols;
    PWDefl pg = pw;
    pg.off = off;
    View<double> dst{out.p, out.cps, out.off + off};
    if (gr.prec == 0) lift_sub<double, TN, double>(View<const double>{static_cast<const double*>(gr.ptr), gr.cps, gr.off}, cview(phi, nc, off), dst, g0, s->ph_d, Lg, &pg);
    else lift_sub<float, TN, double>(View<const float>{static_cast<const float*>(gr.ptr), gr.cps, gr.off}, cview(phi, nc, off), dst, g0, s->ph_d, Lg, &pg);
    off += gr.cols;
    s->launches += 1;
  }
  if (!gslots.empty()) {
    Launch Lgam = make_launch(s, gslots, total);
    gamma_deflate(out, g0, s->mean_scratch, Lgam);
    s->launches += 3;
  }
  return BL_OK;
}

int project(bl_solver* s, const std::vector<Group>& groups, View<double> out,
            const std::vector<int>& slots, int lev = 0) {
  std::vector<int> gs;
  for (int sl : slots)
    if (s->slot[sl].gamma) gs.push_back(sl);
  if (s->opts.precision) return project_groups<float>(s, groups, out, slots, gs, lev);
  return project_groups<double>(s, groups, out, slots, gs, lev);
}

}  // namespace

// Output tile of the Rayleigh-Ritz products: the 48- or 64-wide tiling that pads q least.
int rr_tile(int q) {
  const int64_t p3 = (int64_t)((q + 47) / 48) * 48, p4 = (int64_t)((q + 63) / 64) * 64;
  return p4 < p3 ? 4 : 3;
}

namespace {

// Ritz step on the q columns of S (FP64) of the listed slots: G = S^* M S, H = S^* A S,
// generalised eigenproblem, E <- S Y for the p smallest Ritz values above the slot's
// zero threshold (zthr_d, or none), Ritz values into lam_d.
int ritz_step(bl_solver* s, const std::vector<int>& slots, int q, int nfix, bool use_zthr, int lev = 0) {
  const Level& L0 = s->lv[lev];
  const Geo& g = L0.g;
  const int sc = level_scale(s, lev);
  Launch L = make_launch(s, slots, q);
  View<double> Sv = view(s->Sb, s->qmax * sc);
  const int tile = (q == 2 * s->p && s->tune_rr) ? s->tune_rr : rr_tile(q);
  if (rr_gram(cv(Sv), q, L0.kappa64, g, s->ph_d, s->gram_partial, s->gram_cap, s->Gm, s->Hm, tile, L) != 0)
    return set_error(BL_EINVAL, "Gram scratch too small%s");
  ritz_small(s->Gm, s->Hm, q, nfix, s->p, use_zthr ? s->zthr_d : nullptr, kDropRel, s->ritz_work,
             s->ritz_stride, s->Yd, s->lam_d, s->count_d, L);
  block_combine(cv(Sv), q, s->Yd, s->p, g.ne, view(s->E, s->p * sc), L);
  s->launches += 4;
  if (s->debug && !slots.empty()) {
    double sw[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double* base = s->ritz_work + (size_t)slots[0] * s->ritz_stride;
    (void)hipMemcpyAsync(sw, base + 10 * q * q + 8 * q, 11 * 8, hipMemcpyDeviceToHost, s->st);
    (void)hipStreamSynchronize(s->st);
    std::fprintf(stderr, "bloch: ritz q=%d slots=%zu rank %.0f  shader MHz %.0f  phase us: chol %.1f basis %.1f hprime %.1f tridiag %.1f bisect %.1f invit %.1f back %.1f\n",
                 q, slots.size(), sw[0], (sw[9] - sw[8]) / ((sw[7] - sw[1]) * 0.01), (sw[2] - sw[1]) * 0.01, (sw[3] - sw[2]) * 0.01, (sw[4] - sw[3]) * 0.01,
                 (sw[5] - sw[4]) * 0.01, (sw[10] - sw[5]) * 0.01, (sw[6] - sw[10]) * 0.01, (sw[7] - sw[6]) * 0.01);
  }
  return BL_OK;
}

// Coarsest-level direct solvers of the listed slots for their current phases: the coarse
// operators are probed with unit vectors, assembled, (at k = 0 the nodal one is made
// definite by the constant rank-one term) and inverted.
void setup_coarse(bl_solver* s, const std::vector<int>& slots) {
  Level& C = s->lv.back();
  std::vector<int> gs;
  for (int sl : slots)
    if (s->slot[sl].gamma) gs.push_back(sl);
  // launches over nact * n columns are split so that grid.y stays below 65536
  const int per_e = std::max<int>(1, (int)(65535 / s->nce));
  for (size_t c0 = 0; c0 < slots.size(); c0 += per_e) {
    std::vector<int> part(slots.begin() + c0, slots.begin() + std::min(slots.size(), c0 + per_e));
    Launch L = make_launch(s, part, (int)s->nce);
    edge_apply<double, double>(EM_K, View<const double>{s->probe_e, 0, 0}, View<const double>{nullptr, 0, 0},
                               view(s->probe_out, (int)s->nce), C.kappa64, C.kappa32, nullptr, 0, C.g,
                               s->ph_d, s->mu_d, L, nullptr, nullptr);
    planar_to_matrix(s->probe_out, s->nce, s->kc_inv64, L);
    L.ncps = (int)s->ncn;
    nodal_apply<double>(View<const double>{s->probe_n, 0, 0}, View<const double>{nullptr, 0, 0},
                        view(s->probe_out, (int)s->ncn), C.g, s->ph_d, s->ns, false, L);
    planar_to_matrix(s->probe_out, s->ncn, s->pc_inv64, L);
  }
  Launch L = make_launch(s, slots, 0);
  if (!gs.empty()) add_constant_rank_one(s->pc_inv64, s->ncn, s->ns.c0, make_launch(s, gs, 0));
  invert_hpd(s->kc_inv64, s->nce, L);
  matrix_to_float(s->kc_inv64, s->kc_inv32, 2 * s->nce * s->nce, L);
  invert_hpd(s->pc_inv64, s->ncn, L);
  matrix_to_float(s->pc_inv64, s->pc_inv32, 2 * s->ncn * s->ncn, L);
  s->launches += 10;
}

// Per-slot phases and zero thresholds to the device through the pinned staging area (it is
// rewritten only after the stream has been synchronised).
int upload_slot_params(bl_solver* s) {
  char* h = static_cast<char*>(s->param_h);
  const size_t np = s->ph_h.size() * sizeof(Phase);
  const size_t nz = s->zthr_h.size() * 8;
  const size_t nw = s->pw_h.size() * sizeof(PlaneWave);
  std::memcpy(h, s->ph_h.data(), np);
  std::memcpy(h + np, s->zthr_h.data(), nz);
  std::memcpy(h + np + nz, s->pw_h.data(), nw);
  HIP_OK(hipMemcpyAsync(s->ph_d, h, np, hipMemcpyHostToDevice, s->st));
  HIP_OK(hipMemcpyAsync(s->zthr_d, h + np, nz, hipMemcpyHostToDevice, s->st));
  HIP_OK(hipMemcpyAsync(s->pw_d, h + np + nz, nw, hipMemcpyHostToDevice, s->st));
  pw_tables(s->pw_d, s->pw_tab, 2 * (int64_t)(s->grid.n + s->grid.m), s->grid.n, s->grid.m, s->nslots, s->st);
  s->launches += 1;
  return BL_OK;
}

// Plane-wave deflation parameters for k (PlaneWave): t = k' h with k' = k - 2 pi (p/a, r/b),
// p, r the nearest integers (ties to even), and lambda_w of P in the cancellation-free form
// 4 s1 (h2/h1)(1 - 2/3 s2) + 4 s2 (h1/h2)(1 - 2/3 s1), s_i = sin^2(t_i / 2).
PlaneWave plane_wave_params(const Geo& g, double a, double b, double k1, double k2, bool gamma) {
  PlaneWave q{};
  q.inm = 1.0 / (double)g.nm;
  if (gamma) return q;
  const double tau = 2.0 * M_PI;
  const double r1 = k1 - tau * std::nearbyint(k1 * a / tau) / a;
  const double r2 = k2 - tau * std::nearbyint(k2 * b / tau) / b;
  q.t1 = r1 * g.h1;
  q.t2 = r2 * g.h2;
  const double h1s = std::sin(0.5 * q.t1), h2s = std::sin(0.5 * q.t2);
  const double s1 = h1s * h1s, s2 = h2s * h2s;
  q.exr = -2.0 * s1;
  q.exi = std::sin(q.t1);
  q.eyr = -2.0 * s2;
  q.eyi = std::sin(q.t2);
  const double lw = 4.0 * s1 * g.mx * (1.0 - 2.0 / 3.0 * s2) + 4.0 * s2 * g.my * (1.0 - 2.0 / 3.0 * s1);
  q.ilw = lw > 0 ? 1.0 / ((double)g.nm * lw) : 0.0;
  return q;
}

// Phases of slot `sl` for (k1, k2); false for a non-finite parameter.
bool set_phase(bl_solver* s, int sl, double k1, double k2) {
  if (!std::isfinite(k1) || !std::isfinite(k2)) return false;
  SlotState& ss = s->slot[sl];
  ss.gamma = is_gamma(k1, k2, s->grid.a, s->grid.b);
  if (ss.gamma) s->ph_h[sl] = {1.0, 0.0, 1.0, 0.0};
  else s->ph_h[sl] = {std::cos(k1 * s->grid.a), std::sin(k1 * s->grid.a), std::cos(k2 * s->grid.b), std::sin(k2 * s->grid.b)};
  s->pw_h[sl] = plane_wave_params(s->lv[0].g, s->grid.a, s->grid.b, k1, k2, ss.gamma);
  return true;
}

// Permittivity of slot `sl`: kappa on every level, mu, stabilised patch factors.
int load_eps(bl_solver* s, int sl, const std::vector<double>& kappa, double eps_min) {
  // default shift (Section 5 leaves it open): half the first non-zero eigenvalue of the
  // homogeneous cell, or lambda_p / 40 when larger; much smaller shifts amplify the gradient
  // part that the inexact nodal projection leaves faster than the projection removes it
  const double mu = (s->opts.mu > 0)
                        ? s->opts.mu
                        : std::max(homogeneous_lambda(s->grid.n, s->grid.m, s->grid.a, s->grid.b, eps_min, s->p) / kMuDivisor,
                                   homogeneous_lambda(s->grid.n, s->grid.m, s->grid.a, s->grid.b, eps_min, 1) / 2.0);
  s->mu_h[sl] = mu;
  s->slot[sl].mu = mu;
  s->slot[sl].kappa_max = eps_min > 0 ? 1.0 / eps_min : 1.0;
  HIP_OK(hipMemcpyAsync(s->mu_d + sl, &s->mu_h[sl], 8, hipMemcpyHostToDevice, s->st));
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    double* k64 = L.kappa64 + (int64_t)sl * L.g.nm;
    if (l == 0) HIP_OK(hipMemcpyAsync(k64, kappa.data(), kappa.size() * 8, hipMemcpyHostToDevice, s->st));
    else coarsen_kappa(s->lv[l - 1].kappa64 + (int64_t)sl * s->lv[l - 1].g.nm, s->lv[l - 1].g, k64, 1, s->st);
    to_float(k64, L.kappa32 + (int64_t)sl * L.g.nm, L.g.nm, s->st);
    if (l + 1 < s->lv.size())
      patch_setup(k64, L.g, L.Q, L.T4, s->mu_d + sl, L.sinv64 + (int64_t)sl * L.g.nm * kPatchW,
                  L.sinv32 + (int64_t)sl * L.g.nm * kPatchW, 1, s->st);
    s->launches += 3;
  }
  // the host sources (the task's kappa, mu_h[sl]) stay unchanged until the copies have run:
  // both are rewritten only when the slot takes its next task, after a synchronisation
  return BL_OK;
}

int check_hip() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BL_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return BL_OK;
}

// ---- nested iteration for a first Bloch parameter (Section 6) ------------------------------
// The coarsest level's pencil (A_c, M_c) is probed with unit vectors and solved densely for
// its p smallest non-zero eigenpairs (the gradients are its exact zeros and are skipped); the
// block is then prolongated level by level and, on every level between, iterated to the
// relative residual opts.nested_tol with the level as the finest one of its own hierarchy.
// Everything stays on the device in the engine's own buffers: level-l blocks use the slot's
// regions of E and S (level_scale), the V-cycle and nodal blocks of level l are the ones the
// finest-level cycles use below it, and the dense pencil has buffers of its own.

// Buffers of the coarsest pencil (one slot at a time), allocated on the first nested start.
int ensure_nested(bl_solver* s) {
  const int q = (int)s->nce;
  if (s->nst_q >= q) return BL_OK;
  int rc;
  if ((rc = dalloc_t(s, &s->nst_G, (size_t)q * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->nst_H, (size_t)q * q * 2))) return rc;
  if ((rc = dalloc_t(s, &s->nst_Y, (size_t)q * s->p * 2))) return rc;
  if ((rc = dalloc_t(s, &s->nst_work, ritz_small_work_doubles(q)))) return rc;
  s->nst_q = q;
  return BL_OK;
}

// Plane-wave parameters and tables of slot sl for the geometry of level lev (the projection
// on that level deflates its own discrete plane wave).
int plane_wave_level(bl_solver* s, int sl, int lev, double k1, double k2) {
  const Geo& g = s->lv[lev].g;
  s->pw_h[sl] = plane_wave_params(g, s->grid.a, s->grid.b, k1, k2, s->slot[sl].gamma);
  char* h = static_cast<char*>(s->param_h);   // free: its last copies completed at a synchronisation
  std::memcpy(h, &s->pw_h[sl], sizeof(PlaneWave));
  HIP_OK(hipMemcpyAsync(s->pw_d + sl, h, sizeof(PlaneWave), hipMemcpyHostToDevice, s->st));
  const int64_t stride = 2 * (int64_t)(s->grid.n + s->grid.m);
  pw_tables(s->pw_d + sl, s->pw_tab + sl * stride, stride, g.n, g.m, 1, s->st);
  HIP_OK(hipStreamSynchronize(s->st));
  s->launches += 1;
  return BL_OK;
}

// E (level lev + 1) -> E (level lev) of slot sl by the edge prolongation, through S.
void prolong_block(bl_solver* s, int sl, int lev) {
  const int p = s->p;
  const Level& F = s->lv[lev];
  const Level& C = s->lv[lev + 1];
  Launch L = make_launch(s, {sl}, p);
  const View<double> Sf = view(s->Sb, s->qmax * level_scale(s, lev));
  zero_cols<double>(Sf, F.g.ne, L);
  edge_prolong_add<double>(cview(s->E, p * level_scale(s, lev + 1)), C.g, Sf, F.g, s->ph_d, L);
  sub_cols<double>(cv(Sf), View<const double>{nullptr, 0, 0}, view(s->E, p * level_scale(s, lev)), F.g.ne, L);
  s->launches += 3;
}

// Block iteration of slot sl on level lev >= 1 from the block in E to the relative residual
// tol over the first nev pairs (at most max_it iterations); the iterations go to *its.
int iterate_level(bl_solver* s, int sl, int lev, int nev, double tol, int max_it, int* its) {
  const int p = s->p, ip = s->opts.precision, sc = level_scale(s, lev);
  Level& Lv = s->lv[lev];
  const std::vector<int> one{sl};
  const View<const double> none{nullptr, 0, 0};
  int rc;
  if ((rc = project(s, {{s->E, p * sc, 0, 0, p}}, view(s->Sb, s->qmax * sc), one, lev))) return rc;
  if ((rc = ritz_step(s, one, p, 0, false, lev))) return rc;
  for (int it = 0;; ++it) {
    Launch L = make_launch(s, one, p);
    int nblk = 0;
    if (ip)
      edge_apply<double, float>(EM_EIGRES, cview(s->E, p * sc), none, view(static_cast<float*>(Lv.eb[1]), Lv.ecap[1]),
                                Lv.kappa64, Lv.kappa32, s->lam_d, p, Lv.g, s->ph_d, s->mu_d, L, s->partial, &nblk);
    else
      edge_apply<double, double>(EM_EIGRES, cview(s->E, p * sc), none, view(static_cast<double*>(Lv.eb[0]), Lv.ecap[0]),
                                 Lv.kappa64, Lv.kappa32, s->lam_d, p, Lv.g, s->ph_d, s->mu_d, L, s->partial, &nblk);
    reduce_partials(s->partial, nblk, p, 2, s->norms, s->st);
    s->launches += 2;
    HIP_OK(hipMemcpyAsync(s->norms_h, s->norms, s->readback_bytes, hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    s->lists_used = 0;
    if ((rc = check_hip())) return rc;
    if (it == 0 && s->count_h[sl] < p) return set_error(BL_ENOCONV, "nested start: the block lost rank%s");
    const double* lam = s->lam_h + (size_t)sl * p;
    bool conv = true;
    for (int j = 0; j < nev; ++j) {
      const double den = std::fabs(lam[j]) * std::sqrt(s->norms_h[2 * j + 1]);
      conv = conv && den > 0 && std::sqrt(s->norms_h[2 * j]) <= tol * den;
    }
    if (conv || it >= max_it) {
      *its = it;
      return BL_OK;
    }
    if (ip) vcycle_edge<float>(s, lev, cview(static_cast<const float*>(Lv.eb[1]), Lv.ecap[1]), view(static_cast<float*>(Lv.ex[1]), Lv.ecap[1]), L);
    else vcycle_edge<double>(s, lev, cview(static_cast<const double*>(Lv.eb[0]), Lv.ecap[0]), view(static_cast<double*>(Lv.ex[0]), Lv.ecap[0]), L);
    if ((rc = project(s, {{s->E, p * sc, 0, 0, p}, {Lv.ex[ip], Lv.ecap[ip], 0, ip, p}}, view(s->Sb, s->qmax * sc), one, lev)))
      return rc;
    if ((rc = ritz_step(s, one, 2 * p, p, false, lev))) return rc;
  }
}

// The start block of slot sl at (k1, k2) by nested iteration, left in E (finest level); the
// iterations per level (finest first, 0 for the finest and the coarsest) go to its.  The
// slot's phases must be set; on return its plane-wave parameters are those of the finest
// level again.
int nested_start_slot(bl_solver* s, int sl, double k1, double k2, int nev, std::vector<int>& its) {
  const int nl = (int)s->lv.size(), lc = nl - 1, p = s->p;
  its.assign(nl, 0);
  if (nl < 2 || s->nce > kMaxNestedCoarse)
    return set_error(BL_EINVAL, "nested start needs a coarsest level of at most 512 edges%s");
  int rc;
  if ((rc = ensure_nested(s))) return rc;
  SlotState& ss = s->slot[sl];
  const Level& C = s->lv[lc];
  const int q = (int)s->nce;
  // zero threshold of the dense pencil: far above the rounding of its zero eigenvalues
  // (u times the stencil's Gershgorin bound 8 kappa_max (1/h1^2 + 1/h2^2)), far below the
  // smallest non-zero one
  s->zthr_h[sl] = 1e-8 * 8.0 * ss.kappa_max * (1.0 / (C.g.h1 * C.g.h1) + 1.0 / (C.g.h2 * C.g.h2));
  if ((rc = upload_slot_params(s))) return rc;
  setup_coarse(s, {sl});
  // coarsest pencil: columns of A_c and M_c from the unit vectors (shared by every slot, so
  // the output columns are addressed without a slot offset), to row-major matrices
  Launch Lp = make_launch(s, {sl}, q);
  const View<const double> unit{s->probe_e, 0, 0}, none{nullptr, 0, 0};
  const Launch L1{nullptr, 1, 0, s->st};
  edge_apply<double, double>(EM_A, unit, none, View<double>{s->probe_out, 0, 0}, C.kappa64, C.kappa32, nullptr, 0, C.g,
                             s->ph_d, s->mu_d, Lp, nullptr, nullptr);
  planar_to_matrix(s->probe_out, q, s->nst_H, L1);
  edge_apply<double, double>(EM_M, unit, none, View<double>{s->probe_out, 0, 0}, C.kappa64, C.kappa32, nullptr, 0, C.g,
                             s->ph_d, s->mu_d, Lp, nullptr, nullptr);
  planar_to_matrix(s->probe_out, q, s->nst_G, L1);
  ritz_small(s->nst_G, s->nst_H, q, 0, p, s->zthr_d + sl, kDropRel, s->nst_work, 0, s->nst_Y, s->lam_d + (size_t)sl * p,
             s->count_d + sl, L1);
  // E (coarsest level) = the unit vectors combined with the Ritz vectors
  block_combine(unit, q, s->nst_Y, p, C.g.ne, View<double>{s->E + (size_t)sl * p * 2 * s->lv[0].g.ne, p * level_scale(s, lc), 0},
                L1);
  s->launches += 7;
  HIP_OK(hipMemcpyAsync(s->norms_h, s->norms, s->readback_bytes, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  s->lists_used = 0;
  if ((rc = check_hip())) return rc;
  if (s->count_h[sl] < p) return set_error(BL_ENOCONV, "the coarsest mesh has fewer than p non-zero eigenvalues%s");
  const double tol = s->opts.nested_tol > 0 ? s->opts.nested_tol : 1e-2;
  for (int l = lc - 1; l >= 0 && !rc; --l) {
    prolong_block(s, sl, l);
    if (l == 0) break;
    if ((rc = plane_wave_level(s, sl, l, k1, k2))) break;
    rc = iterate_level(s, sl, l, nev, tol, s->opts.max_iter, &its[l]);
  }
  const int rc2 = plane_wave_level(s, sl, 0, k1, k2);
  return rc ? rc : rc2;
}

void end_task(bl_solver* s, int sl, int status, const char* msg) {
  SlotState& ss = s->slot[sl];
  Task* t = ss.task;
  if (t) {
    if (status != BL_OK && t->status == BL_OK) {
      t->status = status;
      t->message = msg ? msg : "";
    }
    t->finished = true;
    s->retired.push_back(t);
    if (sl == 0) {
      s->last_res_hist = t->res_hist;
      s->last_res_rows = t->nev ? (int)(t->res_hist.size() / t->nev) : 0;
    }
  }
  ss.task = nullptr;
  ss.phase = SLOT_FREE;
}

// Point t of slot sl is done (converged or out of iterations): push E onto the history,
// record the results, continue with the next point or end the task.
int retire_point(bl_solver* s, int sl, bool conv, const double* lam, const double* rel) {
  SlotState& ss = s->slot[sl];
  Task* t = ss.task;
  const size_t colb = (size_t)2 * s->lv[0].g.ne * 8;
  const size_t blk = (size_t)s->p * colb;
  const size_t off = (size_t)sl * s->p * 2 * s->lv[0].g.ne;
  if (ss.hist_count >= 2) HIP_OK(hipMemcpyAsync(s->hist[2] + off, s->hist[1] + off, blk, hipMemcpyDeviceToDevice, s->st));
  if (ss.hist_count >= 1) HIP_OK(hipMemcpyAsync(s->hist[1] + off, s->hist[0] + off, blk, hipMemcpyDeviceToDevice, s->st));
  HIP_OK(hipMemcpyAsync(s->hist[0] + off, s->E + off, blk, hipMemcpyDeviceToDevice, s->st));
  ss.hist_count = std::min(3, ss.hist_count + 1);
  ss.hist_lam1 = lam[0];
  const int nev = t->nev;
  const int nk = (int)(t->ks.size() / 2);
  for (int j = 0; j < nev; ++j) {
    t->evals[(size_t)ss.t * nev + j] = lam[j];
    t->relres[(size_t)ss.t * nev + j] = rel[j];
  }
  t->iters[ss.t] = ss.it;
  t->t_points.push_back(now_seconds());
  if (!conv && t->status == BL_OK) {
    t->status = BL_ENOCONV;
    t->message = "max_iter reached";
  }
  t->res_hist = ss.res_rows;
  ss.res_rows.clear();
  if (ss.t == nk - 1 && t->evecs_dev)
    HIP_OK(hipMemcpyAsync(t->evecs_dev, s->E + off, (size_t)nev * colb, hipMemcpyDeviceToDevice, s->st));
  ss.t += 1;
  ss.it = 0;
  if (ss.t < nk) ss.phase = SLOT_START;
  else end_task(s, sl, BL_OK, nullptr);
  return BL_OK;
}

}  // namespace

// =========================================================================================
size_t engine_footprint(const bl_grid* grid, const bl_opts* o, int nslots) {
  const int p = o->nev + o->nthrow;
  const int q = 3 * p;
  auto lv = hierarchy(grid->n, grid->m, o->levels, o->coarsest_min > 0 ? o->coarsest_min : 8);
  const int pr = o->precision ? 1 : 0;
  size_t per = 0, fixed = 0;
  for (size_t l = 0; l < lv.size(); ++l) {
    Geo g = make_geo(lv[l].first, lv[l].second, grid->a, grid->b);
    per += g.nm * (8 + 4) + (l + 1 < lv.size() ? g.nm * 6 * 12 : 0);
    per += edge_block_bytes(g, p, pr) * 3 + nodal_block_bytes(g, q, pr) * 3;
  }
  Geo g0 = make_geo(grid->n, grid->m, grid->a, grid->b);
  const size_t col = (size_t)2 * g0.ne * 8;
  per += col * (p + q + 3 * p);                   // E, S, history
  per += nodal_block_bytes(g0, q, pr) * 2;        // nodal multi-cycle work
  Geo gc = make_geo(lv.back().first, lv.back().second, grid->a, grid->b);
  per += (size_t)gc.ne * gc.ne * 16 * 2 + (size_t)gc.nm * gc.nm * 16 * 2;   // inverses (FP64 + FP32)
  per += (size_t)gc.ne * gc.ne * 16;                                         // probe results
  per += (size_t)rr_partial_blocks(g0) * q * q * 32 + (size_t)10 * q * q * 16;
  per += (size_t)p * ((g0.ne + 255) / 256) * 16;
  per += (size_t)q * pw_blocks(g0) * 16 + (size_t)q * 48 + (size_t)(grid->n + grid->m) * 16 + sizeof(PlaneWave);
  fixed += (size_t)gc.ne * gc.ne * 16 + (size_t)gc.nm * gc.nm * 16;           // probes
  if (o->nested_start)   // the coarsest pencil of the nested start, its Ritz vectors and work
    fixed += (size_t)gc.ne * gc.ne * 32 + (size_t)gc.ne * p * 16 + ritz_small_work_doubles((int)gc.ne) * 8;
  return fixed + per * (size_t)std::max(1, nslots);
}

int engine_create(const bl_grid* grid, const bl_opts* opts, int nslots, hipStream_t st,
                  const double* eps, bl_solver** out) {
  if (!out) return set_error(BL_EINVAL, "out is NULL%s");
  *out = nullptr;
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  int rc = validate_opts(&o);
  if (rc) return rc;
  if ((rc = validate_grid(grid, o.nev + o.nthrow))) return rc;
  if (nslots < 1 || nslots > kMaxSlots) return set_error(BL_EINVAL, "slot count must be 1..256%s");
  if (eps && (rc = validate_eps(eps, (int64_t)grid->n * grid->m))) return rc;
  bl_solver* s = new (std::nothrow) bl_solver();
  if (!s) return set_error(BL_ENOMEM, "host allocation failed%s");
  s->grid = *grid;
  s->opts = o;
  s->st = st;
  s->nslots = nslots;
  s->p = o.nev + o.nthrow;
  s->qmax = 3 * s->p;
  s->debug = std::getenv("BL_DEBUG") != nullptr;
  s->slot.resize(nslots);
  s->ph_h.assign(nslots, Phase{1.0, 0.0, 1.0, 0.0});
  s->pw_h.assign(nslots, PlaneWave{});
  s->mu_h.assign(nslots, 1.0);
  s->zthr_h.assign(nslots, -INFINITY);
  auto fail = [&](int code) {
    engine_destroy(s);
    return code;
  };
  if (hipGetDevice(&s->device) != hipSuccess) return fail(set_error(BL_EHIP, "no HIP device%s"));
  const bl_grid& gr = s->grid;
  auto sizes = hierarchy(gr.n, gr.m, o.levels, o.coarsest_min);
  s->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) s->lv[l].g = make_geo(sizes[l].first, sizes[l].second, gr.a, gr.b);
  const Geo& c = s->lv.back().g;
  s->nce = c.ne;
  s->ncn = c.nm;
  if (s->nce > kMaxCoarse) return fail(set_error(BL_EINVAL, "grid cannot be coarsened to a small enough level%s"));
  if (o.nested_start && (s->nce > kMaxNestedCoarse || s->lv.size() < 2))
    return fail(set_error(BL_EINVAL, "nested_start needs a hierarchy whose coarsest level has at most 512 edges%s"));
  {  // nodal stencil (same on every level: depends on h2/h1 only)
    const double r = s->lv[0].g.mx, q = s->lv[0].g.my;
    s->ns = {(4.0 / 3.0) * (r + q), -(2.0 / 3.0) * r + (1.0 / 3.0) * q, (1.0 / 3.0) * r - (2.0 / 3.0) * q, -(1.0 / 6.0) * (r + q)};
  }
  const int S = nslots;
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    if ((rc = dalloc_t(s, &L.kappa64, L.g.nm * S))) return fail(rc);
    if ((rc = dalloc_t(s, &L.kappa32, L.g.nm * S))) return fail(rc);
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
      if ((rc = dalloc_t(s, &L.sinv64, L.g.nm * kPatchW * S))) return fail(rc);
      if ((rc = dalloc_t(s, &L.sinv32, L.g.nm * kPatchW * S))) return fail(rc);
    }
  }
  const Geo& g0 = s->lv[0].g;
  const int p = s->p, q = s->qmax;
  const size_t col = (size_t)2 * g0.ne;
  if ((rc = dalloc_t(s, &s->ph_d, S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->mu_d, S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->zthr_d, S))) return fail(rc);
  for (auto& q : s->pw_h) q.inm = 1.0 / (double)g0.nm;
  if ((rc = dalloc_t(s, &s->pw_d, S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->pw_tab, (size_t)2 * (gr.n + gr.m) * S))) return fail(rc);
  if ((rc = ensure_pw(s, q))) return fail(rc);
  if ((rc = dalloc_t(s, &s->E, col * p * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->Sb, col * q * S))) return fail(rc);
  for (int h = 0; h < 3; ++h)
    if ((rc = dalloc_t(s, &s->hist[h], col * p * S))) return fail(rc);
  if (o.variant == 1) {
    if ((rc = dalloc_t(s, &s->Eprev, col * p * S))) return fail(rc);
    if ((rc = dalloc_t(s, &s->Dbuf, col * p * S))) return fail(rc);
  }
  // the round's read-back block: residual norms (2 p per slot), Ritz values (p per slot) and
  // basis counts (per slot), contiguous so that one copy brings them to the host
  const size_t rb = (size_t)3 * p * S + ((size_t)S + 1) / 2;
  if ((rc = dalloc_t(s, &s->norms, rb))) return fail(rc);
  s->lam_d = s->norms + (size_t)2 * p * S;
  s->count_d = reinterpret_cast<int*>(s->norms + (size_t)3 * p * S);
  s->readback_bytes = rb * 8;
  if ((rc = dalloc_t(s, &s->partial, (size_t)p * S * apply_blocks(g0) * 2))) return fail(rc);
  s->gram_cap = (int64_t)rr_partial_blocks(g0) * q * q * 4 * S;
  if ((rc = dalloc_t(s, &s->gram_partial, s->gram_cap))) return fail(rc);
  if ((rc = dalloc_t(s, &s->Gm, (size_t)q * q * 2 * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->Hm, (size_t)q * q * 2 * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->Yd, (size_t)q * q * 2 * S))) return fail(rc);
  s->ritz_stride = ritz_small_work_doubles(q);
  if ((rc = dalloc_t(s, &s->ritz_work, s->ritz_stride * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->mean_scratch, gamma_scratch_doubles(q * S)))) return fail(rc);
  if ((rc = dalloc_t(s, &s->probe_e, (size_t)2 * s->nce * s->nce))) return fail(rc);
  if ((rc = dalloc_t(s, &s->probe_n, (size_t)2 * s->ncn * s->ncn))) return fail(rc);
  if ((rc = dalloc_t(s, &s->probe_out, (size_t)2 * s->nce * s->nce * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->kc_inv64, (size_t)2 * s->nce * s->nce * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->kc_inv32, (size_t)2 * s->nce * s->nce * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->pc_inv64, (size_t)2 * s->ncn * s->ncn * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->pc_inv32, (size_t)2 * s->ncn * s->ncn * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->lists_d, (size_t)kMaxLists * S))) return fail(rc);
  if ((rc = dalloc_t(s, &s->colidx_d, (size_t)S * p))) return fail(rc);
  if (hipHostMalloc((void**)&s->lists_h, (size_t)kMaxLists * S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->colidx_h, (size_t)S * p * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->norms_h, s->readback_bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&s->param_h, (size_t)S * (sizeof(Phase) + 8 + sizeof(PlaneWave)), hipHostMallocDefault) != hipSuccess)
    return fail(set_error(BL_ENOMEM, "pinned host allocation failed%s"));
  s->lam_h = s->norms_h + (size_t)2 * p * S;
  s->count_h = reinterpret_cast<int*>(s->norms_h + (size_t)3 * p * S);
  const int ip = o.precision;
  if ((rc = ensure_level_buffers(s, ip, p, q))) return fail(rc);
  identity_block(s->probe_e, s->nce, s->st);
  identity_block(s->probe_n, s->ncn, s->st);
  if ((rc = upload_slot_params(s))) return fail(rc);
  HIP_OK(hipMemcpyAsync(s->mu_d, s->mu_h.data(), (size_t)S * 8, hipMemcpyHostToDevice, s->st));
  if (!eps) {   // slots receive their permittivity with their first task; keep the rest finite
    for (auto& L : s->lv) {
      fill_zero<double>(L.kappa64, L.g.nm * S, s->st);
      fill_zero<float>(L.kappa32, L.g.nm * S, s->st);
      if (L.sinv64) fill_zero<double>(L.sinv64, L.g.nm * kPatchW * S, s->st);
      if (L.sinv32) fill_zero<float>(L.sinv32, L.g.nm * kPatchW * S, s->st);
    }
  }
  if (eps) {
    std::vector<double> kap((size_t)gr.n * gr.m);
    double eps_min = eps[0];
    for (size_t i = 0; i < kap.size(); ++i) {
      kap[i] = 1.0 / eps[i];
      eps_min = std::min(eps_min, eps[i]);
    }
    for (int sl = 0; sl < S; ++sl)
      if ((rc = load_eps(s, sl, kap, eps_min))) return fail(rc);
  }
  HIP_OK(hipStreamSynchronize(s->st));
  if ((rc = check_hip())) return fail(rc);
  for (int pr = 0; pr < 2; ++pr) {
    s->fuse_edge[pr] = plan_fusion(s, true, pr ? 4 : 8);
    s->fuse_nodal[pr] = plan_fusion(s, false, pr ? 4 : 8);
  }
  if (o.autotune && (rc = engine_autotune(s))) return fail(rc);
  *out = s;
  return BL_OK;
}

void engine_destroy(bl_solver* s) {
  if (!s) return;
  if (s->st) (void)hipStreamSynchronize(s->st);
  else (void)hipDeviceSynchronize();
  if (s->debug && s->rounds > 0)
    std::fprintf(stderr, "bloch: %lld rounds, %.2f columns per round without a preconditioned direction\n", (long long)s->rounds,
                 (double)s->locked_cols / (double)s->rounds);
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->lists_h) (void)hipHostFree(s->lists_h);
  if (s->colidx_h) (void)hipHostFree(s->colidx_h);
  if (s->norms_h) (void)hipHostFree(s->norms_h);   // lam_h and count_h point into it
  if (s->param_h) (void)hipHostFree(s->param_h);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  delete s;
}

int engine_free_slot(const bl_solver* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (s->slot[i].phase == SLOT_FREE) return i;
  return -1;
}

int engine_busy(const bl_solver* s) {
  int b = 0;
  for (auto& ss : s->slot) b += ss.phase != SLOT_FREE;
  return b;
}

int engine_assign(bl_solver* s, int sl, Task* t) {
  if (sl < 0 || sl >= s->nslots || s->slot[sl].phase != SLOT_FREE) return set_error(BL_ESTATE, "slot not free%s");
  SlotState& ss = s->slot[sl];
  const int nk = (int)(t->ks.size() / 2);
  if (nk < 1 || t->nev < 1 || t->nev > s->opts.nev) return set_error(BL_EINVAL, "invalid task%s");
  if (!t->kappa.empty()) {
    if ((int64_t)t->kappa.size() != (int64_t)s->grid.n * s->grid.m) return set_error(BL_EINVAL, "eps size mismatch%s");
    int rc = load_eps(s, sl, t->kappa, t->eps_min);
    if (rc) return rc;
    ss.hist_count = 0;
  }
  if (!t->start_dev && ss.hist_count == 0 && !s->opts.nested_start)
    return set_error(BL_ESTATE, "no start block and no history to extrapolate from%s");
  t->evals.assign((size_t)nk * t->nev, 0.0);
  t->relres.assign((size_t)nk * t->nev, INFINITY);
  t->iters.assign(nk, 0);
  t->status = BL_OK;
  t->finished = t->done = false;
  t->t_start = now_seconds();
  t->t_points.clear();
  ss.task = t;
  ss.phase = SLOT_START;
  ss.t = 0;
  ss.it = 0;
  ss.res_rows.clear();
  return BL_OK;
}

int engine_issue(bl_solver* s) {
  const int p = s->p;
  const Geo& g0 = s->lv[0].g;
  // ---- A. start steps of new points -------------------------------------------------------
  std::vector<int> starting;
  for (int sl = 0; sl < s->nslots; ++sl) {
    SlotState& ss = s->slot[sl];
    ss.fresh = false;
    if (ss.phase != SLOT_START) continue;
    const double k1 = ss.task->ks[2 * ss.t], k2 = ss.task->ks[2 * ss.t + 1];
    if (!set_phase(s, sl, k1, k2)) {
      end_task(s, sl, BL_EINVAL, "non-finite Bloch parameter");
      continue;
    }
    starting.push_back(sl);
  }
  if (!starting.empty()) {
    // a task's first point with neither a start block nor a history to extrapolate from:
    // nested iteration (Section 6) when enabled; should the block lose rank on the way, the
    // point starts from the block in E
    for (int sl : starting) {
      SlotState& ss = s->slot[sl];
      ss.e_start = false;
      if (ss.t != 0 || ss.task->start_dev || ss.hist_count > 0 || !s->opts.nested_start) continue;
      const int rc = nested_start_slot(s, sl, ss.task->ks[0], ss.task->ks[1], ss.task->nev, ss.task->nested_its);
      if (rc == BL_OK) ss.e_start = true;
      else if (rc != BL_ENOCONV) return rc;
    }
    // group by the width of the start basis: a start block (p) or 1..3 history blocks
    std::vector<int> by_q[4];
    for (int sl : starting) {
      SlotState& ss = s->slot[sl];
      const bool from_start = ss.t == 0 && (ss.task->start_dev || ss.e_start);
      const int depth = from_start ? 0 : std::min(ss.hist_count, s->opts.extrap_depth);
      s->zthr_h[sl] = from_start ? -INFINITY : s->opts.zero_rel * ss.hist_lam1;
      by_q[depth].push_back(sl);
      if (from_start && ss.task->start_dev)
        HIP_OK(hipMemcpyAsync(s->E + (size_t)sl * p * 2 * g0.ne, ss.task->start_dev, (size_t)p * 2 * g0.ne * 8,
                              hipMemcpyDeviceToDevice, s->st));
    }
    int rc = upload_slot_params(s);
    if (rc) return rc;
    setup_coarse(s, starting);
    for (int d = 0; d < 4; ++d) {
      if (by_q[d].empty()) continue;
      std::vector<Group> gs;
      if (d == 0) gs.push_back({s->E, p, 0, 0, p});
      for (int h = 0; h < d; ++h) gs.push_back({s->hist[h], p, 0, 0, p});
      const int q = std::max(1, d) * p;
      if ((rc = project(s, gs, view(s->Sb, s->qmax), by_q[d]))) return rc;
      if ((rc = ritz_step(s, by_q[d], q, 0, d > 0))) return rc;
    }
    for (int sl : starting) {
      s->slot[sl].phase = SLOT_ITER;
      s->slot[sl].it = 0;
      s->slot[sl].fresh = true;
    }
  }
  // ---- B. residuals of every iterating slot -------------------------------------------------
  s->issued.clear();
  for (int sl = 0; sl < s->nslots; ++sl)
    if (s->slot[sl].phase == SLOT_ITER) s->issued.push_back(sl);
  if (!s->issued.empty()) {
    const int ip = s->opts.precision;
    const Level& L0 = s->lv[0];
    Launch L = make_launch(s, s->issued, p);
    int nblk = 0;
    if (ip)
      edge_apply<double, float>(EM_EIGRES, cview(s->E, p), View<const double>{nullptr, 0, 0}, view(static_cast<float*>(L0.eb[1]), L0.ecap[1]),
                                L0.kappa64, L0.kappa32, s->lam_d, p, L0.g, s->ph_d, s->mu_d, L, s->partial, &nblk);
    else
      edge_apply<double, double>(EM_EIGRES, cview(s->E, p), View<const double>{nullptr, 0, 0}, view(static_cast<double*>(L0.eb[0]), L0.ecap[0]),
                                 L0.kappa64, L0.kappa32, s->lam_d, p, L0.g, s->ph_d, s->mu_d, L, s->partial, &nblk);
    reduce_partials(s->partial, nblk, (int)s->issued.size() * p, 2, s->norms, s->st);
    s->launches += 2;
    HIP_OK(hipMemcpyAsync(s->norms_h, s->norms, s->readback_bytes, hipMemcpyDeviceToHost, s->st));
  }
  return BL_OK;
}

int engine_finish(bl_solver* s) {
  const int p = s->p;
  HIP_OK(hipStreamSynchronize(s->st));
  timing_collect(s);
  int rc = check_hip();
  if (rc) return rc;
  s->lists_used = 0;
  s->rounds += 1;
  // tasks retired in the previous round: their device copies have completed now
  const double tnow = now_seconds();
  for (Task* t : s->retired) {
    t->done = true;
    t->t_done = tnow;
  }
  s->retired.clear();
  std::vector<int> cont;
  for (size_t z = 0; z < s->issued.size(); ++z) {
    const int sl = s->issued[z];
    SlotState& ss = s->slot[sl];
    Task* t = ss.task;
    if (!t) continue;
    if (ss.fresh && s->count_h[sl] < p) {
      end_task(s, sl, BL_ENOCONV, "start block spans fewer than p non-null directions");
      continue;
    }
    const double* nr = s->norms_h + z * p * 2;
    const double* lam = s->lam_h + (size_t)sl * p;
    double rel[256];
    for (int j = 0; j < p; ++j) {
      const double den = std::fabs(lam[j]) * std::sqrt(nr[2 * j + 1]);
      rel[j] = s->opts.tol_abs ? std::sqrt(nr[2 * j]) : den > 0 ? std::sqrt(nr[2 * j]) / den : INFINITY;
    }
    // optional rounding floor of the relative residual (see bl_opts.tol_floor)
    double floor_num = 0.0;
    if (s->opts.tol_floor && !s->opts.tol_abs) {
      const Geo& g0 = s->lv[0].g;
      floor_num = std::ldexp(1.0, -53) * 8.0 * ss.kappa_max * g0.s / std::min(g0.mx, g0.my);
    }
    bool conv = true;
    int lead = 0;   // leading pairs within the locking bound
    ss.lockmask.assign(p, 0);
    for (int j = 0; j < t->nev; ++j) {
      ss.res_rows.push_back(rel[j]);
      const double tol_j = std::max(s->opts.tol, lam[j] != 0.0 ? floor_num / std::fabs(lam[j]) : 0.0);
      conv = conv && (rel[j] <= tol_j);
      ss.lockmask[j] = s->opts.lock_rel > 0 && rel[j] <= s->opts.lock_rel * tol_j;
      if (lead == j && ss.lockmask[j]) ++lead;
    }
    // throw-away vectors past the first throw_precond get no preconditioned direction either
    if (s->opts.throw_precond > 0)
      for (int j = t->nev + s->opts.throw_precond; j < p; ++j) ss.lockmask[j] = 1;
    if (conv || ss.it >= s->opts.max_iter) {
      if ((rc = retire_point(s, sl, conv, lam, rel))) return rc;
    } else {
      cont.push_back(sl);
      ss.lock = lead;
    }
  }
  s->issued.clear();
  if (!cont.empty()) {
    const int ip = s->opts.precision;
    const bool lob = s->opts.variant == 1;
    Level& L0 = s->lv[0];
    Launch L = make_launch(s, cont, p);
    // soft locking (gradient variant): the pairs within the locking bound, and the throw-away
    // vectors past the first throw_precond, get no preconditioned direction.  The c leading
    // columns locked in every continuing slot are skipped through the views' offset; further
    // locked columns are squeezed out of the residual block in place, so that the V-cycle,
    // the projection and the Ritz step run on the a columns from c on (a = p minus the fewest
    // locked columns of a slot; a slot with more locked columns keeps its highest locked ones
    // to that width).  c < nev and a > 0: an unconverged slot has a wanted pair above tol.
    int c = 0, a = p;
    bool moved = false;
    if (!lob && (s->opts.lock_rel > 0 || s->opts.throw_precond > 0)) {
      c = p;
      int fewest = p;
      for (int sl : cont) {
        const SlotState& ss = s->slot[sl];
        c = std::min(c, ss.lock);
        int nl = 0;
        for (int j = 0; j < p; ++j) nl += ss.lockmask[j] ? 1 : 0;
        fewest = std::min(fewest, nl);
      }
      a = p - fewest;
      for (size_t z = 0; z < cont.size(); ++z) {
        const SlotState& ss = s->slot[cont[z]];
        std::vector<char> keep(p, 0);
        int nk = 0;
        for (int j = c; j < p; ++j)
          if (!ss.lockmask[j]) keep[j] = 1, ++nk;
        for (int j = p - 1; j >= c && nk < a; --j)
          if (!keep[j]) keep[j] = 1, ++nk;
        int k = 0;
        for (int j = c; j < p; ++j)
          if (keep[j]) {
            s->colidx_h[z * p + k] = j - c;
            moved = moved || j - c != k;
            ++k;
          }
      }
      if (moved)
        HIP_OK(hipMemcpyAsync(s->colidx_d, s->colidx_h, cont.size() * p * sizeof(int), hipMemcpyHostToDevice, s->st));
    }
    s->locked_cols += (int64_t)(p - a) * (int64_t)cont.size();
    Launch Lc = L;
    Lc.ncps = a;
    if (ip) {
      const View<float> R = view(static_cast<float*>(L0.eb[1]), L0.ecap[1], c);
      if (moved) compact_cols<float>(R, L0.g.ne, s->colidx_d, p, a, L);
      vcycle_edge<float>(s, 0, cv(R), view(static_cast<float*>(L0.ex[1]), L0.ecap[1], c), Lc);
    } else {
      const View<double> R = view(static_cast<double*>(L0.eb[0]), L0.ecap[0], c);
      if (moved) compact_cols<double>(R, L0.g.ne, s->colidx_d, p, a, L);
      vcycle_edge<double>(s, 0, cv(R), view(static_cast<double*>(L0.ex[0]), L0.ecap[0], c), Lc);
    }
    s->launches += moved ? 1 : 0;
    // LOBPCG (Section 4): from the second iteration of a point on, the basis also holds the
    // previous block's direction D = E_prev - E (E^* M E_prev); the gradient variant, and the
    // first iteration, use [E, C]
    std::vector<int> three, two;
    for (int sl : cont) (lob && s->slot[sl].it > 0 ? three : two).push_back(sl);
    const View<const double> none{nullptr, 0, 0};
    if (!three.empty()) {
      Launch Lt = make_launch(s, three, p);
      edge_apply<double, double>(EM_M, cview(s->Eprev, p), none, view(s->Dbuf, p), L0.kappa64, L0.kappa32, nullptr,
                                 0, L0.g, s->ph_d, s->mu_d, Lt, nullptr, nullptr);
      if (gram(cview(s->E, p), p, cview(s->Dbuf, p), p, L0.g.ne, s->gram_partial, s->gram_cap, s->Gm, Lt) != 0)
        return set_error(BL_EINVAL, "Gram scratch too small%s");
      block_combine(cview(s->E, p), p, s->Gm, p, L0.g.ne, view(s->Dbuf, p), Lt);
      sub_cols<double>(cview(s->Eprev, p), cview(s->Dbuf, p), view(s->Dbuf, p), L0.g.ne, Lt);
      s->launches += 5;
      if ((rc = project(s, {{s->E, p, 0, 0, p}, {L0.ex[ip], L0.ecap[ip], 0, ip, p}, {s->Dbuf, p, 0, 0, p}},
                        view(s->Sb, s->qmax), three)))
        return rc;
      sub_cols<double>(cview(s->E, p), none, view(s->Eprev, p), L0.g.ne, Lt);
      if ((rc = ritz_step(s, three, 3 * p, p, false))) return rc;
    }
    if (!two.empty()) {
      if ((rc = project(s, {{s->E, p, 0, 0, p}, {L0.ex[ip], L0.ecap[ip], c, ip, a}}, view(s->Sb, s->qmax), two)))
        return rc;
      if (lob) sub_cols<double>(cview(s->E, p), none, view(s->Eprev, p), L0.g.ne, make_launch(s, two, p));
      if ((rc = ritz_step(s, two, p + a, p, false))) return rc;
    }
    for (int sl : cont) s->slot[sl].it += 1;
  }
  return BL_OK;
}

int engine_run(bl_solver* s) {
  int rc;
  while (engine_busy(s)) {
    if ((rc = engine_issue(s))) return rc;
    if ((rc = engine_finish(s))) return rc;
  }
  return engine_sync_retired(s);
}

int engine_sync_retired(bl_solver* s) {
  HIP_OK(hipStreamSynchronize(s->st));
  int rc = check_hip();
  if (rc) return rc;
  s->lists_used = 0;
  const double tnow = now_seconds();
  for (Task* t : s->retired) {
    t->done = true;
    t->t_done = tnow;
  }
  s->retired.clear();
  return BL_OK;
}

int engine_set_timing(bl_solver* s, bool enable) {
  if (enable && s->ev_pool.empty()) {
    s->ev_pool.resize(4096);
    for (auto& e : s->ev_pool) HIP_OK(hipEventCreate(&e));
  }
  s->timing = enable;
  s->timed_ms = 0.0;
  s->timed_count = 0;
  s->timed_cols = 0;
  s->timed_bytes = 0.0;
  s->ev_used = 0;
  return BL_OK;
}

// ---- operator-level entry points on slot 0 -------------------------------------------------
int engine_set_k0(bl_solver* s, double k1, double k2) {
  if (!set_phase(s, 0, k1, k2)) return set_error(BL_EINVAL, "non-finite Bloch parameter%s");
  int rc = upload_slot_params(s);
  if (rc) return rc;
  setup_coarse(s, {0});
  s->kset = true;
  HIP_OK(hipStreamSynchronize(s->st));
  s->lists_used = 0;
  return check_hip();
}

int engine_nested_start(bl_solver* s, int sl, double k1, double k2, int nev, std::vector<int>& its) {
  return nested_start_slot(s, sl, k1, k2, nev, its);
}

namespace {
template <typename T>
int apply_t(bl_solver* s, int op, int level, int ncols, const void* xv, const void* yv, void* outv) {
  const int pr = PrecOf<T>::v;
  const int nl = (int)s->lv.size();
  if (level < 0 || level >= nl) return set_error(BL_EINVAL, "level out of range%s");
  Level& L = s->lv[level];
  View<const T> x{static_cast<const T*>(xv), ncols, 0};
  View<const T> y{static_cast<const T*>(yv), ncols, 0};
  View<T> out{static_cast<T*>(outv), ncols, 0};
  const View<const T> none{nullptr, 0, 0};
  Launch La{nullptr, 1, ncols, s->st};
  const bool smoothed = level < nl - 1;
  int rc;
  switch (op) {
    case BL_OP_A: edge_apply<T, T>(EM_A, x, none, out, L.kappa64, L.kappa32, nullptr, 0, L.g, s->ph_d, s->mu_d, La, nullptr, nullptr); break;
    case BL_OP_M: edge_apply<T, T>(EM_M, x, none, out, L.kappa64, L.kappa32, nullptr, 0, L.g, s->ph_d, s->mu_d, La, nullptr, nullptr); break;
    case BL_OP_K: edge_apply<T, T>(EM_K, x, none, out, L.kappa64, L.kappa32, nullptr, 0, L.g, s->ph_d, s->mu_d, La, nullptr, nullptr); break;
    case BL_OP_LIFT: lift<T, T>(x, out, L.g, s->ph_d, La); break;
    case BL_OP_LHM: lhm<T, T>(x, out, L.g, s->ph_d, La); break;
    case BL_OP_P: nodal_apply<T>(x, none, out, L.g, s->ph_d, s->ns, false, La); break;
    case BL_OP_EDGE_SMOOTH:
    case BL_OP_EDGE_SMOOTH_BACK:
      if (!smoothed || !yv) return set_error(BL_EINVAL, "no smoother on this level / rhs missing%s");
      for (int c = 0; c < 4; ++c)
        edge_gs<T>(out, y, L.kappa64, L.kappa32, L.sinv64, L.sinv32, L.g, s->ph_d, s->mu_d, L.T4,
                   op == BL_OP_EDGE_SMOOTH ? c : 3 - c, s->tune_edge, La);
      break;
    case BL_OP_NODAL_SMOOTH:
      if (!smoothed || !yv) return set_error(BL_EINVAL, "no smoother on this level / rhs missing%s");
      for (int c = 0; c < 4; ++c) nodal_gs<T>(out, y, L.g, s->ph_d, s->ns, c, s->tune_nodal, La);
      break;
    case BL_OP_EDGE_VCYCLE:
    case BL_OP_NODAL_VCYCLE: {
      if ((rc = ensure_level_buffers(s, pr, ncols, ncols))) return rc;
      if (op == BL_OP_EDGE_VCYCLE) vcycle_edge<T>(s, level, x, out, La);
      else vcycle_nodal<T>(s, level, x, out, La);
      break;
    }
    case BL_OP_EDGE_PROLONG:
    case BL_OP_EDGE_RESTRICT:
    case BL_OP_NODAL_PROLONG:
    case BL_OP_NODAL_RESTRICT: {
      if (!smoothed) return set_error(BL_EINVAL, "no coarser level%s");
      Level& C = s->lv[level + 1];
      if (op == BL_OP_EDGE_PROLONG) {
        zero_cols<T>(out, L.g.ne, La);
        edge_prolong_add<T>(x, C.g, out, L.g, s->ph_d, La);
      } else if (op == BL_OP_EDGE_RESTRICT) {
        edge_restrict<T>(x, L.g, out, C.g, s->ph_d, La);
      } else if (op == BL_OP_NODAL_PROLONG) {
        zero_cols<T>(out, L.g.nm, La);
        nodal_prolong_add<T>(x, C.g, out, L.g, s->ph_d, La);
      } else {
        nodal_restrict<T>(x, L.g, out, C.g, s->ph_d, La);
      }
      break;
    }
    case BL_OP_PROJECT: {
      if (level != 0 || pr != 0) return set_error(BL_EINVAL, "projection runs on FP64 level-0 blocks%s");
      if (ncols > s->qmax) return set_error(BL_EINVAL, "too many columns%s");
      rc = project(s, {{xv, ncols, 0, 0, ncols}}, View<double>{static_cast<double*>(outv), ncols, 0}, {0});
      if (rc) return rc;
      break;
    }
    case BL_OP_COARSE_EDGE:
      if (level != nl - 1) return set_error(BL_EINVAL, "coarse solve only on the coarsest level%s");
      dense_apply<T>(kc_inv<T>(s), s->nce, x, out, La);
      break;
    case BL_OP_COARSE_NODAL:
      if (level != nl - 1) return set_error(BL_EINVAL, "coarse solve only on the coarsest level%s");
      dense_apply<T>(pc_inv<T>(s), s->ncn, x, out, La);
      break;
    case BL_OP_EIGRES:
      if (!yv) return set_error(BL_EINVAL, "eigenvalues (y) missing%s");
      if ((size_t)ncols * 2 * apply_blocks(L.g) > (size_t)s->p * s->nslots * apply_blocks(s->lv[0].g) * 2)
        return set_error(BL_EINVAL, "too many columns%s");
      edge_apply<T, T>(EM_EIGRES, x, none, out, L.kappa64, L.kappa32, static_cast<const double*>(yv), ncols, L.g,
                       s->ph_d, s->mu_d, La, s->partial, nullptr);
      break;
    case BL_OP_EDGE_SWEEP:
    case BL_OP_EDGE_SWEEP_BACK:
    case BL_OP_NODAL_SWEEP:
    case BL_OP_NODAL_SWEEP_BACK: {
      if (!smoothed || !yv) return set_error(BL_EINVAL, "no smoother on this level / rhs missing%s");
      if (xv == outv) return set_error(BL_EINVAL, "a sweep reads x and writes out: different blocks required%s");
      const bool back = op == BL_OP_EDGE_SWEEP_BACK || op == BL_OP_NODAL_SWEEP_BACK;
      if (op == BL_OP_EDGE_SWEEP || op == BL_OP_EDGE_SWEEP_BACK)
        edge_sweep<T>(x, out, y, L.kappa64, L.kappa32, L.sinv64, L.sinv32, L.g, s->ph_d, s->mu_d, L.T4, back, false,
                      s->tune_sweep[0], La);
      else
        nodal_sweep<T>(x, out, y, L.g, s->ph_d, s->ns, back, false, s->tune_sweep[1], La);
      break;
    }
    default: return set_error(BL_EINVAL, "unknown operator%s");
  }
  return BL_OK;
}
}  // namespace

int engine_rr_products(bl_solver* s, const void* S, int q, double* G, double* H) {
  if (!s->kset) return set_error(BL_ESTATE, "call bl_set_k first%s");
  if (q < 1 || q > s->qmax) return set_error(BL_EINVAL, "q must be 1..3p%s");
  const Level& L0 = s->lv[0];
  const Launch L{nullptr, 1, q, s->st};
  if (rr_gram(View<const double>{static_cast<const double*>(S), q, 0}, q, L0.kappa64, L0.g, s->ph_d, s->gram_partial,
              s->gram_cap, s->Gm, s->Hm, rr_tile(q), L) != 0)
    return set_error(BL_EINVAL, "Gram scratch too small%s");
  HIP_OK(hipMemcpyAsync(G, s->Gm, (size_t)q * q * 16, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipMemcpyAsync(H, s->Hm, (size_t)q * q * 16, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  return check_hip();
}

int engine_apply(bl_solver* s, int op, int level, int prec, int ncols, const void* x,
                 const void* y, void* out) {
  if (!s->kset) return set_error(BL_ESTATE, "call bl_set_k first%s");
  if (prec != 0 && prec != 1) return set_error(BL_EINVAL, "prec must be 0 or 1%s");
  int rc = prec ? apply_t<float>(s, op, level, ncols, x, y, out) : apply_t<double>(s, op, level, ncols, x, y, out);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(s->st));
  s->lists_used = 0;
  return check_hip();
}

}  // namespace bl
