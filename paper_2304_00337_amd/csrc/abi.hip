// C ABI of bloch.h for single problems: a handle is an engine with one slot.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace bl {
const char* last_error_message();
}

using namespace bl;

namespace {

#define HIP_OK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e_)); \
  } while (0)

// Device buffer of one call, freed when the call returns (every path, errors included).
struct DeviceScratch {
  void* p = nullptr;
  bool alloc(size_t bytes) { return hipMalloc(&p, bytes) == hipSuccess; }
  double* d() const { return static_cast<double*>(p); }
  ~DeviceScratch() {
    if (p) (void)hipFree(p);
  }
};

int check_hip() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BL_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return BL_OK;
}

// Run one task on slot 0 to the end; outputs stay valid on BL_ENOCONV.
int run_task(bl_solver* s, Task& t) {
  int rc = engine_assign(s, 0, &t);
  if (rc) return rc;
  rc = engine_run(s);
  if (rc) return rc;
  if (t.status != BL_OK) return set_error(t.status, "%s", t.message.c_str());
  return BL_OK;
}

// Section 6 raster: sources of grid point (i, j), oldest first, as (i', j') pairs.
int raster_sources(int kappa, int i, int j, int32_t* src) {
  int c = 0;
  auto put = [&](int a, int b) {
    src[2 * c] = a;
    src[2 * c + 1] = b;
    ++c;
  };
  if (j == 0)
    for (int q = std::max(0, i - 3); q < i; ++q) put(q, 0);
  else if (i <= 2)
    for (int q = std::max(0, j - 3); q < j; ++q) put(i, q);
  else
    for (int q = i - 3; q < i; ++q) put(q, j);
  (void)kappa;
  return c;
}

// Blocks kept while a grid is solved: the points of columns 0..2 in a ring of four rows (a
// point of those columns is a source of the three rows above it), and every point in a ring
// of three along its row (the horizontal sources).
constexpr int kKeepBlocks = 15;
int keep_column(int i, int j) { return i * 4 + (j & 3); }
int keep_row(int i) { return 12 + i % 3; }
int keep_of_source(int si, int sj, int j) { return sj == j ? keep_row(si) : keep_column(si, sj); }

}  // namespace

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
  o->engine_streams = 3;
  o->autotune = 1;
  o->coarse_fuse = 1;
  o->tiled_sweeps = 2;
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

const char* bl_last_error(void) { return last_error_message(); }

size_t bl_footprint_bytes(const bl_grid* grid, const bl_opts* opts) {
  if (!grid) return 0;
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  return engine_footprint(grid, &o, 1);
}

int bl_create(const bl_grid* grid, const double* eps_cells, const bl_opts* opts, void* stream,
              bl_solver** out) {
  if (!eps_cells) return set_error(BL_EINVAL, "eps is NULL%s");
  return engine_create(grid, opts, 1, static_cast<hipStream_t>(stream), eps_cells, out);
}

void bl_destroy(bl_solver* s) { engine_destroy(s); }

int bl_get_info(const bl_solver* s, bl_info* out) {
  if (!s || !out) return set_error(BL_EINVAL, "NULL argument%s");
  bl::fill_info(s, out);
  return BL_OK;
}

}  // extern "C"

void bl::fill_info(const bl_solver* s, bl_info* out) {
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
  out->mu = s->mu_h.empty() ? 0.0 : s->mu_h[0];
  out->device_bytes = s->dev_bytes;
  out->kernel_launches = s->launches;
  out->edge_smooth_shape[0] = s->tune_edge.bs;
  out->edge_smooth_shape[1] = s->tune_edge.cpt;
  out->edge_smooth_shape[2] = s->tune_edge.xcd;
  out->nodal_smooth_shape[0] = s->tune_nodal.bs;
  out->nodal_smooth_shape[1] = s->tune_nodal.cpt;
  out->nodal_smooth_shape[2] = s->tune_nodal.xcd;
  out->rr_tile = 16 * (s->tune_rr ? s->tune_rr : rr_tile(2 * s->p));
  out->autotune_ms = s->tune_ms;
  out->locked_columns = s->locked_cols;
  out->fused_edge_level = s->fuse_edge[s->opts.precision ? 1 : 0];
  out->fused_nodal_level = s->fuse_nodal[s->opts.precision ? 1 : 0];
}

extern "C" {

int bl_solve_k(bl_solver* s, double k1, double k2, const void* start_dev, double* evals,
               double* relres, int32_t* iters, void* evecs_dev) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  Task t;
  t.ks = {k1, k2};
  t.start_dev = start_dev;
  t.nev = s->opts.nev;
  t.evecs_dev = evecs_dev;
  const int rc = run_task(s, t);
  if (rc != BL_OK && rc != BL_ENOCONV) return rc;
  const int nev = s->opts.nev;
  if (evals) std::memcpy(evals, t.evals.data(), (size_t)nev * 8);
  if (relres) std::memcpy(relres, t.relres.data(), (size_t)nev * 8);
  if (iters) *iters = t.iters[0];
  return rc;
}

int bl_solve_path(bl_solver* s, const double* ks, int32_t nk, const void* start_dev,
                  double* evals, double* relres, int32_t* iters, void* evecs_last_dev) {
  if (!s || !ks || nk < 1) return set_error(BL_EINVAL, "invalid path arguments%s");
  Task t;
  t.ks.assign(ks, ks + 2 * (size_t)nk);
  t.start_dev = start_dev;
  t.nev = s->opts.nev;
  t.evecs_dev = evecs_last_dev;
  const int rc = run_task(s, t);
  if (rc != BL_OK && rc != BL_ENOCONV) return rc;
  const size_t cnt = (size_t)nk * s->opts.nev;
  if (evals) std::memcpy(evals, t.evals.data(), cnt * 8);
  if (relres) std::memcpy(relres, t.relres.data(), cnt * 8);
  if (iters) std::memcpy(iters, t.iters.data(), (size_t)nk * 4);
  return rc;
}

int bl_raster_sources(int32_t kappa, int32_t i, int32_t j, int32_t* src) {
  if (kappa < 2 || !src || i < 0 || j < 0 || i >= kappa || j >= kappa)
    return set_error(BL_EINVAL, "kappa >= 2, src and a point of the grid required%s");
  return raster_sources(kappa, i, j, src);
}

int bl_solve_kgrid(bl_solver* s, int32_t kappa, const void* start_dev, double* evals, double* relres,
                   int32_t* iters) {
  if (!s || kappa < 2 || kappa > 4096 || !start_dev || !evals || !relres || !iters)
    return set_error(BL_EINVAL, "invalid grid arguments%s");
  const int nev = s->opts.nev;
  const size_t blk = (size_t)s->p * 2 * s->lv[0].g.ne;   // doubles per block (slot 0)
  double* keep = nullptr;
  if (hipMalloc((void**)&keep, kKeepBlocks * blk * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(BL_ENOMEM, "no device memory for the grid's kept blocks%s");
  }
  double keep_lam1[kKeepBlocks] = {};
  int first = BL_OK, rc = BL_OK;
  const double pa = M_PI / s->grid.a, pb = M_PI / s->grid.b;
  for (int j = 0; j < kappa && rc == BL_OK; ++j)
    for (int i = 0; i < kappa; ++i) {
      int32_t src[6];
      const int c = raster_sources(kappa, i, j, src);
      const int d = std::min(c, s->opts.extrap_depth);
      SlotState& ss = s->slot[0];
      for (int h = 0; h < d; ++h) {   // hist[0] = the most recent source
        const int q = c - 1 - h;
        const int id = keep_of_source(src[2 * q], src[2 * q + 1], j);
        if (hipMemcpyAsync(s->hist[h], keep + id * blk, blk * sizeof(double), hipMemcpyDeviceToDevice, s->st) !=
            hipSuccess) {
          rc = set_error(BL_EHIP, "history copy failed%s");
          break;
        }
      }
      if (rc) break;
      if (c > 0) {
        ss.hist_count = d;
        ss.hist_lam1 = keep_lam1[keep_of_source(src[2 * c - 2], src[2 * c - 1], j)];
      }
      Task t;
      t.ks = {pa * (2.0 * i / (kappa - 1) - 1.0), pb * (2.0 * j / (kappa - 1) - 1.0)};
      t.start_dev = c == 0 ? start_dev : nullptr;
      t.nev = nev;
      const int r = run_task(s, t);
      if (r != BL_OK && r != BL_ENOCONV) {
        rc = r;
        break;
      }
      if (r != BL_OK && first == BL_OK) first = r;
      const size_t row = (size_t)j * kappa + i;
      std::memcpy(evals + row * nev, t.evals.data(), (size_t)nev * 8);
      std::memcpy(relres + row * nev, t.relres.data(), (size_t)nev * 8);
      iters[row] = t.iters[0];
      // the solved block is the newest history entry now
      const int ids[2] = {keep_row(i), i <= 2 ? keep_column(i, j) : -1};
      for (int id : ids) {
        if (id < 0) continue;
        if (hipMemcpyAsync(keep + id * blk, s->hist[0], blk * sizeof(double), hipMemcpyDeviceToDevice, s->st) !=
            hipSuccess) {
          rc = set_error(BL_EHIP, "history copy failed%s");
          break;
        }
        keep_lam1[id] = ss.hist_lam1;
      }
      if (rc) break;
    }
  const hipError_t se = hipStreamSynchronize(s->st);
  (void)hipFree(keep);
  if (rc) return rc;
  if (se != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(se));
  return first;
}

int bl_nested_start(bl_solver* s, double k1, double k2, double tol_levels, void* out_dev, int32_t* level_iters) {
  if (!s || !out_dev || !(tol_levels > 0) || !(tol_levels < 1)) return set_error(BL_EINVAL, "invalid nested-start arguments%s");
  const int L = (int)s->lv.size();
  if (level_iters)
    for (int l = 0; l < L; ++l) level_iters[l] = 0;
  int rc = engine_set_k0(s, k1, k2);
  if (rc) return rc;
  const double saved = s->opts.nested_tol;
  s->opts.nested_tol = tol_levels;
  std::vector<int> its;
  rc = engine_nested_start(s, 0, k1, k2, s->opts.nev, its);
  s->opts.nested_tol = saved;
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(out_dev, s->E, (size_t)s->p * 2 * s->lv[0].g.ne * 8, hipMemcpyDeviceToDevice, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  if (level_iters)
    for (int l = 0; l < L; ++l) level_iters[l] = its[l];
  return check_hip();
}

int bl_reset_history(bl_solver* s) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  for (auto& ss : s->slot) ss.hist_count = 0;
  return BL_OK;
}

int bl_last_residual_history(const bl_solver* s, double* relres, int32_t cap) {
  if (!s || !relres) return set_error(BL_EINVAL, "NULL argument%s");
  if (cap < 0) return set_error(BL_EINVAL, "cap must be >= 0%s");
  const int nev = s->opts.nev;
  const int rows = std::min(cap, s->last_res_rows);
  std::memcpy(relres, s->last_res_hist.data(), (size_t)rows * nev * 8);
  return rows;
}

int bl_set_timing(bl_solver* s, int32_t enable) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  return engine_set_timing(s, enable != 0);
}

int bl_get_timing(const bl_solver* s, double* total_ms, int64_t* launches, int64_t* columns, double* alg_bytes) {
  if (!s || !total_ms || !launches || !columns || !alg_bytes) return set_error(BL_EINVAL, "NULL argument%s");
  *total_ms = s->timed_ms;
  *launches = s->timed_count;
  *columns = s->timed_cols;
  *alg_bytes = s->timed_bytes;
  return BL_OK;
}

int bl_set_k(bl_solver* s, double k1, double k2) {
  if (!s) return set_error(BL_EINVAL, "solver is NULL%s");
  return engine_set_k0(s, k1, k2);
}

int bl_apply(bl_solver* s, int32_t op, int32_t level, int32_t prec, int32_t ncols, const void* x,
             const void* y, void* out) {
  if (!s || !x || !out || ncols < 1) return set_error(BL_EINVAL, "invalid apply arguments%s");
  return engine_apply(s, op, level, prec, ncols, x, y, out);
}

int bl_gram(bl_solver* s, const void* X, int32_t q, const void* W, int32_t r, int64_t len,
            double* out) {
  if (!s || !X || !W || !out || q < 1 || r < 1 || len < 1) return set_error(BL_EINVAL, "invalid gram arguments%s");
  DeviceScratch part, res;
  const int64_t cap = (int64_t)gram_blocks(len) * q * r * 2;
  if (!part.alloc(cap * 8) || !res.alloc((size_t)q * r * 2 * 8)) return set_error(BL_ENOMEM, "device allocation failed%s");
  const Launch L{nullptr, 1, 0, s->st};
  gram(View<const double>{static_cast<const double*>(X), q, 0}, q, View<const double>{static_cast<const double*>(W), r, 0}, r,
       len, part.d(), cap, res.d(), L);
  hipError_t e = hipMemcpyAsync(out, res.p, (size_t)q * r * 2 * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e));
  return check_hip();
}

int bl_rr_products(bl_solver* s, const void* S, int32_t q, double* G, double* H) {
  if (!s || !S || !G || !H) return set_error(BL_EINVAL, "NULL argument%s");
  return engine_rr_products(s, S, q, G, H);
}

int bl_ritz_small(bl_solver* s, const double* G, const double* H, int32_t q, int32_t want,
                  double zero_thr, double* theta, double* Y) {
  if (!s || !G || !H || !theta || !Y || q < 1 || q > 512 || want < 1 || want > q)
    return set_error(BL_EINVAL, "invalid ritz arguments%s");
  const size_t m2 = (size_t)q * q * 2 * 8;
  DeviceScratch dG, dH, dW, dY, dT, dZ, dc;
  if (!dG.alloc(m2) || !dH.alloc(m2) || !dW.alloc(ritz_small_work_doubles(q) * 8) ||
      !dY.alloc((size_t)q * want * 2 * 8) || !dT.alloc((size_t)want * 8) || !dZ.alloc(8) || !dc.alloc(sizeof(int)))
    return set_error(BL_ENOMEM, "device allocation failed%s");
  HIP_OK(hipMemcpyAsync(dG.p, G, m2, hipMemcpyHostToDevice, s->st));
  HIP_OK(hipMemcpyAsync(dH.p, H, m2, hipMemcpyHostToDevice, s->st));
  HIP_OK(hipMemcpyAsync(dZ.p, &zero_thr, 8, hipMemcpyHostToDevice, s->st));
  const Launch L{nullptr, 1, 0, s->st};
  ritz_small(dG.d(), dH.d(), q, 0, want, dZ.d(), 1e-10, dW.d(), 0, dY.d(), dT.d(), static_cast<int*>(dc.p), L);
  int cnt = 0;
  hipError_t e = hipMemcpyAsync(Y, dY.p, (size_t)q * want * 2 * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(theta, dT.p, (size_t)want * 8, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipMemcpyAsync(&cnt, dc.p, sizeof(int), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return set_error(BL_EHIP, "HIP error: %s", hipGetErrorString(e));
  if (std::getenv("BL_DEBUG")) {
    // the kernel's phase stamps (wall clock, 100 MHz): Cholesky, Z, orthonormality repair,
    // reduction and tridiagonalisation, eigenvalues, eigenvectors, back-transformation
    double st[10] = {};
    if (hipMemcpy(st, dW.d() + 10 * (size_t)q * q + 8 * q + 1, sizeof(st), hipMemcpyDeviceToHost) == hipSuccess)
      std::fprintf(stderr, "bloch: ritz q=%d want=%d phases us: %.1f %.1f %.1f %.1f %.1f %.1f %.1f total %.1f\n", q,
                   want, (st[1] - st[0]) / 100, (st[2] - st[1]) / 100, (st[3] - st[2]) / 100, (st[4] - st[3]) / 100,
                   (st[9] - st[4]) / 100, (st[5] - st[9]) / 100, (st[6] - st[5]) / 100, (st[6] - st[0]) / 100);
  }
  int rc = check_hip();
  return rc ? rc : cnt;
}

}  // extern "C"
