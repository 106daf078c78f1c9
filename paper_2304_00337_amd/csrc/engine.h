// The batched eigensolver engine behind every entry point of bloch.h.
//
// An engine (the bl_solver handle) holds `nslots` problem slots of one grid shape and block
// width p = nev + nthrow.  Each slot carries its own permittivity, shift mu, Bloch phases,
// coarse direct solvers, iteration block, Ritz values and extrapolation history, and works
// through a task: a list of Bloch parameters solved one after the other with Rayleigh-
// quotient extrapolation between them (Section 6).  All slots advance in lock-step rounds;
// every kernel launch of a round covers the list of slots that take that step, so the
// launch count of a round does not grow with the number of slots.
#pragma once

#include "bloch.h"
#include "internal.h"

#include <cstdint>
#include <string>
#include <vector>

namespace bl {

constexpr int kMaxLevels = 16;
constexpr int64_t kMaxCoarse = 2048;   // largest coarsest-level edge count solved densely
constexpr int64_t kMaxNestedCoarse = 512;   // largest coarsest pencil of the nested start (Ritz kernel)
constexpr int kMaxSlots = 256;
// default shift of the preconditioned A + mu M: lambda_p of the homogeneous cell (eps_min,
// k = 0) over this divisor, at least half of its lambda_1 (Section 5 leaves mu open)
constexpr double kMuDivisor = 40.0;
constexpr int kMaxLists = 32;          // device slot lists alive between two synchronisations

// One problem: a path of Bloch parameters on one permittivity.
struct Task {
  int64_t id = 0;
  std::vector<double> kappa;     // 1/eps per cell; empty = keep what the slot holds
  double eps_min = 0.0;
  std::vector<double> ks;        // 2 * nk
  const void* start_dev = nullptr;   // p FP64 planar columns, or null = extrapolate
  int nev = 0;
  void* evecs_dev = nullptr;     // nev columns of the last point, optional
  // results
  std::vector<double> evals, relres;   // nk * nev
  std::vector<int32_t> iters;          // nk
  std::vector<double> res_hist;        // nev per iteration of the last point
  std::vector<double> t_points;        // host time at which each point was retired
  std::vector<int> nested_its;         // nested start: iterations per level (finest first)
  int status = BL_OK;
  std::string message;
  bool finished = false;         // host side finished; results valid once `done`
  bool done = false;
  double t_submit = 0, t_start = 0, t_done = 0;   // seconds, steady clock
};

enum SlotPhase { SLOT_FREE = 0, SLOT_START = 1, SLOT_ITER = 2 };

struct SlotState {
  Task* task = nullptr;
  int phase = SLOT_FREE;
  int t = 0;          // point index within the task
  int it = 0;         // iterations at the current point
  bool fresh = false; // started this round (its Ritz count is checked)
  int hist_count = 0;
  double hist_lam1 = 0.0;
  bool gamma = false;
  double mu = 1.0;
  double kappa_max = 1.0;   // largest 1/eps of the slot's permittivity (residual floor)
  bool e_start = false;     // E holds the start block of the task's first point (nested start)
  int lock = 0;             // leading pairs within the soft-locking bound after the last round
  std::vector<char> lockmask;   // pairs within the soft-locking bound after the last round
  std::vector<double> res_rows;
};

struct Level {
  Geo g{};
  double* kappa64 = nullptr;   // nslots * nm
  float* kappa32 = nullptr;
  double* sinv64 = nullptr;    // nslots * nm * 6 (smoothed levels)
  float* sinv32 = nullptr;
  PatchT T4{};
  double Q[16]{};
  // V-cycle work blocks per precision (0 = FP64, 1 = FP32), nslots * cap columns
  void* ex[2] = {nullptr, nullptr};
  void* eb[2] = {nullptr, nullptr};
  void* er[2] = {nullptr, nullptr};
  int ecap[2] = {0, 0};
  void* nx[2] = {nullptr, nullptr};
  void* nb[2] = {nullptr, nullptr};
  void* nr[2] = {nullptr, nullptr};
  int ncap[2] = {0, 0};
};

Geo make_geo(int n, int m, double a, double b);
bool is_gamma(double k1, double k2, double a, double b);
double homogeneous_lambda(int n, int m, double a, double b, double eps0, int p);
std::vector<std::pair<int, int>> hierarchy(int n, int m, int max_levels, int cmin);
double now_seconds();

int set_error(int code, const char* fmt, const char* detail = "");
int validate_opts(const bl_opts* o);
int validate_grid(const bl_grid* g, int p);
int validate_eps(const double* eps, int64_t count);
void fill_defaults(bl_opts* o);

}  // namespace bl

struct bl_solver {
  bl_grid grid{};
  bl_opts opts{};
  hipStream_t st = nullptr;
  int device = 0;
  int nslots = 1;
  int p = 0, qmax = 0;
  std::vector<bl::Level> lv;
  bl::NodalStencil ns{};
  int64_t nce = 0, ncn = 0;
  // per-slot parameters (host mirror and device copy)
  std::vector<bl::Phase> ph_h;
  std::vector<bl::PlaneWave> pw_h;   // plane-wave deflation parameters per slot
  bl::PlaneWave* pw_d = nullptr;
  double* pw_tab = nullptr;          // per slot 2 (n + m) doubles
  double* pw_part = nullptr;         // nslots * pw_cap columns * pw_blocks partials
  double* pw_coef = nullptr;         // nslots * pw_cap columns * 6
  int pw_cap = 0;
  std::vector<double> mu_h, zthr_h;
  bl::Phase* ph_d = nullptr;
  double* mu_d = nullptr;
  double* zthr_d = nullptr;
  std::vector<bl::SlotState> slot;
  // coarsest-level direct solvers, per slot
  double* kc_inv64 = nullptr;
  float* kc_inv32 = nullptr;
  double* pc_inv64 = nullptr;
  float* pc_inv32 = nullptr;
  double* probe_e = nullptr;
  double* probe_n = nullptr;
  double* probe_out = nullptr;
  // iteration blocks, slot-major
  double* E = nullptr;       // p columns per slot
  double* Sb = nullptr;      // qmax columns per slot
  double* hist[3] = {nullptr, nullptr, nullptr};   // p columns per slot, most recent first
  double* Eprev = nullptr;   // LOBPCG: the previous iteration's block (p columns per slot)
  double* Dbuf = nullptr;    // LOBPCG: its direction E_prev - E (E^* M E_prev), p columns per slot
  double* lam_d = nullptr;   // p per slot
  int* count_d = nullptr;    // per slot
  double* partial = nullptr;
  double* norms = nullptr;   // read-back block: norms, then lam_d and count_d
  size_t readback_bytes = 0;
  double* gram_partial = nullptr;
  int64_t gram_cap = 0;
  double* Gm = nullptr;
  double* Hm = nullptr;
  double* Yd = nullptr;
  double* ritz_work = nullptr;
  size_t ritz_stride = 0;
  double* mean_scratch = nullptr;
  // nested start: the coarsest level's dense pencil and its Ritz step (one slot at a time)
  double* nst_G = nullptr;
  double* nst_H = nullptr;
  double* nst_Y = nullptr;
  double* nst_work = nullptr;
  int nst_q = 0;
  void* nodal_extra[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int nodal_extra_cap[2] = {0, 0};
  // slot lists: pinned host staging and device copies, recycled after each synchronisation
  int* lists_h = nullptr;
  int* lists_d = nullptr;
  int* colidx_h = nullptr;   // soft locking: per slot of a round, the source of each kept column
  int* colidx_d = nullptr;   // (nslots * p)
  int lists_used = 0;
  // read-back of the residual round (pinned)
  double* norms_h = nullptr;
  double* lam_h = nullptr;
  int* count_h = nullptr;
  std::vector<int> issued;    // slots whose residuals were issued in this round
  std::vector<bl::Task*> retired;   // finished tasks whose last device copies may be in flight
  void* param_h = nullptr;    // pinned staging of the per-slot phases and thresholds
  bool kset = false;          // operator entry points: k fixed for slot 0
  std::vector<void*> allocs;
  size_t dev_bytes = 0;
  int64_t launches = 0;
  int64_t locked_cols = 0;   // soft-locked columns summed over slots and iterations
  int64_t rounds = 0;
  std::vector<double> last_res_hist;   // slot 0, last point
  int last_res_rows = 0;
  // opt-in HIP-event timing of the finest-level smoother launches
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  double timed_ms = 0.0;
  int64_t timed_count = 0;
  int64_t timed_cols = 0;
  double timed_bytes = 0.0;   // algorithmic HBM bytes of the timed launches
  bool debug = false;
  // first fused coarse level of the edge / nodal V-cycles per precision (-1: none)
  int fuse_edge[2] = {-1, -1};
  int fuse_nodal[2] = {-1, -1};
  // launch shapes chosen by the autotuner (defaults when it is off)
  bl::SmoothShape tune_edge, tune_nodal;
  int tune_rr = 0;            // Rayleigh-Ritz output tile for q = 2p (0 = by padding)
  double tune_ms = 0.0;       // time the autotuner spent
  int tune_sweep[2] = {0, 0}; // tile shapes of the edge and nodal sweeps (see edge_sweep)
};

namespace bl {

// Engine life cycle.  eps (host, n*m) may be null for a batched engine whose slots receive
// their permittivity with each task.
int engine_create(const bl_grid* grid, const bl_opts* opts, int nslots, hipStream_t st,
                  const double* eps, bl_solver** out);
void engine_destroy(bl_solver* s);
size_t engine_footprint(const bl_grid* grid, const bl_opts* opts, int nslots);
// Put a task on a free slot (uploads its permittivity when it carries one).
int engine_assign(bl_solver* s, int slot, Task* t);
int engine_free_slot(const bl_solver* s);
int engine_busy(const bl_solver* s);
// One round: engine_issue queues the start steps of new points and the residuals of every
// iterating slot; engine_finish waits for them, retires converged points and queues the
// next iteration of the others.  Errors returned are device errors; task-level errors end
// up in Task::status.
int engine_issue(bl_solver* s);
int engine_finish(bl_solver* s);
// Run rounds until every slot is free.
int engine_run(bl_solver* s);
// Wait for the stream and mark the retired tasks done.
int engine_sync_retired(bl_solver* s);

// Autotuner: time the candidate launch shapes of the finest-level smoothers and of the
// Rayleigh-Ritz products on the engine's own buffers and keep the fastest; results are
// cached per (n, m, p, precision) for the process, seeded from the shipped table.
int engine_autotune(bl_solver* s);
int rr_tile(int q);

// Opt-in HIP-event timing of the finest-level smoother launches (resets the totals).
int engine_set_timing(bl_solver* s, bool enable);

// bl_info of an engine (bl_get_info, bl_batch_engine_info).
void fill_info(const bl_solver* s, bl_info* out);

// Operator-level helpers on slot 0.
int engine_set_k0(bl_solver* s, double k1, double k2);
int engine_apply(bl_solver* s, int op, int level, int prec, int ncols, const void* x,
                 const void* y, void* out);
int engine_rr_products(bl_solver* s, const void* S, int q, double* G, double* H);
// Nested iteration (Section 6) for slot sl at (k1, k2), whose phases are set: the start block
// in E on return, iterations per level in its.
int engine_nested_start(bl_solver* s, int sl, double k1, double k2, int nev, std::vector<int>& its);

}  // namespace bl
