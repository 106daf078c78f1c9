// Internal interface between the host solver and the gfx950 kernels.
//
// Every block of complex vectors is stored as "planar column blocks": column j of a block
// of vectors of length N starts at base + j * 2N and holds N real parts followed by N
// imaginary parts.  Edge vectors have N = 2nm (x-edges then y-edges), nodal vectors N = nm.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bl {

// Geometry of one multigrid level (Section 3 mesh, Section 5 bisection hierarchy).
struct Geo {
  int n, m;          // cells per direction
  double h1, h2;     // mesh widths
  double s;          // 1 / (h1 h2): curl-curl scale
  double mx, my;     // h2/h1 (x-edge mass scale) and h1/h2 (y-edge mass scale)
  int64_t nm, ne;    // nodes (= cells) and edges
};

// Bloch phases alpha = exp(i k1 a), beta = exp(i k2 b).
struct Phase {
  double ar, ai, br, bi;
};

// Plane-wave deflation of the nodal solve (null-space elimination, Sections 4-5).  The nodal
// vector w_j = exp(i (t1 j1 + t2 j2)), t = k' h with k' the first-zone representative of k, is
// an exact eigenvector of P = L^* M L with eigenvalue lambda_w (-> 0 like |k|^2 h^2 at Gamma).
// Per slot: t1, t2; ex = exp(i t1) - 1, ey = exp(i t2) - 1 (the gradient of w on an x- / y-edge
// is w_j ex / w_j ey); inm = 1 / nm; ilw = 1 / (nm lambda_w), zero at Gamma.
struct PlaneWave {
  double t1, t2, exr, exi, eyr, eyi, inm, ilw;
};
// Arguments of the deflated projection's kernels.  tab: per slot (stride tabstride doubles)
// the factors exp(i t1 j1), j1 < n, then exp(i t2 j2), j2 < m (interleaved complex).  part:
// per launch column (index slot_in_launch * pcols + off + j) `nblk` block partials of two
// doubles.  coef: per launch column six doubles: w^* b / nm, the exact coefficient
// c = w^* b / (nm lambda_w), and gamma = c - w^* phi' / nm.
struct PWDefl {
  const double* tab;
  const PlaneWave* par;
  double* part;
  double* coef;
  int64_t tabstride;
  int pcols;
  int off;
  int nblk;
};

// Real 4x4 transform T = D^{-1/2} Q of the stabilised node-patch solve (row-major).
struct PatchT {
  double t[16];
};

// Per node, the smoother keeps the stabilised patch inverse W = T diag(1/mu, S^{-1}) T^T as
// its 10 upper-triangle entries (w00 w01 w02 w03 w11 w12 w13 w22 w23 w33), formed in FP64
// from the factors when the coefficients are loaded.
constexpr int kPatchW = 10;

// 9-point coefficients of P = L^* M L (centre, x-neighbours, y-neighbours, diagonals).
struct NodalStencil {
  double c0, cx, cy, cd;
};

enum EdgeMode { EM_A = 0, EM_M = 1, EM_K = 2, EM_RESID_K = 3, EM_EIGRES = 4 };

// Batched launches.  A solver holds `slots` independent problems of one grid shape; slot s
// has its own Bloch phases (ph[s]), shift mu (mu[s], device), permittivity (kappa and patch
// factors at offset s * nm of every level) and coarse inverses.  A launch covers `nact` slots (the device list `slots`,
// or slots 0..nact-1 when it is null) and `ncps` columns per slot: grid.y = nact * ncps.
struct Launch {
  const int* slots;
  int nact;
  int ncps;
  hipStream_t st;
};
// Columns of a slot-major buffer: column j of slot s is at base + (s * cps + off + j) * 2N.
template <typename T>
struct View {
  T* p;
  int cps;
  int off;
};
template <typename T>
inline View<T> view(T* p, int cps, int off = 0) { return View<T>{p, cps, off}; }
template <typename T>
inline View<const T> cview(const T* p, int cps, int off = 0) { return View<const T>{p, cps, off}; }

// tab for slots 0..nslots-1 from par (after the parameters were uploaded).
void pw_tables(const PlaneWave* par, double* tab, int64_t tabstride, int n, int m, int nslots, hipStream_t st);
// mode 0: reduce the w^* b partials (count blocks) of every launch column into coef[0..3];
// mode 1: reduce the w^* phi' partials into coef[4..5] = c - w^* phi' / nm.
void pw_reduce(const PWDefl& d, int mode, int count, const Launch& L);
// b -= w (w^* b / nm) on the launch's nodal columns (partial-free).
template <typename T>
void pw_rhs(View<T> b, const Geo& g, const PWDefl& d, const Launch& L);
// partials of w^* phi on the launch's nodal columns; returns the block count.
template <typename T>
int pw_dot(View<const T> phi, const Geo& g, const PWDefl& d, const Launch& L);
int pw_blocks(const Geo& g);

// ---- launch wrappers (all asynchronous on L.st) --------------------------------------------
// out = op(x); EM_RESID_K: out = b - (A + mu M) x; EM_EIGRES: out = A x - lam M x with lam of
// the column at lam[s * lam_cps + j], and partial[(y * nblk + block) * 2 + {0,1}] =
// (|out|^2, |M x|^2) block sums, y = the launch column index blockIdx.y.
template <typename TI, typename TO>
void edge_apply(int mode, View<const TI> x, View<const TI> b, View<TO> out, const double* kappa64,
                const float* kappa32, const double* lam, int lam_cps, const Geo& g,
                const Phase* ph, const double* mu, const Launch& L, double* partial, int* nblk_out);
void reduce_partials(const double* partial, int nblk, int ncols, int nval, double* out,
                     hipStream_t st);
// blocks per column of the point kernels (edge_apply's partials per column)
int apply_blocks(const Geo& g);

// Launch shape of the colour passes of the smoothers (chosen per engine shape by the
// autotuner; results do not depend on it): threads per block, columns per thread (1 or 2,
// sharing the patch coefficients) and the XCD-major block order.
struct SmoothShape {
  int bs = 256;
  int cpt = 1;
  int xcd = 0;
};

template <typename T>
void edge_gs(View<T> x, View<const T> b, const double* kappa64, const float* kappa32,
             const double* sinv64, const float* sinv32, const Geo& g, const Phase* ph,
             const double* mu, const PatchT& T4, int colour, const SmoothShape& sh, const Launch& L);
// Level transfers folded into a tiled sweep.  bc set (forward sweeps): the sweep also forms
// the residual b - K x of its result and writes its restriction to the coarse right-hand
// side bc (level geometry gc).  xc set: the sweep starts from xin + Pr xc (the coarse
// correction prolongated on the fly).  base set: the sweep writes base + result (xout may be
// base itself).  Each result equals that of the separate kernels bit for bit.
template <typename T>
struct SweepFuse {
  View<T> bc{nullptr, 0, 0};
  View<const T> xc{nullptr, 0, 0};
  View<const T> base{nullptr, 0, 0};
  View<T> res{nullptr, 0, 0};   // nodal backward sweeps: also write b - P xout here
  Geo gc{};
};

// One whole smoothing sweep (four colours; reverse colour order when backward) as one launch
// over LDS tiles with halos, bit-identical to the four colour launches; `tile` selects the
// tile shape (0: 32 x 32, 1: 64 x 32 nodes; FP64 edge sweeps 32 x 32).  Reads the iterate
// from xin and writes it to xout, which must be different buffers; zero_start: the iterate is
// zero on entry (xin is then not read).  sweep.hip.
template <typename T>
void edge_sweep(View<const T> xin, View<T> xout, View<const T> b, const double* kappa64, const float* kappa32,
                const double* sinv64, const float* sinv32, const Geo& g, const Phase* ph, const double* mu,
                const PatchT& T4, bool backward, bool zero_start, int tile, const Launch& L,
                const SweepFuse<T>& fz = SweepFuse<T>{});
// Whether edge sweeps of this element size can restrict (SweepFuse::bc): FP32 only (the
// FP64 residual window exceeds the static LDS of a workgroup).
bool edge_sweep_restricts(size_t elem);
template <typename T>
void nodal_sweep(View<const T> xin, View<T> xout, View<const T> b, const Geo& g, const Phase* ph,
                 const NodalStencil& c, bool backward, bool zero_start, int tile, const Launch& L,
                 const SweepFuse<T>& fz = SweepFuse<T>{});
void patch_setup(const double* kappa, const Geo& g, const double* q, const PatchT& T4, const double* mu,
                 double* sinv64, float* sinv32, int nslots, hipStream_t st);
void coarsen_kappa(const double* kf, const Geo& gf, double* kc, int nslots, hipStream_t st);
void to_float(const double* in, float* out, int64_t count, hipStream_t st);

template <typename T>
void edge_restrict(View<const T> rf, const Geo& gf, View<T> bc, const Geo& gc, const Phase* ph,
                   const Launch& L);
template <typename T>
void edge_prolong_add(View<const T> xc, const Geo& gc, View<T> xf, const Geo& gf,
                      const Phase* ph, const Launch& L);
// out = base + Pr xc (base may be out itself)
template <typename T>
void edge_prolong_to(View<const T> xc, const Geo& gc, View<const T> base, View<T> out, const Geo& gf,
                     const Phase* ph, const Launch& L);

template <typename T>
void nodal_apply(View<const T> x, View<const T> b, View<T> out, const Geo& g, const Phase* ph,
                 const NodalStencil& c, bool resid, const Launch& L);
template <typename T>
void nodal_gs(View<T> x, View<const T> b, const Geo& g, const Phase* ph, const NodalStencil& c,
              int colour, const SmoothShape& sh, const Launch& L);
template <typename T>
void nodal_restrict(View<const T> rf, const Geo& gf, View<T> bc, const Geo& gc, const Phase* ph,
                    const Launch& L);
template <typename T>
void nodal_prolong_add(View<const T> xc, const Geo& gc, View<T> xf, const Geo& gf,
                       const Phase* ph, const Launch& L);
template <typename T>
void nodal_prolong_to(View<const T> xc, const Geo& gc, View<const T> base, View<T> out, const Geo& gf,
                      const Phase* ph, const Launch& L);
// out = L^* M u; with pw, also the partials of w^* out (FP64, before rounding to TO).
template <typename TI, typename TO>
void lhm(View<const TI> u, View<TO> out, const Geo& g, const Phase* ph, const Launch& L,
         const PWDefl* pw = nullptr);
// out = u - L phi; with pw, also minus gamma L w (gamma = coef[4..5] of the column).
template <typename TI, typename TP, typename TO>
void lift_sub(View<const TI> u, View<const TP> phi, View<TO> out, const Geo& g, const Phase* ph,
              const Launch& L, const PWDefl* pw = nullptr);
template <typename TI, typename TO>
void lift(View<const TI> phi, View<TO> out, const Geo& g, const Phase* ph, const Launch& L);
// k = 0 deflation of the constant edge fields on the launch's columns of u; scratch holds
// gamma_scratch_doubles(columns of the launch) doubles.
void gamma_deflate(View<double> u, const Geo& g, double* scratch, const Launch& L);
size_t gamma_scratch_doubles(int cols);
template <typename T>
void axpy(View<T> y, View<const T> x, int64_t len, const Launch& L);
// out = a - b, or out = a when b.p is null (columns of length len)
template <typename T>
void sub_cols(View<const T> a, View<const T> b, View<T> out, int64_t len, const Launch& L);

// Column k of v (columns of length len, k < ncols) receives column src[z * src_stride + k]
// of the same slot (z the launch's slot index), in place; per slot src[k] >= k and strictly
// increasing.  Columns with src[k] == k are not touched.
template <typename T>
void compact_cols(View<T> v, int64_t len, const int* src, int src_stride, int ncols, const Launch& L);

template <typename T>
void fill_zero(T* p, int64_t count, hipStream_t st);
template <typename T>
void zero_cols(View<T> x, int64_t len, const Launch& L);
// Fused coarse levels of a V-cycle: from the first fused level down to the coarsest, one
// workgroup per column runs the whole rest of the cycle in LDS (coarse.hip).  Level 0 of the
// description is the first fused level; the last one is solved with the dense inverse.
constexpr int kMaxFused = 6;
struct CoarseLevel {
  Geo g;
  PatchT T4;
  const double* k64;    // kappa, slot-major (nm per slot)
  const float* k32;
  const double* si64;   // patch inverses, slot-major (6 nm per slot); null on the coarsest
  const float* si32;
};
struct CoarseCycle {
  int nlev;             // fused levels including the coarsest
  int nu_pre, nu_post;
  int64_t nc;           // unknowns of the coarsest level (edges or nodes)
  const void* inv;      // its inverse in the cycle's precision, slot-major (nc x nc complex)
  NodalStencil ns;      // nodal cycles
  CoarseLevel L[kMaxFused];
};
// LDS bytes of a fused cycle with elements of `elem` bytes, and the device's limit.
size_t fused_lds_bytes(const CoarseCycle& C, bool edge, size_t elem);
size_t fused_lds_limit();
template <typename T>
void edge_vcycle_fused(View<const T> b, View<T> x, const CoarseCycle& C, const Phase* ph, const double* mu,
                       const Launch& L);
template <typename T>
void nodal_vcycle_fused(View<const T> b, View<T> x, const CoarseCycle& C, const Phase* ph, const Launch& L);

// Coarsest-level direct solvers.  Probe columns: n shared unit vectors (identity_block);
// per slot s the probe results (n columns) at cols + s * n * 2n and the matrices (row-major
// interleaved complex) at mat + s * n * n * 2.
void identity_block(double* out, int64_t n, hipStream_t st);
void planar_to_matrix(const double* cols, int64_t n, double* mat, const Launch& L);
void add_constant_rank_one(double* mat, int64_t n, double gamma, const Launch& L);
void invert_hpd(double* mat, int64_t n, const Launch& L);
// out[s * count + i] = (float) mat[s * count + i] on the launch's slots
void matrix_to_float(const double* mat, float* out, int64_t count, const Launch& L);
// x = Inv_s b per column, Inv_s = inv + s * n * n (complex, Hermitian)
template <typename T>
void dense_apply(const void* inv, int64_t n, View<const T> b, View<T> x, const Launch& L);

// Per slot: G_s (q x r, row-major interleaved complex, at out + s * q * r * 2) = X_s^* W_s of
// planar FP64 column views of length len.  Returns -1 (nothing launched) when partial_cap
// (doubles) is below gram_blocks(len) * q * r * 2 * nact.
int gram(View<const double> X, int q, View<const double> W, int r, int64_t len, double* partial,
         int64_t partial_cap, double* out, const Launch& L);
int gram_blocks(int64_t len);

// Rayleigh-Ritz products straight from the basis (no stored M S or A S): per slot
// G_s = S_s^* M S_s and H_s = S_s^* A S_s (q x q, row-major interleaved complex, at
// G/H + s * q * q * 2).  q <= 48 runs on the matrix cores; wider bases on the vector units
// with 48- or 64-wide output tiles (`tile` 3 or 4).  Returns -1 (nothing launched) when
// partial_cap (doubles) is below rr_partial_blocks(g) * q * q * 4 * nact.
int rr_gram(View<const double> S, int q, const double* kappa, const Geo& g, const Phase* ph,
            double* partial, int64_t partial_cap, double* G, double* H, int tile, const Launch& L);
int rr_blocks(int64_t nm);
int rr_partial_blocks(const Geo& g);

// Generalised Hermitian eigenproblem H y = theta G y per slot (q x q, row-major interleaved,
// FP64, at G/H + s * q * q * 2), one workgroup per slot.  The first nfix basis vectors may
// be declared G-orthonormal (previous Ritz vectors).  Writes `want` G-orthonormal coefficient
// vectors (q x want, at Y + s * q * want * 2), their Ritz values (theta + s * want) and the
// count found (count[s]).  zero_thr per slot (zthr[s]), or -inf when zthr is null.
void ritz_small(const double* G, const double* H, int q, int nfix, int want, const double* zthr,
                double drop_rel, double* work, size_t work_stride, double* Y, double* theta,
                int* count, const Launch& L);
size_t ritz_small_work_doubles(int q);

// out_s (want columns) = S_s (q columns) * Y_s (q x want, at Y + s * q * want * 2).
void block_combine(View<const double> S, int q, const double* Y, int want, int64_t len,
                   View<double> out, const Launch& L);

}  // namespace bl
