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

// Real 4x4 transform T = D^{-1/2} Q of the stabilised node-patch solve (row-major).
struct PatchT {
  double t[16];
};

// 9-point coefficients of P = L^* M L (centre, x-neighbours, y-neighbours, diagonals).
struct NodalStencil {
  double c0, cx, cy, cd;
};

enum EdgeMode { EM_A = 0, EM_M = 1, EM_K = 2, EM_RESID_K = 3, EM_EIGRES = 4 };

// ---- launch wrappers (all asynchronous on `st`) ------------------------------------------
// out = op(x) for `ncols` columns; EM_RESID_K: out = b - (A + mu M) x;
// EM_EIGRES: out = A x - lam[j] M x, and norms_partial[j][blk] = (|out|^2, |M x|^2).
template <typename TI, typename TO>
void edge_apply(int mode, const TI* x, const TI* b, TO* out, const double* kappa64,
                const float* kappa32, const double* lam, const Geo& g, const Phase& ph,
                double mu, int ncols, double* norms_partial, int* nblk_out, hipStream_t st);
void reduce_partials(const double* partial, int nblk, int ncols, int nval, double* out,
                     hipStream_t st);

template <typename T>
void edge_gs(T* x, const T* b, const double* kappa64, const float* kappa32,
             const double* sinv64, const float* sinv32, const Geo& g, const Phase& ph,
             double mu, const PatchT& T4, int colour, int ncols, hipStream_t st);
void patch_setup(const double* kappa, const Geo& g, const PatchT& T4, const double* q,
                 double mu, double* sinv64, float* sinv32, hipStream_t st);
void coarsen_kappa(const double* kf, const Geo& gf, double* kc, hipStream_t st);
void to_float(const double* in, float* out, int64_t count, hipStream_t st);

template <typename T>
void edge_restrict(const T* rf, const Geo& gf, T* bc, const Geo& gc, const Phase& ph,
                   int ncols, hipStream_t st);
template <typename T>
void edge_prolong_add(const T* xc, const Geo& gc, T* xf, const Geo& gf, const Phase& ph,
                      int ncols, hipStream_t st);

template <typename T>
void nodal_apply(const T* x, const T* b, T* out, const Geo& g, const Phase& ph,
                 const NodalStencil& c, bool resid, int ncols, hipStream_t st);
template <typename T>
void nodal_gs(T* x, const T* b, const Geo& g, const Phase& ph, const NodalStencil& c,
              int colour, int ncols, hipStream_t st);
template <typename T>
void nodal_restrict(const T* rf, const Geo& gf, T* bc, const Geo& gc, const Phase& ph,
                    int ncols, hipStream_t st);
template <typename T>
void nodal_prolong_add(const T* xc, const Geo& gc, T* xf, const Geo& gf, const Phase& ph,
                       int ncols, hipStream_t st);
template <typename TI, typename TO>
void lhm(const TI* u, TO* out, const Geo& g, const Phase& ph, int ncols, hipStream_t st);
template <typename TI, typename TP, typename TO>
void lift_sub(const TI* u, const TP* phi, TO* out, const Geo& g, const Phase& ph, int ncols,
              hipStream_t st);
template <typename TI, typename TO>
void lift(const TI* phi, TO* out, const Geo& g, const Phase& ph, int ncols, hipStream_t st);
void gamma_deflate(double* u, const Geo& g, int ncols, double* scratch, hipStream_t st);

template <typename T>
void fill_zero(T* p, int64_t count, hipStream_t st);
void identity_block(double* out, int64_t n, hipStream_t st);
void planar_to_matrix(const double* cols, int64_t n, double* mat, hipStream_t st);
void add_constant_rank_one(double* mat, int64_t n, double gamma, hipStream_t st);
void invert_hpd(double* mat, int64_t n, hipStream_t st);
void matrix_to_float(const double* mat, float* out, int64_t count, hipStream_t st);
template <typename T>
void dense_apply(const void* inv, int64_t n, const T* b, T* x, int ncols, hipStream_t st);

// G (q x r, row-major interleaved complex) = X^* W, X and W planar FP64 blocks of length len.
void gram(const double* X, int q, const double* W, int r, int64_t len, double* partial,
          int64_t partial_cap, double* out, hipStream_t st);
int gram_blocks(int64_t len);

// Generalised Hermitian eigenproblem H y = theta G y (q x q, row-major interleaved, FP64,
// device).  The first nfix basis vectors may be declared G-orthonormal and H-diagonal
// (previous Ritz vectors).  Writes `want` G-orthonormal coefficient vectors (q x want
// row-major interleaved) to Y, their Ritz values to theta and the count found to *count.
void ritz_small(const double* G, const double* H, int q, int nfix, int want, double zero_thr,
                double drop_rel, double* work, double* Y, double* theta, int* count,
                hipStream_t st);
size_t ritz_small_work_doubles(int q);

// out (planar, want columns) = S (planar, q columns) * Y (q x want, row-major interleaved).
void block_combine(const double* S, int q, const double* Y, int want, int64_t len, double* out,
                   hipStream_t st);

}  // namespace bl
