// Dense kernels of the iteration (Section 4 and 5) for gfx950:
//  * coarsest-level direct solve: the coarse operator is assembled by applying the stencil
//    to unit vectors, inverted in place by Gauss-Jordan (Hermitian positive definite, no
//    pivoting) in one workgroup, and applied as a dense matrix-vector product;
//  * tall-skinny Gram products X^* W of planar FP64 blocks (LDS-staged, register-tiled);
//  * the Ritz step: generalised Hermitian eigenproblem H y = theta G y of size <= 3p solved
//    in one workgroup by scaling, pivoted Cholesky of G (numerically dependent directions
//    dropped) with a second orthonormalisation pass, a Jacobi eigensolve of the reduced H,
//    and ascending sort;
//  * block recombination S Y.
#include "internal.h"

#include <cmath>

namespace bl {

struct c2 {
  double r, i;
};
__device__ __forceinline__ c2 cm(c2 a, c2 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ c2 cmc(c2 a, c2 b) { return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r}; }  // conj(a)*b

// ------------------------------------------------------------------------------------------
__global__ void k_identity_block(double* __restrict__ out, int64_t n) {
  const int64_t j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[j * 2 * n + i] = (i == j) ? 1.0 : 0.0;
  out[j * 2 * n + n + i] = 0.0;
}
void identity_block(double* out, int64_t n, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  k_identity_block<<<grid, 256, 0, st>>>(out, n);
}

// mat (row-major interleaved) [i][j] = column j of the probe result at row i
__global__ void k_planar_to_matrix(const double* __restrict__ cols, int64_t n, double* __restrict__ mat) {
  const int64_t j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  mat[2 * (i * n + j)] = cols[j * 2 * n + i];
  mat[2 * (i * n + j) + 1] = cols[j * 2 * n + n + i];
}
void planar_to_matrix(const double* cols, int64_t n, double* mat, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  k_planar_to_matrix<<<grid, 256, 0, st>>>(cols, n, mat);
}

__global__ void k_add_rank_one(double* __restrict__ mat, int64_t n, double gamma) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) mat[2 * e] += gamma / (double)n;
}
void add_constant_rank_one(double* mat, int64_t n, double gamma, hipStream_t st) {
  k_add_rank_one<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(mat, n, gamma);
}

// In-place Gauss-Jordan inversion of a Hermitian positive definite matrix (no pivoting).
__global__ __launch_bounds__(1024) void k_invert(c2* __restrict__ A, int n) {
  extern __shared__ c2 colk[];
  __shared__ c2 piv;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const c2 a = A[(int64_t)k * n + k];
      const double d = a.r * a.r + a.i * a.i;
      piv = {a.r / d, -a.i / d};
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) colk[i] = A[(int64_t)i * n + k];
    __syncthreads();
    const c2 p = piv;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      if (j != k) A[(int64_t)k * n + j] = cm(A[(int64_t)k * n + j], p);
    }
    __syncthreads();
    if (threadIdx.x == 0) A[(int64_t)k * n + k] = p;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
      const int i = (int)(e / n), j = (int)(e % n);
      if (i == k) continue;
      const c2 f = colk[i];
      if (j == k) {
        const c2 v = cm(f, p);
        A[e] = {-v.r, -v.i};
      } else {
        const c2 v = cm(f, A[(int64_t)k * n + j]);
        A[e] = {A[e].r - v.r, A[e].i - v.i};
      }
    }
    __syncthreads();
  }
}
void invert_hpd(double* mat, int64_t n, hipStream_t st) {
  k_invert<<<1, 1024, (size_t)n * sizeof(c2), st>>>(reinterpret_cast<c2*>(mat), (int)n);
}

__global__ void k_mat_to_float(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}
void matrix_to_float(const double* mat, float* out, int64_t count, hipStream_t st) {
  k_mat_to_float<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(mat, out, count);
}

// x = Inv b for a Hermitian Inv (row-major interleaved); row i of Inv is read as the
// conjugate of column i, so that consecutive threads read consecutive entries.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_apply(const T* __restrict__ inv, int64_t n,
                                                     const T* __restrict__ b, T* __restrict__ x) {
  const int col = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T* bc = b + (int64_t)col * 2 * n;
  T sr = 0, si = 0;
  for (int64_t l = 0; l < n; ++l) {
    const T ar = inv[2 * (l * n + i)], ai = -inv[2 * (l * n + i) + 1];
    const T br = bc[l], bi = bc[n + l];
    sr += ar * br - ai * bi;
    si += ar * bi + ai * br;
  }
  T* xc = x + (int64_t)col * 2 * n;
  xc[i] = sr;
  xc[n + i] = si;
}
template <typename T>
void dense_apply(const void* inv, int64_t n, const T* b, T* x, int ncols, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  k_dense_apply<T><<<grid, 256, 0, st>>>(reinterpret_cast<const T*>(inv), n, b, x);
}
template void dense_apply<double>(const void*, int64_t, const double*, double*, int, hipStream_t);
template void dense_apply<float>(const void*, int64_t, const float*, float*, int, hipStream_t);

// ------------------------------------------------------------------------------------------
// Gram products.  Block (16 x 16 threads) computes a 64 x 64 tile of X^* W over a range of
// rows; rows are staged through LDS 16 at a time; each thread owns a 4 x 4 register tile.
constexpr int GB = 64, GTR = 16;

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ X, int q,
                                              const double* __restrict__ W, int r, int64_t len,
                                              int64_t rows_per_blk, double* __restrict__ partial) {
  __shared__ double xr[GTR][GB], xi[GTR][GB], wr[GTR][GB], wi[GTR][GB];
  const int ntj = (r + GB - 1) / GB;
  const int i0 = (blockIdx.y / ntj) * GB, j0 = (blockIdx.y % ntj) * GB;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t rs = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t re = rs + rows_per_blk < len ? rs + rows_per_blk : len;
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) { ar[a][b] = 0; ai[a][b] = 0; }
  for (int64_t r0 = rs; r0 < re; r0 += GTR) {
    for (int e = tid; e < GTR * GB; e += 256) {
      const int rr = e % GTR, cc = e / GTR;
      const int64_t row = r0 + rr;
      const bool okr = row < re;
      const int cx = i0 + cc, cw = j0 + cc;
      xr[rr][cc] = (okr && cx < q) ? X[(int64_t)cx * 2 * len + row] : 0.0;
      xi[rr][cc] = (okr && cx < q) ? X[(int64_t)cx * 2 * len + len + row] : 0.0;
      wr[rr][cc] = (okr && cw < r) ? W[(int64_t)cw * 2 * len + row] : 0.0;
      wi[rr][cc] = (okr && cw < r) ? W[(int64_t)cw * 2 * len + len + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < GTR; ++rr) {
      double x_r[4], x_i[4], w_r[4], w_i[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) { x_r[a] = xr[rr][ty * 4 + a]; x_i[a] = xi[rr][ty * 4 + a]; }
#pragma unroll
      for (int b = 0; b < 4; ++b) { w_r[b] = wr[rr][tx * 4 + b]; w_i[b] = wi[rr][tx * 4 + b]; }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          ar[a][b] += x_r[a] * w_r[b] + x_i[a] * w_i[b];
          ai[a][b] += x_r[a] * w_i[b] - x_i[a] * w_r[b];
        }
    }
    __syncthreads();
  }
  double* pp = partial + (int64_t)blockIdx.x * q * r * 2;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
      if (i < q && j < r) {
        pp[2 * ((int64_t)i * r + j)] = ar[a][b];
        pp[2 * ((int64_t)i * r + j) + 1] = ai[a][b];
      }
    }
}

__global__ void k_gram_reduce(const double* __restrict__ partial, int nblk, int64_t count,
                              double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * count + e];
  out[e] = s;
}

int gram_blocks(int64_t len) {
  int64_t nb = (len + 1023) / 1024;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return (int)nb;
}

void gram(const double* X, int q, const double* W, int r, int64_t len, double* partial,
          int64_t partial_cap, double* out, hipStream_t st) {
  int nb = gram_blocks(len);
  while ((int64_t)nb * q * r * 2 > partial_cap && nb > 1) nb /= 2;
  int64_t rpb = (len + nb - 1) / nb;
  rpb = (rpb + GTR - 1) / GTR * GTR;
  nb = (int)((len + rpb - 1) / rpb);
  const int nti = (q + GB - 1) / GB, ntj = (r + GB - 1) / GB;
  dim3 grid((unsigned)nb, (unsigned)(nti * ntj));
  k_gram<<<grid, 256, 0, st>>>(X, q, W, r, len, rpb, partial);
  const int64_t count = (int64_t)q * r * 2;
  k_gram_reduce<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(partial, nb, count, out);
}

// ------------------------------------------------------------------------------------------
// Ritz step solver, one workgroup.  For the Gram matrix G = S^* M S and H = S^* A S of a
// basis S (q columns):
//   1. unit-diagonal scaling D, pivoted Cholesky P^T (D G D) P = L L^*, stopped when the
//      largest remaining pivot falls below drop_rel (the directions of S that are
//      numerically dependent are dropped; rank r);
//   2. Z = D P [L11^{-*}; 0] (q x r), an M-orthonormal basis of the kept span;
//   3. H' = Z^* H Z, Hermitian r x r, diagonalised by cyclic parallel Jacobi: in each
//      round the r/2 disjoint pairs of a round-robin schedule get rotations
//      J = [[c, s e^{i phi}], [-s e^{-i phi}, c]] that zero H'_pq, and all 2x2 blocks
//      (pair, pair) are updated at once, V <- V J alongside;
//   4. ascending order, values at or below zero_thr skipped, Y = Z V[:, selected].
// A (the working matrix) and V live in LDS when they fit, otherwise in the global work
// array.
constexpr int RT = 512;

__device__ void block_reduce_max(double& v, int& idx, double* shv, int* shi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_down(v, o, 64);
    const int oi = __shfl_down(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { shv[w] = v; shi[w] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = shv[0];
    int bi = shi[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
      if (shv[k] > bv || (shv[k] == bv && shi[k] < bi)) { bv = shv[k]; bi = shi[k]; }
    shv[16] = bv;
    shi[16] = bi;
  }
  __syncthreads();
  v = shv[16];
  idx = shi[16];
}

__device__ double block_sum(double a, double* sh) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    sh[16] = t;
  }
  __syncthreads();
  return sh[16];
}

size_t ritz_small_work_doubles(int q) { return (size_t)5 * q * q * 2 + 8 * (size_t)q + 64; }

// Out (r x r, stride ldo) = Z^* X Z for X (q x q, row-major global) and Z (q x r); T is a
// q x r scratch.  Ends with a barrier.
__device__ void dense_aha(const c2* X, int q, const c2* Z, int r, c2* T, c2* Out, int ldo) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < q * r; e += nt) {
    const int i = e / r, c = e % r;
    c2 s = {0, 0};
    for (int l = 0; l < q; ++l) {
      const c2 t = cm(X[i * q + l], Z[l * r + c]);
      s.r += t.r;
      s.i += t.i;
    }
    T[i * r + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int a = e / r, b = e % r;
    c2 s = {0, 0};
    for (int l = 0; l < q; ++l) {
      const c2 t = cmc(Z[l * r + a], T[l * r + b]);
      s.r += t.r;
      s.i += t.i;
    }
    Out[a * ldo + b] = s;
  }
  __syncthreads();
}

// In-place Cholesky A = L L^* (lower triangle, stride ld) of a Hermitian positive definite
// r x r matrix; non-positive pivots are clamped to a tiny positive value.
__device__ void cholesky_inplace(c2* A, int r, int ld, double* sh) {
  (void)sh;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < r; ++k) {
    double d = A[k * ld + k].r;
    d = d > 1e-300 ? sqrt(d) : 1e-150;
    __syncthreads();
    for (int i = k + 1 + tid; i < r; i += nt) {
      const c2 a = A[i * ld + k];
      A[i * ld + k] = {a.r / d, a.i / d};
    }
    if (tid == 0) A[k * ld + k] = {d, 0.0};
    __syncthreads();
    const int rem = r - k - 1;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j > i) continue;
      const c2 t = cmc(A[j * ld + k], A[i * ld + k]);
      A[i * ld + j] = {A[i * ld + j].r - t.r, A[i * ld + j].i - t.i};
    }
    __syncthreads();
  }
}

// Linv (stride ldv) = inverse of the lower-triangular L (stride ld, r x r), one column per
// thread by forward substitution.  Ends with a barrier.
__device__ void lower_inverse(const c2* L, int ld, c2* Linv, int ldv, int r) {
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    for (int i = 0; i < r; ++i) {
      if (i < c) {
        Linv[i * ldv + c] = {0.0, 0.0};
        continue;
      }
      c2 s = {(i == c) ? 1.0 : 0.0, 0.0};
      for (int l = c; l < i; ++l) {
        const c2 t = cm(L[i * ld + l], Linv[l * ldv + c]);
        s.r -= t.r;
        s.i -= t.i;
      }
      const double d = L[i * ld + i].r;
      Linv[i * ldv + c] = {s.r / d, s.i / d};
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(RT) void k_ritz_small(const c2* __restrict__ G, const c2* __restrict__ H,
                                                   int q, int want, double zero_thr, double drop_rel,
                                                   double* __restrict__ work, int lds_mode,
                                                   c2* __restrict__ Y, double* __restrict__ theta,
                                                   int* __restrict__ count) {
  extern __shared__ c2 smem[];
  __shared__ double shv[32];
  __shared__ int shi[32];
  __shared__ double rot[4 * 128];
  __shared__ int perm[256];
  __shared__ int pinv[256];
  __shared__ int sel_idx[256];
  __shared__ double ev[256];
  __shared__ double dsc[256];
  __shared__ int rank_s, nsel_s;
  // working storage: A (q x q) and V (q x q) in LDS or global; Z and T1 global
  c2* gw = reinterpret_cast<c2*>(work);
  c2* A = (lds_mode >= 1) ? smem : gw;
  c2* V = (lds_mode >= 2) ? smem + q * q : gw + q * q;
  c2* Z = gw + 2 * q * q;
  c2* T1 = gw + 3 * q * q;
  const int tid = threadIdx.x, nt = blockDim.x;
  // 1. scaling and pivoted Cholesky of D G D (lower triangle is the working part)
  for (int i = tid; i < q; i += nt) {
    const double gd = G[i * q + i].r;
    dsc[i] = gd > 0 ? 1.0 / sqrt(gd) : 0.0;
    perm[i] = i;
  }
  __syncthreads();
  for (int e = tid; e < q * q; e += nt) {
    const int i = e / q, j = e % q;
    const c2 g = G[e], gt = G[j * q + i];
    const double s = dsc[i] * dsc[j];
    A[e] = {0.5 * (g.r + gt.r) * s, 0.5 * (g.i - gt.i) * s};
  }
  __syncthreads();
  int r = 0;
  for (int k = 0; k < q; ++k) {
    double v = -1.0;
    int idx = q;
    for (int j = k + tid; j < q; j += nt) {
      const double d = A[j * q + j].r;
      if (d > v || (d == v && j < idx)) { v = d; idx = j; }
    }
    block_reduce_max(v, idx, shv, shi);
    if (!(v > drop_rel)) break;   // unit diagonal: the pivot is relative to the original size
    if (idx != k) {               // symmetric swap of rows/columns k and idx
      for (int c = tid; c < q; c += nt) {
        const c2 t = A[k * q + c];
        A[k * q + c] = A[idx * q + c];
        A[idx * q + c] = t;
      }
      __syncthreads();
      for (int c = tid; c < q; c += nt) {
        const c2 t = A[c * q + k];
        A[c * q + k] = A[c * q + idx];
        A[c * q + idx] = t;
      }
      if (tid == 0) {
        const int t = perm[k];
        perm[k] = perm[idx];
        perm[idx] = t;
      }
      __syncthreads();
    }
    const double piv = sqrt(A[k * q + k].r);
    __syncthreads();
    for (int i = k + 1 + tid; i < q; i += nt) {
      const c2 a = A[i * q + k];
      A[i * q + k] = {a.r / piv, a.i / piv};
    }
    if (tid == 0) A[k * q + k] = {piv, 0.0};
    __syncthreads();
    // trailing update of the full (Hermitian) square, so later symmetric swaps stay valid
    const int rem = q - k - 1;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      const c2 li = A[i * q + k], lj = A[j * q + k];
      const c2 t = cmc(lj, li);   // l_i conj(l_j)
      A[i * q + j] = {A[i * q + j].r - t.r, A[i * q + j].i - t.i};
    }
    __syncthreads();
    r = k + 1;
  }
  if (tid == 0) rank_s = r;
  __syncthreads();
  r = rank_s;
  // 2. Linv = L11^{-1} into V's storage; Z[i][c] = d_i conj(Linv[c][pinv(i)])
  lower_inverse(A, q, V, q, r);
  for (int i = tid; i < q; i += nt) pinv[perm[i]] = i;
  __syncthreads();
  for (int e = tid; e < q * r; e += nt) {
    const int i = e / r, c = e % r;
    const int pi = pinv[i];
    c2 z = {0.0, 0.0};
    if (pi < r && pi <= c) {
      const c2 l = V[c * q + pi];
      z = {dsc[i] * l.r, -dsc[i] * l.i};
    }
    Z[i * r + c] = z;
  }
  __syncthreads();
  // second pass: G2 = Z^* G Z = L2 L2^*, Z <- Z L2^{-*} (removes the rounding of the first
  // factorisation of a possibly ill-conditioned G)
  dense_aha(G, q, Z, r, T1, A, r);
  cholesky_inplace(A, r, r, shv);
  lower_inverse(A, r, V, r, r);
  for (int e = tid; e < q * r; e += nt) {
    const int i = e / r, c = e % r;
    c2 s = {0, 0};
    for (int l = 0; l <= c; ++l) {
      const c2 t = cmc(V[c * r + l], Z[i * r + l]);   // Z[i][l] conj(Linv2[c][l])
      s.r += t.r;
      s.i += t.i;
    }
    T1[i * r + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < q * r; e += nt) Z[e] = T1[e];
  __syncthreads();
  // 3. H' = Z^* H Z into A (r x r, stride r), symmetrised
  dense_aha(H, q, Z, r, T1, A, r);
  for (int e = tid; e < r * r; e += nt) {
    const int a = e / r, b = e % r;
    if (a < b) {
      const c2 x = A[a * r + b], y = A[b * r + a];
      const c2 h = {0.5 * (x.r + y.r), 0.5 * (x.i - y.i)};
      A[a * r + b] = h;
      A[b * r + a] = {h.r, -h.i};
    } else if (a == b) {
      A[e].i = 0.0;
    }
  }
  for (int e = tid; e < r * r; e += nt) V[e] = {(e / r == e % r) ? 1.0 : 0.0, 0.0};
  __syncthreads();
  // 4. Jacobi on A (r x r)
  if (r >= 2) {
    const int rp = r + (r & 1), np = rp / 2;
    for (int sweep = 0; sweep < 30; ++sweep) {
      double off = 0, dn = 0;
      for (int e = tid; e < r * r; e += nt) {
        const c2 a = A[e];
        const double v = a.r * a.r + a.i * a.i;
        if (e / r == e % r) dn += v; else off += v;
      }
      off = block_sum(off, shv);
      dn = block_sum(dn, shv);
      if (off <= 1e-30 * dn || off == 0.0) break;
      for (int t = 0; t < rp - 1; ++t) {
        for (int k = tid; k < np; k += nt) {
          int a, b;
          if (k == 0) { a = t; b = rp - 1; }
          else { a = (t + k) % (rp - 1); b = (t - k + rp - 1) % (rp - 1); }
          const int p = a < b ? a : b, qq = a < b ? b : a;
          double c = 1, s = 0, er = 1, ei = 0;
          if (qq < r) {
            const c2 apq = A[p * r + qq];
            const double g = sqrt(apq.r * apq.r + apq.i * apq.i);
            const double app = A[p * r + p].r, aqq = A[qq * r + qq].r;
            if (g > 1e-300 && g > 1e-18 * (fabs(app) + fabs(aqq))) {
              const double tau = (aqq - app) / (2.0 * g);
              const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + tt * tt);
              s = tt * c;
              er = apq.r / g;
              ei = apq.i / g;
            }
          }
          perm[2 * k] = p;
          perm[2 * k + 1] = qq;
          rot[4 * k] = c;
          rot[4 * k + 1] = s;
          rot[4 * k + 2] = er;
          rot[4 * k + 3] = ei;
        }
        __syncthreads();
        // every 2x2 block (pair u rows, pair w columns): B <- J_u^* B J_w; V rows: V J_w
        for (int e = tid; e < np * np + np * ((r + 1) / 2); e += nt) {
          if (e < np * np) {
            const int u = e / np, w = e % np;
            const int pu = perm[2 * u], qu = perm[2 * u + 1], pw = perm[2 * w], qw = perm[2 * w + 1];
            const bool ru = qu < r, rw = qw < r;
            // rows present: pu always (< r), qu if ru; columns likewise
            const double cu = rot[4 * u], su = rot[4 * u + 1], cw = rot[4 * w], sw = rot[4 * w + 1];
            const c2 eu = {rot[4 * u + 2], rot[4 * u + 3]}, ew = {rot[4 * w + 2], rot[4 * w + 3]};
            const c2 ewc = {ew.r, -ew.i}, euc = {eu.r, -eu.i};
            if (pu >= r || pw >= r) continue;
            c2 b00 = A[pu * r + pw];
            c2 b01 = rw ? A[pu * r + qw] : c2{0, 0};
            c2 b10 = ru ? A[qu * r + pw] : c2{0, 0};
            c2 b11 = (ru && rw) ? A[qu * r + qw] : c2{0, 0};
            // columns: [b0p, b0q] J_w
            c2 t1 = cm(ewc, b01), t2 = cm(ew, b00);
            const c2 n00 = {cw * b00.r - sw * t1.r, cw * b00.i - sw * t1.i};
            const c2 n01 = {sw * t2.r + cw * b01.r, sw * t2.i + cw * b01.i};
            t1 = cm(ewc, b11);
            t2 = cm(ew, b10);
            const c2 n10 = {cw * b10.r - sw * t1.r, cw * b10.i - sw * t1.i};
            const c2 n11 = {sw * t2.r + cw * b11.r, sw * t2.i + cw * b11.i};
            // rows: J_u^* [n0; n1]
            t1 = cm(eu, n10);
            t2 = cm(euc, n00);
            A[pu * r + pw] = {cu * n00.r - su * t1.r, cu * n00.i - su * t1.i};
            if (ru) A[qu * r + pw] = {su * t2.r + cu * n10.r, su * t2.i + cu * n10.i};
            if (rw) {
              t1 = cm(eu, n11);
              t2 = cm(euc, n01);
              A[pu * r + qw] = {cu * n01.r - su * t1.r, cu * n01.i - su * t1.i};
              if (ru) A[qu * r + qw] = {su * t2.r + cu * n11.r, su * t2.i + cu * n11.i};
            }
          } else {
            const int f = e - np * np;
            const int w = f % np, rowpair = f / np;
            const int pw = perm[2 * w], qw = perm[2 * w + 1];
            if (qw >= r) continue;
            const double cw = rot[4 * w], sw = rot[4 * w + 1];
            const c2 ew = {rot[4 * w + 2], rot[4 * w + 3]}, ewc = {ew.r, -ew.i};
            for (int row = 2 * rowpair; row < 2 * rowpair + 2 && row < r; ++row) {
              const c2 x = V[row * r + pw], y = V[row * r + qw];
              const c2 t1 = cm(ewc, y), t2 = cm(ew, x);
              V[row * r + pw] = {cw * x.r - sw * t1.r, cw * x.i - sw * t1.i};
              V[row * r + qw] = {sw * t2.r + cw * y.r, sw * t2.i + cw * y.i};
            }
          }
        }
        __syncthreads();
      }
    }
  }
  // 5. ascending order (ties by index), skip values <= zero_thr, take `want`
  for (int i = tid; i < r; i += nt) {
    const double v = A[i * r + i].r;
    int rank = 0;
    for (int j = 0; j < r; ++j) {
      const double w = A[j * r + j].r;
      if (w < v || (w == v && j < i)) ++rank;
    }
    ev[rank] = v;
    sel_idx[rank] = i;
  }
  __syncthreads();
  if (tid == 0) {
    int c = 0;
    for (int i = 0; i < r && c < want; ++i) {
      if (ev[i] > zero_thr) {
        pinv[c] = sel_idx[i];
        theta[c] = ev[i];
        ++c;
      }
    }
    for (int i = c; i < want; ++i) theta[i] = 0.0;
    nsel_s = c;
    *count = c;
  }
  __syncthreads();
  const int ns = nsel_s;
  for (int e = tid; e < q * want; e += nt) {
    const int i = e / want, c = e % want;
    c2 s = {0, 0};
    if (c < ns) {
      const int kk = pinv[c];
      for (int l = 0; l < r; ++l) {
        const c2 v = cm(Z[i * r + l], V[l * r + kk]);
        s.r += v.r;
        s.i += v.i;
      }
    }
    Y[i * want + c] = s;
  }
}

static int g_lds_cap = -1;

void ritz_small(const double* G, const double* H, int q, int want, double zero_thr,
                double drop_rel, double* work, double* Y, double* theta, int* count,
                hipStream_t st) {
  if (g_lds_cap < 0) {
    int dev = 0, cap = 65536;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) cap = 65536;
    // static LDS of the kernel (reduction, rotation and index arrays) stays below 12 KB
    cap -= 12 * 1024;
    if (cap > 0 && hipFuncSetAttribute((const void*)k_ritz_small, hipFuncAttributeMaxDynamicSharedMemorySize, cap) != hipSuccess)
      cap = 64 * 1024 - 12 * 1024;
    g_lds_cap = cap > 0 ? cap : 0;
  }
  const size_t mat = (size_t)q * q * sizeof(c2);
  int mode = 0;
  size_t lds = 0;
  if (2 * mat <= (size_t)g_lds_cap) { mode = 2; lds = 2 * mat; }
  else if (mat <= (size_t)g_lds_cap) { mode = 1; lds = mat; }
  k_ritz_small<<<1, RT, lds, st>>>(reinterpret_cast<const c2*>(G), reinterpret_cast<const c2*>(H), q,
                                   want, zero_thr, drop_rel, work, mode, reinterpret_cast<c2*>(Y), theta,
                                   count);
}

// ------------------------------------------------------------------------------------------
// out[:, j] = sum_l S[:, l] Y[l][j]; thread per row, 8 output columns per block row.
constexpr int CB = 8;
__global__ __launch_bounds__(256) void k_block_combine(const double* __restrict__ S, int q,
                                                       const c2* __restrict__ Y, int want, int64_t len,
                                                       double* __restrict__ out) {
  extern __shared__ c2 ys[];   // q x CB
  const int j0 = blockIdx.y * CB;
  for (int e = threadIdx.x; e < q * CB; e += blockDim.x) {
    const int l = e / CB, c = e % CB;
    ys[e] = (j0 + c < want) ? Y[l * want + j0 + c] : c2{0, 0};
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double accr[CB], acci[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) { accr[c] = 0; acci[c] = 0; }
  for (int l = 0; l < q; ++l) {
    const double sr = S[(int64_t)l * 2 * len + i], si = S[(int64_t)l * 2 * len + len + i];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const c2 y = ys[l * CB + c];
      accr[c] += sr * y.r - si * y.i;
      acci[c] += sr * y.i + si * y.r;
    }
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (j0 + c < want) {
      out[(int64_t)(j0 + c) * 2 * len + i] = accr[c];
      out[(int64_t)(j0 + c) * 2 * len + len + i] = acci[c];
    }
  }
}

void block_combine(const double* S, int q, const double* Y, int want, int64_t len, double* out,
                   hipStream_t st) {
  dim3 grid((unsigned)((len + 255) / 256), (unsigned)((want + CB - 1) / CB));
  k_block_combine<<<grid, 256, (size_t)q * CB * sizeof(c2), st>>>(S, q, reinterpret_cast<const c2*>(Y),
                                                                   want, len, out);
}

}  // namespace bl
