// Dense kernels of the iteration (Section 4 and 5) for gfx950:
//  * coarsest-level direct solve: the coarse operator is assembled by applying the stencil
//    to unit vectors, inverted in place by Gauss-Jordan (Hermitian positive definite, no
//    pivoting) in one workgroup, and applied as a dense matrix-vector product;
//  * tall-skinny Gram products X^* W of planar FP64 blocks (LDS-staged, register-tiled);
//  * the Ritz step: generalised Hermitian eigenproblem H y = theta G y of size <= 3p solved
//    in one workgroup by scaling, a Jacobi eigensolve of G (directions of negligible
//    G-eigenvalue dropped), a second Jacobi eigensolve of the reduced H, and ascending sort;
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
// Cyclic parallel Jacobi for a Hermitian r x r matrix A (row-major, global memory) in one
// workgroup, accumulating V <- V J.  Round-robin ordering: in round t the pairs are
// (t, rp-1) and ((t+k) mod (rp-1), (t-k) mod (rp-1)), k = 1..rp/2-1 (rp = r rounded up to
// even; pairs with the padding index are skipped).  Each rotation J = [[c, s e^{i phi}],
// [-s e^{-i phi}, c]] zeroes A_pq.
constexpr int RT = 1024;

__device__ void block_sum2(double& a, double& b, double* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sh[2 * w] = a; sh[2 * w + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0, tb = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { ta += sh[2 * k]; tb += sh[2 * k + 1]; }
    sh[32] = ta;
    sh[33] = tb;
  }
  __syncthreads();
  a = sh[32];
  b = sh[33];
}

__device__ void jacobi(c2* A, c2* V, int r, double* sh, double* rot /* 4 * rp/2 */, int* rpair) {
  const int rp = r + (r & 1);
  const int np = rp / 2;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) V[e] = {(e / r == e % r) ? 1.0 : 0.0, 0.0};
  __syncthreads();
  if (r < 2) return;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0, dn = 0;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
      const c2 a = A[e];
      const double v = a.r * a.r + a.i * a.i;
      if (e / r == e % r) dn += v; else off += v;
    }
    block_sum2(off, dn, sh);
    if (off <= 1e-30 * dn || off == 0.0) break;
    for (int t = 0; t < rp - 1; ++t) {
      for (int k = threadIdx.x; k < np; k += blockDim.x) {
        int a, b;
        if (k == 0) { a = t; b = rp - 1; }
        else { a = (t + k) % (rp - 1); b = (t - k + rp - 1) % (rp - 1); }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1, s = 0, er = 1, ei = 0;
        if (q < r) {
          const c2 apq = A[p * r + q];
          const double g = sqrt(apq.r * apq.r + apq.i * apq.i);
          if (g > 1e-300) {
            const double app = A[p * r + p].r, aqq = A[q * r + q].r;
            const double tau = (aqq - app) / (2.0 * g);
            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            er = apq.r / g;
            ei = apq.i / g;
          }
        }
        rpair[2 * k] = p;
        rpair[2 * k + 1] = q;
        rot[4 * k] = c;
        rot[4 * k + 1] = s;
        rot[4 * k + 2] = er;
        rot[4 * k + 3] = ei;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = threadIdx.x; e < np * r; e += blockDim.x) {
        const int k = e / r, row = e % r;
        const int p = rpair[2 * k], q = rpair[2 * k + 1];
        if (q >= r) continue;
        const double c = rot[4 * k], s = rot[4 * k + 1];
        const c2 ep = {rot[4 * k + 2], rot[4 * k + 3]}, em = {rot[4 * k + 2], -rot[4 * k + 3]};
        c2 x = A[row * r + p], y = A[row * r + q];
        c2 t1 = cm(em, y), t2 = cm(ep, x);
        A[row * r + p] = {c * x.r - s * t1.r, c * x.i - s * t1.i};
        A[row * r + q] = {s * t2.r + c * y.r, s * t2.i + c * y.i};
        x = V[row * r + p];
        y = V[row * r + q];
        t1 = cm(em, y);
        t2 = cm(ep, x);
        V[row * r + p] = {c * x.r - s * t1.r, c * x.i - s * t1.i};
        V[row * r + q] = {s * t2.r + c * y.r, s * t2.i + c * y.i};
      }
      __syncthreads();
      // rows: A <- J^* A
      for (int e = threadIdx.x; e < np * r; e += blockDim.x) {
        const int k = e / r, cc = e % r;
        const int p = rpair[2 * k], q = rpair[2 * k + 1];
        if (q >= r) continue;
        const double c = rot[4 * k], s = rot[4 * k + 1];
        const c2 ep = {rot[4 * k + 2], rot[4 * k + 3]}, em = {rot[4 * k + 2], -rot[4 * k + 3]};
        const c2 x = A[p * r + cc], y = A[q * r + cc];
        const c2 t1 = cm(ep, y), t2 = cm(em, x);
        A[p * r + cc] = {c * x.r - s * t1.r, c * x.i - s * t1.i};
        A[q * r + cc] = {s * t2.r + c * y.r, s * t2.i + c * y.i};
      }
      __syncthreads();
    }
  }
}

size_t ritz_small_work_doubles(int q) { return (size_t)6 * q * q * 2 + 8 * (size_t)q + 64; }

__global__ __launch_bounds__(RT) void k_ritz_small(const c2* __restrict__ G, const c2* __restrict__ H,
                                                   int q, int want, double zero_thr, double drop_rel,
                                                   double* __restrict__ work, c2* __restrict__ Y,
                                                   double* __restrict__ theta, int* __restrict__ count) {
  __shared__ double sh[64];
  __shared__ double rot[4 * 128];
  __shared__ int rpair[2 * 128];
  __shared__ int keep_idx[256];
  __shared__ int sel_idx[256];
  __shared__ int nkeep, nsel;
  c2* A = reinterpret_cast<c2*>(work);
  c2* V = A + q * q;
  c2* Z = V + q * q;
  c2* T1 = Z + q * q;
  double* dsc = reinterpret_cast<double*>(T1 + q * q);   // q scale factors
  double* ev = dsc + q;                                  // q eigenvalues
  // 1. scaled G
  for (int i = threadIdx.x; i < q; i += blockDim.x) {
    const double gd = G[i * q + i].r;
    dsc[i] = gd > 0 ? 1.0 / sqrt(gd) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
    const int i = e / q, j = e % q;
    const c2 g = G[e];
    const c2 gt = G[j * q + i];
    const double s = dsc[i] * dsc[j];
    A[e] = {0.5 * (g.r + gt.r) * s, 0.5 * (g.i - gt.i) * s};
  }
  __syncthreads();
  jacobi(A, V, q, sh, rot, rpair);
  // 2. keep directions with G-eigenvalue above drop_rel * max
  if (threadIdx.x == 0) {
    double mx = 0;
    for (int i = 0; i < q; ++i) mx = fmax(mx, A[i * q + i].r);
    int c = 0;
    for (int i = 0; i < q; ++i)
      if (A[i * q + i].r > drop_rel * mx && dsc[i] >= 0) keep_idx[c++] = i;
    nkeep = c;
  }
  __syncthreads();
  const int rk = nkeep;
  // Z[:, c] = D V[:, keep_c] / sqrt(sigma)
  for (int e = threadIdx.x; e < q * rk; e += blockDim.x) {
    const int i = e / rk, c = e % rk;
    const int kk = keep_idx[c];
    const double sc = dsc[i] / sqrt(A[kk * q + kk].r);
    const c2 v = V[i * q + kk];
    Z[i * rk + c] = {v.r * sc, v.i * sc};
  }
  __syncthreads();
  // 3. T1 = H Z (q x rk), A = Z^* T1 (rk x rk), symmetrised
  for (int e = threadIdx.x; e < q * rk; e += blockDim.x) {
    const int i = e / rk, c = e % rk;
    c2 s = {0, 0};
    for (int l = 0; l < q; ++l) {
      const c2 v = cm(H[i * q + l], Z[l * rk + c]);
      s.r += v.r;
      s.i += v.i;
    }
    T1[i * rk + c] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rk * rk; e += blockDim.x) {
    const int a = e / rk, b = e % rk;
    c2 s = {0, 0};
    for (int l = 0; l < q; ++l) {
      const c2 v = cmc(Z[l * rk + a], T1[l * rk + b]);
      s.r += v.r;
      s.i += v.i;
    }
    A[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rk * rk; e += blockDim.x) {
    const int a = e / rk, b = e % rk;
    if (a < b) {
      const c2 x = A[a * rk + b], y = A[b * rk + a];
      const c2 h = {0.5 * (x.r + y.r), 0.5 * (x.i - y.i)};
      A[a * rk + b] = h;
      A[b * rk + a] = {h.r, -h.i};
    } else if (a == b) {
      A[e].i = 0.0;
    }
  }
  __syncthreads();
  jacobi(A, V, rk, sh, rot, rpair);
  // 4. ascending order (ties by index), skip values <= zero_thr, take `want`
  for (int i = threadIdx.x; i < rk; i += blockDim.x) {
    const double v = A[i * rk + i].r;
    int rank = 0;
    for (int j = 0; j < rk; ++j) {
      const double w = A[j * rk + j].r;
      if (w < v || (w == v && j < i)) ++rank;
    }
    ev[rank] = v;
    sel_idx[rank] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < rk && c < want; ++i) {
      if (ev[i] > zero_thr) {
        keep_idx[c] = sel_idx[i];
        theta[c] = ev[i];
        ++c;
      }
    }
    for (int i = c; i < want; ++i) theta[i] = 0.0;
    nsel = c;
    *count = c;
  }
  __syncthreads();
  const int ns = nsel;
  // 5. Y[:, c] = Z V[:, sel_c]
  for (int e = threadIdx.x; e < q * want; e += blockDim.x) {
    const int i = e / want, c = e % want;
    c2 s = {0, 0};
    if (c < ns) {
      const int kk = keep_idx[c];
      for (int l = 0; l < rk; ++l) {
        const c2 v = cm(Z[i * rk + l], V[l * rk + kk]);
        s.r += v.r;
        s.i += v.i;
      }
    }
    Y[i * want + c] = s;
  }
}

void ritz_small(const double* G, const double* H, int q, int want, double zero_thr,
                double drop_rel, double* work, double* Y, double* theta, int* count,
                hipStream_t st) {
  k_ritz_small<<<1, RT, 0, st>>>(reinterpret_cast<const c2*>(G), reinterpret_cast<const c2*>(H), q,
                                 want, zero_thr, drop_rel, work, reinterpret_cast<c2*>(Y), theta, count);
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
