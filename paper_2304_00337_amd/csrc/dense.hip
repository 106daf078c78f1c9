// Dense kernels of the iteration (Section 4 and 5) for gfx950:
//  * coarsest-level direct solve: the coarse operator is assembled by applying the stencil
//    to unit vectors, inverted in place by Gauss-Jordan (Hermitian positive definite, no
//    pivoting) in one workgroup, and applied as a dense matrix-vector product;
//  * tall-skinny Gram products X^* W of planar FP64 blocks (LDS-staged, register-tiled);
//  * block recombination S Y.
#include "internal.h"

#include <type_traits>

#include <cmath>
#include <cstdio>
#include <cstdlib>

// The coarse solve is repeated inside the fused coarse cycles (coarse.hip) with the same
// operations; no contraction on either side keeps the two bit-identical.
#pragma clang fp contract(off)

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

// mat_s (row-major interleaved) [i][j] = column j of slot s's probe result at row i
__global__ void k_planar_to_matrix(const double* __restrict__ cols, int64_t n, double* __restrict__ mat,
                                   const int* __restrict__ slots) {
  const int64_t j = blockIdx.y;
  const int64_t s = slots ? slots[blockIdx.z] : blockIdx.z;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* c = cols + s * n * 2 * n;
  double* o = mat + s * n * n * 2;
  o[2 * (i * n + j)] = c[j * 2 * n + i];
  o[2 * (i * n + j) + 1] = c[j * 2 * n + n + i];
}
void planar_to_matrix(const double* cols, int64_t n, double* mat, const Launch& L) {
  if (L.nact <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)L.nact);
  k_planar_to_matrix<<<grid, 256, 0, L.st>>>(cols, n, mat, L.slots);
}

__global__ void k_add_rank_one(double* __restrict__ mat, int64_t n, double gamma, const int* __restrict__ slots) {
  const int64_t s = slots ? slots[blockIdx.y] : blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) mat[s * n * n * 2 + 2 * e] += gamma / (double)n;
}
void add_constant_rank_one(double* mat, int64_t n, double gamma, const Launch& L) {
  if (L.nact <= 0) return;
  k_add_rank_one<<<dim3((unsigned)((n * n + 255) / 256), (unsigned)L.nact), 256, 0, L.st>>>(mat, n, gamma, L.slots);
}

// In-place Gauss-Jordan inversion of a Hermitian positive definite matrix (no pivoting),
// one workgroup per slot.
__global__ __launch_bounds__(1024) void k_invert(c2* __restrict__ A, int n, const int* __restrict__ slots) {
  extern __shared__ c2 colk[];
  __shared__ c2 piv;
  A += (int64_t)(slots ? slots[blockIdx.x] : (int)blockIdx.x) * n * n;
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
void invert_hpd(double* mat, int64_t n, const Launch& L) {
  if (L.nact <= 0) return;
  k_invert<<<L.nact, 1024, (size_t)n * sizeof(c2), L.st>>>(reinterpret_cast<c2*>(mat), (int)n, L.slots);
}

__global__ void k_mat_to_float(const double* __restrict__ in, float* __restrict__ out, int64_t count,
                               const int* __restrict__ slots) {
  const int64_t s = slots ? slots[blockIdx.y] : blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[s * count + i] = (float)in[s * count + i];
}
void matrix_to_float(const double* mat, float* out, int64_t count, const Launch& L) {
  if (L.nact <= 0) return;
  k_mat_to_float<<<dim3((unsigned)((count + 255) / 256), (unsigned)L.nact), 256, 0, L.st>>>(mat, out, count, L.slots);
}

// x = Inv_s b for a Hermitian Inv_s (row-major interleaved); row i of Inv_s is read as the
// conjugate of column i, so that consecutive threads read consecutive entries.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_apply(const T* __restrict__ inv, int64_t n, View<const T> bv,
                                                     View<T> xv, const int* __restrict__ slots, int ncps) {
  const int si = (int)blockIdx.y / ncps;
  const int slot = slots ? slots[si] : si, col = (int)blockIdx.y % ncps;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  inv += (int64_t)slot * n * n * 2;
  const T* bc = bv.p + ((int64_t)slot * bv.cps + bv.off + col) * 2 * n;
  T sr = 0, si_ = 0;
  // (unrolled: the loads of several terms are in flight; the summation order is unchanged)
#pragma unroll 8
  for (int64_t l = 0; l < n; ++l) {
    const T ar = inv[2 * (l * n + i)], ai = -inv[2 * (l * n + i) + 1];
    const T br = bc[l], bi = bc[n + l];
    sr += ar * br - ai * bi;
    si_ += ar * bi + ai * br;
  }
  T* xc = xv.p + ((int64_t)slot * xv.cps + xv.off + col) * 2 * n;
  xc[i] = sr;
  xc[n + i] = si_;
}
template <typename T>
void dense_apply(const void* inv, int64_t n, View<const T> b, View<T> x, const Launch& L) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_dense_apply<T><<<grid, 256, 0, L.st>>>(reinterpret_cast<const T*>(inv), n, b, x, L.slots, L.ncps);
}
template void dense_apply<double>(const void*, int64_t, View<const double>, View<double>, const Launch&);
template void dense_apply<float>(const void*, int64_t, View<const float>, View<float>, const Launch&);

// ------------------------------------------------------------------------------------------
// Gram products.  Block (16 x 16 threads) computes a 64 x 64 tile of X^* W over a range of
// rows; rows are staged through LDS 16 at a time; each thread owns a 4 x 4 register tile.
constexpr int GB = 64, GTR = 16;

__global__ __launch_bounds__(256) void k_gram(View<const double> Xv, int q, View<const double> Wv, int r,
                                              int64_t len, int64_t rows_per_blk,
                                              double* __restrict__ partial,
                                              const int* __restrict__ slots) {
  __shared__ double xr[GTR][GB], xi[GTR][GB], wr[GTR][GB], wi[GTR][GB];
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  const double* X = Xv.p + ((int64_t)slot * Xv.cps + Xv.off) * 2 * len;
  const double* W = Wv.p + ((int64_t)slot * Wv.cps + Wv.off) * 2 * len;
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
  double* pp = partial + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * q * r * 2;
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

// out_s = sum over the row blocks of the launch entry z (slot s = slots[z]) in block order
__global__ void k_gram_reduce(const double* __restrict__ partial, int nblk, int64_t count,
                              double* __restrict__ out, const int* __restrict__ slots) {
  const int z = blockIdx.y;
  const int64_t slot = slots ? slots[z] : z;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double* p = partial + (int64_t)z * nblk * count;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += p[(int64_t)b * count + e];
  out[slot * count + e] = s;
}

// Row blocks of one Gram product: a function of the vector length only, so that a slot's
// sums do not depend on which other slots share the launch.
int gram_blocks(int64_t len) {
  int64_t nb = (len + 1023) / 1024;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  int64_t rpb = (len + nb - 1) / nb;
  rpb = (rpb + GTR - 1) / GTR * GTR;
  return (int)((len + rpb - 1) / rpb);
}

int gram(View<const double> X, int q, View<const double> W, int r, int64_t len, double* partial,
         int64_t partial_cap, double* out, const Launch& L) {
  if (L.nact <= 0) return 0;
  const int nb = gram_blocks(len);
  if ((int64_t)nb * q * r * 2 * L.nact > partial_cap) return -1;
  int64_t rpb = (len + nb - 1) / nb;
  rpb = (rpb + GTR - 1) / GTR * GTR;
  const int nti = (q + GB - 1) / GB, ntj = (r + GB - 1) / GB;
  dim3 grid((unsigned)nb, (unsigned)(nti * ntj), (unsigned)L.nact);
  k_gram<<<grid, 256, 0, L.st>>>(X, q, W, r, len, rpb, partial, L.slots);
  const int64_t count = (int64_t)q * r * 2;
  k_gram_reduce<<<dim3((unsigned)((count + 255) / 256), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, count, out, L.slots);
  return 0;
}

// ------------------------------------------------------------------------------------------
// out_s[:, j] = sum_l S_s[:, l] Y_s[l][j]; thread per row, 8 output columns per workgroup.  The
// column blocks of one row range are neighbouring workgroups (blockIdx.x = range * blocks +
// column block), so they run together and read the basis rows through L2 once from memory.
namespace {

// Block combination out_s = S_s Y_s on the matrix cores (FP64 MFMA 16x16x4), computed as
// out^T = Y^T S^T so that each lane's results are consecutive rows of one output column
// (coalesced stores): the A operand is Y (staged in LDS once per workgroup, real and
// imaginary parts apart, zero-padded to whole tiles), the B operand the basis rows straight
// from memory.  A complex product takes three real ones (Gauss's three-multiplication form):
//   P1 = Yr Sr,  P2 = Yi Si,  P3 = (Yr + Yi)(Sr + Si),  Re = P1 - P2,  Im = P3 - P1 - P2,
// each summed over the basis columns in its own accumulator.  The workgroups are persistent:
// each wave walks row tiles of BCR rows (tile t, t + stride, ...) for the NTC output column
// tiles of its workgroup (blockIdx.y selects the tile group when the block is wider), one
// stream of steps of four basis columns across its tiles, with the columns two steps ahead
// (possibly of the next tile) loaded while the current ones are multiplied.  (The file is
// compiled with MFMA results in ordinary VGPRs, so the accumulators stay put across the loop.)
typedef double bd4 __attribute__((ext_vector_type(4)));
constexpr int BCW = 4;    // waves per workgroup
constexpr int BCR = 32;   // rows per tile (two 16-row MFMA tiles)

template <int NTC>
__global__ __launch_bounds__(64 * BCW) void k_block_combine(View<const double> Sv, int q, const c2* __restrict__ Y,
                                                            int want, int64_t len, View<double> ov,
                                                            const int* __restrict__ slots) {
  extern __shared__ double yl[];   // yr then yi, each q4 x 16 NTC
  constexpr int WC = 16 * NTC;
  const int q4 = (q + 3) & ~3;
  const int cbase = (int)blockIdx.y * WC;   // first output column of the workgroup
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  const double* S = Sv.p + ((int64_t)slot * Sv.cps + Sv.off) * 2 * len;
  double* out = ov.p + ((int64_t)slot * ov.cps + ov.off) * 2 * len;
  Y += (int64_t)slot * q * want;
  double* yr = yl;
  double* yi = yl + (size_t)q4 * WC;
  {
    // all of a thread's loads first, then the stores
    constexpr int PER = 8;
    for (int e0 = threadIdx.x; e0 < q4 * WC; e0 += PER * (int)blockDim.x) {
      c2 v[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * (int)blockDim.x, l = e / WC, c = cbase + e % WC;
        v[u] = (e < q4 * WC && l < q && c < want) ? Y[(int64_t)l * want + c] : c2{0, 0};
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < q4 * WC) {
          yr[e] = v[u].r;
          yi[e] = v[u].i;
        }
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t ntiles = (len + BCR - 1) / BCR;
  const int64_t tstride = (int64_t)gridDim.x * BCW;
  int64_t ct = (int64_t)blockIdx.x * BCW + wv;   // tile being multiplied
  if (ct >= ntiles) return;
  const int kk = lane >> 4, cc = lane & 15;
  bd4 p1[2][NTC], p2[2][NTC], p3[2][NTC];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int c = 0; c < NTC; ++c) p1[rt][c] = p2[rt][c] = p3[rt][c] = bd4{0, 0, 0, 0};
  // basis column l0 + kk of this lane's two rows of tile t (zero past the basis, the rows or
  // the last tile)
  auto load = [&](int64_t t, int l0, double* sr, double* si) {
    const int l = l0 + kk;
    const int64_t off = (int64_t)(l < q ? l : q - 1) * 2 * len;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t row = t * BCR + 16 * rt + cc;
      const bool ok = t < ntiles && l < q && row < len;
      const double* rp = S + (ok ? row : 0) + (ok ? off : 0);
      const double a = rp[0], b = rp[len];
      sr[rt] = ok ? a : 0.0;
      si[rt] = ok ? b : 0.0;
    }
  };
  // prefetch position (tile pt, columns pl0 ..), two steps ahead of the multiplication
  int64_t pt = ct;
  int pl0 = 0;
  auto advance = [&]() {
    pl0 += 4;
    if (pl0 >= q4) {
      pl0 = 0;
      pt += tstride;
    }
  };
  double s0r[2], s0i[2], s1r[2], s1i[2], s2r[2], s2i[2];
  load(pt, pl0, s0r, s0i);
  advance();
  load(pt, pl0, s1r, s1i);
  advance();
  int cl0 = 0;
  for (;;) {
    load(pt, pl0, s2r, s2i);
    advance();
    const int l = cl0 + kk;
    double ss[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) ss[rt] = s0r[rt] + s0i[rt];
#pragma unroll
    for (int c = 0; c < NTC; ++c) {
      const double yre = yr[l * WC + 16 * c + cc], yim = yi[l * WC + 16 * c + cc];
      const double ys = yre + yim;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        p1[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(yre, s0r[rt], p1[rt][c], 0, 0, 0);
        p2[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(yim, s0i[rt], p2[rt][c], 0, 0, 0);
        p3[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ys, ss[rt], p3[rt][c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      s0r[rt] = s1r[rt];
      s0i[rt] = s1i[rt];
      s1r[rt] = s2r[rt];
      s1i[rt] = s2i[rt];
    }
    cl0 += 4;
    if (cl0 < q4) continue;
    // tile ct done: accumulator entry v of lane (kk, cc) is output column 16 c + 4 v + kk of
    // row 16 rt + cc of the tile (the 16 x 16 result of the instruction has row 4 v + lane / 16
    // and column lane % 16)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t row = ct * BCR + 16 * rt + cc;
#pragma unroll
      for (int c = 0; c < NTC; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = cbase + 16 * c + 4 * v + kk;
          if (col < want && row < len) {
            const double a = p1[rt][c][v], b = p2[rt][c][v];
            out[(int64_t)col * 2 * len + row] = a - b;
            out[(int64_t)col * 2 * len + len + row] = (p3[rt][c][v] - a) - b;
          }
        }
    }
    ct += tstride;
    if (ct >= ntiles) break;
    cl0 = 0;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int c = 0; c < NTC; ++c) p1[rt][c] = p2[rt][c] = p3[rt][c] = bd4{0, 0, 0, 0};
  }
}

}  // namespace

void block_combine(View<const double> S, int q, const double* Y, int want, int64_t len,
                   View<double> out, const Launch& L) {
  if (L.nact <= 0 || want <= 0) return;
  const int q4 = (q + 3) & ~3;
  const int ntc = (want + 15) / 16;
  // column tiles per workgroup: up to three, as many as the staged Y allows in 160 KB of LDS
  const size_t tile_lds = (size_t)2 * q4 * 16 * sizeof(double);
  int per = 3;
  while (per > 1 && tile_lds * per > (size_t)160 * 1024) --per;
  if (per > ntc) per = ntc;
  const int ny = (ntc + per - 1) / per;
  // persistent workgroups: as many as stay resident together (by LDS, at most two per compute
  // unit), spread over the column groups and slots of the launch
  static const int cus = [] {   // initialised once, thread-safely
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    return c;
  }();
  const int per_cu = tile_lds * per <= (size_t)80 * 1024 ? 2 : 1;
  const int64_t tiles_wg = ((len + BCR - 1) / BCR + BCW - 1) / BCW;
  int64_t nx = ((int64_t)cus * per_cu + (int64_t)ny * L.nact - 1) / ((int64_t)ny * L.nact);
  if (nx < 1) nx = 1;
  if (nx > tiles_wg) nx = tiles_wg;
  const dim3 grid((unsigned)nx, (unsigned)ny, (unsigned)L.nact);
  auto go = [&](auto nt) {
    constexpr int NTC = decltype(nt)::value;
    static const bool attr = [&] {   // once per instantiation, thread-safely
      (void)hipFuncSetAttribute((const void*)k_block_combine<NTC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
      return true;
    }();
    (void)attr;
    k_block_combine<NTC><<<grid, 64 * BCW, tile_lds * NTC, L.st>>>(S, q, reinterpret_cast<const c2*>(Y), want, len,
                                                                  out, L.slots);
  };
  if (per == 1) go(std::integral_constant<int, 1>{});
  else if (per == 2) go(std::integral_constant<int, 2>{});
  else go(std::integral_constant<int, 3>{});
}

// ------------------------------------------------------------------------------------------
// In-place column compaction: column k of the view receives column src[k] (k < ncols,
// src[k] >= k, strictly increasing per slot).  Every thread owns one 16-byte position of
// all columns, so threads never touch each other's data; a thread loads a chunk of source
// columns before it stores them (a destination may be the source of a later column of the
// chunk), and a later chunk's sources lie above every earlier destination.
template <typename T>
__global__ void k_compact_cols(View<T> v, int64_t len, const int* __restrict__ src, int src_stride, int ncols,
                               const int* __restrict__ slots) {
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int CH = 8;
  const int z = blockIdx.y;
  const int sl = slots ? slots[z] : z;
  const int* sk = src + (int64_t)z * src_stride;
  const int64_t nvec = 2 * len * (int64_t)sizeof(T) / (int64_t)sizeof(V);
  V* base = reinterpret_cast<V*>(v.p + ((int64_t)sl * v.cps + v.off) * 2 * len);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += (int64_t)gridDim.x * blockDim.x) {
    for (int k0 = 0; k0 < ncols; k0 += CH) {
      V buf[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int k = k0 + u;
        if (k < ncols && sk[k] != k) buf[u] = base[(int64_t)sk[k] * nvec + i];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int k = k0 + u;
        if (k < ncols && sk[k] != k) base[(int64_t)k * nvec + i] = buf[u];
      }
    }
  }
}
template <typename T>
void compact_cols(View<T> v, int64_t len, const int* src, int src_stride, int ncols, const Launch& L) {
  if (L.nact <= 0 || ncols <= 0) return;
  const int64_t nvec = 2 * len * (int64_t)sizeof(T) / 16;
  int64_t nb = (nvec + 255) / 256;
  if (nb > 2048) nb = 2048;
  k_compact_cols<T><<<dim3((unsigned)nb, (unsigned)L.nact), 256, 0, L.st>>>(v, len, src, src_stride, ncols, L.slots);
}
template void compact_cols<float>(View<float>, int64_t, const int*, int, int, const Launch&);
template void compact_cols<double>(View<double>, int64_t, const int*, int, int, const Launch&);

}  // namespace bl
