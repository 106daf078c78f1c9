// Ritz step of the block iteration (Section 4, Ritz vectors and values) for gfx950: the
// generalised Hermitian eigenproblem  H y = theta G y  of the basis S (q <= 512 columns),
// G = S^* M S and H = S^* A S, solved in one workgroup per problem slot, in LDS:
//
//  1. unit-diagonal scaling D; pivoted Cholesky P^T (D G D) P = L L^* (the first nfix
//     columns, previous Ritz vectors, keep their order), stopped when the largest remaining
//     pivot is below drop_rel: numerically dependent directions of S are dropped (rank r);
//  2. Z = D P [L^{-*}; 0] (q x r) spans the kept directions M-orthonormally; if a kept pivot
//     was small, G2 = Z^* G Z is formed and orthonormality restored to rounding: by one
//     Newton-Schulz step Z <- Z (3I - G2)/2 when G2 is within 1e-3 of the identity (its error
//     squares), else by a second Cholesky pass;
//  3. H' = Z^* H Z (r x r) is reduced to real symmetric tridiagonal form by Householder
//     reflections and a diagonal unitary scaling;
//  4. the wanted eigenvalues (the `want` smallest above zero_thr) by Sturm-count
//     multisection, eight lanes per eigenvalue; eigenvectors of isolated eigenvalues from
//     the twisted factorisation, of clusters of close eigenvalues by inverse iteration with
//     the tridiagonal LU, re-orthogonalised inside the cluster;
//  5. back-transformation through the scaling and the reflections (eight lanes per vector,
//     each lane owning a fixed residue class of the rows), Y = Z y.
//
// The sequential parts (pivot steps, reflector steps) keep few barriers per step: the
// Cholesky pivots without moving data (one barrier per step), pivot searches and vector
// reductions are wave-level shuffle reductions, every wave computes the small reductions it
// needs itself instead of waiting for one thread, and the recurrences use a Newton-refined
// hardware reciprocal instead of division.
#include "internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace bl {

namespace {

struct c2 {
  double r, i;
};
__device__ __forceinline__ c2 cmul(c2 a, c2 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ c2 cmulc(c2 a, c2 b) { return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r}; }  // conj(a) b

// threads per workgroup: a 16 x 16 grid for q <= 48 (the register paths hold 3 x 3 entries
// per thread), a 32 x 32 grid above (register paths up to q = 96, four times the threads for
// the rest)
constexpr int GS = 8;     // lanes per eigenvalue / eigenvector group

// size of the per-index arrays (one complex, eight doubles, four ints per basis index) in
// complex units, rounded up
__host__ __device__ inline int index_block_c2(int q) { return (q * (16 + 64 + 16) + 15) / 16; }

// 1 / x from the hardware reciprocal and two Newton steps (full FP64 accuracy, without the
// long division sequence on the Sturm and factorisation recurrences)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// Cross-lane exchanges through DPP (data-parallel primitives: operand swizzles of the vector
// ALU, a few cycles) instead of LDS permutes (a round trip through the LDS crossbar each).
// Patterns within rows of 16 lanes: partner lane^1 and lane^2 (quad permutations), then the
// mirror within 8 lanes and within 16 lanes, which after the first two stages reach the
// other quad / the other half-row.  All lanes of the wave must be active.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16 lanes

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// sum over groups of 4 / 8 / 16 aligned lanes, the same value in every lane of the group
// (each stage adds two equal-order pairs, so partners agree bit for bit)
__device__ __forceinline__ double sum4(double a) {
  a += dpp_d<kDppXor1>(a);
  return a + dpp_d<kDppXor2>(a);
}
__device__ __forceinline__ double sum8(double a) { a = sum4(a); return a + dpp_d<kDppHalfMirror>(a); }
__device__ __forceinline__ double sum16(double a) { a = sum8(a); return a + dpp_d<kDppMirror>(a); }
// sum over the TG threads of a row of the TG x TG thread grid (16: one row of 16 lanes; 32:
// two, the second pair of partial sums exchanged across the half-wave)
template <int TG>
__device__ __forceinline__ double row_sum(double a) {
  a = sum16(a);
  if constexpr (TG == 32) a += __shfl_xor(a, 16, 64);
  return a;
}

__device__ __forceinline__ double wave_sum(double a) {
  a = sum16(a);
  return (readlane_d(a, 0) + readlane_d(a, 16)) + (readlane_d(a, 32) + readlane_d(a, 48));
}

// (v, idx, pos) of the partner lane replaces this lane's when larger, ties to the smaller
// index (a strict order, so both partners keep the same triple)
template <int CTRL>
__device__ __forceinline__ void pick_max(double& v, int& idx, int& pos) {
  const double ov = dpp_d<CTRL>(v);
  const int oi = dpp_i<CTRL>(idx), op = dpp_i<CTRL>(pos);
  if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; pos = op; }
}

// C (M x N, row-major, leading dimension ldc) = op(X) op(Y) on the matrix cores (FP64 MFMA
// 16x16x4, four real products per complex one), every wave of the workgroup taking 16 x 16
// output tiles in turn; op(X) = X (M x K, row-major) or, with CX, X^* for X stored K x M;
// op(Y) = Y (K x N, row-major) or, with TY, the transpose of Y stored N x K.  Columns j >= NB
// of op(Y) are taken as zero.  Operands may live in LDS or global memory; the next four-wide
// step's operands are loaded while the current one is multiplied.  Call between barriers.
typedef double rd4 __attribute__((ext_vector_type(4)));
template <bool CX, bool TY>
__device__ __forceinline__ void mm_mfma(const c2* X, int ldx, const c2* Y, int ldy, c2* C, int ldc, int M, int N,
                                        int K, int NB) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  const int r16 = lane & 15, k4 = lane >> 4;
  for (int t = wv; t < tm * tn; t += nw) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
    const int ia = i0 + r16, jb = j0 + r16;   // the operand row of X and column of Y this lane supplies
    auto lda = [&](int l) -> c2 {
      if (ia >= M || l >= K) return c2{0.0, 0.0};
      if (CX) {
        const c2 v = X[(int64_t)l * ldx + ia];
        return c2{v.r, -v.i};
      }
      return X[(int64_t)ia * ldx + l];
    };
    auto ldb = [&](int l) -> c2 {
      if (jb >= NB || l >= K) return c2{0.0, 0.0};
      return TY ? Y[(int64_t)jb * ldy + l] : Y[(int64_t)l * ldy + jb];
    };
    rd4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
    c2 a = lda(k4), b = ldb(k4);
    for (int l0 = 0; l0 < K; l0 += 4) {
      const c2 an = lda(l0 + 4 + k4), bn = ldb(l0 + 4 + k4);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.r, b.r, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.i, b.i, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.r, b.i, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.i, b.r, ci, 0, 0, 0);
      a = an;
      b = bn;
    }
    // accumulator entry v of lane (k4, r16) is C[i0 + 4 v + k4][j0 + r16]
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 4 * v + k4, j = j0 + r16;
      if (i < M && j < N) C[(int64_t)i * ldc + j] = c2{cr[v], ci[v]};
    }
  }
}

// Linv (stride ldv) = L^{-1} for lower-triangular L (stride ld, r x r).  Row i of the
// inverse depends on rows < i; four lanes share each column's inner sum.
__device__ __forceinline__ void lower_inv(const c2* L, int ld, c2* Linv, int ldv, int r) {
  const int tid = threadIdx.x, sub = tid & 3;
  for (int i = 0; i < r; ++i) {
    const double d = L[i * ld + i].r;
    for (int cb = 0; cb < r; cb += (int)blockDim.x / 4) {
      const int c = cb + tid / 4;
      c2 s = {0, 0};
      if (c < i)
        for (int l = c + sub; l < i; l += 4) {
          const c2 t = cmul(L[i * ld + l], Linv[l * ldv + c]);
          s.r += t.r;
          s.i += t.i;
        }
      s.r = sum4(s.r);
      s.i = sum4(s.i);
      if (sub == 0 && c < r) {
        c2 v = {0, 0};
        if (c == i) v = {1.0, 0.0};
        else if (c < i) v = {-s.r, -s.i};
        Linv[i * ldv + c] = {v.r / d, v.i / d};
      }
    }
    __syncthreads();
  }
}

// Unpivoted Cholesky of the Hermitian positive definite r x r matrix A (full square kept,
// overwritten); the factor's columns go to L (stride ld, lower triangle).
__device__ __forceinline__ void chol(c2* A, c2* L, int r, int ld) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < r; ++k) {
    double d = A[k * ld + k].r;
    d = d > 1e-300 ? d : 1e-300;
    const double piv = sqrt(d), invd = 1.0 / d;
    const int rem = r - k;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = k + e / rem, j = k + e % rem;
      if (j == k) {
        L[i * ld + k] = (i == k) ? c2{piv, 0.0} : c2{A[i * ld + k].r / piv, A[i * ld + k].i / piv};
      } else if (i > k) {
        const c2 t = cmulc(A[j * ld + k], A[i * ld + k]);
        A[i * ld + j] = {A[i * ld + j].r - t.r * invd, A[i * ld + j].i - t.i * invd};
      }
    }
    __syncthreads();
  }
}

// Number of eigenvalues of the real symmetric tridiagonal (d, e; e[i] couples i, i+1)
// that are below x (Sturm sequence of the LDL^T factorisation of T - x I).
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int r, double x, double tiny) {
  int c = 0;
  double qv = d[0] - x;
  if (qv < 0) ++c;
#pragma unroll 8
  for (int i = 1; i < r; ++i) {
    if (fabs(qv) < tiny) qv = qv < 0 ? -tiny : tiny;
    qv = d[i] - x - e2[i - 1] * rcp_nr(qv);
    if (qv < 0) ++c;
  }
  return c;
}

}  // namespace

// 4 matrices of q rows and stride q | 1 (at most 8 q (q + 1) doubles), then diagnostics at
// 10 q^2 + 8 q
size_t ritz_small_work_doubles(int q) { return (size_t)10 * q * q + 8 * (size_t)q + 64; }

// LDS layout (when it fits): index arrays | A | B | Z | T, each q rows of stride q | 1.
template <int MEM, int TG>
__global__ __launch_bounds__(TG * TG) void k_ritz(const c2* __restrict__ G, const c2* __restrict__ H, int q,
                                             int nfix, int want, const double* __restrict__ zthr,
                                             double drop_rel, double* __restrict__ work,
                                             size_t work_stride, c2* __restrict__ Y,
                                             double* __restrict__ theta, int* __restrict__ count,
                                             const int* __restrict__ slots) {
  extern __shared__ c2 smem[];
  // one workgroup per problem slot
  const int slot = slots ? slots[blockIdx.x] : (int)blockIdx.x;
  G += (size_t)slot * q * q;
  H += (size_t)slot * q * q;
  work += (size_t)slot * work_stride;
  Y += (size_t)slot * q * want;
  theta += (size_t)slot * want;
  count += slot;
  const double zero_thr = zthr ? zthr[slot] : -INFINITY;
  __shared__ int rank_s, second_s;
  __shared__ double red_s[16];
  // per-index arrays at the start of the dynamic LDS block, matrices after them (or in the
  // global work array when they do not fit)
  c2* phase = smem;
  double* dsc = reinterpret_cast<double*>(phase + q);
  double* dd = dsc + q;
  double* ee = dd + q;
  double* ee2 = ee + q;
  double* tau = ee2 + q;
  double* lam = tau + q;
  int* perm = reinterpret_cast<int*>(lam + q);
  int* pinv = perm + q;
  c2* gw = reinterpret_cast<c2*>(work);
  // compile-time choice, so that LDS pointers keep their address space (no flat accesses)
  // row strides are odd (q | 1 for q-wide matrices, r | 1 once the rank is known), so that
  // the rows read side by side by neighbouring lanes fall in different LDS banks
  // MEM 2: the four matrices in LDS; 1: A (the matrix being factorised, reduced or holding
  // the vectors) in LDS, B, Z, T in the work array; 0: all four in the work array
  const int lq = q | 1;
  c2* A = MEM >= 1 ? smem + index_block_c2(q) : gw;
  c2* B = (MEM == 2 ? A : gw) + q * lq;
  c2* Z = B + q * lq;
  c2* T = Z + q * lq;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  double* stamp = work + 10 * q * q + 8 * q + 1;
  if (tid == 0) { stamp[0] = (double)wall_clock64(); stamp[7] = (double)clock64(); }

  // ---- 1. scaled G and pivoted Cholesky -----------------------------------------------------
  // Implicit pivoting: A keeps the original index order; the remaining indices are a compact
  // list and the current diagonal a separate array, both double-buffered by step parity, so
  // that a step needs one barrier (pivot search and update read this step's buffers, the
  // update writes the next step's).  L_{i,k} of the original index i goes to B[i][k]; the
  // rows are put in pivot order afterwards.
  double* dg = reinterpret_cast<double*>(pinv + q);   // [2][q]
  int* rem = reinterpret_cast<int*>(dg + 2 * q);      // [2][q]
  for (int i = tid; i < q; i += nt) {
    const double gd = G[i * q + i].r;
    dsc[i] = gd > 0 ? 1.0 / sqrt(gd) : 0.0;
    rem[i] = i;
  }
  if (tid == 0) second_s = 0;
  __syncthreads();
  int r = 0;
  const int ty = tid / TG, tx = tid % TG;   // TG x TG thread grid
  if (TG == 16 && q <= 3 * TG) {
    // The matrix in registers: thread (ty, tx) holds the entries (ty + TG a, tx + TG b),
    // a, b < 3.  A step broadcasts the pivot column through LDS (colbuf, by step parity)
    // and updates every held entry; entries of already pivoted indices are updated too but
    // never read again, and their diagonal is published as -1, below every candidate, so
    // that the search runs over all indices (dead: bit mask of the pivoted indices).  Two
    // barriers per step.
    c2* colbuf = T;   // [2][q], T is free until the factor is gathered
    c2 ar[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int i = ty + TG * a, j = tx + TG * b;
        ar[a][b] = {0.0, 0.0};
        if (i < q && j < q) {
          const c2 g = G[i * q + j], gt = G[j * q + i];
          const double sc = dsc[i] * dsc[j];
          ar[a][b] = {0.5 * (g.r + gt.r) * sc, 0.5 * (g.i - gt.i) * sc};
          if (i == j) dg[i] = ar[a][b].r;
        }
      }
    __syncthreads();
    unsigned long long dead0 = 0, dead1 = 0;   // indices 0..63, 64..127
    auto is_dead = [&](int i) { return ((i < 64 ? dead0 >> i : dead1 >> (i - 64)) & 1ull) != 0; };
    for (int k = 0; k < q; ++k) {
      const double* dcur = dg + (k & 1) * q;
      double* dnext = dg + ((k + 1) & 1) * q;
      c2* col = colbuf + (k & 1) * q;
      double v;
      int idx;
      if (k < nfix) {
        idx = k;
        v = dcur[k];
      } else {
        v = -1.0;
        idx = q;
        for (int t = lane; t < q; t += 64) {
          const double dv = dcur[t];
          if (dv > v || (dv == v && t < idx)) { v = dv; idx = t; }
        }
        int pos = 0;   // unused here
        pick_max<kDppXor1>(v, idx, pos);
        pick_max<kDppXor2>(v, idx, pos);
        pick_max<kDppHalfMirror>(v, idx, pos);
        pick_max<kDppMirror>(v, idx, pos);
        double bv = readlane_d(v, 0);
        int bi = __builtin_amdgcn_readlane(idx, 0);
        for (int rw = 16; rw < 64; rw += 16) {
          const double ov = readlane_d(v, rw);
          const int oi = __builtin_amdgcn_readlane(idx, rw);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        v = bv;
        idx = bi;
      }
      if (!(v > drop_rel)) break;
      if (idx < 64) dead0 |= 1ull << idx; else dead1 |= 1ull << (idx - 64);
      if (tid == 0) {
        if (v < 1e-4) second_s = 1;
        perm[k] = idx;
      }
      const double piv = sqrt(v), rpiv = 1.0 / piv, invd = 1.0 / v;
      // the pivot column to LDS, and column k of the factor (original rows) to B
      if (tx == idx % TG) {
        const int bsel = idx / TG;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int i = ty + TG * a;
          if (i >= q) continue;
          c2 c = ar[a][0];
#pragma unroll
          for (int b = 1; b < 3; ++b) {   // component-wise selects keep ar in registers
            c.r = (bsel == b) ? ar[a][b].r : c.r;
            c.i = (bsel == b) ? ar[a][b].i : c.i;
          }
          col[i] = c;
          B[i * lq + k] = (i == idx) ? c2{piv, 0.0} : c2{c.r * rpiv, c.i * rpiv};
        }
      }
      __syncthreads();
      c2 ci[3], cj[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        ci[u] = (ty + TG * u < q) ? col[ty + TG * u] : c2{0.0, 0.0};
        cj[u] = (tx + TG * u < q) ? col[tx + TG * u] : c2{0.0, 0.0};
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const c2 t = cmulc(cj[b], ci[a]);   // A_i,idx conj(A_j,idx)
          ar[a][b] = {ar[a][b].r - t.r * invd, ar[a][b].i - t.i * invd};
        }
      if (ty == tx)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int i = ty + TG * a;
          if (i < q) dnext[i] = is_dead(i) ? -1.0 : ar[a][a].r;
        }
      __syncthreads();
      r = k + 1;
    }
    // the dropped indices follow the kept ones in index order
    if (tid == 0) {
      int t = r;
      for (int i = 0; i < q; ++i)
        if (!is_dead(i)) perm[t++] = i;
    }
  } else {
    for (int e = tid; e < q * q; e += nt) {
      const int i = e / q, j = e % q;
      const c2 g = G[e], gt = G[j * q + i];
      const double s = dsc[i] * dsc[j];
      const c2 a = {0.5 * (g.r + gt.r) * s, 0.5 * (g.i - gt.i) * s};
      A[i * lq + j] = a;
      if (i == j) dg[i] = a.r;
    }
    __syncthreads();
    for (int k = 0; k < q; ++k) {
      const double* dcur = dg + (k & 1) * q;
      double* dnext = dg + ((k + 1) & 1) * q;
      const int* rcur = rem + (k & 1) * q;
      int* rnext = rem + ((k + 1) & 1) * q;
      const int nr = q - k;
      // pivot: largest remaining diagonal, ties to the smaller index (the first nfix stay in
      // order: they lead the list); every wave finds it itself (same lanes, same order)
      double v;
      int idx, pos;
      if (k < nfix) {
        pos = 0;
        idx = rcur[0];
        v = dcur[idx];
      } else {
        v = -1.0;
        idx = q;
        pos = q;
        for (int t = lane; t < nr; t += 64) {
          const int i = rcur[t];
          const double dv = dcur[i];
          if (dv > v || (dv == v && i < idx)) { v = dv; idx = i; pos = t; }
        }
        pick_max<kDppXor1>(v, idx, pos);
        pick_max<kDppXor2>(v, idx, pos);
        pick_max<kDppHalfMirror>(v, idx, pos);
        pick_max<kDppMirror>(v, idx, pos);
        // the four rows' winners, in row order (uniform values)
        double bv = readlane_d(v, 0);
        int bi = __builtin_amdgcn_readlane(idx, 0), bp = __builtin_amdgcn_readlane(pos, 0);
        for (int rw = 16; rw < 64; rw += 16) {
          const double ov = readlane_d(v, rw);
          const int oi = __builtin_amdgcn_readlane(idx, rw), op = __builtin_amdgcn_readlane(pos, rw);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; bp = op; }
        }
        v = bv;
        idx = bi;
        pos = bp;
      }
      if (!(v > drop_rel)) break;
      if (tid == 0) {
        if (v < 1e-4) second_s = 1;
        perm[k] = idx;
      }
      const double piv = sqrt(v), invd = 1.0 / v;
      // factor column k (original rows) and the next step's list
      for (int t = tid; t < nr; t += nt) {
        const int i = rcur[t];
        const c2 a = A[i * lq + idx];
        B[i * lq + k] = (i == idx) ? c2{piv, 0.0} : c2{a.r / piv, a.i / piv};
        if (t != pos) rnext[t < pos ? t : t - 1] = i;
      }
      // trailing update of the remaining indices but idx (column idx is only read here)
      if (TG == 16 && nr <= 3 * TG) {
        // register block of up to 3 x 3 entries: every load before any store, so that the
        // loads are not held behind stores the compiler cannot tell apart
        int ib[3], jb[3];
        c2 ai[3], aj[3], cur[3][3];
  #pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int a = ty + TG * u, b = tx + TG * u;
          ib[u] = (a < nr && a != pos) ? rcur[a] : -1;
          jb[u] = (b < nr && b != pos) ? rcur[b] : -1;
        }
  #pragma unroll
        for (int u = 0; u < 3; ++u) {
          if (ib[u] >= 0) ai[u] = A[ib[u] * lq + idx];
          if (jb[u] >= 0) aj[u] = A[jb[u] * lq + idx];
        }
  #pragma unroll
        for (int v = 0; v < 3; ++v)
  #pragma unroll
          for (int u = 0; u < 3; ++u)
            if (ib[v] >= 0 && jb[u] >= 0) cur[v][u] = A[ib[v] * lq + jb[u]];
  #pragma unroll
        for (int v = 0; v < 3; ++v)
  #pragma unroll
          for (int u = 0; u < 3; ++u)
            if (ib[v] >= 0 && jb[u] >= 0) {
              const c2 t = cmulc(aj[u], ai[v]);
              const c2 nv = {cur[v][u].r - t.r * invd, cur[v][u].i - t.i * invd};
              A[ib[v] * lq + jb[u]] = nv;
              if (ib[v] == jb[u]) dnext[ib[v]] = nv.r;
            }
      } else {
        for (int a = ty; a < nr; a += TG) {
          if (a == pos) continue;
          const int i = rcur[a];
          const c2 aik = A[i * lq + idx];
          for (int b = tx; b < nr; b += TG) {
            if (b == pos) continue;
            const int j = rcur[b];
            const c2 t = cmulc(A[j * lq + idx], aik);
            const c2 nv = {A[i * lq + j].r - t.r * invd, A[i * lq + j].i - t.i * invd};
            A[i * lq + j] = nv;
            if (a == b) dnext[i] = nv.r;
          }
        }
      }
      __syncthreads();
      r = k + 1;
    }

  }
  // pivot order of the dropped indices (after the kept ones; the register path has set
  // them), and the factor's rows in pivot order into T (rows of A are free from here on)
  if (!(TG == 16 && q <= 3 * TG))
    for (int t = tid; t < q - r; t += nt) perm[r + t] = rem[(r & 1) * q + t];
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int ip = e / r, k = e % r;
    if (k <= ip) T[ip * lq + k] = B[perm[ip] * lq + k];
  }
  if (tid == 0) rank_s = r;
  __syncthreads();
  r = rank_s;
  const int lr = r | 1;
  if (tid == 0) stamp[1] = (double)wall_clock64();

  // ---- 2. Z = D P [L^{-*}; 0] -------------------------------------------------------------
  lower_inv(T, lq, A, lq, r);
  for (int i = tid; i < q; i += nt) pinv[perm[i]] = i;
  __syncthreads();
  for (int e = tid; e < q * r; e += nt) {
    const int i = e / r, c = e % r;
    const int pi = pinv[i];
    c2 z = {0.0, 0.0};
    if (pi < r && pi <= c) {
      const c2 l = A[c * lq + pi];
      z = {dsc[i] * l.r, -dsc[i] * l.i};
    }
    Z[i * lr + c] = z;
  }
  __syncthreads();
  if (second_s) {   // G2 = Z^* G Z = L2 L2^*, Z <- Z L2^{-*}
    for (int e = tid; e < q * q; e += nt) B[(e / q) * lq + e % q] = G[e];   // G into the free B region
    __syncthreads();
    mm_mfma<false, false>(B, lq, Z, lr, T, lr, q, r, q, r);
    __syncthreads();
    mm_mfma<true, false>(Z, lr, T, lr, A, lr, r, r, q, r);
    __syncthreads();
    // distance of G2 from the identity (max entry); when it is small, one Newton-Schulz step
    // Z <- Z (3I - G2) / 2 restores orthonormality to O(dev^2), else the Cholesky route
    double dloc = 0;
    for (int e = tid; e < r * r; e += nt) {
      const int i = e / r, j = e % r;
      const c2 a = A[i * lr + j];
      dloc = fmax(dloc, fabs(a.r - (i == j ? 1.0 : 0.0)) + fabs(a.i));
    }
    for (int o = 32; o > 0; o >>= 1) dloc = fmax(dloc, __shfl_xor(dloc, o, 64));
    if (lane == 0) red_s[tid >> 6] = dloc;
    __syncthreads();
    double dev = 0;
    for (int w = 0; w < (nt >> 6); ++w) dev = fmax(dev, red_s[w]);
    if (dev < 1e-3) {
      for (int e = tid; e < r * r; e += nt) {
        const int i = e / r, j = e % r;
        const c2 a = A[i * lr + j];
        A[i * lr + j] = (i == j) ? c2{1.5 - 0.5 * a.r, -0.5 * a.i} : c2{-0.5 * a.r, -0.5 * a.i};
      }
      __syncthreads();
      mm_mfma<false, false>(Z, lr, A, lr, T, lr, q, r, r, r);
    } else {
      chol(A, B, r, lr);
      lower_inv(B, lr, A, lr, r);
      for (int e = tid; e < q * r; e += nt) {
        const int i = e / r, c = e % r;
        c2 s = {0, 0};
        for (int l = 0; l <= c; ++l) {
          const c2 t = cmulc(A[c * lr + l], Z[i * lr + l]);
          s.r += t.r;
          s.i += t.i;
        }
        T[i * lr + c] = s;
      }
    }
    __syncthreads();
    for (int e = tid; e < q * lr; e += nt) Z[e] = T[e];
    __syncthreads();
  }
  if (tid == 0) stamp[2] = (double)wall_clock64();

  // ---- 3. H' = Z^* H Z (A, stride r), Hermitian part, then tridiagonalisation ----------------
  for (int e = tid; e < q * q; e += nt) B[(e / q) * lq + e % q] = H[e];   // H into the free B region
  __syncthreads();
  mm_mfma<false, false>(B, lq, Z, lr, T, lr, q, r, q, r);
  __syncthreads();
  mm_mfma<true, false>(Z, lr, T, lr, A, lr, r, r, q, r);
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int a = e / r, b = e % r;
    if (a < b) {
      const c2 x = A[a * lr + b], y = A[b * lr + a];
      const c2 h = {0.5 * (x.r + y.r), 0.5 * (x.i - y.i)};
      A[a * lr + b] = h;
      A[b * lr + a] = {h.r, -h.i};
    } else if (a == b) {
      A[a * lr + a].i = 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) stamp[3] = (double)wall_clock64();
  // Householder: at step k the column below the diagonal, x = A[k+1:, k], is mapped to
  // beta e1 by H_k = I - tau v v^* (v stored in row k of B, entries k+1..r-1); the trailing
  // block becomes H_k A22 H_k via p = tau A22 v, w = p - (tau/2)(v^* p) v,
  // A22 <- A22 - v w^* - w v^*.  T holds p.  Every wave forms the column norm and v^* p
  // itself (same lanes, same order: identical values in all waves).
  if (TG == 16 && r <= 3 * TG) {
    // The matrix in registers as in the Cholesky (thread (ty, tx) holds (ty + TG a, tx + TG b)).
    // Per step: column k through LDS (colv, by step parity), the reflector from it in every
    // wave, p = tau A22 v as per-thread partial sums combined across the TG threads of a
    // row with DPP, p through LDS (pv) for v^* p and the column side of w, then the rank-2
    // update of the held entries.  Two barriers per step.  The subdiagonal (beta) and the
    // diagonal go to A's LDS copy, where the extraction below reads them.
    c2* colv = T;             // [2][r]
    c2* pv = T + 2 * r;       // [r]
    c2 ar[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int i = ty + TG * a, j = tx + TG * b;
        ar[a][b] = (i < r && j < r) ? A[i * lr + j] : c2{0.0, 0.0};
      }
    __syncthreads();   // A's copy is written below
    for (int k = 0; k + 2 < r; ++k) {
      c2* col = colv + (k & 1) * r;
      if (tx == k % TG) {
        const int bsel = k / TG;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int i = ty + TG * a;
          if (i >= r) continue;
          c2 c = ar[a][0];
#pragma unroll
          for (int b = 1; b < 3; ++b) {
            c.r = (bsel == b) ? ar[a][b].r : c.r;
            c.i = (bsel == b) ? ar[a][b].i : c.i;
          }
          col[i] = c;
          if (i == k) dd[k] = c.r;
        }
      }
      __syncthreads();
      double part = 0;
      for (int l = lane; l < r; l += 64)
        if (l > k) {
          const c2 x = col[l];
          part += x.r * x.r + x.i * x.i;
        }
      const double xn2 = wave_sum(part);
      const c2 x0 = col[k + 1];
      const double ax0 = sqrt(x0.r * x0.r + x0.i * x0.i);
      const double sig = xn2 - ax0 * ax0;
      if (sig <= 1e-30 * xn2 || xn2 == 0.0) {   // already reduced in this column
        if (tid == 0) {
          tau[k] = 0.0;
          A[(k + 1) * lr + k] = x0;
        }
        for (int j = tid; j < r; j += nt) B[k * lr + j] = {0.0, 0.0};
        continue;
      }
      const double xn = sqrt(xn2);
      const c2 ph0 = ax0 > 0 ? c2{x0.r / ax0, x0.i / ax0} : c2{1.0, 0.0};
      const c2 beta = {-ph0.r * xn, -ph0.i * xn};
      const double tk = 1.0 / (xn2 + xn * ax0);      // 2 / (v^* v)
      // v_j: x0 - beta at k + 1, x_j below, 0 above
      auto vat = [&](int j) -> c2 {
        if (j == k + 1) return c2{x0.r - beta.r, x0.i - beta.i};
        return j > k + 1 && j < r ? col[j] : c2{0.0, 0.0};
      };
      if (tid < r) B[k * lr + tid] = vat(tid);
      if (tid == 0) {
        tau[k] = tk;
        A[(k + 1) * lr + k] = beta;
      }
      c2 vi[3], vj[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        vi[u] = vat(ty + TG * u);
        vj[u] = vat(tx + TG * u);
      }
      // p_i = tau sum_j A_ij v_j for the held rows (partials over the held columns, summed
      // across the row's TG threads)
      c2 pi[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        c2 sacc = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const c2 t = cmul(ar[a][b], vj[b]);
          sacc.r += t.r;
          sacc.i += t.i;
        }
        pi[a] = {tk * row_sum<TG>(sacc.r), tk * row_sum<TG>(sacc.i)};
        const int i = ty + TG * a;
        if (tx == 0 && i > k && i < r) pv[i] = pi[a];
      }
      __syncthreads();
      double kp = 0;
      for (int l = lane; l < r; l += 64)
        if (l > k) kp += cmulc(vat(l), pv[l]).r;
      const double Kh = 0.5 * tk * wave_sum(kp);
      c2 wi[3], wj[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        wi[u] = {pi[u].r - Kh * vi[u].r, pi[u].i - Kh * vi[u].i};
        const int j = tx + TG * u;
        const c2 pj = (j > k && j < r) ? pv[j] : c2{0.0, 0.0};
        wj[u] = {pj.r - Kh * vj[u].r, pj.i - Kh * vj[u].i};
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (ty + TG * a > k && tx + TG * b > k) {
            const c2 t1 = cmulc(wj[b], vi[a]), t2 = cmulc(vj[b], wi[a]);   // v_i conj(w_j), w_i conj(v_j)
            ar[a][b] = {ar[a][b].r - t1.r - t2.r, ar[a][b].i - t1.i - t2.i};
          }
    }
    // the last 2 x 2 block (diagonal and subdiagonal) to A's copy
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int i = ty + TG * a, j = tx + TG * b;
        if (i < r && j < r && i >= r - 2 && j >= r - 2 && j <= i) A[i * lr + j] = ar[a][b];
      }
    __syncthreads();
  } else {
    // with A in LDS and the other matrices in the work array (MEM 1), the reflector and p
    // are also kept in LDS (after A) for the products; the reflector still goes to B for the
    // back-transformation
    c2* vst = MEM == 1 ? A + q * lq : nullptr;
    c2* pv = MEM == 1 ? vst + q : T;
    for (int k = 0; k + 2 < r; ++k) {
      const int m = r - k - 1;
      double part = 0;
      for (int j = lane; j < m; j += 64) {
        const c2 x = A[(k + 1 + j) * lr + k];
        part += x.r * x.r + x.i * x.i;
      }
      const double xn2 = wave_sum(part);
      const c2 x0 = A[(k + 1) * lr + k];
      const double ax0 = sqrt(x0.r * x0.r + x0.i * x0.i);
      const double sig = xn2 - ax0 * ax0;
      if (sig <= 1e-30 * xn2 || xn2 == 0.0) {   // already reduced in this column
        if (tid == 0) { tau[k] = 0.0; dd[k] = A[k * lr + k].r; }
        for (int j = tid; j < r; j += nt) B[k * lr + j] = {0.0, 0.0};
        __syncthreads();
        continue;
      }
      const double xn = sqrt(xn2);
      const c2 ph0 = ax0 > 0 ? c2{x0.r / ax0, x0.i / ax0} : c2{1.0, 0.0};
      const c2 beta = {-ph0.r * xn, -ph0.i * xn};
      const double tk = 1.0 / (xn2 + xn * ax0);      // 2 / (v^* v)
      for (int j = tid; j < r; j += nt) {
        c2 vj = {0.0, 0.0};
        if (j == k + 1) vj = {x0.r - beta.r, x0.i - beta.i};
        else if (j > k + 1) vj = A[j * lr + k];
        B[k * lr + j] = vj;
        if (MEM == 1) vst[j] = vj;
      }
      if (tid == 0) { tau[k] = tk; dd[k] = A[k * lr + k].r; }
      __syncthreads();
      const c2* v = MEM == 1 ? vst : B + k * lr;
      {   // p = tau A22 v, four lanes per row
        const int sub = tid & 3;
        for (int rb = 0; rb < m; rb += nt / 4) {
          const int i = rb + tid / 4;
          c2 s = {0, 0};
          if (i < m) {
            const c2* row = A + (k + 1 + i) * lr + k + 1;
            for (int l = sub; l < m; l += 4) {
              const c2 t = cmul(row[l], v[k + 1 + l]);
              s.r += t.r;
              s.i += t.i;
            }
          }
          s.r = sum4(s.r);
          s.i = sum4(s.i);
          if (sub == 0 && i < m) pv[i] = {tk * s.r, tk * s.i};
        }
      }
      __syncthreads();
      double kp = 0;
      for (int i = lane; i < m; i += 64) kp += cmulc(v[k + 1 + i], pv[i]).r;
      const double Kh = 0.5 * tk * wave_sum(kp);
      if (TG == 16 && m <= 3 * TG) {
        // register block of up to 3 x 3 entries, all loads before the stores (as in the
        // Cholesky update)
        c2 vi[3], wi[3], vj[3], wj[3], cur[3][3];
  #pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int i = ty + TG * u, j = tx + TG * u;
          if (i < m) {
            vi[u] = v[k + 1 + i];
            const c2 pi = pv[i];
            wi[u] = {pi.r - Kh * vi[u].r, pi.i - Kh * vi[u].i};
          }
          if (j < m) {
            vj[u] = v[k + 1 + j];
            const c2 pj = pv[j];
            wj[u] = {pj.r - Kh * vj[u].r, pj.i - Kh * vj[u].i};
          }
        }
  #pragma unroll
        for (int a = 0; a < 3; ++a)
  #pragma unroll
          for (int b = 0; b < 3; ++b)
            if (ty + TG * a < m && tx + TG * b < m) cur[a][b] = A[(k + 1 + ty + TG * a) * lr + k + 1 + tx + TG * b];
  #pragma unroll
        for (int a = 0; a < 3; ++a)
  #pragma unroll
          for (int b = 0; b < 3; ++b)
            if (ty + TG * a < m && tx + TG * b < m) {
              const c2 t1 = cmulc(wj[b], vi[a]), t2 = cmulc(vj[b], wi[a]);   // v_i conj(w_j), w_i conj(v_j)
              A[(k + 1 + ty + TG * a) * lr + k + 1 + tx + TG * b] = {cur[a][b].r - t1.r - t2.r,
                                                                      cur[a][b].i - t1.i - t2.i};
            }
      } else {
        for (int i = ty; i < m; i += TG) {
          const c2 vi = v[k + 1 + i];
          const c2 wi = {pv[i].r - Kh * vi.r, pv[i].i - Kh * vi.i};
          for (int j = tx; j < m; j += TG) {
            const c2 vj = v[k + 1 + j];
            const c2 wj = {pv[j].r - Kh * vj.r, pv[j].i - Kh * vj.i};
            const c2 t1 = cmulc(wj, vi), t2 = cmulc(vj, wi);   // v_i conj(w_j), w_i conj(v_j)
            c2& a = A[(k + 1 + i) * lr + k + 1 + j];
            a = {a.r - t1.r - t2.r, a.i - t1.i - t2.i};
          }
        }
      }
      if (tid == 0) A[(k + 1) * lr + k] = beta;   // column k: outside the updated block
      __syncthreads();
    }
  }
  // real tridiagonal: T' = Phi^* T Phi with Phi = diag(phase), off-diagonals |T_{k+1,k}|
  if (tid == 0) {
    for (int k = (r >= 2 ? r - 2 : 0); k < r; ++k) dd[k] = A[k * lr + k].r;
    phase[0] = {1.0, 0.0};
    for (int k = 0; k + 1 < r; ++k) {
      const c2 b = A[(k + 1) * lr + k];
      const double ab = sqrt(b.r * b.r + b.i * b.i);
      ee[k] = ab;
      ee2[k] = ab * ab;
      // phase[k+1] = phase[k] * b / |b|
      const c2 u = ab > 0 ? c2{b.r / ab, b.i / ab} : c2{1.0, 0.0};
      phase[k + 1] = cmul(phase[k], u);
    }
    if (r >= 1) { ee[r - 1] = 0.0; ee2[r - 1] = 0.0; }
  }
  __syncthreads();
  if (tid == 0) stamp[4] = (double)wall_clock64();

  // ---- 4. wanted eigenvalues (multisection) and eigenvectors (inverse iteration) ----------
  double tn = 0;   // infinity norm of the tridiagonal
  for (int i = 0; i < r; ++i) tn = fmax(tn, fabs(dd[i]) + (i > 0 ? ee[i - 1] : 0.0) + ee[i]);
  const double lo0 = -tn - 1.0, hi0 = tn + 1.0;
  const double tiny = 1e-300 + 1e-16 * tn * 1e-10;
  const int nz = (zero_thr > lo0) ? sturm_count(dd, ee2, r, zero_thr * (1 + 1e-14) + 1e-300, tiny) : 0;
  const int ns = min(want, r - nz);
  {
    // eight lanes per eigenvalue: each round splits [lo, hi] at 7 interior points and keeps
    // the eighth that holds the (nz + j)-th eigenvalue (all lanes of a group agree)
    const int sub = tid % GS;
    for (int jb = 0; jb < ns; jb += nt / GS) {
      const int j = jb + tid / GS;
      if (j < ns) {
        const int target = nz + j;
        double lo = lo0, hi = hi0;
        for (int it = 0; it < 100; ++it) {
          if (!(hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
          const double x = lo + (hi - lo) * (double)(sub + 1) / (double)GS;
          const bool inside = sub < GS - 1 && x > lo && x < hi;
          const int c = inside ? sturm_count(dd, ee2, r, x, tiny) : -1;
          double nlo = (inside && c <= target) ? x : lo;
          double nhi = (inside && c > target) ? x : hi;
          // combine the group of eight (GS) lanes: max of the lower, min of the upper ends
          nlo = fmax(nlo, dpp_d<kDppXor1>(nlo));
          nhi = fmin(nhi, dpp_d<kDppXor1>(nhi));
          nlo = fmax(nlo, dpp_d<kDppXor2>(nlo));
          nhi = fmin(nhi, dpp_d<kDppXor2>(nhi));
          nlo = fmax(nlo, dpp_d<kDppHalfMirror>(nlo));
          nhi = fmin(nhi, dpp_d<kDppHalfMirror>(nhi));
          if (nlo == lo && nhi == hi) break;   // no representable interior point left
          lo = nlo;
          hi = nhi;
        }
        if (sub == 0) lam[j] = 0.5 * (lo + hi);
      }
    }
  }
  __syncthreads();
  if (tid == 0) stamp[9] = (double)wall_clock64();
  // Eigenvectors: an isolated eigenvalue's from the twisted factorisation (one thread each);
  // eigenvalues closer than 1e-6 tn form a cluster, whose vectors come from inverse iteration
  // on T' - lambda I with partial pivoting, one wave per cluster: every lane factorises and
  // solves for one member, and after each of the three solves the members are Gram-Schmidt-
  // orthogonalised in order (lanes over the rows, wave reductions).  Real vectors of length r
  // are kept in T (as doubles): vec j at xs + j*r.  Per index j the LU of T' - lambda_j I
  // (3 arrays of length r) lies in the free A region, continued in T's tail (at most want*r +
  // 3*want*r <= 4 q^2 doubles, the size of A and T together).
  double* xs = reinterpret_cast<double*>(T);
  const int clus_in_a = (2 * q * q) / (3 * r > 0 ? 3 * r : 1);
  auto lu_at = [&](int j) -> double* {
    return j < clus_in_a ? reinterpret_cast<double*>(A) + (size_t)j * 3 * r
                         : xs + (size_t)want * r + (size_t)(j - clus_in_a) * 3 * r;
  };
  auto in_cluster = [&](int j) {
    return (j > 0 && lam[j] - lam[j - 1] <= 1e-6 * tn) || (j + 1 < ns && lam[j + 1] - lam[j] <= 1e-6 * tn);
  };
  for (int j = tid; j < ns; j += nt) {
    if (in_cluster(j)) continue;
    double* u = lu_at(j);
    double* u1 = u + r;        // L+ / D+ of the twisted factorisation
    double* lm = u1 + r;
    {
      // an isolated eigenvalue: its vector from the twisted factorisation of T' - lambda I
      // (one forward LDL^T and one backward UDU^T pass; the twist index k minimises
      // |gamma_k| = |D+_k + D-_k - (d_k - lambda)|, and z_k = 1 is propagated both ways)
      double* x = xs + (size_t)j * r;
      const double shift = lam[j];
      double dp = dd[0] - shift;
      for (int i = 0; i + 1 < r; ++i) {
        if (fabs(dp) < tiny) dp = dp < 0 ? -tiny : tiny;
        u[i] = dp;                           // D+_i
        const double l = ee[i] * rcp_nr(dp);
        u1[i] = l;                           // L+_i
        dp = dd[i + 1] - shift - l * ee[i];
      }
      if (fabs(dp) < tiny) dp = dp < 0 ? -tiny : tiny;
      u[r - 1] = dp;
      double dm = dd[r - 1] - shift;
      double best = fabs(u[r - 1]);
      int kt = r - 1;
      for (int i = r - 2; i >= 0; --i) {
        if (fabs(dm) < tiny) dm = dm < 0 ? -tiny : tiny;
        const double uu = ee[i] * rcp_nr(dm);
        lm[i] = uu;                          // U-_i
        dm = dd[i] - shift - uu * ee[i];     // D-_i
        const double gam = fabs(u[i] + dm - (dd[i] - shift));
        if (gam < best) { best = gam; kt = i; }
      }
      x[kt] = 1.0;
      double nrm = 1.0;
      for (int i = kt - 1; i >= 0; --i) {
        x[i] = -u1[i] * x[i + 1];
        nrm += x[i] * x[i];
      }
      for (int i = kt + 1; i < r; ++i) {
        x[i] = -lm[i - 1] * x[i - 1];
        nrm += x[i] * x[i];
      }
      const double inv = 1.0 / sqrt(nrm);
      for (int i = 0; i < r; ++i) x[i] *= inv;
    }
  }
  {
    const int wv = tid >> 6, nw = nt >> 6;
    int ci = 0;
    for (int j = 0; j < ns;) {
      int jend = j + 1;
      while (jend < ns && lam[jend] - lam[jend - 1] <= 1e-6 * tn) ++jend;
      if (jend - j > 1 && (ci++ % nw) == wv) {
        const int k = jend - j;
        for (int c0 = 0; c0 < k; c0 += 64) {   // members, 64 at a time (lanes)
          const int c = j + c0 + lane;
          if (c0 + lane < k) {
            double* u = lu_at(c);
            double* u1 = u + r;    // U: diagonal and first super-diagonal; the second
            double* lm = u1 + r;   // super-diagonal is e_{i+1} after a row swap, else 0.
                                   // Multipliers; a row swap is encoded as -(mult) - 4.
            const double shift = lam[c];
            // Gaussian elimination with partial pivoting of the tridiagonal T' - shift I: the
            // carried row has entries (a_i, b_i) in columns (i, i+1); the next row is
            // (e_i, d_{i+1} - shift, e_{i+1}) in columns (i, i+1, i+2).
            // u keeps the reciprocals of U's diagonal (the back substitution multiplies)
            double a_i = dd[0] - shift, b_i = ee[0];
            for (int i = 0; i < r - 1; ++i) {
              const double sub = ee[i];
              const double dnext = dd[i + 1] - shift, bnext = ee[i + 1];
              if (fabs(sub) > fabs(a_i)) {              // swap rows i and i+1
                const double rs = rcp_nr(sub);
                const double mlt = a_i * rs;
                u[i] = rs;
                u1[i] = dnext;
                lm[i] = -mlt - 4.0;                     // |mult| <= 1, so lm <= -3 marks a swap
                a_i = b_i - mlt * dnext;
                b_i = -mlt * bnext;
              } else {
                const double aa = fabs(a_i) > tiny ? a_i : (a_i < 0 ? -tiny : tiny);
                const double ra = rcp_nr(aa);
                const double mlt = sub * ra;
                u[i] = ra;
                u1[i] = b_i;
                lm[i] = mlt;                            // |mult| <= 1
                a_i = dnext - mlt * b_i;
                b_i = bnext;
              }
            }
            u[r - 1] = rcp_nr(fabs(a_i) > tiny ? a_i : (a_i < 0 ? -tiny : tiny));
            u1[r - 1] = 0.0;
            lm[r - 1] = 0.0;
            double* x = xs + (size_t)c * r;
            for (int i = 0; i < r; ++i) x[i] = 1.0 + 0.0625 * (double)((i * 7 + c * 3) % 11);
          }
        }
        for (int rep = 0; rep < 3; ++rep) {
          for (int c0 = 0; c0 < k; c0 += 64) {
            const int c = j + c0 + lane;
            if (c0 + lane < k) {
              const double* u = lu_at(c);
              const double* u1 = u + r;
              const double* lm = u1 + r;
              double* x = xs + (size_t)c * r;
              // forward: apply the row operations to x (the running entry carried in a register)
              double xi = x[0];
              for (int i = 0; i < r - 1; ++i) {
                const double l = lm[i], xn = x[i + 1];
                if (l <= -3.0) {   // swapped: new row i <- old row i+1; row i+1 <- old i - mult*old i+1
                  const double mlt = -(l + 4.0);
                  x[i] = xn;
                  xi = xi - mlt * xn;
                } else {
                  x[i] = xi;
                  xi = xn - l * xi;
                }
              }
              x[r - 1] = xi;
              // back substitution with U (reciprocal diagonal u, super u1, super-super e_{i+1}
              // on swaps; the two entries below carried in registers)
              double x1 = 0.0, x2 = 0.0;
              for (int i = r - 1; i >= 0; --i) {
                double sacc = x[i];
                if (i + 1 < r) sacc -= u1[i] * x1;
                if (i + 2 < r && lm[i] <= -3.0) sacc -= ee[i + 1] * x2;
                const double xv = sacc * u[i];
                x[i] = xv;
                x2 = x1;
                x1 = xv;
              }
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          // orthogonalise each member against the earlier ones, normalise (lanes over rows)
          for (int c = j; c < jend; ++c) {
            double* x = xs + (size_t)c * r;
            for (int pc = j; pc < c; ++pc) {
              const double* y = xs + (size_t)pc * r;
              double part = 0;
              for (int i = lane; i < r; i += 64) part += y[i] * x[i];
              const double dot = wave_sum(part);
              for (int i = lane; i < r; i += 64) x[i] -= dot * y[i];
            }
            double part = 0;
            for (int i = lane; i < r; i += 64) part += x[i] * x[i];
            const double nrm = sqrt(wave_sum(part));
            const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
            for (int i = lane; i < r; i += 64) x[i] *= inv;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
      j = jend;
    }
  }
  __syncthreads();
  if (tid == 0) stamp[5] = (double)wall_clock64();

  // ---- 5. back-transformation: y = H_0 ... H_{r-3} Phi x, then Y = Z y ----------------------
  // complex vectors of length r, column-major in the A region: yv[c * lr + i]
  c2* yv = A;
  for (int e = tid; e < ns * r; e += nt) {
    const int c = e / r, i = e % r;
    const double xv = xs[(size_t)c * r + i];
    yv[c * lr + i] = {phase[i].r * xv, phase[i].i * xv};
  }
  __syncthreads();
  {
    // eight lanes per vector; lane `sub` owns the rows i = sub mod 8 throughout, so the
    // reflections need no barrier (v^* y is combined by shuffles inside the group)
    const int sub = tid % GS;
    for (int cb = 0; cb < ns; cb += nt / GS) {
      const int c = cb + tid / GS;
      if (c < ns) {
        c2* y = yv + (size_t)c * lr;
        for (int k = r - 3; k >= 0; --k) {
          const double tk = tau[k];
          if (tk == 0.0) continue;
          const c2* v = B + k * lr;
          const int i0 = k + 1 + ((sub - (k + 1)) % GS + GS) % GS;
          c2 s = {0, 0};
          for (int i = i0; i < r; i += GS) {
            const c2 t = cmulc(v[i], y[i]);
            s.r += t.r;
            s.i += t.i;
          }
          s.r = sum8(s.r);   // the vector's eight lanes (GS)
          s.i = sum8(s.i);
          for (int i = i0; i < r; i += GS) {
            const c2 t = cmul(v[i], s);
            y[i] = {y[i].r - tk * t.r, y[i].i - tk * t.i};
          }
        }
      }
    }
  }
  __syncthreads();
  // Y (q x want) = Z (q x r) y; columns ns..want-1 zero
  mm_mfma<false, true>(Z, lr, yv, lr, Y, want, q, want, r, ns);
  for (int c = tid; c < want; c += nt) theta[c] = c < ns ? lam[c] : 0.0;
  if (tid == 0) {
    *count = ns;
    work[10 * q * q + 8 * q] = (double)r;       // diagnostic: kept rank
    stamp[5 + 1] = (double)wall_clock64();
    stamp[8] = (double)clock64();
  }
}

static int g_cap = -1;

void ritz_small(const double* G, const double* H, int q, int nfix, int want, const double* zthr,
                double drop_rel, double* work, size_t work_stride, double* Y, double* theta,
                int* count, const Launch& L) {
  if (g_cap < 0) {
    int dev = 0, cap = 65536;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) cap = 65536;
    cap -= 1024;   // the kernel's static LDS (scalars) is below 1 KB
    bool ok = cap > 0;
    const void* fns[6] = {(const void*)k_ritz<0, 16>, (const void*)k_ritz<1, 16>, (const void*)k_ritz<2, 16>,
                          (const void*)k_ritz<0, 32>, (const void*)k_ritz<1, 32>, (const void*)k_ritz<2, 32>};
    for (const void* f : fns)
      if (ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, cap) != hipSuccess) ok = false;
    if (!ok)
      cap = 64 * 1024 - 1024;
    g_cap = cap > 0 ? cap : 0;
    if (std::getenv("BL_DEBUG")) std::fprintf(stderr, "bloch: ritz dynamic LDS cap %d bytes\n", g_cap);
  }
  if (L.nact <= 0) return;
  const size_t idx = (size_t)index_block_c2(q) * sizeof(c2);
  const size_t need = idx + (size_t)4 * q * (q | 1) * sizeof(c2);
  const size_t need1 = idx + ((size_t)q * (q | 1) + 2 * (size_t)q) * sizeof(c2);
  const int mem = need <= (size_t)g_cap ? 2 : (need1 <= (size_t)g_cap ? 1 : 0);
  const size_t lds = mem == 2 ? need : (mem == 1 ? need1 : idx);
  const c2* g = reinterpret_cast<const c2*>(G);
  const c2* h = reinterpret_cast<const c2*>(H);
  c2* y = reinterpret_cast<c2*>(Y);
#define BL_RITZ(M, TGV)                                                                                    \
  k_ritz<M, TGV><<<L.nact, TGV * TGV, lds, L.st>>>(g, h, q, nfix, want, zthr, drop_rel, work, work_stride, y, \
                                                   theta, count, L.slots)
  if (q <= 48) {
    if (mem == 2) BL_RITZ(2, 16);
    else if (mem == 1) BL_RITZ(1, 16);
    else BL_RITZ(0, 16);
  } else {
    if (mem == 2) BL_RITZ(2, 32);
    else if (mem == 1) BL_RITZ(1, 32);
    else BL_RITZ(0, 32);
  }
#undef BL_RITZ
}

}  // namespace bl
