// Device helpers shared by the stencil kernels: complex arithmetic, Bloch-extended reads
// and writes ("extended" coordinates: a vector index outside [0,n) x [0,m) is read through
// the Bloch extension u(j1 + s1 n, j2 + s2 m) = alpha^s1 beta^s2 u(j1, j2)), slot/column
// addressing of batched launches and the cell curl.
#pragma once

#include "internal.h"

// No contraction into FMAs in these helpers either: they are inlined into the per-level
// kernels and the fused coarse cycles alike, which must round identically.
#pragma clang fp contract(off)

namespace bl {

template <typename T>
struct Cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, T br, T bi) {
  return {a.re * br - a.im * bi, a.re * bi + a.im * br};
}

// Phases in the kernel's arithmetic type.
template <typename T>
struct Ph {
  T ar, ai, br, bi;
};
template <typename T>
__host__ __device__ inline Ph<T> cast_phase(const Phase& p) {
  return {(T)p.ar, (T)p.ai, (T)p.br, (T)p.bi};
}

// Read component `off` (0 for x-edges / nodes, nm for y-edges) at extended (j1, j2),
// j1 in [-n, 2n), j2 in [-m, 2m).
template <typename TS, typename T>
__device__ __forceinline__ Cx<T> fetch(const TS* __restrict__ col, int64_t N, int n, int m,
                                       int64_t off, int j1, int j2, const Ph<T>& p) {
  int s1 = 0, s2 = 0;
  if (j1 < 0) { j1 += n; s1 = -1; } else if (j1 >= n) { j1 -= n; s1 = 1; }
  if (j2 < 0) { j2 += m; s2 = -1; } else if (j2 >= m) { j2 -= m; s2 = 1; }
  const int64_t i = off + (int64_t)j2 * n + j1;
  Cx<T> v = {(T)col[i], (T)col[N + i]};
  if (s1 > 0) v = cmul(v, p.ar, p.ai);
  else if (s1 < 0) v = cmul(v, p.ar, -p.ai);
  if (s2 > 0) v = cmul(v, p.br, p.bi);
  else if (s2 < 0) v = cmul(v, p.br, -p.bi);
  return v;
}

// Add delta (given in extended coordinates) to the stored value at extended (j1, j2),
// j1 in [-1, n), j2 in [-1, m): u_can = conj(phase) * u_ext.
template <typename TS, typename T>
__device__ __forceinline__ void add_ext(TS* __restrict__ col, int64_t N, int n, int m, int64_t off,
                                        int j1, int j2, Cx<T> d, const Ph<T>& p) {
  if (j1 < 0) { j1 += n; d = cmul(d, p.ar, p.ai); }
  if (j2 < 0) { j2 += m; d = cmul(d, p.br, p.bi); }
  const int64_t i = off + (int64_t)j2 * n + j1;
  col[i] = (TS)((T)col[i] + d.re);
  col[N + i] = (TS)((T)col[N + i] + d.im);
}

__device__ __forceinline__ int wrapi(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// Slot and in-slot column of this block (grid.y = active slots * columns per slot).
struct SJ {
  int slot, j;
};
__device__ __forceinline__ SJ slot_col(const int* slots, int ncps) {
  const int si = (int)blockIdx.y / ncps;
  return {slots ? slots[si] : si, (int)blockIdx.y % ncps};
}
template <typename T>
__device__ __forceinline__ T* colp(View<T> v, SJ s, int64_t N) {
  return v.p + ((int64_t)s.slot * v.cps + v.off + s.j) * 2 * N;
}

// Plane wave w_j = exp(i t1 j1) exp(i t2 j2) of a slot from its factor tables.
__device__ __forceinline__ Cx<double> pw_value(const PWDefl& d, int slot, int n, int j1, int j2) {
  const double* t = d.tab + (int64_t)slot * d.tabstride;
  const double ar = t[2 * j1], ai = t[2 * j1 + 1];
  const double br = t[2 * (n + j2)], bi = t[2 * (n + j2) + 1];
  return {ar * br - ai * bi, ar * bi + ai * br};
}

// Sum of (a, b) over the workgroup (waves of 64, at most 1024 threads) in a fixed order;
// thread 0 stores it at out[0..1].
__device__ __forceinline__ void block_sum2(double a, double b, double* out) {
  __shared__ double sh[2][16];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wv] = a; sh[1][wv] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0, tb = 0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) { ta += sh[0][w]; tb += sh[1][w]; }
    out[0] = ta;
    out[1] = tb;
  }
}

// (i mod n, i / n) in 32-bit unsigned arithmetic, for 0 <= i < 2^32 (node and edge indices of
// a level fit); a 64-bit division costs several times as many instructions
__device__ __forceinline__ void split_index(int64_t i, int n, int& j1, int& j2) {
  const unsigned u = (unsigned)i, q = u / (unsigned)n;
  j2 = (int)q;
  j1 = (int)(u - q * (unsigned)n);
}

// Block order that gives each of the 8 XCDs (which receive the blocks round-robin) one
// contiguous range of logical blocks, so that the rows shared by neighbouring blocks stay in
// one L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

template <typename T>
__device__ __forceinline__ T kap(const double* k64, const float* k32, int64_t i);
template <>
__device__ __forceinline__ double kap<double>(const double* k64, const float*, int64_t i) { return k64[i]; }
template <>
__device__ __forceinline__ float kap<float>(const double*, const float* k32, int64_t i) { return k32[i]; }

// Cell curl (circulation) of cell (c1, c2), extended c in [-1, n).
template <typename TS, typename T>
__device__ __forceinline__ Cx<T> cell_curl(const TS* col, int64_t N, int n, int m, int64_t nm,
                                           int c1, int c2, const Ph<T>& p) {
  return fetch<TS, T>(col, N, n, m, 0, c1, c2 + 1, p) - fetch<TS, T>(col, N, n, m, 0, c1, c2, p) +
         fetch<TS, T>(col, N, n, m, nm, c1, c2, p) - fetch<TS, T>(col, N, n, m, nm, c1 + 1, c2, p);
}

}  // namespace bl
