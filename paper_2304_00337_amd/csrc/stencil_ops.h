// Per-point bodies of the stencil kernels (Sections 3-5), shared by the per-level kernels of
// stencils.hip and the fused coarse-level V-cycles of coarse.hip, so that both perform the
// same operations in the same order (and, with contraction off, round identically).
// Vectors are planar (re at [0, N), im at [N, 2N)) and read in Bloch-extended coordinates.
#pragma once

#include "stencil_common.h"

#include <type_traits>

#pragma clang fp contract(off)

namespace bl {

// Edge values around a patch node (p1, p2), given in canonical indices, read and updated in
// Bloch-extended coordinates: get(c, d1, d2) is component c (0 = x-edges, 1 = y-edges) at
// (p1 + d1, p2 + d2) times the phase of the crossing, add(c, d1, d2, v) adds v (given in
// extended coordinates) to the stored value.  This accessor reads a whole column in memory;
// the tiled sweeps have one over an LDS copy of a tile (same operations, same rounding).
template <typename T, typename TS = T>
struct ColumnEdges {
  TS* xc;
  int64_t N, nm;
  int n, m, p1, p2;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    return fetch<typename std::remove_const<TS>::type, T>(xc, N, n, m, c ? nm : 0, p1 + d1, p2 + d2, p);
  }
  __device__ __forceinline__ void add(int c, int d1, int d2, Cx<T> v) const {
    add_ext<T, T>(xc, N, n, m, c ? nm : 0, p1 + d1, p2 + d2, v, p);
  }
};

// The same reads for a node whose whole neighbourhood lies inside the grid (no seam): plain
// indexing, no phase.  (Identical values to ColumnEdges there.)
template <typename T, typename TS>
struct DirectEdges {
  const TS* xc;
  int64_t N, nm, d;
  int n;
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    const int64_t i = (c ? nm : 0) + d + (int64_t)d2 * n + d1;
    return {(T)xc[i], (T)xc[N + i]};
  }
};
template <typename T, typename TS>
struct DirectNodes {
  const TS* xc;
  int64_t N, d;
  int n;
  __device__ __forceinline__ Cx<T> get(int d1, int d2) const {
    const int64_t i = d + (int64_t)d2 * n + d1;
    return {(T)xc[i], (T)xc[N + i]};
  }
};

// Workgroup tiles of the point kernels: kPtW x kPtH nodes (one per thread), row-major tiles;
// `inner` (uniform in the workgroup) when every node of the tile and its 3 x 3 neighbourhood
// lie inside the grid, so that the reads need no seam handling.
constexpr int kPtW = 64, kPtH = 4;
struct PointTile {
  int p1, p2;
  bool inner;
};
__device__ __forceinline__ PointTile point_tile(int n, int m) {
  const int tiles_x = (n + kPtW - 1) / kPtW;
  // XCD-major order (consecutive blocks go to the eight XCDs in turn): each XCD takes a
  // contiguous range of tile rows, so the rows a tile shares with its neighbours above and
  // below are read through the same L2
  const int nb = (int)gridDim.x;
  const int t = nb >= 8 ? xcd_block((int)blockIdx.x, nb) : (int)blockIdx.x;
  const int tx0 = (t % tiles_x) * kPtW, ty0 = (t / tiles_x) * kPtH;
  return {tx0 + (int)(threadIdx.x % kPtW), ty0 + (int)(threadIdx.x / kPtW),
          tx0 >= 1 && tx0 + kPtW <= n - 1 && ty0 >= 1 && ty0 + kPtH <= m - 1};
}
inline int point_tiles(int n, int m) { return ((n + kPtW - 1) / kPtW) * ((m + kPtH - 1) / kPtH); }

// Workgroups that walk kPtPer consecutive tiles (k = 0 .. kPtPer - 1) of their XCD-major block
// in turn, paying the set-up (slot, phase and column pointers) once; tiles past the last are
// empty (no live point).
constexpr int kPtPer = 4;
__device__ __forceinline__ PointTile point_tile_k(int n, int m, int k) {
  const int tiles_x = (n + kPtW - 1) / kPtW;
  const int nb = (int)gridDim.x;
  const int t = (nb >= 8 ? xcd_block((int)blockIdx.x, nb) : (int)blockIdx.x) * kPtPer + k;
  const int tx0 = (t % tiles_x) * kPtW, ty0 = (t / tiles_x) * kPtH;
  return {tx0 + (int)(threadIdx.x % kPtW), ty0 + (int)(threadIdx.x / kPtW),
          tx0 >= 1 && tx0 + kPtW <= n - 1 && ty0 >= 1 && ty0 + kPtH <= m - 1};
}
inline int point_blocks(int n, int m) { return (point_tiles(n, m) + kPtPer - 1) / kPtPer; }

// (A x) and (M x) at the edge of component c (0: x-edge, 1: y-edge) owned by the accessor's
// node, from the curls of its two cells and its two parallel neighbours.  ka, kb: kappa of
// the cells below and above an x-edge, right and left of a y-edge; mm: the edge's mass scale.
template <typename T, typename XA>
__device__ __forceinline__ void edge_AM_acc(const XA& X, int c, T ka, T kb, T s, T mm, Cx<T>& Au, Cx<T>& Mu) {
  const T two3 = (T)(2.0 / 3.0), one6 = (T)(1.0 / 6.0);
  if (c == 0) {
    const Cx<T> wlo = X.get(0, 0, 0) - X.get(0, 0, -1) + X.get(1, 0, -1) - X.get(1, 1, -1);
    const Cx<T> whi = X.get(0, 0, 1) - X.get(0, 0, 0) + X.get(1, 0, 0) - X.get(1, 1, 0);
    Au = s * ((ka * wlo) - (kb * whi));
    const Cx<T> u0 = X.get(0, 0, 0);
    Mu = mm * ((two3 * u0) + one6 * (X.get(0, 0, 1) + X.get(0, 0, -1)));
  } else {
    const Cx<T> wr = X.get(0, 0, 1) - X.get(0, 0, 0) + X.get(1, 0, 0) - X.get(1, 1, 0);
    const Cx<T> wl = X.get(0, -1, 1) - X.get(0, -1, 0) + X.get(1, -1, 0) - X.get(1, 0, 0);
    Au = s * ((ka * wr) - (kb * wl));
    const Cx<T> u0 = X.get(1, 0, 0);
    Mu = mm * ((two3 * u0) + one6 * (X.get(1, 1, 0) + X.get(1, -1, 0)));
  }
}

// (A x)_d and (M x)_d at edge d of a column in memory; kapf(i) gives kappa of cell i in T.
template <typename TI, typename T, typename KF>
__device__ __forceinline__ void edge_AM(const TI* xc, int64_t N, int n, int m, int64_t nm, int64_t d,
                                        const KF& kapf, T s, T mx, T my, const Ph<T>& p, Cx<T>& Au,
                                        Cx<T>& Mu) {
  static_assert(sizeof(TI) == sizeof(T), "edge_AM reads the column in its compute type");
  if (d < nm) {
    const int j1 = (int)(d % n), j2 = (int)(d / n);
    const ColumnEdges<T, const TI> X{xc, N, nm, n, m, j1, j2, p};
    edge_AM_acc<T>(X, 0, kapf((int64_t)wrapi(j2 - 1, m) * n + j1), kapf((int64_t)j2 * n + j1), s, mx, Au, Mu);
  } else {
    const int64_t e = d - nm;
    const int j1 = (int)(e % n), j2 = (int)(e / n);
    const ColumnEdges<T, const TI> X{xc, N, nm, n, m, j1, j2, p};
    edge_AM_acc<T>(X, 1, kapf((int64_t)j2 * n + j1), kapf((int64_t)j2 * n + wrapi(j1 - 1, n)), s, my, Au, Mu);
  }
}

// Explicit fused multiply-adds (contraction is otherwise off), so that every kernel sharing
// these bodies rounds the same way.
template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c);
template <>
__device__ __forceinline__ float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ __forceinline__ Cx<T> cfma(T w, Cx<T> r, Cx<T> acc) {
  return {fmat<T>(w, r.re, acc.re), fmat<T>(w, r.im, acc.im)};
}
template <typename T>
__device__ __forceinline__ Cx<T> cfma(T w, Cx<T> r, T c, Cx<T> u) {   // w r + c u
  return {fmat<T>(w, r.re, c * u.re), fmat<T>(w, r.im, c * u.im)};
}

// Residual of K = A + mu M on one patch edge: b - (s (k_a w_a - k_b w_b) + mm (2/3 u0 +
// 1/6 (u1 + u2))), for the edge's two cells (curls w_a, w_b) and its two parallel neighbours.
template <typename T>
__device__ __forceinline__ Cx<T> patch_resid(Cx<T> b, T ka, Cx<T> wa, T kb, Cx<T> wb, T s, T mm, Cx<T> u0, Cx<T> u1,
                                             Cx<T> u2) {
  const T two3 = (T)(2.0 / 3.0), one6 = (T)(1.0 / 6.0);
  const Cx<T> c = cfma<T>(ka, wa, (T)-1, kb * wb);                 // ka wa - kb wb
  const Cx<T> mass = cfma<T>(one6, u1 + u2, two3, u0);             // 2/3 u0 + 1/6 (u1 + u2)
  return b - cfma<T>(s, c, mm, mass);
}

// Stabilised node-patch update at node (p1, p2) (Section 5): residual r of K = A + mu M on
// the four patch edges, delta = W r with the node's patch inverse W = T diag(1/mu, S^{-1})
// T^T (10 upper-triangle entries at w), x += delta.  k* are the kappas of the four cells
// around the node, X the accessor of the iterate and B that of the right-hand side (both
// around the patch node).
template <typename T, typename XA, typename BA>
__device__ __forceinline__ void patch_update(const XA& X, const BA& B, T kne, T knw, T ksw, T kse, const T* w,
                                             T s, T mmx, T mmy) {
  const Cx<T> X00 = X.get(0, 0, 0);
  const Cx<T> X01 = X.get(0, 0, 1);
  const Cx<T> X0m = X.get(0, 0, -1);
  const Cx<T> Xm0 = X.get(0, -1, 0);
  const Cx<T> Xm1 = X.get(0, -1, 1);
  const Cx<T> Xmm = X.get(0, -1, -1);
  const Cx<T> Y00 = X.get(1, 0, 0);
  const Cx<T> Y10 = X.get(1, 1, 0);
  const Cx<T> Ym0 = X.get(1, -1, 0);
  const Cx<T> Y0m = X.get(1, 0, -1);
  const Cx<T> Y1m = X.get(1, 1, -1);
  const Cx<T> Ymm = X.get(1, -1, -1);
  const Cx<T> wne = X01 - X00 + Y00 - Y10;
  const Cx<T> wnw = Xm1 - Xm0 + Ym0 - Y00;
  const Cx<T> wsw = Xm0 - Xmm + Ymm - Y0m;
  const Cx<T> wse = X00 - X0m + Y0m - Y1m;
  const Cx<T> r0 = patch_resid<T>(B.get(0, 0, 0), kse, wse, kne, wne, s, mmx, X00, X01, X0m);
  const Cx<T> r1 = patch_resid<T>(B.get(0, -1, 0), ksw, wsw, knw, wnw, s, mmx, Xm0, Xm1, Xmm);
  const Cx<T> r2 = patch_resid<T>(B.get(1, 0, 0), kne, wne, knw, wnw, s, mmy, Y00, Y10, Ym0);
  const Cx<T> r3 = patch_resid<T>(B.get(1, 0, -1), kse, wse, ksw, wsw, s, mmy, Y0m, Y1m, Ymm);
  const T w00 = w[0], w01 = w[1], w02 = w[2], w03 = w[3], w11 = w[4], w12 = w[5], w13 = w[6], w22 = w[7],
          w23 = w[8], w33 = w[9];
  X.add(0, 0, 0, cfma<T>(w03, r3, cfma<T>(w02, r2, cfma<T>(w01, r1, w00 * r0))));
  X.add(0, -1, 0, cfma<T>(w13, r3, cfma<T>(w12, r2, cfma<T>(w11, r1, w01 * r0))));
  X.add(1, 0, 0, cfma<T>(w23, r3, cfma<T>(w22, r2, cfma<T>(w12, r1, w02 * r0))));
  X.add(1, 0, -1, cfma<T>(w33, r3, cfma<T>(w23, r2, cfma<T>(w13, r1, w03 * r0))));
}

// The patch update on a column in memory.
template <typename T>
__device__ __forceinline__ void edge_patch_gs(T* xc, const T* bc, int64_t N, int n, int m, int64_t nm, int p1,
                                              int p2, T kne, T knw, T ksw, T kse, const T* w, T s, T mmx, T mmy,
                                              const Ph<T>& p) {
  const ColumnEdges<T> X{xc, N, nm, n, m, p1, p2, p};
  const ColumnEdges<T, const T> B{bc, N, nm, n, m, p1, p2, p};
  patch_update<T>(X, B, kne, knw, ksw, kse, w, s, mmx, mmy);
}

// Restriction (adjoint of the edge embedding: 1/2 collinear, 1/4 parallel) at the coarse
// edge of component c owned by a coarse node, from the fine values around its fine node 2J
// given by an accessor R (R.get(c, d1, d2) as fetch()).
template <typename T, typename RA>
__device__ __forceinline__ Cx<T> edge_restrict_acc(const RA& R, int c) {
  const T h = (T)0.5, q = (T)0.25;
  if (c == 0)
    return h * (R.get(0, 0, 0) + R.get(0, 1, 0)) +
           q * (R.get(0, 0, 1) + R.get(0, 1, 1) + R.get(0, 0, -1) + R.get(0, 1, -1));
  return h * (R.get(1, 0, 0) + R.get(1, 0, 1)) +
         q * (R.get(1, 1, 0) + R.get(1, 1, 1) + R.get(1, -1, 0) + R.get(1, -1, 1));
}

// Coarse edge d of (Pr^* r) for the fine column r.
template <typename T>
__device__ __forceinline__ Cx<T> edge_restrict_at(const T* r, const Geo& gf, const Geo& gc, int64_t d,
                                                  const Ph<T>& p) {
  const int c = d < gc.nm ? 0 : 1;
  const int64_t e = c ? d - gc.nm : d;
  const int J1 = (int)(e % gc.n), J2 = (int)(e / gc.n);
  const ColumnEdges<T, const T> R{r, gf.ne, gf.nm, gf.n, gf.m, 2 * J1, 2 * J2, p};
  return edge_restrict_acc<T>(R, c);
}

template <typename T>
__device__ __forceinline__ Cx<T> pick_cx(bool c, Cx<T> a, Cx<T> b) {
  return {c ? a.re : b.re, c ? a.im : b.im};
}

// Fine edge of component c owned by fine node (f1, f2) of (Pr x_c): the embedding of the
// coarse Nedelec function (1/2 of the coarse edge's value on its halves, 1/4 of the two
// parallel coarse edges' values in between).  The transfers form every candidate and select
// one, so that lanes of either parity run the same instructions.
// A fine edge from the coarse edge a it lies on (even position across the edge direction:
// half of it) or from the two coarse edges a, b it lies between (odd: a quarter of their sum).
template <typename T>
__device__ __forceinline__ Cx<T> edge_prolong_combine(const Cx<T>& a, const Cx<T>& b, bool odd) {
  return pick_cx<T>(!odd, (T)0.5 * a, (T)0.25 * (a + b));
}

template <typename T>
__device__ __forceinline__ Cx<T> edge_prolong_xy(const T* c, const Geo& gc, int comp, int f1, int f2,
                                                 const Ph<T>& p) {
  const int nc = gc.n, mc = gc.m;
  const int64_t Nc = gc.ne, nmc = gc.nm;
  if (comp == 0) {
    const int J1 = f1 >> 1, J2 = f2 >> 1;
    const Cx<T> a = fetch<T, T>(c, Nc, nc, mc, 0, J1, J2, p);
    const Cx<T> b = fetch<T, T>(c, Nc, nc, mc, 0, J1, J2 + 1, p);
    return edge_prolong_combine<T>(a, b, (f2 & 1) != 0);
  }
  const int J1 = f1 >> 1, J2 = f2 >> 1;
  const Cx<T> a = fetch<T, T>(c, Nc, nc, mc, nmc, J1, J2, p);
  const Cx<T> b = fetch<T, T>(c, Nc, nc, mc, nmc, J1 + 1, J2, p);
  return edge_prolong_combine<T>(a, b, (f1 & 1) != 0);
}

// Fine edge d of (Pr x_c).
template <typename T>
__device__ __forceinline__ Cx<T> edge_prolong_at(const T* c, const Geo& gc, const Geo& gf, int64_t d,
                                                 const Ph<T>& p) {
  const int comp = d < gf.nm ? 0 : 1;
  const int64_t e = comp ? d - gf.nm : d;
  return edge_prolong_xy<T>(c, gc, comp, (int)(e % gf.n), (int)(e / gf.n), p);
}

// Nodal values around node (p1, p2) in Bloch-extended coordinates (as ColumnEdges, one
// component): get(d1, d2) is the value at (p1 + d1, p2 + d2) times the crossing's phase.
template <typename T>
struct ColumnNodes {
  const T* c;
  int64_t N;
  int n, m, p1, p2;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int d1, int d2) const { return fetch<T, T>(c, N, n, m, 0, p1 + d1, p2 + d2, p); }
};

// 9-point P = L^* M L at the accessor's node; the coefficients depend only on h2/h1.
template <typename T, typename XA>
__device__ __forceinline__ Cx<T> nodal_stencil_at(const XA& X, const NodalStencil& s) {
  const Cx<T> u = X.get(0, 0);
  const Cx<T> ex = X.get(1, 0) + X.get(-1, 0);
  const Cx<T> ey = X.get(0, 1) + X.get(0, -1);
  const Cx<T> ed = X.get(1, 1) + X.get(-1, 1) + X.get(1, -1) + X.get(-1, -1);
  return ((T)s.c0 * u) + ((T)s.cx * ex) + ((T)s.cy * ey) + ((T)s.cd * ed);
}

template <typename T>
__device__ __forceinline__ Cx<T> nodal_stencil(const T* c, int64_t N, int n, int m, int p1, int p2,
                                               const NodalStencil& s, const Ph<T>& p) {
  return nodal_stencil_at<T>(ColumnNodes<T>{c, N, n, m, p1, p2, p}, s);
}

// Full-weighting restriction (adjoint of bilinear interpolation) at a coarse node, from the
// fine values around its fine node 2J given by an accessor R (R.get(d1, d2) as fetch()).
template <typename T, typename RA>
__device__ __forceinline__ Cx<T> nodal_restrict_acc(const RA& R) {
  Cx<T> v = {0, 0};
#pragma unroll
  for (int d2 = -1; d2 <= 1; ++d2)
#pragma unroll
    for (int d1 = -1; d1 <= 1; ++d1) {
      const T w = (T)((d1 == 0 ? 1.0 : 0.5) * (d2 == 0 ? 1.0 : 0.5));
      v = v + (w * R.get(d1, d2));
    }
  return v;
}

// Coarse node d of the full-weighting restriction of the fine column r.
template <typename T>
__device__ __forceinline__ Cx<T> nodal_restrict_at(const T* r, const Geo& gf, const Geo& gc, int64_t d,
                                                   const Ph<T>& p) {
  const int J1 = (int)(d % gc.n), J2 = (int)(d / gc.n);
  return nodal_restrict_acc<T>(ColumnNodes<T>{r, gf.nm, gf.n, gf.m, 2 * J1, 2 * J2, p});
}

// Fine node (f1, f2) of the bilinear interpolation of the coarse nodal function.
// Bilinear interpolation at a fine node from the four coarse values around it (coarse node
// (J1, J2) = fine (f1 >> 1, f2 >> 1) and its neighbours one up in x, y and both); o1, o2 the
// parities of f1, f2.
template <typename T>
__device__ __forceinline__ Cx<T> nodal_prolong_combine(const Cx<T>& c00, const Cx<T>& c10, const Cx<T>& c01,
                                                       const Cx<T>& c11, bool o1, bool o2) {
  const Cx<T> vx = (T)0.5 * (c00 + c10);                   // odd f1, even f2
  const Cx<T> vy = (T)0.5 * (c00 + c01);                   // even f1, odd f2
  const Cx<T> vd = (T)0.25 * (c00 + c10 + c01 + c11);      // both odd
  return pick_cx<T>(o1, pick_cx<T>(o2, vd, vx), pick_cx<T>(o2, vy, c00));
}

template <typename T>
__device__ __forceinline__ Cx<T> nodal_prolong_xy(const T* c, const Geo& gc, int f1, int f2, const Ph<T>& p) {
  const int J1 = f1 >> 1, J2 = f2 >> 1;
  const bool o1 = f1 & 1, o2 = f2 & 1;
  const Cx<T> c00 = fetch<T, T>(c, gc.nm, gc.n, gc.m, 0, J1, J2, p);
  const Cx<T> c10 = fetch<T, T>(c, gc.nm, gc.n, gc.m, 0, J1 + 1, J2, p);
  const Cx<T> c01 = fetch<T, T>(c, gc.nm, gc.n, gc.m, 0, J1, J2 + 1, p);
  const Cx<T> c11 = fetch<T, T>(c, gc.nm, gc.n, gc.m, 0, J1 + 1, J2 + 1, p);
  return nodal_prolong_combine<T>(c00, c10, c01, c11, o1, o2);
}

// Fine node d of the bilinear interpolation of the coarse nodal function.
template <typename T>
__device__ __forceinline__ Cx<T> nodal_prolong_at(const T* c, const Geo& gc, const Geo& gf, int64_t d,
                                                  const Ph<T>& p) {
  return nodal_prolong_xy<T>(c, gc, (int)(d % gf.n), (int)(d / gf.n), p);
}

}  // namespace bl
