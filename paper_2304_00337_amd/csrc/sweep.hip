// Tiled smoother sweeps (Section 5) for gfx950: one launch performs a whole sweep of the
// four-colour node-patch block Gauss-Seidel (edge smoother) or of the four-colour point
// Gauss-Seidel (nodal smoother) instead of one launch per colour.
//
// Each workgroup owns a TX x TY tile of nodes of one column and keeps in LDS the iterate on
// the tile plus a halo (kLo nodes below/left, kHi above/right).  The four colour passes run
// on the LDS copy, updating every patch whose stencil lies inside the box, halo included;
// values near the box edge go stale (their neighbours outside are not updated), but the
// staleness moves inwards by at most one node per pass on the low side and two on the high
// side, so after four passes the tile itself holds exactly what the per-colour launches
// produce.  The halo widths are the smallest for which this holds for both colour orders
// (checked by propagating the set of exact values through the passes).  Patches are
// computed by the same per-point code as the per-colour kernels, through an accessor that
// reads the LDS copy with the same Bloch-phase arithmetic, so the results agree bit for bit.
//
// The sweep reads the iterate from one buffer and writes it to another: a tile's halo is the
// neighbours' state before the sweep, which an in-place update could already have replaced.
//
// HBM traffic per sweep and column: the right-hand side once, the iterate once (not at all
// when the sweep starts from zero) and the iterate written once, against four reads of the
// iterate and two of the right-hand side for four colour launches.
#include "stencil_ops.h"

#pragma clang fp contract(off)

namespace bl {

namespace {

constexpr int kLo = 4;    // halo below / left of a tile, nodes (even: keeps colour parity)
constexpr int kHiE = 5;   // halo above / right, edge sweeps
constexpr int kHiN = 4;   // halo above / right, nodal sweeps
constexpr int kThreads = 256;

__device__ __forceinline__ int wrapm(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ const T* pick_si(const double* a, const float* b);
template <>
__device__ __forceinline__ const double* pick_si<double>(const double* a, const float*) { return a; }
template <>
__device__ __forceinline__ const float* pick_si<float>(const double*, const float* b) { return b; }

// Phase of an extended index as fetch() applies it: j < 0 one period back, j >= n one ahead.
template <typename T>
__device__ __forceinline__ Cx<T> phased(Cx<T> v, int j1, int j2, int n, int m, const Ph<T>& p) {
  if (j1 >= n) v = cmul(v, p.ar, p.ai);
  else if (j1 < 0) v = cmul(v, p.ar, -p.ai);
  if (j2 >= m) v = cmul(v, p.br, p.bi);
  else if (j2 < 0) v = cmul(v, p.br, -p.bi);
  return v;
}

// Edge values of the box in LDS (planes: x-edge re, x-edge im, y-edge re, y-edge im; index
// by * BX + bx), seen from the patch at box position (bx, by) = canonical node (p1, p2).
// Same reads and phase products as ColumnEdges on the column in memory.
template <typename T, int BX>
struct TileEdges {
  T* re0;
  T* im0;
  T* re1;
  T* im1;
  int bx, by, n, m, p1, p2;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    const int i = (by + d2) * BX + bx + d1;
    const Cx<T> v = c ? Cx<T>{re1[i], im1[i]} : Cx<T>{re0[i], im0[i]};
    return phased<T>(v, p1 + d1, p2 + d2, n, m, p);
  }
  __device__ __forceinline__ void add(int c, int d1, int d2, Cx<T> v) const {
    const int i = (by + d2) * BX + bx + d1;
    if (p1 + d1 < 0) v = cmul(v, p.ar, p.ai);
    if (p2 + d2 < 0) v = cmul(v, p.br, p.bi);
    T* re = c ? re1 : re0;
    T* im = c ? im1 : im0;
    re[i] = re[i] + v.re;
    im[i] = im[i] + v.im;
  }
};

template <typename T, int BX>
struct TileNodes {
  const T* re;
  const T* im;
  int bx, by, n, m, p1, p2;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int d1, int d2) const {
    const int i = (by + d2) * BX + bx + d1;
    return phased<T>(Cx<T>{re[i], im[i]}, p1 + d1, p2 + d2, n, m, p);
  }
};

// Column and tile of this workgroup: blockIdx.y = active slot x column, blockIdx.x = tile
// (XCD-major order when there are at least 8 tiles, so that neighbouring tiles share an L2).
struct TileRef {
  int slot, j, t0x, t0y;
};
__device__ __forceinline__ TileRef tile_ref(const int* slots, int ncps, int tiles_x, int TX, int TY) {
  const int si = (int)blockIdx.y / ncps;
  const int nb = (int)gridDim.x;
  const int t = nb >= 8 ? xcd_block((int)blockIdx.x, nb) : (int)blockIdx.x;
  return {slots ? slots[si] : si, (int)blockIdx.y % ncps, (t % tiles_x) * TX, (t / tiles_x) * TY};
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_edge_sweep(View<const T> xin, View<T> xout, View<const T> bv,
                                                         const double* __restrict__ k64,
                                                         const float* __restrict__ k32,
                                                         const double* __restrict__ si64,
                                                         const float* __restrict__ si32, Geo g,
                                                         const Phase* __restrict__ phs,
                                                         const double* __restrict__ mus, PatchT T4, int backward,
                                                         int zero_start, const int* __restrict__ slots, int ncps,
                                                         int tiles_x) {
  constexpr int BX = TX + kLo + kHiE, BY = TY + kLo + kHiE, BN = BX * BY;
  __shared__ T lds[4 * BN];
  T* const re0 = lds;
  T* const im0 = lds + BN;
  T* const re1 = lds + 2 * BN;
  T* const im1 = lds + 3 * BN;
  const TileRef tr = tile_ref(slots, ncps, tiles_x, TX, TY);
  const int n = g.n, m = g.m, tid = threadIdx.x;
  const int64_t N = g.ne, nm = g.nm;
  const SJ sj{tr.slot, tr.j};
  const T* xc = zero_start ? nullptr : colp(xin, sj, N);
  T* xo = colp(xout, sj, N);
  const T* bc = colp(bv, sj, N);
  const Ph<T> p = cast_phase<T>(phs[tr.slot]);
  for (int e = tid; e < BN; e += kThreads) {
    if (zero_start) {
      re0[e] = im0[e] = re1[e] = im1[e] = (T)0;
    } else {
      const int c1 = wrapm(tr.t0x - kLo + e % BX, n), c2 = wrapm(tr.t0y - kLo + e / BX, m);
      const int64_t i = (int64_t)c2 * n + c1;
      re0[e] = xc[i];
      im0[e] = xc[N + i];
      re1[e] = xc[nm + i];
      im1[e] = xc[N + nm + i];
    }
  }
  __syncthreads();
  k64 += (int64_t)tr.slot * nm;
  k32 += (int64_t)tr.slot * nm;
  const T* sib = pick_si<T>(si64, si32) + 6 * (int64_t)tr.slot * nm;
  const T s = (T)g.s, mu = (T)mus[tr.slot];
  const T mmx = mu * (T)g.mx, mmy = mu * (T)g.my;
  for (int q = 0; q < 4; ++q) {
    const int colour = backward ? 3 - q : q;
    // patch nodes: box positions 1 .. B-2 whose canonical parity is the colour's (the box
    // origin t0 - kLo is even and n, m are even, so the parity is that of the position)
    const int b0x = (colour & 1) ? 1 : 2, b0y = (colour >> 1) ? 1 : 2;
    const int cx = (BX - 2 - b0x) / 2 + 1, cy = (BY - 2 - b0y) / 2 + 1;
    for (int t = tid; t < cx * cy; t += kThreads) {
      const int bx = b0x + 2 * (t % cx), by = b0y + 2 * (t / cx);
      const int p1 = wrapm(tr.t0x - kLo + bx, n), p2 = wrapm(tr.t0y - kLo + by, m);
      const int p1m = wrapi(p1 - 1, n), p2m = wrapi(p2 - 1, m);
      const T kne = kap<T>(k64, k32, (int64_t)p2 * n + p1);
      const T knw = kap<T>(k64, k32, (int64_t)p2 * n + p1m);
      const T ksw = kap<T>(k64, k32, (int64_t)p2m * n + p1m);
      const T kse = kap<T>(k64, k32, (int64_t)p2m * n + p1);
      const T* si = sib + 6 * ((int64_t)p2 * n + p1);
      const TileEdges<T, BX> X{re0, im0, re1, im1, bx, by, n, m, p1, p2, p};
      patch_update<T>(X, bc, N, n, m, nm, p1, p2, kne, knw, ksw, kse, si, T4, s, mu, mmx, mmy, p);
    }
    __syncthreads();
  }
  for (int e = tid; e < TX * TY; e += kThreads) {
    const int ix = e % TX, iy = e / TX;
    const int c1 = tr.t0x + ix, c2 = tr.t0y + iy;
    if (c1 >= n || c2 >= m) continue;
    const int bi = (iy + kLo) * BX + ix + kLo;
    const int64_t i = (int64_t)c2 * n + c1;
    xo[i] = re0[bi];
    xo[N + i] = im0[bi];
    xo[nm + i] = re1[bi];
    xo[N + nm + i] = im1[bi];
  }
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_nodal_sweep(View<const T> xin, View<T> xout, View<const T> bv, Geo g,
                                                          const Phase* __restrict__ phs, NodalStencil st,
                                                          int backward, int zero_start,
                                                          const int* __restrict__ slots, int ncps, int tiles_x) {
  constexpr int BX = TX + kLo + kHiN, BY = TY + kLo + kHiN, BN = BX * BY;
  __shared__ T lds[2 * BN];
  T* const re = lds;
  T* const im = lds + BN;
  const TileRef tr = tile_ref(slots, ncps, tiles_x, TX, TY);
  const int n = g.n, m = g.m, tid = threadIdx.x;
  const int64_t N = g.nm;
  const SJ sj{tr.slot, tr.j};
  const T* xc = zero_start ? nullptr : colp(xin, sj, N);
  T* xo = colp(xout, sj, N);
  const T* bc = colp(bv, sj, N);
  const Ph<T> p = cast_phase<T>(phs[tr.slot]);
  for (int e = tid; e < BN; e += kThreads) {
    if (zero_start) {
      re[e] = im[e] = (T)0;
    } else {
      const int c1 = wrapm(tr.t0x - kLo + e % BX, n), c2 = wrapm(tr.t0y - kLo + e / BX, m);
      const int64_t i = (int64_t)c2 * n + c1;
      re[e] = xc[i];
      im[e] = xc[N + i];
    }
  }
  __syncthreads();
  const T inv = (T)1 / (T)st.c0;
  for (int q = 0; q < 4; ++q) {
    const int colour = backward ? 3 - q : q;
    const int b0x = (colour & 1) ? 1 : 2, b0y = (colour >> 1) ? 1 : 2;
    const int cx = (BX - 2 - b0x) / 2 + 1, cy = (BY - 2 - b0y) / 2 + 1;
    for (int t = tid; t < cx * cy; t += kThreads) {
      const int bx = b0x + 2 * (t % cx), by = b0y + 2 * (t / cx);
      const int p1 = wrapm(tr.t0x - kLo + bx, n), p2 = wrapm(tr.t0y - kLo + by, m);
      const int64_t i = (int64_t)p2 * n + p1;
      const TileNodes<T, BX> X{re, im, bx, by, n, m, p1, p2, p};
      const Cx<T> r = Cx<T>{bc[i], bc[N + i]} - nodal_stencil_at<T>(X, st);
      const int bi = by * BX + bx;
      re[bi] += inv * r.re;
      im[bi] += inv * r.im;
    }
    __syncthreads();
  }
  for (int e = tid; e < TX * TY; e += kThreads) {
    const int ix = e % TX, iy = e / TX;
    const int c1 = tr.t0x + ix, c2 = tr.t0y + iy;
    if (c1 >= n || c2 >= m) continue;
    const int bi = (iy + kLo) * BX + ix + kLo;
    const int64_t i = (int64_t)c2 * n + c1;
    xo[i] = re[bi];
    xo[N + i] = im[bi];
  }
}

constexpr int kTX = 32, kTY = 32;

}  // namespace

template <typename T>
void edge_sweep(View<const T> xin, View<T> xout, View<const T> b, const double* kappa64, const float* kappa32,
                const double* sinv64, const float* sinv32, const Geo& g, const Phase* ph, const double* mu,
                const PatchT& T4, bool backward, bool zero_start, const Launch& L) {
  const int tx = (g.n + kTX - 1) / kTX, ty = (g.m + kTY - 1) / kTY;
  dim3 grid((unsigned)(tx * ty), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_edge_sweep<T, kTX, kTY><<<grid, kThreads, 0, L.st>>>(xin, xout, b, kappa64, kappa32, sinv64, sinv32, g, ph, mu, T4,
                                                         backward ? 1 : 0, zero_start ? 1 : 0, L.slots, L.ncps, tx);
}

template <typename T>
void nodal_sweep(View<const T> xin, View<T> xout, View<const T> b, const Geo& g, const Phase* ph,
                 const NodalStencil& c, bool backward, bool zero_start, const Launch& L) {
  const int tx = (g.n + kTX - 1) / kTX, ty = (g.m + kTY - 1) / kTY;
  dim3 grid((unsigned)(tx * ty), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_nodal_sweep<T, kTX, kTY><<<grid, kThreads, 0, L.st>>>(xin, xout, b, g, ph, c, backward ? 1 : 0, zero_start ? 1 : 0,
                                                          L.slots, L.ncps, tx);
}

template void edge_sweep<double>(View<const double>, View<double>, View<const double>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, bool, bool, const Launch&);
template void edge_sweep<float>(View<const float>, View<float>, View<const float>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, bool, bool, const Launch&);
template void nodal_sweep<double>(View<const double>, View<double>, View<const double>, const Geo&, const Phase*, const NodalStencil&, bool, bool, const Launch&);
template void nodal_sweep<float>(View<const float>, View<float>, View<const float>, const Geo&, const Phase*, const NodalStencil&, bool, bool, const Launch&);

}  // namespace bl
