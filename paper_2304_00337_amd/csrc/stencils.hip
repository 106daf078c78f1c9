// Edge and nodal stencil kernels for gfx950: the Bloch-phase Nedelec curl-curl and mass
// operators (Section 3), the node-patch block Gauss-Seidel smoother with the stabilised
// 4x4 solve and the grid transfers of the bisection hierarchy (Section 5), the null-space
// projection operators L, L^* M and P = L^* M L (Section 4 and 5).
//
// All kernels work in "extended" coordinates: a vector index outside [0,n) x [0,m) is
// read through the Bloch extension u(j1 + s1 n, j2 + s2 m) = alpha^s1 beta^s2 u(j1, j2),
// so every stencil is the plain translation-invariant one and the phases enter only
// through the reads (and writes) that cross the cell boundary.  The local patch matrices
// are therefore real and independent of k.
#include "stencil_ops.h"

#include <cmath>

// No contraction of multiplies and adds into FMAs: every launch-shape variant of a kernel
// (and the fused coarse-level cycles) then performs exactly the written operations, so
// results do not depend on the shape the autotuner picks.  The kernels are bandwidth-bound;
// the extra instructions cost nothing.
#pragma clang fp contract(off)

namespace bl {

// ------------------------------------------------------------------------------------------
// Edge operators: A (curl-curl with kappa = 1/eps), M (mass), K = A + mu M and residuals.
// Thread per (node, column): the node's x-edge and y-edge; T is the arithmetic type (double,
// or float with float data).  Tiles away from the seam read without the Bloch extension.
template <typename T, int MODE, typename XA>
__device__ __forceinline__ void edge_point(const XA& X, int c, T ka, T kb, T s, T mm, T mu, T lam, Cx<T> b,
                                           Cx<T>& r, Cx<T>& Mu) {
  Cx<T> Au;
  edge_AM_acc<T>(X, c, ka, kb, s, mm, Au, Mu);
  if (MODE == EM_A) r = Au;
  else if (MODE == EM_M) r = Mu;
  else if (MODE == EM_K) r = Au + (mu * Mu);
  else if (MODE == EM_RESID_K) r = b - (Au + (mu * Mu));
  else r = Au - (lam * Mu);
}

template <typename TI, typename TO, typename T, int MODE>
__global__ __launch_bounds__(256) void k_edge_apply(View<const TI> xv, View<const TI> bv, View<TO> ov,
                                                    const double* __restrict__ k64,
                                                    const float* __restrict__ k32,
                                                    const double* __restrict__ lam, int lam_cps,
                                                    Geo g, const Phase* __restrict__ phs,
                                                    const double* __restrict__ mus,
                                                    const int* __restrict__ slots, int ncps,
                                                    double* __restrict__ partial) {
  const SJ sj = slot_col(slots, ncps);
  const int n = g.n, m = g.m;
  const int64_t nm = g.nm, N = g.ne;
  T rr = 0, mmv = 0;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const TI* xc = colp(xv, sj, N);
  k64 += (int64_t)sj.slot * nm;
  k32 += (int64_t)sj.slot * nm;
  const T mu = (MODE == EM_K || MODE == EM_RESID_K) ? (T)mus[sj.slot] : (T)0;
  const T lm = MODE == EM_EIGRES ? (T)lam[(int64_t)sj.slot * lam_cps + sj.j] : (T)0;
  const TI* bc = MODE == EM_RESID_K ? colp(bv, sj, N) : nullptr;
  TO* oc = colp(ov, sj, N);
  for (int kt = 0; kt < kPtPer; ++kt) {
    const PointTile pt = point_tile_k(n, m, kt);
    if (pt.p1 >= n || pt.p2 >= m) continue;
    const int64_t d = (int64_t)pt.p2 * n + pt.p1;
    const T kh = kap<T>(k64, k32, d);
    const T kbelow = kap<T>(k64, k32, (int64_t)wrapi(pt.p2 - 1, m) * n + pt.p1);
    const T kleft = kap<T>(k64, k32, (int64_t)pt.p2 * n + wrapi(pt.p1 - 1, n));
    Cx<T> bx{0, 0}, by{0, 0};
    if (MODE == EM_RESID_K) {
      bx = Cx<T>{(T)bc[d], (T)bc[N + d]};
      by = Cx<T>{(T)bc[nm + d], (T)bc[N + nm + d]};
    }
    Cx<T> rx, ry, mx, my;
    if (pt.inner) {
      const DirectEdges<T, TI> X{xc, N, nm, d, n};
      edge_point<T, MODE>(X, 0, kbelow, kh, (T)g.s, (T)g.mx, mu, lm, bx, rx, mx);
      edge_point<T, MODE>(X, 1, kh, kleft, (T)g.s, (T)g.my, mu, lm, by, ry, my);
    } else {
      const ColumnEdges<T, const TI> X{xc, N, nm, n, m, pt.p1, pt.p2, p};
      edge_point<T, MODE>(X, 0, kbelow, kh, (T)g.s, (T)g.mx, mu, lm, bx, rx, mx);
      edge_point<T, MODE>(X, 1, kh, kleft, (T)g.s, (T)g.my, mu, lm, by, ry, my);
    }
    oc[d] = (TO)rx.re;
    oc[N + d] = (TO)rx.im;
    oc[nm + d] = (TO)ry.re;
    oc[N + nm + d] = (TO)ry.im;
    if (MODE == EM_EIGRES) {
      rr += (rx.re * rx.re + rx.im * rx.im) + (ry.re * ry.re + ry.im * ry.im);
      mmv += (mx.re * mx.re + mx.im * mx.im) + (my.re * my.re + my.im * my.im);
    }
  }
  if (MODE == EM_EIGRES) {
    // block reduction of the two squared norms, one partial per block
    __shared__ double sh[2][256 / 64];
    double a = rr, c = mmv;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_down(a, o, 64);
      c += __shfl_down(c, o, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { sh[0][wv] = a; sh[1][wv] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double ta = 0, tc = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { ta += sh[0][w]; tc += sh[1][w]; }
      double* pp = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
      pp[0] = ta;
      pp[1] = tc;
    }
  }
}

int apply_blocks(const Geo& g) { return point_blocks(g.n, g.m); }

template <typename TI, typename TO>
void edge_apply(int mode, View<const TI> x, View<const TI> b, View<TO> out, const double* kappa64,
                const float* kappa32, const double* lam, int lam_cps, const Geo& g,
                const Phase* ph, const double* mu, const Launch& L, double* partial, int* nblk_out) {
  using T = typename std::conditional<std::is_same<TI, double>::value, double, float>::type;
  dim3 grid((unsigned)point_blocks(g.n, g.m), (unsigned)(L.nact * L.ncps));
  if (nblk_out) *nblk_out = (int)grid.x;
  if (grid.y == 0) return;
#define BL_EA(MD) k_edge_apply<TI, TO, T, MD><<<grid, kPtW * kPtH, 0, L.st>>>(x, b, out, kappa64, kappa32, lam, lam_cps, g, ph, mu, L.slots, L.ncps, partial)
  switch (mode) {
    case EM_A: BL_EA(EM_A); break;
    case EM_M: BL_EA(EM_M); break;
    case EM_K: BL_EA(EM_K); break;
    case EM_RESID_K: BL_EA(EM_RESID_K); break;
    default: BL_EA(EM_EIGRES); break;
  }
#undef BL_EA
}

template void edge_apply<double, double>(int, View<const double>, View<const double>, View<double>, const double*, const float*, const double*, int, const Geo&, const Phase*, const double*, const Launch&, double*, int*);
template void edge_apply<double, float>(int, View<const double>, View<const double>, View<float>, const double*, const float*, const double*, int, const Geo&, const Phase*, const double*, const Launch&, double*, int*);
template void edge_apply<float, float>(int, View<const float>, View<const float>, View<float>, const double*, const float*, const double*, int, const Geo&, const Phase*, const double*, const Launch&, double*, int*);

// Sum per-block partials: out[j*nval + v] = sum_b partial[(j*nblk + b)*nval + v].
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int nval,
                                  double* __restrict__ out) {
  const int col = blockIdx.x;
  __shared__ double sh[4][256];
  for (int v = 0; v < nval; ++v) {
    double a = 0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += partial[((int64_t)col * nblk + b) * nval + v];
    sh[v][threadIdx.x] = a;
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int v = 0; v < nval; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int v = 0; v < nval; ++v) out[(int64_t)col * nval + v] = sh[v][0];
}

void reduce_partials(const double* partial, int nblk, int ncols, int nval, double* out,
                     hipStream_t st) {
  if (ncols <= 0) return;
  k_reduce_partials<<<ncols, 256, 0, st>>>(partial, nblk, nval, out);
}

// ------------------------------------------------------------------------------------------
// Node-patch block Gauss-Seidel (Section 5): for every node of one colour, the residual of
// K = A + mu M on the four edges touching the node (e0 = right x-edge, e1 = left x-edge,
// e2 = upper y-edge, e3 = lower y-edge, extended coordinates) is computed, the 4x4 patch
// system is solved in the stabilised form  delta = T diag(1/mu, S^{-1}) T^T r  (the first
// column of T spans the node's gradient, on which K acts as mu times the mass), and the
// four edges are updated.  Same-colour patches are uncoupled, so the nodes of a colour are
// processed in parallel with the same result as one after the other.
template <typename T>
__device__ __forceinline__ const T* pick(const double* a, const float* b);
template <>
__device__ __forceinline__ const double* pick<double>(const double* a, const float*) { return a; }
template <>
__device__ __forceinline__ const float* pick<float>(const double*, const float* b) { return b; }

template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_edge_gs(View<T> xv, View<const T> bv,
                                                 const double* __restrict__ k64,
                                                 const float* __restrict__ k32,
                                                 const double* __restrict__ si64,
                                                 const float* __restrict__ si32, Geo g,
                                                 const Phase* __restrict__ phs,
                                                 const double* __restrict__ mus, PatchT T4,
                                                 int colour, const int* __restrict__ slots,
                                                 int ncps, int xcd) {
  const int ncg = (ncps + CPT - 1) / CPT;
  const int si_ = (int)blockIdx.y / ncg;
  const int slot = slots ? slots[si_] : si_;
  const int j0 = ((int)blockIdx.y % ncg) * CPT;
  const int n = g.n, m = g.m, nh = n >> 1, mh = m >> 1;
  const int bx = xcd ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nh * mh) return;
  const int p1 = 2 * (int)(t % nh) + (colour & 1);
  const int p2 = 2 * (int)(t / nh) + (colour >> 1);
  const int64_t nm = g.nm, N = g.ne;
  const Ph<T> p = cast_phase<T>(phs[slot]);
  k64 += (int64_t)slot * nm;
  k32 += (int64_t)slot * nm;
  const int p1m = wrapi(p1 - 1, n), p2m = wrapi(p2 - 1, m);
  const T kne = kap<T>(k64, k32, (int64_t)p2 * n + p1);
  const T knw = kap<T>(k64, k32, (int64_t)p2 * n + p1m);
  const T ksw = kap<T>(k64, k32, (int64_t)p2m * n + p1m);
  const T kse = kap<T>(k64, k32, (int64_t)p2m * n + p1);
  const T* si = pick<T>(si64, si32) + kPatchW * ((int64_t)slot * nm + (int64_t)p2 * n + p1);
  const T s = (T)g.s, mu = (T)mus[slot];
  const T mmx = mu * (T)g.mx, mmy = mu * (T)g.my;
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int j = j0 + cc;
    if (j >= ncps) break;
    const SJ sj{slot, j};
    edge_patch_gs<T>(colp(xv, sj, N), colp(bv, sj, N), N, n, m, nm, p1, p2, kne, knw, ksw, kse, si, s, mmx, mmy, p);
  }
}

template <typename T>
void edge_gs(View<T> x, View<const T> b, const double* kappa64, const float* kappa32,
             const double* sinv64, const float* sinv32, const Geo& g, const Phase* ph,
             const double* mu, const PatchT& T4, int colour, const SmoothShape& sh, const Launch& L) {
  const int64_t cnt = (int64_t)(g.n / 2) * (g.m / 2);
  const int bs = sh.bs > 0 ? sh.bs : 256, cpt = sh.cpt == 2 ? 2 : 1;
  dim3 grid((unsigned)((cnt + bs - 1) / bs), (unsigned)(L.nact * ((L.ncps + cpt - 1) / cpt)));
  if (grid.y == 0) return;
  if (cpt == 2)
    k_edge_gs<T, 2><<<grid, bs, 0, L.st>>>(x, b, kappa64, kappa32, sinv64, sinv32, g, ph, mu, T4, colour, L.slots, L.ncps, sh.xcd);
  else
    k_edge_gs<T, 1><<<grid, bs, 0, L.st>>>(x, b, kappa64, kappa32, sinv64, sinv32, g, ph, mu, T4, colour, L.slots, L.ncps, sh.xcd);
}
template void edge_gs<double>(View<double>, View<const double>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, int, const SmoothShape&, const Launch&);
template void edge_gs<float>(View<float>, View<const float>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, int, const SmoothShape&, const Launch&);

// Per-node inverse of the 3x3 block S = (Q'^T D^{-1/2} A_loc D^{-1/2} Q') + mu I of the
// stabilised patch system, Q' = columns 2..4 of the orthogonal Q (passed row-major in q).
// A_loc = (1/(h1 h2)) sum over the four cells of kappa_c c_c c_c^T with the cell
// circulation vectors c over (e0, e1, e2, e3): NE (-1,0,1,0), NW (0,-1,-1,0),
// SW (0,1,0,-1), SE (1,0,0,1).  Stored as (s00, s01, s02, s11, s12, s22).  Thread per
// (node, slot); kappa and the output are slot-major.
struct Q16 {
  double q[16];
};
__global__ void k_patch_setup(const double* __restrict__ kappa, Geo g, Q16 Q, PatchT T4,
                              const double* __restrict__ mus, double* __restrict__ s64, float* __restrict__ s32,
                              int nslots) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.nm * nslots) return;
  const int64_t slot = gid / g.nm, node = gid % g.nm;
  kappa += slot * g.nm;
  const double mu = mus[slot];
  const int n = g.n, m = g.m;
  const int p1 = (int)(node % n), p2 = (int)(node / n);
  const int p1m = wrapi(p1 - 1, n), p2m = wrapi(p2 - 1, m);
  const double kc[4] = {kappa[(int64_t)p2 * n + p1], kappa[(int64_t)p2 * n + p1m],
                        kappa[(int64_t)p2m * n + p1m], kappa[(int64_t)p2m * n + p1]};
  const double cv[4][4] = {{-1, 0, 1, 0}, {0, -1, -1, 0}, {0, 1, 0, -1}, {1, 0, 0, 1}};
  const double dx = g.mx * 2.0 / 3.0, dy = g.my * 2.0 / 3.0;
  const double dinv[4] = {1.0 / sqrt(dx), 1.0 / sqrt(dx), 1.0 / sqrt(dy), 1.0 / sqrt(dy)};
  double Ah[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double a = 0;
      for (int c = 0; c < 4; ++c) a += kc[c] * cv[c][i] * cv[c][j];
      Ah[i][j] = a * g.s * dinv[i] * dinv[j];
    }
  double S[3][3];
  for (int a = 0; a < 3; ++a)
    for (int bb = 0; bb < 3; ++bb) {
      double v = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) v += Q.q[i * 4 + a + 1] * Ah[i][j] * Q.q[j * 4 + bb + 1];
      S[a][bb] = v + (a == bb ? mu : 0.0);
    }
  // symmetric 3x3 inverse by cofactors (S is SPD and well conditioned)
  const double c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
  const double c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
  const double c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
  const double det = S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02;
  const double id = 1.0 / det;
  const double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
  const double i11 = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) * id;
  const double i12 = (S[0][2] * S[1][0] - S[0][0] * S[1][2]) * id;
  const double i22 = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) * id;
  // W = T diag(1/mu, S^{-1}) T^T (symmetric), upper triangle row by row
  const double D[4][4] = {{1.0 / mu, 0, 0, 0}, {0, i00, i01, i02}, {0, i01, i11, i12}, {0, i02, i12, i22}};
  int o = 0;
  for (int l = 0; l < 4; ++l)
    for (int k = l; k < 4; ++k) {
      double w = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) w += T4.t[l * 4 + a] * D[a][b] * T4.t[k * 4 + b];
      s64[gid * kPatchW + o] = w;
      s32[gid * kPatchW + o] = (float)w;
      ++o;
    }
}

void patch_setup(const double* kappa, const Geo& g, const double* q, const PatchT& T4, const double* mu,
                 double* sinv64, float* sinv32, int nslots, hipStream_t st) {
  Q16 Q;
  for (int i = 0; i < 16; ++i) Q.q[i] = q[i];
  const int64_t cnt = g.nm * nslots;
  k_patch_setup<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(kappa, g, Q, T4, mu, sinv64, sinv32, nslots);
}

// kappa on the next coarser level: mean over the 2x2 children (Galerkin coarse operator
// of the edge embedding equals rediscretisation with this coefficient); slot-major.
__global__ void k_coarsen_kappa(const double* __restrict__ kf, int nf, int mf, double* __restrict__ kc,
                                int nc, int mc, int nslots) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncm = (int64_t)nc * mc;
  if (gid >= ncm * nslots) return;
  const int64_t slot = gid / ncm, c = gid % ncm;
  const int c1 = (int)(c % nc), c2 = (int)(c / nc);
  const double* k = kf + slot * (int64_t)nf * mf;
  const int64_t f = (int64_t)(2 * c2) * nf + 2 * c1;
  kc[gid] = 0.25 * (k[f] + k[f + 1] + k[f + nf] + k[f + nf + 1]);
}
void coarsen_kappa(const double* kf, const Geo& gf, double* kc, int nslots, hipStream_t st) {
  const int nc = gf.n / 2, mc = gf.m / 2;
  const int64_t cnt = (int64_t)nc * mc * nslots;
  k_coarsen_kappa<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(kf, gf.n, gf.m, kc, nc, mc, nslots);
}

__global__ void k_to_float(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}
void to_float(const double* in, float* out, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  k_to_float<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(in, out, count);
}

// ------------------------------------------------------------------------------------------
// Edge grid transfers.  The prolongation is the embedding of the coarse Nedelec space:
// a coarse x-edge contributes 1/2 to its two collinear fine x-edges and 1/4 to the four
// parallel fine x-edges half a coarse cell above and below (y-edges alike); the
// restriction is its adjoint.
template <typename T>
__global__ __launch_bounds__(256) void k_edge_restrict(View<const T> rv, Geo gf, View<T> bv, Geo gc,
                                                       const Phase* __restrict__ phs,
                                                       const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= gc.ne) return;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const Cx<T> v = edge_restrict_at<T>(colp(rv, sj, gf.ne), gf, gc, d, p);
  T* o = colp(bv, sj, gc.ne);
  o[d] = v.re;
  o[gc.ne + d] = v.im;
}

template <typename T>
__global__ __launch_bounds__(256) void k_edge_prolong_add(View<const T> cv, Geo gc, View<const T> basev, View<T> fv,
                                                          Geo gf, const Phase* __restrict__ phs,
                                                          const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= gf.ne) return;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const Cx<T> v = edge_prolong_at<T>(colp(cv, sj, gc.ne), gc, gf, d, p);
  const T* x0 = colp(basev, sj, gf.ne);   // may be the output itself (same element)
  T* o = colp(fv, sj, gf.ne);
  o[d] = x0[d] + v.re;
  o[gf.ne + d] = x0[gf.ne + d] + v.im;
}

template <typename T>
void edge_restrict(View<const T> rf, const Geo& gf, View<T> bc, const Geo& gc, const Phase* ph,
                   const Launch& L) {
  dim3 grid((unsigned)((gc.ne + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_edge_restrict<T><<<grid, 256, 0, L.st>>>(rf, gf, bc, gc, ph, L.slots, L.ncps);
}
template <typename T>
void edge_prolong_add(View<const T> xc, const Geo& gc, View<T> xf, const Geo& gf,
                      const Phase* ph, const Launch& L) {
  edge_prolong_to<T>(xc, gc, View<const T>{xf.p, xf.cps, xf.off}, xf, gf, ph, L);
}
template <typename T>
void edge_prolong_to(View<const T> xc, const Geo& gc, View<const T> base, View<T> out, const Geo& gf,
                     const Phase* ph, const Launch& L) {
  dim3 grid((unsigned)((gf.ne + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_edge_prolong_add<T><<<grid, 256, 0, L.st>>>(xc, gc, base, out, gf, ph, L.slots, L.ncps);
}
template void edge_restrict<double>(View<const double>, const Geo&, View<double>, const Geo&, const Phase*, const Launch&);
template void edge_restrict<float>(View<const float>, const Geo&, View<float>, const Geo&, const Phase*, const Launch&);
template void edge_prolong_add<double>(View<const double>, const Geo&, View<double>, const Geo&, const Phase*, const Launch&);
template void edge_prolong_add<float>(View<const float>, const Geo&, View<float>, const Geo&, const Phase*, const Launch&);
template void edge_prolong_to<double>(View<const double>, const Geo&, View<const double>, View<double>, const Geo&, const Phase*, const Launch&);
template void edge_prolong_to<float>(View<const float>, const Geo&, View<const float>, View<float>, const Geo&, const Phase*, const Launch&);

// ------------------------------------------------------------------------------------------
// Nodal operators.  P = L^* M L is the 9-point Bloch Q1 Laplacian; its coefficients depend
// only on h2/h1, which bisection keeps, so every level uses the same stencil.
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_nodal_apply(View<const T> xv, View<const T> bv, View<T> ov,
                                                     Geo g, const Phase* __restrict__ phs,
                                                     NodalStencil s, const int* __restrict__ slots,
                                                     int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t N = g.nm;
  const T* xc = colp(xv, sj, N);
  const T* bc = RESID ? colp(bv, sj, N) : nullptr;
  T* o = colp(ov, sj, N);
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  for (int kt = 0; kt < kPtPer; ++kt) {
    const PointTile pt = point_tile_k(g.n, g.m, kt);
    if (pt.p1 >= g.n || pt.p2 >= g.m) continue;
    const int64_t d = (int64_t)pt.p2 * g.n + pt.p1;
    Cx<T> v;
    if (pt.inner) v = nodal_stencil_at<T>(DirectNodes<T, T>{xc, N, d, g.n}, s);
    else v = nodal_stencil<T>(xc, N, g.n, g.m, pt.p1, pt.p2, s, p);
    if (RESID) v = Cx<T>{bc[d], bc[N + d]} - v;
    o[d] = v.re;
    o[N + d] = v.im;
  }
}

template <typename T>
void nodal_apply(View<const T> x, View<const T> b, View<T> out, const Geo& g, const Phase* ph,
                 const NodalStencil& c, bool resid, const Launch& L) {
  dim3 grid((unsigned)point_blocks(g.n, g.m), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  if (resid) k_nodal_apply<T, true><<<grid, kPtW * kPtH, 0, L.st>>>(x, b, out, g, ph, c, L.slots, L.ncps);
  else k_nodal_apply<T, false><<<grid, kPtW * kPtH, 0, L.st>>>(x, b, out, g, ph, c, L.slots, L.ncps);
}
template void nodal_apply<double>(View<const double>, View<const double>, View<double>, const Geo&, const Phase*, const NodalStencil&, bool, const Launch&);
template void nodal_apply<float>(View<const float>, View<const float>, View<float>, const Geo&, const Phase*, const NodalStencil&, bool, const Launch&);

// Point Gauss-Seidel for P on the nodes of one colour (same-colour nodes are not
// neighbours of the 9-point stencil).
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_nodal_gs(View<T> xv, View<const T> bv, Geo g,
                                                  const Phase* __restrict__ phs, NodalStencil s,
                                                  int colour, const int* __restrict__ slots, int ncps,
                                                  int xcd) {
  const int ncg = (ncps + CPT - 1) / CPT;
  const int si_ = (int)blockIdx.y / ncg;
  const int slot = slots ? slots[si_] : si_;
  const int j0 = ((int)blockIdx.y % ncg) * CPT;
  const int nh = g.n >> 1, mh = g.m >> 1;
  const int bx = xcd ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nh * mh) return;
  const int p1 = 2 * (int)(t % nh) + (colour & 1);
  const int p2 = 2 * (int)(t / nh) + (colour >> 1);
  const Ph<T> p = cast_phase<T>(phs[slot]);
  const int64_t N = g.nm;
  const int64_t i = (int64_t)p2 * g.n + p1;
  const T inv = (T)1 / (T)s.c0;
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int j = j0 + cc;
    if (j >= ncps) break;
    const SJ sj{slot, j};
    T* xc = colp(xv, sj, N);
    const T* bc = colp(bv, sj, N);
    const Cx<T> r = Cx<T>{bc[i], bc[N + i]} - nodal_stencil<T>(xc, N, g.n, g.m, p1, p2, s, p);
    xc[i] += inv * r.re;
    xc[N + i] += inv * r.im;
  }
}

template <typename T>
void nodal_gs(View<T> x, View<const T> b, const Geo& g, const Phase* ph, const NodalStencil& c,
              int colour, const SmoothShape& sh, const Launch& L) {
  const int64_t cnt = (int64_t)(g.n / 2) * (g.m / 2);
  const int bs = sh.bs > 0 ? sh.bs : 256, cpt = sh.cpt == 2 ? 2 : 1;
  dim3 grid((unsigned)((cnt + bs - 1) / bs), (unsigned)(L.nact * ((L.ncps + cpt - 1) / cpt)));
  if (grid.y == 0) return;
  if (cpt == 2) k_nodal_gs<T, 2><<<grid, bs, 0, L.st>>>(x, b, g, ph, c, colour, L.slots, L.ncps, sh.xcd);
  else k_nodal_gs<T, 1><<<grid, bs, 0, L.st>>>(x, b, g, ph, c, colour, L.slots, L.ncps, sh.xcd);
}
template void nodal_gs<double>(View<double>, View<const double>, const Geo&, const Phase*, const NodalStencil&, int, const SmoothShape&, const Launch&);
template void nodal_gs<float>(View<float>, View<const float>, const Geo&, const Phase*, const NodalStencil&, int, const SmoothShape&, const Launch&);

// Nodal transfers: bilinear interpolation of the coarse Q1 function (embedding) and its
// adjoint (full weighting with Bloch phases).
template <typename T>
__global__ __launch_bounds__(256) void k_nodal_restrict(View<const T> rv, Geo gf, View<T> bv, Geo gc,
                                                        const Phase* __restrict__ phs,
                                                        const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= gc.nm) return;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const Cx<T> v = nodal_restrict_at<T>(colp(rv, sj, gf.nm), gf, gc, d, p);
  T* o = colp(bv, sj, gc.nm);
  o[d] = v.re;
  o[gc.nm + d] = v.im;
}

template <typename T>
__global__ __launch_bounds__(256) void k_nodal_prolong_add(View<const T> cv, Geo gc, View<const T> basev, View<T> fv,
                                                           Geo gf, const Phase* __restrict__ phs,
                                                           const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= gf.nm) return;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const Cx<T> v = nodal_prolong_at<T>(colp(cv, sj, gc.nm), gc, gf, d, p);
  const T* x0 = colp(basev, sj, gf.nm);   // may be the output itself (same element)
  T* o = colp(fv, sj, gf.nm);
  o[d] = x0[d] + v.re;
  o[gf.nm + d] = x0[gf.nm + d] + v.im;
}

template <typename T>
void nodal_restrict(View<const T> rf, const Geo& gf, View<T> bc, const Geo& gc, const Phase* ph,
                    const Launch& L) {
  dim3 grid((unsigned)((gc.nm + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_nodal_restrict<T><<<grid, 256, 0, L.st>>>(rf, gf, bc, gc, ph, L.slots, L.ncps);
}
template <typename T>
void nodal_prolong_add(View<const T> xc, const Geo& gc, View<T> xf, const Geo& gf,
                       const Phase* ph, const Launch& L) {
  nodal_prolong_to<T>(xc, gc, View<const T>{xf.p, xf.cps, xf.off}, xf, gf, ph, L);
}
template <typename T>
void nodal_prolong_to(View<const T> xc, const Geo& gc, View<const T> base, View<T> out, const Geo& gf,
                      const Phase* ph, const Launch& L) {
  dim3 grid((unsigned)((gf.nm + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_nodal_prolong_add<T><<<grid, 256, 0, L.st>>>(xc, gc, base, out, gf, ph, L.slots, L.ncps);
}
template void nodal_restrict<double>(View<const double>, const Geo&, View<double>, const Geo&, const Phase*, const Launch&);
template void nodal_restrict<float>(View<const float>, const Geo&, View<float>, const Geo&, const Phase*, const Launch&);
template void nodal_prolong_add<double>(View<const double>, const Geo&, View<double>, const Geo&, const Phase*, const Launch&);
template void nodal_prolong_add<float>(View<const float>, const Geo&, View<float>, const Geo&, const Phase*, const Launch&);
template void nodal_prolong_to<double>(View<const double>, const Geo&, View<const double>, View<double>, const Geo&, const Phase*, const Launch&);
template void nodal_prolong_to<float>(View<const float>, const Geo&, View<const float>, View<float>, const Geo&, const Phase*, const Launch&);

// out (nodal) = L^* M u (edge).  (L^* v)(p) = v_x(p1-1,p2) - v_x(p1,p2) + v_y(p1,p2-1) - v_y(p1,p2)
// in extended coordinates, with v = M u evaluated on the fly.  Arithmetic in FP64 (the
// right-hand side of the projection keeps the outer precision).
template <typename T, typename XA>
__device__ __forceinline__ Cx<T> lhm_at(const XA& X, T mx, T my) {
  const T two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
  auto mx_at = [&](int d1) {
    return mx * ((two3 * X.get(0, d1, 0)) + one6 * (X.get(0, d1, 1) + X.get(0, d1, -1)));
  };
  auto my_at = [&](int d2) {
    return my * ((two3 * X.get(1, 0, d2)) + one6 * (X.get(1, 1, d2) + X.get(1, -1, d2)));
  };
  return mx_at(-1) - mx_at(0) + my_at(-1) - my_at(0);
}

template <typename TI, typename TO, bool PW>
__global__ __launch_bounds__(256) void k_lhm(View<const TI> uv, View<TO> ov, Geo g,
                                             const Phase* __restrict__ phs,
                                             const int* __restrict__ slots, int ncps, PWDefl pw) {
  using T = double;
  const SJ sj = slot_col(slots, ncps);
  const int n = g.n, m = g.m;
  const int64_t N = g.ne, nm = g.nm;
  const TI* c = colp(uv, sj, N);
  TO* o = colp(ov, sj, nm);
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  double sr = 0.0, si = 0.0;
  for (int kt = 0; kt < kPtPer; ++kt) {
    const PointTile pt = point_tile_k(n, m, kt);
    if (pt.p1 >= n || pt.p2 >= m) continue;
    const int64_t d = (int64_t)pt.p2 * n + pt.p1;
    Cx<T> v;
    if (pt.inner) v = lhm_at<T>(DirectEdges<T, TI>{c, N, nm, d, n}, (T)g.mx, (T)g.my);
    else v = lhm_at<T>(ColumnEdges<T, const TI>{c, N, nm, n, m, pt.p1, pt.p2, p}, (T)g.mx, (T)g.my);
    o[d] = (TO)v.re;
    o[nm + d] = (TO)v.im;
    if (PW) {   // conj(w_j) v_j in FP64, before the rounding to TO
      const Cx<double> w = pw_value(pw, sj.slot, n, pt.p1, pt.p2);
      sr += w.re * v.re + w.im * v.im;
      si += w.re * v.im - w.im * v.re;
    }
  }
  if (PW) {
    const int64_t col = (int64_t)(blockIdx.y / ncps) * pw.pcols + pw.off + sj.j;
    block_sum2(sr, si, pw.part + (col * pw.nblk + blockIdx.x) * 2);
  }
}

template <typename TI, typename TO>
void lhm(View<const TI> u, View<TO> out, const Geo& g, const Phase* ph, const Launch& L, const PWDefl* pw) {
  dim3 grid((unsigned)point_blocks(g.n, g.m), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  if (pw) k_lhm<TI, TO, true><<<grid, kPtW * kPtH, 0, L.st>>>(u, out, g, ph, L.slots, L.ncps, *pw);
  else k_lhm<TI, TO, false><<<grid, kPtW * kPtH, 0, L.st>>>(u, out, g, ph, L.slots, L.ncps, PWDefl{});
}
template void lhm<double, double>(View<const double>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lhm<double, float>(View<const double>, View<float>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lhm<float, float>(View<const float>, View<float>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lhm<float, double>(View<const float>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);

// out (edge) = u - L phi, (L phi)_x(j1,j2) = phi(j1+1,j2) - phi(j1,j2),
// (L phi)_y(j1,j2) = phi(j1,j2+1) - phi(j1,j2) (extended reads).  FP64 arithmetic.  PW: the
// plane-wave part of the nodal solution is added as gamma L w, (L w)_x = w_j ex, (L w)_y = w_j ey.
// A thread takes kLiftPer edges (256 apart, so that every load stays coalesced): the
// workgroup's set-up is paid once for all of them and every edge's loads are issued before the
// first result is formed (the arithmetic per edge is fetch()'s, in the same order).
constexpr int kLiftPer = 4;

template <typename TI, typename TP, typename TO, bool SUB, bool PW>
__global__ __launch_bounds__(256) void k_lift(View<const TI> uv, View<const TP> fv, View<TO> ov, Geo g,
                                              const Phase* __restrict__ phs,
                                              const int* __restrict__ slots, int ncps, PWDefl pw) {
  using T = double;
  const SJ sj = slot_col(slots, ncps);
  const int64_t d0 = (int64_t)blockIdx.x * (kLiftPer * 256) + threadIdx.x;
  if (d0 >= g.ne) return;
  const Ph<T> p = cast_phase<T>(phs[sj.slot]);
  const int n = g.n, m = g.m;
  const int64_t N = g.ne, nm = g.nm;
  const TP* f = colp(fv, sj, nm);
  const TI* uc = SUB ? colp(uv, sj, N) : nullptr;
  TO* o = colp(ov, sj, N);
  // loads: phi at the edge's far node (a, Bloch code sa) and its own node (b), u, the plane wave
  TP ar[kLiftPer], ai[kLiftPer], br[kLiftPer], bi[kLiftPer];
  TI ur[kLiftPer], ui[kLiftPer];
  int sa[kLiftPer];
  double w1r[kLiftPer], w1i[kLiftPer], w2r[kLiftPer], w2i[kLiftPer];
  const double* tab = PW ? pw.tab + (int64_t)sj.slot * pw.tabstride : nullptr;
#pragma unroll
  for (int k = 0; k < kLiftPer; ++k) {
    const int64_t d = d0 + k * 256;
    if (d >= N) continue;
    const bool xe = d < nm;
    int j1, j2;
    split_index(xe ? d : d - nm, n, j1, j2);
    // far node (j1 + 1, j2) or (j1, j2 + 1), wrapped: code 1 one period ahead in x, 2 in y
    int f1 = j1 + (xe ? 1 : 0), f2 = j2 + (xe ? 0 : 1), code = 0;
    if (f1 >= n) { f1 -= n; code = 1; }
    if (f2 >= m) { f2 -= m; code = 2; }
    const int64_t ia = (int64_t)f2 * n + f1, ib = (int64_t)j2 * n + j1;
    sa[k] = code;
    ar[k] = f[ia];
    ai[k] = f[nm + ia];
    br[k] = f[ib];
    bi[k] = f[nm + ib];
    if (SUB) {
      ur[k] = uc[d];
      ui[k] = uc[N + d];
    }
    if (PW) {
      w1r[k] = tab[2 * j1];
      w1i[k] = tab[2 * j1 + 1];
      w2r[k] = tab[2 * (n + j2)];
      w2i[k] = tab[2 * (n + j2) + 1];
    }
  }
  const double* gm = nullptr;
  if (PW) {
    const int64_t col = (int64_t)(blockIdx.y / ncps) * pw.pcols + pw.off + sj.j;
    gm = pw.coef + col * 6 + 4;
  }
#pragma unroll
  for (int k = 0; k < kLiftPer; ++k) {
    const int64_t d = d0 + k * 256;
    if (d >= N) continue;
    const bool xe = d < nm;
    Cx<T> a = {(T)ar[k], (T)ai[k]};
    if (sa[k] == 1) a = cmul(a, p.ar, p.ai);
    else if (sa[k] == 2) a = cmul(a, p.br, p.bi);
    Cx<T> lp = a - Cx<T>{(T)br[k], (T)bi[k]};
    if (PW) {
      const PlaneWave& q = pw.par[sj.slot];
      const Cx<double> w = {w1r[k] * w2r[k] - w1i[k] * w2i[k], w1r[k] * w2i[k] + w1i[k] * w2r[k]};
      const Cx<double> lw = xe ? cmul(w, q.exr, q.exi) : cmul(w, q.eyr, q.eyi);
      lp = lp + cmul(lw, gm[0], gm[1]);
    }
    Cx<T> v = lp;
    if (SUB) v = Cx<T>{(T)ur[k], (T)ui[k]} - lp;
    o[d] = (TO)v.re;
    o[N + d] = (TO)v.im;
  }
}

template <typename TI, typename TP, typename TO>
void lift_sub(View<const TI> u, View<const TP> phi, View<TO> out, const Geo& g, const Phase* ph,
              const Launch& L, const PWDefl* pw) {
  dim3 grid((unsigned)((g.ne + kLiftPer * 256 - 1) / (kLiftPer * 256)), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  if (pw) k_lift<TI, TP, TO, true, true><<<grid, 256, 0, L.st>>>(u, phi, out, g, ph, L.slots, L.ncps, *pw);
  else k_lift<TI, TP, TO, true, false><<<grid, 256, 0, L.st>>>(u, phi, out, g, ph, L.slots, L.ncps, PWDefl{});
}
template <typename TI, typename TO>
void lift(View<const TI> phi, View<TO> out, const Geo& g, const Phase* ph, const Launch& L) {
  dim3 grid((unsigned)((g.ne + kLiftPer * 256 - 1) / (kLiftPer * 256)), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_lift<TO, TI, TO, false, false><<<grid, 256, 0, L.st>>>(View<const TO>{nullptr, 0, 0}, phi, out, g, ph, L.slots, L.ncps, PWDefl{});
}
template void lift_sub<double, double, double>(View<const double>, View<const double>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lift_sub<double, float, double>(View<const double>, View<const float>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lift_sub<float, float, double>(View<const float>, View<const float>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lift_sub<float, double, double>(View<const float>, View<const double>, View<double>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lift_sub<float, float, float>(View<const float>, View<const float>, View<float>, const Geo&, const Phase*, const Launch&, const PWDefl*);
template void lift<double, double>(View<const double>, View<double>, const Geo&, const Phase*, const Launch&);
template void lift<float, float>(View<const float>, View<float>, const Geo&, const Phase*, const Launch&);

// k = 0: remove the constant x- and y-edge fields M-orthogonally.  With alpha = beta = 1,
// M applied to a constant x-field is h2/h1 times it, so the M-projection onto the constant
// fields subtracts the mean of the x-part and of the y-part of every column.  The sums are
// formed by kGammaBlocks workgroups per column (partials in a fixed order), then reduced.
constexpr int kGammaBlocks = 64;
__global__ __launch_bounds__(256) void k_col_sums(View<const double> uv, Geo g, double* __restrict__ part,
                                                  const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t N = g.ne, nm = g.nm;
  const double* c = colp(uv, sj, N);
  const int64_t per = (nm + kGammaBlocks - 1) / kGammaBlocks;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < nm ? i0 + per : nm;
  double a[4] = {0, 0, 0, 0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    a[0] += c[i];
    a[1] += c[N + i];
    a[2] += c[nm + i];
    a[3] += c[N + nm + i];
  }
  __shared__ double sh[4][256];
  for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] = a[v];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int v = 0; v < 4; ++v) part[((int64_t)blockIdx.y * kGammaBlocks + blockIdx.x) * 4 + v] = sh[v][0];
}
__global__ void k_sub_means(View<double> uv, Geo g, const double* __restrict__ sums,
                            const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= g.ne) return;
  const int64_t N = g.ne;
  double* c = colp(uv, sj, N);
  const int part = d < g.nm ? 0 : 2;
  const double inv = 1.0 / (double)g.nm;
  c[d] -= sums[(int64_t)blockIdx.y * 4 + part] * inv;
  c[N + d] -= sums[(int64_t)blockIdx.y * 4 + part + 1] * inv;
}
size_t gamma_scratch_doubles(int cols) { return (size_t)(kGammaBlocks + 1) * 4 * cols; }
void gamma_deflate(View<double> u, const Geo& g, double* scratch, const Launch& L) {
  const int cols = L.nact * L.ncps;
  if (cols == 0) return;
  double* sums = scratch + (size_t)kGammaBlocks * 4 * cols;
  k_col_sums<<<dim3(kGammaBlocks, (unsigned)cols), 256, 0, L.st>>>(View<const double>{u.p, u.cps, u.off}, g, scratch,
                                                                   L.slots, L.ncps);
  reduce_partials(scratch, kGammaBlocks, cols, 4, sums, L.st);
  dim3 grid((unsigned)((g.ne + 255) / 256), (unsigned)cols);
  k_sub_means<<<grid, 256, 0, L.st>>>(u, g, sums, L.slots, L.ncps);
}

// y += x on the launch's columns (vectors of length len)
template <typename T>
__global__ void k_axpy(View<T> yv, View<const T> xv, int64_t len, const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * len) return;
  colp(yv, sj, len)[i] += colp(xv, sj, len)[i];
}
template <typename T>
void axpy(View<T> y, View<const T> x, int64_t len, const Launch& L) {
  dim3 grid((unsigned)((2 * len + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_axpy<T><<<grid, 256, 0, L.st>>>(y, x, len, L.slots, L.ncps);
}
template void axpy<double>(View<double>, View<const double>, int64_t, const Launch&);
template void axpy<float>(View<float>, View<const float>, int64_t, const Launch&);

// out = a - b (b null: out = a) on the launch's columns of length len (complex, planar)
template <typename T>
__global__ void k_sub_cols(View<const T> av, View<const T> bv, View<T> ov, int64_t len, const int* __restrict__ slots,
                           int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * len) return;
  const T a = colp(av, sj, len)[i];
  colp(ov, sj, len)[i] = bv.p ? a - colp(bv, sj, len)[i] : a;
}
template <typename T>
void sub_cols(View<const T> a, View<const T> b, View<T> out, int64_t len, const Launch& L) {
  dim3 grid((unsigned)((2 * len + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_sub_cols<T><<<grid, 256, 0, L.st>>>(a, b, out, len, L.slots, L.ncps);
}
template void sub_cols<double>(View<const double>, View<const double>, View<double>, int64_t, const Launch&);

template <typename T>
__global__ void k_fill_zero(T* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = (T)0;
}
template <typename T>
void fill_zero(T* p, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  k_fill_zero<T><<<(unsigned)((count + 255) / 256), 256, 0, st>>>(p, count);
}
template void fill_zero<double>(double*, int64_t, hipStream_t);
template void fill_zero<float>(float*, int64_t, hipStream_t);

template <typename T>
__global__ void k_zero_cols(View<T> xv, int64_t len, const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * len) return;
  colp(xv, sj, len)[i] = (T)0;
}
template <typename T>
void zero_cols(View<T> x, int64_t len, const Launch& L) {
  dim3 grid((unsigned)((2 * len + 255) / 256), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_zero_cols<T><<<grid, 256, 0, L.st>>>(x, len, L.slots, L.ncps);
}
template void zero_cols<double>(View<double>, int64_t, const Launch&);
template void zero_cols<float>(View<float>, int64_t, const Launch&);

}  // namespace bl
