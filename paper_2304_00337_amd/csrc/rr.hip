// Rayleigh-Ritz products of the Ritz step (Section 4) for gfx950, straight from the basis:
//
//   G = S^* M S = sum over edges e of conj(s_e) (M s)_e,
//   H = S^* A S = sum over cells c of (kappa_c / (h1 h2)) conj(w_c) w_c,
//
// with w_c the Bloch-extended circulation of cell c (A = C^* K C, C the discrete curl, K the
// diagonal of kappa / (h1 h2)), so H is a weighted Gram product of the cell curls and the
// products M S and A S are never stored.  One workgroup owns a range of node indices d
// (x-edge d, y-edge d and cell d) and an output tile of TB x TB entries; it stages, per
// chunk of CH nodes, the basis values, the mass products and the scaled curls of the tile's
// columns in LDS and accumulates RT x RT complex register tiles per thread.  Partial sums
// per node range are reduced in a fixed order, so a slot's G and H do not depend on the
// other slots of the launch.
//
// Bases of at most 48 columns (the iteration's [X, W] for p <= 24) take the matrix cores
// instead: FP64 MFMA 16x16x4 products, one workgroup of eight waves per node range (four for
// G, four for H; two waves per SIMD hide each other's loads).  Each lane forms, for one node
// of a group of four and one column of each 16-column tile, the basis values and mass
// products (G) or the scaled cell curls (H) directly in the operand layout of the
// instruction (no LDS staging); the six upper tile pairs are accumulated in registers and
// the waves' sums are combined in a fixed order before one partial per node range is written.
#include "stencil_common.h"

// Contractions are explicit (fma in the accumulations, none elsewhere), so the 48- and
// 64-wide tile variants round identically.
#pragma clang fp contract(off)

namespace bl {

namespace {

constexpr int CH = 8;   // nodes per LDS chunk

template <int RT>
__global__ __launch_bounds__(256) void k_rr_gram(View<const double> Sv, int q,
                                                 const double* __restrict__ kappa, Geo g,
                                                 const Phase* __restrict__ phs, int64_t rows_per_blk,
                                                 double* __restrict__ partial,
                                                 const int* __restrict__ slots) {
  constexpr int TB = 16 * RT;
  __shared__ double xr[2 * CH][TB], xi[2 * CH][TB], yr[2 * CH][TB], yi[2 * CH][TB];
  __shared__ double ar_[CH][TB], ai_[CH][TB], br_[CH][TB], bi_[CH][TB];
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  const int64_t N = g.ne, nm = g.nm;
  const int n = g.n, m = g.m;
  const double* S = Sv.p + ((int64_t)slot * Sv.cps + Sv.off) * 2 * N;
  const double* kap = kappa + (int64_t)slot * nm;
  const Ph<double> p = cast_phase<double>(phs[slot]);
  const int ntj = (q + TB - 1) / TB;
  const int ti0 = (blockIdx.y / ntj) * TB, tj0 = (blockIdx.y % ntj) * TB;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t rs = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t re = rs + rows_per_blk < nm ? rs + rows_per_blk : nm;
  const double two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
  double gr[RT][RT], gi[RT][RT], hr[RT][RT], hi[RT][RT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) { gr[a][b] = 0; gi[a][b] = 0; hr[a][b] = 0; hi[a][b] = 0; }
  // diagonal tiles (all of them when q fits one tile) stage one column range: the curls of
  // the i- and j-ranges coincide and are formed once
  const bool diag = ti0 == tj0;
  for (int64_t r0 = rs; r0 < re; r0 += CH) {
    // consecutive threads take consecutive nodes of one column (coalesced reads)
    for (int e = tid; e < CH * TB; e += 256) {
      const int r = e % CH, c = e / CH;
      const int64_t d = r0 + r;
      const bool ok = d < re;
      const int j1 = ok ? (int)(d % n) : 0, j2 = ok ? (int)(d / n) : 0;
      const double wsc = ok ? sqrt(kap[ok ? d : 0] * g.s) : 0.0;
      const int ci = ti0 + c, cj = tj0 + c;
      if (ok && ci < q) {
        const double* col = S + (int64_t)ci * 2 * N;
        xr[r][c] = col[d];
        xi[r][c] = col[N + d];
        xr[CH + r][c] = col[nm + d];
        xi[CH + r][c] = col[N + nm + d];
        if (!diag) {
          const Cx<double> w = cell_curl<double, double>(col, N, n, m, nm, j1, j2, p);
          ar_[r][c] = wsc * w.re;
          ai_[r][c] = wsc * w.im;
        }
      } else {
        xr[r][c] = 0; xi[r][c] = 0; xr[CH + r][c] = 0; xi[CH + r][c] = 0;
        ar_[r][c] = 0; ai_[r][c] = 0;
      }
      if (ok && cj < q) {
        const double* col = S + (int64_t)cj * 2 * N;
        const Cx<double> ux = {col[d], col[N + d]};
        const Cx<double> mxv = g.mx * ((two3 * ux) + one6 * (fetch<double, double>(col, N, n, m, 0, j1, j2 + 1, p) +
                                                              fetch<double, double>(col, N, n, m, 0, j1, j2 - 1, p)));
        const Cx<double> uy = {col[nm + d], col[N + nm + d]};
        const Cx<double> myv = g.my * ((two3 * uy) + one6 * (fetch<double, double>(col, N, n, m, nm, j1 + 1, j2, p) +
                                                              fetch<double, double>(col, N, n, m, nm, j1 - 1, j2, p)));
        yr[r][c] = mxv.re;
        yi[r][c] = mxv.im;
        yr[CH + r][c] = myv.re;
        yi[CH + r][c] = myv.im;
        const Cx<double> w = cell_curl<double, double>(col, N, n, m, nm, j1, j2, p);
        br_[r][c] = wsc * w.re;
        bi_[r][c] = wsc * w.im;
      } else {
        yr[r][c] = 0; yi[r][c] = 0; yr[CH + r][c] = 0; yi[CH + r][c] = 0;
        br_[r][c] = 0; bi_[r][c] = 0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 2 * CH; ++rr) {
      double u_r[RT], u_i[RT], v_r[RT], v_i[RT];
#pragma unroll
      for (int a = 0; a < RT; ++a) { u_r[a] = xr[rr][ty * RT + a]; u_i[a] = xi[rr][ty * RT + a]; }
#pragma unroll
      for (int b = 0; b < RT; ++b) { v_r[b] = yr[rr][tx * RT + b]; v_i[b] = yi[rr][tx * RT + b]; }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < RT; ++b) {
          gr[a][b] = fma(u_i[a], v_i[b], fma(u_r[a], v_r[b], gr[a][b]));
          gi[a][b] = fma(-u_i[a], v_r[b], fma(u_r[a], v_i[b], gi[a][b]));
        }
    }
#pragma unroll 4
    for (int rr = 0; rr < CH; ++rr) {
      double u_r[RT], u_i[RT], v_r[RT], v_i[RT];
      if (diag) {
#pragma unroll
        for (int a = 0; a < RT; ++a) { u_r[a] = br_[rr][ty * RT + a]; u_i[a] = bi_[rr][ty * RT + a]; }
      } else {
#pragma unroll
        for (int a = 0; a < RT; ++a) { u_r[a] = ar_[rr][ty * RT + a]; u_i[a] = ai_[rr][ty * RT + a]; }
      }
#pragma unroll
      for (int b = 0; b < RT; ++b) { v_r[b] = br_[rr][tx * RT + b]; v_i[b] = bi_[rr][tx * RT + b]; }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < RT; ++b) {
          hr[a][b] = fma(u_i[a], v_i[b], fma(u_r[a], v_r[b], hr[a][b]));
          hi[a][b] = fma(-u_i[a], v_r[b], fma(u_r[a], v_i[b], hi[a][b]));
        }
    }
    __syncthreads();
  }
  // partial layout per (launch entry z, node range): G (q x q) then H (q x q), interleaved
  double* pg = partial + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * (int64_t)q * q * 4;
  double* ph = pg + (int64_t)q * q * 2;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int i = ti0 + ty * RT + a, j = tj0 + tx * RT + b;
      if (i < q && j < q) {
        const int64_t e = 2 * ((int64_t)i * q + j);
        pg[e] = gr[a][b];
        pg[e + 1] = gi[a][b];
        ph[e] = hr[a][b];
        ph[e + 1] = hi[a][b];
      }
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int MQ = 48;          // widest basis of the matrix-core path (3 tiles of 16 columns,
                                // written out below as the pairs of three tiles)
constexpr int MT = MQ / 16;     // column tiles
constexpr int MP = MT * (MT + 1) / 2;   // tile pairs ti <= tj
constexpr int MW = 4;           // waves per product (G or H) in a workgroup

#define BL_MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

// Lane l of a wave takes node d (the group's node l / 16) and column 16 t + l % 16 of each
// tile t.  Neighbour indices and the Bloch phases of the seam follow fetch().
struct NodeRef {
  int64_t d, up, dn, rt, lf;
  bool ok, cu, cd, cr, cl;
};
__device__ __forceinline__ NodeRef node_ref(int64_t d, bool ok, int n, int m) {
  NodeRef r;
  r.ok = ok;
  const int j1 = ok ? (int)(d % n) : 0, j2 = ok ? (int)(d / n) : 0;
  r.d = ok ? d : 0;
  r.cu = j2 == m - 1;
  r.cd = j2 == 0;
  r.cr = j1 == n - 1;
  r.cl = j1 == 0;
  r.up = r.cu ? r.d - (int64_t)(m - 1) * n : r.d + n;   // x-edge (j1, j2 + 1)
  r.dn = r.cd ? r.d + (int64_t)(m - 1) * n : r.d - n;   // x-edge (j1, j2 - 1)
  r.rt = r.cr ? r.d - (n - 1) : r.d + 1;                // y-edge (j1 + 1, j2)
  r.lf = r.cl ? r.d + (n - 1) : r.d - 1;                // y-edge (j1 - 1, j2)
  return r;
}

__device__ __forceinline__ Cx<double> sel(bool c, Cx<double> a, Cx<double> b) {
  return {c ? a.re : b.re, c ? a.im : b.im};
}

// Operands of one 16-column tile for G = sum over edges of conj(u) (M u): the x- and y-edge
// values (u) and their mass products (v), per component [0] x, [1] y.
struct GTile {
  double ur[2], ui[2], vr[2], vi[2];
};
__device__ __forceinline__ GTile g_tile(const double* __restrict__ S, int q, int64_t N, int64_t nm, const Geo& g,
                                        const Ph<double>& p, const NodeRef& r, int t) {
  GTile o = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  const int c = 16 * t + (int)(threadIdx.x & 15);
  if (r.ok && c < q) {
    const double two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
    const double* col = S + (int64_t)c * 2 * N;
    const Cx<double> x0 = {col[r.d], col[N + r.d]};
    const Cx<double> xu = sel(r.cu, cmul(Cx<double>{col[r.up], col[N + r.up]}, p.br, p.bi),
                              Cx<double>{col[r.up], col[N + r.up]});
    const Cx<double> xd = sel(r.cd, cmul(Cx<double>{col[r.dn], col[N + r.dn]}, p.br, -p.bi),
                              Cx<double>{col[r.dn], col[N + r.dn]});
    const Cx<double> y0 = {col[nm + r.d], col[N + nm + r.d]};
    const Cx<double> yr = sel(r.cr, cmul(Cx<double>{col[nm + r.rt], col[N + nm + r.rt]}, p.ar, p.ai),
                              Cx<double>{col[nm + r.rt], col[N + nm + r.rt]});
    const Cx<double> yl = sel(r.cl, cmul(Cx<double>{col[nm + r.lf], col[N + nm + r.lf]}, p.ar, -p.ai),
                              Cx<double>{col[nm + r.lf], col[N + nm + r.lf]});
    const Cx<double> mx = g.mx * ((two3 * x0) + one6 * (xu + xd));
    const Cx<double> my = g.my * ((two3 * y0) + one6 * (yr + yl));
    o.ur[0] = x0.re; o.ui[0] = x0.im; o.ur[1] = y0.re; o.ui[1] = y0.im;
    o.vr[0] = mx.re; o.vi[0] = mx.im; o.vr[1] = my.re; o.vi[1] = my.im;
  }
  return o;
}

// Operands of one tile for H = sum over cells of (kappa s) conj(w) w: the cell curl scaled
// by sqrt(kappa s).
struct HTile {
  double wr, wi;
};
__device__ __forceinline__ HTile h_tile(const double* __restrict__ S, int q, int64_t N, int64_t nm,
                                        const Ph<double>& p, double wsc, const NodeRef& r, int t) {
  HTile o = {0, 0};
  const int c = 16 * t + (int)(threadIdx.x & 15);
  if (r.ok && c < q) {
    const double* col = S + (int64_t)c * 2 * N;
    const Cx<double> x0 = {col[r.d], col[N + r.d]};
    const Cx<double> xu = sel(r.cu, cmul(Cx<double>{col[r.up], col[N + r.up]}, p.br, p.bi),
                              Cx<double>{col[r.up], col[N + r.up]});
    const Cx<double> y0 = {col[nm + r.d], col[N + nm + r.d]};
    const Cx<double> yr = sel(r.cr, cmul(Cx<double>{col[nm + r.rt], col[N + nm + r.rt]}, p.ar, p.ai),
                              Cx<double>{col[nm + r.rt], col[N + nm + r.rt]});
    const Cx<double> c0 = wsc * (xu - x0 + y0 - yr);
    o.wr = c0.re;
    o.wi = c0.im;
  }
  return o;
}

// G and H updates of tile pair (A, B), accumulator k
#define BL_GPAIR(k, A, B)                                  \
  ar[k] = BL_MFMA(A.ur[0], B.vr[0], ar[k]);                \
  ar[k] = BL_MFMA(A.ui[0], B.vi[0], ar[k]);                \
  ar[k] = BL_MFMA(A.ur[1], B.vr[1], ar[k]);                \
  ar[k] = BL_MFMA(A.ui[1], B.vi[1], ar[k]);                \
  ai[k] = BL_MFMA(A.ur[0], B.vi[0], ai[k]);                \
  ai[k] = BL_MFMA(-A.ui[0], B.vr[0], ai[k]);               \
  ai[k] = BL_MFMA(A.ur[1], B.vi[1], ai[k]);                \
  ai[k] = BL_MFMA(-A.ui[1], B.vr[1], ai[k]);
#define BL_HPAIR(k, A, B)                                  \
  ar[k] = BL_MFMA(A.wr, B.wr, ar[k]);                      \
  ar[k] = BL_MFMA(A.wi, B.wi, ar[k]);                      \
  ai[k] = BL_MFMA(A.wr, B.wi, ai[k]);                      \
  ai[k] = BL_MFMA(-A.wi, B.wr, ai[k]);

// Workgroup of 2 MW waves per node range [rs, re): waves 0..MW-1 accumulate G, waves
// MW..2MW-1 accumulate H, wave w of a product taking the 4-node groups w, w + MW, ...
__global__ __launch_bounds__(128 * MW) void k_rr_mfma(View<const double> Sv, int q, const double* __restrict__ kappa,
                                                      Geo g, const Phase* __restrict__ phs, int64_t rows_per_blk,
                                                      double* __restrict__ partial, const int* __restrict__ slots) {
  extern __shared__ double red[];   // per product: 2 MP d4 per lane (re, im), lane-major
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  const int64_t N = g.ne, nm = g.nm;
  const int n = g.n, m = g.m;
  const double* S = Sv.p + ((int64_t)slot * Sv.cps + Sv.off) * 2 * N;
  const double* kap = kappa + (int64_t)slot * nm;
  const Ph<double> p = cast_phase<double>(phs[slot]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool is_h = wv >= MW;
  const int w = is_h ? wv - MW : wv;
  const int64_t rs = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t re = rs + rows_per_blk < nm ? rs + rows_per_blk : nm;
  const int64_t ngroups = (re - rs + 3) / 4;
  d4 ar[MP], ai[MP];
#pragma unroll
  for (int k = 0; k < MP; ++k) ar[k] = ai[k] = d4{0, 0, 0, 0};
  // tile pairs k = 0..5: (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
  if (!is_h) {
    for (int64_t grp = w; grp < ngroups; grp += MW) {
      const int64_t d = rs + 4 * grp + (lane >> 4);
      const NodeRef r = node_ref(d, d < re, n, m);
      const GTile t0 = g_tile(S, q, N, nm, g, p, r, 0);
      const GTile t1 = g_tile(S, q, N, nm, g, p, r, 1);
      const GTile t2 = g_tile(S, q, N, nm, g, p, r, 2);
      BL_GPAIR(0, t0, t0)
      BL_GPAIR(1, t0, t1)
      BL_GPAIR(2, t0, t2)
      BL_GPAIR(3, t1, t1)
      BL_GPAIR(4, t1, t2)
      BL_GPAIR(5, t2, t2)
    }
  } else {
    for (int64_t grp = w; grp < ngroups; grp += MW) {
      const int64_t d = rs + 4 * grp + (lane >> 4);
      const NodeRef r = node_ref(d, d < re, n, m);
      const double wsc = r.ok ? sqrt(kap[r.d] * g.s) : 0.0;
      const HTile t0 = h_tile(S, q, N, nm, p, wsc, r, 0);
      const HTile t1 = h_tile(S, q, N, nm, p, wsc, r, 1);
      const HTile t2 = h_tile(S, q, N, nm, p, wsc, r, 2);
      BL_HPAIR(0, t0, t0)
      BL_HPAIR(1, t0, t1)
      BL_HPAIR(2, t0, t2)
      BL_HPAIR(3, t1, t1)
      BL_HPAIR(4, t1, t2)
      BL_HPAIR(5, t2, t2)
    }
  }
  // combine the waves of each product in order 0 .. MW-1
  double* mine = red + ((size_t)(is_h ? 1 : 0) * 64 + lane) * 8 * MP;
  for (int src = 0; src < MW; ++src) {
    if (w == src) {
#pragma unroll
      for (int k = 0; k < MP; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* e = mine + 8 * k + 2 * v;
          if (src == 0) {
            e[0] = ar[k][v];
            e[1] = ai[k][v];
          } else {
            e[0] += ar[k][v];
            e[1] += ai[k][v];
          }
        }
    }
    __syncthreads();
  }
  // write the range's full G and H (q x q, interleaved complex; lower tiles mirrored)
  double* pg = partial + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * (int64_t)q * q * 4;
  for (int e = threadIdx.x; e < 2 * 64 * MP * 4; e += 128 * MW) {
    const int prod = e / (64 * MP * 4), l = (e / (MP * 4)) % 64, k = (e / 4) % MP, v = e % 4;
    int ti = 0, tj = 0, kk = k;
    for (ti = 0; ti < MT; ++ti) {
      if (kk < MT - ti) { tj = ti + kk; break; }
      kk -= MT - ti;
    }
    const int i = 16 * ti + 4 * v + (l >> 4), j = 16 * tj + (l & 15);
    if (i >= q || j >= q) continue;
    const double* src = red + ((size_t)prod * 64 + l) * 8 * MP + 8 * k + 2 * v;
    double* out = pg + (int64_t)prod * q * q * 2;
    const int64_t a = 2 * ((int64_t)i * q + j), b = 2 * ((int64_t)j * q + i);
    out[a] = src[0];
    out[a + 1] = src[1];
    if (ti != tj) {
      out[b] = src[0];
      out[b + 1] = -src[1];
    }
  }
}

#undef BL_GPAIR
#undef BL_HPAIR
#undef BL_MFMA

// G_s, H_s = sums over the node ranges of launch entry z: 64 entries per block, the ranges
// split into four consecutive quarters summed in range order, the quarters then added in
// order (a fixed order, independent of timing).
__global__ __launch_bounds__(256) void k_rr_reduce(const double* __restrict__ partial, int nblk, int q,
                                                   double* __restrict__ G, double* __restrict__ H,
                                                   const int* __restrict__ slots) {
  __shared__ double part[4][64];
  const int z = blockIdx.y;
  const int64_t slot = slots ? slots[z] : z;
  const int64_t cnt = (int64_t)q * q * 4;
  const int lo = threadIdx.x & 63, qt = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lo;
  const double* pz = partial + (int64_t)z * nblk * cnt;
  const int b0 = (int)((int64_t)nblk * qt / 4), b1 = (int)((int64_t)nblk * (qt + 1) / 4);
  double sum = 0;
  if (e < cnt)
    for (int b = b0; b < b1; ++b) sum += pz[(int64_t)b * cnt + e];
  part[qt][lo] = sum;
  __syncthreads();
  if (qt == 0 && e < cnt) {
    const double s = ((part[0][lo] + part[1][lo]) + part[2][lo]) + part[3][lo];
    const int64_t half = (int64_t)q * q * 2;
    if (e < half) G[slot * half + e] = s;
    else H[slot * half + e - half] = s;
  }
}

}  // namespace

// node ranges of the matrix-core path: up to one workgroup per compute unit, >= 64 nodes each
int rr_mfma_blocks(int64_t nm) {
  int64_t nb = (nm + 255) / 256;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  int64_t rpb = (nm + nb - 1) / nb;
  rpb = (rpb + 3) / 4 * 4;
  return (int)((nm + rpb - 1) / rpb);
}

int rr_partial_blocks(int64_t nm) {
  const int a = rr_blocks(nm), b = rr_mfma_blocks(nm);
  return a > b ? a : b;
}

int rr_blocks(int64_t nm) {
  int64_t nb = (nm + 511) / 512;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  int64_t rpb = (nm + nb - 1) / nb;
  rpb = (rpb + CH - 1) / CH * CH;
  return (int)((nm + rpb - 1) / rpb);
}

int rr_gram(View<const double> S, int q, const double* kappa, const Geo& g, const Phase* ph,
            double* partial, int64_t partial_cap, double* G, double* H, int tile, const Launch& L) {
  if (L.nact <= 0) return 0;
  if (q <= MQ) {
    const int nb = rr_mfma_blocks(g.nm);
    if ((int64_t)nb * q * q * 4 * L.nact > partial_cap) return -1;
    int64_t rpb = (g.nm + nb - 1) / nb;
    rpb = (rpb + 3) / 4 * 4;
    const size_t lds = (size_t)2 * 64 * 8 * MP * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)k_rr_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr = true;
    }
    k_rr_mfma<<<dim3((unsigned)nb, 1, (unsigned)L.nact), 128 * MW, lds, L.st>>>(S, q, kappa, g, ph, rpb, partial,
                                                                                L.slots);
    const int64_t cnt = (int64_t)q * q * 4;
    k_rr_reduce<<<dim3((unsigned)((cnt + 63) / 64), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H,
                                                                                      L.slots);
    return 0;
  }
  const int nb = rr_blocks(g.nm);
  if ((int64_t)nb * q * q * 4 * L.nact > partial_cap) return -1;
  int64_t rpb = (g.nm + nb - 1) / nb;
  rpb = (rpb + CH - 1) / CH * CH;
  const int TB = tile == 4 ? 64 : 48;
  const int nt = (q + TB - 1) / TB;
  dim3 grid((unsigned)nb, (unsigned)(nt * nt), (unsigned)L.nact);
  if (tile == 4) k_rr_gram<4><<<grid, 256, 0, L.st>>>(S, q, kappa, g, ph, rpb, partial, L.slots);
  else k_rr_gram<3><<<grid, 256, 0, L.st>>>(S, q, kappa, g, ph, rpb, partial, L.slots);
  const int64_t cnt = (int64_t)q * q * 4;
  k_rr_reduce<<<dim3((unsigned)((cnt + 63) / 64), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H, L.slots);
  return 0;
}

}  // namespace bl
