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
// instead: FP64 MFMA 16x16x4 products.  One workgroup of eight waves (four for G, four for
// H) owns a slice of 16 nodes of a band of rows and streams the rows through an LDS ring:
// x-edge rows r-1, r, r+1 and the y-edge row r (with one halo node either side), stored as
// fetch() returns them, with the next rows prefetched into registers while the current row
// is computed (one barrier per row; every basis value is read from memory once per band).
// Each lane forms, for one node of a group of four and one column of each 16-column tile,
// the basis values and mass products (G) or the scaled cell curls (H) from LDS directly in
// the operand layout of the instruction; the six upper tile pairs are accumulated in
// registers and the waves' sums are combined in a fixed order before one partial per slice
// and band is written.
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
constexpr int SW = 4 * MW;      // nodes per row of a workgroup's slice (one group of 4 per wave)
constexpr int CP = MQ + 4;      // LDS stride of a node's columns (complex; padded against bank conflicts)
constexpr int XS = 4;           // x-edge row slots of the ring (rows r-1, r, r+1 in use, r+2 filling)
constexpr int YW = SW + 2;      // y-edge row with one node either side

#define BL_MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

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

// Operands of one 16-column tile for G = sum over edges of conj(u) (M u): the x- and y-edge
// values (u) and their mass products (v), per component [0] x, [1] y.
struct GTile {
  double ur[2], ui[2], vr[2], vi[2];
};
// Operands of one tile for H = sum over cells of (kappa s) conj(w) w: the cell curl scaled
// by sqrt(kappa s).
struct HTile {
  double wr, wi;
};

// The workgroup's staging: x-edge rows in a ring of XS slots (row e in slot (e - r0 + 1) mod
// XS), y-edge rows in two slots with the scaled curl weights of their cells; per node the
// columns at stride CP (complex).  Values are stored as fetch() returns them for the row's
// extended index (times beta one period up, conj(beta) one period back; the y halo times
// alpha / conj(alpha)), zero for columns >= q and nodes past the grid.
struct RRStage {
  double2 x[XS][SW][CP];
  double2 y[2][YW][CP];
  double w[2][SW];
};

// Staged item e of a row pair: x-edge (node, column) of row xrow for e < SW MQ, then y-edge
// (halo node, column) of row yrow, then the cell coefficient kappa of the cells of row yrow.
// rr_fetch issues the loads only (from a valid address in every case, so that no value is
// waited for before it is stored), with a code for what rr_put applies: bit 3 zero (not
// wanted, or outside the basis / grid), bits 0-1 the Bloch factor (1: times the phase, 2:
// times its conjugate), bit 2 the factor is alpha (y halo) instead of beta (x rows).
struct RRRaw {
  double a, b;
  int code;
};

__device__ __forceinline__ RRRaw rr_fetch(int e, const double* S, int q, int64_t N, int64_t nm, int n, int m,
                                          const double* kap, int c0, int xrow, int yrow, bool want) {
  // branch-free: the three kinds' addresses are formed side by side and selected, and every
  // lane issues its two loads, so that nothing waits for the values here
  constexpr int NX = SW * MQ, NY = YW * MQ;
  const bool isx = e < NX, isy = !isx && e < NX + NY, isw = !isx && !isy;
  const int ey = e - NX, ew = e - NX - NY;
  // x-edge rows: the row's wrap is the same for the whole workgroup
  int r = xrow, cx = 0;
  if (r < 0) { r += m; cx = 2; } else if (r >= m) { r -= m; cx = 1; }
  const int colx = e / SW, jx = c0 + e % SW;
  const bool okx = colx < q && jx < n;
  // y-edge halo
  const int coly = ey / YW;
  int jy = c0 - 1 + ey % YW, cy = 4;
  cy = jy < 0 ? (cy | 2) : (jy == n ? (cy | 1) : cy);
  const bool oky = coly < q && jy <= n;
  jy = jy < 0 ? jy + n : (jy == n ? 0 : jy);
  // curl weight
  const int jw = c0 + ew;
  const bool okw = jw < n;
  const bool ok = want && (isx ? okx : (isy ? oky : okw));
  const int col = isx ? colx : coly;
  const double* base = isw ? kap : S + (int64_t)((ok && col < q) ? col : 0) * 2 * N;
  int64_t off = isx ? (int64_t)r * n + jx : (isy ? nm + (int64_t)yrow * n + jy : (int64_t)yrow * n + jw);
  off = ok ? off : 0;
  const int64_t str = isw ? 0 : N;
  const int code = ok ? (isx ? cx : (isy ? cy : 0)) : 8;
  return RRRaw{base[off], base[off + str], code};
}

// store item e (applying its code) into the x slot / y slot
__device__ __forceinline__ void rr_put(RRStage& st, int e, const RRRaw& raw, const Ph<double>& p, double s, int xslot,
                                       int yslot, bool with_x, bool with_y) {
  constexpr int NX = SW * MQ, NY = YW * MQ;
  const bool zero = (raw.code & 8) != 0;
  if (e >= NX + NY) {
    if (with_y) st.w[yslot][e - NX - NY] = zero ? 0.0 : sqrt(raw.a * s);
    return;
  }
  Cx<double> v = {raw.a, raw.b};
  const double fr = (raw.code & 4) ? p.ar : p.br, fi = (raw.code & 4) ? p.ai : p.bi;
  if (raw.code & 1) v = cmul(v, fr, fi);
  else if (raw.code & 2) v = cmul(v, fr, -fi);
  const double2 w = zero ? double2{0.0, 0.0} : double2{v.re, v.im};
  if (e < NX) {
    if (with_x) st.x[xslot][e % SW][e / SW] = w;
  } else {
    e -= NX;
    if (with_y) st.y[yslot][e % YW][e / YW] = w;
  }
}

constexpr int RR_ITEMS = SW * MQ + YW * MQ + SW;
constexpr int RR_THREADS = 128 * MW;
constexpr int RR_PER_THREAD = (RR_ITEMS + RR_THREADS - 1) / RR_THREADS;

// One workgroup per slice of SW nodes x band of rows [r0, r1) of a slot: waves 0..MW-1 form
// G, waves MW..2MW-1 form H, wave w of a product taking the nodes 4w .. 4w+3 of each row.
// Rows stream through the LDS ring with a one-row prefetch in registers and one barrier per
// row; the waves' sums are combined in a fixed order and the slice's full G and H written.
__global__ __launch_bounds__(RR_THREADS) void k_rr_mfma(View<const double> Sv, int q, const double* __restrict__ kappa,
                                                        Geo g, const Phase* __restrict__ phs, int slices, int band,
                                                        double* __restrict__ partial, const int* __restrict__ slots) {
  extern __shared__ double lds[];
  RRStage& st = *reinterpret_cast<RRStage*>(lds);
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  const int64_t N = g.ne, nm = g.nm;
  const int n = g.n, m = g.m;
  const double* S = Sv.p + ((int64_t)slot * Sv.cps + Sv.off) * 2 * N;
  const double* kap = kappa + (int64_t)slot * nm;
  const Ph<double> p = cast_phase<double>(phs[slot]);
  const int c0 = (int)(blockIdx.x % slices) * SW;
  const int r0 = (int)(blockIdx.x / slices) * band;
  const int r1 = r0 + band < m ? r0 + band : m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool is_h = wv >= MW;
  const int w = is_h ? wv - MW : wv;
  const int tid = threadIdx.x;
  auto xslot = [&](int e) { return (e - r0 + 1) & (XS - 1); };
  // rows r0-1, r0, r0+1 (x) and r0 (y) straight into LDS (all loads issued first)
  {
    RRRaw ini[3][RR_PER_THREAD];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int u = 0; u < RR_PER_THREAD; ++u) {
        const int e = tid + u * RR_THREADS;
        ini[k][u] = rr_fetch(e < RR_ITEMS ? e : 0, S, q, N, nm, n, m, kap, c0, r0 - 1 + k, r0, e < RR_ITEMS);
      }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int u = 0; u < RR_PER_THREAD; ++u) {
        const int e = tid + u * RR_THREADS;
        if (e < RR_ITEMS) rr_put(st, e, ini[k][u], p, g.s, xslot(r0 - 1 + k), r0 & 1, true, k == 1);
      }
  }
  // prefetch of rows r0+2 (x) and r0+1 (y)
  RRRaw pf[RR_PER_THREAD];
#pragma unroll
  for (int u = 0; u < RR_PER_THREAD; ++u) {
    const int e = tid + u * RR_THREADS;
    pf[u] = rr_fetch(e < RR_ITEMS ? e : 0, S, q, N, nm, n, m, kap, c0, r0 + 2, r0 + 1, e < RR_ITEMS && r0 + 1 < r1);
  }
  d4 ar[MP], ai[MP];
#pragma unroll
  for (int k = 0; k < MP; ++k) ar[k] = ai[k] = d4{0, 0, 0, 0};
  const double two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
  const int jn = 4 * w + (lane >> 4);   // this lane's node in the slice
  const int cl = lane & 15;             // and column in each tile
  for (int r = r0; r < r1; ++r) {
    __syncthreads();   // rows up to r + 1 staged; the slots written below are no longer read
    if (r + 1 < r1) {
#pragma unroll
      for (int u = 0; u < RR_PER_THREAD; ++u) {
        const int e = tid + u * RR_THREADS;
        if (e < RR_ITEMS) rr_put(st, e, pf[u], p, g.s, xslot(r + 2), (r + 1) & 1, true, true);
      }
#pragma unroll
      for (int u = 0; u < RR_PER_THREAD; ++u) {
        const int e = tid + u * RR_THREADS;
        pf[u] = rr_fetch(e < RR_ITEMS ? e : 0, S, q, N, nm, n, m, kap, c0, r + 3, r + 2, e < RR_ITEMS && r + 2 < r1);
      }
    }
    const int sm = xslot(r - 1), s0 = xslot(r), sp = xslot(r + 1), sy = r & 1;
    if (!is_h) {
      const bool node_ok = c0 + jn < n;
      GTile t[MT];
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) {
        const int c = 16 * tt + cl;
        const double2 x0 = st.x[s0][jn][c], xu = st.x[sp][jn][c], xd = st.x[sm][jn][c];
        const double2 y0 = st.y[sy][jn + 1][c], yr = st.y[sy][jn + 2][c], yl = st.y[sy][jn][c];
        const Cx<double> mx = g.mx * ((two3 * Cx<double>{x0.x, x0.y}) + one6 * (Cx<double>{xu.x, xu.y} + Cx<double>{xd.x, xd.y}));
        const Cx<double> my = g.my * ((two3 * Cx<double>{y0.x, y0.y}) + one6 * (Cx<double>{yr.x, yr.y} + Cx<double>{yl.x, yl.y}));
        // u of nodes past the grid is zero (their y-edge slot may hold the wrapped halo value)
        t[tt].ur[0] = x0.x; t[tt].ui[0] = x0.y;
        t[tt].ur[1] = node_ok ? y0.x : 0.0; t[tt].ui[1] = node_ok ? y0.y : 0.0;
        t[tt].vr[0] = mx.re; t[tt].vi[0] = mx.im; t[tt].vr[1] = my.re; t[tt].vi[1] = my.im;
      }
      BL_GPAIR(0, t[0], t[0])
      BL_GPAIR(1, t[0], t[1])
      BL_GPAIR(2, t[0], t[2])
      BL_GPAIR(3, t[1], t[1])
      BL_GPAIR(4, t[1], t[2])
      BL_GPAIR(5, t[2], t[2])
    } else {
      HTile t[MT];
      const double wsc = st.w[sy][jn];
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) {
        const int c = 16 * tt + cl;
        const double2 x0 = st.x[s0][jn][c], xu = st.x[sp][jn][c];
        const double2 y0 = st.y[sy][jn + 1][c], yr = st.y[sy][jn + 2][c];
        const Cx<double> c0v = wsc * (Cx<double>{xu.x, xu.y} - Cx<double>{x0.x, x0.y} + Cx<double>{y0.x, y0.y} -
                                      Cx<double>{yr.x, yr.y});
        t[tt].wr = c0v.re;
        t[tt].wi = c0v.im;
      }
      BL_HPAIR(0, t[0], t[0])
      BL_HPAIR(1, t[0], t[1])
      BL_HPAIR(2, t[0], t[2])
      BL_HPAIR(3, t[1], t[1])
      BL_HPAIR(4, t[1], t[2])
      BL_HPAIR(5, t[2], t[2])
    }
  }
  __syncthreads();   // the ring is reused for the combination
  // combine the waves of each product in order 0 .. MW-1
  double* red = lds;
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
  // write the slice's full G and H (q x q, interleaved complex; lower tiles mirrored)
  double* pg = partial + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * (int64_t)q * q * 4;
  for (int e = threadIdx.x; e < 2 * 64 * MP * 4; e += RR_THREADS) {
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

// G_s, H_s = sums over the node ranges of launch entry z: 16 entries per block, the ranges
// split into sixteen consecutive groups summed in range order, the groups' sums then added
// in order (a fixed order, independent of timing).
__global__ __launch_bounds__(256) void k_rr_reduce(const double* __restrict__ partial, int nblk, int q,
                                                   double* __restrict__ G, double* __restrict__ H,
                                                   const int* __restrict__ slots) {
  __shared__ double part[16][17];
  const int z = blockIdx.y;
  const int64_t slot = slots ? slots[z] : z;
  const int64_t cnt = (int64_t)q * q * 4;
  const int lo = threadIdx.x & 15, gq = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + lo;
  const double* pz = partial + (int64_t)z * nblk * cnt;
  const int b0 = (int)((int64_t)nblk * gq / 16), b1 = (int)((int64_t)nblk * (gq + 1) / 16);
  double sum = 0;
  if (e < cnt)
    for (int b = b0; b < b1; ++b) sum += pz[(int64_t)b * cnt + e];
  part[gq][lo] = sum;
  __syncthreads();
  if (gq == 0 && e < cnt) {
    double t = part[0][lo];
    for (int k = 1; k < 16; ++k) t += part[k][lo];
    const int64_t half = (int64_t)q * q * 2;
    if (e < half) G[slot * half + e] = t;
    else H[slot * half + e - half] = t;
  }
}

}  // namespace

// slices x bands of the matrix-core path: slices of SW nodes, bands of rows so that about
// one workgroup per compute unit runs
struct RRGrid {
  int slices, band, blocks;
};
RRGrid rr_mfma_grid(const Geo& g) {
  const int slices = (g.n + SW - 1) / SW;
  int nbands = 256 / slices;
  if (nbands < 1) nbands = 1;
  if (nbands > g.m) nbands = g.m;
  const int band = (g.m + nbands - 1) / nbands;
  nbands = (g.m + band - 1) / band;
  return {slices, band, slices * nbands};
}

int rr_partial_blocks(const Geo& g) {
  const int a = rr_blocks(g.nm), b = rr_mfma_grid(g).blocks;
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
    const RRGrid grd = rr_mfma_grid(g);
    const int nb = grd.blocks;
    if ((int64_t)nb * q * q * 4 * L.nact > partial_cap) return -1;
    const size_t lds = sizeof(RRStage) > (size_t)2 * 64 * 8 * MP * sizeof(double) ? sizeof(RRStage)
                                                                                 : (size_t)2 * 64 * 8 * MP * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)k_rr_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr = true;
    }
    k_rr_mfma<<<dim3((unsigned)nb, 1, (unsigned)L.nact), RR_THREADS, lds, L.st>>>(S, q, kappa, g, ph, grd.slices,
                                                                                  grd.band, partial, L.slots);
    const int64_t cnt = (int64_t)q * q * 4;
    k_rr_reduce<<<dim3((unsigned)((cnt + 15) / 16), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H,
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
  k_rr_reduce<<<dim3((unsigned)((cnt + 15) / 16), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H, L.slots);
  return 0;
}

}  // namespace bl
