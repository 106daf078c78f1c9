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
// Bases of at most 144 columns take the matrix cores instead: FP64 MFMA 16x16x4 products, the
// columns cut into groups of 48 (three 16-column tiles): one launch for the diagonal blocks
// (each group against itself, the upper tile pairs), one for the cross blocks (two groups
// staged side by side, all nine tile pairs, mirrored into the lower triangle).  One
// workgroup of eight waves (four for G, four for H) owns a slice of 16 nodes of a band of
// rows and one block, and streams the rows through an LDS ring:
// x-edge rows r-1, r, r+1 and the y-edge row r (with one halo node either side), stored as
// fetch() returns them, with the next rows prefetched into registers while the current row
// is computed (one barrier per row; every basis value is read from memory once per band).
// Each lane forms, for one node of a group of four and one column of each 16-column tile,
// the basis values and mass products (G) or the scaled cell curls (H) from LDS directly in
// the operand layout of the instruction; the six upper tile pairs are accumulated in
// registers and the waves' sums are combined in a fixed order before one partial per slice
// and band is written.
#include "stencil_common.h"

#include <type_traits>

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
  // blockIdx.y enumerates the upper tile blocks (bi <= bj) row by row; entries below the
  // diagonal are not summed but mirrored from the upper ones (Hermitian), so every kept entry
  // (i <= j) is summed in the same order whatever the tile width
  const int ntj = (q + TB - 1) / TB;
  int bi = 0, rem = (int)blockIdx.y;
  while (rem >= ntj - bi) { rem -= ntj - bi; ++bi; }
  const int ti0 = bi * TB, tj0 = (bi + rem) * TB;
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
      if (i <= j && j < q) {
        const int64_t e = 2 * ((int64_t)i * q + j), f = 2 * ((int64_t)j * q + i);
        pg[e] = gr[a][b];
        pg[e + 1] = gi[a][b];
        ph[e] = hr[a][b];
        ph[e + 1] = hi[a][b];
        if (i != j) {
          pg[f] = gr[a][b];
          pg[f + 1] = -gi[a][b];
          ph[f] = hr[a][b];
          ph[f + 1] = -hi[a][b];
        }
      }
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int MQ = 48;          // columns of one group of the matrix-core path (3 tiles of 16)
constexpr int MT = MQ / 16;     // column tiles per group
constexpr int MW = 4;           // waves per product (G or H) in a workgroup
constexpr int SW = 4 * MW;      // nodes per row of a workgroup's slice (one group of 4 per wave)
constexpr int XS = 4;           // x-edge row slots of the ring (rows r-1, r, r+1 in use, r+2 filling)
constexpr int YW = SW + 2;      // y-edge row with one node either side
constexpr int RR_THREADS = 128 * MW;
constexpr int kMfmaGroups = 3;  // bases up to 3 groups (144 columns) take the matrix cores

// A workgroup stages NG column groups: NG = 1 for a diagonal block of G and H (the upper tile
// pairs of its three tiles), NG = 2 for the cross block of two groups (all nine tile pairs).
template <int NG>
struct RRConf {
  static constexpr int NC = NG * MQ;           // staged columns
  static constexpr int CP = NC + 4;            // LDS stride of a node's columns (complex; padded)
  static constexpr int NT = NG * MT;           // staged tiles
  static constexpr int MP = NG == 1 ? MT * (MT + 1) / 2 : MT * MT;   // tile pairs
  static constexpr int ITEMS = SW * NC + YW * NC + SW;
  static constexpr int PER_THREAD = (ITEMS + RR_THREADS - 1) / RR_THREADS;
};
// tile pair k -> staged tiles (ti, tj): NG = 1 the upper pairs of tiles 0..2, NG = 2 tiles
// 0..2 (first group) against 3..5 (second group)
template <int NG>
__host__ __device__ constexpr int pair_ti(int k) { return NG == 1 ? (k < 3 ? 0 : (k < 5 ? 1 : 2)) : k / 3; }
template <int NG>
__host__ __device__ constexpr int pair_tj(int k) { return NG == 1 ? (k < 3 ? k : (k < 5 ? k - 2 : 2)) : 3 + k % 3; }

#define BL_MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

// The workgroup's staging: x-edge rows in a ring of XS slots (row e in slot (e - r0 + 1) mod
// XS), y-edge rows in two slots with the scaled curl weights of their cells; per node the
// staged columns at stride CP (complex).  Values are stored as fetch() returns them for the
// row's extended index (times beta one period up, conj(beta) one period back; the y halo
// times alpha / conj(alpha)), zero for columns >= q and nodes past the grid.
template <int NG>
struct RRStage {
  double2 x[XS][SW][RRConf<NG>::CP];
  double2 y[2][YW][RRConf<NG>::CP];
  double2 w[2][SW];   // scaled curl weight of the row's cells (first component)
};

// Staged column c of a workgroup with group bases cA (and cB): global column.
template <int NG>
__device__ __forceinline__ int staged_col(int c, int cA, int cB) {
  return (NG == 1 || c < MQ) ? cA + c : cB + (c - MQ);
}

// Staged item e of a row pair: x-edge (node, column) of a row for e < SW NC, then y-edge
// (halo node, column) of a row, then the cell coefficient kappa of the cells of that row.
// What does not change from row to row is worked out once per thread (RRItem): the address
// of the item's value in row 0, its LDS position within a row slot, its kind, the Bloch
// factor of a y halo node (alpha or its conjugate past the slice's left / right end of the
// period) and whether it lies inside the basis and the grid.  A row then costs a pointer
// offset, two loads and, at the store, the Bloch factor of the row (x rows one period up or
// back take beta or its conjugate) or of the halo node.
struct RRItem {
  const double* base;   // value of the item in row 0; the slot's first value when not in use
  int info;             // LDS offset (bits 0-15), kind (16-17: 0 x, 1 y, 2 kappa, 3 none),
                        // halo phase (18-19: 1 times alpha, 2 times conj(alpha)), in use (20)
};
struct RRRaw {
  double a, b;
};

template <int NG>
__device__ __forceinline__ RRItem rr_plan(int e, const double* S, int q, int64_t N, int64_t nm, int n,
                                          const double* kap, int c0, int cA, int cB) {
  constexpr int NC = RRConf<NG>::NC, CP = RRConf<NG>::CP, NX = SW * NC, NY = YW * NC;
  if (e >= RRConf<NG>::ITEMS) return RRItem{S, 3 << 16};
  if (e < NX) {
    const int col = staged_col<NG>(e / SW, cA, cB), j = c0 + e % SW;
    const bool ok = col < q && j < n;
    return RRItem{ok ? S + (int64_t)col * 2 * N + j : S, ((e % SW) * CP + e / SW) | (ok ? 1 << 20 : 0)};
  }
  if (e < NX + NY) {
    const int ey = e - NX;
    const int col = staged_col<NG>(ey / YW, cA, cB);
    int j = c0 - 1 + ey % YW;
    const int ph = j < 0 ? 2 : (j == n ? 1 : 0);
    const bool ok = col < q && j <= n;
    j = j < 0 ? j + n : (j == n ? 0 : j);
    return RRItem{ok ? S + (int64_t)col * 2 * N + nm + j : S,
                  ((ey % YW) * CP + ey / YW) | (1 << 16) | (ph << 18) | (ok ? 1 << 20 : 0)};
  }
  const int ew = e - NX - NY, j = c0 + ew;
  const bool ok = j < n;
  return RRItem{ok ? kap + j : kap, ew | (2 << 16) | (ok ? 1 << 20 : 0)};
}

// Issue the item's loads for x row offset xoff / y row offset yoff (in values); an item not in
// use (or a row not wanted) reads its base, a valid address.
__device__ __forceinline__ RRRaw rr_load(const RRItem& it, int64_t xoff, int64_t yoff, bool want, int64_t N) {
  const int kind = (it.info >> 16) & 3;
  const bool use = want && (it.info & (1 << 20));
  const int64_t off = use ? (kind == 0 ? xoff : yoff) : 0;
  const double* ptr = it.base + off;
  return RRRaw{ptr[0], ptr[kind == 2 ? 0 : N]};
}

// Store the item into its x slot / y slot / weight slot, with the Bloch factor of its row
// (x: code xcode, uniform over the workgroup; 1 times beta, 2 times conj(beta)) or of its halo
// node (y); zero when not in use.
template <int NG>
__device__ __forceinline__ void rr_store(RRStage<NG>& st, const RRItem& it, const RRRaw& raw, bool want, int xcode,
                                         const Ph<double>& p, double s, int xslot, int yslot, bool with_y) {
  const int kind = (it.info >> 16) & 3;
  if (kind == 3 || (kind != 0 && !with_y)) return;
  const bool use = want && (it.info & (1 << 20));
  Cx<double> v = {raw.a, raw.b};
  if (kind == 0) {
    if (xcode) v = cmul(v, p.br, xcode & 2 ? -p.bi : p.bi);
  } else if (kind == 1) {
    const int hcode = (it.info >> 18) & 3;
    if (hcode) v = cmul(v, p.ar, hcode & 2 ? -p.ai : p.ai);
  } else {
    v = Cx<double>{sqrt(raw.a * s), 0.0};
  }
  double2* dst = kind == 0 ? &st.x[xslot][0][0] : (kind == 1 ? &st.y[yslot][0][0] : &st.w[yslot][0]);
  dst[it.info & 0xffff] = use ? double2{v.re, v.im} : double2{0.0, 0.0};
}

// x row xr (in [-1, m + 1]) of the extended grid: its stored row offset and Bloch code
__device__ __forceinline__ void rr_xrow(int xr, int n, int m, int64_t& off, int& code) {
  code = 0;
  if (xr < 0) { xr += m; code = 2; } else if (xr >= m) { xr -= m; code = 1; }
  off = (int64_t)xr * n;
}

// Group bases of workgroup row blockIdx.y: NG = 1, diagonal block y (columns 48 y ..);
// NG = 2, the y-th cross pair (I < J) in row order.
template <int NG>
__device__ __forceinline__ void group_bases(int y, int ngroups, int& cA, int& cB) {
  if (NG == 1) {
    cA = MQ * y;
    cB = cA;
    return;
  }
  int I = 0, rem = y;
  while (rem >= ngroups - 1 - I) { rem -= ngroups - 1 - I; ++I; }
  cA = MQ * I;
  cB = MQ * (I + 1 + rem);
}

// Cross blocks (NG = 2): wave w of a product takes the tile pairs [KB, KB + KC) of the nine
// (KB = 0, KC = 5 for w < 2; KB = 5, KC = 4 otherwise) over the eight nodes 8 (w & 1) .. + 7 of
// the slice (two groups of four), so that its accumulators and operands stay in registers.
template <int KB, int KC>
__device__ __forceinline__ void cross_g(const RRStage<2>& st, int s0, int sp, int sm, int sy, int nb8, int lane,
                                        bool node_ok0, bool node_ok1, double mxs, double mys, d4* ar, d4* ai) {
  constexpr int TI0 = pair_ti<2>(KB), TI1 = pair_ti<2>(KB + KC - 1);   // first-side tiles used
  const double two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
  const int cl = lane & 15;
#pragma unroll
  for (int gsub = 0; gsub < 2; ++gsub) {
    const int jn = nb8 + 4 * gsub + (lane >> 4);
    const bool node_ok = gsub ? node_ok1 : node_ok0;
    double ur[MT][2], ui[MT][2], vr[MT][2], vi[MT][2];
#pragma unroll
    for (int ta = TI0; ta <= TI1; ++ta) {
      const int c = 16 * ta + cl;
      const double2 x0 = st.x[s0][jn][c], y0 = st.y[sy][jn + 1][c];
      ur[ta][0] = x0.x; ui[ta][0] = x0.y;
      ur[ta][1] = node_ok ? y0.x : 0.0; ui[ta][1] = node_ok ? y0.y : 0.0;
    }
#pragma unroll
    for (int tb = 0; tb < MT; ++tb) {
      const int c = MQ + 16 * tb + cl;
      const double2 x0 = st.x[s0][jn][c], xu = st.x[sp][jn][c], xd = st.x[sm][jn][c];
      const double2 y0 = st.y[sy][jn + 1][c], yr = st.y[sy][jn + 2][c], yl = st.y[sy][jn][c];
      const Cx<double> mx = mxs * ((two3 * Cx<double>{x0.x, x0.y}) + one6 * (Cx<double>{xu.x, xu.y} + Cx<double>{xd.x, xd.y}));
      const Cx<double> my = mys * ((two3 * Cx<double>{y0.x, y0.y}) + one6 * (Cx<double>{yr.x, yr.y} + Cx<double>{yl.x, yl.y}));
      vr[tb][0] = mx.re; vi[tb][0] = mx.im; vr[tb][1] = my.re; vi[tb][1] = my.im;
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int A = pair_ti<2>(KB + kk), B = pair_tj<2>(KB + kk) - MT;
      ar[kk] = BL_MFMA(ur[A][0], vr[B][0], ar[kk]);
      ar[kk] = BL_MFMA(ui[A][0], vi[B][0], ar[kk]);
      ar[kk] = BL_MFMA(ur[A][1], vr[B][1], ar[kk]);
      ar[kk] = BL_MFMA(ui[A][1], vi[B][1], ar[kk]);
      ai[kk] = BL_MFMA(ur[A][0], vi[B][0], ai[kk]);
      ai[kk] = BL_MFMA(-ui[A][0], vr[B][0], ai[kk]);
      ai[kk] = BL_MFMA(ur[A][1], vi[B][1], ai[kk]);
      ai[kk] = BL_MFMA(-ui[A][1], vr[B][1], ai[kk]);
    }
  }
}
template <int KB, int KC>
__device__ __forceinline__ void cross_h(const RRStage<2>& st, int s0, int sp, int sy, int nb8, int lane, d4* ar,
                                        d4* ai) {
  constexpr int TI0 = pair_ti<2>(KB), TI1 = pair_ti<2>(KB + KC - 1);
  const int cl = lane & 15;
#pragma unroll
  for (int gsub = 0; gsub < 2; ++gsub) {
    const int jn = nb8 + 4 * gsub + (lane >> 4);
    const double wsc = st.w[sy][jn].x;
    double wr[2 * MT], wi[2 * MT];
#pragma unroll
    for (int tt = 0; tt < 2 * MT; ++tt) {
      if (tt < MT && (tt < TI0 || tt > TI1)) continue;
      const int c = 16 * tt + cl;
      const double2 x0 = st.x[s0][jn][c], xu = st.x[sp][jn][c];
      const double2 y0 = st.y[sy][jn + 1][c], yr = st.y[sy][jn + 2][c];
      const Cx<double> c0v = wsc * (Cx<double>{xu.x, xu.y} - Cx<double>{x0.x, x0.y} + Cx<double>{y0.x, y0.y} -
                                    Cx<double>{yr.x, yr.y});
      wr[tt] = c0v.re;
      wi[tt] = c0v.im;
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int A = pair_ti<2>(KB + kk), B = pair_tj<2>(KB + kk);
      ar[kk] = BL_MFMA(wr[A], wr[B], ar[kk]);
      ar[kk] = BL_MFMA(wi[A], wi[B], ar[kk]);
      ai[kk] = BL_MFMA(wr[A], wi[B], ai[kk]);
      ai[kk] = BL_MFMA(-wi[A], wr[B], ai[kk]);
    }
  }
}

// One workgroup per slice of SW nodes x band of rows [r0, r1) of a slot and per column block
// (blockIdx.y): waves 0..MW-1 form G, waves MW..2MW-1 form H, wave w of a product taking the
// nodes 4w .. 4w+3 of each row.  Rows stream through the LDS ring with a one-row prefetch in
// registers and one barrier per row; the waves' sums are combined in a fixed order and the
// block's entries of G and H (with their Hermitian mirrors) written to the slice's partial.
template <int NG>
__global__ __launch_bounds__(RR_THREADS) void k_rr_mfma(View<const double> Sv, int q, const double* __restrict__ kappa,
                                                        Geo g, const Phase* __restrict__ phs, int slices, int band,
                                                        int ngroups, double* __restrict__ partial,
                                                        const int* __restrict__ slots) {
  using C = RRConf<NG>;
  constexpr int NT = C::NT, MP = C::MP, PT = C::PER_THREAD;
  extern __shared__ double lds[];
  RRStage<NG>& st = *reinterpret_cast<RRStage<NG>*>(lds);
  const int slot = slots ? slots[blockIdx.z] : (int)blockIdx.z;
  int cA, cB;
  group_bases<NG>((int)blockIdx.y, ngroups, cA, cB);
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
  RRItem items[PT];
#pragma unroll
  for (int u = 0; u < PT; ++u) items[u] = rr_plan<NG>(tid + u * RR_THREADS, S, q, N, nm, n, kap, c0, cA, cB);
  // rows r0-1, r0, r0+1 (x) and r0 (y) straight into LDS (all loads issued first)
  {
    RRRaw ini[3][PT];
    int xc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int64_t xo;
      rr_xrow(r0 - 1 + k, n, m, xo, xc[k]);
#pragma unroll
      for (int u = 0; u < PT; ++u) ini[k][u] = rr_load(items[u], xo, (int64_t)r0 * n, true, N);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int u = 0; u < PT; ++u)
        rr_store<NG>(st, items[u], ini[k][u], true, xc[k], p, g.s, xslot(r0 - 1 + k), r0 & 1, k == 1);
  }
  // prefetch of rows r0+2 (x) and r0+1 (y)
  RRRaw pf[PT];
  int pf_code;
  {
    int64_t xo;
    rr_xrow(r0 + 2, n, m, xo, pf_code);
#pragma unroll
    for (int u = 0; u < PT; ++u) pf[u] = rr_load(items[u], xo, (int64_t)(r0 + 1) * n, r0 + 1 < r1, N);
  }
  constexpr int NA = NG == 1 ? MP : 5;   // accumulators per wave (cross blocks: half the pairs)
  d4 ar[NA], ai[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) ar[k] = ai[k] = d4{0, 0, 0, 0};
  const double two3 = 2.0 / 3.0, one6 = 1.0 / 6.0;
  const int half = w >> 1, nb8 = 8 * (w & 1);   // cross blocks: pair half and node octet
  const int jn = 4 * w + (lane >> 4);   // this lane's node in the slice
  const int cl = lane & 15;             // and column in each tile
  for (int r = r0; r < r1; ++r) {
    __syncthreads();   // rows up to r + 1 staged; the slots written below are no longer read
    if (r + 1 < r1) {
#pragma unroll
      for (int u = 0; u < PT; ++u)
        rr_store<NG>(st, items[u], pf[u], true, pf_code, p, g.s, xslot(r + 2), (r + 1) & 1, true);
      int64_t xo;
      rr_xrow(r + 3, n, m, xo, pf_code);
      const bool want = r + 2 < r1;
#pragma unroll
      for (int u = 0; u < PT; ++u) pf[u] = rr_load(items[u], xo, (int64_t)(r + 2) * n, want, N);
    }
    const int sm = xslot(r - 1), s0 = xslot(r), sp = xslot(r + 1), sy = r & 1;
    if (NG == 2) {
      if (!is_h) {
        const bool ok0 = c0 + nb8 + (lane >> 4) < n, ok1 = c0 + nb8 + 4 + (lane >> 4) < n;
        if (half == 0) cross_g<0, 5>(*reinterpret_cast<const RRStage<2>*>(&st), s0, sp, sm, sy, nb8, lane, ok0, ok1, g.mx, g.my, ar, ai);
        else cross_g<5, 4>(*reinterpret_cast<const RRStage<2>*>(&st), s0, sp, sm, sy, nb8, lane, ok0, ok1, g.mx, g.my, ar, ai);
      } else {
        if (half == 0) cross_h<0, 5>(*reinterpret_cast<const RRStage<2>*>(&st), s0, sp, sy, nb8, lane, ar, ai);
        else cross_h<5, 4>(*reinterpret_cast<const RRStage<2>*>(&st), s0, sp, sy, nb8, lane, ar, ai);
      }
    } else if (!is_h) {
      // G = sum over edges of conj(u) (M u): u of the pairs' first tiles, M u of their second
      const bool node_ok = c0 + jn < n;
      double ur[NT][2], ui[NT][2], vr[NT][2], vi[NT][2];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const int c = 16 * tt + cl;
        const double2 x0 = st.x[s0][jn][c], y0 = st.y[sy][jn + 1][c];
        // u of nodes past the grid is zero (their y-edge slot may hold the wrapped halo value)
        ur[tt][0] = x0.x; ui[tt][0] = x0.y;
        ur[tt][1] = node_ok ? y0.x : 0.0; ui[tt][1] = node_ok ? y0.y : 0.0;
        const double2 xu = st.x[sp][jn][c], xd = st.x[sm][jn][c];
        const double2 yr = st.y[sy][jn + 2][c], yl = st.y[sy][jn][c];
        const Cx<double> mx = g.mx * ((two3 * Cx<double>{x0.x, x0.y}) + one6 * (Cx<double>{xu.x, xu.y} + Cx<double>{xd.x, xd.y}));
        const Cx<double> my = g.my * ((two3 * Cx<double>{y0.x, y0.y}) + one6 * (Cx<double>{yr.x, yr.y} + Cx<double>{yl.x, yl.y}));
        vr[tt][0] = mx.re; vi[tt][0] = mx.im; vr[tt][1] = my.re; vi[tt][1] = my.im;
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        const int A = pair_ti<NG>(k), B = pair_tj<NG>(k);
        ar[k] = BL_MFMA(ur[A][0], vr[B][0], ar[k]);
        ar[k] = BL_MFMA(ui[A][0], vi[B][0], ar[k]);
        ar[k] = BL_MFMA(ur[A][1], vr[B][1], ar[k]);
        ar[k] = BL_MFMA(ui[A][1], vi[B][1], ar[k]);
        ai[k] = BL_MFMA(ur[A][0], vi[B][0], ai[k]);
        ai[k] = BL_MFMA(-ui[A][0], vr[B][0], ai[k]);
        ai[k] = BL_MFMA(ur[A][1], vi[B][1], ai[k]);
        ai[k] = BL_MFMA(-ui[A][1], vr[B][1], ai[k]);
      }
    } else {
      // H = sum over cells of (kappa s) conj(w) w, w the cell curl
      double wr[NT], wi[NT];
      const double wsc = st.w[sy][jn].x;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const int c = 16 * tt + cl;
        const double2 x0 = st.x[s0][jn][c], xu = st.x[sp][jn][c];
        const double2 y0 = st.y[sy][jn + 1][c], yr = st.y[sy][jn + 2][c];
        const Cx<double> c0v = wsc * (Cx<double>{xu.x, xu.y} - Cx<double>{x0.x, x0.y} + Cx<double>{y0.x, y0.y} -
                                      Cx<double>{yr.x, yr.y});
        wr[tt] = c0v.re;
        wi[tt] = c0v.im;
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        const int A = pair_ti<NG>(k), B = pair_tj<NG>(k);
        ar[k] = BL_MFMA(wr[A], wr[B], ar[k]);
        ar[k] = BL_MFMA(wi[A], wi[B], ar[k]);
        ai[k] = BL_MFMA(wr[A], wi[B], ai[k]);
        ai[k] = BL_MFMA(-wi[A], wr[B], ai[k]);
      }
    }
  }
  __syncthreads();   // the ring is reused for the combination
  // combine the waves of each product in a fixed order: diagonal blocks waves 0 .. MW-1 (each
  // holds every pair for its nodes); cross blocks the two node octets of each pair half
  double* red = lds;
  if (NG == 1) {
    double* mine = red + ((size_t)(is_h ? 1 : 0) * 64 + lane) * 8 * MP;
    for (int src = 0; src < MW; ++src) {
      if (w == src) {
#pragma unroll
        for (int k = 0; k < NA; ++k)
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
  } else {
    const int kb = half ? 5 : 0, kc = half ? 4 : 5;
    double* mine = red + ((size_t)(is_h ? 1 : 0) * 64 + lane) * 8 * MP;
    for (int oct = 0; oct < 2; ++oct) {
      if ((w & 1) == oct) {
#pragma unroll
        for (int kk = 0; kk < NA; ++kk) {
          if (kk >= kc) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* e = mine + 8 * (kb + kk) + 2 * v;
            if (oct == 0) {
              e[0] = ar[kk][v];
              e[1] = ai[kk][v];
            } else {
              e[0] += ar[kk][v];
              e[1] += ai[kk][v];
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // write the block's entries of G and H (q x q, interleaved complex) with their mirrors
  double* pg = partial + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * (int64_t)q * q * 4;
  for (int e = threadIdx.x; e < 2 * 64 * MP * 4; e += RR_THREADS) {
    const int prod = e / (64 * MP * 4), l = (e / (MP * 4)) % 64, k = (e / 4) % MP, v = e % 4;
    const int ti = pair_ti<NG>(k), tj = pair_tj<NG>(k);
    const int i = staged_col<NG>(16 * ti + 4 * v + (l >> 4), cA, cB), j = staged_col<NG>(16 * tj + (l & 15), cA, cB);
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
  if (q <= kMfmaGroups * MQ) {
    const RRGrid grd = rr_mfma_grid(g);
    const int nb = grd.blocks;
    if ((int64_t)nb * q * q * 4 * L.nact > partial_cap) return -1;
    const int ngroups = (q + MQ - 1) / MQ;
    auto launch = [&](auto ngt, int blocks_y) {
      constexpr int NG = decltype(ngt)::value;
      const size_t red = (size_t)2 * 64 * 8 * RRConf<NG>::MP * sizeof(double);
      const size_t lds = sizeof(RRStage<NG>) > red ? sizeof(RRStage<NG>) : red;
      static const bool attr = [&] {   // once per instantiation, thread-safely
        (void)hipFuncSetAttribute((const void*)k_rr_mfma<NG>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return true;
      }();
      (void)attr;
      k_rr_mfma<NG><<<dim3((unsigned)nb, (unsigned)blocks_y, (unsigned)L.nact), RR_THREADS, lds, L.st>>>(
          S, q, kappa, g, ph, grd.slices, grd.band, ngroups, partial, L.slots);
    };
    launch(std::integral_constant<int, 1>{}, ngroups);
    if (ngroups > 1) launch(std::integral_constant<int, 2>{}, ngroups * (ngroups - 1) / 2);
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
  dim3 grid((unsigned)nb, (unsigned)(nt * (nt + 1) / 2), (unsigned)L.nact);
  if (tile == 4) k_rr_gram<4><<<grid, 256, 0, L.st>>>(S, q, kappa, g, ph, rpb, partial, L.slots);
  else k_rr_gram<3><<<grid, 256, 0, L.st>>>(S, q, kappa, g, ph, rpb, partial, L.slots);
  const int64_t cnt = (int64_t)q * q * 4;
  k_rr_reduce<<<dim3((unsigned)((cnt + 15) / 16), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H, L.slots);
  return 0;
}

}  // namespace bl
