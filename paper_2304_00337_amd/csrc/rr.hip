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

// G_s, H_s = sums over the node ranges of launch entry z, in range order.
__global__ void k_rr_reduce(const double* __restrict__ partial, int nblk, int q, double* __restrict__ G,
                            double* __restrict__ H, const int* __restrict__ slots) {
  const int z = blockIdx.y;
  const int64_t slot = slots ? slots[z] : z;
  const int64_t cnt = (int64_t)q * q * 4;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const double* p = partial + (int64_t)z * nblk * cnt;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += p[(int64_t)b * cnt + e];
  const int64_t half = (int64_t)q * q * 2;
  if (e < half) G[slot * half + e] = s;
  else H[slot * half + e - half] = s;
}

}  // namespace

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
  k_rr_reduce<<<dim3((unsigned)((cnt + 255) / 256), (unsigned)L.nact), 256, 0, L.st>>>(partial, nb, q, G, H, L.slots);
  return 0;
}

}  // namespace bl
