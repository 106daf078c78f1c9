// Plane-wave deflation of the nodal solve in the null-space elimination (Sections 4-5).
//
// P = L^* M L is a constant-coefficient stencil, so the nodal plane wave w of the first-zone
// representative of k is an exact eigenvector; its eigenvalue lambda_w shrinks like
// |k|^2 h^2 next to the Gamma point, where P turns singular.  The projection splits the nodal
// solve along w: the right-hand side b is orthogonalised against w before the V-cycles, the
// cycles' result phi' is orthogonalised after them, and the exact component
// c = w^* b / (nm lambda_w) is added back, all coefficients in FP64.  A single-precision
// cycle therefore never carries the near-singular mode, whose residual it would lose to
// rounding.  The partial sums come in a fixed order (bit-reproducible).
#include "stencil_common.h"
#include "stencil_ops.h"

#include <algorithm>

namespace bl {

__global__ void k_pw_tables(const PlaneWave* __restrict__ par, double* __restrict__ tab, int64_t stride,
                            int n, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n + m) return;
  const PlaneWave q = par[blockIdx.y];
  const double ang = i < n ? q.t1 * (double)i : q.t2 * (double)(i - n);
  double sn, cs;
  sincos(ang, &sn, &cs);
  double* t = tab + (int64_t)blockIdx.y * stride;
  t[2 * i] = cs;
  t[2 * i + 1] = sn;
}

void pw_tables(const PlaneWave* par, double* tab, int64_t tabstride, int n, int m, int nslots, hipStream_t st) {
  if (nslots <= 0) return;
  dim3 grid((unsigned)((n + m + 255) / 256), (unsigned)nslots);
  k_pw_tables<<<grid, 256, 0, st>>>(par, tab, tabstride, n, m);
}

int pw_blocks(const Geo& g) {
  return std::max(point_tiles(g.n, g.m), (int)((g.nm + 255) / 256));
}

// One workgroup per launch column: the column's partials in a fixed order.
__global__ __launch_bounds__(256) void k_pw_reduce(PWDefl d, int mode, int count, const int* __restrict__ slots) {
  const int64_t col = blockIdx.y;
  const double* pp = d.part + col * d.nblk * 2;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
    sr += pp[2 * b];
    si += pp[2 * b + 1];
  }
  __shared__ double tot[2];
  block_sum2(sr, si, tot);
  if (threadIdx.x == 0) {
    const int sidx = (int)(col / d.pcols);
    const PlaneWave& q = d.par[slots ? slots[sidx] : sidx];
    double* c = d.coef + col * 6;
    if (mode == 0) {
      c[0] = tot[0] * q.inm;
      c[1] = tot[1] * q.inm;
      c[2] = tot[0] * q.ilw;
      c[3] = tot[1] * q.ilw;
    } else {
      c[4] = c[2] - tot[0] * q.inm;
      c[5] = c[3] - tot[1] * q.inm;
    }
  }
}

void pw_reduce(const PWDefl& d, int mode, int count, const Launch& L) {
  const int cols = L.nact * d.pcols;
  if (cols == 0) return;
  k_pw_reduce<<<dim3(1, (unsigned)cols), 256, 0, L.st>>>(d, mode, count, L.slots);
}

// kPwPer elements per thread (strided by the block size, so that a wave's accesses stay
// contiguous): fewer, fuller blocks for these streaming passes
constexpr int kPwPer = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_pw_rhs(View<T> bv, Geo g, PWDefl d, const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int n = g.n;
  const int64_t col = (int64_t)(blockIdx.y / ncps) * d.pcols + d.off + sj.j;
  const double* c = d.coef + col * 6;
  T* b = colp(bv, sj, g.nm);
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kPwPer + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kPwPer; ++u) {
    const int64_t i = i0 + (int64_t)u * blockDim.x;
    if (i >= g.nm) break;
    int j1, j2;
    split_index(i, n, j1, j2);
    const Cx<double> w = pw_value(d, sj.slot, n, j1, j2);
    const Cx<double> ws = cmul(w, c[0], c[1]);
    b[i] = (T)((double)b[i] - ws.re);
    b[g.nm + i] = (T)((double)b[g.nm + i] - ws.im);
  }
}

template <typename T>
void pw_rhs(View<T> b, const Geo& g, const PWDefl& d, const Launch& L) {
  dim3 grid((unsigned)((g.nm + 256 * kPwPer - 1) / (256 * kPwPer)), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return;
  k_pw_rhs<T><<<grid, 256, 0, L.st>>>(b, g, d, L.slots, L.ncps);
}
template void pw_rhs<double>(View<double>, const Geo&, const PWDefl&, const Launch&);
template void pw_rhs<float>(View<float>, const Geo&, const PWDefl&, const Launch&);

template <typename T>
__global__ __launch_bounds__(256) void k_pw_dot(View<const T> fv, Geo g, PWDefl d, const int* __restrict__ slots, int ncps) {
  const SJ sj = slot_col(slots, ncps);
  const int n = g.n;
  const T* f = colp(fv, sj, g.nm);
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kPwPer + threadIdx.x;
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int u = 0; u < kPwPer; ++u) {
    const int64_t i = i0 + (int64_t)u * blockDim.x;
    if (i >= g.nm) break;
    int j1, j2;
    split_index(i, n, j1, j2);
    const Cx<double> w = pw_value(d, sj.slot, n, j1, j2);
    const double fr = (double)f[i], fi = (double)f[g.nm + i];
    sr += w.re * fr + w.im * fi;
    si += w.re * fi - w.im * fr;
  }
  const int64_t col = (int64_t)(blockIdx.y / ncps) * d.pcols + d.off + sj.j;
  block_sum2(sr, si, d.part + (col * d.nblk + blockIdx.x) * 2);
}

template <typename T>
int pw_dot(View<const T> phi, const Geo& g, const PWDefl& d, const Launch& L) {
  dim3 grid((unsigned)((g.nm + 256 * kPwPer - 1) / (256 * kPwPer)), (unsigned)(L.nact * L.ncps));
  if (grid.y == 0) return (int)grid.x;
  k_pw_dot<T><<<grid, 256, 0, L.st>>>(phi, g, d, L.slots, L.ncps);
  return (int)grid.x;
}
template int pw_dot<double>(View<const double>, const Geo&, const PWDefl&, const Launch&);
template int pw_dot<float>(View<const float>, const Geo&, const PWDefl&, const Launch&);

}  // namespace bl
