// Fused coarse levels of the V-cycles (Section 5) for gfx950.  Below a size where the
// per-level launches are latency-bound (a few microseconds of dispatch for a few thousand
// unknowns), the rest of a V-cycle — smoothing, residual, restriction, the dense coarsest
// solve, prolongation and post-smoothing on every remaining level — runs in one workgroup
// per column, with all levels' vectors in LDS and a barrier between dependent passes.  The
// per-point bodies are those of the per-level kernels (stencil_ops.h) and the coarsest solve
// sums in the same order as k_dense_apply, so a fused cycle reproduces the per-level one bit
// for bit.
#include "stencil_ops.h"

#include <cstdlib>

#pragma clang fp contract(off)

namespace bl {

namespace {

// Threads per fused workgroup.  Only one workgroup per column runs, so the cycle is latency
// bound: more threads shorten every pass (a 64 x 64 nodal colour pass is one node per thread
// at 1024), at the price of slightly dearer barriers.
constexpr int kFusedMaxThreads = 1024;

template <typename T>
__device__ __forceinline__ const T* pickp(const double* a, const float* b);
template <>
__device__ __forceinline__ const double* pickp<double>(const double* a, const float*) { return a; }
template <>
__device__ __forceinline__ const float* pickp<float>(const double*, const float* b) { return b; }

// LDS vector `which` (0 = iterate x, 1 = right-hand side b, 2 = residual r) of fused level
// l: per level l < nlev-1 the three vectors (2 ne or 2 nm values each), on the coarsest x
// and b.  Offsets are recomputed from the cycle description (no pointer tables in scratch).
template <typename T>
__device__ __forceinline__ T* lds_vec(T* base, const CoarseCycle& C, bool edge, int l, int which) {
  int64_t off = 0;
  for (int i = 0; i < l; ++i) {
    const int64_t len = 2 * (edge ? C.L[i].g.ne : C.L[i].g.nm);
    off += len * (i + 1 < C.nlev ? 3 : 2);
  }
  return base + off + which * 2 * (edge ? C.L[l].g.ne : C.L[l].g.nm);
}

// x = Inv b for the Hermitian inverse of one slot (row i read as the conjugate of column i).
template <typename T>
__device__ void dense_solve(const T* inv, int64_t n, const T* b, T* x) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    T sr = 0, si = 0;
    // (unrolled: the loads of several terms are in flight; the summation order is unchanged)
#pragma unroll 8
    for (int64_t l = 0; l < n; ++l) {
      const T ar = inv[2 * (l * n + i)], ai = -inv[2 * (l * n + i) + 1];
      const T br = b[l], bi = b[n + l];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    x[i] = sr;
    x[n + i] = si;
  }
}

template <typename T>
__device__ void edge_colour(const CoarseCycle& C, int l, int slot, T* x, const T* b, int colour, T mu,
                            const Ph<T>& p) {
  const CoarseLevel& lv = C.L[l];
  const Geo& g = lv.g;
  const int n = g.n, m = g.m, nh = n >> 1, mh = m >> 1;
  const int64_t nm = g.nm;
  const double* k64 = lv.k64 + (int64_t)slot * nm;
  const float* k32 = lv.k32 + (int64_t)slot * nm;
  const T s = (T)g.s, mmx = mu * (T)g.mx, mmy = mu * (T)g.my;
  for (int t = threadIdx.x; t < nh * mh; t += blockDim.x) {
    const int p1 = 2 * (t % nh) + (colour & 1);
    const int p2 = 2 * (t / nh) + (colour >> 1);
    const int p1m = wrapi(p1 - 1, n), p2m = wrapi(p2 - 1, m);
    const T kne = kap<T>(k64, k32, (int64_t)p2 * n + p1);
    const T knw = kap<T>(k64, k32, (int64_t)p2 * n + p1m);
    const T ksw = kap<T>(k64, k32, (int64_t)p2m * n + p1m);
    const T kse = kap<T>(k64, k32, (int64_t)p2m * n + p1);
    const T* si = pickp<T>(lv.si64, lv.si32) + kPatchW * ((int64_t)slot * nm + (int64_t)p2 * n + p1);
    edge_patch_gs<T>(x, b, g.ne, n, m, nm, p1, p2, kne, knw, ksw, kse, si, s, mmx, mmy, p);
  }
}

template <typename T>
__global__ __launch_bounds__(kFusedMaxThreads) void k_edge_vcycle_fused(View<const T> bv, View<T> xv, CoarseCycle C,
                                                           const Phase* __restrict__ phs,
                                                           const double* __restrict__ mus,
                                                           const int* __restrict__ slots, int ncps) {
  extern __shared__ unsigned char lds_raw[];
  const int zi = (int)blockIdx.x / ncps;
  const int slot = slots ? slots[zi] : zi;
  const SJ sj{slot, (int)blockIdx.x % ncps};
  const Ph<T> p = cast_phase<T>(phs[slot]);
  const T mu = (T)mus[slot];
  T* const base = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  {
    const T* bg = colp(bv, sj, C.L[0].g.ne);
    T* b0 = lds_vec(base, C, true, 0, 1);
    for (int64_t i = tid; i < 2 * C.L[0].g.ne; i += nt) b0[i] = bg[i];
  }
  __syncthreads();
  const int last = C.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const Geo& g = C.L[l].g;
    const int64_t N = g.ne;
    T* x = lds_vec(base, C, true, l, 0);
    const T* b = lds_vec(base, C, true, l, 1);
    T* r = lds_vec(base, C, true, l, 2);
    for (int64_t i = tid; i < 2 * N; i += nt) x[i] = (T)0;
    __syncthreads();
    for (int it = 0; it < C.nu_pre; ++it)
      for (int c = 0; c < 4; ++c) {
        edge_colour<T>(C, l, slot, x, b, c, mu, p);
        __syncthreads();
      }
    const double* k64 = C.L[l].k64 + (int64_t)slot * g.nm;
    const float* k32 = C.L[l].k32 + (int64_t)slot * g.nm;
    for (int64_t d = tid; d < N; d += nt) {
      Cx<T> Au, Mu;
      edge_AM<T, T>(x, N, g.n, g.m, g.nm, d, [&](int64_t i) { return kap<T>(k64, k32, i); }, (T)g.s, (T)g.mx,
                    (T)g.my, p, Au, Mu);
      const Cx<T> v = Cx<T>{b[d], b[N + d]} - (Au + (mu * Mu));
      r[d] = v.re;
      r[N + d] = v.im;
    }
    __syncthreads();
    const Geo& gc = C.L[l + 1].g;
    T* bc = lds_vec(base, C, true, l + 1, 1);
    for (int64_t d = tid; d < gc.ne; d += nt) {
      const Cx<T> v = edge_restrict_at<T>(r, g, gc, d, p);
      bc[d] = v.re;
      bc[gc.ne + d] = v.im;
    }
    __syncthreads();
  }
  dense_solve<T>(static_cast<const T*>(C.inv) + (int64_t)slot * C.nc * C.nc * 2, C.nc, lds_vec(base, C, true, last, 1),
                 lds_vec(base, C, true, last, 0));
  __syncthreads();
  for (int l = last - 1; l >= 0; --l) {
    const Geo& g = C.L[l].g;
    const Geo& gc = C.L[l + 1].g;
    T* x = lds_vec(base, C, true, l, 0);
    const T* xc = lds_vec(base, C, true, l + 1, 0);
    for (int64_t d = tid; d < g.ne; d += nt) {
      const Cx<T> v = edge_prolong_at<T>(xc, gc, g, d, p);
      x[d] += v.re;
      x[g.ne + d] += v.im;
    }
    __syncthreads();
    const T* b = lds_vec(base, C, true, l, 1);
    for (int it = 0; it < C.nu_post; ++it)
      for (int c = 3; c >= 0; --c) {
        edge_colour<T>(C, l, slot, x, b, c, mu, p);
        __syncthreads();
      }
  }
  T* xg = colp(xv, sj, C.L[0].g.ne);
  const T* x0 = lds_vec(base, C, true, 0, 0);
  for (int64_t i = tid; i < 2 * C.L[0].g.ne; i += nt) xg[i] = x0[i];
}

template <typename T>
__device__ void nodal_colour(const Geo& g, T* x, const T* b, int colour, const NodalStencil& s, const Ph<T>& p) {
  const int nh = g.n >> 1, mh = g.m >> 1;
  const int64_t N = g.nm;
  const T inv = (T)1 / (T)s.c0;
  for (int t = threadIdx.x; t < nh * mh; t += blockDim.x) {
    const int p1 = 2 * (t % nh) + (colour & 1);
    const int p2 = 2 * (t / nh) + (colour >> 1);
    const int64_t i = (int64_t)p2 * g.n + p1;
    const Cx<T> r = Cx<T>{b[i], b[N + i]} - nodal_stencil<T>(x, N, g.n, g.m, p1, p2, s, p);
    x[i] += inv * r.re;
    x[N + i] += inv * r.im;
  }
}

template <typename T>
__global__ __launch_bounds__(kFusedMaxThreads) void k_nodal_vcycle_fused(View<const T> bv, View<T> xv, CoarseCycle C,
                                                            const Phase* __restrict__ phs,
                                                            const int* __restrict__ slots, int ncps) {
  extern __shared__ unsigned char lds_raw[];
  const int zi = (int)blockIdx.x / ncps;
  const int slot = slots ? slots[zi] : zi;
  const SJ sj{slot, (int)blockIdx.x % ncps};
  const Ph<T> p = cast_phase<T>(phs[slot]);
  T* const base = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  {
    const T* bg = colp(bv, sj, C.L[0].g.nm);
    T* b0 = lds_vec(base, C, false, 0, 1);
    for (int64_t i = tid; i < 2 * C.L[0].g.nm; i += nt) b0[i] = bg[i];
  }
  __syncthreads();
  const int last = C.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const Geo& g = C.L[l].g;
    const int64_t N = g.nm;
    T* x = lds_vec(base, C, false, l, 0);
    const T* b = lds_vec(base, C, false, l, 1);
    T* r = lds_vec(base, C, false, l, 2);
    for (int64_t i = tid; i < 2 * N; i += nt) x[i] = (T)0;
    __syncthreads();
    for (int it = 0; it < C.nu_pre; ++it)
      for (int c = 0; c < 4; ++c) {
        nodal_colour<T>(g, x, b, c, C.ns, p);
        __syncthreads();
      }
    for (int64_t d = tid; d < N; d += nt) {
      const Cx<T> v = Cx<T>{b[d], b[N + d]} - nodal_stencil<T>(x, N, g.n, g.m, (int)(d % g.n), (int)(d / g.n), C.ns, p);
      r[d] = v.re;
      r[N + d] = v.im;
    }
    __syncthreads();
    const Geo& gc = C.L[l + 1].g;
    T* bc = lds_vec(base, C, false, l + 1, 1);
    for (int64_t d = tid; d < gc.nm; d += nt) {
      const Cx<T> v = nodal_restrict_at<T>(r, g, gc, d, p);
      bc[d] = v.re;
      bc[gc.nm + d] = v.im;
    }
    __syncthreads();
  }
  dense_solve<T>(static_cast<const T*>(C.inv) + (int64_t)slot * C.nc * C.nc * 2, C.nc, lds_vec(base, C, false, last, 1),
                 lds_vec(base, C, false, last, 0));
  __syncthreads();
  for (int l = last - 1; l >= 0; --l) {
    const Geo& g = C.L[l].g;
    const Geo& gc = C.L[l + 1].g;
    T* x = lds_vec(base, C, false, l, 0);
    const T* xc = lds_vec(base, C, false, l + 1, 0);
    for (int64_t d = tid; d < g.nm; d += nt) {
      const Cx<T> v = nodal_prolong_at<T>(xc, gc, g, d, p);
      x[d] += v.re;
      x[g.nm + d] += v.im;
    }
    __syncthreads();
    const T* b = lds_vec(base, C, false, l, 1);
    for (int it = 0; it < C.nu_post; ++it)
      for (int c = 3; c >= 0; --c) {
        nodal_colour<T>(g, x, b, c, C.ns, p);
        __syncthreads();
      }
  }
  T* xg = colp(xv, sj, C.L[0].g.nm);
  const T* x0 = lds_vec(base, C, false, 0, 0);
  for (int64_t i = tid; i < 2 * C.L[0].g.nm; i += nt) xg[i] = x0[i];
}

int g_lds_cap = -1;

int lds_cap() {
  if (g_lds_cap < 0) {
    int dev = 0, cap = 65536;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) cap = 65536;
    const void* ks[] = {(const void*)k_edge_vcycle_fused<double>, (const void*)k_edge_vcycle_fused<float>,
                        (const void*)k_nodal_vcycle_fused<double>, (const void*)k_nodal_vcycle_fused<float>};
    for (const void* k : ks)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, cap) != hipSuccess) cap = 65536;
    g_lds_cap = cap;
  }
  return g_lds_cap;
}

}  // namespace

size_t fused_lds_bytes(const CoarseCycle& C, bool edge, size_t elem) {
  size_t b = 0;
  for (int l = 0; l < C.nlev; ++l) {
    const int64_t len = 2 * (edge ? C.L[l].g.ne : C.L[l].g.nm);
    b += (size_t)len * elem * (l + 1 < C.nlev ? 3 : 2);
  }
  return b;
}

size_t fused_lds_limit() { return (size_t)lds_cap(); }

namespace {
// Enough threads for one patch node (edge) or node (nodal) of a colour on the first fused
// level each, between 256 and kFusedMaxThreads.  Results do not depend on it.
int fused_threads(const CoarseCycle& C) {
  static const int forced = [] {
    const char* e = std::getenv("BL_FUSED_THREADS");
    const int v = e ? std::atoi(e) : 0;
    return v >= 64 && v <= kFusedMaxThreads && v % 64 == 0 ? v : 0;
  }();
  if (forced) return forced;
  const int64_t per_colour = C.L[0].g.nm / 4;
  int nt = 256;
  while (nt < kFusedMaxThreads && nt < per_colour) nt *= 2;
  return nt;
}
}  // namespace

template <typename T>
void edge_vcycle_fused(View<const T> b, View<T> x, const CoarseCycle& C, const Phase* ph, const double* mu,
                       const Launch& L) {
  const int nb = L.nact * L.ncps;
  if (nb <= 0) return;
  const size_t lds = fused_lds_bytes(C, true, sizeof(T));
  (void)lds_cap();
  k_edge_vcycle_fused<T><<<nb, fused_threads(C), lds, L.st>>>(b, x, C, ph, mu, L.slots, L.ncps);
}
template <typename T>
void nodal_vcycle_fused(View<const T> b, View<T> x, const CoarseCycle& C, const Phase* ph, const Launch& L) {
  const int nb = L.nact * L.ncps;
  if (nb <= 0) return;
  const size_t lds = fused_lds_bytes(C, false, sizeof(T));
  (void)lds_cap();
  k_nodal_vcycle_fused<T><<<nb, fused_threads(C), lds, L.st>>>(b, x, C, ph, L.slots, L.ncps);
}
template void edge_vcycle_fused<double>(View<const double>, View<double>, const CoarseCycle&, const Phase*, const double*, const Launch&);
template void edge_vcycle_fused<float>(View<const float>, View<float>, const CoarseCycle&, const Phase*, const double*, const Launch&);
template void nodal_vcycle_fused<double>(View<const double>, View<double>, const CoarseCycle&, const Phase*, const Launch&);
template void nodal_vcycle_fused<float>(View<const float>, View<float>, const CoarseCycle&, const Phase*, const Launch&);

}  // namespace bl
