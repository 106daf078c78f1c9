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
// computed by the same per-point code as the per-colour kernels, through accessors that
// read the LDS copy with the same Bloch-phase arithmetic, so the results agree bit for bit.
//
// LDS layout: the box is split by node parity into four sub-grids, so that the patches of
// one colour, which are two nodes apart, sit at consecutive addresses (no bank conflicts)
// and every neighbour of a patch is at a compile-time offset from it.  Only workgroups whose
// box crosses the periodic seam run the phase checks of the Bloch extension.
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
constexpr int kMaxThreads = 512;   // workgroups of 256 threads, or 512 where the launch has few tiles
// (a colour pass of a 32 x 32 tile then takes one round instead of two: the coarser levels'
// launches are too small to hide the rounds' latency behind other workgroups)
__device__ __forceinline__ int nthreads() { return (int)blockDim.x; }

// MODE bits of a sweep with level transfers folded in: kRestrict (forward sweeps) also forms
// the residual of the result and restricts it to the coarse right-hand side; kProlong starts
// from xin + Pr xc; kBase writes base + result.  The residual at the fine nodes that the
// restriction reads (one node below/left of the tile to its last row/column) needs the swept
// iterate two nodes below/left and one node above/right of the tile: the halos grow to kLoR
// below (nodal and edge) and kHiER above (edge; the nodal forward sweep's kHiN suffices).
constexpr int kRestrict = 1, kProlong = 2, kBase = 4;
// kResid (nodal backward sweeps): the sweep also writes the residual b - P x of its result at
// the tile's nodes (as the residual kernel computes it), for which the iterate must be exact
// one node around the tile.
constexpr int kResid = 8;
constexpr int kLoR = 6;
constexpr int kHiER = 6;

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

// Parity-split box: position (bx, by) of a BX x BY box is entry (by/2) HX + bx/2 of
// sub-grid (bx mod 2) + 2 (by mod 2).
template <int BX, int BY>
struct Split {
  static constexpr int HX = (BX + 1) / 2, HY = (BY + 1) / 2, SUB = HX * HY, N = 4 * SUB;
  __device__ static __forceinline__ int at(int bx, int by) {
    return ((bx & 1) + 2 * (by & 1)) * SUB + (by >> 1) * HX + (bx >> 1);
  }
};

// Which neighbours of a node lie across the periodic seam: for a node at canonical (p1, p2)
// the neighbour at offset d1 = -1 crosses when p1 = 0, d1 = +1 when p1 = n - 1 (y alike).
// Only the directions in which the box crosses the seam (CX, CY) are checked.
template <bool CX, bool CY>
struct Seam {
  bool lx, hx, ly, hy;
  __device__ __forceinline__ Seam(int p1, int p2, int n, int m)
      : lx(CX && p1 == 0), hx(CX && p1 == n - 1), ly(CY && p2 == 0), hy(CY && p2 == m - 1) {}
  __device__ __forceinline__ bool cross_x(int d1) const { return CX && ((d1 < 0 && lx) || (d1 > 0 && hx)); }
  __device__ __forceinline__ bool cross_y(int d2) const { return CY && ((d2 < 0 && ly) || (d2 > 0 && hy)); }
};

template <typename T>
__device__ __forceinline__ Cx<T> pick(bool c, Cx<T> a, Cx<T> b) {
  return {c ? a.re : b.re, c ? a.im : b.im};
}

// The value at offset (d1, d2) as fetch() returns it: times alpha (one period ahead) or
// conj(alpha) (one period back) across the x seam, then beta likewise across the y seam.
// The products are formed unconditionally and selected per lane, so that workgroups on the
// seam run the same instructions in every lane.
template <bool CX, bool CY, typename T>
__device__ __forceinline__ Cx<T> phased(Cx<T> v, int d1, int d2, const Seam<CX, CY>& sm, const Ph<T>& p) {
  if (CX && d1 != 0) v = pick(sm.cross_x(d1), cmul(v, p.ar, d1 > 0 ? p.ai : -p.ai), v);
  if (CY && d2 != 0) v = pick(sm.cross_y(d2), cmul(v, p.br, d2 > 0 ? p.bi : -p.bi), v);
  return v;
}

// Iterate around the patch node at box position (2i + PX, 2j + PY) = canonical (p1, p2), in
// the LDS planes (x-edge re, x-edge im, y-edge re, y-edge im, Split::N values each).
template <typename T, int BX, int BY, int PX, int PY, bool CX, bool CY>
struct TileEdges {
  using S = Split<BX, BY>;
  T* pl;
  int i, j;
  Seam<CX, CY> sm;
  Ph<T> p;
  __device__ __forceinline__ int idx(int d1, int d2) const {
    const int sx = (PX + d1) & 1, sy = (PY + d2) & 1;
    return (sx + 2 * sy) * S::SUB + (j + ((PY + d2) >> 1)) * S::HX + i + ((PX + d1) >> 1);
  }
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    const T* q = pl + c * 2 * S::N + idx(d1, d2);
    return phased<CX, CY, T>(Cx<T>{q[0], q[S::N]}, d1, d2, sm, p);
  }
  // as add_ext(): a value written one period back is stored times alpha (beta)
  __device__ __forceinline__ void add(int c, int d1, int d2, Cx<T> v) const {
    if (CX && d1 < 0) v = pick(sm.lx, cmul(v, p.ar, p.ai), v);
    if (CY && d2 < 0) v = pick(sm.ly, cmul(v, p.br, p.bi), v);
    T* q = pl + c * 2 * S::N + idx(d1, d2);
    q[0] = q[0] + v.re;
    q[S::N] = q[S::N] + v.im;
  }
};

// Right-hand side around the patch node, read in memory (as fetch()).
template <typename T, bool CX, bool CY>
struct TileRhs {
  const T* bc;
  int64_t N, nm;
  int n, m, p1, p2;
  Seam<CX, CY> sm;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    int j1 = p1 + d1, j2 = p2 + d2;
    if (CX && d1 != 0) j1 = sm.cross_x(d1) ? (d1 < 0 ? n - 1 : 0) : j1;
    if (CY && d2 != 0) j2 = sm.cross_y(d2) ? (d2 < 0 ? m - 1 : 0) : j2;
    const int64_t k = (c ? nm : 0) + (int64_t)j2 * n + j1;
    return phased<CX, CY, T>(Cx<T>{bc[k], bc[N + k]}, d1, d2, sm, p);
  }
};

// Nodal values around the node at box position (2i + PX, 2j + PY), two LDS planes.
template <typename T, int BX, int BY, int PX, int PY, bool CX, bool CY>
struct TileNodes {
  using S = Split<BX, BY>;
  const T* pl;
  int i, j;
  Seam<CX, CY> sm;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int d1, int d2) const {
    const int sx = (PX + d1) & 1, sy = (PY + d2) & 1;
    const T* q = pl + (sx + 2 * sy) * S::SUB + (j + ((PY + d2) >> 1)) * S::HX + i + ((PX + d1) >> 1);
    return phased<CX, CY, T>(Cx<T>{q[0], q[S::N]}, d1, d2, sm, p);
  }
};

// Patches each colour pass has to update.  Walking the passes backwards from the region that
// must be exact after the sweep (the tile, or the residual window's inputs), a pass needs the
// patches of its colour that write into the region still required, and the values those
// patches read must then be exact before it; every other patch of the box only feeds values
// that never reach the tile.  The bounding rectangle of the needed patches (box positions,
// inclusive) is formed at compile time for every box shape and colour order.
struct PassRect {
  int x0, x1, y0, y1;
};
struct SweepRects {
  PassRect r[4];   // in sweep order
  bool ok;         // no needed patch lies on the box's outermost ring (the halo suffices)
};
constexpr int kMaxBox = 80;
constexpr SweepRects sweep_rects(bool edge, int BX, int BY, int LO, int TX, int TY, int EA, int EB, bool bwd) {
  // need[c][by][bx]: component c (x-edge / y-edge; nodal values use c = 0) must be exact
  bool need[2][kMaxBox][kMaxBox] = {};
  for (int y = LO - EA; y < LO + TY + EB; ++y)
    for (int x = LO - EA; x < LO + TX + EB; ++x) need[0][y][x] = need[1][y][x] = true;
  // an edge patch at P reads x-edges at P + XR and y-edges at P + YR (patch_update) and writes
  // the x-edges of P and P - (1, 0) and the y-edges of P and P - (0, 1); a nodal point reads
  // its 3 x 3 neighbourhood and writes P
  constexpr int XR[6][2] = {{0, 0}, {0, 1}, {0, -1}, {-1, 0}, {-1, 1}, {-1, -1}};
  constexpr int YR[6][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, -1}, {1, -1}, {-1, -1}};
  SweepRects out{};
  out.ok = BX <= kMaxBox && BY <= kMaxBox;
  for (int k = 3; k >= 0; --k) {
    const int colour = bwd ? 3 - k : k;
    const int px = colour & 1, py = colour >> 1;
    PassRect r{kMaxBox, -1, kMaxBox, -1};
    bool hit[kMaxBox][kMaxBox] = {};
    for (int y = 0; y < BY; ++y)
      for (int x = 0; x < BX; ++x) {
        if ((x & 1) != px || (y & 1) != py) continue;
        hit[y][x] = edge ? (need[0][y][x] || (x > 0 && need[0][y][x - 1]) || need[1][y][x] ||
                            (y > 0 && need[1][y - 1][x]))
                         : need[0][y][x];
        if (!hit[y][x]) continue;
        if (x == 0 || y == 0 || x == BX - 1 || y == BY - 1) {   // not updatable: the halo is short
          out.ok = false;
          continue;
        }
        if (x < r.x0) r.x0 = x;
        if (x > r.x1) r.x1 = x;
        if (y < r.y0) r.y0 = y;
        if (y > r.y1) r.y1 = y;
      }
    // the needed patches' reads must be exact before the pass (the other patches of the
    // rectangle are updated too, but nothing needed reads what they write)
    for (int y = 1; y < BY - 1; ++y)
      for (int x = 1; x < BX - 1; ++x) {
        if (!hit[y][x]) continue;
        if (edge) {
          for (int q = 0; q < 6; ++q) {
            need[0][y + XR[q][1]][x + XR[q][0]] = true;
            need[1][y + YR[q][1]][x + YR[q][0]] = true;
          }
        } else {
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) need[0][y + dy][x + dx] = true;
        }
      }
    out.r[k] = r;
  }
  return out;
}

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

struct EdgeArgs {
  const double* k64;
  const float* k32;
  const double* si64;
  const float* si32;
  PatchT T4;
  double s, mx, my;
};

// One colour pass of the edge smoother on the box (patch nodes at box positions 1 .. B-2 of
// the colour's parity; the box origin t0 - kLo is even and n, m are even, so the parity of a
// position is that of its canonical node).
template <typename T, int BX, int BY, int COLOUR, bool CX, bool CY, int X0, int X1, int Y0, int Y1>
__device__ __forceinline__ void edge_pass(T* pl, const T* bc, const EdgeArgs& a, int slot, int ox, int oy, int n,
                                          int m, int64_t N, int64_t nm, T mu, const Ph<T>& p) {
  constexpr int PX = COLOUR & 1, PY = COLOUR >> 1;
  static_assert((X0 & 1) == PX && (Y0 & 1) == PY && X0 >= 1 && Y0 >= 1 && X1 <= BX - 2 && Y1 <= BY - 2, "pass rectangle");
  constexpr int B0X = X0, B0Y = Y0;
  constexpr int CNX = (X1 - X0) / 2 + 1, CNY = (Y1 - Y0) / 2 + 1;
  const double* k64 = a.k64 + (int64_t)slot * nm;
  const float* k32 = a.k32 + (int64_t)slot * nm;
  const T* sib = pick_si<T>(a.si64, a.si32) + kPatchW * (int64_t)slot * nm;
  const T s = (T)a.s;
  const T mmx = mu * (T)a.mx, mmy = mu * (T)a.my;
  for (int t = threadIdx.x; t < CNX * CNY; t += nthreads()) {
    const int i = (B0X >> 1) + t % CNX, j = (B0Y >> 1) + t / CNX;
    const int bx = 2 * i + PX, by = 2 * j + PY;
    const int p1 = CX ? wrapm(ox + bx, n) : ox + bx;
    const int p2 = CY ? wrapm(oy + by, m) : oy + by;
    const T* si = sib + kPatchW * ((int64_t)p2 * n + p1);
    const Seam<CX, CY> sm(p1, p2, n, m);
    const TileEdges<T, BX, BY, PX, PY, CX, CY> X{pl, i, j, sm, p};
    const int p1m = wrapi(p1 - 1, n), p2m = wrapi(p2 - 1, m);
    const T kne = kap<T>(k64, k32, (int64_t)p2 * n + p1);
    const T knw = kap<T>(k64, k32, (int64_t)p2 * n + p1m);
    const T ksw = kap<T>(k64, k32, (int64_t)p2m * n + p1m);
    const T kse = kap<T>(k64, k32, (int64_t)p2m * n + p1);
    const TileRhs<T, CX, CY> B{bc, N, nm, n, m, p1, p2, sm, p};
    patch_update<T>(X, B, kne, knw, ksw, kse, si, s, mmx, mmy);
  }
}

template <typename T, int BX, int BY, bool BWD, bool CX, bool CY, int LO, int TX, int TY, int EA, int EB>
__device__ __forceinline__ void edge_passes(T* pl, const T* bc, const EdgeArgs& a, int slot, int ox, int oy, int n,
                                            int m, int64_t N, int64_t nm, T mu, const Ph<T>& p) {
  constexpr SweepRects R = sweep_rects(true, BX, BY, LO, TX, TY, EA, EB, BWD);
  static_assert(R.ok, "the halo does not cover the sweep's dependency cone");
#define BL_EPASS(k, c)                                                                                             \
  edge_pass<T, BX, BY, c, CX, CY, R.r[k].x0, R.r[k].x1, R.r[k].y0, R.r[k].y1>(pl, bc, a, slot, ox, oy, n, m, N, nm, mu, \
                                                                            p);                                       \
  __syncthreads();
  BL_EPASS(0, BWD ? 3 : 0)
  BL_EPASS(1, BWD ? 2 : 1)
  BL_EPASS(2, BWD ? 1 : 2)
  BL_EPASS(3, BWD ? 0 : 3)
#undef BL_EPASS
}

// Residual b - (A + mu M) x at both edges owned by the box positions of parity (PX, PY)
// inside the residual window (as the residual kernel computes them), into rl (row-major
// window; planes x re, x im, y re, y im).
template <typename T, int BX, int BY, int PX, int PY, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void edge_resid_pass(T* pl, T* rl, const T* bc, const EdgeArgs& a, int slot, int ox,
                                                int oy, int n, int m, int64_t N, int64_t nm, T mu, const Ph<T>& p) {
  constexpr int R0 = LO - 1, RW = TX + 1, RH = TY + 1, RP = RW * RH;
  constexpr int I0 = (R0 - PX + 1) / 2, I1 = (LO + TX - 1 - PX) / 2;
  constexpr int J0 = (R0 - PY + 1) / 2, J1 = (LO + TY - 1 - PY) / 2;
  constexpr int CNX = I1 - I0 + 1, CNY = J1 - J0 + 1;
  const double* k64 = a.k64 + (int64_t)slot * nm;
  const float* k32 = a.k32 + (int64_t)slot * nm;
  const T s = (T)a.s, mx = (T)a.mx, my = (T)a.my;
  for (int t = threadIdx.x; t < CNX * CNY; t += nthreads()) {
    const int i = I0 + t % CNX, j = J0 + t / CNX;
    const int bx = 2 * i + PX, by = 2 * j + PY;
    const int p1 = CX ? wrapm(ox + bx, n) : ox + bx;
    const int p2 = CY ? wrapm(oy + by, m) : oy + by;
    const int64_t k = (int64_t)p2 * n + p1;
    const TileEdges<T, BX, BY, PX, PY, CX, CY> X{pl, i, j, Seam<CX, CY>(p1, p2, n, m), p};
    const T kh = kap<T>(k64, k32, k);
    const int q = (by - R0) * RW + (bx - R0);
    Cx<T> Au, Mu;
    edge_AM_acc<T>(X, 0, kap<T>(k64, k32, (int64_t)wrapi(p2 - 1, m) * n + p1), kh, s, mx, Au, Mu);
    const Cx<T> rx = Cx<T>{bc[k], bc[N + k]} - (Au + (mu * Mu));
    edge_AM_acc<T>(X, 1, kh, kap<T>(k64, k32, (int64_t)p2 * n + wrapi(p1 - 1, n)), s, my, Au, Mu);
    const Cx<T> ry = Cx<T>{bc[nm + k], bc[N + nm + k]} - (Au + (mu * Mu));
    rl[q] = rx.re;
    rl[RP + q] = rx.im;
    rl[2 * RP + q] = ry.re;
    rl[3 * RP + q] = ry.im;
  }
}

// Residual window values of component c around window position (x, y) (as fetch()).
template <typename T, int RW, int RH, bool CX, bool CY>
struct WindowEdges {
  const T* rl;
  int x, y;
  Seam<CX, CY> sm;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int c, int d1, int d2) const {
    const int q = c * 2 * RW * RH + (y + d2) * RW + x + d1;
    return phased<CX, CY, T>(Cx<T>{rl[q], rl[RW * RH + q]}, d1, d2, sm, p);
  }
};

// Residual of the swept tile and its restriction to the edges of the tile's coarse nodes.
template <typename T, int BX, int BY, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void edge_restrict_tile(T* pl, T* rl, const T* bc, T* bco, const EdgeArgs& a,
                                                   int slot, int ox, int oy, int t0x, int t0y, int n, int m,
                                                   int64_t N, int64_t nm, T mu, const Geo& gc, const Ph<T>& p) {
  edge_resid_pass<T, BX, BY, 0, 0, CX, CY, LO, TX, TY>(pl, rl, bc, a, slot, ox, oy, n, m, N, nm, mu, p);
  edge_resid_pass<T, BX, BY, 1, 0, CX, CY, LO, TX, TY>(pl, rl, bc, a, slot, ox, oy, n, m, N, nm, mu, p);
  edge_resid_pass<T, BX, BY, 0, 1, CX, CY, LO, TX, TY>(pl, rl, bc, a, slot, ox, oy, n, m, N, nm, mu, p);
  edge_resid_pass<T, BX, BY, 1, 1, CX, CY, LO, TX, TY>(pl, rl, bc, a, slot, ox, oy, n, m, N, nm, mu, p);
  __syncthreads();
  constexpr int HX = TX / 2, HY = TY / 2;
  for (int t = threadIdx.x; t < HX * HY; t += nthreads()) {
    const int jx = t % HX, jy = t / HX;
    const int f1 = t0x + 2 * jx, f2 = t0y + 2 * jy;
    if (f1 >= n || f2 >= m) continue;
    const WindowEdges<T, TX + 1, TY + 1, CX, CY> R{rl, 2 * jx + 1, 2 * jy + 1, Seam<CX, CY>(f1, f2, n, m), p};
    const int64_t J = (int64_t)(f2 >> 1) * gc.n + (f1 >> 1);
    const Cx<T> vx = edge_restrict_acc<T>(R, 0);
    const Cx<T> vy = edge_restrict_acc<T>(R, 1);
    bco[J] = vx.re;
    bco[gc.ne + J] = vx.im;
    bco[gc.nm + J] = vy.re;
    bco[gc.ne + gc.nm + J] = vy.im;
  }
}

template <typename T, int TX, int TY, bool BWD, int MODE>
__global__ __launch_bounds__(kMaxThreads) void k_edge_sweep(View<const T> xin, View<T> xout, View<const T> bv, EdgeArgs a,
                                                         Geo g, const Phase* __restrict__ phs,
                                                         const double* __restrict__ mus, int zero_start,
                                                         const int* __restrict__ slots, int ncps, int tiles_x,
                                                         SweepFuse<T> fz) {
  static_assert(!((MODE & kRestrict) && BWD), "the residual window halo is sized for forward sweeps");
  static_assert(!(MODE & kBase), "edge sweeps have no base update");
  constexpr bool RES = (MODE & kRestrict) != 0, PRO = (MODE & kProlong) != 0;
  constexpr int LO = RES ? kLoR : kLo;
  constexpr int BX = TX + LO + (RES ? kHiER : kHiE), BY = TY + LO + (RES ? kHiER : kHiE);
  using S = Split<BX, BY>;
  // coarse edges under the box (prolongating sweeps of boxes inside the period, FP32): fine box
  // position b lies over coarse box position b >> 1 and its neighbours one up
  constexpr bool STAGE = PRO && sizeof(T) == 4;
  constexpr int CBX = (BX - 1) / 2 + 2, CBY = (BY - 1) / 2 + 2, CB = CBX * CBY;
  __shared__ T pl[4 * S::N];
  __shared__ T rl[RES ? 4 * (TX + 1) * (TY + 1) : 1];
  __shared__ T cl[STAGE ? 4 * CB : 1];   // x-edge re, im, y-edge re, im
  const TileRef tr = tile_ref(slots, ncps, tiles_x, TX, TY);
  const int n = g.n, m = g.m, tid = threadIdx.x;
  const int64_t N = g.ne, nm = g.nm;
  const int ox = tr.t0x - LO, oy = tr.t0y - LO;   // canonical node of box position 0 (unwrapped)
  const bool cx = !(ox >= 0 && ox + BX <= n), cy = !(oy >= 0 && oy + BY <= m);
  const SJ sj{tr.slot, tr.j};
  T* xo = colp(xout, sj, N);
  const T* bc = colp(bv, sj, N);
  const Ph<T> p = cast_phase<T>(phs[tr.slot]);
  if (zero_start) {
    for (int e = tid; e < 4 * S::N; e += nthreads()) pl[e] = (T)0;
  } else {
    const T* xc = colp(xin, sj, N);
    const T* cc = PRO ? colp(fz.xc, sj, fz.gc.ne) : nullptr;
    if (STAGE && !cx && !cy) {
      // as the prolongation kernel, x + Pr xc, with the coarse edges (as fetch() returns them
      // at the box's coarse positions, ox and oy being even) staged once in LDS, and the
      // iterate's loads issued four positions at a time
      const Geo& gc = fz.gc;
      const int J0 = ox >> 1, K0 = oy >> 1;
      for (int e = tid; e < CB; e += nthreads()) {
        const int a = e % CBX, b = e / CBX;
        const Cx<T> vx = fetch<T, T>(cc, gc.ne, gc.n, gc.m, 0, J0 + a, K0 + b, p);
        const Cx<T> vy = fetch<T, T>(cc, gc.ne, gc.n, gc.m, gc.nm, J0 + a, K0 + b, p);
        cl[e] = vx.re;
        cl[CB + e] = vx.im;
        cl[2 * CB + e] = vy.re;
        cl[3 * CB + e] = vy.im;
      }
      __syncthreads();
      constexpr int LB = 4;
      for (int e0 = tid; e0 < BX * BY; e0 += LB * nthreads()) {
        T u[LB][4];
#pragma unroll
        for (int v = 0; v < LB; ++v) {
          const int e = e0 + v * nthreads();
          if (e >= BX * BY) continue;
          const int64_t i = (int64_t)(oy + e / BX) * n + ox + e % BX;
          u[v][0] = xc[i];
          u[v][1] = xc[N + i];
          u[v][2] = xc[nm + i];
          u[v][3] = xc[N + nm + i];
        }
#pragma unroll
        for (int v = 0; v < LB; ++v) {
          const int e = e0 + v * nthreads();
          if (e >= BX * BY) continue;
          const int bx = e % BX, by = e / BX;
          const int q = (by >> 1) * CBX + (bx >> 1);
          const Cx<T> vx = edge_prolong_combine<T>(Cx<T>{cl[q], cl[CB + q]}, Cx<T>{cl[q + CBX], cl[CB + q + CBX]},
                                                   (by & 1) != 0);
          const Cx<T> vy = edge_prolong_combine<T>(Cx<T>{cl[2 * CB + q], cl[3 * CB + q]},
                                                   Cx<T>{cl[2 * CB + q + 1], cl[3 * CB + q + 1]}, (bx & 1) != 0);
          const int k = S::at(bx, by);
          pl[k] = u[v][0] + vx.re;
          pl[S::N + k] = u[v][1] + vx.im;
          pl[2 * S::N + k] = u[v][2] + vy.re;
          pl[3 * S::N + k] = u[v][3] + vy.im;
        }
      }
    } else {
      for (int e = tid; e < BX * BY; e += nthreads()) {
        const int bx = e % BX, by = e / BX;
        const int c1 = cx ? wrapm(ox + bx, n) : ox + bx, c2 = cy ? wrapm(oy + by, m) : oy + by;
        const int64_t i = (int64_t)c2 * n + c1;
        const int k = S::at(bx, by);
        if constexpr (PRO) {   // as the prolongation kernel: x + Pr xc
          const Cx<T> vx = edge_prolong_xy<T>(cc, fz.gc, 0, c1, c2, p);
          const Cx<T> vy = edge_prolong_xy<T>(cc, fz.gc, 1, c1, c2, p);
          pl[k] = xc[i] + vx.re;
          pl[S::N + k] = xc[N + i] + vx.im;
          pl[2 * S::N + k] = xc[nm + i] + vy.re;
          pl[3 * S::N + k] = xc[N + nm + i] + vy.im;
        } else {
          pl[k] = xc[i];
          pl[S::N + k] = xc[N + i];
          pl[2 * S::N + k] = xc[nm + i];
          pl[3 * S::N + k] = xc[N + nm + i];
        }
      }
    }
  }
  __syncthreads();
  const T mu = (T)mus[tr.slot];
  constexpr int EA = RES ? 2 : 0, EB = RES ? 1 : 0;   // exact margin the residual window needs
  if (!cx && !cy)
    edge_passes<T, BX, BY, BWD, false, false, LO, TX, TY, EA, EB>(pl, bc, a, tr.slot, ox, oy, n, m, N, nm, mu, p);
  else if (!cy)
    edge_passes<T, BX, BY, BWD, true, false, LO, TX, TY, EA, EB>(pl, bc, a, tr.slot, ox, oy, n, m, N, nm, mu, p);
  else if (!cx)
    edge_passes<T, BX, BY, BWD, false, true, LO, TX, TY, EA, EB>(pl, bc, a, tr.slot, ox, oy, n, m, N, nm, mu, p);
  else
    edge_passes<T, BX, BY, BWD, true, true, LO, TX, TY, EA, EB>(pl, bc, a, tr.slot, ox, oy, n, m, N, nm, mu, p);
  for (int e = tid; e < TX * TY; e += nthreads()) {
    const int ix = e % TX, iy = e / TX;
    const int c1 = tr.t0x + ix, c2 = tr.t0y + iy;
    if (c1 >= n || c2 >= m) continue;
    const int k = S::at(ix + LO, iy + LO);
    const int64_t i = (int64_t)c2 * n + c1;
    xo[i] = pl[k];
    xo[N + i] = pl[S::N + k];
    xo[nm + i] = pl[2 * S::N + k];
    xo[N + nm + i] = pl[3 * S::N + k];
  }
  if constexpr (RES) {
    T* bco = colp(fz.bc, sj, fz.gc.ne);
    if (!cx && !cy)
      edge_restrict_tile<T, BX, BY, false, false, LO, TX, TY>(pl, rl, bc, bco, a, tr.slot, ox, oy, tr.t0x, tr.t0y, n,
                                                             m, N, nm, mu, fz.gc, p);
    else if (!cy)
      edge_restrict_tile<T, BX, BY, true, false, LO, TX, TY>(pl, rl, bc, bco, a, tr.slot, ox, oy, tr.t0x, tr.t0y, n,
                                                            m, N, nm, mu, fz.gc, p);
    else if (!cx)
      edge_restrict_tile<T, BX, BY, false, true, LO, TX, TY>(pl, rl, bc, bco, a, tr.slot, ox, oy, tr.t0x, tr.t0y, n,
                                                            m, N, nm, mu, fz.gc, p);
    else
      edge_restrict_tile<T, BX, BY, true, true, LO, TX, TY>(pl, rl, bc, bco, a, tr.slot, ox, oy, tr.t0x, tr.t0y, n,
                                                           m, N, nm, mu, fz.gc, p);
  }
}

// One colour pass of the nodal point Gauss-Seidel on the box.
template <typename T, int BX, int BY, int COLOUR, bool CX, bool CY, int X0, int X1, int Y0, int Y1>
__device__ __forceinline__ void nodal_pass(T* pl, const T* bc, const NodalStencil& st, int ox, int oy, int n, int m,
                                           int64_t N, const Ph<T>& p) {
  using S = Split<BX, BY>;
  constexpr int PX = COLOUR & 1, PY = COLOUR >> 1;
  static_assert((X0 & 1) == PX && (Y0 & 1) == PY && X0 >= 1 && Y0 >= 1 && X1 <= BX - 2 && Y1 <= BY - 2, "pass rectangle");
  constexpr int B0X = X0, B0Y = Y0;
  constexpr int CNX = (X1 - X0) / 2 + 1, CNY = (Y1 - Y0) / 2 + 1;
  const T inv = (T)1 / (T)st.c0;
  for (int t = threadIdx.x; t < CNX * CNY; t += nthreads()) {
    const int i = (B0X >> 1) + t % CNX, j = (B0Y >> 1) + t / CNX;
    const int bx = 2 * i + PX, by = 2 * j + PY;
    const int p1 = CX ? wrapm(ox + bx, n) : ox + bx;
    const int p2 = CY ? wrapm(oy + by, m) : oy + by;
    const int64_t k = (int64_t)p2 * n + p1;
    const TileNodes<T, BX, BY, PX, PY, CX, CY> X{pl, i, j, Seam<CX, CY>(p1, p2, n, m), p};
    const Cx<T> r = Cx<T>{bc[k], bc[N + k]} - nodal_stencil_at<T>(X, st);
    T* q = pl + (PX + 2 * PY) * S::SUB + j * S::HX + i;
    q[0] += inv * r.re;
    q[S::N] += inv * r.im;
  }
}

template <typename T, int BX, int BY, bool BWD, bool CX, bool CY, int LO, int TX, int TY, int EA, int EB>
__device__ __forceinline__ void nodal_passes(T* pl, const T* bc, const NodalStencil& st, int ox, int oy, int n, int m,
                                             int64_t N, const Ph<T>& p) {
  constexpr SweepRects R = sweep_rects(false, BX, BY, LO, TX, TY, EA, EB, BWD);
  static_assert(R.ok, "the halo does not cover the sweep's dependency cone");
#define BL_NPASS(k, c)                                                                                             \
  nodal_pass<T, BX, BY, c, CX, CY, R.r[k].x0, R.r[k].x1, R.r[k].y0, R.r[k].y1>(pl, bc, st, ox, oy, n, m, N, p); \
  __syncthreads();
  BL_NPASS(0, BWD ? 3 : 0)
  BL_NPASS(1, BWD ? 2 : 1)
  BL_NPASS(2, BWD ? 1 : 2)
  BL_NPASS(3, BWD ? 0 : 3)
#undef BL_NPASS
}

// Residual b - P x on the box positions of parity (PX, PY) inside the residual window
// [LO - 1, LO + TX - 1] x [LO - 1, LO + TY - 1] (the fine nodes that the restriction to the
// tile's coarse nodes reads), as the residual kernel computes it, into rl (row-major window,
// re plane then im plane).
template <typename T, int BX, int BY, int PX, int PY, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void nodal_resid_pass(const T* pl, T* rl, const T* bc, const NodalStencil& st, int ox,
                                                 int oy, int n, int m, int64_t N, const Ph<T>& p) {
  constexpr int R0 = LO - 1, RW = TX + 1, RH = TY + 1;
  constexpr int I0 = (R0 - PX + 1) / 2, I1 = (LO + TX - 1 - PX) / 2;
  constexpr int J0 = (R0 - PY + 1) / 2, J1 = (LO + TY - 1 - PY) / 2;
  constexpr int CNX = I1 - I0 + 1, CNY = J1 - J0 + 1;
  for (int t = threadIdx.x; t < CNX * CNY; t += nthreads()) {
    const int i = I0 + t % CNX, j = J0 + t / CNX;
    const int bx = 2 * i + PX, by = 2 * j + PY;
    const int p1 = CX ? wrapm(ox + bx, n) : ox + bx;
    const int p2 = CY ? wrapm(oy + by, m) : oy + by;
    const int64_t k = (int64_t)p2 * n + p1;
    const TileNodes<T, BX, BY, PX, PY, CX, CY> X{pl, i, j, Seam<CX, CY>(p1, p2, n, m), p};
    const Cx<T> r = Cx<T>{bc[k], bc[N + k]} - nodal_stencil_at<T>(X, st);
    const int q = (by - R0) * RW + (bx - R0);
    rl[q] = r.re;
    rl[RW * RH + q] = r.im;
  }
}

// Residual b - P x at the tile's nodes (box positions LO .. LO + TX - 1, LO .. LO + TY - 1),
// straight to memory, as the residual kernel computes it.
template <typename T, int BX, int BY, int PAR, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void nodal_tile_resid_par(const T* pl, const T* bc, T* ro, const NodalStencil& st, int ox,
                                                     int oy, int n, int m, int64_t N, const Ph<T>& p) {
  constexpr int PX = PAR & 1, PY = PAR >> 1;
  constexpr int I0 = (LO - PX + 1) / 2, I1 = (LO + TX - 1 - PX) / 2;
  constexpr int J0 = (LO - PY + 1) / 2, J1 = (LO + TY - 1 - PY) / 2;
  constexpr int CNX = I1 - I0 + 1, CNY = J1 - J0 + 1;
  for (int t = threadIdx.x; t < CNX * CNY; t += nthreads()) {
    const int i = I0 + t % CNX, j = J0 + t / CNX;
    const int bx = 2 * i + PX, by = 2 * j + PY;
    const int p1 = CX ? wrapm(ox + bx, n) : ox + bx;
    const int p2 = CY ? wrapm(oy + by, m) : oy + by;
    if (ox + bx >= n || oy + by >= m) continue;   // past the grid's last tile column / row
    const int64_t k = (int64_t)p2 * n + p1;
    const TileNodes<T, BX, BY, PX, PY, CX, CY> X{pl, i, j, Seam<CX, CY>(p1, p2, n, m), p};
    const Cx<T> r = Cx<T>{bc[k], bc[N + k]} - nodal_stencil_at<T>(X, st);
    ro[k] = r.re;
    ro[N + k] = r.im;
  }
}
template <typename T, int BX, int BY, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void nodal_tile_resid(const T* pl, const T* bc, T* ro, const NodalStencil& st, int ox,
                                                 int oy, int n, int m, int64_t N, const Ph<T>& p) {
  nodal_tile_resid_par<T, BX, BY, 0, CX, CY, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
  nodal_tile_resid_par<T, BX, BY, 1, CX, CY, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
  nodal_tile_resid_par<T, BX, BY, 2, CX, CY, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
  nodal_tile_resid_par<T, BX, BY, 3, CX, CY, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
}

// Residual window values around window position (x, y) (as fetch()).
template <typename T, int RW, int RH, bool CX, bool CY>
struct WindowNodes {
  const T* rl;
  int x, y;
  Seam<CX, CY> sm;
  Ph<T> p;
  __device__ __forceinline__ Cx<T> get(int d1, int d2) const {
    const int q = (y + d2) * RW + x + d1;
    return phased<CX, CY, T>(Cx<T>{rl[q], rl[RW * RH + q]}, d1, d2, sm, p);
  }
};

// Residual of the swept tile and its restriction to the tile's coarse nodes.
template <typename T, int BX, int BY, bool CX, bool CY, int LO, int TX, int TY>
__device__ __forceinline__ void nodal_restrict_tile(const T* pl, T* rl, const T* bc, T* bco, const NodalStencil& st,
                                                    int ox, int oy, int t0x, int t0y, int n, int m, int64_t N,
                                                    const Geo& gc, const Ph<T>& p) {
  nodal_resid_pass<T, BX, BY, 0, 0, CX, CY, LO, TX, TY>(pl, rl, bc, st, ox, oy, n, m, N, p);
  nodal_resid_pass<T, BX, BY, 1, 0, CX, CY, LO, TX, TY>(pl, rl, bc, st, ox, oy, n, m, N, p);
  nodal_resid_pass<T, BX, BY, 0, 1, CX, CY, LO, TX, TY>(pl, rl, bc, st, ox, oy, n, m, N, p);
  nodal_resid_pass<T, BX, BY, 1, 1, CX, CY, LO, TX, TY>(pl, rl, bc, st, ox, oy, n, m, N, p);
  __syncthreads();
  constexpr int HX = TX / 2, HY = TY / 2;
  for (int t = threadIdx.x; t < HX * HY; t += nthreads()) {
    const int jx = t % HX, jy = t / HX;
    const int f1 = t0x + 2 * jx, f2 = t0y + 2 * jy;
    if (f1 >= n || f2 >= m) continue;
    const WindowNodes<T, TX + 1, TY + 1, CX, CY> R{rl, 2 * jx + 1, 2 * jy + 1, Seam<CX, CY>(f1, f2, n, m), p};
    const Cx<T> v = nodal_restrict_acc<T>(R);
    const int64_t J = (int64_t)(f2 >> 1) * gc.n + (f1 >> 1);
    bco[J] = v.re;
    bco[gc.nm + J] = v.im;
  }
}

template <typename T, int TX, int TY, bool BWD, int MODE>
__global__ __launch_bounds__(kMaxThreads) void k_nodal_sweep(View<const T> xin, View<T> xout, View<const T> bv, Geo g,
                                                          const Phase* __restrict__ phs, NodalStencil st,
                                                          int zero_start, const int* __restrict__ slots, int ncps,
                                                          int tiles_x, SweepFuse<T> fz) {
  static_assert(!((MODE & kRestrict) && BWD), "the residual window halo is sized for forward sweeps");
  static_assert(!((MODE & kResid) && !BWD), "the tile residual rides on backward sweeps");
  constexpr bool RES = (MODE & kRestrict) != 0, PRO = (MODE & kProlong) != 0, BAS = (MODE & kBase) != 0;
  constexpr bool TRES = (MODE & kResid) != 0;
  constexpr int LO = RES ? kLoR : kLo;
  constexpr int HI = TRES ? kHiN + 1 : kHiN;   // (the tile residual: exact one node above / right too)
  constexpr int BX = TX + LO + HI, BY = TY + LO + HI;
  using S = Split<BX, BY>;
  // coarse nodes under the box (prolongating sweeps of boxes inside the period): fine box
  // position b lies over coarse box position b >> 1 and its neighbours one up
  constexpr int CBX = (BX - 1) / 2 + 2, CBY = (BY - 1) / 2 + 2, CB = CBX * CBY;
  __shared__ T pl[2 * S::N];
  __shared__ T rl[RES ? 2 * (TX + 1) * (TY + 1) : 1];
  __shared__ T cl[PRO && (sizeof(T) == 4 || TX * TY <= 1024) ? 2 * CB : 1];
  const TileRef tr = tile_ref(slots, ncps, tiles_x, TX, TY);
  const int n = g.n, m = g.m, tid = threadIdx.x;
  const int64_t N = g.nm;
  const int ox = tr.t0x - LO, oy = tr.t0y - LO;
  const bool cx = !(ox >= 0 && ox + BX <= n), cy = !(oy >= 0 && oy + BY <= m);
  const SJ sj{tr.slot, tr.j};
  T* xo = colp(xout, sj, N);
  const T* bc = colp(bv, sj, N);
  const Ph<T> p = cast_phase<T>(phs[tr.slot]);
  if (zero_start) {
    for (int e = tid; e < 2 * S::N; e += nthreads()) pl[e] = (T)0;
  } else {
    const T* xc = colp(xin, sj, N);
    const T* cc = PRO ? colp(fz.xc, sj, fz.gc.nm) : nullptr;
    // (not for FP64 64 x 32 tiles, whose registers would then cost occupancy)
    constexpr bool STAGE = PRO && (sizeof(T) == 4 || TX * TY <= 1024);
    if (STAGE && !cx && !cy) {
      // as the prolongation kernel, x + Pr xc, with the coarse values (as fetch() returns them
      // at the box's coarse positions, ox and oy being even) staged once in LDS, and the
      // iterate's loads issued four positions at a time
      const int J0 = ox >> 1, K0 = oy >> 1;
      for (int e = tid; e < CB; e += nthreads()) {
        const Cx<T> v = fetch<T, T>(cc, fz.gc.nm, fz.gc.n, fz.gc.m, 0, J0 + e % CBX, K0 + e / CBX, p);
        cl[e] = v.re;
        cl[CB + e] = v.im;
      }
      __syncthreads();
      constexpr int LB = 4;
      for (int e0 = tid; e0 < BX * BY; e0 += LB * nthreads()) {
        T ur[LB], ui[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int e = e0 + u * nthreads();
          if (e >= BX * BY) continue;
          const int64_t i = (int64_t)(oy + e / BX) * n + ox + e % BX;
          ur[u] = xc[i];
          ui[u] = xc[N + i];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int e = e0 + u * nthreads();
          if (e >= BX * BY) continue;
          const int bx = e % BX, by = e / BX;
          const int q = (by >> 1) * CBX + (bx >> 1);
          const Cx<T> v = nodal_prolong_combine<T>(Cx<T>{cl[q], cl[CB + q]}, Cx<T>{cl[q + 1], cl[CB + q + 1]},
                                                   Cx<T>{cl[q + CBX], cl[CB + q + CBX]},
                                                   Cx<T>{cl[q + CBX + 1], cl[CB + q + CBX + 1]}, bx & 1, by & 1);
          const int k = S::at(bx, by);
          pl[k] = ur[u] + v.re;
          pl[S::N + k] = ui[u] + v.im;
        }
      }
    } else {
      for (int e = tid; e < BX * BY; e += nthreads()) {
        const int bx = e % BX, by = e / BX;
        const int c1 = cx ? wrapm(ox + bx, n) : ox + bx, c2 = cy ? wrapm(oy + by, m) : oy + by;
        const int64_t i = (int64_t)c2 * n + c1;
        const int k = S::at(bx, by);
        if constexpr (PRO) {   // as the prolongation kernel: base + Pr xc
          const Cx<T> v = nodal_prolong_xy<T>(cc, fz.gc, c1, c2, p);
          pl[k] = xc[i] + v.re;
          pl[S::N + k] = xc[N + i] + v.im;
        } else {
          pl[k] = xc[i];
          pl[S::N + k] = xc[N + i];
        }
      }
    }
  }
  __syncthreads();
  // exact margin the residual window (restriction) or the tile residual needs
  constexpr int EA = RES ? 2 : (TRES ? 1 : 0), EB = (RES || TRES) ? 1 : 0;
  if (!cx && !cy) nodal_passes<T, BX, BY, BWD, false, false, LO, TX, TY, EA, EB>(pl, bc, st, ox, oy, n, m, N, p);
  else if (!cy) nodal_passes<T, BX, BY, BWD, true, false, LO, TX, TY, EA, EB>(pl, bc, st, ox, oy, n, m, N, p);
  else if (!cx) nodal_passes<T, BX, BY, BWD, false, true, LO, TX, TY, EA, EB>(pl, bc, st, ox, oy, n, m, N, p);
  else nodal_passes<T, BX, BY, BWD, true, true, LO, TX, TY, EA, EB>(pl, bc, st, ox, oy, n, m, N, p);
  const T* bs = BAS ? colp(fz.base, sj, N) : nullptr;
  if constexpr (BAS) {   // as the update kernel: base + x (the base loads four positions at a time)
    constexpr int LB = 4;
    for (int e0 = tid; e0 < TX * TY; e0 += LB * nthreads()) {
      T br[LB], bi[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int e = e0 + u * nthreads();
        const int c1 = tr.t0x + e % TX, c2 = tr.t0y + e / TX;
        if (e >= TX * TY || c1 >= n || c2 >= m) continue;
        const int64_t i = (int64_t)c2 * n + c1;
        br[u] = bs[i];
        bi[u] = bs[N + i];
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int e = e0 + u * nthreads();
        const int ix = e % TX, iy = e / TX;
        const int c1 = tr.t0x + ix, c2 = tr.t0y + iy;
        if (e >= TX * TY || c1 >= n || c2 >= m) continue;
        const int k = S::at(ix + LO, iy + LO);
        const int64_t i = (int64_t)c2 * n + c1;
        xo[i] = br[u] + pl[k];
        xo[N + i] = bi[u] + pl[S::N + k];
      }
    }
  } else {
    for (int e = tid; e < TX * TY; e += nthreads()) {
      const int ix = e % TX, iy = e / TX;
      const int c1 = tr.t0x + ix, c2 = tr.t0y + iy;
      if (c1 >= n || c2 >= m) continue;
      const int k = S::at(ix + LO, iy + LO);
      const int64_t i = (int64_t)c2 * n + c1;
      xo[i] = pl[k];
      xo[N + i] = pl[S::N + k];
    }
  }
  if constexpr (TRES) {
    T* ro = colp(fz.res, sj, N);
    if (!cx && !cy) nodal_tile_resid<T, BX, BY, false, false, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
    else if (!cy) nodal_tile_resid<T, BX, BY, true, false, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
    else if (!cx) nodal_tile_resid<T, BX, BY, false, true, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
    else nodal_tile_resid<T, BX, BY, true, true, LO, TX, TY>(pl, bc, ro, st, ox, oy, n, m, N, p);
  }
  if constexpr (RES) {
    T* bco = colp(fz.bc, sj, fz.gc.nm);
    if (!cx && !cy)
      nodal_restrict_tile<T, BX, BY, false, false, LO, TX, TY>(pl, rl, bc, bco, st, ox, oy, tr.t0x, tr.t0y, n, m, N,
                                                              fz.gc, p);
    else if (!cy)
      nodal_restrict_tile<T, BX, BY, true, false, LO, TX, TY>(pl, rl, bc, bco, st, ox, oy, tr.t0x, tr.t0y, n, m, N,
                                                             fz.gc, p);
    else if (!cx)
      nodal_restrict_tile<T, BX, BY, false, true, LO, TX, TY>(pl, rl, bc, bco, st, ox, oy, tr.t0x, tr.t0y, n, m, N,
                                                             fz.gc, p);
    else
      nodal_restrict_tile<T, BX, BY, true, true, LO, TX, TY>(pl, rl, bc, bco, st, ox, oy, tr.t0x, tr.t0y, n, m, N,
                                                            fz.gc, p);
  }
}

// Tile shapes (nodes): 0: 32 x 32, 1: 64 x 32.  FP64 edge sweeps, and FP64 nodal sweeps with
// the residual window, use 32 x 32 only (the larger boxes exceed the static LDS limit).
// 512 threads when the launch has fewer than four tile workgroups per compute unit
inline unsigned sweep_threads(const dim3& grid) { return (uint64_t)grid.x * grid.y < 1024 ? 512u : 256u; }

template <typename T, int TX, int TY, bool BWD, int MODE>
void edge_go(View<const T> xin, View<T> xout, View<const T> b, const EdgeArgs& a, const Geo& g, const Phase* ph,
             const double* mu, bool zero_start, const SweepFuse<T>& fz, const Launch& L) {
  const int tx = (g.n + TX - 1) / TX, ty = (g.m + TY - 1) / TY;
  dim3 grid((unsigned)(tx * ty), (unsigned)(L.nact * L.ncps));
  // the restricting sweep's LDS (box and residual window) admits three workgroups per compute
  // unit: 512 threads each keep the occupancy up
  k_edge_sweep<T, TX, TY, BWD, MODE><<<grid, (MODE & kRestrict) ? 512u : sweep_threads(grid), 0, L.st>>>(xin, xout, b, a, g, ph, mu, zero_start ? 1 : 0,
                                                                  L.slots, L.ncps, tx, fz);
}

template <typename T, int TX, int TY>
void edge_launch(View<const T> xin, View<T> xout, View<const T> b, const EdgeArgs& a, const Geo& g, const Phase* ph,
                 const double* mu, bool backward, bool zero_start, const SweepFuse<T>& fz, const Launch& L) {
  if (backward) {
    if (fz.xc.p) edge_go<T, TX, TY, true, kProlong>(xin, xout, b, a, g, ph, mu, zero_start, fz, L);
    else edge_go<T, TX, TY, true, 0>(xin, xout, b, a, g, ph, mu, zero_start, fz, L);
    return;
  }
  if constexpr (sizeof(T) == 4 && TX * TY <= 1024) {   // the residual window fits LDS: FP32, 32 x 32
    if (fz.bc.p) {
      edge_go<T, TX, TY, false, kRestrict>(xin, xout, b, a, g, ph, mu, zero_start, fz, L);
      return;
    }
  }
  edge_go<T, TX, TY, false, 0>(xin, xout, b, a, g, ph, mu, zero_start, fz, L);
}

template <typename T, int TX, int TY, bool BWD, int MODE>
void nodal_go(View<const T> xin, View<T> xout, View<const T> b, const Geo& g, const Phase* ph, const NodalStencil& c,
              bool zero_start, const SweepFuse<T>& fz, const Launch& L) {
  const int tx = (g.n + TX - 1) / TX, ty = (g.m + TY - 1) / TY;
  dim3 grid((unsigned)(tx * ty), (unsigned)(L.nact * L.ncps));
  k_nodal_sweep<T, TX, TY, BWD, MODE><<<grid, sweep_threads(grid), 0, L.st>>>(xin, xout, b, g, ph, c, zero_start ? 1 : 0,
                                                                   L.slots, L.ncps, tx, fz);
}

template <typename T, int TX, int TY>
void nodal_launch(View<const T> xin, View<T> xout, View<const T> b, const Geo& g, const Phase* ph,
                  const NodalStencil& c, bool backward, bool zero_start, const SweepFuse<T>& fz, const Launch& L) {
  const int mode = (fz.bc.p ? kRestrict : 0) | (fz.xc.p ? kProlong : 0) | (fz.base.p ? kBase : 0) |
                   (fz.res.p ? kResid : 0);
  if (!backward) {
    if constexpr (sizeof(T) == 4 || TX * TY <= 1024) {   // (the FP64 64 x 32 window is routed to 32 x 32)
      if (mode == kRestrict) {
        nodal_go<T, TX, TY, false, kRestrict>(xin, xout, b, g, ph, c, zero_start, fz, L);
        return;
      }
    }
    nodal_go<T, TX, TY, false, 0>(xin, xout, b, g, ph, c, zero_start, fz, L);
    return;
  }
  switch (mode) {
    case kProlong: nodal_go<T, TX, TY, true, kProlong>(xin, xout, b, g, ph, c, zero_start, fz, L); break;
    case kBase: nodal_go<T, TX, TY, true, kBase>(xin, xout, b, g, ph, c, zero_start, fz, L); break;
    case kProlong | kBase:
      nodal_go<T, TX, TY, true, kProlong | kBase>(xin, xout, b, g, ph, c, zero_start, fz, L);
      break;
    case kProlong | kResid:
      nodal_go<T, TX, TY, true, kProlong | kResid>(xin, xout, b, g, ph, c, zero_start, fz, L);
      break;
    case kResid: nodal_go<T, TX, TY, true, kResid>(xin, xout, b, g, ph, c, zero_start, fz, L); break;
    default: nodal_go<T, TX, TY, true, 0>(xin, xout, b, g, ph, c, zero_start, fz, L); break;
  }
}

}  // namespace

bool edge_sweep_restricts(size_t elem) { return elem == 4; }

template <typename T>
void edge_sweep(View<const T> xin, View<T> xout, View<const T> b, const double* kappa64, const float* kappa32,
                const double* sinv64, const float* sinv32, const Geo& g, const Phase* ph, const double* mu,
                const PatchT& T4, bool backward, bool zero_start, int tile, const Launch& L, const SweepFuse<T>& fz) {
  if (L.nact * L.ncps == 0) return;
  const EdgeArgs a{kappa64, kappa32, sinv64, sinv32, T4, g.s, g.mx, g.my};
  if constexpr (sizeof(T) == 4) {
    if (tile == 1 && !fz.bc.p) {
      edge_launch<T, 64, 32>(xin, xout, b, a, g, ph, mu, backward, zero_start, fz, L);
      return;
    }
  }
  edge_launch<T, 32, 32>(xin, xout, b, a, g, ph, mu, backward, zero_start, fz, L);
}

template <typename T>
void nodal_sweep(View<const T> xin, View<T> xout, View<const T> b, const Geo& g, const Phase* ph,
                 const NodalStencil& c, bool backward, bool zero_start, int tile, const Launch& L,
                 const SweepFuse<T>& fz) {
  if (L.nact * L.ncps == 0) return;
  if (tile == 1 && (sizeof(T) == 4 || !fz.bc.p))
    nodal_launch<T, 64, 32>(xin, xout, b, g, ph, c, backward, zero_start, fz, L);
  else
    nodal_launch<T, 32, 32>(xin, xout, b, g, ph, c, backward, zero_start, fz, L);
}

template void edge_sweep<double>(View<const double>, View<double>, View<const double>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, bool, bool, int, const Launch&, const SweepFuse<double>&);
template void edge_sweep<float>(View<const float>, View<float>, View<const float>, const double*, const float*, const double*, const float*, const Geo&, const Phase*, const double*, const PatchT&, bool, bool, int, const Launch&, const SweepFuse<float>&);
template void nodal_sweep<double>(View<const double>, View<double>, View<const double>, const Geo&, const Phase*, const NodalStencil&, bool, bool, int, const Launch&, const SweepFuse<double>&);
template void nodal_sweep<float>(View<const float>, View<float>, View<const float>, const Geo&, const Phase*, const NodalStencil&, bool, bool, int, const Launch&, const SweepFuse<float>&);

}  // namespace bl
