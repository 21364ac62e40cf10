// Shared device helpers: complex arithmetic, index maps and merge-tree geometry.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 cd;  // complex double, interleaved (re, im)
typedef float2 cf;   // complex float

__host__ __device__ inline cd cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline cd cadd(cd a, cd b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cd csub(cd a, cd b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cd cmul(cd a, cd b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a*b + c
__host__ __device__ inline cd cfma(cd a, cd b, cd c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__host__ __device__ inline cd cconj(cd a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cd cscale(cd a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline cd cinv(cd a) {
  // 1/a with a scaling step so that |a| near the range limits stays finite
  double s = fmax(fabs(a.x), fabs(a.y));
  double ar = a.x / s, ai = a.y / s;
  double d = ar * ar + ai * ai;
  return make_double2(ar / (d * s), -ai / (d * s));
}

// complex float counterparts
__host__ __device__ inline cf cmkf(float r, float i) { return make_float2(r, i); }
__host__ __device__ inline cf cadd(cf a, cf b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cf csub(cf a, cf b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cf cmul(cf a, cf b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cf cfma(cf a, cf b, cf c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__host__ __device__ inline float cabs2(cf a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cf cinv(cf a) {
  const float s = fmaxf(fabsf(a.x), fabsf(a.y));
  const float ar = a.x / s, ai = a.y / s;
  const float d = ar * ar + ai * ai;
  return make_float2(ar / (d * s), -ai / (d * s));
}
// widening / narrowing
__host__ __device__ inline cd to_cd(cd a) { return a; }
__host__ __device__ inline cd to_cd(cf a) { return make_double2((double)a.x, (double)a.y); }
__host__ __device__ inline cf to_cf(cd a) { return make_float2((float)a.x, (float)a.y); }

// Traits of the two complex storage types.
template <class T> struct cx;
template <> struct cx<cd> {
  typedef double real;
  __host__ __device__ static cd make(double r, double i) { return make_double2(r, i); }
  __host__ __device__ static cd from(cd a) { return a; }
};
template <> struct cx<cf> {
  typedef float real;
  __host__ __device__ static cf make(double r, double i) { return make_float2((float)r, (float)i); }
  __host__ __device__ static cf from(cd a) { return to_cf(a); }
};

// Index map: i -> map ? map[i] : off + i + (i >= gap_start ? gap_len : 0).
// Describes a row or column selection of a matrix operand.
struct IdxMap {
  const int* map;
  int off;
  int gap_start;
  int gap_len;
};
__host__ __device__ inline int imap(const IdxMap& m, int i) {
  return m.map ? m.map[i] : m.off + i + (i >= m.gap_start ? m.gap_len : 0);
}
// The same map when it is known not to be a table: no load, so that a loop
// evaluating it does not wait on the loads it has in flight.
__host__ __device__ inline int imap_arith(const IdxMap& m, int i) {
  return m.off + i + (i >= m.gap_start ? m.gap_len : 0);
}
__host__ __device__ inline IdxMap im_off(int off) { return IdxMap{nullptr, off, 1 << 30, 0}; }
__host__ __device__ inline IdxMap im_gap(int off, int gap_start, int gap_len) {
  return IdxMap{nullptr, off, gap_start, gap_len};
}
__host__ __device__ inline IdxMap im_tab(const int* tab) { return IdxMap{tab, 0, 1 << 30, 0}; }

// ---------------------------------------------------------------------------
// Merge-tree geometry of an nx x ny mesh (both powers of two, 2^ax x 2^ay).
// Merge l (1-based) joins pairs of level-l boxes along x when l is odd and
// along y when l is even while both directions have merges left (the first
// 2 min(ax, ay) merges; all of them on a square mesh), and along the longer
// direction after that.  A level-l box is 2^dx x 2^dy elements, dx and dy
// the merges along x and y among merges 1..l-1.  Boxes of every level are
// stored in merge-tree order: an element's tree code has bit l-1 equal to the
// bit of its x or y index that merge l consumes (the next unused one of that
// direction), and box j of level l covers the elements whose code shifted
// right by l-1 equals j, so the pair merged at level l is (2j, 2j+1) and
// produces box j of level l+1.  On a square mesh the code is the Morton code
// (x bits at even positions, y bits at odd positions).
struct Geom {
  int nx, ny, ax, ay, p, level;
  int wx, wy, nbx, nby, nboxes, b;
  int off[5];  // side offsets in the box-local [l; r; b; t] order
};

// 0: merge l runs along x, 1: along y.
__host__ __device__ inline int merge_axis_of(int ax, int ay, int l) {
  const int c = ax < ay ? ax : ay;
  if (l <= 2 * c) return (l & 1) ? 0 : 1;
  return ax > ay ? 0 : 1;
}

// Merges along x (dx) and y (dy) among merges 1..l-1.
__host__ __device__ inline void merges_before(int ax, int ay, int l, int& dx, int& dy) {
  const int c = ax < ay ? ax : ay, k = l - 1;
  if (k <= 2 * c) {
    dx = (k + 1) / 2;
    dy = k / 2;
  } else if (ax > ay) {
    dx = k - c;
    dy = c;
  } else {
    dx = c;
    dy = k - c;
  }
}

inline int log2_exact(int v) {
  int q = 0;
  while ((1 << q) < v) ++q;
  return q;
}

inline Geom make_geom(int nx, int ny, int p, int level) {
  Geom g;
  g.nx = nx;
  g.ny = ny;
  g.ax = log2_exact(nx);
  g.ay = log2_exact(ny);
  g.p = p;
  g.level = level;
  int dx, dy;
  merges_before(g.ax, g.ay, level, dx, dy);
  g.wx = 1 << dx;
  g.wy = 1 << dy;
  g.nbx = nx / g.wx;
  g.nby = ny / g.wy;
  g.nboxes = g.nbx * g.nby;
  g.off[0] = 0;
  g.off[1] = g.wy * p;
  g.off[2] = 2 * g.wy * p;
  g.off[3] = 2 * g.wy * p + g.wx * p;
  g.off[4] = 2 * (g.wx + g.wy) * p;
  g.b = g.off[4];
  return g;
}

// Tree code of element (x, y) (its level-1 box index) and its inverse.
__host__ __device__ inline uint32_t tree_code(int ax, int ay, uint32_t x, uint32_t y) {
  const int c = ax < ay ? ax : ay;
  uint32_t code = 0;
  for (int k = 0; k < c; ++k) {
    code |= ((x >> k) & 1u) << (2 * k);
    code |= ((y >> k) & 1u) << (2 * k + 1);
  }
  code |= (ax > ay ? (x >> c) : (y >> c)) << (2 * c);
  return code;
}

__host__ __device__ inline void tree_decode(int ax, int ay, uint32_t code, uint32_t& x, uint32_t& y) {
  const int c = ax < ay ? ax : ay;
  x = 0;
  y = 0;
  for (int k = 0; k < c; ++k) {
    x |= ((code >> (2 * k)) & 1u) << k;
    y |= ((code >> (2 * k + 1)) & 1u) << k;
  }
  if (ax > ay) x |= (code >> (2 * c)) << c;
  else y |= (code >> (2 * c)) << c;
}

__host__ __device__ inline void box_xy(const Geom& g, int j, int& bx, int& by) {
  uint32_t ex, ey;
  tree_decode(g.ax, g.ay, (uint32_t)j << (g.level - 1), ex, ey);
  bx = (int)(ex / (uint32_t)g.wx);
  by = (int)(ey / (uint32_t)g.wy);
}

__host__ __device__ inline int box_index(const Geom& g, int bx, int by) {
  return (int)(tree_code(g.ax, g.ay, (uint32_t)bx * g.wx, (uint32_t)by * g.wy) >> (g.level - 1));
}

__host__ __device__ inline int side_of(const Geom& g, int k) {
  return (k >= g.off[1]) + (k >= g.off[2]) + (k >= g.off[3]);
}

__host__ __device__ inline bool side_physical(const Geom& g, int bx, int by, int s) {
  return (s == 0 && bx == 0) || (s == 1 && bx == g.nbx - 1) || (s == 2 && by == 0) ||
         (s == 3 && by == g.nby - 1);
}

// Canonical slot of box-local boundary index k of box (bx, by).
__host__ __device__ inline int box_slot(const Geom& g, int bx, int by, int k) {
  const int s = side_of(g, k);
  const int kk = k - g.off[s];
  const int q = kk / g.p, r = kk - q * g.p;
  int ex, ey;
  if (s == 0) { ex = bx * g.wx; ey = by * g.wy + q; }
  else if (s == 1) { ex = bx * g.wx + g.wx - 1; ey = by * g.wy + q; }
  else if (s == 2) { ex = bx * g.wx + q; ey = by * g.wy; }
  else { ex = bx * g.wx + q; ey = by * g.wy + g.wy - 1; }
  return ((ex + g.nx * ey) * 4 + s) * g.p + r;
}

// Slot across the face from canonical slot `s` of an nx x ny mesh, or -1 on
// the physical boundary.
__host__ __device__ inline int slot_partner(int nx, int ny, int p, int s) {
  const int k = s % p;
  const int side = (s / p) & 3;
  const int e = s / (4 * p);
  const int ix = e % nx, iy = e / nx;
  if (side == 0) return ix == 0 ? -1 : (((e - 1) * 4 + 1) * p + k);
  if (side == 1) return ix == nx - 1 ? -1 : (((e + 1) * 4 + 0) * p + k);
  if (side == 2) return iy == 0 ? -1 : (((e - nx) * 4 + 3) * p + k);
  return iy == ny - 1 ? -1 : (((e + nx) * 4 + 2) * p + k);
}

// Allow up to `bytes` of dynamic LDS for `kernel` (gfx950 has 160 KB per CU).
template <class K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Values that are the same in every lane of a wave (the wave index, data read
// from one LDS address) held in scalar registers, so that conditions on them
// compile to scalar branches instead of divergent ones.
__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Logical index of workgroup b of a 1-D grid of G workgroups such that each
// XCD's workgroups take one contiguous range: the dispatcher deals hardware
// indices round-robin over the 8 XCDs (b % 8), so neighbouring logical
// workgroups, which share the cache lines at their boundaries, then run
// behind one L2.  A bijection on [0, G) for any G.
#ifndef HPS_XCDS
#define HPS_XCDS 8
#endif
__device__ inline int xcd_swizzle(int b, int G) {
  const int q = G / HPS_XCDS, r = G % HPS_XCDS;  // XCD x runs q + (x < r) of them
  const int x = b % HPS_XCDS, k = b / HPS_XCDS;
  return x * q + min(x, r) + k;
}
__device__ inline unsigned long long wave_uniform(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ inline double wave_uniform(double v) {
  return __longlong_as_double((long long)wave_uniform((unsigned long long)__double_as_longlong(v)));
}

// Device error words of a problem (kFlagWords ints in its workspace):
//   word 0: bits kFlagSingular (exact zero pivot), kFlagNonFinite (NaN or Inf
//           in b_nodes or s_nodes);
//   words 2-3: the first zero pivot as (level << 40) | batch index, kept as the
//           minimum (level 0: the leaf build, index = element of the group;
//           level l >= 1: merge l, index = pair of the group's level batch);
//   words 4-5: the first element (index in the group) with a non-finite input;
//   word 6: the lowest merge level whose inverse without row interchanges
//           failed its threshold test (0x7FFFFFFF: none).
constexpr int kFlagWords = 8;
constexpr int kFlagSingular = 2;
constexpr int kFlagNonFinite = 4;
__host__ __device__ inline unsigned long long flag_where(int level, long long index) {
  return ((unsigned long long)level << 40) | (unsigned long long)index;
}
__device__ inline void flag_singular(int* flag, unsigned long long where) {
  atomicOr(flag, kFlagSingular);
  atomicMin(reinterpret_cast<unsigned long long*>(flag + 2), where);
}
__device__ inline void flag_nonfinite(int* flag, unsigned long long element) {
  atomicOr(flag, kFlagNonFinite);
  atomicMin(reinterpret_cast<unsigned long long*>(flag + 4), element);
}
