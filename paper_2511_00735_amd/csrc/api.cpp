// Host side of the HPS library: workspace layout, the level scheduler (leaf
// build, merges), the multigrid V-cycle, the coarse GMRES and the outer
// flexible GMRES, exported through the C ABI of include/hps.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hps.h"
#include "host.h"
#include "solve.h"
#include "gemv.h"

// Elements per leaf launch (each holds its bordered matrix, ~0.65 MB at
// N = 16, in the scratch buffer while it is factored).  One launch of many
// rounds of workgroups ends with one tail instead of one per launch.
#ifndef HPS_LEAF_CHUNK
#define HPS_LEAF_CHUNK 4096
#endif

// One timed launch: events recorded on the context's stream around it.
struct TimedLaunch {
  hipEvent_t start, stop;
  int kernel;
  long long units;
};

struct hps_ctx {
  hipStream_t stream;
  std::string err;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  int use_graphs = 0;
  int timing = 0;
  std::vector<TimedLaunch> timed;
  // pinned host copies (two, alternating) of a solve's Hessenberg columns,
  // read back once per FGMRES iteration (a pageable destination is staged by
  // the runtime), and the events that mark each copy done.  Held by the
  // context and grown as needed, so that short-lived problems do not allocate
  // and free pinned memory (a free can wait for the whole device).
  void* hbuf = nullptr;
  size_t hbuf_bytes = 0;
  hipEvent_t hev[2] = {nullptr, nullptr};
  // live problem handles of this context, whose device error words
  // hps_sync reads
  std::vector<hps_problem*> problems;
};

namespace hps {

namespace {

inline size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kWorkVectors = 9;  // canonical group vectors in a workspace (see workv)
constexpr int kMaxGroup = 4096;  // problems in one group
constexpr int kMaxGamma = 4;     // coarse calls per level of a gamma-cycle

struct Level {
  Geom g;
  size_t T_off = 0;     // box maps: complex FP64, or FP32 when f32 (level 1: always FP64)
  bool f32 = false;     // mixed precision: this level's merge and V-cycle run in FP32
  size_t T32_off = 0;   // level 1 in mixed mode: FP32 copy of the leaf maps
  // merge of this level's box pairs (level < L, or the top pair in exact mode)
  int pairs = 0, m = 0, e = 0, axis = 0, a0 = 0, b0 = 0;
  IdxMap E1{}, E2{};
  bool has_merge = false;
  // Per pair, with x = [Q.beta; P.alpha] (2m) and y = [P.E1; Q.E2] (2e):
  size_t Ainv_off = 0;  // [pairs][2m][2m] A^-1, A = [[I, -T^P_aa], [-T^Q_bb, I]]
  size_t X_off = 0;     // [pairs][2m][2e] A^-1 B (the shared-face data as a function of y)
  size_t map_off = 0;   // int32 [2e]: merged-box position of y
  size_t xtab_off = 0;  // int32 [pairs][2m]: canonical slots of x
  size_t ytab_off = 0;  // int32 [pairs][2e]: canonical slots of y (-1: physical)
  size_t dtab_off = 0;  // int32 [pairs][2e]: slots across the face of y (-1: physical)
  size_t Z0_off = 0;    // complex FP64 [pairs][2m]: A^-1 r_x of the down sweep
  // levels 1..K of a fused V-cycle launch: the slot tables as positions in the
  // level-(K+1) box's LDS vector (int32 [pairs][2m], [pairs][2e], [pairs][2e])
  size_t xl_off = 0, dl_off = 0, yl_off = 0;
};

// Workspace of a group of nq problems of one shape.  Every per-problem array
// is repeated nq times, problem after problem, so that the boxes (and pairs) of
// one level form one contiguous batch of nq * boxes entries and the canonical
// vectors of the group one vector of nq * nslots entries.
struct Layout {
  int nq;
  int nx, ny, N, p, E, L, Lmax, k, restart;  // mesh nx x ny elements
  int gamma;             // coarse calls per level (1: V-cycle)
  size_t gam_off = 0;    // gamma > 1: per level l < L the vectors W, Y, R, D (see mg_gamma)
  bool exact, mixed;
  size_t stage_off = 0;  // FP32 output of the last FP32 merge, widened into FP64 maps
  long long nslots;
  int nL;  // number of coarse unknowns
  int leaf_chunk;
  size_t tables_off, H_off;
  std::vector<Level> lev;  // 1..L
  size_t scratch_off, scratch_bytes;
  size_t V_off, Z_off, work_off;  // Krylov bases and 5 canonical work vectors
  size_t cV_off, cw_off, cx_off, cidx_off, cH_off, cy_off, cs_off;  // coarse GMRES
  size_t part_off, hh_off, one_off, flag_off;
  size_t jctr_off;                 // int: the FGMRES iteration index of the captured iteration
  // V-cycle levels 1..fuse in one launch per direction (0: none): per
  // level-(fuse+1) box, fnloc local slots and their canonical slots (down and up sets)
  int fuse = 0, fnloc = 0;
  size_t fgd_off = 0, fgu_off = 0;
  size_t fb_off;                   // int [1 + leaf_chunk]: the leaf fallback's element list
  size_t ysol_off;                 // [nq][restart] FGMRES update coefficients
  size_t gpart_off, gpart_elems;  // split-K GEMV partial sums
  size_t total;
};

// Elements along y (0 in the descriptor: a square mesh) and the element side:
// square elements of side 1 / max(nx, ny) on (0, nx h) x (0, ny h).
inline int desc_ny(const hps_desc* d) { return d->ny ? d->ny : d->n; }
inline double element_size(int nx, int ny) { return 1.0 / std::max(nx, ny); }

int ilog2(int v) {
  int q = 0;
  while ((1 << q) < v) ++q;
  return q;
}

Level make_level(int nx, int ny, int p, int l) {
  Level lv;
  lv.g = make_geom(nx, ny, p, l);
  return lv;
}

// Merge geometry of level l: shared side alpha of P, beta of Q, exterior maps.
void set_merge_geom(Level& lv) {
  const Geom& g = lv.g;
  lv.has_merge = true;
  lv.pairs = g.nboxes / 2;
  lv.axis = merge_axis_of(g.ax, g.ay, g.level);
  if (lv.axis == 0) {  // x-merge: alpha = r of P, beta = l of Q
    lv.m = g.off[2] - g.off[1];
    lv.a0 = g.off[1];
    lv.b0 = g.off[0];
    lv.E1 = im_gap(0, g.off[1], lv.m);
    lv.E2 = im_off(g.off[1]);
  } else {             // y-merge: alpha = t of P, beta = b of Q
    lv.m = g.off[4] - g.off[3];
    lv.a0 = g.off[3];
    lv.b0 = g.off[2];
    lv.E1 = im_off(0);
    lv.E2 = im_gap(0, g.off[2], lv.m);
  }
  lv.e = g.b - lv.m;
}

// Merged-box position of every y index (y = [P.E1; Q.E2], each in the child's
// [l; r; b; t] order without the shared side).
std::vector<int> merge_map(const Level& lv) {
  const Geom& g = lv.g;
  const int p = g.p, wx = g.wx, wy = g.wy;
  std::vector<int> out;
  out.reserve(2 * lv.e);
  auto seg = [&](int start, int len) { for (int k = 0; k < len; ++k) out.push_back(start + k); };
  if (lv.axis == 0) {
    // merged box 2wx x wy: l [0, wy p), r [wy p, 2wy p), b [2wy p, 2wy p + 2wx p), t after
    const int ml = 0, mr = wy * p, mb = 2 * wy * p, mt = 2 * wy * p + 2 * wx * p;
    seg(ml, wy * p);            // P.l
    seg(mb, wx * p);            // P.b
    seg(mt, wx * p);            // P.t
    seg(mr, wy * p);            // Q.r
    seg(mb + wx * p, wx * p);   // Q.b
    seg(mt + wx * p, wx * p);   // Q.t
  } else {
    // merged box wx x 2wy: l [0, 2wy p), r [2wy p, 4wy p), b [4wy p, 4wy p + wx p), t after
    const int ml = 0, mr = 2 * wy * p, mb = 4 * wy * p, mt = 4 * wy * p + wx * p;
    seg(ml, wy * p);            // P.l
    seg(mr, wy * p);            // P.r
    seg(mb, wx * p);            // P.b
    seg(ml + wy * p, wy * p);   // Q.l
    seg(mr + wy * p, wy * p);   // Q.r
    seg(mt, wx * p);            // Q.t
  }
  return out;
}

// Canonical slots of the level-L unknowns, box by box in storage order.
std::vector<int> coarse_slots(const Level& lv) {
  const Geom& g = lv.g;
  std::vector<int> out;
  for (int j = 0; j < g.nboxes; ++j) {
    int bx, by;
    box_xy(g, j, bx, by);
    for (int k = 0; k < g.b; ++k)
      if (!side_physical(g, bx, by, side_of(g, k))) out.push_back(box_slot(g, bx, by, k));
  }
  return out;
}

// Slot tables of a level's pairs (pair j: P = box 2j, Q = box 2j+1):
// x = [Q.beta; P.alpha] (never physical), y = [P.E1; Q.E2] and the slots
// across the face of y; physical entries of y are -1.
void pair_tables(const Level& lv, std::vector<int>& xt, std::vector<int>& yt, std::vector<int>& dt) {
  const Geom& g = lv.g;
  xt.clear();
  yt.clear();
  dt.clear();
  for (int j = 0; j < lv.pairs; ++j) {
    int px, py, qx, qy;
    box_xy(g, 2 * j, px, py);
    box_xy(g, 2 * j + 1, qx, qy);
    for (int i = 0; i < lv.m; ++i) xt.push_back(box_slot(g, qx, qy, lv.b0 + i));
    for (int i = 0; i < lv.m; ++i) xt.push_back(box_slot(g, px, py, lv.a0 + i));
    for (int side = 0; side < 2; ++side) {
      const int bx = side ? qx : px, by = side ? qy : py;
      const IdxMap& E = side ? lv.E2 : lv.E1;
      for (int i = 0; i < lv.e; ++i) {
        const int k = imap(E, i);
        if (side_physical(g, bx, by, side_of(g, k))) {
          yt.push_back(-1);
          dt.push_back(-1);
        } else {
          const int s = box_slot(g, bx, by, k);
          yt.push_back(s);
          dt.push_back(slot_partner(g.nx, g.ny, g.p, s));
        }
      }
    }
  }
}

// Tables of the fused levels 1..K for one problem.  Box B of level K+1 holds
// its elements' slots at local index (lx + wx ly) 4p + (side p + k).  The down
// sweep's local set is the box's slots off its boundary plus, at the position
// of each boundary slot, the slot across it (-1 where physical); the up sweep's
// is every slot of the box.
struct FusedTables {
  std::vector<int> gdown, gup;
  std::vector<std::vector<int>> xl, dl, yl;   // index: level
};

FusedTables fused_tables(const Layout& lay) {
  const int K = lay.fuse, p = lay.p, m4 = 4 * p, nx = lay.nx, ny = lay.ny;
  const Geom& gb = lay.lev[K + 1].g;
  const int nloc = gb.wx * gb.wy * m4;
  FusedTables ft;
  ft.gdown.assign((size_t)gb.nboxes * nloc, -1);
  ft.gup.assign((size_t)gb.nboxes * nloc, -1);
  auto local_of = [&](int bx, int by, int s) {
    const int e = s / m4, ix = e % nx, iy = e / nx;
    const int lx = ix - bx * gb.wx, ly = iy - by * gb.wy;
    if (lx < 0 || lx >= gb.wx || ly < 0 || ly >= gb.wy) return -1;
    return (lx + gb.wx * ly) * m4 + s % m4;
  };
  for (int jb = 0; jb < gb.nboxes; ++jb) {
    int bx, by;
    box_xy(gb, jb, bx, by);
    for (int i = 0; i < nloc; ++i) {
      const int le = i / m4, ix = bx * gb.wx + le % gb.wx, iy = by * gb.wy + le / gb.wx;
      const int s = (ix + nx * iy) * m4 + i % m4;
      const int ps = slot_partner(nx, ny, p, s);
      const bool boundary = ps < 0 || local_of(bx, by, ps) < 0;
      ft.gup[(size_t)jb * nloc + i] = s;
      ft.gdown[(size_t)jb * nloc + i] = boundary ? ps : s;
    }
  }
  ft.xl.resize(K + 1);
  ft.dl.resize(K + 1);
  ft.yl.resize(K + 1);
  for (int l = 1; l <= K; ++l) {
    const Level& lv = lay.lev[l];
    std::vector<int> xt, yt, dt;
    pair_tables(lv, xt, yt, dt);
    const int m2 = 2 * lv.m, e2 = 2 * lv.e;
    for (int j = 0; j < lv.pairs; ++j) {
      int bx, by;
      box_xy(gb, j >> (K - l), bx, by);
      for (int i = 0; i < m2; ++i) ft.xl[l].push_back(local_of(bx, by, xt[(size_t)j * m2 + i]));
      for (int i = 0; i < e2; ++i) {
        const int y = yt[(size_t)j * e2 + i], d = dt[(size_t)j * e2 + i];
        ft.yl[l].push_back(y < 0 ? -1 : local_of(bx, by, y));
        // across the face: inside the box, or outside it at the kept slot's position
        ft.dl[l].push_back(d < 0 ? -1 : (local_of(bx, by, d) >= 0 ? local_of(bx, by, d) : local_of(bx, by, y)));
      }
    }
  }
  return ft;
}

const char* check_desc(const hps_desc* d) {
  if (!d) return "null descriptor";
  const int ny = desc_ny(d);
  if (d->n < 1 || d->n > 1024 || (d->n & (d->n - 1)) || ny < 1 || ny > 1024 || (ny & (ny - 1)) ||
      d->n * ny < 2)
    return "n and ny must be powers of two in [1, 1024] with at least two elements";
  if (d->order < 2 || d->order > 16) return "order N must be in [2, 16]";
  if (!(std::isfinite(d->kappa) && d->kappa > 0)) return "kappa must be finite and > 0";
  if (!(std::isfinite(d->eta) && d->eta > 0)) return "eta must be finite and > 0";
  const int Lmax = ilog2(d->n) + ilog2(ny);
  if (d->levels < 0 || d->levels > Lmax) return "levels out of range";
  if (d->coarse_iters == 0 || d->coarse_iters < -1 || d->coarse_iters > kMaxCoarse)
    return "coarse_iters must be -1 (exact) or 1..32";
  const int L = d->levels ? d->levels : Lmax;
  if (d->coarse_iters == -1 && L != Lmax) return "exact coarse solve requires levels = L_max";
  if (d->gamma < 0 || d->gamma > kMaxGamma) return "gamma must be in [1, 4] (0 => 1)";
  if (d->restart < 0 || d->restart > 200) return "restart must be in [1, 200]";
  if (d->precision != HPS_FP64 && d->precision != HPS_MIXED) return "precision must be HPS_FP64 or HPS_MIXED";
  return nullptr;
}

// Per-problem device scratch of the outer Arnoldi step: h (R+2), h2 (R+2), |w|^2, norm, spare.
inline size_t hh_stride(int restart) { return (size_t)2 * (restart + 2) + 4; }

// Shape-only arguments of the fused launch over levels 1..K (for the checks).
FusedArgs fused_shape(const Layout& lay, int K) {
  FusedArgs a{};
  const Geom& gb = lay.lev[K + 1].g;
  a.nloc = gb.wx * gb.wy * 4 * lay.p;
  a.nloc_pad = (a.nloc + 3) & ~3;
  for (int l = 1; l <= K; ++l) {
    const Level& lv = lay.lev[l];
    a.lev[l - 1].m = lv.m;
    a.lev[l - 1].e = lv.e;
  }
  return a;
}

// The V-cycle's levels 1..K run in one launch per direction (one workgroup per
// level-(K+1) box) when every one of them is a merged level of the level-1
// precision with enough pairs for the two-workgroups-per-pair kernels and the
// box's slots and the largest level's group buffers fit the LDS; K = 4 at
// most (groups of 64 threads per pair half at level 1), 2 at least.
void choose_fuse(Layout& lay) {
  lay.fuse = 0;
  if (lay.gamma > 1) return;   // the gamma-cycle revisits levels one at a time
  int K = 0;
  for (int k = 1; k <= kFuseMax && k + 1 <= lay.L; ++k) {
    const Level& lv = lay.lev[k];
    if (!lv.has_merge || lv.f32 != lay.lev[1].f32 || !vc_small_ok(lv.m, lv.e, lay.nq * lv.pairs)) break;
    K = k;
  }
  while (K >= 2 && !fused_ok(fused_shape(lay, K), K)) --K;
  if (K < 2) return;
  lay.fuse = K;
  lay.fnloc = fused_shape(lay, K).nloc;
}

Layout make_layout(const hps_desc* d, int nq) {
  Layout lay;
  lay.nq = nq;
  lay.nx = d->n;
  lay.ny = desc_ny(d);
  lay.N = d->order;
  lay.p = d->order - 1;
  lay.E = lay.nx * lay.ny;
  lay.Lmax = ilog2(lay.nx) + ilog2(lay.ny);
  lay.L = d->levels ? d->levels : lay.Lmax;
  lay.exact = (d->coarse_iters == -1);
  lay.mixed = (d->precision == HPS_MIXED);
  lay.k = lay.exact ? 0 : d->coarse_iters;
  lay.restart = d->restart ? d->restart : 60;
  lay.gamma = d->gamma > 1 ? d->gamma : 1;
  lay.nslots = (long long)lay.E * 4 * lay.p;
  lay.leaf_chunk = (int)std::min<long long>((long long)lay.E * nq, HPS_LEAF_CHUNK);
  const size_t Q = (size_t)nq;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += up256(bytes); return o; };
  const int N1 = lay.N + 1;
  lay.tables_off = take(sizeof(double) * (2 * N1 * N1 + N1));
  lay.H_off = take(sizeof(cd) * Q * lay.E * 4 * lay.p);
  lay.lev.resize(lay.L + 1);
  size_t merge_scratch = 0;
  for (int l = 1; l <= lay.L; ++l) {
    Level& lv = lay.lev[l];
    lv = make_level(lay.nx, lay.ny, lay.p, l);
    // mixed precision: merges 1 .. L-3 (and the V-cycle on those levels) in FP32,
    // the top two merges, the coarse level and the outer operator in FP64
    lv.f32 = lay.mixed && l <= lay.L - 3;
    const size_t nmap = Q * lv.g.nboxes * lv.g.b * lv.g.b;
    lv.T_off = take((l == 1 || !lv.f32 ? sizeof(cd) : sizeof(cf)) * nmap);
    if (l == 1 && lv.f32) lv.T32_off = take(sizeof(cf) * nmap);
    if (lay.mixed && l == lay.L - 2 && l >= 2) lay.stage_off = take(sizeof(cf) * nmap);
    if (l < lay.L || (lay.exact && l == lay.L)) {
      set_merge_geom(lv);
      const size_t es = lv.f32 ? sizeof(cf) : sizeof(cd);
      const size_t np = Q * lv.pairs;
      lv.Ainv_off = take(es * np * 4 * lv.m * lv.m);
      if (l < lay.L) lv.X_off = take(es * np * 4 * lv.m * lv.e);
      lv.map_off = take(sizeof(int) * 2 * (size_t)lv.e);
      lv.xtab_off = take(sizeof(int) * np * 2 * lv.m);
      lv.ytab_off = take(sizeof(int) * np * 2 * lv.e);
      lv.dtab_off = take(sizeof(int) * np * 2 * lv.e);
      lv.Z0_off = take(sizeof(cd) * np * 2 * lv.m);
      const size_t zbytes = sizeof(cd) * np * lv.m * 2 * lv.e;
      merge_scratch = std::max(merge_scratch, up256(zbytes) + up256(inverse_scratch_bytes<cd>(lv.m, (int)np)));
    }
  }
  lay.scratch_bytes = std::max(merge_scratch, sizeof(double) * leaf_scratch_doubles(lay.N, lay.leaf_chunk));
  lay.scratch_off = take(lay.scratch_bytes);
  const size_t vb = sizeof(cd) * Q * lay.nslots;
  lay.V_off = take(vb * (lay.restart + 1));
  lay.Z_off = take(vb * lay.restart);
  lay.work_off = take(up256(vb) * kWorkVectors);
  if (lay.gamma > 1) lay.gam_off = take(up256(vb) * 4 * (size_t)lay.L);
  {
    Level& top = lay.lev[lay.L];
    int nL = 0;
    for (int j = 0; j < top.g.nboxes; ++j) {
      int bx, by;
      box_xy(top.g, j, bx, by);
      for (int s = 0; s < 4; ++s)
        if (!side_physical(top.g, bx, by, s)) nL += top.g.off[s + 1] - top.g.off[s];
    }
    lay.nL = nL;
  }
  const int kk = std::max(lay.k, 1);
  const size_t nL1 = std::max(lay.nL, 1);
  lay.cV_off = take(sizeof(cd) * Q * (kk + 1) * nL1);
  lay.cw_off = take(sizeof(cd) * Q * nL1);
  lay.cx_off = take(sizeof(cd) * Q * nL1);
  lay.cidx_off = take(sizeof(int) * Q * nL1);
  lay.cH_off = take(sizeof(cd) * Q * (kk + 1) * kk);
  lay.cy_off = take(sizeof(cd) * Q * (kk + 1));
  lay.cs_off = take(sizeof(cd) * Q * 8);
  lay.part_off = take(sizeof(cd) * Q * (lay.restart + 2) * kMaxDotBlocks);
  lay.hh_off = take(sizeof(cd) * Q * hh_stride(lay.restart));
  lay.one_off = take(sizeof(cd));
  lay.jctr_off = take(sizeof(int));
  choose_fuse(lay);
  if (lay.fuse) {
    const Geom& gb = lay.lev[lay.fuse + 1].g;
    lay.fgd_off = take(sizeof(int) * Q * gb.nboxes * lay.fnloc);
    lay.fgu_off = take(sizeof(int) * Q * gb.nboxes * lay.fnloc);
    for (int l = 1; l <= lay.fuse; ++l) {
      Level& lv = lay.lev[l];
      const size_t np = Q * lv.pairs;
      lv.xl_off = take(sizeof(int) * np * 2 * lv.m);
      lv.dl_off = take(sizeof(int) * np * 2 * lv.e);
      lv.yl_off = take(sizeof(int) * np * 2 * lv.e);
    }
  }
  lay.ysol_off = take(sizeof(cd) * Q * lay.restart);
  {
    // split-K GEMV partials: at most two descriptors per launch, of the shapes
    // (2m x 2m), (e x m), (2m x 2e) per merge level and (nL/2 x nL/2) for the
    // coarse pair
    size_t mx = 0;
    auto need = [&](int M, int K, int batch, bool always) {
      const int ns = gemv_nsplit(M, K, batch);
      if (ns > 1 || always) mx = std::max(mx, (size_t)ns * batch * M);
    };
    for (int l = 1; l <= lay.L; ++l) {
      const Level& lv = lay.lev[l];
      if (!lv.has_merge) continue;
      const int np = nq * lv.pairs;
      need(2 * lv.m, 2 * lv.m, np, true);  // A^-1 r_x: partial sums even unsplit
      need(lv.e, lv.m, np, false);
      need(2 * lv.m, 2 * lv.e, np, false);
    }
    if (lay.nL > 0) {  // the coarse pair-form product always goes through partial sums
      const int ns = gemv_nsplit(lay.nL / 2, lay.nL / 2, nq);
      mx = std::max(mx, (size_t)ns * nq * (lay.nL / 2));
    }
    // two descriptors' partials, plus those of A^-1 r_x consumed by the T products
    lay.gpart_elems = 3 * mx + 128;
    lay.gpart_off = take(sizeof(cd) * lay.gpart_elems);
  }
  lay.flag_off = take(sizeof(int) * kFlagWords);
  lay.fb_off = take(sizeof(int) * (1 + (size_t)lay.leaf_chunk));
  lay.total = off;
  return lay;
}

enum State { kCreated = 0, kLeaves = 1 };

}  // namespace
}  // namespace hps

// A problem handle holds a group of lay.nq problems of one shape (one for
// hps_problem_create); kappa and eta may differ between them.
struct hps_problem {
  hps_ctx* ctx;
  hps_desc desc;
  std::vector<double> kappa, eta;
  hps::Layout lay;
  char* ws;
  int state;
  int merged;     // highest merge level done
  bool have_T1;
  hipGraphExec_t pgraph = nullptr;  // captured V-cycle (work vector 5 -> 6)
  bool graph_failed = false;
  hipGraphExec_t igraph = nullptr;  // captured FGMRES iteration (index on the device)
  bool igraph_failed = false;
  // levels whose merge inverse uses partial pivoting (set when the inverse
  // without row interchanges failed its threshold test; kept for later builds)
  std::vector<char> pivot_level;
  // build and solve times (hps_info): events on the context's stream at the
  // start of the leaf build, after its latest build step, and around a solve
  hipEvent_t ev_build0 = nullptr, ev_build1 = nullptr, ev_solve0 = nullptr, ev_solve1 = nullptr;
};

using namespace hps;

namespace {

template <class T>
T* at(hps_problem* p, size_t off) { return reinterpret_cast<T*>(p->ws + off); }

hps_status fail(hps_ctx* c, hps_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                                \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail((ctx), HPS_ERR_HIP, std::string("HIP error: ") + hipGetErrorString(_e) + \
                                          " at " #expr);                                 \
  } while (0)

cd* Tlev(hps_problem* p, int l) { return at<cd>(p, p->lay.lev[l].T_off); }

// ---- merge of one level (1 <= l < L): level-l pairs -> level-(l+1) boxes --
// T is the precision of this merge (complex FP64 or FP32); Tin are the level-l
// box maps and Tout receives the level-(l+1) maps, both in that precision.
// Besides the merged maps it leaves, per pair, the explicit A^-1 and X = A^-1 B
// that the V-cycle applies (Sec. 4.3): with W = I - T^P_aa T^Q_bb,
//   A^-1 = [[W^-1, W^-1 T^P_aa], [T^Q_bb W^-1, I + T^Q_bb W^-1 T^P_aa]].
// At the top of an exact solve (l == L) only A^-1 is formed.
template <class T>
hps_status merge_impl(hps_problem* p, int l, const T* Tin, T* Tout) {
  typedef OperandT<T> Operand;
  typedef GemmArgsT<T> GemmArgs;
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const Level& lv = lay.lev[l];
  const int b = lv.g.b, m = lv.m, e = lv.e, np = lay.nq * lv.pairs, m2 = 2 * m;
  const long long pstride = 2LL * b * b;
  const T* TP = Tin;
  const T* TQ = Tin + (size_t)b * b;
  T* Ai = at<T>(p, lv.Ainv_off);
  const long long as = (long long)m2 * m2;
  T* A11 = Ai;
  T* A21 = Ai + m;
  T* A12 = Ai + (size_t)m * m2;
  T* A22 = A12 + m;
  const T one = cx<T>::make(1, 0), zero = cx<T>::make(0, 0), mone = cx<T>::make(-1, 0);
  const Operand none{nullptr, 0, 0, im_off(0), im_off(0)};
  int* flag = at<int>(p, lay.flag_off);
  const bool top = l == lay.L;   // exact top: only A^-1 is needed
  char* scr = at<char>(p, lay.scratch_off);
  const size_t zb = up256(sizeof(cd) * (size_t)np * m * 2 * e);
  T* Z = reinterpret_cast<T*>(scr);
  void* invs = scr + zb;
  const long long zs = (long long)m * 2 * e;
  T* X = top ? nullptr : at<T>(p, lv.X_off);
  const long long xs = (long long)m2 * 2 * e;
  T* YQ = X;
  T* YP = X ? X + m : nullptr;
  const Level& nx = lay.lev[top ? l : l + 1];
  const int* mp = top ? nullptr : at<int>(p, lv.map_off);
  // only rows/columns of the merged boxes' interior sides are ever needed
  auto skip = [&](int row_y, int row_off, int col_y, int col_off) {
    PhysSkip k{};
    k.enabled = 1;
    k.g = nx.g;
    k.nbox = nx.g.nboxes;
    k.ymap = mp;
    k.row_y = row_y;
    k.row_off = row_off;
    k.col_y = col_y;
    k.col_off = col_off;
    return k;
  };
  const PhysSkip sk_c0 = top ? PhysSkip{} : skip(0, 0, 1, 0), sk_ce = top ? PhysSkip{} : skip(0, 0, 1, e);
  // Every block below is written by a GEMM whose C operand (or B operand) is
  // read in place from the children's box maps, so no block is staged by a
  // copy: with y = [P.E1; Q.E2] split into its halves,
  //   W        = I - T^P_aa T^Q_bb   (inverted in place: the (1,1) block of A^-1)
  //   A12 = W^-1 T^P_aa,  A21 = T^Q_bb W^-1,  A22 = I + T^Q_bb A12
  //   Zr       = T^P_aa T^Q_{b,E2}                  (m x e, in Z)
  //   YQ[:, 1] = W^-1 T^P_{a,E1},  YQ[:, 2] = W^-1 Zr          (f^Q_b of y)
  //   YP[:, 1] = T^Q_bb YQ[:, 1],  YP[:, 2] = T^Q_bb YQ[:, 2] + T^Q_{b,E2}
  //   T_new(P.E1, P.E1) = T^P_{E1,a} YP[:, 1] + T^P_{E1,E1}, T_new(P.E1, Q.E2) = T^P_{E1,a} YP[:, 2]
  //   T_new(Q.E2, P.E1) = T^Q_{E2,b} YQ[:, 1], T_new(Q.E2, Q.E2) = T^Q_{E2,b} YQ[:, 2] + T^Q_{E2,E2}
  // (X = A^-1 B: rows [0, m) YQ, rows [m, 2m) YP.)  Products that do not
  // depend on each other share a launch: {W, Zr}, the inverse, {A12, A21,
  // YQ}, {A22, YP}, {T_new}.
  auto gemm = [&](int M_, int N_, int K_) {
    GemmArgs g{};
    g.M = M_; g.N = N_; g.K = K_; g.batch = np;
    g.alpha = one; g.beta = zero; g.C = none;
    return g;
  };
  const Operand Taa{TP, pstride, b, im_off(lv.a0), im_off(lv.a0)};
  const Operand Tbb{TQ, pstride, b, im_off(lv.b0), im_off(lv.b0)};
  const Operand Wi{A11, as, m2, im_off(0), im_off(0)};
  GemmArgs grp[kGemmGroup];
  int ng = 0;
  {
    GemmArgs g = gemm(m, m, m);
    g.A = Taa; g.B = Tbb; g.alpha = mone;
    g.D = A11; g.Dstride = as; g.ldd = m2; g.dr = im_off(0); g.dc = im_off(0);
    g.diag_add = one; g.has_diag = 1;
    grp[ng++] = g;
    if (!top) {
      GemmArgs z = gemm(m, e, m);
      z.A = Taa; z.B = Operand{TQ, pstride, b, im_off(lv.b0), lv.E2};
      z.D = Z; z.Dstride = zs; z.ldd = m; z.dr = im_off(0); z.dc = im_off(0);
      z.skip = sk_ce;
      grp[ng++] = z;
    }
    HIPCHK(c, zgemm_group(grp, ng, st));
  }
  HIPCHK(c, zinverse<T>(A11, m, m2, as, np, invs, flag, l, p->pivot_level[l] != 0, st));
  ng = 0;
  {
    GemmArgs g = gemm(m, m, m);
    g.Dstride = as; g.ldd = m2; g.dr = im_off(0); g.dc = im_off(0);
    g.A = Wi; g.B = Taa; g.D = A12;
    grp[ng++] = g;
    g.A = Tbb; g.B = Wi; g.D = A21;
    grp[ng++] = g;
    if (!top) {
      GemmArgs y = gemm(m, e, m);
      y.A = Wi; y.D = YQ; y.Dstride = xs; y.ldd = m2; y.dr = im_off(0);
      y.B = Operand{TP, pstride, b, im_off(lv.a0), lv.E1};
      y.dc = im_off(0);
      y.skip = sk_c0;
      grp[ng++] = y;
      y.B = Operand{Z, zs, m, im_off(0), im_off(0)};
      y.dc = im_off(e);
      y.skip = sk_ce;
      grp[ng++] = y;
    }
    HIPCHK(c, zgemm_group(grp, ng, st));
  }
  ng = 0;
  {
    GemmArgs g = gemm(m, m, m);
    g.Dstride = as; g.ldd = m2; g.dr = im_off(0); g.dc = im_off(0);
    g.A = Tbb; g.B = Operand{A12, as, m2, im_off(0), im_off(0)}; g.D = A22;
    g.diag_add = one; g.has_diag = 1;
    grp[ng++] = g;
    if (!top) {
      GemmArgs y = gemm(m, e, m);
      y.A = Tbb; y.D = YP; y.Dstride = xs; y.ldd = m2; y.dr = im_off(0);
      y.B = Operand{YQ, xs, m2, im_off(0), im_off(0)};
      y.dc = im_off(0);
      y.skip = sk_c0;
      grp[ng++] = y;
      y.B = Operand{YQ, xs, m2, im_off(0), im_off(e)};
      y.beta = one; y.C = Operand{TQ, pstride, b, im_off(lv.b0), lv.E2}; y.dc = im_off(e);
      y.skip = sk_ce;
      grp[ng++] = y;
    }
    HIPCHK(c, zgemm_group(grp, ng, st));
  }
  if (top) return HPS_OK;
  T* Tn = Tout;
  const int bn = nx.g.b;
  const long long ns = (long long)bn * bn;
  const IdxMap rowP = im_tab(mp), rowQ = im_tab(mp + e), colP = im_tab(mp), colQ = im_tab(mp + e);
  const PhysSkip s00 = skip(1, 0, 1, 0), s0e = skip(1, 0, 1, e), se0 = skip(1, e, 1, 0), see = skip(1, e, 1, e);
  {
    GemmArgs g = gemm(e, e, m);
    g.D = Tn; g.Dstride = ns; g.ldd = bn;
    // rows P.E1
    g.A = Operand{TP, pstride, b, lv.E1, im_off(lv.a0)};
    g.dr = rowP;
    g.B = Operand{YP, xs, m2, im_off(0), im_off(0)};
    g.beta = one; g.C = Operand{TP, pstride, b, lv.E1, lv.E1}; g.dc = colP;
    g.skip = s00;
    grp[0] = g;
    g.B = Operand{YP, xs, m2, im_off(0), im_off(e)};
    g.beta = zero; g.C = none; g.dc = colQ;
    g.skip = s0e;
    grp[1] = g;
    // rows Q.E2
    g.A = Operand{TQ, pstride, b, lv.E2, im_off(lv.b0)};
    g.dr = rowQ;
    g.B = Operand{YQ, xs, m2, im_off(0), im_off(0)};
    g.beta = zero; g.C = none; g.dc = colP;
    g.skip = se0;
    grp[2] = g;
    g.B = Operand{YQ, xs, m2, im_off(0), im_off(e)};
    g.beta = one; g.C = Operand{TQ, pstride, b, lv.E2, lv.E2}; g.dc = colQ;
    g.skip = see;
    grp[3] = g;
    HIPCHK(c, zgemm_group(grp, 4, st));
  }
  return HPS_OK;
}

template <class M>
M* Tmat(hps_problem* p, int l) {
  const Level& lv = p->lay.lev[l];
  return at<M>(p, (l == 1 && lv.f32) ? lv.T32_off : lv.T_off);
}

hps_status merge_one(hps_problem* p, int l) {
  const Layout& lay = p->lay;
  const Level& lv = lay.lev[l];
  if (!lv.f32) {
    cd* out = (l < lay.L) ? Tlev(p, l + 1) : nullptr;
    return merge_impl<cd>(p, l, Tlev(p, l), out);
  }
  const Level& nx = lay.lev[l + 1];
  cf* out = nx.f32 ? at<cf>(p, nx.T_off) : at<cf>(p, lay.stage_off);
  hps_status s = merge_impl<cf>(p, l, Tmat<cf>(p, l), out);
  if (s != HPS_OK || nx.f32) return s;
  // the next merge runs in FP64: widen the level-(l+1) maps
  HIPCHK(p->ctx, convert_c32_c64(out, Tlev(p, l + 1), (long long)lay.nq * nx.g.nboxes * nx.g.b * nx.g.b,
                                 p->ctx->stream));
  return HPS_OK;
}

// ---- V-cycle -------------------------------------------------------------
bool small_level(const Level& lv, int nq) {
  return vc_small_ok(lv.m, lv.e, nq * lv.pairs);
}

template <class M>
SmallLevelT<M> small_args(hps_problem* p, const Level& lv) {
  SmallLevelT<M> a;
  a.g = lv.g;
  a.m = lv.m;
  a.e = lv.e;
  a.a0 = lv.a0;
  a.b0 = lv.b0;
  a.E1 = lv.E1;
  a.E2 = lv.E2;
  a.T = Tmat<M>(p, lv.g.level);
  a.Ainv = at<M>(p, lv.Ainv_off);
  a.X = lv.X_off ? at<M>(p, lv.X_off) : nullptr;
  a.xtab = at<int>(p, lv.xtab_off);
  a.ytab = at<int>(p, lv.ytab_off);
  a.dtab = at<int>(p, lv.dtab_off);
  a.Z0 = at<cd>(p, lv.Z0_off);
  return a;
}

VecIn vin_compact(const cd* ptr, long long stride) {
  VecIn v{};
  v.p = ptr;
  v.stride = stride;
  return v;
}
// x = the sum of a (pM x pbatch) GEMV's split-K partials from row proff on;
// row tile 0 stores it at save + b * save_stride + proff.
VecIn vin_partials(const cd* ps, int pns, int pbatch, int pM, int proff, cd* save, long long save_stride) {
  VecIn v{};
  v.ps = ps;
  v.pns = pns;
  v.pbatch = pbatch;
  v.pM = pM;
  v.proff = proff;
  v.save = save;
  v.save_stride = save_stride;
  v.save_off = proff;
  return v;
}
VecIn vin_table(const cd* vec, const int* tab, long long tstride) {
  VecIn v{};
  v.vec = vec;
  v.tab = tab;
  v.tstride = tstride;
  return v;
}
void vout_table(VecOut& v, cd* vec, const int* tab, long long tstride, bool add) {
  v.vec = vec;
  v.tab = tab;
  v.tstride = tstride;
  v.add = add ? 1 : 0;
}
VecOut vout_compact(cd* ptr, long long stride, const cd* y0 = nullptr, long long y0s = 0) {
  VecOut v{};
  v.p = ptr;
  v.stride = stride;
  v.y0 = y0;
  v.y0stride = y0s;
  v.beta = cmk(1, 0);
  return v;
}
template <class M>
GemvDescT<M> gdesc(int Mr, int K, OperandT<M> A, VecIn x, VecOut y, cd alpha = cmk(1, 0)) {
  GemvDescT<M> d{};
  d.M_ = Mr;
  d.K = K;
  d.A = A;
  d.alpha = alpha;
  d.x = x;
  d.y = y;
  return d;
}

// Down sweep of level l on the residual w (canonical, updated in place):
// z0 = A^-1 r_x for every pair (kept in Z0), then the rows across the kept
// faces receive C~ z0: w[Pi(P.E1)] += T^P_{E1,a} z0_P, w[Pi(Q.E2)] += T^Q_{E2,b} z0_Q.
// M is the storage precision of the level's operators.
template <class M>
hps_status vcycle_down_t(hps_problem* p, int l, cd* wv) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Level& lv = p->lay.lev[l];
  if (small_level(lv, p->lay.nq)) {
    HIPCHK(c, vc_down_small(small_args<M>(p, lv), p->lay.nq * lv.pairs, wv, st));
    return HPS_OK;
  }
  const int b = lv.g.b, m = lv.m, e = lv.e, np = p->lay.nq * lv.pairs, m2 = 2 * m;
  const long long ps = 2LL * b * b;
  const M* T = Tmat<M>(p, l);
  cd* Z0 = at<cd>(p, lv.Z0_off);
  const int* dtab = at<int>(p, lv.dtab_off);
  cd* part = at<cd>(p, p->lay.gpart_off);
  // z0 = A^-1 r_x as split-K partial sums only: the T products below sum them
  // while staging their x (and row tile 0 stores z0 in Z0), so no reduction
  // launch sits between the two products
  GemvDescT<M> d0 = gdesc<M>(m2, m2, OperandT<M>{at<M>(p, lv.Ainv_off), (long long)m2 * m2, m2, im_off(0), im_off(0)},
                             vin_table(wv, at<int>(p, lv.xtab_off), m2), vout_compact(nullptr, 0));
  GemvPartLayout pl{};
  HIPCHK(c, zgemv_partials(&d0, 1, np, part, &pl, st));
  const cd* pz = part + pl.poff[0];
  cd* part2 = part + up256(sizeof(cd) * (size_t)pl.nsplit[0] * np * m2) / sizeof(cd);
  VecOut oP{}, oQ{};
  vout_table(oP, wv, dtab, 2 * e, true);
  vout_table(oQ, wv, dtab + e, 2 * e, true);
  GemvDescT<M> d[2] = {gdesc<M>(e, m, OperandT<M>{T, ps, b, lv.E1, im_off(lv.a0)}, vin_partials(pz, pl.nsplit[0], np, m2, m, Z0, m2), oP),
                       gdesc<M>(e, m, OperandT<M>{T + (size_t)b * b, ps, b, lv.E2, im_off(lv.b0)},
                                vin_partials(pz, pl.nsplit[0], np, m2, 0, Z0, m2), oQ)};
  HIPCHK(c, zgemv_batched(d, 2, np, part2, st));
  return HPS_OK;
}

// Up sweep of level l: x = z0 + X y with y the kept-face values already in z,
// written into z at the shared-face slots.
template <class M>
hps_status vcycle_up_t(hps_problem* p, int l, cd* z) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Level& lv = p->lay.lev[l];
  if (vc_up_small_ok(lv.m, lv.e, p->lay.nq * lv.pairs)) {
    HIPCHK(c, vc_up_small(small_args<M>(p, lv), p->lay.nq * lv.pairs, z, st));
    return HPS_OK;
  }
  const int m2 = 2 * lv.m, e2 = 2 * lv.e, np = p->lay.nq * lv.pairs;
  const cd* Z0 = at<cd>(p, lv.Z0_off);
  VecOut o = vout_compact(nullptr, 0, Z0, m2);
  vout_table(o, z, at<int>(p, lv.xtab_off), m2, false);
  GemvDescT<M> d = gdesc<M>(m2, e2, OperandT<M>{at<M>(p, lv.X_off), (long long)m2 * e2, m2, im_off(0), im_off(0)},
                            vin_table(z, at<int>(p, lv.ytab_off), e2), o);
  HIPCHK(c, zgemv_batched(&d, 1, np, at<cd>(p, p->lay.gpart_off), st));
  return HPS_OK;
}

// Levels 1..fuse of the down (r updated in place) or up (z) sweep in one launch.
hipError_t fused_levels(hps_problem* p, bool down, cd* vec) {
  const Layout& lay = p->lay;
  const int K = lay.fuse;
  FusedArgs a = fused_shape(lay, K);
  a.gdown = at<int>(p, lay.fgd_off);
  a.gup = at<int>(p, lay.fgu_off);
  const bool f32 = lay.lev[1].f32;
  for (int l = 1; l <= K; ++l) {
    const Level& lv = lay.lev[l];
    FusedLevel& L = a.lev[l - 1];
    L.a0 = lv.a0;
    L.b0 = lv.b0;
    L.b = lv.g.b;
    L.E1 = lv.E1;
    L.E2 = lv.E2;
    L.T = f32 ? (const void*)Tmat<cf>(p, l) : (const void*)Tmat<cd>(p, l);
    L.Ainv = p->ws + lv.Ainv_off;
    L.X = p->ws + lv.X_off;
    L.xl = at<int>(p, lv.xl_off);
    L.dl = at<int>(p, lv.dl_off);
    L.yl = at<int>(p, lv.yl_off);
    L.Z0 = at<cd>(p, lv.Z0_off);
  }
  const int boxes = lay.nq * lay.lev[K + 1].g.nboxes;
  return f32 ? vc_fused<cf>(a, K, boxes, vec, down, p->ctx->stream)
             : vc_fused<cd>(a, K, boxes, vec, down, p->ctx->stream);
}

hps_status vcycle_down(hps_problem* p, int l, cd* wv) {
  return p->lay.lev[l].f32 ? vcycle_down_t<cf>(p, l, wv) : vcycle_down_t<cd>(p, l, wv);
}

hps_status vcycle_up(hps_problem* p, int l, cd* z) {
  return p->lay.lev[l].f32 ? vcycle_up_t<cf>(p, l, z) : vcycle_up_t<cd>(p, l, z);
}

// Canonical group vectors (nq * nslots entries): 0 the V-cycle residual, 1 the
// FGMRES residual, 2-3 coarse scratch, 4 the Arnoldi vector, 5-6 the captured
// V-cycle's input and output, 7-8 the group's right-hand side and solution.
cd* workv(hps_problem* p, int i) {
  return reinterpret_cast<cd*>(p->ws + p->lay.work_off +
                               i * up256(sizeof(cd) * (size_t)p->lay.nslots * p->lay.nq));
}

// Classical Gram-Schmidt, two passes, against V[0..nv) for each problem of
// the group (segments of n entries), then the normalisation: the passes'
// coefficients in h and h2 (problem q at + q*hs; the Hessenberg column is
// their sum, which the host forms when it reads them back), the new basis
// vector in out (displaced by (*jdev + 1) * jstride with jdev set) and its
// norm in hout (+ q*hs).  The second pass's dot products also give |w'|^2
// (into nrm2 + q*hs), and its update is fused with the normalisation: with V
// orthonormal |w''|^2 = |w'|^2 - |h2|^2.  w holds w' afterwards.
// With nvdev set the vector count is *nvdev + 1, read on the device, and nv
// is the largest it may be.
hps_status cgs2_normalize(hps_problem* p, const cd* V, long long vstride, int nv, cd* w, long long n, cd* h,
                          cd* h2, cd* nrm2, cd* out, cd* hout, long long hs, const int* nvdev = nullptr,
                          const int* jdev = nullptr, long long jstride = 0) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const int nq = p->lay.nq;
  cd* part = at<cd>(p, p->lay.part_off);
  HIPCHK(c, multi_dot(V, vstride, nv, w, n, part, h, false, st, nq, hs, nvdev));
  HIPCHK(c, multi_axpy(V, vstride, nv, h, w, n, -1, st, nq, hs, nvdev));
  HIPCHK(c, multi_dot(V, vstride, nv, w, n, part, h2, false, st, nq, hs, nvdev, nrm2));
  HIPCHK(c, axpy_normalize(V, vstride, nv, h2, hs, w, n, nrm2, hs, out, hout, hs, st, nq, nvdev, jdev, jstride));
  return HPS_OK;
}

// Coarse matvec w = M_L v on compact coarse vectors below the top level: the
// level-L skeleton matvec on canonical scratch vectors.  v: problem q's vector
// at v + q*vstride; w: [nq][nL].  (At the top level the coarse system is the
// single pair's A_L; coarse_solve forms that product from split-K partial sums
// inside its Arnoldi step.)
hps_status coarse_matvec(hps_problem* p, const cd* v, long long vstride, cd* w) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const Level& top = lay.lev[lay.L];
  const int* idx = at<int>(p, lay.cidx_off);
  cd* u1 = workv(p, 2);
  cd* u2 = workv(p, 3);
  HIPCHK(c, index_scatter(idx, lay.nL, v, u1, st, lay.nq, vstride));
  HIPCHK(c, skeleton_apply(top.g, Tlev(p, lay.L), u1, u2, false, st, lay.nq));
  HIPCHK(c, index_gather(idx, lay.nL, u2, w, st, lay.nq));
  return HPS_OK;
}

// Coarse solve at level L on the level-L unknowns held in wv; result into z.
hps_status coarse_solve(hps_problem* p, cd* wv, cd* z) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const Level& top = lay.lev[lay.L];
  const int nq = lay.nq;
  if (lay.exact) {
    // z at the top pair's shared face = A_L^-1 r_x
    const int m2 = 2 * top.m;
    const int* xtab = at<int>(p, top.xtab_off);
    VecOut o = vout_compact(nullptr, 0);
    vout_table(o, z, xtab, m2, false);
    GemvDesc d = gdesc<cd>(m2, m2, Operand{at<cd>(p, top.Ainv_off), (long long)m2 * m2, m2, im_off(0), im_off(0)},
                           vin_table(wv, xtab, m2), o);
    HIPCHK(c, zgemv_batched(&d, 1, nq, at<cd>(p, lay.gpart_off), st));
    return HPS_OK;
  }
  const int nL = lay.nL, k = lay.k;
  if (nL == 0) return HPS_OK;
  const long long vq = (long long)(k + 1) * nL;  // one problem's coarse basis
  const int hsize = (k + 1) * k;
  const int* idx = at<int>(p, lay.cidx_off);
  cd* V = at<cd>(p, lay.cV_off);
  cd* w = at<cd>(p, lay.cw_off);
  cd* wt = at<cd>(p, lay.cx_off);
  cd* H = at<cd>(p, lay.cH_off);
  cd* sc = at<cd>(p, lay.cs_off);  // beta^2 per problem
  cd* part = at<cd>(p, lay.gpart_off);
  const bool pair_form = lay.L == lay.Lmax;
  // pair form on short coarse vectors: the start and the finish run inside the
  // first and last Arnoldi launches, and the first product reads w0 = wv[idx]
  const bool fold = pair_form && coarse_fast_ok(nL, k);
  const CoarseEnds ends{idx, wv, z, sc, k};
  if (!fold) HIPCHK(c, coarse_start(idx, nL, wv, V, vq, H, hsize, sc, nq, st));
  for (int j = 0; j < k; ++j) {
    const cd* vj = V + (size_t)j * nL;
    CoarseW src{};
    if (pair_form) {
      // M_L v = [v_P - T^Q_bb v_Q ; v_Q - T^P_aa v_P] on [P.alpha; Q.beta]
      const int b = top.g.b;
      const int m = nL / 2;
      const cd* T = Tlev(p, lay.L);
      const long long ts = 2LL * b * b;  // one problem's two top boxes
      // the shared face: P's right and Q's left side (a merge along x, e.g. the
      // last merge of a wide rectangular mesh), else P's top and Q's bottom
      const bool along_x = merge_axis_of(top.g.ax, top.g.ay, lay.L) == 0;
      const int aP = along_x ? top.g.off[1] : top.g.off[3], bQ = along_x ? top.g.off[0] : top.g.off[2];
      const bool w0 = fold && j == 0;   // the product of w0 = wv[idx] (V_0 is formed after it)
      GemvDesc d[2] = {gdesc<cd>(m, m, Operand{T + (size_t)b * b, ts, b, im_off(bQ), im_off(bQ)},
                                 w0 ? vin_table(wv, idx + m, nL) : vin_compact(vj + m, vq), vout_compact(nullptr, 0)),
                       gdesc<cd>(m, m, Operand{T, ts, b, im_off(aP), im_off(aP)},
                                 w0 ? vin_table(wv, idx, nL) : vin_compact(vj, vq), vout_compact(nullptr, 0))};
      // at most 8 splits: the single-workgroup Arnoldi step reads every partial
      GemvPartLayout pl{};
      HIPCHK(c, zgemv_partials(d, 2, nq, part, &pl, st, 8));
      src.part = part;
      src.poff0 = pl.poff[0];
      src.poff1 = pl.poff[1];
      src.ns0 = pl.nsplit[0];
      src.ns1 = pl.nsplit[1];
      src.m = m;
      src.nb = nq;
    } else {
      hps_status s = coarse_matvec(p, vj, vq, w);
      if (s != HPS_OK) return s;
      src.w = w;
    }
    HIPCHK(c, coarse_arnoldi(V, nL, vq, j, src, wt, H + (size_t)j * (k + 1), hsize, nq, st, fold ? &ends : nullptr));
  }
  if (!fold) HIPCHK(c, coarse_finish(H, k, hsize, sc, V, nL, vq, idx, z, nq, st));
  return HPS_OK;
}

hps_status mg_gamma(hps_problem* p, int l, const cd* r, cd* z);

hps_status precond_one(hps_problem* p, const cd* r, cd* z) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  if (lay.gamma > 1) {
    HIPCHK(c, vfill(z, lay.nslots * lay.nq, cmk(0, 0), st));
    return mg_gamma(p, 1, r, z);
  }
  cd* wv = workv(p, 0);
  const long long ntot = lay.nslots * lay.nq;
  HIPCHK(c, vcopy_zero(r, wv, z, ntot, st));   // wv = r, z = 0
  if (lay.fuse) HIPCHK(c, fused_levels(p, true, wv));
  for (int l = lay.fuse + 1; l < lay.L; ++l) {
    hps_status s = vcycle_down(p, l, wv);
    if (s != HPS_OK) return s;
  }
  hps_status s = coarse_solve(p, wv, z);
  if (s != HPS_OK) return s;
  for (int l = lay.L - 1; l > lay.fuse; --l) {
    s = vcycle_up(p, l, z);
    if (s != HPS_OK) return s;
  }
  if (lay.fuse) HIPCHK(c, fused_levels(p, false, z));
  return HPS_OK;
}

// gamma-cycle (gamma > 1, Sec. 4.3 "multiple coarse calls"): at every level
// the coarse correction is a stationary iteration of gamma steps on the
// level's Schur complement M_{l+1},
//   y = 0;  repeat gamma times:  y += MG_{l+1}(r~ - M_{l+1} y),
// with r~ the level-(l+1) residual left by the down sweep; gamma = 1 is the
// V-cycle.  Vectors are canonical (only the level's unknowns are meaningful);
// level l uses its own W (the residual, reduced in place by the down sweep),
// Y (the iterate), R (the stationary residual) and D (the correction), so
// the recursion needs no allocation.  r is read at level-l slots; z receives
// MG_l r at level-l slots (other slots untouched).
cd* gamv(hps_problem* p, int l, int which) {
  const size_t vb = up256(sizeof(cd) * (size_t)p->lay.nslots * p->lay.nq);
  return reinterpret_cast<cd*>(p->ws + p->lay.gam_off + ((size_t)(l - 1) * 4 + which) * vb);
}

hps_status mg_gamma(hps_problem* p, int l, const cd* r, cd* z) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const long long ntot = lay.nslots * lay.nq;
  if (l == lay.L) {
    HIPCHK(c, vcopy(r, workv(p, 0), ntot, st));
    return coarse_solve(p, workv(p, 0), z);
  }
  cd* W = gamv(p, l, 0);
  cd* Y = gamv(p, l, 1);
  cd* R = gamv(p, l, 2);
  cd* D = gamv(p, l, 3);
  HIPCHK(c, vcopy_zero(r, W, Y, ntot, st));   // W = r, Y = 0
  hps_status s = vcycle_down(p, l, W);        // z0 in Z0; W at level-(l+1) slots = r~
  if (s != HPS_OK) return s;
  const Level& nx = lay.lev[l + 1];
  for (int it = 0; it < lay.gamma; ++it) {
    const cd* src = W;
    if (it > 0) {
      // R = r~ - M_{l+1} Y (M_{l+1} in the precision its maps are stored in)
      if (nx.f32)
        HIPCHK(c, skeleton_apply(nx.g, at<cf>(p, nx.T_off), Y, R, false, st, lay.nq));
      else
        HIPCHK(c, skeleton_apply(nx.g, Tlev(p, l + 1), Y, R, false, st, lay.nq));
      HIPCHK(c, axpby(cmk(1, 0), W, cmk(-1, 0), R, R, ntot, st));
      src = R;
    }
    HIPCHK(c, vfill(D, ntot, cmk(0, 0), st));
    s = mg_gamma(p, l + 1, src, D);
    if (s != HPS_OK) return s;
    HIPCHK(c, axpby(cmk(1, 0), Y, cmk(1, 0), D, Y, ntot, st));
  }
  HIPCHK(c, vcopy(Y, z, ntot, st));            // z = y at level-(l+1) slots
  return vcycle_up(p, l, z);                    // x = z0 + X y at the level's shared faces
}

// The V-cycle is a fixed sequence of launches for a given problem, so it is
// captured once into a HIP graph (reading work vector 5, writing work vector 6)
// and replayed; this removes the host launch cost of ~10^2 small kernels per
// application.  The graph holds no memset nodes and no host synchronisation.
hps_status precond_graphed(hps_problem* p, const cd* r, cd* z) {
  hps_ctx* c = p->ctx;
  const long long n = p->lay.nslots * p->lay.nq;
  cd* rin = workv(p, 5);
  cd* zout = workv(p, 6);
  if (!p->pgraph && !p->graph_failed) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // run once eagerly so that every kernel attribute is set outside the capture
    HIPCHK(c, vcopy(r, rin, n, c->stream));
    hps_status s = precond_one(p, rin, zout);
    if (s != HPS_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      s = precond_one(p, rin, zout);
      e = hipStreamEndCapture(c->stream, &graph);
    }
    c->stream = saved;
    if (e == hipSuccess && s == HPS_OK && graph) e = hipGraphInstantiate(&p->pgraph, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || s != HPS_OK || !p->pgraph) {
      p->pgraph = nullptr;
      p->graph_failed = true;
      (void)hipGetLastError();
    }
  }
  if (!p->pgraph) return precond_one(p, r, z);
  HIPCHK(c, vcopy(r, rin, n, c->stream));
  HIPCHK(c, hipGraphLaunch(p->pgraph, c->stream));
  HIPCHK(c, vcopy(zout, z, n, c->stream));
  return HPS_OK;
}

hps_status precond_any(hps_problem* p, const cd* r, cd* z) {
  return p->ctx->use_graphs ? precond_graphed(p, r, z) : precond_one(p, r, z);
}

hps_status check_ready(hps_problem* p, bool need_merges) {
  if (!p) return HPS_ERR_ARG;
  if (p->state < kLeaves) return fail(p->ctx, HPS_ERR_STATE, "leaves not built");
  if (need_merges) {
    const int need = p->lay.exact ? p->lay.L : p->lay.L - 1;
    if (p->merged < need) return fail(p->ctx, HPS_ERR_STATE, "merge levels missing");
  }
  return HPS_OK;
}

// Reads the problem's device error words (synchronises) and turns a recorded
// failure into a status and a message naming where it happened; `first` is
// the caller's index of the handle's first problem.
hps_status read_flag(hps_problem* p, int first = 0) {
  int f[kFlagWords];
  HIPCHK(p->ctx, hipMemcpyAsync(f, at<int>(p, p->lay.flag_off), sizeof(f), hipMemcpyDeviceToHost, p->ctx->stream));
  HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
  const Layout& lay = p->lay;
  auto word = [&](int i) {
    unsigned long long v;
    std::memcpy(&v, f + i, sizeof(v));
    return v;
  };
  if (f[0] & kFlagNonFinite) {
    const long long G = (long long)word(4);
    const long long q = G / lay.E, e = G % lay.E;
    return fail(p->ctx, HPS_ERR_ARG,
                "non-finite value in b_nodes or s_nodes of problem " + std::to_string(first + q) + ", element " +
                    std::to_string(e) + " (ix " + std::to_string(e % lay.nx) + ", iy " + std::to_string(e / lay.nx) +
                    "); its leaf map was not built");
  }
  if (f[0] & kFlagSingular) {
    const unsigned long long w = word(2);
    const int level = (int)(w >> 40);
    const long long idx = (long long)(w & ((1ull << 40) - 1));
    std::string where;
    if (level == 0) {
      const long long q = idx / lay.E, e = idx % lay.E;
      where = "the leaf map of problem " + std::to_string(first + q) + ", element " + std::to_string(e);
    } else {
      const int pairs = (level <= lay.L && lay.lev[level].has_merge) ? lay.lev[level].pairs : 1;
      const long long q = idx / pairs, j = idx % pairs;
      where = "merge level " + std::to_string(level) + " of problem " + std::to_string(first + q) + ", pair " +
              std::to_string(j) + " (boxes " + std::to_string(2 * j) + " and " + std::to_string(2 * j + 1) +
              " in merge-tree order)";
    }
    return fail(p->ctx, HPS_ERR_SINGULAR, "zero pivot in " + where);
  }
  return HPS_OK;
}

// The blocked merge inverses run without row interchanges across blocks
// under a threshold test (inverse.hip); a level that failed it is recorded in
// error word 6.  This switches that level to partial pivoting and redoes the
// merges from it up to the last one done, until no level fails (at most L
// rounds).  Synchronises.
hps_status stabilize_merges(hps_problem* p) {
  static const int kNone = 0x7FFFFFFF;
  int* w6 = at<int>(p, p->lay.flag_off) + 6;
  for (int round = 0; round <= p->lay.L; ++round) {
    int lv = kNone;
    HIPCHK(p->ctx, hipMemcpyAsync(&lv, w6, sizeof(int), hipMemcpyDeviceToHost, p->ctx->stream));
    HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
    if (lv == kNone || lv < 1 || lv > p->merged) return HPS_OK;
    p->pivot_level[lv] = 1;
    HIPCHK(p->ctx, hipMemcpyAsync(w6, &kNone, sizeof(int), hipMemcpyHostToDevice, p->ctx->stream));
    for (int l = lv; l <= p->merged; ++l) {
      const hps_status s = merge_one(p, l);
      if (s != HPS_OK) return s;
    }
  }
  return fail(p->ctx, HPS_ERR_STATE, "merge inverses did not stabilise");
}

// ---- outer flexible GMRES ------------------------------------------------
typedef std::complex<double> zc;

// Flexible GMRES(R) for all nq problems of a group in lock step: every
// iteration runs one V-cycle, one M_1 product and one CGS2 step for the whole
// group and copies the group's Hessenberg columns to the host once; Givens
// rotations, estimates and stopping are per problem.  A problem that has
// converged (or reached maxit) stops taking part in the least-squares updates,
// so its solution stays as it was.  rhs, g: group vectors.
// One FGMRES iteration with its index j read on the device (the int at
// jctr_off): V_j into the V-cycle's input vector, the preconditioner, its
// output into Z_j, the M_1 product, CGS2 against V_0..V_j with V_{j+1} and its
// norm formed by the second pass's update, then j + 1.  Every launch has the same arguments for every j, so one
// captured graph serves all iterations of all cycles.
hps_status iteration_kernels(hps_problem* p) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const int nq = lay.nq;
  const long long n = lay.nslots, ntot = n * nq;
  const int R = lay.restart;
  const long long HS = (long long)hh_stride(R);
  cd* V = at<cd>(p, lay.V_off);
  cd* Z = at<cd>(p, lay.Z_off);
  cd* w = workv(p, 4);
  cd* rin = workv(p, 5);
  cd* zout = workv(p, 6);
  cd* hh = at<cd>(p, lay.hh_off);
  cd* nrm2 = hh + 2 * (R + 2);
  int* jctr = at<int>(p, lay.jctr_off);
  HIPCHK(c, vcopy_at(V, rin, ntot, jctr, nullptr, ntot, st));
  hps_status s = precond_one(p, rin, zout);
  if (s != HPS_OK) return s;
  HIPCHK(c, vcopy_at(zout, Z, ntot, nullptr, jctr, ntot, st));
  HIPCHK(c, skeleton_apply(lay.lev[1].g, Tlev(p, 1), zout, w, true, st, nq));
  s = cgs2_normalize(p, V, ntot, R, w, n, hh, hh + (R + 2), nrm2, V, nrm2 + 1, HS, jctr, jctr, ntot);
  if (s != HPS_OK) return s;
  HIPCHK(c, counter_add(jctr, 1, st));
  return HPS_OK;
}

// Captures iteration_kernels into p->igraph on first use; the caller has just
// run them eagerly (so every kernel attribute is set outside the capture).  A
// capture that fails leaves the problem on eager launches.
void capture_iteration(hps_problem* p) {
  hps_ctx* c = p->ctx;
  if (p->igraph || p->igraph_failed) return;
  p->igraph_failed = true;
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  hipStream_t saved = c->stream;
  c->stream = c->cap_stream;
  hipGraph_t graph = nullptr;
  hps_status s = HPS_ERR_HIP;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    s = iteration_kernels(p);
    e = hipStreamEndCapture(c->stream, &graph);
  }
  c->stream = saved;
  if (e == hipSuccess && s == HPS_OK && graph) e = hipGraphInstantiate(&p->igraph, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e == hipSuccess && s == HPS_OK && p->igraph) {
    p->igraph_failed = false;
  } else {
    p->igraph = nullptr;
    (void)hipGetLastError();
  }
}

hps_status fgmres_group(hps_problem* p, const cd* rhs, cd* g, double tol, int maxit, hps_info* info) {
  hps_ctx* c = p->ctx;
  hipStream_t st = c->stream;
  const Layout& lay = p->lay;
  const int nq = lay.nq;
  const long long n = lay.nslots;
  const long long ntot = n * nq;
  const int R = lay.restart;
  const long long HS = (long long)hh_stride(R);
  cd* V = at<cd>(p, lay.V_off);
  cd* Z = at<cd>(p, lay.Z_off);
  cd* res = workv(p, 1);
  cd* w = workv(p, 4);
  cd* hh = at<cd>(p, lay.hh_off);  // per problem q at hh + q*HS: h [R+2], h2 [R+2], |w|^2, norm
  cd* hcol = hh;
  cd* h2 = hh + (R + 2);
  cd* nrm2 = hh + 2 * (R + 2);
  cd* hnorm = nrm2 + 1;
  cd* part = at<cd>(p, lay.part_off);
  cd* ysol = at<cd>(p, lay.ysol_off);
  const Geom& g1 = lay.lev[1].g;
  const cd* T1 = Tlev(p, 1);
  const size_t hn = (size_t)HS * nq;
  if (c->hbuf_bytes < sizeof(cd) * 2 * hn) {
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    c->hbuf = nullptr;
    c->hbuf_bytes = 0;
    const size_t bytes = std::max<size_t>(sizeof(cd) * 2 * hn, 64 << 10);
    HIPCHK(c, hipHostMalloc(&c->hbuf, bytes, hipHostMallocDefault));
    c->hbuf_bytes = bytes;
  }
  for (int i = 0; i < 2; ++i)
    if (!c->hev[i]) HIPCHK(c, hipEventCreateWithFlags(&c->hev[i], hipEventDisableTiming));
  cd* hbuf = static_cast<cd*>(c->hbuf);
  const cd* host = hbuf;
  // graphs on: every iteration replays one captured graph
  int* jctr = at<int>(p, lay.jctr_off);
  bool graphed = c->use_graphs != 0 && !p->igraph_failed;
  auto fetch = [&]() -> hps_status {
    HIPCHK(c, hipMemcpyAsync(hbuf, hh, sizeof(cd) * hn, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return HPS_OK;
  };
  for (int q = 0; q < nq; ++q) info[q] = hps_info{HPS_OK, 0, 0.0, 0.0, 0.0, 0.0};
  // ||rhs|| per problem
  HIPCHK(c, multi_dot(rhs, 0, 1, rhs, n, part, nrm2, false, st, nq, HS));
  hps_status s = fetch();
  if (s != HPS_OK) return s;
  std::vector<double> bnorm(nq);
  for (int q = 0; q < nq; ++q) bnorm[q] = std::sqrt(std::max(host[q * HS + 2 * (R + 2)].x, 0.0));
  HIPCHK(c, vfill(g, ntot, cmk(0, 0), st));
  HIPCHK(c, vcopy(rhs, res, ntot, st));
  std::vector<int> it(nq, 0), done(nq, 0), jend(nq, 0), live(nq, 0);
  std::vector<double> est(nq, 1.0);
  std::vector<std::vector<zc>> Hm(nq), cs(nq), sn(nq), gv(nq);
  for (int q = 0; q < nq; ++q) {
    Hm[q].assign((size_t)(R + 1) * R, zc(0, 0));
    cs[q].assign(R, zc(0, 0));
    sn[q].assign(R, zc(0, 0));
    gv[q].assign(R + 1, zc(0, 0));
    if (bnorm[q] == 0.0) done[q] = 1;  // g = 0 is exact
  }
  while (true) {
    // true residual norms; a problem at tolerance or at maxit is done
    HIPCHK(c, multi_dot(res, 0, 1, res, n, part, nrm2, false, st, nq, HS));
    s = fetch();
    if (s != HPS_OK) return s;
    int active = 0;
    for (int q = 0; q < nq; ++q) {
      if (bnorm[q] == 0.0) continue;
      const double beta = std::sqrt(std::max(host[q * HS + 2 * (R + 2)].x, 0.0));
      info[q].relres_true = beta / bnorm[q];
      if (info[q].relres_true <= tol || it[q] >= maxit) done[q] = 1;
      live[q] = !done[q];
      jend[q] = 0;
      if (live[q]) {
        ++active;
        std::fill(gv[q].begin(), gv[q].end(), zc(0, 0));
        gv[q][0] = beta;
      }
    }
    if (active == 0) break;
    HIPCHK(c, normalize(res, nrm2, V, n, nullptr, st, nq, HS, 0));
    if (graphed) HIPCHK(c, counter_set(jctr, 0, st));
    // Iteration j on the device: V-cycle, M_1 product, CGS2, V_{j+1}, and its
    // Hessenberg column copied to host buffer j % 2.  The next iteration needs
    // nothing from the host, so it is enqueued before the host waits for this
    // one's column (its writes to hh follow the copy in stream order), unless
    // the convergence rate so far predicts that this one reaches the tolerance;
    // a column computed past the stopping point is simply not used.
    auto enqueue = [&](int j) -> hps_status {
      if (graphed) {
        // the iteration graph (the device index equals j: set to 0 above,
        // advanced once per iteration in stream order)
        if (p->igraph) {
          HIPCHK(c, hipGraphLaunch(p->igraph, st));
        } else {
          hps_status e = iteration_kernels(p);
          if (e != HPS_OK) return e;
          HIPCHK(c, hipStreamSynchronize(st));
          capture_iteration(p);
          if (!p->igraph) graphed = false;  // later iterations of this cycle use the eager path
        }
        HIPCHK(c, hipMemcpyAsync(hbuf + (size_t)(j & 1) * hn, hh, sizeof(cd) * hn, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipEventRecord(c->hev[j & 1], st));
        return HPS_OK;
      }
      hps_status e = precond_any(p, V + (size_t)j * ntot, Z + (size_t)j * ntot);
      if (e != HPS_OK) return e;
      HIPCHK(c, skeleton_apply(g1, T1, Z + (size_t)j * ntot, w, true, st, nq));
      e = cgs2_normalize(p, V, ntot, j + 1, w, n, hcol, h2, nrm2, V + (size_t)(j + 1) * ntot, hnorm, HS);
      if (e != HPS_OK) return e;
      HIPCHK(c, hipMemcpyAsync(hbuf + (size_t)(j & 1) * hn, hh, sizeof(cd) * hn, hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipEventRecord(c->hev[j & 1], st));
      return HPS_OK;
    };
    std::vector<double> prev(nq, 1.0);
    int enq = 0;  // iterations of this cycle enqueued
    for (int j = 0; j < R; ++j) {
      if (enq == j) {
        s = enqueue(j);
        if (s != HPS_OK) return s;
        ++enq;
      }
      bool likely_last = false;
      for (int q = 0; q < nq; ++q) {
        if (!live[q] || j == 0) continue;
        const double rate = std::min(1.0, est[q] / std::max(prev[q], 1e-300));
        if (est[q] * rate <= 2.0 * tol || it[q] + 1 >= maxit) likely_last = true;
      }
      if (!likely_last && j + 1 < R) {
        s = enqueue(j + 1);
        if (s != HPS_OK) return s;
        ++enq;
      }
      HIPCHK(c, hipEventSynchronize(c->hev[j & 1]));
      int still = 0;
      for (int q = 0; q < nq; ++q) {
        if (!live[q]) continue;
        prev[q] = est[q];
        const cd* hq = hbuf + (size_t)(j & 1) * hn + (size_t)q * HS;
        zc* col = &Hm[q][(size_t)j * (R + 1)];
        for (int i = 0; i <= j; ++i) col[i] = zc(hq[i].x + hq[R + 2 + i].x, hq[i].y + hq[R + 2 + i].y);
        col[j + 1] = zc(hq[2 * (R + 2) + 1].x, 0.0);
        for (int i = 0; i < j; ++i) {  // G_i = [[conj c, conj s], [-s, c]]
          const zc t = std::conj(cs[q][i]) * col[i] + std::conj(sn[q][i]) * col[i + 1];
          col[i + 1] = -sn[q][i] * col[i] + cs[q][i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
        cs[q][j] = den > 0 ? col[j] / den : zc(1, 0);
        sn[q][j] = den > 0 ? col[j + 1] / den : zc(0, 0);
        col[j] = den;
        col[j + 1] = 0;
        gv[q][j + 1] = -sn[q][j] * gv[q][j];
        gv[q][j] = std::conj(cs[q][j]) * gv[q][j];
        ++it[q];
        jend[q] = j + 1;
        est[q] = std::abs(gv[q][j + 1]) / bnorm[q];
        if (est[q] <= tol || it[q] >= maxit) live[q] = 0;
        else ++still;
      }
      if (still == 0) break;
    }
    // g += Z y per problem (y zero beyond a problem's own Krylov dimension)
    int jmax = 0;
    for (int q = 0; q < nq; ++q) jmax = std::max(jmax, jend[q]);
    std::vector<cd> yd((size_t)nq * R, cmk(0, 0));
    for (int q = 0; q < nq; ++q) {
      const int je = jend[q];
      std::vector<zc> yv(je);
      for (int i = je - 1; i >= 0; --i) {
        zc acc = gv[q][i];
        for (int k = i + 1; k < je; ++k) acc -= Hm[q][(size_t)k * (R + 1) + i] * yv[k];
        yv[i] = acc / Hm[q][(size_t)i * (R + 1) + i];
      }
      for (int i = 0; i < je; ++i) yd[(size_t)q * R + i] = cmk(yv[i].real(), yv[i].imag());
    }
    HIPCHK(c, hipMemcpyAsync(ysol, yd.data(), sizeof(cd) * yd.size(), hipMemcpyHostToDevice, st));
    HIPCHK(c, multi_axpy(Z, ntot, jmax, ysol, g, n, +1, st, nq, R));
    HIPCHK(c, hipStreamSynchronize(st));  // yd must outlive the copy
    // true residual
    HIPCHK(c, skeleton_apply(g1, T1, g, w, true, st, nq));
    HIPCHK(c, axpby(cmk(1, 0), rhs, cmk(-1, 0), w, res, ntot, st));
  }
  for (int q = 0; q < nq; ++q) {
    info[q].iterations = it[q];
    info[q].relres_est = bnorm[q] == 0.0 ? 0.0 : est[q];
    info[q].status = (info[q].relres_true <= tol) ? HPS_OK : HPS_NOT_CONVERGED;
  }
  return HPS_OK;
}

}  // namespace

namespace {

hps_status group_create(hps_ctx* ctx, const hps_desc* desc, int count, const double* kappa, const double* eta,
                        void* workspace, size_t bytes, hps_problem** out) {
  if (!ctx || !out) return HPS_ERR_ARG;
  if (const char* m = check_desc(desc)) return fail(ctx, HPS_ERR_ARG, m);
  if (count < 1 || count > kMaxGroup) return fail(ctx, HPS_ERR_ARG, "group size out of range");
  for (int q = 0; q < count; ++q)
    if (!(std::isfinite(kappa[q]) && kappa[q] > 0 && std::isfinite(eta[q]) && eta[q] > 0))
      return fail(ctx, HPS_ERR_ARG, "kappa and eta must be finite and > 0");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(ctx, HPS_ERR_ARG, "workspace must be a non-null 256-byte aligned device pointer");
  Layout lay = make_layout(desc, count);
  if (bytes < lay.total)
    return fail(ctx, HPS_ERR_OOM, "workspace too small: need " + std::to_string(lay.total) + " bytes");
  hps_problem* p = new hps_problem;
  p->ctx = ctx;
  p->desc = *desc;
  p->kappa.assign(kappa, kappa + count);
  p->eta.assign(eta, eta + count);
  p->lay = lay;
  p->ws = reinterpret_cast<char*>(workspace);
  p->state = kCreated;
  p->merged = 0;
  p->have_T1 = false;
  p->pivot_level.assign(lay.L + 2, 0);
  for (hipEvent_t* ev : {&p->ev_build0, &p->ev_build1, &p->ev_solve0, &p->ev_solve1}) {
    const hipError_t e = hipEventCreate(ev);
    if (e != hipSuccess) {
      hps_problem_destroy(p);
      return fail(ctx, HPS_ERR_HIP, std::string("HIP error: ") + hipGetErrorString(e) + " at hipEventCreate");
    }
  }
  // small tables: GLL data, merge maps, slot tables (with each problem's offset
  // into the group vectors), coarse index list, constants
  GllTables t = gll_tables(desc->order);
  std::vector<double> tab;
  tab.insert(tab.end(), t.D.begin(), t.D.end());
  tab.insert(tab.end(), t.w.begin(), t.w.end());
  tab.insert(tab.end(), t.Kr.begin(), t.Kr.end());
  HIPCHK(ctx, hipMemcpyAsync(p->ws + lay.tables_off, tab.data(), sizeof(double) * tab.size(),
                             hipMemcpyHostToDevice, ctx->stream));
  auto replicate = [&](const std::vector<int>& one) {
    std::vector<int> all;
    all.reserve(one.size() * count);
    for (int q = 0; q < count; ++q)
      for (int v : one) all.push_back(v < 0 ? -1 : (int)(v + (long long)q * lay.nslots));
    return all;
  };
  // all uploads are ordered on the context's stream (after whatever last used
  // this memory); the host copies stay alive until the synchronisation below
  std::vector<std::vector<int>> keep;
  auto upload = [&](size_t off, std::vector<int> v) -> hipError_t {
    keep.push_back(std::move(v));
    const std::vector<int>& h = keep.back();
    return hipMemcpyAsync(p->ws + off, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, ctx->stream);
  };
  for (int l = 1; l <= lay.L; ++l) {
    const Level& lv = lay.lev[l];
    if (!lv.has_merge) continue;
    std::vector<int> xt, yt, dt;
    pair_tables(lv, xt, yt, dt);
    HIPCHK(ctx, upload(lv.map_off, merge_map(lv)));
    HIPCHK(ctx, upload(lv.xtab_off, replicate(xt)));
    HIPCHK(ctx, upload(lv.ytab_off, replicate(yt)));
    HIPCHK(ctx, upload(lv.dtab_off, replicate(dt)));
  }
  if (!lay.exact && lay.nL > 0) HIPCHK(ctx, upload(lay.cidx_off, replicate(coarse_slots(lay.lev[lay.L]))));
  if (lay.fuse) {
    FusedTables ft = fused_tables(lay);
    auto copies = [&](const std::vector<int>& one) {   // local indices: the same for every problem
      std::vector<int> all;
      all.reserve(one.size() * count);
      for (int q = 0; q < count; ++q) all.insert(all.end(), one.begin(), one.end());
      return all;
    };
    HIPCHK(ctx, upload(lay.fgd_off, replicate(ft.gdown)));
    HIPCHK(ctx, upload(lay.fgu_off, replicate(ft.gup)));
    for (int l = 1; l <= lay.fuse; ++l) {
      HIPCHK(ctx, upload(lay.lev[l].xl_off, copies(ft.xl[l])));
      HIPCHK(ctx, upload(lay.lev[l].dl_off, copies(ft.dl[l])));
      HIPCHK(ctx, upload(lay.lev[l].yl_off, copies(ft.yl[l])));
    }
  }
  const cd one = cmk(1, 0);
  HIPCHK(ctx, hipMemcpyAsync(p->ws + lay.one_off, &one, sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
  // error words: no flags, no first failure (records keep a minimum)
  const int words[kFlagWords] = {0, 0, -1, -1, -1, -1, 0x7FFFFFFF, 0};
  HIPCHK(ctx, hipMemcpyAsync(p->ws + lay.flag_off, words, sizeof(words), hipMemcpyHostToDevice, ctx->stream));
  // Box maps of merged levels: entries on physical sides are never computed;
  // they are kept at zero so that products with zero data stay zero.
  for (int l = 2; l <= lay.L; ++l) {
    const Level& lv = lay.lev[l];
    const long long nmap = (long long)count * lv.g.nboxes * lv.g.b * lv.g.b;
    HIPCHK(ctx, vfill(Tlev(p, l), lv.f32 ? (nmap + 1) / 2 : nmap, cmk(0, 0), ctx->stream));
    if (lay.mixed && l == lay.L - 2 && l >= 2)
      HIPCHK(ctx, vfill(at<cd>(p, lay.stage_off), (nmap + 1) / 2, cmk(0, 0), ctx->stream));
  }
  // Columns of X = A^-1 B on physical sides are likewise never computed.
  for (int l = 1; l < lay.L; ++l) {
    const Level& lv = lay.lev[l];
    const long long nx = (long long)count * lv.pairs * 4 * lv.m * lv.e;
    HIPCHK(ctx, vfill(at<cd>(p, lv.X_off), lv.f32 ? (nx + 1) / 2 : nx, cmk(0, 0), ctx->stream));
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->problems.push_back(p);
  *out = p;
  return HPS_OK;
}

// Visits the problems behind `count` handles in order: f(handle, member q,
// index of that problem in the caller's per-problem arrays).
template <class F>
hps_status for_each_problem(hps_problem* const* pp, int count, F f) {
  int base = 0;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    if (!p) return HPS_ERR_ARG;
    for (int q = 0; q < p->lay.nq; ++q) {
      hps_status s = f(p, q, base + q);
      if (s != HPS_OK) return s;
    }
    base += p->lay.nq;
  }
  return HPS_OK;
}

}  // namespace

// Context access for the library's other sources.
void hps_ctx_set_error(hps_ctx* ctx, const char* msg) {
  if (ctx) ctx->err = msg;
}
void* hps_ctx_stream(hps_ctx* ctx) { return ctx ? static_cast<void*>(ctx->stream) : nullptr; }

// ============================ C ABI ========================================
extern "C" {

hps_status hps_ctx_create(void* hip_stream, hps_ctx** out) {
  if (!out) return HPS_ERR_ARG;
  hps_ctx* c = new hps_ctx;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  *out = c;
  return HPS_OK;
}

namespace {
void drop_timed(hps_ctx* ctx) {
  for (TimedLaunch& t : ctx->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  ctx->timed.clear();
}
}  // namespace

hps_status hps_ctx_destroy(hps_ctx* ctx) {
  if (ctx) {
    for (hps_problem* p : ctx->problems) p->ctx = nullptr;
    (void)hipStreamSynchronize(ctx->stream);
    drop_timed(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
    for (int i = 0; i < 2; ++i)
      if (ctx->hev[i]) (void)hipEventDestroy(ctx->hev[i]);
  }
  delete ctx;
  return HPS_OK;
}

hps_status hps_kernel_time(hps_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms, int64_t* units) {
  if (!ctx || !launches || !total_ms || !units) return HPS_ERR_ARG;
  if (kernel != HPS_KERNEL_LEAF) return fail(ctx, HPS_ERR_ARG, "unknown kernel id");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *launches = 0;
  *total_ms = 0;
  *units = 0;
  for (const TimedLaunch& t : ctx->timed) {
    if (t.kernel != kernel) continue;
    float ms = 0;
    HIPCHK(ctx, hipEventElapsedTime(&ms, t.start, t.stop));
    *launches += 1;
    *total_ms += ms;
    *units += t.units;
  }
  return HPS_OK;
}

hps_status hps_set_option(hps_ctx* ctx, int32_t option, int32_t value) {
  if (!ctx) return HPS_ERR_ARG;
  if (option == HPS_OPT_GRAPHS) {
    ctx->use_graphs = value ? 1 : 0;
    return HPS_OK;
  }
  if (option == HPS_OPT_TIMING) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    drop_timed(ctx);
    ctx->timing = value ? 1 : 0;
    return HPS_OK;
  }
  return fail(ctx, HPS_ERR_ARG, "unknown option");
}

const char* hps_last_error(const hps_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hps_status hps_sync(hps_ctx* ctx) {
  if (!ctx) return HPS_ERR_ARG;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (hps_problem* p : ctx->problems) {
    hps_status s = p->state >= kLeaves ? stabilize_merges(p) : HPS_OK;
    if (s == HPS_OK) s = read_flag(p);
    if (s != HPS_OK) return s;
  }
  return HPS_OK;
}

hps_status hps_workspace_bytes(const hps_desc* desc, size_t* bytes) {
  if (!bytes || check_desc(desc)) return HPS_ERR_ARG;
  *bytes = make_layout(desc, 1).total;
  return HPS_OK;
}

hps_status hps_choose_levels(const hps_desc* desc, int32_t count, size_t budget, int32_t* levels) {
  if (!levels || check_desc(desc) || count < 1 || count > kMaxGroup) return HPS_ERR_ARG;
  hps_desc d = *desc;
  const int Lmax = ilog2(d.n) + ilog2(desc_ny(&d));
  // the exact coarse solve exists only at the top level
  const int lo = d.coarse_iters == -1 ? Lmax : 1;
  for (int L = Lmax; L >= lo; --L) {
    d.levels = L;
    if (make_layout(&d, count).total <= budget) {
      *levels = L;
      return HPS_OK;
    }
  }
  return HPS_ERR_OOM;
}

hps_status hps_group_workspace_bytes(const hps_desc* desc, int32_t count, size_t* bytes) {
  if (!bytes || check_desc(desc) || count < 1 || count > kMaxGroup) return HPS_ERR_ARG;
  *bytes = make_layout(desc, count).total;
  return HPS_OK;
}

hps_status hps_gll_nodes(int32_t order, double* xi) {
  if (order < 1 || order > 64 || !xi) return HPS_ERR_ARG;
  GllTables t = gll_tables(order);
  std::memcpy(xi, t.xi.data(), sizeof(double) * (order + 1));
  return HPS_OK;
}

hps_status hps_node_coords(const hps_desc* desc, double* x, double* y) {
  if (check_desc(desc) || !x || !y) return HPS_ERR_ARG;
  const int nx = desc->n, ny = desc_ny(desc), N = desc->order, N1 = N + 1;
  const double h = element_size(nx, ny);
  GllTables t = gll_tables(N);
  for (int e = 0; e < nx * ny; ++e) {
    const int ix = e % nx, iy = e / nx;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N; ++j) {
        const size_t q = (size_t)e * N1 * N1 + i * N1 + j;
        x[q] = ix * h + (1.0 + t.xi[i]) * h / 2;
        y[q] = iy * h + (1.0 + t.xi[j]) * h / 2;
      }
  }
  return HPS_OK;
}

hps_status hps_slot_coords(const hps_desc* desc, double* x, double* y, double* nx, double* ny) {
  if (check_desc(desc) || !x || !y || !nx || !ny) return HPS_ERR_ARG;
  const int mx = desc->n, my = desc_ny(desc), N = desc->order, p = N - 1;
  const double h = element_size(mx, my);
  GllTables t = gll_tables(N);
  const double nrm[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
  for (int e = 0; e < mx * my; ++e) {
    const int ix = e % mx, iy = e / mx;
    for (int s = 0; s < 4; ++s)
      for (int k = 0; k < p; ++k) {
        const size_t q = ((size_t)e * 4 + s) * p + k;
        const double along = (1.0 + t.xi[k + 1]) * h / 2;
        double xx, yy;
        if (s == 0) { xx = ix * h; yy = iy * h + along; }
        else if (s == 1) { xx = (ix + 1) * h; yy = iy * h + along; }
        else if (s == 2) { xx = ix * h + along; yy = iy * h; }
        else { xx = ix * h + along; yy = (iy + 1) * h; }
        x[q] = xx;
        y[q] = yy;
        nx[q] = nrm[s][0];
        ny[q] = nrm[s][1];
      }
  }
  return HPS_OK;
}

hps_status hps_problem_create(hps_ctx* ctx, const hps_desc* desc, void* workspace, size_t bytes,
                              hps_problem** out) {
  if (!desc) return HPS_ERR_ARG;
  return group_create(ctx, desc, 1, &desc->kappa, &desc->eta, workspace, bytes, out);
}

hps_status hps_group_create(hps_ctx* ctx, const hps_desc* desc, int32_t count, const double* kappa,
                            const double* eta, void* workspace, size_t bytes, hps_problem** out) {
  if (!desc || !kappa || !eta) return HPS_ERR_ARG;
  return group_create(ctx, desc, count, kappa, eta, workspace, bytes, out);
}

int32_t hps_group_size(const hps_problem* p) { return p ? p->lay.nq : 0; }

hps_status hps_problem_destroy(hps_problem* p) {
  if (!p) return HPS_OK;
  if (p->pgraph) (void)hipGraphExecDestroy(p->pgraph);
  if (p->igraph) (void)hipGraphExecDestroy(p->igraph);
  for (hipEvent_t ev : {p->ev_build0, p->ev_build1, p->ev_solve0, p->ev_solve1})
    if (ev) (void)hipEventDestroy(ev);
  if (p->ctx) {
    std::vector<hps_problem*>& v = p->ctx->problems;
    v.erase(std::remove(v.begin(), v.end(), p), v.end());
  }
  delete p;
  return HPS_OK;
}

hps_status hps_member_level_view(const hps_problem* pc, int32_t member, int32_t level, hps_level_view* out) {
  hps_problem* p = const_cast<hps_problem*>(pc);
  if (!p || !out || level < 1 || level > p->lay.L || member < 0 || member >= p->lay.nq) return HPS_ERR_ARG;
  const Level& lv = p->lay.lev[level];
  const bool f32 = lv.f32;
  const size_t es = f32 ? sizeof(cf) : sizeof(cd);
  const size_t q = (size_t)member;
  out->level = level;
  out->boxes = lv.g.nboxes;
  out->box_nodes = lv.g.b;
  out->morton = 1;
  const size_t nmap = (size_t)lv.g.nboxes * lv.g.b * lv.g.b;
  if (level == 1 && f32) out->T = p->ws + lv.T32_off + q * nmap * sizeof(cf);
  else out->T = p->ws + lv.T_off + q * nmap * (level == 1 ? sizeof(cd) : es);
  out->fp32 = f32 ? 1 : 0;
  out->pairs = lv.has_merge ? lv.pairs : 0;
  out->shared_nodes = lv.has_merge ? lv.m : 0;
  out->Ainv = lv.has_merge ? (const void*)(p->ws + lv.Ainv_off + q * lv.pairs * 4 * lv.m * lv.m * es) : nullptr;
  out->X = (lv.has_merge && lv.X_off) ? (const void*)(p->ws + lv.X_off + q * lv.pairs * 4 * lv.m * lv.e * es)
                                      : nullptr;
  return HPS_OK;
}

hps_status hps_level_view_get(const hps_problem* pc, int32_t level, hps_level_view* out) {
  return hps_member_level_view(pc, 0, level, out);
}

hps_status hps_build_leaves(hps_problem* const* pp, int32_t count, const double* const* b_nodes,
                            const double* const* s_nodes) {
  if (!pp || count <= 0 || !b_nodes) return HPS_ERR_ARG;
  int base = 0;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    if (!p) return HPS_ERR_ARG;
    const Layout& lay = p->lay;
    for (int q = 0; q < lay.nq; ++q)
      if (!b_nodes[base + q]) return fail(p->ctx, HPS_ERR_ARG, "null b_nodes");
    const int N1 = lay.N + 1;
    LeafArgs a{};
    a.nx = lay.nx;
    a.ny = lay.ny;
    a.ax = ilog2(lay.nx);
    a.ay = ilog2(lay.ny);
    a.N = lay.N;
    a.E = lay.E;
    a.h = element_size(lay.nx, lay.ny);
    const double* tab = at<double>(p, lay.tables_off);
    a.D = tab;
    a.w = tab + N1 * N1;
    a.Kr = tab + N1 * N1 + N1;
    a.scratch = at<double>(p, lay.scratch_off);
    a.T = Tlev(p, 1);
    a.H = at<cd>(p, lay.H_off);
    a.flag = at<int>(p, lay.flag_off);
    a.fb_list = at<int>(p, lay.fb_off);
    HIPCHK(p->ctx, hipEventRecord(p->ev_build0, p->ctx->stream));
    HIPCHK(p->ctx, flag_reset(a.flag, p->ctx->stream));   // a new build: earlier failures are gone
    const long long Gtot = (long long)lay.E * lay.nq;
    for (long long G0 = 0; G0 < Gtot;) {
      // one launch: at most leaf_chunk elements of at most kLeafMaxQ problems
      const int q0 = (int)(G0 / lay.E);
      const long long lim = std::min<long long>(Gtot, (long long)(q0 + kLeafMaxQ) * lay.E);
      const int cnt = (int)std::min<long long>(lay.leaf_chunk, lim - G0);
      a.G0 = (int)G0;
      a.count = cnt;
      a.q0 = q0;
      for (int u = 0; u < kLeafMaxQ; ++u) {
        const int q = q0 + u;
        const bool ok = q < lay.nq;
        a.b_nodes[u] = ok ? b_nodes[base + q] : nullptr;
        a.s_nodes[u] = ok && s_nodes ? s_nodes[base + q] : nullptr;
        a.kappa[u] = ok ? p->kappa[q] : 1.0;
        a.eta[u] = ok ? p->eta[q] : 1.0;
      }
      TimedLaunch tl{};
      if (p->ctx->timing) {
        HIPCHK(p->ctx, hipEventCreate(&tl.start));
        HIPCHK(p->ctx, hipEventCreate(&tl.stop));
        tl.kernel = HPS_KERNEL_LEAF;
        tl.units = cnt;
        HIPCHK(p->ctx, hipEventRecord(tl.start, p->ctx->stream));
      }
      HIPCHK(p->ctx, leaf_build(a, p->ctx->stream));
      if (p->ctx->timing) {
        HIPCHK(p->ctx, hipEventRecord(tl.stop, p->ctx->stream));
        p->ctx->timed.push_back(tl);
      }
      G0 += cnt;
    }
    if (lay.lev[1].f32) {
      // FP64 leaf maps serve the outer operator M_1; the FP32 copy feeds the
      // FP32 merges and the FP32 levels of the V-cycle
      const Level& l1 = lay.lev[1];
      HIPCHK(p->ctx, convert_c64_c32(Tlev(p, 1), at<cf>(p, l1.T32_off),
                                     (long long)lay.nq * l1.g.nboxes * l1.g.b * l1.g.b, p->ctx->stream));
    }
    HIPCHK(p->ctx, hipEventRecord(p->ev_build1, p->ctx->stream));
    p->state = kLeaves;
    p->merged = 0;
    base += lay.nq;
  }
  return HPS_OK;
}

hps_status hps_merge_level(hps_problem* const* pp, int32_t count, int32_t level) {
  if (!pp || count <= 0) return HPS_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    if (!p) return HPS_ERR_ARG;
    if (p->state < kLeaves) return fail(p->ctx, HPS_ERR_STATE, "merge before build_leaves");
    const int Lm = p->lay.exact ? p->lay.L : p->lay.L - 1;
    if (level < 1 || level > Lm) return fail(p->ctx, HPS_ERR_ARG, "merge level out of range");
    if (level != p->merged + 1) return fail(p->ctx, HPS_ERR_STATE, "merge levels must run in order");
    hps_status s = merge_one(p, level);
    if (s != HPS_OK) return s;
    HIPCHK(p->ctx, hipEventRecord(p->ev_build1, p->ctx->stream));
    p->merged = level;
  }
  return HPS_OK;
}

hps_status hps_set_rhs(hps_problem* const* pp, int32_t count, const double* const* t, double* const* rhs) {
  if (!pp || count <= 0 || !t || !rhs) return HPS_ERR_ARG;
  return for_each_problem(pp, count, [&](hps_problem* p, int q, int k) -> hps_status {
    hps_status s = check_ready(p, false);
    if (s != HPS_OK) return s;
    if (!t[k] || !rhs[k]) return fail(p->ctx, HPS_ERR_ARG, "null t or rhs");
    const Layout& lay = p->lay;
    const Geom& g1 = lay.lev[1].g;
    const size_t m = (size_t)4 * lay.p;
    HIPCHK(p->ctx, rhs_build(g1, Tlev(p, 1) + (size_t)q * lay.E * m * m, at<cd>(p, lay.H_off) + (size_t)q * lay.E * m,
                             reinterpret_cast<const cd*>(t[k]), reinterpret_cast<cd*>(rhs[k]), p->ctx->stream));
    return HPS_OK;
  });
}

hps_status hps_skeleton_apply(hps_problem* const* pp, int32_t count, int32_t level, const double* const* g,
                              double* const* out) {
  if (!pp || count <= 0 || !g || !out) return HPS_ERR_ARG;
  return for_each_problem(pp, count, [&](hps_problem* p, int q, int k) -> hps_status {
    hps_status s = check_ready(p, false);
    if (s != HPS_OK) return s;
    if (level < 1 || level > p->lay.L) return fail(p->ctx, HPS_ERR_ARG, "level out of range");
    if (level > p->merged + 1) return fail(p->ctx, HPS_ERR_STATE, "level maps not built yet");
    if (!g[k] || !out[k]) return fail(p->ctx, HPS_ERR_ARG, "null vector");
    const Level& lv = p->lay.lev[level];
    const Geom& gl = lv.g;
    const size_t moff = (size_t)q * gl.nboxes * gl.b * gl.b;
    if (level > 1 && lv.f32)
      HIPCHK(p->ctx, skeleton_apply(gl, at<cf>(p, lv.T_off) + moff, reinterpret_cast<const cd*>(g[k]),
                                    reinterpret_cast<cd*>(out[k]), false, p->ctx->stream));
    else
      HIPCHK(p->ctx, skeleton_apply(gl, Tlev(p, level) + moff, reinterpret_cast<const cd*>(g[k]),
                                    reinterpret_cast<cd*>(out[k]), level == 1, p->ctx->stream));
    return HPS_OK;
  });
}

hps_status hps_precond_apply(hps_problem* const* pp, int32_t count, const double* const* r, double* const* z) {
  if (!pp || count <= 0 || !r || !z) return HPS_ERR_ARG;
  int base = 0;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    hps_status s = check_ready(p, true);
    if (s != HPS_OK) return s;
    s = stabilize_merges(p);
    if (s != HPS_OK) return s;
    const long long n = p->lay.nslots;
    const int nq = p->lay.nq;
    for (int q = 0; q < nq; ++q)
      if (!r[base + q] || !z[base + q]) return fail(p->ctx, HPS_ERR_ARG, "null vector");
    if (nq == 1) {
      s = precond_any(p, reinterpret_cast<const cd*>(r[base]), reinterpret_cast<cd*>(z[base]));
    } else {
      cd* rg = workv(p, 7);
      cd* zg = workv(p, 8);
      for (int q = 0; q < nq; ++q)
        HIPCHK(p->ctx, vcopy(reinterpret_cast<const cd*>(r[base + q]), rg + q * n, n, p->ctx->stream));
      s = precond_any(p, rg, zg);
      for (int q = 0; s == HPS_OK && q < nq; ++q)
        HIPCHK(p->ctx, vcopy(zg + q * n, reinterpret_cast<cd*>(z[base + q]), n, p->ctx->stream));
    }
    if (s != HPS_OK) return s;
    base += nq;
  }
  return HPS_OK;
}

hps_status hps_recover_field(hps_problem* const* pp, int32_t count, const double* const* b_nodes,
                             const double* const* s_nodes, const double* const* t, const double* const* g,
                             double* const* u) {
  if (!pp || count <= 0 || !b_nodes || !t || !g || !u) return HPS_ERR_ARG;
  int base = 0;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    hps_status s = check_ready(p, false);
    if (s != HPS_OK) return s;
    const Layout& lay = p->lay;
    for (int q = 0; q < lay.nq; ++q)
      if (!b_nodes[base + q] || !t[base + q] || !g[base + q] || !u[base + q])
        return fail(p->ctx, HPS_ERR_ARG, "null b_nodes, t, g or u");
    const int N = lay.N, N1 = N + 1;
    FieldArgs a{};
    a.nx = lay.nx;
    a.ny = lay.ny;
    a.N = N;
    a.E = lay.E;
    a.h = element_size(lay.nx, lay.ny);
    const double* tab = at<double>(p, lay.tables_off);
    a.D = tab;
    a.w = tab + N1 * N1;
    a.Kr = tab + N1 * N1 + N1;
    a.scratch = at<double>(p, lay.scratch_off);
    a.flag = at<int>(p, lay.flag_off);
    // Lagrange weights of the degree-(N-2) polynomial through the inner GLL
    // nodes, evaluated at -1 and +1 (the corner extrapolation)
    const GllTables gt = gll_tables(N);
    for (int k = 1; k < N; ++k) {
      double wl = 1.0, wr = 1.0;
      for (int j = 1; j < N; ++j) {
        if (j == k) continue;
        wl *= (-1.0 - gt.xi[j]) / (gt.xi[k] - gt.xi[j]);
        wr *= (1.0 - gt.xi[j]) / (gt.xi[k] - gt.xi[j]);
      }
      a.xl[k - 1] = wl;
      a.xr[k - 1] = wr;
    }
    const int per = (int)std::min<size_t>(1024, lay.scratch_bytes / (sizeof(double) * field_scratch_doubles(N, 1)));
    if (per < 1) return fail(p->ctx, HPS_ERR_OOM, "workspace scratch too small for the field recovery");
    for (int q0 = 0; q0 < lay.nq; q0 += kFieldMaxQ) {
      const int nq = std::min(kFieldMaxQ, lay.nq - q0);
      for (int k = 0; k < nq; ++k) {
        const int qq = base + q0 + k;
        a.b_nodes[k] = b_nodes[qq];
        a.s_nodes[k] = s_nodes ? s_nodes[qq] : nullptr;
        a.t[k] = reinterpret_cast<const cd*>(t[qq]);
        a.g[k] = reinterpret_cast<const cd*>(g[qq]);
        a.u[k] = reinterpret_cast<cd*>(u[qq]);
        a.kappa[k] = p->kappa[q0 + k];
        a.eta[k] = p->eta[q0 + k];
      }
      a.count = nq * lay.E;
      HIPCHK(p->ctx, field_recover(a, per, p->ctx->stream));
    }
    base += lay.nq;
  }
  return HPS_OK;
}

hps_status hps_gmres_solve(hps_problem* const* pp, int32_t count, const double* const* rhs, double* const* g,
                           double tol, int32_t maxit, hps_info* info) {
  if (!pp || count <= 0 || !rhs || !g || !info || !(tol > 0) || maxit < 0) return HPS_ERR_ARG;
  hps_status worst = HPS_OK;
  int base = 0;
  for (int i = 0; i < count; ++i) {
    hps_problem* p = pp[i];
    hps_status s = check_ready(p, true);
    if (s != HPS_OK) return s;
    const long long n = p->lay.nslots;
    const int nq = p->lay.nq;
    for (int q = 0; q < nq; ++q)
      if (!rhs[base + q] || !g[base + q]) return fail(p->ctx, HPS_ERR_ARG, "null vector");
    // a failure recorded by the build (zero pivot, non-finite input) ends the
    // call before any iteration
    s = stabilize_merges(p);
    if (s != HPS_OK) return s;
    s = read_flag(p, base);
    if (s != HPS_OK) return s;
    HIPCHK(p->ctx, hipEventRecord(p->ev_solve0, p->ctx->stream));
    if (nq == 1) {
      s = fgmres_group(p, reinterpret_cast<const cd*>(rhs[base]), reinterpret_cast<cd*>(g[base]), tol, maxit,
                       &info[base]);
    } else {
      cd* rg = workv(p, 7);
      cd* gg = workv(p, 8);
      for (int q = 0; q < nq; ++q)
        HIPCHK(p->ctx, vcopy(reinterpret_cast<const cd*>(rhs[base + q]), rg + q * n, n, p->ctx->stream));
      s = fgmres_group(p, rg, gg, tol, maxit, &info[base]);
      for (int q = 0; s == HPS_OK && q < nq; ++q)
        HIPCHK(p->ctx, vcopy(gg + q * n, reinterpret_cast<cd*>(g[base + q]), n, p->ctx->stream));
    }
    if (s != HPS_OK) return s;
    HIPCHK(p->ctx, hipEventRecord(p->ev_solve1, p->ctx->stream));
    s = read_flag(p, base);
    if (s != HPS_OK) return s;
    float tb = 0.0f, ts = 0.0f;
    HIPCHK(p->ctx, hipEventElapsedTime(&tb, p->ev_build0, p->ev_build1));
    HIPCHK(p->ctx, hipEventElapsedTime(&ts, p->ev_solve0, p->ev_solve1));
    for (int q = 0; q < nq; ++q) {
      info[base + q].t_build_s = 1e-3 * tb;
      info[base + q].t_solve_s = 1e-3 * ts;
      if (info[base + q].status == HPS_NOT_CONVERGED) worst = HPS_NOT_CONVERGED;
    }
    base += nq;
  }
  return worst;
}

}  // extern "C"
