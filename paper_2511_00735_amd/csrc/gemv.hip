// Streaming kernels of the multigrid V-cycle (Sec. 4.3): batched split-K complex
// GEMVs with the gathers from / scatters to the canonical skeleton vector fused
// into their load and store paths, and one-workgroup-per-pair kernels that run a
// whole level of the V-cycle for levels with many small pairs.
//
// All of this is HBM-bound: every stored operator is read once per application,
// 16 bytes per complex entry, with column-major tiles read 64 rows at a time so
// that a wavefront loads 1 KB contiguous per column.
#include "common.h"
#include "gemv.h"

namespace hps {

namespace {

constexpr int kRowsT = 64;   // rows per tile (one per lane)
constexpr int kThreads = 256;

__device__ inline cd load_x(const VecIn& x, int b, int k) {
  if (x.ps) {
    const cd* pp = x.ps + (long long)b * x.pM + x.proff + k;
    const long long ss = (long long)x.pbatch * x.pM;
    cd s = cmk(0.0, 0.0);
    int q = 0;
    for (; q + 4 <= x.pns; q += 4) {  // four loads in flight, summed in split order
      cd v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = pp[(q + u) * ss];
#pragma unroll
      for (int u = 0; u < 4; ++u) s = cadd(s, v[u]);
    }
    for (; q < x.pns; ++q) s = cadd(s, pp[q * ss]);
    return s;
  }
  if (x.p) return x.p[(long long)b * x.stride + k];
  const int s = x.tab[(long long)b * x.tstride + k];
  return s >= 0 ? x.vec[s] : cmk(0.0, 0.0);
}

__device__ inline void store_y(const VecOut& y, int b, int i, cd v) {
  if (y.y0) v = cfma(y.beta, y.y0[(long long)b * y.y0stride + i], v);
  if (y.p) y.p[(long long)b * y.stride + i] = v;
  if (y.vec) {
    const int s = y.tab[(long long)b * y.tstride + i];
    if (s >= 0) y.vec[s] = y.add ? cadd(y.vec[s], v) : v;
  }
}

// grid: x = row tile * nsplit (flattened), y = batch, z = descriptor.  NT / 64
// waves per workgroup, wave w taking columns k0 + w, k0 + w + NW, ...
template <class Mt, int NT>
__global__ __launch_bounds__(NT) void gemv_kernel(GemvBatchT<Mt> gb, cd* partial) {
  constexpr int NW = NT / 64;
  __shared__ cd xs[kGemvKChunkMax];
  __shared__ cd red[NW][kRowsT];
  const GemvDescT<Mt>& d = gb.d[blockIdx.z];
  const int tiles = (d.M_ + kRowsT - 1) / kRowsT;
  const int nsplit = gb.nsplit[blockIdx.z];
  if ((int)blockIdx.x >= tiles * nsplit) return;
  const int tile = blockIdx.x % tiles, split = blockIdx.x / tiles;
  const int b = blockIdx.y;
  const int kc = (d.K + nsplit - 1) / nsplit;
  const int k0 = split * kc;
  const int k1 = min(d.K, k0 + kc);
  const int t = threadIdx.x, lane = t & 63, grp = t >> 6;
  const int r = tile * kRowsT + lane;
  const bool rok = r < d.M_ && k0 < k1;
  const Mt* Ab = d.A.base + (long long)b * d.A.bstride;
  const long long row = imap(d.A.r, r < d.M_ ? r : 0);
  // The first U entries of the thread are requested before x is staged (two
  // dependent loads through the slot table), clamped into the operator; the
  // barrier keeps them in flight together.
  constexpr int U = 8;  // independent loads in flight per thread
  Mt a0[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a0[u] = cx<Mt>::make(0.0, 0.0);
  if (k0 < k1) {  // uniform over the workgroup
#pragma unroll
    for (int u = 0; u < U; ++u) a0[u] = Ab[(long long)imap_arith(d.A.c, min(k0 + grp + NW * u, k1 - 1)) * d.A.ld + row];
  }
  for (int k = k0 + t; k < k1; k += NT) {
    const cd v = load_x(d.x, b, k);
    xs[k - k0] = v;
    if (d.x.save && tile == 0) d.x.save[(long long)b * d.x.save_stride + d.x.save_off + k] = v;
  }
  __syncthreads();
  cd acc = cmk(0.0, 0.0);
  if (rok) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + grp + NW * u;
      acc = cfma(k < k1 ? to_cd(a0[u]) : cmk(0.0, 0.0), xs[min(k, k1 - 1) - k0], acc);
    }
    int k = k0 + grp + NW * U;
    for (; k + NW * (U - 1) < k1; k += NW * U) {
      Mt a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = Ab[(long long)imap_arith(d.A.c, k + NW * u) * d.A.ld + row];
#pragma unroll
      for (int u = 0; u < U; ++u) acc = cfma(to_cd(a[u]), xs[k + NW * u - k0], acc);
    }
    for (; k < k1; k += NW) acc = cfma(to_cd(Ab[(long long)imap_arith(d.A.c, k) * d.A.ld + row]), xs[k - k0], acc);
  }
  red[grp][lane] = acc;
  __syncthreads();
  if (grp != 0 || r >= d.M_) return;
  cd s = red[0][lane];
#pragma unroll
  for (int w = 1; w < NW; ++w) s = cadd(s, red[w][lane]);
  if (nsplit == 1 && !gb.partials_only)
    store_y(d.y, b, r, cmul(d.alpha, s));
  else
    partial[gb.poff[blockIdx.z] + ((long long)split * gb.batch + b) * d.M_ + r] = s;
}

// Sum the split-K partials in split order (deterministic) and apply the epilogue.
// (A device-scope fence per workgroup to let the last split reduce in place
// forces an L2 write-back on this chip and costs more than this launch.)
template <class Mt>
__global__ void gemv_reduce_kernel(GemvBatchT<Mt> gb, const cd* partial) {
  const GemvDescT<Mt>& d = gb.d[blockIdx.z];
  const int nsplit = gb.nsplit[blockIdx.z];
  if (nsplit == 1) return;
  const int b = blockIdx.y;
  const long long ps = (long long)gb.batch * d.M_;  // between splits
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.M_; r += gridDim.x * blockDim.x) {
    const cd* pp = partial + gb.poff[blockIdx.z] + (long long)b * d.M_ + r;
    cd s = cmk(0.0, 0.0);
    int q = 0;
    for (; q + 8 <= nsplit; q += 8) {  // eight loads in flight, summed in split order
      cd v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(q + u) * ps];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = cadd(s, v[u]);
    }
    for (; q < nsplit; ++q) s = cadd(s, pp[q * ps]);
    store_y(d.y, b, r, cmul(d.alpha, s));
  }
}

// ---- two workgroups per pair: a whole V-cycle level ---------------------------
// Levels with many small pairs are bound by the latency of their dependent
// loads (slot index -> vector value -> product -> scatter), not by bandwidth:
// every workgroup of such a level is resident at once, so the launch lasts as
// long as one workgroup's chain of round trips.  Each half of a pair is
// therefore independent work for its own workgroup, and every load that does
// not depend on a computed value (slot indices, the operator entries of the
// thread, the vector values read through those slots) is issued before the
// first product is formed.

// One GEMV piece of a workgroup, y[i] = (y0 ? y0[i] : 0) + sum_k A(rm(i), cm(k)) x[k]
// for i < M, k < K, with x, y0, y in LDS.  Rows go in tiles of RT = min(M, 64),
// one row per lane; S tiles are in flight per pass, each with G column groups;
// the first CAP columns of a thread in the first pass are prefetched into
// registers by load(), the rest are read in run().
template <class Mt, int NT, int CAP>
struct RegGemv {
  static_assert(CAP % 4 == 0, "prefetch groups of four");
  Mt a[CAP];
  int M, K, RT, S, G, slot, r, g, passes, tid;
  bool act;
  // t: the thread's index among the NT threads that form this product (the
  // workgroup's, or one group's of a workgroup split into equal groups that
  // all run products of one shape, so that they meet the same barriers)
  __device__ void setup(int M_, int K_, int t = threadIdx.x) {
    tid = t;
    M = M_;
    K = K_;
    RT = M < 64 ? M : 64;
    const int tiles = (M + RT - 1) / RT;
    S = min(tiles, NT / RT);
    const int tpt = NT / S;
    G = tpt / RT;
    slot = t / tpt;
    const int u = t - slot * tpt;
    r = u % RT;
    g = u / RT;
    act = slot < S && g < G;
    passes = (tiles + S - 1) / S;
  }
  // Unconditional loads: indices outside the operator are clamped into it, and
  // run() zeroes those entries; a barrier must separate load() from run(), so
  // that the loads stay in flight together instead of sinking to their uses.
  __device__ void load(const Mt* A, int ld, IdxMap rm, IdxMap cm) {
    const int row = slot * RT + r;
    const Mt* Ar = A + imap(rm, act && row < M ? row : 0);
#pragma unroll
    for (int c = 0; c < CAP; ++c) a[c] = Ar[(long long)imap(cm, min(g + c * G, K - 1)) * ld];
  }
  // red: NT entries of LDS.  Ends with the workgroup synchronised.
  __device__ void run(const Mt* A, int ld, IdxMap rm, IdxMap cm, const cd* x, const cd* y0, cd* y, cd* red) {
    for (int ps = 0; ps < passes; ++ps) {
      const int row = (ps * S + slot) * RT + r;
      cd acc = cmk(0.0, 0.0);
      if (act && row < M) {
        int c = 0;
        if (ps == 0) {
          // four entries at a time: the empty asm orders each group after the
          // previous one's products, so that the compiler does not widen every
          // prefetched entry (and read every x) ahead of the first product
#pragma unroll
          for (int q0 = 0; q0 < CAP; q0 += 4) {
            int col[4];
            Mt w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              col[q] = g + (q0 + q) * G;
              w[q] = a[q0 + q];
            }
            asm volatile("" : "+v"(acc.x), "+v"(acc.y), "+v"(col[0]), "+v"(col[1]), "+v"(col[2]), "+v"(col[3]),
                         "+v"(w[0].x), "+v"(w[0].y), "+v"(w[1].x), "+v"(w[1].y), "+v"(w[2].x), "+v"(w[2].y),
                         "+v"(w[3].x), "+v"(w[3].y));
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc = cfma(col[q] < K ? to_cd(w[q]) : cmk(0.0, 0.0), x[min(col[q], K - 1)], acc);
          }
          c = CAP;
        }
        const long long ar = imap(rm, row);
#ifndef HPS_SMALL_U
#define HPS_SMALL_U 8
#endif
        constexpr int U = sizeof(Mt) == sizeof(cd) ? 4 : HPS_SMALL_U;  // independent loads in flight per thread
#pragma unroll 1
        for (; g + (c + U - 1) * G < K; c += U) {
          Mt v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) v[u] = A[(long long)imap(cm, g + (c + u) * G) * ld + ar];
#pragma unroll
          for (int u = 0; u < U; ++u) acc = cfma(to_cd(v[u]), x[g + (c + u) * G], acc);
        }
#pragma unroll 1
        for (; g + c * G < K; ++c) acc = cfma(to_cd(A[(long long)imap(cm, g + c * G) * ld + ar]), x[g + c * G], acc);
      }
      if (act) red[(slot * G + g) * RT + r] = acc;
      __syncthreads();
      for (int q = tid; q < S * RT; q += NT) {
        const int sl = q / RT, rr = q - sl * RT;
        const int i = (ps * S + sl) * RT + rr;
        if (i < M) {
          cd sum = y0 ? y0[i] : cmk(0.0, 0.0);
          for (int gg = 0; gg < G; ++gg) sum = cadd(sum, red[(sl * G + gg) * RT + rr]);
          y[i] = sum;
        }
      }
      __syncthreads();
    }
  }
};

// Register budgets (entries per thread prefetched per operator).
template <class Mt> struct SmallCap { static constexpr int A = 8, T = 12, X = 16; };
template <> struct SmallCap<cd> { static constexpr int A = 4, T = 8, X = 12; };

// The map i -> m(i + r0).
__device__ inline IdxMap im_shift(IdxMap m, int r0) {
  if (m.map) {
    m.map += r0;
  } else {
    m.off += r0;
    m.gap_start -= r0;
  }
  return m;
}

// Down sweep, half h of pair j, row piece pc of P (workgroup (2j + h) P + pc;
// levels with few pairs split each half's T rows over P workgroups, each of
// which forms the whole z0 half again).  x = [Q.beta; P.alpha]:
// h = 0 forms z0_P = rows [m, 2m) of A^-1 r_x and adds T^P_{E1,a} z0_P to the
// slots across P's kept faces; h = 1 forms z0_Q = rows [0, m) and adds
// T^Q_{E2,b} z0_Q across Q's.  The two halves touch disjoint slots, and no
// other pair of the level reads or writes those slots.
template <class Mt, int NT>
__global__ __launch_bounds__(NT) void vc_down_small_kernel(SmallLevelT<Mt> a, cd* vec, int P) {
  extern __shared__ cd sm[];
  const int m = a.m, e = a.e, m2 = 2 * m;
  const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
  const int jh = bid / P, pc = bid - jh * P;
  const int j = jh >> 1, h = jh & 1, t = threadIdx.x;
  const int R = (e + P - 1) / P, r0 = pc * R, Me = min(R, e - r0);   // this piece's T rows
  if (Me <= 0) return;   // uniform over the workgroup
  cd* r = sm;             // [2m] r_x
  cd* z = r + m2;         // [m]  z0 half
  cd* dv = z + m;         // [e]  vector values across the faces
  cd* dd = dv + e;        // [e]  T z0 half
  cd* red = dd + e;       // [NT]
  int* ds = reinterpret_cast<int*>(red + NT);  // [e] slots across the faces
  const long long bb = (long long)a.g.b * a.g.b;
  const int xi = t < m2 ? a.xtab[(long long)j * m2 + t] : -1;
  const int di = t < Me ? a.dtab[(long long)j * 2 * e + h * e + r0 + t] : -1;
  RegGemv<Mt, NT, SmallCap<Mt>::A> ga;
  RegGemv<Mt, NT, SmallCap<Mt>::T> gt;
  ga.setup(m, m2);
  gt.setup(Me, m);
  const Mt* Ai = a.Ainv + (long long)j * m2 * m2;
  const IdxMap arow = im_off(h == 0 ? m : 0);
  const Mt* Th = a.T + (2LL * j + h) * bb;
  const IdxMap trow = im_shift(h == 0 ? a.E1 : a.E2, r0);
  const IdxMap tcol = im_off(h == 0 ? a.a0 : a.b0);
  ga.load(Ai, m2, arow, im_off(0));
  gt.load(Th, a.g.b, trow, tcol);
  if (t < m2) r[t] = vec[xi];
  if (t < Me) {
    ds[t] = di;
    dv[t] = di >= 0 ? vec[di] : cmk(0.0, 0.0);
  }
  __syncthreads();
  ga.run(Ai, m2, arow, im_off(0), r, nullptr, z, red);
  if (pc == 0 && t < m) a.Z0[(long long)j * m2 + (h == 0 ? m : 0) + t] = z[t];
  gt.run(Th, a.g.b, trow, tcol, z, dv, dd, red);
  if (t < Me && ds[t] >= 0) vec[ds[t]] = dd[t];
}

// Up sweep, piece p of pair j (workgroup P j + p): rows [p R, p R + M) of
// x = z0 + X y (R = ceil(2m / P), M = min(R, 2m - p R)), y the kept-face
// values of z, written into z at the shared-face slots.  The rows are
// independent, so levels with few pairs split them over many workgroups,
// each of which forms complete rows (no partial sums to reduce).
template <class Mt, int NT>
__global__ __launch_bounds__(NT) void vc_up_small_kernel(SmallLevelT<Mt> a, cd* z, int P) {
  extern __shared__ cd sm[];
  const int m = a.m, e = a.e, m2 = 2 * m, e2 = 2 * e;
  const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
  const int j = bid / P, pc = bid - j * P, t = threadIdx.x;
  const int R = (m2 + P - 1) / P, r0 = pc * R, M = min(R, m2 - r0);
  if (M <= 0) return;   // uniform over the workgroup
  cd* y = sm;          // [2e]
  cd* z0 = y + e2;     // [R]
  cd* x = z0 + R;      // [R]
  cd* red = x + R;     // [NT]
  constexpr int kY = 4;   // y entries gathered per thread with their loads in flight together
  int yi[kY];
#pragma unroll
  for (int u = 0; u < kY; ++u) yi[u] = t + u * NT < e2 ? a.ytab[(long long)j * e2 + t + u * NT] : -1;
  const int xi = t < M ? a.xtab[(long long)j * m2 + r0 + t] : -1;
  const cd zv = t < M ? a.Z0[(long long)j * m2 + r0 + t] : cmk(0.0, 0.0);
  RegGemv<Mt, NT, SmallCap<Mt>::X> gx;
  gx.setup(M, e2);
  const Mt* Xj = a.X + (long long)j * m2 * e2;
  const IdxMap xrow = im_off(r0);
  gx.load(Xj, m2, xrow, im_off(0));
#pragma unroll
  for (int u = 0; u < kY; ++u)
    if (t + u * NT < e2) y[t + u * NT] = yi[u] >= 0 ? z[yi[u]] : cmk(0.0, 0.0);
  for (int i = t + kY * NT; i < e2; i += NT) {
    const int s = a.ytab[(long long)j * e2 + i];
    y[i] = s >= 0 ? z[s] : cmk(0.0, 0.0);
  }
  if (t < M) z0[t] = zv;
  __syncthreads();
  gx.run(Xj, m2, xrow, im_off(0), y, z0, x, red);
  if (t < M) z[xi] = x[t];
}


// ---- levels 1..K in one launch: one workgroup per level-(K+1) box ------------
// Below level K+1 a box's pairs touch only the slots of its own elements and,
// in the down sweep, the slots across its boundary (the rows of the kept faces'
// neighbours), which no other box touches before level K+1.  One workgroup of
// 1024 threads therefore runs all K levels of one box with the box's slot
// values in LDS: the level-l pairs of the box (2^(K-l) of them, consecutive in
// merge-tree order) split the threads into equal groups, so every group runs
// products of one shape and meets the same barriers.  Only the operators and
// z0 go through global memory; the vector is read and written once.
constexpr int kFusedThreads = 1024;

template <class Mt, int NTG>
__device__ void fused_down_level(const FusedLevel& L, int box, int ppb, cd* v, cd* w, int tid) {
  const int m = L.m, e = L.e, m2 = 2 * m;
  const int grp = tid / NTG, t = tid - grp * NTG;
  const int j = box * ppb + (grp >> 1), h = grp & 1;
  const int reg = 3 * m + 2 * e + NTG + (e + 3) / 4;   // one group's LDS, in cd
  cd* r = w + (long long)grp * reg;   // [2m] r_x
  cd* z = r + m2;                      // [m]  z0 half
  cd* dv = z + m;                      // [e]  values across the kept faces
  cd* dd = dv + e;                     // [e]  T z0 half
  cd* red = dd + e;                    // [NTG]
  int* ds = reinterpret_cast<int*>(red + NTG);   // [e]
  const long long bb = (long long)L.b * L.b;
  const Mt* T = static_cast<const Mt*>(L.T);
  const Mt* Ai = static_cast<const Mt*>(L.Ainv) + (long long)j * m2 * m2;
  const IdxMap arow = im_off(h == 0 ? m : 0);
  const Mt* Th = T + (2LL * j + h) * bb;
  const IdxMap trow = h == 0 ? L.E1 : L.E2;
  const IdxMap tcol = im_off(h == 0 ? L.a0 : L.b0);
  RegGemv<Mt, NTG, SmallCap<Mt>::A> ga;
  RegGemv<Mt, NTG, SmallCap<Mt>::T> gt;
  ga.setup(m, m2, t);
  gt.setup(e, m, t);
  ga.load(Ai, m2, arow, im_off(0));
  gt.load(Th, L.b, trow, tcol);
  for (int i = t; i < m2; i += NTG) r[i] = v[L.xl[(long long)j * m2 + i]];
  for (int i = t; i < e; i += NTG) {
    const int di = L.dl[(long long)j * 2 * e + h * e + i];
    ds[i] = di;
    dv[i] = di >= 0 ? v[di] : cmk(0.0, 0.0);
  }
  __syncthreads();
  ga.run(Ai, m2, arow, im_off(0), r, nullptr, z, red);
  for (int i = t; i < m; i += NTG) L.Z0[(long long)j * m2 + (h == 0 ? m : 0) + i] = z[i];
  gt.run(Th, L.b, trow, tcol, z, dv, dd, red);
  for (int i = t; i < e; i += NTG)
    if (ds[i] >= 0) v[ds[i]] = dd[i];
  __syncthreads();
}

template <class Mt, int NTP>
__device__ void fused_up_level(const FusedLevel& L, int box, int ppb, cd* v, cd* w, int tid) {
  const int m2 = 2 * L.m, e2 = 2 * L.e;
  const int grp = tid / NTP, t = tid - grp * NTP;
  const int j = box * ppb + grp;
  const int reg = e2 + 2 * m2 + NTP;
  cd* y = w + (long long)grp * reg;   // [2e]
  cd* z0 = y + e2;                     // [2m]
  cd* x = z0 + m2;                     // [2m]
  cd* red = x + m2;                    // [NTP]
  const Mt* Xj = static_cast<const Mt*>(L.X) + (long long)j * m2 * e2;
  RegGemv<Mt, NTP, SmallCap<Mt>::X> gx;
  gx.setup(m2, e2, t);
  gx.load(Xj, m2, im_off(0), im_off(0));
  for (int i = t; i < e2; i += NTP) {
    const int yi = L.yl[(long long)j * e2 + i];
    y[i] = yi >= 0 ? v[yi] : cmk(0.0, 0.0);
  }
  for (int i = t; i < m2; i += NTP) z0[i] = L.Z0[(long long)j * m2 + i];
  __syncthreads();
  gx.run(Xj, m2, im_off(0), im_off(0), y, z0, x, red);
  for (int i = t; i < m2; i += NTP) v[L.xl[(long long)j * m2 + i]] = x[i];
  __syncthreads();
}

// Level l of K (1-based) of the down sweep: 2^(K-l) pairs per box, a group of
// 512 >> (K - l) threads per pair half.
template <class Mt, int K, int l>
__device__ inline void fused_down_from(const FusedArgs& a, int box, cd* v, cd* w, int tid) {
  if constexpr (l <= K) {
    constexpr int kGroup = (kFusedThreads / 2) >> (K - l);
    fused_down_level<Mt, kGroup>(a.lev[l - 1], box, 1 << (K - l), v, w, tid);
    fused_down_from<Mt, K, l + 1>(a, box, v, w, tid);
  }
}

template <class Mt, int K, int l>
__device__ inline void fused_up_from(const FusedArgs& a, int box, cd* v, cd* w, int tid) {
  if constexpr (l >= 1) {
    constexpr int kGroup = kFusedThreads >> (K - l);
    fused_up_level<Mt, kGroup>(a.lev[l - 1], box, 1 << (K - l), v, w, tid);
    fused_up_from<Mt, K, l - 1>(a, box, v, w, tid);
  }
}

template <class Mt, int K>
__global__ __launch_bounds__(kFusedThreads) void vc_down_fused_kernel(FusedArgs a, cd* vec) {
  extern __shared__ cd sm[];
  const int box = blockIdx.x, tid = threadIdx.x;
  cd* v = sm;
  cd* w = sm + a.nloc_pad;
  const int* gs = a.gdown + (long long)box * a.nloc;
  for (int i = tid; i < a.nloc; i += kFusedThreads) {
    const int s = gs[i];
    v[i] = s >= 0 ? vec[s] : cmk(0.0, 0.0);
  }
  __syncthreads();
  fused_down_from<Mt, K, 1>(a, box, v, w, tid);
  for (int i = tid; i < a.nloc; i += kFusedThreads) {
    const int s = gs[i];
    if (s >= 0) vec[s] = v[i];
  }
}

template <class Mt, int K>
__global__ __launch_bounds__(kFusedThreads) void vc_up_fused_kernel(FusedArgs a, cd* z) {
  extern __shared__ cd sm[];
  const int box = blockIdx.x, tid = threadIdx.x;
  cd* v = sm;
  cd* w = sm + a.nloc_pad;
  const int* gs = a.gup + (long long)box * a.nloc;
  for (int i = tid; i < a.nloc; i += kFusedThreads) v[i] = z[gs[i]];
  __syncthreads();
  fused_up_from<Mt, K, K>(a, box, v, w, tid);
  for (int i = tid; i < a.nloc; i += kFusedThreads) z[gs[i]] = v[i];
}

}  // namespace

namespace {
// Launches of few workgroups (a capped split count) take 16 waves per
// workgroup, so that each thread still has about one batch of loads.
template <class Mt>
hipError_t launch_gemv(const GemvBatchT<Mt>& gb, int gx, int batch, int nd, cd* partial, hipStream_t st) {
  if ((long long)gx * batch * nd < kGemvTargetBlocks / 2)
    hipLaunchKernelGGL((gemv_kernel<Mt, 1024>), dim3(gx, batch, nd), dim3(1024), 0, st, gb, partial);
  else
    hipLaunchKernelGGL((gemv_kernel<Mt, kThreads>), dim3(gx, batch, nd), dim3(kThreads), 0, st, gb, partial);
  return hipPeekAtLastError();
}
}  // namespace

int gemv_nsplit(int M, int K, int batch) {
  const int tiles = (M + kRowsT - 1) / kRowsT;
  int ns = (kGemvTargetBlocks + tiles * batch - 1) / (tiles * batch);
  ns = std::max(1, std::min(ns, (K + 63) / 64));
  while ((K + ns - 1) / ns > kGemvKChunkMax) ++ns;
  return ns;
}

template <class Mt>
hipError_t zgemv_batched(const GemvDescT<Mt>* d, int nd, int batch, cd* partial, hipStream_t st) {
  if (nd <= 0 || nd > kGemvMaxDesc || batch <= 0) return hipErrorInvalidValue;
  for (int i = 0; i < nd; ++i)
    if (d[i].A.c.map) return hipErrorInvalidValue;   // column maps are offsets (imap_arith)
  GemvBatchT<Mt> gb{};
  gb.batch = batch;
  int gx = 0;
  long long poff = 0;
  bool any_split = false;
  for (int i = 0; i < nd; ++i) {
    gb.d[i] = d[i];
    const int tiles = (d[i].M_ + kRowsT - 1) / kRowsT;
    const int ns = gemv_nsplit(d[i].M_, d[i].K, batch);
    gb.nsplit[i] = ns;
    gb.poff[i] = poff;
    if (ns > 1) { poff += (long long)ns * batch * d[i].M_; any_split = true; }
    gx = std::max(gx, tiles * ns);
  }
  if (any_split && !partial) return hipErrorInvalidValue;
  hipError_t err = launch_gemv(gb, gx, batch, nd, partial, st);
  if (err != hipSuccess || !any_split) return err;
  int maxM = 0;
  for (int i = 0; i < nd; ++i) maxM = std::max(maxM, d[i].M_);
  hipLaunchKernelGGL(gemv_reduce_kernel<Mt>, dim3((maxM + 63) / 64, batch, nd), dim3(64), 0, st, gb, partial);
  return hipPeekAtLastError();
}

template <class Mt>
hipError_t zgemv_partials(const GemvDescT<Mt>* d, int nd, int batch, cd* partial, GemvPartLayout* lay,
                          hipStream_t st, int max_split) {
  if (nd <= 0 || nd > kGemvMaxDesc || batch <= 0 || !partial || !lay) return hipErrorInvalidValue;
  for (int i = 0; i < nd; ++i)
    if (d[i].A.c.map) return hipErrorInvalidValue;   // column maps are offsets (imap_arith)
  GemvBatchT<Mt> gb{};
  gb.batch = batch;
  gb.partials_only = 1;
  int gx = 0;
  long long poff = 0;
  for (int i = 0; i < nd; ++i) {
    gb.d[i] = d[i];
    const int tiles = (d[i].M_ + kRowsT - 1) / kRowsT;
    int ns = gemv_nsplit(d[i].M_, d[i].K, batch);
    if (max_split > 0 && ns > max_split && (d[i].K + max_split - 1) / max_split <= kGemvKChunkMax) ns = max_split;
    gb.nsplit[i] = ns;
    gb.poff[i] = poff;
    lay->nsplit[i] = ns;
    lay->poff[i] = poff;
    poff += (long long)ns * batch * d[i].M_;
    gx = std::max(gx, tiles * ns);
  }
  return launch_gemv(gb, gx, batch, nd, partial, st);
}

namespace {

// Threads per workgroup: at least one per slot index, and otherwise as many
// as let the level's 2 x pairs workgroups be resident together (about
// kSmallResident threads on the chip at these kernels' register use), but no
// more than one per kSmallMinEntries operator entries.
#ifndef HPS_SMALL_RESIDENT
#define HPS_SMALL_RESIDENT 262144
#endif
#ifndef HPS_SMALL_MIN_ENTRIES
#define HPS_SMALL_MIN_ENTRIES 4
#endif
constexpr long long kSmallResident = HPS_SMALL_RESIDENT;
constexpr long long kSmallMinEntries = HPS_SMALL_MIN_ENTRIES;
int small_threads(long long entries, int need, int pairs) {
  int nt = 64;
  while (nt < 1024 && 2LL * pairs * (2 * nt) <= kSmallResident && 2 * nt * kSmallMinEntries <= entries) nt *= 2;
  while (nt < need) nt *= 2;
  return nt;
}
size_t small_down_lds(int m, int e, int nt) { return sizeof(cd) * (size_t)(3 * m + 2 * e + nt) + sizeof(int) * e; }
// up-sweep LDS for pieces of R rows: y [2e], z0 and x [R], red [nt]
size_t small_up_lds(int R, int e, int nt) { return sizeof(cd) * (size_t)(2 * e + 2 * R + nt); }
#ifndef HPS_SMALL_UP_WGS
#define HPS_SMALL_UP_WGS 256
#endif
constexpr long long kSmallUpWGs = HPS_SMALL_UP_WGS;
#ifndef HPS_SMALL_UP_ROWS
#define HPS_SMALL_UP_ROWS 4
#endif
constexpr int kSmallUpRows = HPS_SMALL_UP_ROWS;

// Row pieces per pair for the up sweep: at least two, more while the level has
// fewer than kSmallUpWGs workgroups and a piece keeps at least kSmallUpRows rows.
int up_pieces(int m, int pairs) {
  int P = 2;
  while ((long long)P * pairs < kSmallUpWGs && 2 * m >= 2 * P * kSmallUpRows) P *= 2;
  return P;
}

// T-row pieces per pair half for the down sweep: more while the level has
// fewer than kSmallDownWGs workgroups and a piece keeps at least 64 rows.
#ifndef HPS_SMALL_DOWN_WGS
#define HPS_SMALL_DOWN_WGS 256
#endif
int down_pieces(int e, int pairs) {
  int P = 1;
  while (2LL * P * pairs < HPS_SMALL_DOWN_WGS && e >= 2 * P * 64 && P < 4) P *= 2;
  return P;
}

template <class Mt, int NT>
hipError_t launch_down(const SmallLevelT<Mt>& a, int pairs, cd* vec, hipStream_t st) {
  const size_t lds = small_down_lds(a.m, a.e, NT);
  hipError_t err = allow_lds(vc_down_small_kernel<Mt, NT>, lds);
  if (err != hipSuccess) return err;
  const int P = down_pieces(a.e, pairs);
  hipLaunchKernelGGL((vc_down_small_kernel<Mt, NT>), dim3(2 * pairs * P), dim3(NT), lds, st, a, vec, P);
  return hipPeekAtLastError();
}

template <class Mt, int NT>
hipError_t launch_up(const SmallLevelT<Mt>& a, int pairs, int P, cd* z, hipStream_t st) {
  const size_t lds = small_up_lds((2 * a.m + P - 1) / P, a.e, NT);
  hipError_t err = allow_lds(vc_up_small_kernel<Mt, NT>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((vc_up_small_kernel<Mt, NT>), dim3(P * pairs), dim3(NT), lds, st, a, z, P);
  return hipPeekAtLastError();
}

}  // namespace

#ifndef HPS_SMALL_MIN_PAIRS
#define HPS_SMALL_MIN_PAIRS 32
#endif
bool vc_up_small_ok(int m, int e, int pairs) {
  if (pairs < 1 || m < 1 || e < 1) return false;
  const int P = up_pieces(m, pairs), R = (2 * m + P - 1) / P;
  return R <= 1024 && small_up_lds(R, e, 1024) <= 64 * 1024;
}

bool vc_small_ok(int m, int e, int pairs) {
  return pairs >= HPS_SMALL_MIN_PAIRS && m >= 1 && e >= 1 && 2 * m <= 1024 && 2 * e <= 1024 &&
         small_down_lds(m, e, 1024) <= 64 * 1024;
}

template <class Mt>
hipError_t vc_down_small(const SmallLevelT<Mt>& a, int pairs, cd* vec, hipStream_t st) {
  if (!vc_small_ok(a.m, a.e, pairs)) return hipErrorInvalidValue;
  const int m = a.m, e = a.e;
  switch (small_threads(2LL * m * m + (long long)e * m, std::max(2 * m, e), pairs)) {
    case 64: return launch_down<Mt, 64>(a, pairs, vec, st);
    case 128: return launch_down<Mt, 128>(a, pairs, vec, st);
    case 256: return launch_down<Mt, 256>(a, pairs, vec, st);
    case 512: return launch_down<Mt, 512>(a, pairs, vec, st);
    default: return launch_down<Mt, 1024>(a, pairs, vec, st);
  }
}

template <class Mt>
hipError_t vc_up_small(const SmallLevelT<Mt>& a, int pairs, cd* z, hipStream_t st) {
  if (!vc_up_small_ok(a.m, a.e, pairs)) return hipErrorInvalidValue;
  const int m = a.m, e = a.e;
  const int P = up_pieces(m, pairs);
  const int R = (2 * m + P - 1) / P;
  switch (small_threads((long long)R * 2 * e, std::max(std::min(2 * e, 1024), R), pairs * P / 2)) {
    case 64: return launch_up<Mt, 64>(a, pairs, P, z, st);
    case 128: return launch_up<Mt, 128>(a, pairs, P, z, st);
    case 256: return launch_up<Mt, 256>(a, pairs, P, z, st);
    case 512: return launch_up<Mt, 512>(a, pairs, P, z, st);
    default: return launch_up<Mt, 1024>(a, pairs, P, z, st);
  }
}

size_t fused_lds_bytes(const FusedArgs& a, int K, bool down) {
  size_t need = 0;
  for (int l = 1; l <= K; ++l) {
    const FusedLevel& L = a.lev[l - 1];
    size_t groups, reg;
    if (down) {
      const int ntg = (kFusedThreads / 2) >> (K - l);
      groups = (size_t)2 << (K - l);
      reg = 3 * L.m + 2 * L.e + ntg + (L.e + 3) / 4;
    } else {
      const int ntp = kFusedThreads >> (K - l);
      groups = (size_t)1 << (K - l);
      reg = 2 * L.e + 4 * L.m + ntp;
    }
    need = std::max(need, groups * reg);
  }
  return sizeof(cd) * ((size_t)a.nloc_pad + need);
}

bool fused_ok(const FusedArgs& a, int K) {
  if (K < 2 || K > kFuseMax) return false;
  for (int l = 1; l <= K; ++l) {
    const FusedLevel& L = a.lev[l - 1];
    if (L.m < 1 || L.e < 1 || 2 * L.m > 1024 || 2 * L.e > 4096) return false;
  }
  return fused_lds_bytes(a, K, true) <= 160 * 1024 && fused_lds_bytes(a, K, false) <= 160 * 1024;
}

namespace {
template <class Mt, int K>
hipError_t launch_fused(const FusedArgs& a, int boxes, cd* vec, bool down, hipStream_t st) {
  const size_t lds = fused_lds_bytes(a, K, down);
  if (down) {
    hipError_t err = allow_lds(vc_down_fused_kernel<Mt, K>, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((vc_down_fused_kernel<Mt, K>), dim3(boxes), dim3(kFusedThreads), lds, st, a, vec);
  } else {
    hipError_t err = allow_lds(vc_up_fused_kernel<Mt, K>, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((vc_up_fused_kernel<Mt, K>), dim3(boxes), dim3(kFusedThreads), lds, st, a, vec);
  }
  return hipPeekAtLastError();
}
}  // namespace

template <class Mt>
hipError_t vc_fused(const FusedArgs& a, int K, int boxes, cd* vec, bool down, hipStream_t st) {
  if (!fused_ok(a, K) || boxes < 1) return hipErrorInvalidValue;
  switch (K) {
    case 2: return launch_fused<Mt, 2>(a, boxes, vec, down, st);
    case 3: return launch_fused<Mt, 3>(a, boxes, vec, down, st);
    default: return launch_fused<Mt, 4>(a, boxes, vec, down, st);
  }
}

template hipError_t vc_fused<cd>(const FusedArgs&, int, int, cd*, bool, hipStream_t);
template hipError_t vc_fused<cf>(const FusedArgs&, int, int, cd*, bool, hipStream_t);
template hipError_t zgemv_batched<cd>(const GemvDescT<cd>*, int, int, cd*, hipStream_t);
template hipError_t zgemv_batched<cf>(const GemvDescT<cf>*, int, int, cd*, hipStream_t);
template hipError_t zgemv_partials<cd>(const GemvDescT<cd>*, int, int, cd*, GemvPartLayout*, hipStream_t, int);
template hipError_t zgemv_partials<cf>(const GemvDescT<cf>*, int, int, cd*, GemvPartLayout*, hipStream_t, int);
template hipError_t vc_down_small<cd>(const SmallLevelT<cd>&, int, cd*, hipStream_t);
template hipError_t vc_down_small<cf>(const SmallLevelT<cf>&, int, cd*, hipStream_t);
template hipError_t vc_up_small<cd>(const SmallLevelT<cd>&, int, cd*, hipStream_t);
template hipError_t vc_up_small<cf>(const SmallLevelT<cf>&, int, cd*, hipStream_t);

}  // namespace hps
