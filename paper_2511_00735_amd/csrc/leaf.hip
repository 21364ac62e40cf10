// Leaf impedance-to-impedance maps (Sec. 3.1, eq. ItIOperator), one workgroup
// per element, one launch per chunk of elements.
//
// With the element unknowns split into interior nodes (i) and boundary nodes
// (G), the element matrix L of Sec. 3.1 is [[N_GG + i eta I, N_Gi], [L_iG, L_ii]]
// where N_G are the normal-derivative rows and L_ii, L_iG the interior rows of
// the real symmetric local operator.  Eliminating the interior gives
//     T = I_o L^-1 I(:, G) = (i eta I - R)(R + i eta I)^-1 = -I + 2 i eta (R + i eta I)^-1,
//     R = N_GG - N_Gi L_ii^-1 L_iG          (real, 4p x 4p),
//     H = -(T + I) N_Gi L_ii^-1 bt = 2 i eta (R + i eta I)^-1 (-q),  q = N_Gi L_ii^-1 bt.
// The expensive part is therefore a REAL Schur complement: the bordered real
// matrix K = [[L_ii, L_iG, bt], [N_Gi, N_GG, 0]] is reduced by partial LU over
// its first p^2 pivots (pivot search restricted to the L_ii rows), which leaves
// [R | -q] in its trailing rows.  Only the 4p x 4p complex Cayley step remains.
// This is the same T as the paper's complex n_loc x n_loc solve, computed with
// about 1/7 of its flops and in real arithmetic.
//
// The reduction is a right-looking blocked LU with panels of kNB columns:
//  * K is never assembled in memory: the first panel, its U12 rows and its
//    trailing update evaluate K's entries (a few dozen nonzeros per row) from
//    their definition, and that first trailing update is the matrix's first
//    write to global memory;
//  * the panel (all remaining rows x kNB columns) sits in registers, each wave
//    holding every fourth column; pivot rows are left where they are during
//    the panel and only marked as used, so a column step needs one barrier:
//    the wave holding the next column publishes it in LDS with its pivot key
//    (64-bit modulus/row keys, DPP arg-max across the wavefront), and every
//    wave reads the pivot row of its own columns by lane broadcasts;
//  * multipliers stay unscaled in the panel, with 1/pivot kept per column;
//    once the panel is done they are scaled into the panel's own (finished)
//    columns of the element matrix, and the LDS is handed to U12 and L11;
//  * the row interchanges are applied once per panel (chunk by chunk, below):
//    the pivot rows of the trailing columns are gathered into U12, and the
//    non-pivot rows among the first kNB move into the slots the pivot rows
//    vacate;
//  * the trailing columns are taken in chunks whose U12 rows fit the LDS
//    (at most 208 columns): per chunk the row interchanges, U12 = L11^-1 A12
//    by per-column forward substitution in LDS, then the trailing update
//    A22 -= L21 U12 with one row and four adjacent columns per thread (U12
//    read as 128-bit broadcasts, L21 rows from the element matrix, three
//    column groups of A22 in flight per lane).
// With 24-column panels and chunks of at most 208 columns the LDS holds about
// 48 KB at N = 16, so three workgroups share a CU (their 164 registers per
// lane allow three waves per SIMD); the trailing matrix is read and written
// once per 24 pivots.  Measured per 4096-element launch at N = 16: 7.44 ms,
// against 7.86 ms with 20-column panels (one chunk) and 7.5-7.7 ms with 24 and
// 28 columns in chunks of 144 or 176 columns.  The same update on the FP64
// matrix cores (16x16x4 tiles of A22^T -= U12^T L21^T, L21 held per row
// block) measured 10.8 ms at 20 columns: the tiles' registers leave no room
// at three workgroups per CU for loads in flight ahead of the products, and
// the FP64 matrix rate of this part equals its vector rate.
#include <algorithm>

#include "common.h"
#include "host.h"
#include "pivot.h"

namespace hps {

namespace {

#ifndef HPS_LEAF_NB
#define HPS_LEAF_NB 24
#endif
constexpr int kNB = HPS_LEAF_NB;  // panel width of the blocked LU (a multiple of 4)
static_assert(kNB % 4 == 0, "panel columns are dealt to four waves and updated four at a time");
#ifndef HPS_LEAF_OCC
#define HPS_LEAF_OCC 3            // workgroups per CU the register budget is set for
#endif
#ifndef HPS_LEAF_PF
#define HPS_LEAF_PF 3
#endif
constexpr int kPF = HPS_LEAF_PF;  // trailing-update column groups in flight per lane
#ifndef HPS_LEAF_ADD_B
#define HPS_LEAF_ADD_B 16
#endif
constexpr int kAddB = HPS_LEAF_ADD_B;  // K entries added per thread with their loads in flight together
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kCPW = kNB / kWaves;  // panel columns per wave
constexpr int kMaxChunks = 5;    // 64-row chunks of a panel: n_loc <= 320 (N <= 16)
#ifndef HPS_LEAF_CW
#define HPS_LEAF_CW 208
#endif
constexpr int kCWMax = HPS_LEAF_CW;  // trailing columns whose U12 rows share the LDS at a time
static_assert(kCWMax % 4 == 0, "trailing columns are updated four at a time");
// An element whose interior elimination meets a pivot below 0.02 times its
// largest (in modulus) lies within about 1e-6 (relative, in kappa^2) of an
// interior Dirichlet eigenvalue; rounding in the large term of its Schur
// complement would then reach 1e-11 of T, so it is recomputed by the complex
// elimination of the whole element system (no resonance: the impedance
// problem is well posed).  Away from resonances the ratio stays near 0.05-0.3.
constexpr float kNearSingular2 = 0.02f * 0.02f;
constexpr int kFbBlocks = 32;    // workgroups of the fallback launch

struct Dims {
  int N, p, pp, nloc, ncol, ldu;
};

__host__ __device__ inline Dims dims_of(int N) {
  Dims d;
  d.N = N;
  d.p = N - 1;
  d.pp = d.p * d.p;
  d.nloc = d.pp + 4 * d.p;
  d.ncol = d.nloc + 2;
  // row stride of U12 in LDS, which holds at most kCWMax trailing columns at a
  // time: 2 mod 4, so that the rows of one column fall in different banks
  const int nc0 = d.ncol - (d.pp < kNB ? d.pp : kNB);
  d.ldu = (((nc0 < kCWMax ? nc0 : kCWMax) + 3) & ~3) + 2;
  return d;
}

// doubles of one element's bordered matrix in the scratch buffer (256-byte
// multiple, so every element's matrix starts 256-byte aligned)
__host__ __device__ inline size_t elem_stride(const Dims& d) {
  return ((size_t)d.nloc * d.ncol + 31) & ~(size_t)31;
}

// Entry (r, c) of the bordered real matrix K of one element, evaluated from its
// definition: rows/cols interior (i,j) -> (i-1)*p + (j-1); boundary l_k, r_k,
// b_k, t_k -> pp + side*p + (k-1); extra columns nloc, nloc+1 = Re/Im of bt.
// An interior row couples to the 2p-1 interior nodes on its grid lines, four
// boundary nodes and the two source columns; a normal-derivative row to p
// interior and two boundary nodes.  The first panel of the partial LU reads K
// this way, so the matrix is never stored before its first trailing update.
struct ElemK {
  int N, p, pp, nloc;
  const double* D;      // (N+1)^2 reference differentiation matrix
  const double* w;      // N+1 GLL weights
  const double* Kr;     // (N+1)^2 reference stiffness
  const double* bnode;  // (N+1)^2 coefficient b at the element's nodes
  const double* snode;  // complex (N+1)^2 source at the nodes, or null
  double kappa, h;

  __device__ double operator()(int r, int c) const {
    const int N1 = N + 1;
    if (r < pp) {
      const int i = r / p + 1, j = r - (i - 1) * p + 1;
      if (c >= nloc) {
        if (!snode) return 0.0;
        return 0.25 * h * h * w[i] * w[j] * snode[2 * (i * N1 + j) + (c - nloc)];
      }
      if (c < pp) {
        const int i2 = c / p + 1, j2 = c - (i2 - 1) * p + 1;
        double v = 0.0;
        if (j == j2) v += Kr[i * N1 + i2] * w[j];
        if (i == i2) v += w[i] * Kr[j * N1 + j2];
        if (i == i2 && j == j2) v -= 0.25 * h * h * kappa * kappa * (1.0 - bnode[i * N1 + j]) * w[i] * w[j];
        return v;
      }
      const int s = (c - pp) / p, k = c - pp - s * p + 1;
      if (s == 0) return (j == k) ? Kr[i * N1 + 0] * w[j] : 0.0;
      if (s == 1) return (j == k) ? Kr[i * N1 + N] * w[j] : 0.0;
      if (s == 2) return (i == k) ? w[i] * Kr[j * N1 + 0] : 0.0;
      return (i == k) ? w[i] * Kr[j * N1 + N] : 0.0;
    }
    if (c >= nloc) return 0.0;
    // normal-derivative row of boundary node (side s, index k)
    const int s = (r - pp) / p, k = r - pp - s * p + 1;
    const bool lo = (s == 0 || s == 2);
    const double sg = lo ? -2.0 / h : 2.0 / h;  // outward normal sign
    const int dr = lo ? 0 : N;                   // D row of the boundary node
    if (c < pp) {
      const int i2 = c / p + 1, j2 = c - (i2 - 1) * p + 1;
      if (s < 2) return (j2 == k) ? sg * D[dr * N1 + i2] : 0.0;   // x-derivative along line j = k
      return (i2 == k) ? sg * D[dr * N1 + j2] : 0.0;              // y-derivative along line i = k
    }
    const int s2 = (c - pp) / p, k2 = c - pp - s2 * p + 1;
    if (k2 != k) return 0.0;
    if (s < 2) return s2 == 0 ? sg * D[dr * N1 + 0] : (s2 == 1 ? sg * D[dr * N1 + N] : 0.0);
    return s2 == 2 ? sg * D[dr * N1 + 0] : (s2 == 3 ? sg * D[dr * N1 + N] : 0.0);
  }

  // The nonzeros of K one by one: it < items() enumerates (row, slot) pairs,
  // 2p+5 slots per interior row (its x-line with the diagonal, its y-line, four
  // boundary nodes, two source columns) and p+2 per boundary row, slot-major.  False for a
  // slot that holds no entry (the source columns without a source).
  __device__ int items() const { return pp * (2 * p + 5) + 4 * p * (p + 2); }
  __device__ bool item(int it, int& r, int& c, double& v) const {
    const int N1 = N + 1, si = 2 * p + 5;
    const double hh = 0.25 * h * h;
    if (it < pp * si) {
      // rows fastest: the lanes of a wave take one slot kind of consecutive
      // rows, so that y-line, top/bottom-node and source entries (a single
      // column for a run of rows) are read and written contiguously
      const int s = it / pp;
      r = it - s * pp;
      const int i = r / p + 1, j = r - (i - 1) * p + 1;
      if (s < p) {                       // (i2, j): x-line, diagonal when i2 == i
        const int i2 = s + 1;
        c = s * p + (j - 1);
        v = Kr[i * N1 + i2] * w[j];
        if (i2 == i) v += w[i] * Kr[j * N1 + j] - hh * kappa * kappa * (1.0 - bnode[i * N1 + j]) * w[i] * w[j];
      } else if (s < 2 * p - 1) {        // (i, j2), j2 != j: y-line
        const int jj = s - p + 1;
        const int j2 = jj + (jj >= j ? 1 : 0);
        c = (i - 1) * p + (j2 - 1);
        v = w[i] * Kr[j * N1 + j2];
      } else if (s < 2 * p + 3) {        // boundary nodes l_j, r_j, b_i, t_i
        const int side = s - (2 * p - 1);
        if (side == 0) { c = pp + (j - 1); v = Kr[i * N1 + 0] * w[j]; }
        else if (side == 1) { c = pp + p + (j - 1); v = Kr[i * N1 + N] * w[j]; }
        else if (side == 2) { c = pp + 2 * p + (i - 1); v = w[i] * Kr[j * N1 + 0]; }
        else { c = pp + 3 * p + (i - 1); v = w[i] * Kr[j * N1 + N]; }
      } else {                           // Re / Im of the source term
        if (!snode) return false;
        const int part = s - (2 * p + 3);
        c = nloc + part;
        v = hh * w[i] * w[j] * snode[2 * (i * N1 + j) + part];
      }
      return true;
    }
    const int jt = it - pp * si;
    const int t = jt / (4 * p), rb = jt - t * (4 * p);
    const int side = rb / p, k = rb - side * p + 1;
    r = pp + rb;
    const bool lo = (side == 0 || side == 2);
    const double sg = lo ? -2.0 / h : 2.0 / h;
    const int dr = lo ? 0 : N;
    if (t < p) {
      c = side < 2 ? t * p + (k - 1) : (k - 1) * p + t;
      v = sg * D[dr * N1 + t + 1];
    } else {
      c = pp + ((side < 2 ? 0 : 2) + (t - p)) * p + (k - 1);
      v = sg * D[dr * N1 + (t == p ? 0 : N)];
    }
    return true;
  }
};

// Lane l's double broadcast to the whole wavefront (l uniform).
__device__ inline double readlane_d(double v, int l) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Called by the one wave holding the next panel column (value of row t*64 +
// lane in v[t]): publishes the column, picks its pivot among the unused
// candidate rows and stores the pivot key and 1/pivot.
__device__ inline void publish_pivot(const double (&v)[kMaxChunks], unsigned used, int rows, int cand,
                                     double* cbn, unsigned long long* key_out, double* inv_out) {
  const int lane = threadIdx.x & 63;
  unsigned long long best = 0;
#pragma unroll
  for (int t = 0; t < kMaxChunks; ++t) {
    const int r = t * 64 + lane;
    if (r < rows) cbn[r] = v[t];
    if (r < cand && !((used >> t) & 1u)) best = max(best, pivot_key(fabs(v[t]), r));
  }
  best = wave_max_key(best);
  const int pn = min(max(pivot_row(best), 0), cand - 1);
  double dn = 0.0;
#pragma unroll
  for (int t = 0; t < kMaxChunks; ++t)
    if (t == (pn >> 6)) dn = readlane_d(v[t], pn & 63);
  if (lane == 0) {
    *key_out = best;
    *inv_out = ((best >> 32) <= 1u) ? 0.0 : 1.0 / dn;
  }
}

// Broadcast of lane l's complex value to the whole wavefront (l uniform).
__device__ inline cd readlane_cd(cd v, int l) {
  const long long x = __double_as_longlong(v.x), y = __double_as_longlong(v.y);
  const unsigned x0 = (unsigned)__builtin_amdgcn_readlane((int)x, l);
  const unsigned x1 = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
  const unsigned y0 = (unsigned)__builtin_amdgcn_readlane((int)y, l);
  const unsigned y1 = (unsigned)__builtin_amdgcn_readlane((int)(y >> 32), l);
  return cmk(__longlong_as_double((long long)(((unsigned long long)x1 << 32) | x0)),
             __longlong_as_double((long long)(((unsigned long long)y1 << 32) | y0)));
}

// Called by the one wave holding the next column of the Cayley inverse (row
// lane in v): publishes the column, picks its pivot among the unused rows and
// stores the pivot key and 1/pivot.
__device__ inline void cayley_publish(cd v, bool used, bool row_ok, cd* cbn, unsigned long long* key_out,
                                      cd* inv_out) {
  const int lane = threadIdx.x & 63;
  cbn[lane] = v;
  unsigned long long key = (row_ok && !used) ? pivot_key(cabs2(v), lane) : 0ull;
  key = wave_max_key(key);
  const cd d = readlane_cd(v, pivot_row(key) & 63);
  if (lane == 0) {
    *key_out = key;
    *inv_out = ((key >> 32) <= 1u) ? cmk(0.0, 0.0) : cinv(d);
  }
}

// T = -I + 2 i eta Z and H = 2 i eta Z (-q), Z = (R + i eta I)^-1, from [R | -q]
// in the trailing rows of the reduced bordered matrix A.
//
// Z by Gauss-Jordan with the 4p x 4p complex matrix in registers: thread
// (row i = lane, wave w) holds columns j = w + 4t.  Pivot rows stay where they
// are (marked used); a step reads the pivot row by lane broadcasts, the pivot
// column from LDS (published by the wave holding it, with the next pivot key),
// and needs one barrier.  With pivot row pr_k at step k, the storage ends as
// S[pr_k][j] = Z[k][pr_j].
__device__ void leaf_cayley(const LeafArgs& a, const Dims& d, const double* A, double* lds) {
  constexpr int kT = 16;  // columns per thread (4p <= 64)
  const int m = 4 * d.p, nloc = d.nloc, npiv = d.pp;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_uniform(tid >> 6);
  const int G = a.G0 + blockIdx.x;
  const int q = G / a.E, e = G % a.E;
  const double eta = a.eta[q - a.q0];
  const double* snode = a.s_nodes[q - a.q0];
  cd* colbuf = reinterpret_cast<cd*>(lds);             // [2][64] pivot column
  cd* hpart = colbuf + 128;                            // [kWaves][64] partial H
  cd* pinv = hpart + kWaves * 64;                      // [2] 1 / next pivot
  unsigned long long* kw = reinterpret_cast<unsigned long long*>(pinv + 2);  // [2]
  int* pivs = reinterpret_cast<int*>(kw + 2);          // [64] pivot row of each step
  const bool row_ok = lane < m;
  cd s[kT];
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const int j = wave + kWaves * t;
    s[t] = (row_ok && j < m) ? cmk(A[(size_t)(npiv + j) * nloc + npiv + lane], lane == j ? eta : 0.0)
                             : cmk(0.0, 0.0);
  }
  if (wave == 0) cayley_publish(s[0], false, row_ok, colbuf, kw, pinv);
  __syncthreads();
  bool used = false;
  int myk = 0;
#pragma unroll 1
  for (int k = 0; k < m; ++k) {
    const int b = k & 1;
    const unsigned long long kk = wave_uniform(kw[b]);
    const cd inv = pinv[b];
    const bool zero = (kk >> 32) <= 1u;
    const int pr = min(max(pivot_row(kk), 0), m - 1);
    const bool isp = lane == pr;
    if (isp) { used = true; myk = k; }
    if (tid == 0) {
      pivs[k] = pr;
      if (zero) flag_singular(a.flag, flag_where(0, G));
    }
    const cd f = isp ? cmk(0.0, 0.0) : cmul(colbuf[b * 64 + lane], inv);
    const int tk = k >> 2, ok = k & 3;
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      if (wave + kWaves * t < m) {
        if (wave == ok && t == tk) {
          s[t] = isp ? inv : cmk(-f.x, -f.y);
        } else {
          const cd pv = readlane_cd(s[t], pr);
          s[t] = isp ? cmul(pv, inv) : csub(s[t], cmul(f, pv));
        }
      }
    }
    // the wave holding column k + 1 publishes it with its pivot and 1/pivot
    const int kn = k + 1;
    if (kn < m && wave == (kn & 3)) {
      const int tn = kn >> 2;
      cd vn = cmk(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < kT; ++t)
        if (t == tn) vn = s[t];
      cayley_publish(vn, used, row_ok, colbuf + (kn & 1) * 64, kw + (kn & 1), pinv + (kn & 1));
    }
    __syncthreads();
  }
  const int ix = e % a.nx, iy = e / a.nx;
  cd* Tout = a.T + (a.linear_out ? (size_t)G : ((size_t)q * a.E + tree_code(a.ax, a.ay, ix, iy))) * m * m;
  const double te = 2.0 * eta;
  cd hacc = cmk(0.0, 0.0);
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const int j = wave + kWaves * t;
    if (row_ok && j < m) {
      const int c = pivs[j];
      const cd z = s[t];
      Tout[(size_t)c * m + myk] = cmk(-te * z.y - (myk == c ? 1.0 : 0.0), te * z.x);
      if (snode) {
        const cd tc = cmk(A[(size_t)nloc * nloc + npiv + c], A[(size_t)(nloc + 1) * nloc + npiv + c]);
        hacc = cfma(z, tc, hacc);
      }
    }
  }
  if (row_ok) hpart[wave * 64 + myk] = hacc;
  __syncthreads();
  if (tid < m) {
    cd acc = hpart[tid];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) acc = cadd(acc, hpart[w * 64 + tid]);
    a.H[(size_t)G * m + tid] = cmk(-te * acc.y, te * acc.x);
  }
}

// LDS doubles shared by the panel's pivot-column exchange and U12 + L11
__host__ __device__ inline size_t leaf_region_doubles(const Dims& d) {
  const size_t a = (size_t)2 * 64 * kMaxChunks, b = (size_t)kNB * d.ldu + (size_t)kNB * kNB;
  const size_t c = (size_t)d.nloc * kWaves;   // the first panel's columns of K, kWaves at least at a time
  const size_t ab = a > b ? a : b;
  return ab > c ? ab : c;
}

// LDS bytes: the LU phase (panel, U12, row map) and the Cayley phase
size_t leaf_lds_bytes(int N) {
  const Dims d = dims_of(N);
  const size_t lu = leaf_region_doubles(d) * sizeof(double) + 2 * (size_t)d.nloc * sizeof(int);
  const size_t cay = (size_t)(130 + kWaves * 64) * sizeof(cd) + 2 * sizeof(unsigned long long) + 64 * sizeof(int);
  return std::max(lu, cay);
}

// One element per workgroup: assembly, the bordered real partial LU, then the
// Cayley step.
__global__ __launch_bounds__(kThreads, HPS_LEAF_OCC) void leaf_kernel(LeafArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lds[];
  __shared__ int piv_s[kNB];              // panel-relative pivot row of each column
  __shared__ int dsrc_s[kNB];             // row moved into the slot of pivot piv_s[c], or -1
  __shared__ double dinv_s[kNB];          // 1 / pivot
  __shared__ unsigned long long kw_s[2];  // next pivot key (double buffered)
  __shared__ double pinv_s[2];            // 1 / next pivot
  const Dims d = dims_of(a.N);
  const int nloc = d.nloc, ncol = d.ncol, npiv = d.pp, ldu = d.ldu;
  // LDS region: the pivot-column exchange while a panel is factorised, then
  // U12 and L11
  double* colbuf = lds;                     // [2][64 * kMaxChunks] pivot column
  double* U = lds;                          // U12, kNB x ldu, row-major
  double* L11 = lds + (size_t)kNB * ldu;    // scaled L11, row-major kNB x kNB
  const size_t region = leaf_region_doubles(d);
  int* rowmap = reinterpret_cast<int*>(lds + region);  // trailing slot -> panel row of its L21
  int* slotof = rowmap + nloc;                         // first panel: row of K -> its trailing slot, or -1
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_uniform(tid >> 6);
  const int G = a.G0 + blockIdx.x;
  const int q = G / a.E, e = G % a.E;
  const int N1 = a.N + 1;
  double* A = a.scratch + (size_t)blockIdx.x * elem_stride(d);
  const double* sq = a.s_nodes[q - a.q0];
  const ElemK K{d.N, d.p, d.pp, nloc, a.D, a.w, a.Kr, a.b_nodes[q - a.q0] + (size_t)e * N1 * N1,
                sq ? sq + (size_t)e * 2 * N1 * N1 : nullptr, a.kappa[q - a.q0], a.h};
  // a NaN or Inf among the element's inputs: recorded, and the element is
  // skipped by the whole workgroup (the call then reports HPS_ERR_ARG)
  {
    bool bad = false;
    for (int i = tid; i < N1 * N1; i += kThreads) {
      bad |= !isfinite(K.bnode[i]);
      if (K.snode) bad |= !isfinite(K.snode[2 * i]) || !isfinite(K.snode[2 * i + 1]);
    }
    if (__syncthreads_or(bad)) {
      if (tid == 0) flag_nonfinite(a.flag, G);
      return;
    }
  }
  // smallest and largest squared pivot modulus of the interior elimination
  // (thread 0): their ratio tells an element close to an interior Dirichlet
  // resonance, whose Schur complement loses accuracy
  float p2min = 3.0e38f, p2max = 0.0f;

  for (int k0 = 0; k0 < npiv; k0 += kNB) {
    const int kb = min(kNB, npiv - k0);
    const int rows = nloc - k0;       // panel rows
    const int cand = npiv - k0;       // pivot candidates: the interior rows
    const int c0 = k0 + kb, nc = ncol - c0;
    // the panel in registers: wave w holds columns j = w + kWaves * u, lane the
    // rows t * 64 + lane
    const bool first = k0 == 0;   // the first panel reads K itself
    double xv[kMaxChunks][kCPW];
    if (first) {
      // K's first kb columns, evaluated into the (still free) U12 area as many
      // at a time as it holds (a multiple of kWaves)
#pragma unroll
      for (int u = 0; u < kCPW; ++u)
#pragma unroll
        for (int t = 0; t < kMaxChunks; ++t) xv[t][u] = 0.0;
      const int kst = min(kNB, (int)(region / nloc) / kWaves * kWaves);
      for (int s0 = 0; s0 < kb; s0 += kst) {
        for (int idx = tid; idx < rows * kst; idx += kThreads) {
          const int r = idx % rows, c = s0 + idx / rows;
          if (c < kb) U[(size_t)(c - s0) * nloc + r] = K(r, c);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCPW; ++u) {
          const int j = wave + kWaves * u;
          if (j >= s0 && j < s0 + kst && j < kb) {
            const double* col = U + (size_t)(j - s0) * nloc;
#pragma unroll
            for (int t = 0; t < kMaxChunks; ++t) {
              const int r = t * 64 + lane;
              xv[t][u] = r < rows ? col[r] : 0.0;
            }
          }
        }
        __syncthreads();   // the next batch, or the column exchange below, reuses that LDS
      }
    } else {
#pragma unroll
      for (int u = 0; u < kCPW; ++u) {
        const int j = wave + kWaves * u;
        const double* col = A + (size_t)(k0 + j) * nloc + k0;
#pragma unroll
        for (int t = 0; t < kMaxChunks; ++t) {
          const int r = t * 64 + lane;
          xv[t][u] = (j < kb && r < rows) ? col[r] : 0.0;
        }
      }
    }
    for (int r = tid; r < rows; r += kThreads) {
      rowmap[r] = r;
      slotof[r] = r;
    }
    if (wave == 0) {
      double v0[kMaxChunks];
#pragma unroll
      for (int t = 0; t < kMaxChunks; ++t) v0[t] = xv[t][0];
      publish_pivot(v0, 0u, rows, cand, colbuf, kw_s, pinv_s);
    }
    __syncthreads();

    // ---- panel: one barrier per column ----
    unsigned used = 0;   // bit t: row t*64 + lane is a pivot row of this panel
#pragma unroll 1
    for (int c = 0; c < kb; ++c) {
      const int bsel = c & 1;
      const double* cb = colbuf + bsel * 64 * kMaxChunks;
      const unsigned long long kk = wave_uniform(kw_s[bsel]);
      const double inv = wave_uniform(pinv_s[bsel]);
      const bool zero = (kk >> 32) <= 1u;
      const int pr = min(max(pivot_row(kk), 0), cand - 1);
      const int tp = pr >> 6, lp = pr & 63;
      if (lane == lp) used |= 1u << tp;
      if (tid == 0) {
        piv_s[c] = pr;
        dinv_s[c] = inv;
        const float p2 = zero ? 0.0f : __uint_as_float((unsigned)(kk >> 32) - 1u);
        p2min = fminf(p2min, p2);
        p2max = fmaxf(p2max, p2);
      }
      // the pivot row of this wave's open columns, by lane broadcast (zero for
      // finished columns: their values stay exactly as they are)
      double pv[kCPW];
#pragma unroll
      for (int u = 0; u < kCPW; ++u) pv[u] = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxChunks; ++t) {
        if (t == tp) {
#pragma unroll
          for (int u = 0; u < kCPW; ++u) {
            const int j = wave + kWaves * u;
            if (j > c && j < kb) pv[u] = readlane_d(xv[t][u], lp);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < kMaxChunks; ++t) {
        const int r = t * 64 + lane;
        const bool act = r < rows && !((used >> t) & 1u);
        const double m = act ? cb[r] * inv : 0.0;
#pragma unroll
        for (int u = 0; u < kCPW; ++u) xv[t][u] -= m * pv[u];
      }
      // the wave holding column c + 1 publishes it with its pivot and 1/pivot
      const int cn = c + 1;
      if (cn < kb && wave == (cn & (kWaves - 1))) {
        const int un = cn / kWaves;
        double vn[kMaxChunks];
#pragma unroll
        for (int t = 0; t < kMaxChunks; ++t) vn[t] = 0.0;
#pragma unroll
        for (int u = 0; u < kCPW; ++u)
          if (u == un) {
#pragma unroll
            for (int t = 0; t < kMaxChunks; ++t) vn[t] = xv[t][u];
          }
        publish_pivot(vn, used, rows, cand, colbuf + (bsel ^ 1) * 64 * kMaxChunks, kw_s + (bsel ^ 1),
                      pinv_s + (bsel ^ 1));
      }
      if (c == kb - 1 && wave == 0) {
        // pair the pivot rows beyond the first kb with the non-pivot rows
        // among the first kb: those rows take the pivot rows' slots
        bool isp = false;
        if (lane < kb)
          for (int qq = 0; qq < kb; ++qq) isp |= (piv_s[qq] == lane);
        const unsigned long long nonpiv = __ballot(lane < kb && !isp);
        const int y = lane < kb ? piv_s[lane] : 0;
        const bool far = lane < kb && y >= kb;
        const unsigned long long farm = __ballot(far);
        if (lane < kb) slotof[y] = -1;   // pivot rows leave the trailing block
        if (far) {
          const int rank = __popcll(farm & ((1ull << lane) - 1ull));
          unsigned long long mm = nonpiv;
          for (int k = 0; k < rank; ++k) mm &= mm - 1ull;
          const int x = __ffsll((long long)mm) - 1;
          dsrc_s[lane] = x;
          rowmap[y] = x;
          slotof[x] = y;
        } else if (lane < kb) {
          dsrc_s[lane] = -1;
        }
      }
      __syncthreads();
    }

    // ---- scaled multipliers to the (finished) panel columns of A ----
#pragma unroll
    for (int u = 0; u < kCPW; ++u) {
      const int j = wave + kWaves * u;
      if (j < kb) {
        const double dj = dinv_s[j];
        double* col = A + (size_t)(k0 + j) * nloc + k0;
#pragma unroll
        for (int t = 0; t < kMaxChunks; ++t) {
          const int r = t * 64 + lane;
          if (r < rows) col[r] = xv[t][u] * dj;
        }
      }
    }
    __syncthreads();
    // L11 (scaled multipliers of the pivot rows) from the panel columns
    for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
      const int qq = idx % kNB, r = idx / kNB;
      L11[idx] = (qq < r && r < kb) ? A[(size_t)(k0 + qq) * nloc + k0 + piv_s[r]] : 0.0;
    }
    // ---- the trailing columns in chunks of at most ldu - 2, whose U12 rows
    // share the LDS: row interchanges, U12, trailing update ----
    const int cwmax = ldu - 2;
    const int nch = (nc + cwmax - 1) / cwmax;
    const int cwid = (nc + nch - 1) / nch;
    for (int cs = 0; cs < nc; cs += cwid) {
      const int cw = min(cwid, nc - cs);
      // Two passes, eight loads in flight per thread in each: the pivot rows of
      // the chunk's columns into U12 (rows past a short last panel are zero
      // and take part in the update; the first panel reads K, whose trailing
      // update goes through rowmap), then the non-pivot rows among the first
      // kb into the vacated pivot slots.  A thread handles the same entries in
      // both passes, so each slot is read before it is overwritten.
      const int nu = kNB * cw;
      for (int base = tid; base < nu; base += 8 * kThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = base + u * kThreads;
          const int qq = idx % kNB, cc = cs + idx / kNB;
          v[u] = 0.0;
          if (idx < nu && qq < kb)
            v[u] = first ? K(piv_s[qq], c0 + cc) : A[(size_t)(c0 + cc) * nloc + k0 + piv_s[qq]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = base + u * kThreads;
          if (idx < nu) U[(idx % kNB) * ldu + idx / kNB] = v[u];
        }
      }
      if (!first) {
        for (int base = tid; base < nu; base += 8 * kThreads) {
          double v[8];
          double* dst[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int idx = base + u * kThreads;
            const int qq = idx % kNB, cc = cs + idx / kNB;
            const int x = (idx < nu && qq < kb) ? dsrc_s[qq] : -1;
            double* col = A + (size_t)(c0 + cc) * nloc + k0;
            dst[u] = x >= 0 ? col + piv_s[qq] : nullptr;
            v[u] = x >= 0 ? col[x] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (dst[u]) *dst[u] = v[u];
        }
      }
      __syncthreads();
      // U12 = L11^-1 (pivot rows of A12): forward substitution per column
      for (int cl = tid; cl < cw; cl += kThreads) {
        double u[kNB];
#pragma unroll
        for (int r = 0; r < kNB; ++r) u[r] = r < kb ? U[r * ldu + cl] : 0.0;
#pragma unroll
        for (int r = 1; r < kNB; ++r) {
          double s = u[r];
#pragma unroll
          for (int qq = 0; qq < r; ++qq) s -= L11[r * kNB + qq] * u[qq];
          u[r] = s;
          asm volatile("" : "+v"(u[r])::"memory");
        }
#pragma unroll
        for (int r = 0; r < kNB; ++r)
          if (r < kb) U[r * ldu + cl] = u[r];
      }
      __syncthreads();
      // A22 -= L21 U12: one row x four adjacent columns per thread (U12 read
      // as 128-bit broadcasts, L21 rows from the element matrix)
      {
        const int tr = rows - kb;
        const int RB = (tr + 63) >> 6, CG = (cw + 3) >> 2;
#pragma unroll 1
        for (int rb = 0; rb < RB; ++rb) {
          const int y = kb + rb * 64 + lane;       // panel-relative slot
          const bool live = y < rows;
          double l[kNB];
          {
            const double* lrow = A + (size_t)k0 * nloc + k0 + (live ? rowmap[y] : 0);
#pragma unroll
            for (int qq = 0; qq < kNB; ++qq) l[qq] = (live && qq < kb) ? lrow[(size_t)qq * nloc] : 0.0;
          }
          double* arow = A + (size_t)(c0 + cs) * nloc + k0 + y;
          // kPF column groups of A22 in flight per lane (a ring indexed at
          // compile time): one group's products take far less than a memory
          // round trip
          double nx[kPF][4];
#pragma unroll
          for (int p = 0; p < kPF; ++p) {
            const int cgp = wave + p * kWaves;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int cc = cgp * 4 + u;
              nx[p][u] = (live && cgp < CG && cc < cw && !first) ? arow[(size_t)cc * nloc] : 0.0;
            }
          }
#pragma unroll 1
          for (int cb = wave; cb < CG; cb += kWaves * kPF) {
#pragma unroll
            for (int p = 0; p < kPF; ++p) {
              const int cg = cb + p * kWaves;
              if (cg >= CG) break;   // uniform over the wave
              double sacc[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) sacc[u] = nx[p][u];
              const int cn = cg + kPF * kWaves;
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int cc = cn * 4 + u;
                nx[p][u] = (live && cn < CG && cc < cw && !first) ? arow[(size_t)cc * nloc] : 0.0;
              }
              const double2* Ub = reinterpret_cast<const double2*>(U + cg * 4);
              // four U12 rows at a time keep the register footprint down
#pragma unroll
              for (int q4 = 0; q4 < kNB; q4 += 4) {
                double2 u01[4], u23[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  u01[k] = Ub[(q4 + k) * (ldu / 2)];
                  u23[k] = Ub[(q4 + k) * (ldu / 2) + 1];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  sacc[0] -= l[q4 + k] * u01[k].x;
                  sacc[1] -= l[q4 + k] * u01[k].y;
                  sacc[2] -= l[q4 + k] * u23[k].x;
                  sacc[3] -= l[q4 + k] * u23[k].y;
                }
                // keeps the products in this group (not sunk into the guarded
                // stores) and the next group's loads behind them
                asm volatile("" : "+v"(sacc[0]), "+v"(sacc[1]), "+v"(sacc[2]), "+v"(sacc[3])::"memory");
              }
              if (live) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                  if (cg * 4 + u < cw) arow[(size_t)(cg * 4 + u) * nloc] = sacc[u];
              }
            }
          }
        }
      }
      __syncthreads();   // the next chunk's U12 reuses the LDS
    }
    if (first) {
      // the first trailing update started from zero: add K's trailing entries
      // at their rows' slots (each slot and column is touched once), kAddB at
      // a time so that their loads are in flight together
      const int items = K.items();
      for (int base = tid; base < items; base += kAddB * kThreads) {
        double* adr[kAddB];
        double val[kAddB], old[kAddB];
#pragma unroll
        for (int u = 0; u < kAddB; ++u) {
          int r = 0, c = 0;
          double v = 0.0;
          const int it = base + u * kThreads;
          const bool ok = it < items && K.item(it, r, c, v) && c >= c0 && slotof[r] >= 0;
          adr[u] = ok ? A + (size_t)c * nloc + slotof[r] : nullptr;
          val[u] = v;
        }
#pragma unroll
        for (int u = 0; u < kAddB; ++u) old[u] = adr[u] ? *adr[u] : 0.0;
#pragma unroll
        for (int u = 0; u < kAddB; ++u)
          if (adr[u]) *adr[u] = old[u] + val[u];
      }
      __syncthreads();
    }
  }
  if (tid == 0 && !(p2min >= kNearSingular2 * p2max)) a.fb_list[1 + atomicAdd(a.fb_list, 1)] = G;
  // the factorisation's LDS is free again: the Cayley step reuses it
  leaf_cayley(a, d, A, lds);
}

__global__ void fb_reset_kernel(int* list) { list[0] = 0; }

__global__ void flag_reset_kernel(int* flag) {
  const int i = threadIdx.x;
  if (i < kFlagWords) flag[i] = (i >= 2 && i < 6) ? -1 : (i == 6 ? 0x7FFFFFFF : 0);
}

// The complex element matrix L of Sec. 3.1 into columns [0, nloc) of S
// (column-major, ld nloc, rows and columns in ElemK's order): K's nonzeros one
// by one (each entry once), i eta on the diagonal of the boundary rows.
// Columns [nloc, ncols) are zeroed for the caller's right-hand sides; the
// load's real and imaginary parts (K's columns nloc, nloc + 1) go to column
// `load_col` when it is >= 0.  Ends with a barrier.
__device__ void element_assemble(cd* S, const ElemK& K, const Dims& d, double eta, int ncols, int load_col) {
  const int nloc = d.nloc, tid = threadIdx.x;
  for (int idx = tid; idx < nloc * ncols; idx += kThreads) S[idx] = cmk(0.0, 0.0);
  __syncthreads();
  for (int it = tid; it < K.items(); it += kThreads) {
    int r = 0, c = 0;
    double v = 0.0;
    if (!K.item(it, r, c, v)) continue;
    if (c < nloc) S[(size_t)c * nloc + r].x = v;
    else if (load_col >= 0) {
      if (c == nloc) S[(size_t)load_col * nloc + r].x = v;
      else S[(size_t)load_col * nloc + r].y = v;
    }
  }
  __syncthreads();
  for (int r = d.pp + tid; r < nloc; r += kThreads) S[(size_t)r * nloc + r].y = eta;
  __syncthreads();
}

// Solves L X = B in place: S = [L | B] (nloc x (nloc + nrhs), column-major,
// ld nloc); LU with partial pivoting over all rows, the right-hand sides
// carried along, then back substitution.  On return columns [nloc, nloc +
// nrhs) hold X.  A zero pivot is recorded as flag_where(0, elem).  Ends with
// a barrier.
__device__ void element_lu_solve(cd* S, int nloc, int nrhs, int* flag, long long elem) {
  __shared__ unsigned long long kw[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ncols = nloc + nrhs;
#define AT(r, c) S[(size_t)(c) * nloc + (r)]
  for (int k = 0; k < nloc; ++k) {
    unsigned long long key = 0;
    for (int r = k + tid; r < nloc; r += kThreads) key = max(key, pivot_key(cabs2(AT(r, k)), r));
    key = wave_max_key(key);
    if (lane == 0) kw[wave] = key;
    __syncthreads();
    unsigned long long kk = kw[0];
    for (int w = 1; w < kWaves; ++w) kk = max(kk, kw[w]);
    const int pr = min(max(pivot_row(kk), k), nloc - 1);
    if (tid == 0 && (kk >> 32) <= 1u) flag_singular(flag, flag_where(0, elem));
    if (pr != k)
      for (int c = k + tid; c < ncols; c += kThreads) {
        const cd t = AT(k, c);
        AT(k, c) = AT(pr, c);
        AT(pr, c) = t;
      }
    __syncthreads();
    const cd inv = cinv(AT(k, k));
    for (int r = k + 1 + tid; r < nloc; r += kThreads) AT(r, k) = cmul(AT(r, k), inv);
    __syncthreads();
    const int nr = nloc - k - 1, nc = ncols - k - 1;
    for (int idx = tid; idx < nr * nc; idx += kThreads) {
      const int r = k + 1 + idx % nr, c = k + 1 + idx / nr;
      AT(r, c) = csub(AT(r, c), cmul(AT(r, k), AT(k, c)));
    }
    __syncthreads();
  }
  for (int k = nloc - 1; k >= 0; --k) {
    const cd inv = cinv(AT(k, k));
    for (int j = tid; j < nrhs; j += kThreads) AT(k, nloc + j) = cmul(AT(k, nloc + j), inv);
    __syncthreads();
    for (int idx = tid; idx < k * nrhs; idx += kThreads) {
      const int i = idx % k, j = idx / k;
      AT(i, nloc + j) = csub(AT(i, nloc + j), cmul(AT(i, k), AT(k, nloc + j)));
    }
    __syncthreads();
  }
#undef AT
}

// ---- fallback: the element system of Sec. 3.1 solved as it stands ----------
// For the elements the leaf kernel lists (interior block nearly singular), the
// complex n_loc x n_loc element matrix L (interior rows of the local operator,
// boundary rows I_i = N_G + i eta E_G) is factored by LU with partial pivoting
// over all rows, with the right-hand sides [E_G^T | bt] carried along; back
// substitution gives X = L^-1 [E_G^T | bt], and T = I_o X_G-columns,
// H = I_o x_bt with I_o = -(N_G - i eta E_G).  One workgroup per listed
// element (grid-stride over the list), the system column-major in scratch.
// Slow (one barrier-separated rank-1 update per pivot) and meant to be rare.
__host__ __device__ inline size_t fb_stride(const Dims& d) {
  return ((size_t)2 * d.nloc * (d.nloc + 4 * d.p + 1) + 31) & ~(size_t)31;
}

__global__ __launch_bounds__(kThreads) void leaf_fallback_kernel(LeafArgs a) {
  const Dims d = dims_of(a.N);
  const int nloc = d.nloc, npiv = d.pp, m = 4 * d.p, nrhs = m + 1;
  const int tid = threadIdx.x;
  const int N1 = a.N + 1;
  // uniform values (scalar registers): the per-problem kernel arguments are
  // then indexed in place
  const int listed = __builtin_amdgcn_readfirstlane(a.fb_list[0]);
  cd* S = reinterpret_cast<cd*>(a.scratch + (size_t)blockIdx.x * fb_stride(d));
  for (int it = blockIdx.x; it < listed; it += gridDim.x) {
    const int G = __builtin_amdgcn_readfirstlane(a.fb_list[1 + it]);
    const int q = G / a.E, e = G % a.E;
    const double eta = a.eta[q - a.q0];
    const double* sq = a.s_nodes[q - a.q0];
    const ElemK K{d.N, d.p, d.pp, nloc, a.D, a.w, a.Kr, a.b_nodes[q - a.q0] + (size_t)e * N1 * N1,
                  sq ? sq + (size_t)e * 2 * N1 * N1 : nullptr, a.kappa[q - a.q0], a.h};
    // [L | E_G^T | bt]
    element_assemble(S, K, d, eta, nloc + nrhs, nloc + m);
    for (int j = tid; j < m; j += kThreads) S[(size_t)(nloc + j) * nloc + npiv + j] = cmk(1.0, 0.0);
    __syncthreads();
    element_lu_solve(S, nloc, nrhs, a.flag, G);
    // T = I_o X on the boundary columns, H = I_o x on the load column; row i
    // of N_G has p + 2 entries (K's items of boundary row i)
    const int ix = e % a.nx, iy = e / a.nx;
    cd* Tout = a.T + (a.linear_out ? (size_t)G : ((size_t)q * a.E + tree_code(a.ax, a.ay, ix, iy))) * m * m;
    const int nb0 = npiv * (2 * d.p + 5);   // first item of the boundary rows
    for (int idx = tid; idx < m * nrhs; idx += kThreads) {
      const int i = idx % m, j = idx / m;
      cd acc = cmk(0.0, 0.0);
      for (int t = 0; t < d.p + 2; ++t) {
        int r = 0, c = 0;
        double v = 0.0;
        K.item(nb0 + t * m + i, r, c, v);
        acc = cadd(acc, cscale(S[(size_t)(nloc + j) * nloc + c], v));
      }
      const cd xg = S[(size_t)(nloc + j) * nloc + npiv + i];
      const cd tv = cmk(-acc.x - eta * xg.y, -acc.y + eta * xg.x);
      if (j < m) Tout[(size_t)j * m + i] = tv;
      else a.H[(size_t)G * m + i] = tv;
    }
    __syncthreads();
  }
}

// ---- field recovery (Sec. 3.1): u = L^-1 [bt; f] per element ---------------
// f: the element's incoming impedances (g on interior sides, t on physical
// sides).  u at the non-corner nodes from the element solve; each corner the
// mean of the two extrapolations along its sides (weights xl at xi = -1, xr at
// xi = +1 of the degree-(N-2) polynomial through the side's inner nodes).
__host__ __device__ inline size_t field_stride(const Dims& d) {
  return ((size_t)2 * d.nloc * (d.nloc + 1) + 31) & ~(size_t)31;
}

__global__ __launch_bounds__(kThreads) void field_kernel(FieldArgs a) {
  const Dims d = dims_of(a.N);
  const int nloc = d.nloc, npiv = d.pp, p = d.p, N = a.N, N1 = N + 1;
  const int tid = threadIdx.x;
  cd* S = reinterpret_cast<cd*>(a.scratch + (size_t)blockIdx.x * field_stride(d));
  __shared__ cd uc[4][2];   // corner extrapolations: [corner][along y, along x]
  for (int G = blockIdx.x; G < a.count; G += gridDim.x) {
    const int q = G / a.E, e = G % a.E;
    const int ix = e % a.nx, iy = e / a.nx;
    const double eta = a.eta[q];
    const double* sq = a.s_nodes[q];
    const ElemK K{d.N, d.p, d.pp, nloc, a.D, a.w, a.Kr, a.b_nodes[q] + (size_t)e * N1 * N1,
                  sq ? sq + (size_t)e * 2 * N1 * N1 : nullptr, a.kappa[q], a.h};
    element_assemble(S, K, d, eta, nloc + 1, nloc);
    // boundary rows: the incoming impedances of the element's four sides
    const cd* g = a.g[q];
    const cd* t = a.t[q];
    for (int k = tid; k < 4 * p; k += kThreads) {
      const int side = k / p;
      const bool phys = (side == 0 && ix == 0) || (side == 1 && ix == a.nx - 1) || (side == 2 && iy == 0) ||
                        (side == 3 && iy == a.ny - 1);
      const size_t slot = (size_t)e * 4 * p + k;
      S[(size_t)nloc * nloc + npiv + k] = phys ? t[slot] : g[slot];
    }
    __syncthreads();
    element_lu_solve(S, nloc, 1, a.flag, G);
    const cd* x = S + (size_t)nloc * nloc;
    cd* u = a.u[q] + (size_t)e * N1 * N1;
    // interior nodes (i, j) = row (i-1) p + (j-1); side nodes after them
    for (int r = tid; r < nloc; r += kThreads) {
      int node;
      if (r < npiv) {
        node = (r / p + 1) * N1 + (r % p + 1);
      } else {
        const int side = (r - npiv) / p, k = (r - npiv) % p + 1;
        node = side == 0 ? k : (side == 1 ? N * N1 + k : (side == 2 ? k * N1 : k * N1 + N));
      }
      u[node] = x[r];
    }
    // corners (0,0), (0,N), (N,0), (N,N): extrapolate along the side in y
    // (nodes (i, k)) and along the side in x (nodes (k, j))
    if (tid < 8) {
      const int corner = tid >> 1, dir = tid & 1;
      const int ci = (corner & 2) ? N : 0, cj = (corner & 1) ? N : 0;
      const double* wgt = dir == 0 ? (cj ? a.xr : a.xl) : (ci ? a.xr : a.xl);
      cd acc = cmk(0.0, 0.0);
      for (int k = 1; k < N; ++k) {
        // row of the side node in the solve's order
        int r;
        if (dir == 0) r = npiv + (ci ? p : 0) + (k - 1);        // side l (i = 0) or r (i = N), node j = k
        else r = npiv + (cj ? 3 * p : 2 * p) + (k - 1);          // side b (j = 0) or t (j = N), node i = k
        acc = cadd(acc, cscale(x[r], wgt[k - 1]));
      }
      uc[corner][dir] = acc;
    }
    __syncthreads();
    if (tid < 4) {
      const int ci = (tid & 2) ? N : 0, cj = (tid & 1) ? N : 0;
      u[ci * N1 + cj] = cscale(cadd(uc[tid][0], uc[tid][1]), 0.5);
    }
    __syncthreads();
  }
}

}  // namespace

size_t field_scratch_doubles(int N, int blocks) { return (size_t)blocks * field_stride(dims_of(N)); }

hipError_t field_recover(const FieldArgs& a, int blocks, hipStream_t st) {
  const Dims d = dims_of(a.N);
  if (d.nloc > 64 * kMaxChunks || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(field_kernel, dim3(std::min(blocks, a.count)), dim3(kThreads), 0, st, a);
  return hipPeekAtLastError();
}

size_t leaf_scratch_doubles(int N, int count) {
  const Dims d = dims_of(N);
  const int fb = count < kFbBlocks ? count : kFbBlocks;
  return std::max((size_t)count * elem_stride(d), (size_t)fb * fb_stride(d));
}

hipError_t flag_reset(int* flag, hipStream_t st) {
  hipLaunchKernelGGL(flag_reset_kernel, dim3(1), dim3(64), 0, st, flag);
  return hipPeekAtLastError();
}

hipError_t leaf_build(const LeafArgs& a, hipStream_t st) {
  const Dims d = dims_of(a.N);
  if (d.nloc > 64 * kMaxChunks || 4 * d.p > 64) return hipErrorInvalidValue;
  const size_t lds = leaf_lds_bytes(a.N);
  hipError_t e0 = allow_lds(leaf_kernel, lds);
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(fb_reset_kernel, dim3(1), dim3(1), 0, st, a.fb_list);
  hipLaunchKernelGGL(leaf_kernel, dim3(a.count), dim3(kThreads), lds, st, a);
  hipLaunchKernelGGL(leaf_fallback_kernel, dim3(std::min(a.count, kFbBlocks)), dim3(kThreads), 0, st, a);
  return hipPeekAtLastError();
}

}  // namespace hps
