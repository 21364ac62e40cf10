// Batched in-place inversion of complex matrices (FP64 or FP32) by
// Gauss-Jordan elimination.
//
// m <= 32 (m <= 128 when partial pivoting is asked for): the whole matrix sits
// in registers, one workgroup per matrix, partial pivoting.
// Otherwise blocked Gauss-Jordan over block columns C = [k0, k0+nb):
//   1. without row interchanges across blocks (the default): the diagonal
//      block is inverted as it stands (gj_diag for the first block; each
//      later one by a look-ahead workgroup of the previous step's update
//      launch, from that launch's inputs), under a threshold test on the
//      multipliers that gj_update repeats for the rows outside the block; a
//      level that fails it is redone by the host with partial pivoting, so a
//      step is one launch.  With partial pivoting (two launches per step):
//      gj_panel (in registers or LDS) picks nb pivot rows (as the row map of
//      this step) and forms Dinv, the inverse of the pivot block;
//   2. gj_update: one pass over the whole matrix, out of place (two buffers),
//      rows read through the row map, P = C, X = Dinv A'[P, :]:
//        rows in P:      out = X           (Dinv on the C columns)
//        rows not in P:  out = A'[i, ~C] - A'[i, C] X   (-A'[i, C] Dinv on C).
// The row interchanges of all steps compose to one map rho; the inverse of the
// original matrix is the result with column j moved to column rho[j], which the
// last update (or a final copy) applies.  Work: m^3 complex multiply-adds in
// m / nb launches (2 m / nb with partial pivoting).  The merge blocks
// W = I - T^P_aa T^Q_bb of these problems need no interchanges (partial
// pivoting keeps every diagonal pivot and the elimination grows entries by
// about 3%), which is why the default skips the pivot search that dominated
// each step.
#include "common.h"
#include "host.h"
#include "pivot.h"

#include <climits>

namespace hps {

namespace {

constexpr int kNB = 32;        // widest block column
constexpr int kSmallNoPivot = 32;   // largest order inverted in registers without pivoting
constexpr int kPanelThreads = 1024;

// LDS bytes of gj_panel for m - k0 = rows and block width kb.
template <class T>
size_t panel_lds_bytes(int rows, int kb) {
  return sizeof(T) * ((size_t)rows * kb + (size_t)kb * kb + 2 * kb) + sizeof(int) * rows;
}

// Block width: the panel of the first step (m rows) must fit in about 150 KB.
template <class T>
int panel_width(int m) {
  int nb = kNB;
  while (nb > 4 && panel_lds_bytes<T>(m, nb) > 150 * 1024) nb /= 2;
  return nb;
}

// 1/a for matrix entries of moderate magnitude (one real division).
template <class T>
__device__ inline T crecip(T a) {
  typedef typename cx<T>::real R;
  const R n = a.x * a.x + a.y * a.y;
  const R s = n > 0 ? R(1) / n : R(0);
  return cx<T>::make(a.x * s, -a.y * s);
}

// Step 1 of a block column: the panel A[k0:m, k0:k0+kb] of matrix blockIdx.x.
// A partial-pivoting LU of the panel (rank-1 updates spread over (row, column
// group) threads; the next pivot found during the update by a per-wave DPP
// arg-max) selects the pivot rows; Dinv = (pivot block)^-1 then comes from an
// in-LDS Gauss-Jordan on the original pivot rows.  Writes Dinv [kb][kb]
// (column-major), rowmap (row i of the next matrix is row rowmap[i] of this
// one) and the composed map rho (row i then holds row rho[i] of the original).
template <class T>
__global__ __launch_bounds__(kPanelThreads) void gj_panel_kernel(const T* A, int m, int lda, long long bstride,
                                                                 int k0, int kb, const int* rho_prev, int* rho,
                                                                 int* rowmap, T* dinv, int* flag, int level) {
  extern __shared__ char smem[];
  const int rows = m - k0;
  T* Pn = reinterpret_cast<T*>(smem);          // rows x kb, column-major (ld rows)
  T* S = Pn + (size_t)rows * kb;               // kb x kb pivot block
  T* colk = S + kb * kb;                       // kb: column k of S
  T* rowk = colk + kb;                         // kb: row k of S
  int* perm = reinterpret_cast<int*>(rowk + kb);  // rows: local row order
  __shared__ unsigned long long kw[kPanelThreads / 64];  // per-wave best pivot key
  const T* Ab = A + (long long)blockIdx.x * bstride;
  const int tid = threadIdx.x, nt = blockDim.x, nw = nt / 64;
  // rank-1 updates: thread (rr, g) takes rows rr, rr + RT, ... and columns
  // c+1+g, c+1+g+G, ...
  const int RT = rows < nt ? rows : nt;
  const int G = nt / RT;
  const int rr = tid % RT, g = tid / RT;
  {
    unsigned long long best = 0;
    constexpr int U = 8;
    for (int base = 0; base < rows * kb; base += U * nt) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * nt + tid;
        v[u] = idx < rows * kb ? Ab[(long long)(k0 + idx / rows) * lda + k0 + idx % rows] : cx<T>::make(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * nt + tid;
        if (idx < rows * kb) {
          Pn[idx] = v[u];
          if (idx < rows) best = max(best, pivot_key(cabs2(v[u]), idx));
        }
      }
    }
    best = wave_max_key(best);
    if ((tid & 63) == 0) kw[tid >> 6] = best;
  }
  for (int r = tid; r < rows; r += nt) perm[r] = r;
  __syncthreads();
  // Only the pivot choice is taken from this factorisation (multipliers are not
  // kept): the block inverse below starts again from the original pivot rows.
  for (int c = 0; c < kb; ++c) {
    unsigned long long kk = 0;
    for (int w = 0; w < nw; ++w) kk = max(kk, kw[w]);
    int pr = pivot_row(kk);
    const bool bad = (kk >> 32) <= 1u || pr < c || pr >= rows;
    if (bad) pr = c;
    if (tid == 0 && bad) flag_singular(flag, flag_where(level, blockIdx.x));
    if (pr != c) {
      if (tid < kb) {
        const T t = Pn[tid * rows + c];
        Pn[tid * rows + c] = Pn[tid * rows + pr];
        Pn[tid * rows + pr] = t;
      } else if (tid == kb) {
        const int t = perm[c];
        perm[c] = perm[pr];
        perm[pr] = t;
      }
    }
    __syncthreads();
    if (c + 1 < kb) {
      const T inv = crecip(Pn[c * rows + c]);
      unsigned long long best = 0;
      if (g < G) {
        for (int r = rr; r < rows; r += RT) {
          if (r <= c) continue;
          const T l = cmul(Pn[c * rows + r], inv);
          for (int j = c + 1 + g; j < kb; j += G) {
            const T v = csub(Pn[j * rows + r], cmul(l, Pn[j * rows + c]));
            Pn[j * rows + r] = v;
            if (j == c + 1) best = max(best, pivot_key(cabs2(v), r));
          }
        }
      }
      best = wave_max_key(best);
      if ((tid & 63) == 0) kw[tid >> 6] = best;
      __syncthreads();
    }
  }
  int* rm = rowmap + (long long)blockIdx.x * m;
  int* ro = rho + (long long)blockIdx.x * m;
  const int* rp = rho_prev ? rho_prev + (long long)blockIdx.x * m : nullptr;
  for (int i = tid; i < m; i += nt) {
    const int src = i < k0 ? i : k0 + perm[i - k0];
    rm[i] = src;
    ro[i] = rp ? rp[src] : src;
  }
  for (int idx = tid; idx < kb * kb; idx += nt) {
    const int r = idx % kb, c = idx / kb;
    S[idx] = Ab[(long long)(k0 + c) * lda + k0 + perm[r]];
  }
  __syncthreads();
  // Gauss-Jordan on the pivot block; its rows are already in pivot order, so
  // the diagonal pivots are the ones the panel factorisation chose
  for (int k = 0; k < kb; ++k) {
    const T inv = crecip(S[k * kb + k]);
    if (tid < kb) {
      colk[tid] = tid == k ? cx<T>::make(0.0, 0.0) : S[k * kb + tid];
      rowk[tid] = tid == k ? inv : cmul(S[tid * kb + k], inv);
    }
    __syncthreads();
    for (int idx = tid; idx < kb * kb; idx += nt) {
      const int i = idx % kb, j = idx / kb;
      const T rk = rowk[j];  // row k scaled by the pivot's inverse
      if (i == k) {
        S[idx] = rk;
      } else {
        const T base = j == k ? cx<T>::make(0.0, 0.0) : S[idx];
        S[idx] = csub(base, cmul(colk[i], rk));
      }
    }
    __syncthreads();
  }
  T* Db = dinv + (long long)blockIdx.x * kNB * kNB;
  for (int idx = tid; idx < kb * kb; idx += nt) Db[idx] = S[idx];
}

// Lane l's complex value broadcast to the wavefront (l uniform).
__device__ inline cd readlane_c(cd v, int l) {
  const long long x = __double_as_longlong(v.x), y = __double_as_longlong(v.y);
  const unsigned x0 = (unsigned)__builtin_amdgcn_readlane((int)x, l);
  const unsigned x1 = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
  const unsigned y0 = (unsigned)__builtin_amdgcn_readlane((int)y, l);
  const unsigned y1 = (unsigned)__builtin_amdgcn_readlane((int)(y >> 32), l);
  return cmk(__longlong_as_double((long long)(((unsigned long long)x1 << 32) | x0)),
             __longlong_as_double((long long)(((unsigned long long)y1 << 32) | y0)));
}
__device__ inline cf readlane_c(cf v, int l) {
  return cmkf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l)),
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l)));
}

// m <= 64 RC: Gauss-Jordan with the matrix in registers, one workgroup of NW
// waves per matrix: thread (rows 64c + lane, wave w) holds columns j = w + NW t.
// Pivot rows stay where they are (marked used); a step reads the pivot row by
// lane broadcasts and the pivot column from LDS, where the wave holding it
// published it with the next pivot key and reciprocal, and takes one barrier.
// With pivot row pr_k at step k the registers end as S[pr_k][j] = A^-1[k][pr_j],
// written back to A^-1's own positions.
template <class T, int NW, int RC>
__global__ __launch_bounds__(64 * NW) void inv_small_kernel(T* A, int m, int lda, long long bstride, int* flag, int level) {
  constexpr int kT = 64 * RC / NW;  // columns per thread
  __shared__ T colbuf[2][64 * RC];
  __shared__ T pinv[2];
  __shared__ unsigned long long kw[2];
  __shared__ int pivs[64 * RC];
  T* Ab = A + (long long)blockIdx.x * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_uniform(tid >> 6);
  T sv[RC][kT];
#pragma unroll
  for (int c = 0; c < RC; ++c)
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int i = 64 * c + lane, j = wave + NW * t;
      sv[c][t] = (i < m && j < m) ? Ab[(long long)j * lda + i] : cx<T>::make(0.0, 0.0);
    }
  unsigned used = 0;   // bit c: row 64c + lane is a pivot row
  int myk[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) myk[c] = 0;
  // the wave holding column kn publishes it with its pivot and reciprocal
  auto publish = [&](int kn, int tn) {
    const int b = kn & 1;
    unsigned long long key = 0;
    T vn[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      vn[c] = cx<T>::make(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < kT; ++t)
        if (t == tn) vn[c] = sv[c][t];
      const int i = 64 * c + lane;
      colbuf[b][i] = vn[c];
      if (i < m && !((used >> c) & 1u)) key = max(key, pivot_key(cabs2(vn[c]), i));
    }
    key = wave_max_key(key);
    const int pn = min(max(pivot_row(key), 0), m - 1);
    T d = cx<T>::make(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < RC; ++c)
      if (c == (pn >> 6)) d = readlane_c(vn[c], pn & 63);
    if (lane == 0) {
      kw[b] = key;
      pinv[b] = ((key >> 32) <= 1u) ? cx<T>::make(0.0, 0.0) : crecip(d);
    }
  };
  if (wave == 0) publish(0, 0);
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < m; ++k) {
    const int b = k & 1;
    const unsigned long long kk = wave_uniform(kw[b]);
    const T inv = pinv[b];
    const int pr = min(max(pivot_row(kk), 0), m - 1);
    const int cp = pr >> 6, lp = pr & 63;
    if (lane == lp) {
      used |= 1u << cp;
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c == cp) myk[c] = k;
    }
    if (tid == 0) {
      pivs[k] = pr;
      if ((kk >> 32) <= 1u) flag_singular(flag, flag_where(level, blockIdx.x));
    }
    T f[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c)
      f[c] = (64 * c + lane == pr) ? cx<T>::make(0.0, 0.0) : cmul(colbuf[b][64 * c + lane], inv);
    const int tk = k / NW, ok = k % NW;
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      if (wave + NW * t >= m) continue;
      if (wave == ok && t == tk) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
          sv[c][t] = (64 * c + lane == pr) ? inv : csub(cx<T>::make(0.0, 0.0), f[c]);
      } else {
        T pv = cx<T>::make(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c == cp) pv = readlane_c(sv[c][t], lp);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          sv[c][t] = (64 * c + lane == pr) ? cmul(pv, inv) : csub(sv[c][t], cmul(f[c], pv));
      }
    }
    const int kn = k + 1;
    if (kn < m && wave == kn % NW) publish(kn, kn / NW);
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < RC; ++c)
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int i = 64 * c + lane, j = wave + NW * t;
      if (i < m && j < m) Ab[(long long)pivs[j] * lda + myk[c]] = sv[c][t];
    }
}

// Called by the one wave holding the next panel column (column U of this
// wave's registers, rows t*64 + lane): publishes the column, picks its pivot
// among the unused rows, stores the pivot key and 1/pivot.
template <int U, class T, int CH, int CPW>
__device__ inline void panel_publish(const T (&x)[CH][CPW], unsigned used, int rows, T* cbn,
                                     unsigned long long* key_out, T* inv_out) {
  const int lane = threadIdx.x & 63;
  unsigned long long best = 0;
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    const int r = t * 64 + lane;
    if (r < rows) {
      cbn[r] = x[t][U];
      if (!((used >> t) & 1u)) best = max(best, pivot_key(cabs2(x[t][U]), r));
    }
  }
  best = wave_max_key(best);
  const int pn = min(max(pivot_row(best), 0), rows - 1);
  T dn = cx<T>::make(0.0, 0.0);
#pragma unroll
  for (int t = 0; t < CH; ++t)
    if (t == (pn >> 6)) dn = readlane_c(x[t][U], pn & 63);
  if (lane == 0) {
    *key_out = best;
    *inv_out = ((best >> 32) <= 1u) ? cx<T>::make(0.0, 0.0) : crecip(dn);
  }
}

// gj_panel with the panel in registers (1024 threads; rows <= 64 CH, kb <= 16
// CPW): wave w holds panel columns j = w + 16u, lane the rows t*64 + lane.
// Pivot rows stay where they are (marked used) during the panel LU, so a column
// step takes one barrier: the wave holding the next column publishes it with
// its pivot key and reciprocal, every wave reads the pivot row of its own
// columns by lane broadcasts.  Only the pivot order is kept.  The row order of
// the step: pivot rows first, the non-pivot rows among the first kb moved into
// the slots the later pivot rows leave.  Dinv = (pivot block)^-1 then comes
// from a Gauss-Jordan of the original pivot rows in pivot order (no further
// pivoting), one entry per thread, one barrier per step.  Same outputs as
// gj_panel_kernel.
template <class T, int CH, int CPW>
__global__ __launch_bounds__(1024) void gj_panel_reg_kernel(const T* A, int m, int lda, long long bstride, int k0,
                                                             int kb, const int* rho_prev, int* rho, int* rowmap,
                                                             T* dinv, int* flag, int level) {
  constexpr int NW = 16;
  __shared__ T colbuf[2][64 * CH];
  __shared__ unsigned long long kw_s[2];
  __shared__ T pinv_s[2];
  __shared__ int piv_s[kNB], dsrc_s[kNB];
  const int rows = m - k0;
  const T* Ab = A + (long long)blockIdx.x * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_uniform(tid >> 6);
  T x[CH][CPW];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    const int j = wave + NW * u;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int r = t * 64 + lane;
      x[t][u] = (j < kb && r < rows) ? Ab[(long long)(k0 + j) * lda + k0 + r] : cx<T>::make(0.0, 0.0);
    }
  }
  if (wave == 0) panel_publish<0>(x, 0u, rows, colbuf[0], kw_s, pinv_s);
  __syncthreads();
  unsigned used = 0;  // bit t: row t*64 + lane is a pivot row
#pragma unroll 1
  for (int c = 0; c < kb; ++c) {
    const int b = c & 1;
    const unsigned long long kk = wave_uniform(kw_s[b]);
    const T inv = pinv_s[b];
    const int pr = min(max(pivot_row(kk), 0), rows - 1);
    const int tp = pr >> 6, lp = pr & 63;
    if (lane == lp) used |= 1u << tp;
    if (tid == 0) {
      piv_s[c] = pr;
      if ((kk >> 32) <= 1u) flag_singular(flag, flag_where(level, blockIdx.x));
    }
    // pivot row entries of this wave's live columns, scaled by 1/pivot once
    // (the column entries then multiply them directly); waves with no live
    // column skip the step
    T pv[CPW];
    bool wlive = false;
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
      pv[u] = cx<T>::make(0.0, 0.0);
      const int j = wave + NW * u;
      wlive |= (j > c && j < kb);
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      if (t == tp) {
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
          const int j = wave + NW * u;
          if (j > c && j < kb) pv[u] = cmul(readlane_c(x[t][u], lp), inv);
        }
      }
    }
    // the wave holding column c + 1 publishes it (during the update) with its
    // pivot and 1/pivot
    const int cn = c + 1;
    const bool own = cn < kb && wave == (cn % NW);
    const int un = cn / NW;
    T* cbn = colbuf[b ^ 1];
    unsigned long long best = 0;
    if (wlive) {
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        // chunks past the live rows (uniform); not taken at CH = 16, where the
        // extra control flow would push the 128-register budget into scratch
        if (CH <= 8 && t * 64 >= rows) continue;
        const int r = t * 64 + lane;
        const bool act = r < rows && !((used >> t) & 1u);
        const T l = act ? colbuf[b][r] : cx<T>::make(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
          const int j = wave + NW * u;
          if (j > c && j < kb) x[t][u] = csub(x[t][u], cmul(l, pv[u]));  // wave-uniform
        }
        if (own && r < rows) {
          const T vn = (CPW == 1 || un == 0) ? x[t][0] : x[t][CPW - 1];
          cbn[r] = vn;
          if (act) best = max(best, pivot_key(cabs2(vn), r));
        }
      }
    }
    if (own) {
      best = wave_max_key(best);
      const T dn = cbn[min(max(pivot_row(best), 0), rows - 1)];
      if (lane == 0) {
        kw_s[b ^ 1] = best;
        pinv_s[b ^ 1] = ((best >> 32) <= 1u) ? cx<T>::make(0.0, 0.0) : crecip(dn);
      }
    }
    if (c == kb - 1 && wave == 0) {
      // pair the pivot rows beyond the first kb with the non-pivot rows among
      // the first kb: those rows take the pivot rows' slots
      bool isp = false;
      if (lane < kb)
        for (int q = 0; q < kb; ++q) isp |= (piv_s[q] == lane);
      const unsigned long long nonpiv = __ballot(lane < kb && !isp);
      const int y = lane < kb ? piv_s[lane] : 0;
      const bool far = lane < kb && y >= kb;
      const unsigned long long farm = __ballot(far);
      if (lane < kb) {
        int xsrc = -1;
        if (far) {
          const int rank = __popcll(farm & ((1ull << lane) - 1ull));
          unsigned long long mm = nonpiv;
          for (int k = 0; k < rank; ++k) mm &= mm - 1ull;
          xsrc = __ffsll((long long)mm) - 1;
        }
        dsrc_s[lane] = xsrc;
      }
    }
    __syncthreads();
  }
  // the step's row order: rm[i] (new row i holds old row rm[i])
  int* rm = rowmap + (long long)blockIdx.x * m;
  int* ro = rho + (long long)blockIdx.x * m;
  const int* rp = rho_prev ? rho_prev + (long long)blockIdx.x * m : nullptr;
  for (int i = tid; i < m; i += 1024) {
    int src = i;
    if (i >= k0) {
      const int r = i - k0;
      int pr = r;
      if (r < kb) {
        pr = piv_s[r];
      } else {
        for (int q = 0; q < kb; ++q)
          if (piv_s[q] == r) pr = dsrc_s[q];
      }
      src = k0 + pr;
    }
    rm[i] = src;
    ro[i] = rp ? rp[src] : src;
  }
  // Dinv: Gauss-Jordan of S = A[k0 + piv, k0 : k0 + kb], thread (i, j) = (tid % 32, tid / 32)
  const int gi = tid & 31, gj = tid >> 5;
  const bool live = gi < kb && gj < kb;
  T sv = live ? Ab[(long long)(k0 + gj) * lda + k0 + piv_s[gi]] : cx<T>::make(0.0, 0.0);
  T* colS = colbuf[0];   // [2][32]: column k of S
  __syncthreads();       // piv_s reads done with the panel buffers
  if (gj == 0) colS[gi] = sv;
  if (tid == 0) pinv_s[0] = crecip(sv);
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < kb; ++k) {
    const int b = k & 1;
    const T inv = pinv_s[b];
    // pivot row entry of this thread's column: thread (k, gj) = lane k or 32 + k of this wave
    const T r0 = readlane_c(sv, k), r1 = readlane_c(sv, 32 + k);
    const T rk = (lane < 32) ? r0 : r1;
    const T ci = colbuf[b][gi];
    T v;
    if (gi == k) v = (gj == k) ? inv : cmul(rk, inv);
    else if (gj == k) v = csub(cx<T>::make(0.0, 0.0), cmul(ci, inv));
    else v = csub(sv, cmul(cmul(ci, inv), rk));
    sv = live ? v : cx<T>::make(0.0, 0.0);
    if (gj == k + 1 && k + 1 < kb) {
      colbuf[b ^ 1][gi] = sv;
      if (gi == k + 1) pinv_s[b ^ 1] = crecip(sv);
    }
    __syncthreads();
  }
  T* Db = dinv + (long long)blockIdx.x * kNB * kNB;
  if (live) Db[gj * kb + gi] = sv;
}

// Step 1 without row interchanges across blocks: the inverse of the diagonal
// block A[k0 : k0+kb, k0 : k0+kb] of matrix blockIdx.x by Gauss-Jordan without
// pivoting, one wave per matrix (lane = row i + 32 h, columns j = 2t + h), so
// a step needs no workgroup barrier.  The row maps of this step are the
// identity.  The elimination is accepted only while every multiplier of a
// row below the pivot stays within 1/kNoPivotTau of the pivot (threshold
// pivoting's test); otherwise the level is recorded in error word 6 and the
// host redoes the merge with partial pivoting.
constexpr double kNoPivotTau = 0.1;

template <class T>
__global__ __launch_bounds__(64) void gj_diag_kernel(const T* A, int m, int lda, long long bstride, int k0, int kb,
                                                     const int* rho_prev, int* rho, int* rowmap, T* dinv,
                                                     int* flag, int level) {
  __shared__ T prow[kNB];
  __shared__ T colk[kNB];
  const T* Ab = A + (long long)blockIdx.x * bstride;
  const int lane = threadIdx.x, i = lane & 31, h = lane >> 5;
  {
    int* rm = rowmap + (long long)blockIdx.x * m;
    int* ro = rho + (long long)blockIdx.x * m;
    const int* rp = rho_prev ? rho_prev + (long long)blockIdx.x * m : nullptr;
    for (int r = lane; r < m; r += 64) {
      rm[r] = r;
      ro[r] = rp ? rp[r] : r;
    }
  }
  // a block narrower than kNB is padded with the identity, so that every
  // step below is the same and the step loop unrolls with static register
  // indices; the padding's inverse is the identity and is not written
  T sv[kNB / 2];
#pragma unroll
  for (int t = 0; t < kNB / 2; ++t) {
    const int j = 2 * t + h;
    sv[t] = (i < kb && j < kb) ? Ab[(long long)(k0 + j) * lda + k0 + i]
                               : cx<T>::make(i == j ? 1.0 : 0.0, 0.0);
  }
  bool grow = false;
  const bool live = i < kb;
#pragma unroll
  for (int k = 0; k < kNB; ++k) {
    // publish row k (its two lanes) and column k (the 32 lanes holding it)
    if (i == k) {
#pragma unroll
      for (int t = 0; t < kNB / 2; ++t) prow[2 * t + h] = sv[t];
    }
    if (h == (k & 1)) colk[i] = sv[k >> 1];
    __syncthreads();
    // all LDS reads of the step together, then branch-free arithmetic: with
    // li = a_ik / a_kk (rows i != k) and li = 1 - 1/a_kk (row k), every entry
    // becomes a_ij - li a_kj; column k is then set to -li (rows i != k) and
    // 1/a_kk (row k)
    T pr[kNB / 2];
#pragma unroll
    for (int t = 0; t < kNB / 2; ++t) pr[t] = prow[2 * t + h];
    const T pk = prow[k];
    const T l = colk[i];
    const T inv = crecip(pk);
    const bool rowk = i == k;
    const T lq = cmul(l, inv);
    const T li = rowk ? csub(cx<T>::make(1.0, 0.0), inv) : lq;
    // threshold test: |a_ik| > |a_kk| / tau for a row below, or a zero pivot
    const double p2 = (double)cabs2(pk);
    if (k < kb && ((i > k && live && !((double)cabs2(l) * (kNoPivotTau * kNoPivotTau) <= p2)) || !(p2 > 0.0)))
      grow = true;
#pragma unroll
    for (int t = 0; t < kNB / 2; ++t) sv[t] = csub(sv[t], cmul(li, pr[t]));
    const T colv = rowk ? inv : csub(cx<T>::make(0.0, 0.0), lq);
    if (h == (k & 1)) sv[k >> 1] = colv;
    __syncthreads();
  }
  if (__ballot(grow)) {
    if (lane == 0) atomicMin(flag + 6, level);
  }
  T* Db = dinv + (long long)blockIdx.x * kNB * kNB;
#pragma unroll
  for (int t = 0; t < kNB / 2; ++t) {
    const int j = 2 * t + h;
    if (i < kb && j < kb) Db[j * kb + i] = sv[t];
  }
}

// Look-ahead of the no-pivot path, run by one extra workgroup (workgroup 0, 256 threads)
// of the update launch of step k: the pivot block of step k + 1 as that update
// will leave it, P = A[K1, K1] - A[K1, K0] Dk A[K0, K1] (K0 = [k0, k0+kb),
// K1 = [k1, k1+kb1), Dk the inverse of this step's pivot block, ld kb), from
// the same inputs as the update, and its inverse into Dn (ld kb1) by the same
// Gauss-Jordan steps and threshold test as gj_diag_kernel.  Thread (i, g)
// holds row i, columns 4g..4g+3; S0..S3 are kNB x kNB entries of LDS each
// (column-major, ld kNB): A[K1, K0], Dk, A[K0, K1] and A[K1, K0] Dk.
// Component-wise choice between two complex values (a choice between whole
// vector-type values can leave a private copy behind).
template <class T>
__device__ inline T csel(bool c, const T& a, const T& b) {
  return cx<T>::make(c ? a.x : b.x, c ? a.y : b.y);
}

template <class T>
__device__ __forceinline__ void gj_next_diag(const T* Ab, int lda, int k0, int kb, int k1, int kb1, const T* Dk, T* Dn,
                             T* S0, T* S1, T* S2, T* S3, int* check, int level) {
  constexpr int W = kNB * kNB;
  const int tid = threadIdx.x, i = tid & 31, g = tid >> 5, j0 = 4 * g;
  const T zero = cx<T>::make(0.0, 0.0);
  for (int idx = tid; idx < W; idx += 256) {
    const int r = idx & 31, c = idx >> 5;   // row r, column c (column-major, ld kNB)
    const bool a0 = r < kb1 && c < kb, a1 = r < kb && c < kb, a2 = r < kb && c < kb1;
    // loads from clamped (valid) addresses, zeros chosen outside
    S0[idx] = csel(a0, Ab[(long long)(k0 + (a0 ? c : 0)) * lda + k1 + (a0 ? r : 0)], zero);
    S1[idx] = csel(a1, Dk[a1 ? c * kb + r : 0], zero);
    S2[idx] = csel(a2, Ab[(long long)(k1 + (a2 ? c : 0)) * lda + k0 + (a2 ? r : 0)], zero);
  }
  // this thread's four entries of the pivot block (the identity past kb1), as
  // four scalars so that every index below is static
  auto init = [&](int j) {
    const bool in = i < kb1 && j < kb1;
    return csel(in, Ab[(long long)(k1 + (in ? j : 0)) * lda + k1 + (in ? i : 0)], cx<T>::make(i == j ? 1.0 : 0.0, 0.0));
  };
  T p0 = init(j0), p1 = init(j0 + 1), p2 = init(j0 + 2), p3 = init(j0 + 3);
  __syncthreads();
  // S3 = A[K1, K0] Dk
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + u;
    T t = zero;
    for (int r = 0; r < kNB; ++r) t = cfma(S0[r * kNB + i], S1[j * kNB + r], t);
    S3[j * kNB + i] = t;
  }
  __syncthreads();
  // P -= S3 A[K0, K1] (rows and columns past kb1 keep the identity)
  auto prod = [&](int j) {
    T t = zero;
    for (int r = 0; r < kNB; ++r) t = cfma(S3[r * kNB + i], S2[j * kNB + r], t);
    return t;
  };
  if (i < kb1) {
    if (j0 < kb1) p0 = csub(p0, prod(j0));
    if (j0 + 1 < kb1) p1 = csub(p1, prod(j0 + 1));
    if (j0 + 2 < kb1) p2 = csub(p2, prod(j0 + 2));
    if (j0 + 3 < kb1) p3 = csub(p3, prod(j0 + 3));
  }
  __syncthreads();   // S0 and S1 hold rows and columns k below
  bool grow = false;
  const bool live = i < kb1;
  for (int k = 0; k < kNB; ++k) {
    // row and column k in one of two buffers (alternating), so that one
    // barrier per step orders both the writes before the reads and this
    // step's reads before the writes two steps on
    T* prow = S0 + (k & 1) * kNB;
    T* colk = S1 + (k & 1) * kNB;
    const int kg = k >> 2, ku = k & 3;
    if (i == k) {
      prow[j0] = p0;
      prow[j0 + 1] = p1;
      prow[j0 + 2] = p2;
      prow[j0 + 3] = p3;
    }
    if (g == kg) colk[i] = csel(ku == 0, p0, csel(ku == 1, p1, csel(ku == 2, p2, p3)));
    __syncthreads();
    const T pk = prow[k];
    const T l = colk[i];
    const T r0 = prow[j0], r1 = prow[j0 + 1], r2 = prow[j0 + 2], r3 = prow[j0 + 3];
    const T inv = crecip(pk);
    const bool rowk = i == k;
    const T lq = cmul(l, inv);
    const T li = csel(rowk, csub(cx<T>::make(1.0, 0.0), inv), lq);
    const double p2k = (double)cabs2(pk);
    if (k < kb1 && ((i > k && live && !((double)cabs2(l) * (kNoPivotTau * kNoPivotTau) <= p2k)) || !(p2k > 0.0)))
      grow = true;
    p0 = csub(p0, cmul(li, r0));
    p1 = csub(p1, cmul(li, r1));
    p2 = csub(p2, cmul(li, r2));
    p3 = csub(p3, cmul(li, r3));
    const T colv = csel(rowk, inv, csub(zero, lq));
    p0 = csel(g == kg && ku == 0, colv, p0);
    p1 = csel(g == kg && ku == 1, colv, p1);
    p2 = csel(g == kg && ku == 2, colv, p2);
    p3 = csel(g == kg && ku == 3, colv, p3);
  }
  if (i < kb1) {
    if (j0 < kb1) Dn[j0 * kb1 + i] = p0;
    if (j0 + 1 < kb1) Dn[(j0 + 1) * kb1 + i] = p1;
    if (j0 + 2 < kb1) Dn[(j0 + 2) * kb1 + i] = p2;
    if (j0 + 3 < kb1) Dn[(j0 + 3) * kb1 + i] = p3;
  }
  if (__syncthreads_or(grow) && tid == 0 && check) atomicMin(check + 6, level);
}

// Step 2 of a block column: out-of-place update of the whole matrix, BT x BT
// tiles (64, or 32 where 64 would leave few workgroups), 256 threads, each
// thread (BT/16)^2 outputs (rows i0 + tx + 16u, columns j0 + ty + 16v), rows
// read through rowmap, P = C = [k0, k0+kb):
//   X = Dinv A'[P, :] (Dinv on the C columns); rows in P: out = X;
//   other rows: out = A'[i, ~C] - A'[i, C] X  (-A'[i, C] Dinv on C).
// With colmap the output column j is written at colmap[j].
// check: without row interchanges (gj_diag_kernel), the block multipliers
// -A'[i, C] Dinv of the rows outside P must stay within 1/kNoPivotTau, else
// the level is recorded in check[6] (null: no check).
template <class T, int BT>
__global__ __launch_bounds__(256) void gj_update_kernel(const T* A, int lda, long long astride, T* O, int ldo,
                                                        long long ostride, int m, int k0, int kb,
                                                        const int* rowmap, const T* dinv, const int* colmap,
                                                        int* check, int level, T* dnext, int k1, int kb1) {
  constexpr int U = BT / 16;
  static_assert(BT >= 32, "the look-ahead workgroup reuses Xs, Bp and Ac as 4 kNB x kNB blocks");
  __shared__ T Ds[kNB * kNB];
  __shared__ T Xs[kNB][BT];
  __shared__ T Bp[kNB][BT];     // A'[P, jtile]
  __shared__ T Ac[kNB][BT + 1]; // A'[itile, C], transposed
  const int tiles = (m + BT - 1) / BT, per = tiles * tiles;
  // one flat grid: with a look-ahead, workgroups 0 .. batch-1 are the
  // matrices' look-aheads (dispatched first), then each matrix's tiles
  const int nla = dnext ? (int)gridDim.x / (per + 1) : 0;
  if ((int)blockIdx.x < nla) {
    // the next step's pivot block inverse of matrix blockIdx.x (no row
    // interchanges; Xs, Bp, Ac and Ds hold the four kNB x kNB blocks it
    // needs), formed while the tiles are updated
    const int b = blockIdx.x;
    gj_next_diag<T>(A + (long long)b * astride, lda, k0, kb, k1, kb1, dinv + (long long)b * kNB * kNB,
                    dnext + (long long)b * kNB * kNB, &Xs[0][0], &Bp[0][0], &Ac[0][0], Ds, check, level);
    return;
  }
  const int q = (int)blockIdx.x - nla;
  const int tile = q % per, b = q / per;
  const int i0 = (tile % tiles) * BT, j0 = (tile / tiles) * BT;
  const T* Ab = A + (long long)b * astride;
  T* Ob = O + (long long)b * ostride;
  const int* rm = rowmap + (long long)b * m;
  const T* Db = dinv + (long long)b * kNB * kNB;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  T aout[U][U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int gi = i0 + tx + 16 * u;
    const bool rowok = gi < m && !(gi >= k0 && gi < k0 + kb);
    const int src = gi < m ? rm[gi] : 0;
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const int gj = j0 + ty + 16 * v;
      const bool ok = rowok && gj < m && !(gj >= k0 && gj < k0 + kb);
      aout[u][v] = ok ? Ab[(long long)gj * lda + src] : cx<T>::make(0.0, 0.0);
    }
  }
  for (int idx = tid; idx < kb * kb; idx += 256) Ds[(idx / kb) * kNB + idx % kb] = Db[idx];
  for (int idx = tid; idx < kb * BT; idx += 256) {
    const int q = idx % kb, j = idx / kb;
    const int gj = j0 + j;
    Bp[q][j] = (gj < m) ? Ab[(long long)gj * lda + rm[k0 + q]] : cx<T>::make(0.0, 0.0);
  }
  for (int idx = tid; idx < BT * kb; idx += 256) {
    const int i = idx % BT, q = idx / BT;
    const int gi = i0 + i;
    Ac[q][i] = (gi < m) ? Ab[(long long)(k0 + q) * lda + rm[gi]] : cx<T>::make(0.0, 0.0);
  }
  __syncthreads();
  for (int idx = tid; idx < kb * BT; idx += 256) {
    const int j = idx % BT, q = idx / BT;
    const int gj = j0 + j;
    T v = cx<T>::make(0.0, 0.0);
    if (gj >= k0 && gj < k0 + kb) {
      v = Ds[(gj - k0) * kNB + q];
    } else if (gj < m) {
      for (int r = 0; r < kb; ++r) v = cfma(Ds[r * kNB + q], Bp[r][j], v);
    }
    Xs[q][j] = v;
  }
  __syncthreads();
  T acc[U][U];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < U; ++v) acc[u][v] = cx<T>::make(0.0, 0.0);
  for (int q = 0; q < kb; ++q) {
    T a[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = Ac[q][tx + 16 * u];
#pragma unroll
    for (int v = 0; v < U; ++v) x[v] = Xs[q][ty + 16 * v];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < U; ++v) acc[u][v] = cfma(a[u], x[v], acc[u][v]);
  }
  bool grow = false;
  const double lim2 = 1.0 / (kNoPivotTau * kNoPivotTau);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int gi = i0 + tx + 16 * u;
    if (gi >= m) continue;
    const bool inP = gi >= k0 && gi < k0 + kb;
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const int j = ty + 16 * v;
      const int gj = j0 + j;
      if (gj >= m) continue;
      const int oc = colmap ? colmap[(long long)b * m + gj] : gj;
      const T val = inP ? Xs[gi - k0][j] : csub(aout[u][v], acc[u][v]);
      if (check && !inP && gi > k0 && gj >= k0 && gj < k0 + kb && !((double)cabs2(val) <= lim2)) grow = true;
      Ob[(long long)oc * ldo + gi] = val;
    }
  }
  if (check && __syncthreads_or(grow) && tid == 0) atomicMin(check + 6, level);
}

// dst(:, colmap[j]) = src(:, j): the inverse of the row-interchanged matrix
// becomes the inverse of the original one.
template <class T>
__global__ void permute_cols_kernel(const T* S, int lds, long long sstride, T* A, int lda, long long bstride,
                                    int m, const int* colmap) {
  const int b = blockIdx.z, j = blockIdx.y;
  const T* Sb = S + (long long)b * sstride;
  T* Ab = A + (long long)b * bstride;
  const int oc = colmap ? colmap[(long long)b * m + j] : j;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    Ab[(long long)oc * lda + i] = Sb[(long long)j * lds + i];
}

template <class T>
struct BlockScratch {
  T* buf;       // [batch][m][m] second buffer (ld m)
  T* dinv;      // [2][batch][kNB][kNB] (alternating pivot block inverses without pivoting)
  int* rho[2];  // [batch][m] composed row maps (alternating)
  int* rowmap;  // [batch][m]
};

template <class T>
inline BlockScratch<T> carve(void* base, int m, int batch) {
  BlockScratch<T> s;
  char* p = (char*)base;
  auto take = [&](size_t bytes) { char* q = p; p += (bytes + 255) & ~size_t(255); return q; };
  s.buf = (T*)take(sizeof(T) * (size_t)batch * m * m);
  s.dinv = (T*)take(sizeof(T) * (size_t)2 * batch * kNB * kNB);
  s.rho[0] = (int*)take(sizeof(int) * (size_t)batch * m);
  s.rho[1] = (int*)take(sizeof(int) * (size_t)batch * m);
  s.rowmap = (int*)take(sizeof(int) * (size_t)batch * m);
  return s;
}

template <class T>
hipError_t inverse_blocked(T* A, int m, int lda, long long bstride, int batch, void* scratch,
                           int* flag, int level, bool pivot, hipStream_t st) {
  BlockScratch<T> s = carve<T>(scratch, m, batch);
  hipError_t err;
  const int nbw = panel_width<T>(m);
  if ((err = allow_lds(gj_panel_kernel<T>, panel_lds_bytes<T>(m, nbw))) != hipSuccess) return err;
  T* cur = A;
  int ldc = lda;
  long long cs = bstride;
  T* nxt = s.buf;
  int ldn = m;
  long long ns = (long long)m * m;
  // 32 x 32 update tiles when 64 x 64 ones would give under 512 workgroups:
  // then a step lasts about as long as its look-ahead (FP64 m = 480 in four
  // matrices: 44 us per step with 256 tiles of 64 x 64, which fill the chip
  // at one per CU, against ~29 us with 900 of 32 x 32)
  const long long w64 = (long long)((m + 63) / 64) * ((m + 63) / 64) * batch;
  const bool tiles32 = w64 < 512;
  const int tiles = tiles32 ? (m + 31) / 32 : (m + 63) / 64;
  // register panels: rows <= 512 with 32 columns, FP64 rows <= 1024 with 16
  // columns; larger matrices keep the LDS panel
  const int reg = m <= 512 ? 1 : (m <= 1024 && sizeof(T) == sizeof(cd) ? 2 : 0);
  const int nb = !pivot ? kNB : (reg == 1 ? kNB : (reg == 2 ? kNB / 2 : nbw));
  static_assert(kNB == 32, "register panels hold 32 (16 x 2) columns");
  const int steps = (m + nb - 1) / nb;
  for (int s_ = 0; s_ < steps; ++s_) {
    const int k0 = s_ * nb;
    const int kb = std::min(nb, m - k0);
    const int* rho_prev = s_ ? s.rho[(s_ - 1) & 1] : nullptr;
    int* rho = s.rho[s_ & 1];
    // without row interchanges the pivot block of step s_ + 1 is inverted by
    // an extra workgroup of step s_'s update launch (from that launch's
    // inputs); the two inverses alternate between the halves of s.dinv
    T* dcur = pivot ? s.dinv : s.dinv + (size_t)(s_ & 1) * batch * kNB * kNB;
    T* dnext = (!pivot && s_ + 1 < steps) ? s.dinv + (size_t)((s_ + 1) & 1) * batch * kNB * kNB : nullptr;
    const int k1 = k0 + nb, kb1 = dnext ? std::min(nb, m - k1) : 0;
    if (!pivot) {
      if (s_ == 0)   // the first pivot block (and the identity row map)
        hipLaunchKernelGGL(gj_diag_kernel<T>, dim3(batch), dim3(64), 0, st, cur, m, ldc, cs, k0, kb, rho_prev, rho,
                           s.rowmap, dcur, flag, level);
    } else if (reg == 1)
      hipLaunchKernelGGL((gj_panel_reg_kernel<T, 8, 2>), dim3(batch), dim3(1024), 0, st, cur, m, ldc, cs, k0, kb,
                         rho_prev, rho, s.rowmap, s.dinv, flag, level);
    else if (reg == 2)
      hipLaunchKernelGGL((gj_panel_reg_kernel<T, 16, 1>), dim3(batch), dim3(1024), 0, st, cur, m, ldc, cs, k0,
                         kb, rho_prev, rho, s.rowmap, s.dinv, flag, level);
    else
      hipLaunchKernelGGL(gj_panel_kernel<T>, dim3(batch), dim3(kPanelThreads), panel_lds_bytes<T>(m - k0, kb), st,
                         cur, m, ldc, cs, k0, kb, rho_prev, rho, s.rowmap, s.dinv, flag, level);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    // the last step writes straight into A, columns permuted, when it can
    // (no row interchanges: the columns stay where they are)
    const bool last_into_A = (s_ == steps - 1) && nxt == A;
    const int* colmap = (last_into_A && pivot) ? rho : nullptr;
    int* check = pivot ? nullptr : flag;
    // the look-aheads are the launch's first workgroups, so that they start at
    // once even where the tiles fill the chip (tiles, not look-aheads, then
    // wait for free slots)
    const long long wgs = (long long)(tiles * tiles + (dnext ? 1 : 0)) * batch;
    if (wgs > INT_MAX) return hipErrorInvalidValue;
    if (tiles32)
      hipLaunchKernelGGL((gj_update_kernel<T, 32>), dim3((unsigned)wgs), dim3(256), 0, st, cur, ldc, cs, nxt, ldn,
                         ns, m, k0, kb, s.rowmap, dcur, colmap, check, level, dnext, k1, kb1);
    else
      hipLaunchKernelGGL((gj_update_kernel<T, 64>), dim3((unsigned)wgs), dim3(256), 0, st, cur, ldc, cs, nxt, ldn,
                         ns, m, k0, kb, s.rowmap, dcur, colmap, check, level, dnext, k1, kb1);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    std::swap(cur, nxt);
    std::swap(ldc, ldn);
    std::swap(cs, ns);
  }
  if (cur != A) {
    hipLaunchKernelGGL(permute_cols_kernel<T>, dim3((m + 255) / 256, m, batch), dim3(256), 0, st, cur, ldc, cs, A,
                       lda, bstride, m, pivot ? s.rho[(steps - 1) & 1] : nullptr);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

template <class T>
size_t inverse_scratch_bytes(int m, int batch) {
  if (m <= kSmallNoPivot) return 0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(sizeof(T) * (size_t)batch * m * m) + up(sizeof(T) * (size_t)2 * batch * kNB * kNB) +
         3 * up(sizeof(int) * (size_t)batch * m);
}

template <class T>
hipError_t zinverse(T* A, int m, int lda, long long bstride, int batch, void* scratch, int* flag,
                    int level, bool pivot, hipStream_t st) {
  if (m <= 0 || batch <= 0) return hipSuccess;
  // without interchanges the blocked path (one launch per 32-column step)
  // beats the register inverse's 2 us column steps from two block columns on
  if (m <= kSmallNoPivot || (m <= 64 && pivot)) {
    hipLaunchKernelGGL((inv_small_kernel<T, 4, 1>), dim3(batch), dim3(256), 0, st, A, m, lda, bstride, flag, level);
    return hipPeekAtLastError();
  }
  if (m <= 128 && pivot) {
    hipLaunchKernelGGL((inv_small_kernel<T, 16, 2>), dim3(batch), dim3(1024), 0, st, A, m, lda, bstride, flag, level);
    return hipPeekAtLastError();
  }
  return inverse_blocked<T>(A, m, lda, bstride, batch, scratch, flag, level, pivot, st);
}

template size_t inverse_scratch_bytes<cd>(int, int);
template size_t inverse_scratch_bytes<cf>(int, int);
template hipError_t zinverse<cd>(cd*, int, int, long long, int, void*, int*, int, bool, hipStream_t);
template hipError_t zinverse<cf>(cf*, int, int, long long, int, void*, int*, int, bool, hipStream_t);

}  // namespace hps
