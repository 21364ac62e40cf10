// In-LDS Gauss-Jordan inversion with partial pivoting for one small complex
// matrix per workgroup (m <= 64).
#pragma once
#include "common.h"
#include "pivot.h"

// S: m x m column-major in LDS (ld = m), inverted in place.  LDS workspace:
// ipiv int[64], colk and rowk T[64], kw u64[16].  Called by every thread of the
// block; blockDim.x is a multiple of 64 and at most 1024.  Sets bit 2 of *flag
// on a zero pivot.
//
// Each step k takes two barriers: (1) the row interchange k <-> pr on every
// column but k, staging the pivot row and column k; (2) the elimination,
// thread (row i = tid % 64, columns j = tid / 64 + G*t), which also forms the
// next column's pivot candidates and reduces them per wavefront (DPP arg-max).
template <class T>
__device__ inline void gj_inplace_small(T* S, int m, int* ipiv, T* colk, T* rowk, unsigned long long* kw,
                                        int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x, nw = nt >> 6;
  const int i = tid & 63, g = tid >> 6, G = nw;
  unsigned long long best = (g == 0 && i < m) ? hps::pivot_key(cabs2(S[i]), i) : 0ull;
  best = hps::wave_max_key(best);
  if ((tid & 63) == 0) kw[g] = best;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    unsigned long long kk = 0;
    for (int w = 0; w < nw; ++w) kk = max(kk, kw[w]);
    int pr = hps::pivot_row(kk);
    const bool bad = (kk >> 32) <= 1u || pr < k || pr >= m;
    if (bad) pr = k;
    const T d = S[k * m + pr];
    for (int j = tid; j < m; j += nt) {
      if (j == k) continue;
      const T u = S[j * m + pr];
      if (pr != k) S[j * m + pr] = S[j * m + k];
      rowk[j] = u;
    }
    for (int r = tid; r < m; r += nt) {
      const int src = (r == pr) ? k : r;
      colk[r] = (r == k) ? cx<T>::make(0.0, 0.0) : S[k * m + src];
    }
    if (tid == 0) {
      ipiv[k] = pr;
      if (bad) atomicOr(flag, 2);
    }
    __syncthreads();
    const T inv = (cabs2(d) > 0) ? cinv(d) : cx<T>::make(0.0, 0.0);
    best = 0;
    if (i < m) {
      const T ci = colk[i];
      for (int j = g; j < m; j += G) {
        T v;
        if (i == k) {
          v = (j == k) ? inv : cmul(rowk[j], inv);
        } else if (j == k) {
          v = csub(cx<T>::make(0.0, 0.0), cmul(ci, inv));
        } else {
          v = csub(S[j * m + i], cmul(ci, cmul(rowk[j], inv)));
        }
        S[j * m + i] = v;
        if (j == k + 1 && i > k) best = max(best, hps::pivot_key(cabs2(v), i));
      }
    }
    best = hps::wave_max_key(best);
    if ((tid & 63) == 0) kw[g] = best;
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last one first
  for (int r = tid; r < m; r += nt) {
    for (int k = m - 1; k >= 0; --k) {
      const int pr = ipiv[k];
      if (pr != k) {
        const T t = S[k * m + r];
        S[k * m + r] = S[pr * m + r];
        S[pr * m + r] = t;
      }
    }
  }
  __syncthreads();
}
