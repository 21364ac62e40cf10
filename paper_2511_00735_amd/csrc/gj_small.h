// In-LDS Gauss-Jordan inversion with partial pivoting for one small complex
// matrix per workgroup (m <= 64: one wave searches the pivot column, lane = row).
#pragma once
#include "common.h"

// S: m x m column-major in LDS (ld = m), inverted in place.
// ipiv: LDS int[m]; colk: LDS cd[m]; must be called by all threads of the block
// (blockDim.x >= 64).  Sets bit 2 of *flag on an exactly zero pivot.
template <class T>
__device__ inline void gj_inplace_small(T* S, int m, int* ipiv, T* colk, int* flag) {
  typedef typename cx<T>::real R;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int k = 0; k < m; ++k) {
    if (tid < 64) {
      R best = -1;
      int bi = k;
      for (int r = k + tid; r < m; r += 64) {
        const R v = cabs2(S[k * m + r]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const R ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (tid == 0) {
        ipiv[k] = bi;
        if (!(best > 0)) atomicOr(flag, 2);
      }
    }
    __syncthreads();
    const int pr = ipiv[k];
    if (pr != k) {
      for (int j = tid; j < m; j += nt) {
        const T t = S[j * m + k];
        S[j * m + k] = S[j * m + pr];
        S[j * m + pr] = t;
      }
      __syncthreads();
    }
    const T d = S[k * m + k];
    const T inv = (cabs2(d) > 0) ? cinv(d) : cx<T>::make(0.0, 0.0);
    __syncthreads();
    for (int j = tid; j < m; j += nt) {
      // row k scaled by 1/d (its diagonal becomes 1/d); column k saved
      const T v = (j == k) ? cx<T>::make(1.0, 0.0) : S[j * m + k];
      S[j * m + k] = cmul(v, inv);
      colk[j] = (j == k) ? cx<T>::make(0.0, 0.0) : S[k * m + j];
    }
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += nt) {
      const int i = idx % m, j = idx / m;
      if (i == k) continue;
      const T base = (j == k) ? cx<T>::make(0.0, 0.0) : S[j * m + i];
      const T f = colk[i];
      const T rk = S[j * m + k];
      S[j * m + i] = csub(base, cmul(f, rk));
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last one first
  for (int i = tid; i < m; i += nt) {
    for (int k = m - 1; k >= 0; --k) {
      const int pr = ipiv[k];
      if (pr != k) {
        const T t = S[k * m + i];
        S[k * m + i] = S[pr * m + i];
        S[pr * m + i] = t;
      }
    }
  }
  __syncthreads();
}
