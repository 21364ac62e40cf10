// Batched in-place inversion of complex FP64 matrices by Gauss-Jordan
// elimination with partial pivoting.
//
// m <= 64: the whole matrix sits in LDS, one workgroup per matrix.
// m  > 64: blocked Gauss-Jordan.  For each block column C = [k0, k0+nb):
//   1. partial-pivoting LU of the panel A[k0:m, C] (a copy) selects nb pivot
//      rows among the rows not yet used as pivots;
//   2. those rows are swapped into P = [k0, k0+nb);
//   3. Dinv = A[P, C]^-1 (small in-LDS Gauss-Jordan);
//   4. X = Dinv A[P, ~C],  Y = -A[~P, C] Dinv,  A[~P, ~C] -= A[~P, C] X,
//      then A[P, ~C] = X, A[~P, C] = Y, A[P, C] = Dinv  (MFMA GEMMs);
// and finally the row interchanges are undone as column interchanges in
// reverse order.  Work: m^3 complex multiply-adds, nearly all in GEMMs.
#include "common.h"
#include "gj_small.h"
#include "host.h"

namespace hps {

namespace {

constexpr int kNB = 32;

__global__ __launch_bounds__(256) void inv_small_kernel(cd* A, int m, int lda, long long bstride,
                                                        int* flag) {
  extern __shared__ cd S[];
  __shared__ int ipiv[64];
  __shared__ cd colk[64];
  cd* Ab = A + (long long)blockIdx.x * bstride;
  for (int base = 0; base < m * m; base += 4 * 256) {
    cd v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + threadIdx.x;
      v[q] = idx < m * m ? Ab[(long long)(idx / m) * lda + idx % m] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + threadIdx.x;
      if (idx < m * m) S[idx] = v[q];
    }
  }
  __syncthreads();
  gj_inplace_small(S, m, ipiv, colk, flag);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    const int r = idx % m, c = idx / m;
    Ab[(long long)c * lda + r] = S[idx];
  }
}

struct BlockScratch {
  cd* panel;  // [batch][m][nb]   (ld m)
  cd* dinv;   // [batch][nb][nb]
  cd* X;      // [batch][nb][m]   (nb x (m - kb), ld nb)
  cd* Y;      // [batch][m][nb]   ((m - kb) x kb, ld m)
  int* ipiv;  // [batch][m]
};

inline BlockScratch carve(void* base, int m, int batch) {
  BlockScratch s;
  char* p = (char*)base;
  auto take = [&](size_t bytes) { char* q = p; p += (bytes + 255) & ~size_t(255); return q; };
  s.panel = (cd*)take(sizeof(cd) * (size_t)batch * m * kNB);
  s.dinv = (cd*)take(sizeof(cd) * (size_t)batch * kNB * kNB);
  s.X = (cd*)take(sizeof(cd) * (size_t)batch * kNB * m);
  s.Y = (cd*)take(sizeof(cd) * (size_t)batch * m * kNB);
  s.ipiv = (int*)take(sizeof(int) * (size_t)batch * m);
  return s;
}

// Panel LU (partial pivoting) of A[k0:m, k0:k0+kb], held in LDS: records the
// absolute pivot rows in ipiv[k0 .. k0+kb) and writes Dinv = (L11 U11)^-1, the
// inverse of the pivot block once its rows are swapped into place.
__global__ __launch_bounds__(256) void panel_lds_kernel(const cd* A, int m, int lda, long long bstride,
                                                        int k0, int kb, int* ipiv, cd* dinv, int* flag) {
  extern __shared__ cd Pn[];          // rows x kb, column-major (ld = rows)
  __shared__ int pr_s;
  __shared__ cd Li[kNB * kNB];        // L11^-1 (unit lower), column-major kb x kb
  const cd* Ab = A + (long long)blockIdx.x * bstride;
  int* ip = ipiv + (long long)blockIdx.x * m;
  const int rows = m - k0;
  const int tid = threadIdx.x;
  for (int base = 0; base < rows * kb; base += 4 * 256) {
    cd v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + tid;
      v[q] = idx < rows * kb ? Ab[(long long)(k0 + idx / rows) * lda + k0 + idx % rows] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + tid;
      if (idx < rows * kb) Pn[(idx / rows) * rows + idx % rows] = v[q];
    }
  }
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    if (tid < 64) {
      double best = -1.0;
      int bi = c;
      for (int r = c + tid; r < rows; r += 64) {
        const double v = cabs2(Pn[c * rows + r]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (tid == 0) {
        pr_s = bi;
        ip[k0 + c] = k0 + bi;
        if (!(best > 0.0)) atomicOr(flag, 2);
      }
    }
    __syncthreads();
    const int pr = pr_s;
    if (pr != c) {
      for (int j = tid; j < kb; j += blockDim.x) {
        const cd t = Pn[j * rows + c];
        Pn[j * rows + c] = Pn[j * rows + pr];
        Pn[j * rows + pr] = t;
      }
      __syncthreads();
    }
    const cd d = Pn[c * rows + c];
    const cd inv = cabs2(d) > 0.0 ? cinv(d) : cmk(0.0, 0.0);
    for (int r = c + 1 + tid; r < rows; r += blockDim.x) {
      const cd l = cmul(Pn[c * rows + r], inv);
      Pn[c * rows + r] = l;
      for (int j = c + 1; j < kb; ++j) Pn[j * rows + r] = csub(Pn[j * rows + r], cmul(l, Pn[j * rows + c]));
    }
    __syncthreads();
  }
  // Li = L11^-1 column by column (unit lower triangular forward substitution)
  if (tid < kb) {
    const int j = tid;
    for (int i = 0; i < kb; ++i) {
      cd v = (i == j) ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
      for (int q = j; q < i; ++q) v = csub(v, cmul(Pn[q * rows + i], Li[j * kNB + q]));
      Li[j * kNB + i] = (i < j) ? cmk(0.0, 0.0) : v;
    }
  }
  __syncthreads();
  // Dinv = U11^-1 Li: back substitution on each column of Li
  cd* Db = dinv + (long long)blockIdx.x * kNB * kNB;
  if (tid < kb) {
    const int j = tid;
    cd x[kNB];
    for (int i = kb - 1; i >= 0; --i) {
      cd v = Li[j * kNB + i];
      for (int q = i + 1; q < kb; ++q) v = csub(v, cmul(Pn[q * rows + i], x[q]));
      const cd u = Pn[i * rows + i];
      x[i] = cabs2(u) > 0.0 ? cmul(v, cinv(u)) : cmk(0.0, 0.0);
    }
    for (int i = 0; i < kb; ++i) Db[j * kb + i] = x[i];
  }
}

// Panel width: the panel (m rows x nb complex) must fit in about 123 KB of LDS.
int panel_width(int m) {
  int nb = kNB;
  while (nb > 4 && (size_t)m * nb * sizeof(cd) > 126 * 1024) nb /= 2;
  return nb;
}

// Apply the interchanges rows k0+j <-> ipiv[k0+j], j = 0..kb-1, in order, to all columns.
__global__ void swap_rows_kernel(cd* A, int m, int lda, long long bstride, int k0, int kb,
                                 const int* ipiv) {
  cd* Ab = A + (long long)blockIdx.y * bstride;
  const int* ip = ipiv + (long long)blockIdx.y * m;
  for (int col = blockIdx.x * blockDim.x + threadIdx.x; col < m; col += gridDim.x * blockDim.x) {
    cd* Ac = Ab + (long long)col * lda;
    for (int j = 0; j < kb; ++j) {
      const int pr = ip[k0 + j];
      if (pr != k0 + j) {
        const cd t = Ac[k0 + j];
        Ac[k0 + j] = Ac[pr];
        Ac[pr] = t;
      }
    }
  }
}

// Undo all row interchanges as column interchanges, last one first.
__global__ void unswap_cols_kernel(cd* A, int m, int lda, long long bstride, const int* ipiv) {
  cd* Ab = A + (long long)blockIdx.y * bstride;
  const int* ip = ipiv + (long long)blockIdx.y * m;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < m; row += gridDim.x * blockDim.x) {
    for (int k = m - 1; k >= 0; --k) {
      const int pr = ip[k];
      if (pr != k) {
        const cd t = Ab[(long long)k * lda + row];
        Ab[(long long)k * lda + row] = Ab[(long long)pr * lda + row];
        Ab[(long long)pr * lda + row] = t;
      }
    }
  }
}

hipError_t inverse_blocked(cd* A, int m, int lda, long long bstride, int batch, void* scratch,
                           int* flag, hipStream_t st) {
  BlockScratch s = carve(scratch, m, batch);
  const cd one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0), mone = cmk(-1.0, 0.0);
  hipError_t err;
  const int nbw = panel_width(m);
  const size_t plds = (size_t)m * nbw * sizeof(cd);
  if ((err = allow_lds(panel_lds_kernel, plds)) != hipSuccess) return err;
  for (int k0 = 0; k0 < m; k0 += nbw) {
    const int kb = std::min(nbw, m - k0);
    hipLaunchKernelGGL(panel_lds_kernel, dim3(batch), dim3(256), (size_t)(m - k0) * kb * sizeof(cd), st, A,
                       m, lda, bstride, k0, kb, s.ipiv, s.dinv, flag);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(swap_rows_kernel, dim3((m + 255) / 256, batch), dim3(256), 0, st, A, m, lda,
                       bstride, k0, kb, s.ipiv);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    const int mr = m - kb;  // rows / columns outside the block
    if (mr > 0) {
      // X = Dinv * A[P, ~C]   (kb x mr)
      GemmArgs g{};
      g.M = kb; g.N = mr; g.K = kb; g.batch = batch;
      g.A = Operand{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)};
      g.B = Operand{A, bstride, lda, im_off(k0), im_gap(0, k0, kb)};
      g.alpha = one; g.beta = zero;
      g.C = Operand{nullptr, 0, 0, im_off(0), im_off(0)};
      g.D = s.X; g.Dstride = (long long)kNB * m; g.ldd = kb; g.dr = im_off(0); g.dc = im_off(0);
      if ((err = zgemm(g, st)) != hipSuccess) return err;
      // Y = -A[~P, C] * Dinv   (mr x kb)
      GemmArgs y{};
      y.M = mr; y.N = kb; y.K = kb; y.batch = batch;
      y.A = Operand{A, bstride, lda, im_gap(0, k0, kb), im_off(k0)};
      y.B = Operand{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)};
      y.alpha = mone; y.beta = zero;
      y.C = Operand{nullptr, 0, 0, im_off(0), im_off(0)};
      y.D = s.Y; y.Dstride = (long long)m * kNB; y.ldd = m; y.dr = im_off(0); y.dc = im_off(0);
      if ((err = zgemm(y, st)) != hipSuccess) return err;
      // A[~P, ~C] -= A[~P, C] * X
      GemmArgs u{};
      u.M = mr; u.N = mr; u.K = kb; u.batch = batch;
      u.A = Operand{A, bstride, lda, im_gap(0, k0, kb), im_off(k0)};
      u.B = Operand{s.X, (long long)kNB * m, kb, im_off(0), im_off(0)};
      u.alpha = mone; u.beta = one;
      u.C = Operand{A, bstride, lda, im_gap(0, k0, kb), im_gap(0, k0, kb)};
      u.D = A; u.Dstride = bstride; u.ldd = lda; u.dr = im_gap(0, k0, kb); u.dc = im_gap(0, k0, kb);
      if ((err = zgemm(u, st)) != hipSuccess) return err;
      // A[P, ~C] = X ; A[~P, C] = Y
      if ((err = zcopy2d(kb, mr, batch, Operand{s.X, (long long)kNB * m, kb, im_off(0), im_off(0)}, one,
                         A, bstride, lda, im_off(k0), im_gap(0, k0, kb), st)) != hipSuccess)
        return err;
      if ((err = zcopy2d(mr, kb, batch, Operand{s.Y, (long long)m * kNB, m, im_off(0), im_off(0)}, one,
                         A, bstride, lda, im_gap(0, k0, kb), im_off(k0), st)) != hipSuccess)
        return err;
    }
    // A[P, C] = Dinv
    if ((err = zcopy2d(kb, kb, batch, Operand{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)},
                       one, A, bstride, lda, im_off(k0), im_off(k0), st)) != hipSuccess)
      return err;
  }
  hipLaunchKernelGGL(unswap_cols_kernel, dim3((m + 255) / 256, batch), dim3(256), 0, st, A, m, lda,
                     bstride, s.ipiv);
  return hipPeekAtLastError();
}

}  // namespace

size_t inverse_scratch_bytes(int m, int batch) {
  if (m <= 64) return 0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(sizeof(cd) * (size_t)batch * m * kNB) + up(sizeof(cd) * (size_t)batch * kNB * kNB) +
         up(sizeof(cd) * (size_t)batch * kNB * m) + up(sizeof(cd) * (size_t)batch * m * kNB) +
         up(sizeof(int) * (size_t)batch * m);
}

hipError_t zinverse(cd* A, int m, int lda, long long bstride, int batch, void* scratch, int* flag,
                    hipStream_t st) {
  if (m <= 0 || batch <= 0) return hipSuccess;
  if (m <= 64) {
    hipError_t e0 = allow_lds(inv_small_kernel, (size_t)m * m * sizeof(cd));
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(inv_small_kernel, dim3(batch), dim3(256), (size_t)m * m * sizeof(cd), st, A, m,
                       lda, bstride, flag);
    return hipPeekAtLastError();
  }
  return inverse_blocked(A, m, lda, bstride, batch, scratch, flag, st);
}

}  // namespace hps
