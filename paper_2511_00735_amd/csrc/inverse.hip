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

template <class T>
__global__ __launch_bounds__(256) void inv_small_kernel(T* A, int m, int lda, long long bstride,
                                                        int* flag) {
  extern __shared__ char smem[];
  T* S = reinterpret_cast<T*>(smem);
  __shared__ int ipiv[64];
  __shared__ T colk[64];
  T* Ab = A + (long long)blockIdx.x * bstride;
  for (int base = 0; base < m * m; base += 4 * 256) {
    T v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + threadIdx.x;
      v[q] = idx < m * m ? Ab[(long long)(idx / m) * lda + idx % m] : cx<T>::make(0.0, 0.0);
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

template <class T>
struct BlockScratch {
  T* panel;   // [batch][m][nb]   (ld m)
  T* dinv;    // [batch][nb][nb]
  T* X;       // [batch][nb][m]   (nb x (m - kb), ld nb)
  T* Y;       // [batch][m][nb]   ((m - kb) x kb, ld m)
  int* ipiv;  // [batch][m]
};

template <class T>
inline BlockScratch<T> carve(void* base, int m, int batch) {
  BlockScratch<T> s;
  char* p = (char*)base;
  auto take = [&](size_t bytes) { char* q = p; p += (bytes + 255) & ~size_t(255); return q; };
  s.panel = (T*)take(sizeof(T) * (size_t)batch * m * kNB);
  s.dinv = (T*)take(sizeof(T) * (size_t)batch * kNB * kNB);
  s.X = (T*)take(sizeof(T) * (size_t)batch * kNB * m);
  s.Y = (T*)take(sizeof(T) * (size_t)batch * m * kNB);
  s.ipiv = (int*)take(sizeof(int) * (size_t)batch * m);
  return s;
}

// Panel LU (partial pivoting) of A[k0:m, k0:k0+kb], held in LDS: records the
// absolute pivot rows in ipiv[k0 .. k0+kb) and writes Dinv = (L11 U11)^-1, the
// inverse of the pivot block once its rows are swapped into place.
template <class T>
__global__ __launch_bounds__(256) void panel_lds_kernel(const T* A, int m, int lda, long long bstride,
                                                        int k0, int kb, int* ipiv, T* dinv, int* flag) {
  typedef typename cx<T>::real R;
  extern __shared__ char smem[];
  T* Pn = reinterpret_cast<T*>(smem);  // rows x kb, column-major (ld = rows)
  __shared__ int pr_s;
  __shared__ T Li[kNB * kNB];          // L11^-1 (unit lower), column-major kb x kb
  const T* Ab = A + (long long)blockIdx.x * bstride;
  int* ip = ipiv + (long long)blockIdx.x * m;
  const int rows = m - k0;
  const int tid = threadIdx.x;
  for (int base = 0; base < rows * kb; base += 4 * 256) {
    T v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = base + q * 256 + tid;
      v[q] = idx < rows * kb ? Ab[(long long)(k0 + idx / rows) * lda + k0 + idx % rows] : cx<T>::make(0.0, 0.0);
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
      R best = -1;
      int bi = c;
      for (int r = c + tid; r < rows; r += 64) {
        const R v = cabs2(Pn[c * rows + r]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const R ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (tid == 0) {
        pr_s = bi;
        ip[k0 + c] = k0 + bi;
        if (!(best > 0)) atomicOr(flag, 2);
      }
    }
    __syncthreads();
    const int pr = pr_s;
    if (pr != c) {
      for (int j = tid; j < kb; j += blockDim.x) {
        const T t = Pn[j * rows + c];
        Pn[j * rows + c] = Pn[j * rows + pr];
        Pn[j * rows + pr] = t;
      }
      __syncthreads();
    }
    const T d = Pn[c * rows + c];
    const T inv = cabs2(d) > 0 ? cinv(d) : cx<T>::make(0.0, 0.0);
    for (int r = c + 1 + tid; r < rows; r += blockDim.x) {
      const T l = cmul(Pn[c * rows + r], inv);
      Pn[c * rows + r] = l;
      for (int j = c + 1; j < kb; ++j) Pn[j * rows + r] = csub(Pn[j * rows + r], cmul(l, Pn[j * rows + c]));
    }
    __syncthreads();
  }
  // Li = L11^-1 column by column (unit lower triangular forward substitution)
  if (tid < kb) {
    const int j = tid;
    for (int i = 0; i < kb; ++i) {
      T v = (i == j) ? cx<T>::make(1.0, 0.0) : cx<T>::make(0.0, 0.0);
      for (int q = j; q < i; ++q) v = csub(v, cmul(Pn[q * rows + i], Li[j * kNB + q]));
      Li[j * kNB + i] = (i < j) ? cx<T>::make(0.0, 0.0) : v;
    }
  }
  __syncthreads();
  // Dinv = U11^-1 Li: back substitution on each column of Li
  T* Db = dinv + (long long)blockIdx.x * kNB * kNB;
  if (tid < kb) {
    const int j = tid;
    T x[kNB];
    for (int i = kb - 1; i >= 0; --i) {
      T v = Li[j * kNB + i];
      for (int q = i + 1; q < kb; ++q) v = csub(v, cmul(Pn[q * rows + i], x[q]));
      const T u = Pn[i * rows + i];
      x[i] = cabs2(u) > 0 ? cmul(v, cinv(u)) : cx<T>::make(0.0, 0.0);
    }
    for (int i = 0; i < kb; ++i) Db[j * kb + i] = x[i];
  }
}

// Panel width: the panel (m rows x nb complex) must fit in about 123 KB of LDS.
template <class T>
int panel_width(int m) {
  int nb = kNB;
  while (nb > 4 && (size_t)m * nb * sizeof(T) > 126 * 1024) nb /= 2;
  return nb;
}

// Apply the interchanges rows k0+j <-> ipiv[k0+j], j = 0..kb-1, in order, to all columns.
template <class T>
__global__ void swap_rows_kernel(T* A, int m, int lda, long long bstride, int k0, int kb,
                                 const int* ipiv) {
  T* Ab = A + (long long)blockIdx.y * bstride;
  const int* ip = ipiv + (long long)blockIdx.y * m;
  for (int col = blockIdx.x * blockDim.x + threadIdx.x; col < m; col += gridDim.x * blockDim.x) {
    T* Ac = Ab + (long long)col * lda;
    for (int j = 0; j < kb; ++j) {
      const int pr = ip[k0 + j];
      if (pr != k0 + j) {
        const T t = Ac[k0 + j];
        Ac[k0 + j] = Ac[pr];
        Ac[pr] = t;
      }
    }
  }
}

// Undo all row interchanges as column interchanges, last one first.
template <class T>
__global__ void unswap_cols_kernel(T* A, int m, int lda, long long bstride, const int* ipiv) {
  T* Ab = A + (long long)blockIdx.y * bstride;
  const int* ip = ipiv + (long long)blockIdx.y * m;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < m; row += gridDim.x * blockDim.x) {
    for (int k = m - 1; k >= 0; --k) {
      const int pr = ip[k];
      if (pr != k) {
        const T t = Ab[(long long)k * lda + row];
        Ab[(long long)k * lda + row] = Ab[(long long)pr * lda + row];
        Ab[(long long)pr * lda + row] = t;
      }
    }
  }
}

template <class T>
hipError_t inverse_blocked(T* A, int m, int lda, long long bstride, int batch, void* scratch,
                           int* flag, hipStream_t st) {
  BlockScratch<T> s = carve<T>(scratch, m, batch);
  const T one = cx<T>::make(1.0, 0.0), zero = cx<T>::make(0.0, 0.0), mone = cx<T>::make(-1.0, 0.0);
  hipError_t err;
  const int nbw = panel_width<T>(m);
  const size_t plds = (size_t)m * nbw * sizeof(T);
  if ((err = allow_lds(panel_lds_kernel<T>, plds)) != hipSuccess) return err;
  for (int k0 = 0; k0 < m; k0 += nbw) {
    const int kb = std::min(nbw, m - k0);
    hipLaunchKernelGGL(panel_lds_kernel<T>, dim3(batch), dim3(256), (size_t)(m - k0) * kb * sizeof(T), st, A,
                       m, lda, bstride, k0, kb, s.ipiv, s.dinv, flag);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(swap_rows_kernel<T>, dim3((m + 255) / 256, batch), dim3(256), 0, st, A, m, lda,
                       bstride, k0, kb, s.ipiv);
    if ((err = hipPeekAtLastError()) != hipSuccess) return err;
    const int mr = m - kb;  // rows / columns outside the block
    if (mr > 0) {
      // X = Dinv * A[P, ~C]   (kb x mr)
      GemmArgsT<T> g{};
      g.M = kb; g.N = mr; g.K = kb; g.batch = batch;
      g.A = OperandT<T>{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)};
      g.B = OperandT<T>{A, bstride, lda, im_off(k0), im_gap(0, k0, kb)};
      g.alpha = one; g.beta = zero;
      g.C = OperandT<T>{nullptr, 0, 0, im_off(0), im_off(0)};
      g.D = s.X; g.Dstride = (long long)kNB * m; g.ldd = kb; g.dr = im_off(0); g.dc = im_off(0);
      if ((err = zgemm(g, st)) != hipSuccess) return err;
      // Y = -A[~P, C] * Dinv   (mr x kb)
      GemmArgsT<T> y{};
      y.M = mr; y.N = kb; y.K = kb; y.batch = batch;
      y.A = OperandT<T>{A, bstride, lda, im_gap(0, k0, kb), im_off(k0)};
      y.B = OperandT<T>{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)};
      y.alpha = mone; y.beta = zero;
      y.C = OperandT<T>{nullptr, 0, 0, im_off(0), im_off(0)};
      y.D = s.Y; y.Dstride = (long long)m * kNB; y.ldd = m; y.dr = im_off(0); y.dc = im_off(0);
      if ((err = zgemm(y, st)) != hipSuccess) return err;
      // A[~P, ~C] -= A[~P, C] * X
      GemmArgsT<T> u{};
      u.M = mr; u.N = mr; u.K = kb; u.batch = batch;
      u.A = OperandT<T>{A, bstride, lda, im_gap(0, k0, kb), im_off(k0)};
      u.B = OperandT<T>{s.X, (long long)kNB * m, kb, im_off(0), im_off(0)};
      u.alpha = mone; u.beta = one;
      u.C = OperandT<T>{A, bstride, lda, im_gap(0, k0, kb), im_gap(0, k0, kb)};
      u.D = A; u.Dstride = bstride; u.ldd = lda; u.dr = im_gap(0, k0, kb); u.dc = im_gap(0, k0, kb);
      if ((err = zgemm(u, st)) != hipSuccess) return err;
      // A[P, ~C] = X ; A[~P, C] = Y
      if ((err = zcopy2d(kb, mr, batch, OperandT<T>{s.X, (long long)kNB * m, kb, im_off(0), im_off(0)}, one,
                         A, bstride, lda, im_off(k0), im_gap(0, k0, kb), st)) != hipSuccess)
        return err;
      if ((err = zcopy2d(mr, kb, batch, OperandT<T>{s.Y, (long long)m * kNB, m, im_off(0), im_off(0)}, one,
                         A, bstride, lda, im_gap(0, k0, kb), im_off(k0), st)) != hipSuccess)
        return err;
    }
    // A[P, C] = Dinv
    if ((err = zcopy2d(kb, kb, batch, OperandT<T>{s.dinv, (long long)kNB * kNB, kb, im_off(0), im_off(0)},
                       one, A, bstride, lda, im_off(k0), im_off(k0), st)) != hipSuccess)
      return err;
  }
  hipLaunchKernelGGL(unswap_cols_kernel<T>, dim3((m + 255) / 256, batch), dim3(256), 0, st, A, m, lda,
                     bstride, s.ipiv);
  return hipPeekAtLastError();
}

}  // namespace

template <class T>
size_t inverse_scratch_bytes(int m, int batch) {
  if (m <= 64) return 0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(sizeof(T) * (size_t)batch * m * kNB) + up(sizeof(T) * (size_t)batch * kNB * kNB) +
         up(sizeof(T) * (size_t)batch * kNB * m) + up(sizeof(T) * (size_t)batch * m * kNB) +
         up(sizeof(int) * (size_t)batch * m);
}

template <class T>
hipError_t zinverse(T* A, int m, int lda, long long bstride, int batch, void* scratch, int* flag,
                    hipStream_t st) {
  if (m <= 0 || batch <= 0) return hipSuccess;
  if (m <= 64) {
    hipError_t e0 = allow_lds(inv_small_kernel<T>, (size_t)m * m * sizeof(T));
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(inv_small_kernel<T>, dim3(batch), dim3(256), (size_t)m * m * sizeof(T), st, A, m,
                       lda, bstride, flag);
    return hipPeekAtLastError();
  }
  return inverse_blocked<T>(A, m, lda, bstride, batch, scratch, flag, st);
}

template size_t inverse_scratch_bytes<cd>(int, int);
template size_t inverse_scratch_bytes<cf>(int, int);
template hipError_t zinverse<cd>(cd*, int, int, long long, int, void*, int*, hipStream_t);
template hipError_t zinverse<cf>(cf*, int, int, long long, int, void*, int*, hipStream_t);

}  // namespace hps
