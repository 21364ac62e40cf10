// Internal declarations of the solve-phase kernels (solve.hip).
#pragma once
#include "host.h"

namespace hps {

constexpr int kMaxCoarse = 32;     // maximum coarse GMRES steps
constexpr int kMaxDotBlocks = 512; // partial sums per vector in the two-stage dot

struct GemvArgs {
  int M, K, batch;
  Operand A;                 // M x K
  const cd* x; long long xs; // x[b], stride xs
  cd alpha;
  const cd* y0; long long y0s; cd beta;  // optional (y0 == null: ignored)
  cd* y; long long ys;
};

hipError_t skeleton_apply(const Geom& g, const cd* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st);
hipError_t rhs_build(const Geom& g, const cd* T, const cd* H, const cd* t, cd* rhs, hipStream_t st);
hipError_t zgemv(const GemvArgs& a, hipStream_t st);
hipError_t pair_gather(const Geom& g, int pairs, int which, IdxMap local, int len, const cd* vec,
                       cd* out, long long ostride, bool partner, hipStream_t st);
hipError_t pair_scatter(const Geom& g, int pairs, int which, IdxMap local, int len, const cd* in,
                        long long istride, cd* vec, bool partner, bool add, hipStream_t st);
hipError_t index_gather(const int* idx, int n, const cd* vec, cd* out, hipStream_t st);
hipError_t index_scatter(const int* idx, int n, const cd* in, cd* vec, hipStream_t st);
hipError_t vfill(cd* v, long long n, cd val, hipStream_t st);
// out = a x + b y
hipError_t axpby(cd a, const cd* x, cd b, const cd* y, cd* out, long long n, hipStream_t st);
hipError_t vcopy(const cd* src, cd* dst, long long n, hipStream_t st);
int dot_blocks(long long n);
// out[v] (+)= sum_i conj(V_v[i]) w[i], v < nvec; partial: nvec * dot_blocks(n) entries.
hipError_t multi_dot(const cd* V, long long vstride, int nvec, const cd* w, long long n, cd* partial,
                     cd* out, bool accumulate, hipStream_t st);
// w += sign * sum_v h[v] V_v
hipError_t multi_axpy(const cd* V, long long vstride, int nvec, const cd* h, cd* w, long long n, int sign,
                      hipStream_t st);
hipError_t normalize(const cd* w, const cd* nrm2, cd* out, long long n, cd* hout, hipStream_t st);
// Coarse k-step GMRES on compact coarse vectors of length n (one workgroup per
// launch).  V: (k+1) x n basis, H: (k+1) x k Hessenberg (ld k+1).
// start: V_0 = w / |w| with w = vec[idx], beta2 = |w|^2, H[0 .. hsize) = 0.
hipError_t coarse_start(const int* idx, int n, const cd* vec, cd* V, cd* H, int hsize, cd* beta2,
                        hipStream_t st);
// The product w = M_L v_j: either given (w), or, for the top pair, v_j minus the
// split-K partial sums of the two off-diagonal blocks (rows [0, m) from poff0,
// rows [m, 2m) from poff1; ns splits each, partial[po + s*m + r]).
struct CoarseW {
  const cd* w;
  const cd* part;
  long long poff0, poff1;
  int ns0, ns1;
  int m;
};
// Arnoldi step j (0 <= j < kMaxCoarse): two-pass classical Gram-Schmidt,
// V_{j+1} and column j of H.  wtmp: n scratch entries.
hipError_t coarse_arnoldi(cd* V, int n, int j, const CoarseW& src, cd* wtmp, cd* Hcol, hipStream_t st);
// y = argmin |beta e1 - H y| (Givens), vec[idx] = V y.
hipError_t coarse_finish(const cd* H, int k, const cd* beta2, const cd* V, int n, const int* idx, cd* vec,
                         hipStream_t st);

}  // namespace hps
