// Internal declarations of the solve-phase kernels (solve.hip).
#pragma once
#include "host.h"

namespace hps {

constexpr int kMaxCoarse = 32;     // maximum coarse GMRES steps
constexpr int kMaxDotBlocks = 512; // partial sums per vector in the two-stage dot

// For nq problems of a group: their level-l boxes follow each other in T and
// their canonical vectors in gin / out.
hipError_t skeleton_apply(const Geom& g, const cd* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st, int nq = 1);
// The same with complex FP32 box maps (FP64 vectors and arithmetic).
hipError_t skeleton_apply(const Geom& g, const cf* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st, int nq = 1);
hipError_t rhs_build(const Geom& g, const cd* T, const cd* H, const cd* t, cd* rhs, hipStream_t st);
// nq lists of n indices one after the other: out[q*ostride + r] = vec[idx[q*n + r]]
// (ostride 0: n) and vec[idx[q*n + r]] = in[q*istride + r].
hipError_t index_gather(const int* idx, int n, const cd* vec, cd* out, hipStream_t st, int nq = 1,
                        long long ostride = 0);
hipError_t index_scatter(const int* idx, int n, const cd* in, cd* vec, hipStream_t st, int nq = 1,
                         long long istride = 0);
hipError_t vfill(cd* v, long long n, cd val, hipStream_t st);
// out = a x + b y
hipError_t axpby(cd a, const cd* x, cd b, const cd* y, cd* out, long long n, hipStream_t st);
hipError_t vcopy(const cd* src, cd* dst, long long n, hipStream_t st);
// dst = src with src displaced by (*isrc) * stride or dst by (*idst) * stride
// (indices held on the device; null: none).
hipError_t vcopy_at(const cd* src, cd* dst, long long n, const int* isrc, const int* idst, long long stride,
                    hipStream_t st);
// *c = value, or *c += value, on the stream (one tiny launch, no memset).
hipError_t counter_set(int* c, int value, hipStream_t st);
hipError_t counter_add(int* c, int value, hipStream_t st);
// dst = src and zero = 0 (n entries each) in one launch.
hipError_t vcopy_zero(const cd* src, cd* dst, cd* zero, long long n, hipStream_t st);
int dot_blocks(long long n);
// Vectors of nq problems are stored one after the other (segments of n).
// out[q*ostride + v] (+)= sum_i conj(V_v[q*n + i]) w[q*n + i], v < nvec;
// partial: nq * (nvec + 1) * dot_blocks(n) entries.  With nvdev set the
// vector count is read on the device, *nvdev + 1, and nvec is the largest it
// may be (the launch's size; entries v > *nvdev of out are left as they were).
// With selfout set, conj(w) . w of problem q also goes to selfout[q*ostride].
hipError_t multi_dot(const cd* V, long long vstride, int nvec, const cd* w, long long n, cd* partial,
                     cd* out, bool accumulate, hipStream_t st, int nq = 1, long long ostride = 0,
                     const int* nvdev = nullptr, cd* selfout = nullptr);
// Second Gram-Schmidt update and normalisation in one pass (V orthonormal):
// out[q*n + i] = (w - sum_v h[q*hstride + v] V_v)[q*n + i] / r_q with
// r_q^2 = Re nrm2[q*nstride] - sum_v |h[q*hstride + v]|^2 (nrm2 holding |w|^2),
// hout[q*houtstride] = r_q; nvdev and jdev (out displaced by (*jdev + 1) *
// jstride) as for multi_axpy and normalize.
hipError_t axpy_normalize(const cd* V, long long vstride, int nvec, const cd* h, long long hstride, const cd* w,
                          long long n, const cd* nrm2, long long nstride, cd* out, cd* hout, long long houtstride,
                          hipStream_t st, int nq = 1, const int* nvdev = nullptr, const int* jdev = nullptr,
                          long long jstride = 0);
// w[q*n + i] += sign * sum_v h[q*hstride + v] V_v[q*n + i] (nvdev as above)
hipError_t multi_axpy(const cd* V, long long vstride, int nvec, const cd* h, cd* w, long long n, int sign,
                      hipStream_t st, int nq = 1, long long hstride = 0, const int* nvdev = nullptr);
// out[q*n + i] = w[q*n + i] / sqrt(Re nrm2[q*nstride]); hout[q*hstride] = the
// norm.  With jdev set, out is displaced by (*jdev + 1) * jstride.
hipError_t normalize(const cd* w, const cd* nrm2, cd* out, long long n, cd* hout, hipStream_t st, int nq = 1,
                     long long nstride = 0, long long hstride = 0, const int* jdev = nullptr,
                     long long jstride = 0);
// Coarse k-step GMRES on compact coarse vectors of length n, one workgroup per
// problem q < nq.  Problem q's basis is V + q*vq ((k+1) x n), its Hessenberg
// H + q*hsize ((k+1) x k, ld k+1), its index list idx + q*n, beta2[q].
// start: V_0 = w / |w| with w = vec[idx], beta2 = |w|^2, H = 0.
hipError_t coarse_start(const int* idx, int n, const cd* vec, cd* V, long long vq, cd* H, int hsize, cd* beta2,
                        int nq, hipStream_t st);
// The product w = M_L v_j: either given (w, problem q at w + q*n), or, for the
// top pair, v_j minus the split-K partial sums of the two off-diagonal blocks
// (rows [0, m) from poff0, rows [m, 2m) from poff1; ns splits each, batch nb =
// the number of problems; partial[po + (s*nb + q)*m + r]).
struct CoarseW {
  const cd* w;
  const cd* part;
  long long poff0, poff1;
  int ns0, ns1;
  int m, nb;
};
// The k-step GMRES's start and end folded into its first and last Arnoldi
// steps (register kernels only: coarse_fast_ok(n, k)): step 0 gathers
// w0 = vin[idx] itself (the product src was formed from w0, not from V_0),
// writes V_0 = w0/|w0|, beta2 and H = 0; step k-1 solves the least squares
// and scatters vout[idx] = V y instead of forming V_k (coarse_start and
// coarse_finish are then not launched).
struct CoarseEnds {
  const int* idx;     // [nq][n] coarse index lists
  const cd* vin;      // gathered at step 0
  cd* vout;           // scattered at step k-1
  cd* beta2;          // [nq]
  int k;
};
bool coarse_fast_ok(int n, int k);
// Arnoldi step j (0 <= j < kMaxCoarse): two-pass classical Gram-Schmidt,
// V_{j+1} and column j of H (Hcol = H + j*(k+1), per problem + q*hsize).
// wtmp: nq * n scratch entries.
hipError_t coarse_arnoldi(cd* V, int n, long long vq, int j, const CoarseW& src, cd* wtmp, cd* Hcol, int hsize,
                          int nq, hipStream_t st, const CoarseEnds* ends = nullptr);
// y = argmin |beta e1 - H y| (Givens), vec[idx] = V y, per problem.
hipError_t coarse_finish(const cd* H, int k, int hsize, const cd* beta2, const cd* V, int n, long long vq,
                         const int* idx, cd* vec, int nq, hipStream_t st);

}  // namespace hps
