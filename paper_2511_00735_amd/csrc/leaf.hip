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
#include <algorithm>

#include "common.h"
#include "gj_small.h"
#include "host.h"

namespace hps {

namespace {

constexpr int kNB = 16;       // panel width of the blocked LU
constexpr int kThreads = 256;
constexpr int kStripes = 8;   // column stripes of the trailing update

struct Dims {
  int N, p, pp, nloc, ncol;
};

__device__ inline Dims dims_of(int N) {
  Dims d;
  d.N = N;
  d.p = N - 1;
  d.pp = d.p * d.p;
  d.nloc = d.pp + 4 * d.p;
  d.ncol = d.nloc + 2;
  return d;
}

// Entry (r, c) of the bordered real matrix K of one element.
// rows/cols: interior (i,j) -> (i-1)*p + (j-1); boundary l_k, r_k, b_k, t_k ->
// pp + side*p + (k-1); extra columns nloc, nloc+1 = Re/Im of bt.
__device__ inline double k_entry(const Dims& d, int r, int c, const double* D, const double* w,
                                 const double* Kr, const double* bnode, const double* snode,
                                 double kappa, double h) {
  const int N = d.N, p = d.p, pp = d.pp, N1 = N + 1;
  const double f = 2.0 / h;
  if (r < pp) {
    const int i = r / p + 1, j = r % p + 1;
    if (c >= d.nloc) {
      if (!snode) return 0.0;
      const double s = snode[2 * (i * N1 + j) + (c - d.nloc)];
      return 0.25 * h * h * w[i] * w[j] * s;
    }
    if (c < pp) {
      const int i2 = c / p + 1, j2 = c % p + 1;
      double v = 0.0;
      if (j == j2) v += Kr[i * N1 + i2] * w[j];
      if (i == i2) v += w[i] * Kr[j * N1 + j2];
      if (i == i2 && j == j2) {
        const double cc = kappa * kappa * (1.0 - bnode[i * N1 + j]);
        v -= 0.25 * h * h * cc * w[i] * w[j];
      }
      return v;
    }
    const int s = (c - pp) / p, k = (c - pp) % p + 1;
    if (s == 0) return (j == k) ? Kr[i * N1 + 0] * w[j] : 0.0;
    if (s == 1) return (j == k) ? Kr[i * N1 + N] * w[j] : 0.0;
    if (s == 2) return (i == k) ? w[i] * Kr[j * N1 + 0] : 0.0;
    return (i == k) ? w[i] * Kr[j * N1 + N] : 0.0;
  }
  if (c >= d.nloc) return 0.0;
  // normal-derivative row of boundary node (side s, index k)
  const int s = (r - pp) / p, k = (r - pp) % p + 1;
  const double sg = (s == 0 || s == 2) ? -f : f;    // outward normal sign
  const int dr = (s == 0 || s == 2) ? 0 : N;         // D row of the boundary node
  if (c < pp) {
    const int i2 = c / p + 1, j2 = c % p + 1;
    if (s < 2) return (j2 == k) ? sg * D[dr * N1 + i2] : 0.0;   // x-derivative along line j = k
    return (i2 == k) ? sg * D[dr * N1 + j2] : 0.0;              // y-derivative along line i = k
  }
  const int s2 = (c - pp) / p, k2 = (c - pp) % p + 1;
  if (k2 != k) return 0.0;
  if (s < 2) {
    if (s2 == 0) return sg * D[dr * N1 + 0];
    if (s2 == 1) return sg * D[dr * N1 + N];
    return 0.0;
  }
  if (s2 == 2) return sg * D[dr * N1 + 0];
  if (s2 == 3) return sg * D[dr * N1 + N];
  return 0.0;
}

// T = -I + 2 i eta (R + i eta I)^-1 and H from [R | -q] in the trailing rows of
// the reduced bordered matrix A; S: (4p)^2 complex LDS workspace.
__device__ void leaf_cayley(const LeafArgs& a, const double* A, cd* S, int* ipiv, cd* colk) {
  const Dims d = dims_of(a.N);
  const int m = 4 * d.p, nloc = d.nloc, npiv = d.pp;
  const int tid = threadIdx.x;
  const int G = a.G0 + blockIdx.x;
  const int q = G / a.E, e = G % a.E;
  const double eta = a.eta[q - a.q0];
  const double* snode = a.s_nodes[q - a.q0];
  for (int idx = tid; idx < m * m; idx += kThreads) {
    const int r = idx % m, c = idx / m;
    S[idx] = cmk(A[(size_t)(npiv + c) * nloc + npiv + r], r == c ? eta : 0.0);
  }
  __syncthreads();
  gj_inplace_small(S, m, ipiv, colk, a.flag);
  const int ix = e % a.n, iy = e / a.n;
  cd* Tout = a.T + ((size_t)q * a.E + morton_xy(ix, iy)) * m * m;
  const double te = 2.0 * eta;
  for (int idx = tid; idx < m * m; idx += kThreads) {
    const int r = idx % m, c = idx / m;
    const cd z = S[idx];
    Tout[idx] = cmk(-te * z.y - (r == c ? 1.0 : 0.0), te * z.x);
  }
  if (tid < m) {
    cd acc = cmk(0.0, 0.0);
    if (snode) {
      for (int c = 0; c < m; ++c) {
        const cd tc = cmk(A[(size_t)nloc * nloc + npiv + c], A[(size_t)(nloc + 1) * nloc + npiv + c]);
        acc = cfma(S[c * m + tid], tc, acc);
      }
    }
    a.H[(size_t)G * m + tid] = cmk(-te * acc.y, te * acc.x);
  }
}


// One element per workgroup: the bordered real partial LU, then the Cayley step.
__global__ __launch_bounds__(kThreads) void leaf_kernel(LeafArgs a) {
  extern __shared__ double lds[];
  __shared__ int piv_s[kNB];
  const Dims d = dims_of(a.N);
  const int nloc = d.nloc, ncol = d.ncol, npiv = d.pp;
  double* P = lds;                          // panel, nloc x kNB, column-major (ld nloc)
  double* U = lds + (size_t)nloc * kNB;     // U12 block, kNB x ncol, row-major (ld ncol)
  const int tid = threadIdx.x;
  const int G = a.G0 + blockIdx.x;
  const int q = G / a.E, e = G % a.E;
  const int N1 = a.N + 1;
  double* A = a.scratch + (size_t)blockIdx.x * nloc * ncol;
  const double* bnode = a.b_nodes[q - a.q0] + (size_t)e * N1 * N1;
  const double* sq = a.s_nodes[q - a.q0];
  const double* snode = sq ? sq + (size_t)e * 2 * N1 * N1 : nullptr;

  for (int idx = tid; idx < nloc * ncol; idx += kThreads) {
    const int r = idx % nloc, c = idx / nloc;
    A[idx] = k_entry(d, r, c, a.D, a.w, a.Kr, bnode, snode, a.kappa[q - a.q0], a.h);
  }
  __syncthreads();

  for (int k0 = 0; k0 < npiv; k0 += kNB) {
    const int kb = min(kNB, npiv - k0);
    const int rows = nloc - k0;
    for (int idx = tid; idx < rows * kb; idx += kThreads) {
      const int r = idx % rows, c = idx / rows;
      P[c * nloc + r] = A[(size_t)(k0 + c) * nloc + k0 + r];
    }
    __syncthreads();
    for (int c = 0; c < kb; ++c) {
      if (tid < 64) {
        double best = -1.0;
        int bi = c;
        for (int r = c + tid; r < npiv - k0; r += 64) {
          const double v = fabs(P[c * nloc + r]);
          if (v > best) { best = v; bi = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (tid == 0) {
          piv_s[c] = bi;
          if (!(best > 0.0)) atomicOr(a.flag, 2);
        }
      }
      __syncthreads();
      const int pr = piv_s[c];
      if (pr != c) {
        for (int j = tid; j < kb; j += kThreads) {
          const double t = P[j * nloc + c];
          P[j * nloc + c] = P[j * nloc + pr];
          P[j * nloc + pr] = t;
        }
        __syncthreads();
      }
      const double piv = P[c * nloc + c];
      const double inv = (piv != 0.0) ? 1.0 / piv : 0.0;
      for (int r = c + 1 + tid; r < rows; r += kThreads) {
        const double l = P[c * nloc + r] * inv;
        P[c * nloc + r] = l;
        for (int j = c + 1; j < kb; ++j) P[j * nloc + r] -= l * P[j * nloc + c];
      }
      __syncthreads();
    }
    // row interchanges on the trailing columns
    const int c0 = k0 + kb;
    for (int col = c0 + tid; col < ncol; col += kThreads) {
      double* Ac = A + (size_t)col * nloc + k0;
      for (int c = 0; c < kb; ++c) {
        const int pr = piv_s[c];
        if (pr != c) {
          const double t = Ac[c];
          Ac[c] = Ac[pr];
          Ac[pr] = t;
        }
      }
    }
    __syncthreads();
    // U12 = L11^-1 A12 (unit lower triangular forward substitution)
    const int nc = ncol - c0;
    for (int cc = tid; cc < nc; cc += kThreads) {
      const double* Ac = A + (size_t)(c0 + cc) * nloc + k0;
      double u[kNB];
#pragma unroll
      for (int r = 0; r < kNB; ++r) {
        if (r < kb) {
          double s = Ac[r];
#pragma unroll
          for (int q = 0; q < kNB; ++q)
            if (q < r) s -= P[q * nloc + r] * u[q];
          u[r] = s;
          U[r * ncol + cc] = s;
        }
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12, rows k0+kb.., cols c0..
    const int tr = rows - kb;
    const int items = tr * kStripes;
    for (int it = tid; it < items; it += kThreads) {
      const int r = it % tr, stripe = it / tr;
      double l[kNB];
#pragma unroll
      for (int q = 0; q < kNB; ++q) l[q] = (q < kb) ? P[q * nloc + kb + r] : 0.0;
      // four columns per iteration keep four loads in flight per thread
      int cc = stripe;
      for (; cc + 3 * kStripes < nc; cc += 4 * kStripes) {
        double* ap[4];
        double sv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ap[u] = A + (size_t)(c0 + cc + u * kStripes) * nloc + k0 + kb + r;
          sv[u] = *ap[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int q = 0; q < kNB; ++q) sv[u] -= l[q] * U[q * ncol + cc + u * kStripes];
          *ap[u] = sv[u];
        }
      }
      for (; cc < nc; cc += kStripes) {
        double* ap = A + (size_t)(c0 + cc) * nloc + k0 + kb + r;
        double s = *ap;
#pragma unroll
        for (int q = 0; q < kNB; ++q) s -= l[q] * U[q * ncol + cc];
        *ap = s;
      }
    }
    __syncthreads();
  }
  // the factorisation's LDS is free again: the Cayley step reuses it
  __shared__ int ipiv_c[64];
  __shared__ cd colk_c[64];
  leaf_cayley(a, A, reinterpret_cast<cd*>(lds), ipiv_c, colk_c);
}

}  // namespace

size_t leaf_scratch_doubles(int N, int count) {
  const int p = N - 1, nloc = p * p + 4 * p;
  return (size_t)count * nloc * (nloc + 2);
}

hipError_t leaf_build(const LeafArgs& a, hipStream_t st) {
  const int p = a.N - 1, nloc = p * p + 4 * p, ncol = nloc + 2;
  const size_t lds_lu = ((size_t)nloc * kNB + (size_t)kNB * ncol) * sizeof(double);
  const size_t lds_cayley = (size_t)(4 * p) * (4 * p) * sizeof(cd);
  const size_t lds = std::max(lds_lu, lds_cayley);
  hipError_t e0 = allow_lds(leaf_kernel, lds);
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(leaf_kernel, dim3(a.count), dim3(kThreads), lds, st, a);
  return hipPeekAtLastError();
}

}  // namespace hps
