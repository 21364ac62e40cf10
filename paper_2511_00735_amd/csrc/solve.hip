// Solve-phase kernels: skeleton matvec M_l g (Sec. 3.2), right-hand side,
// the per-level pieces of the multigrid V-cycle (Sec. 4.3), and deterministic
// reductions for the Krylov methods.  All of them stream stored operators or
// vectors once (HBM-bound); reductions use a fixed two-stage tree, no atomics,
// so results are bitwise reproducible.
#include "common.h"
#include "solve.h"

namespace hps {

namespace {

constexpr int kRows = 64;  // rows per workgroup of the streaming matvec kernels

// out[Pi(s)] = g[Pi(s)] - (T^B g_B)[s] for every interior boundary slot s of
// every level-l box B.  Grid (boxes, ceil(b / 64)), 64 threads.
__global__ __launch_bounds__(kRows) void skeleton_apply_kernel(Geom g, const cd* T, const cd* gin,
                                                               cd* out, int zero_physical) {
  extern __shared__ cd gB[];
  const int j = blockIdx.x;
  const int r0 = blockIdx.y * kRows;
  int bx, by;
  box_xy(g, j, bx, by);
  const int b = g.b;
  const int tid = threadIdx.x;
  const int r = r0 + tid;
  bool phys_side[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) phys_side[s] = side_physical(g, bx, by, s);
  // rows of this chunk that lie on physical sides produce nothing
  bool any = false;
  for (int s = 0; s < 4; ++s)
    if (!phys_side[s] && g.off[s] < r0 + kRows && g.off[s + 1] > r0) any = true;
  if (!any && !zero_physical) return;
  for (int k = tid; k < b; k += kRows) {
    const int s = side_of(g, k);
    gB[k] = phys_side[s] ? cmk(0.0, 0.0) : gin[box_slot(g, bx, by, k)];
  }
  __syncthreads();
  if (r >= b) return;
  const int sr = side_of(g, r);
  const int slot = box_slot(g, bx, by, r);
  if (phys_side[sr]) {
    if (zero_physical) out[slot] = cmk(0.0, 0.0);
    return;
  }
  const cd* Tb = T + (long long)j * b * b;
  cd acc = cmk(0.0, 0.0);
  for (int s = 0; s < 4; ++s) {
    if (phys_side[s]) continue;
    const int c1 = g.off[s + 1];
    int c = g.off[s];
    for (; c + 3 < c1; c += 4) {
      const cd t0 = Tb[(long long)c * b + r], t1 = Tb[(long long)(c + 1) * b + r];
      const cd t2 = Tb[(long long)(c + 2) * b + r], t3 = Tb[(long long)(c + 3) * b + r];
      acc = cfma(t0, gB[c], acc);
      acc = cfma(t1, gB[c + 1], acc);
      acc = cfma(t2, gB[c + 2], acc);
      acc = cfma(t3, gB[c + 3], acc);
    }
    for (; c < c1; ++c) acc = cfma(Tb[(long long)c * b + r], gB[c], acc);
  }
  const int ps = slot_partner(g.n, g.p, slot);
  out[ps] = csub(gin[ps], acc);
}

// Level-1 right-hand side: rhs[Pi(s)] = (H^e + T^e t_phys)[s]; physical slots 0.
__global__ __launch_bounds__(kRows) void rhs_kernel(Geom g, const cd* T, const cd* H, const cd* t,
                                                    cd* rhs) {
  __shared__ cd tl[256];
  const int e = blockIdx.x;
  const int n = g.n, p = g.p, m = 4 * p;
  const int ix = e % n, iy = e / n;
  const cd* Te = T + (long long)morton_xy(ix, iy) * m * m;
  bool phys[4] = {ix == 0, ix == n - 1, iy == 0, iy == n - 1};
  for (int k = threadIdx.x; k < m; k += kRows) {
    const int s = k / p;
    tl[k] = phys[s] ? t[(long long)e * m + k] : cmk(0.0, 0.0);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < m; r += kRows) {
    const int s = r / p;
    const int slot = e * m + r;
    if (phys[s]) {
      rhs[slot] = cmk(0.0, 0.0);
      continue;
    }
    cd acc = H ? H[(long long)e * m + r] : cmk(0.0, 0.0);
    for (int c = 0; c < m; ++c)
      if (phys[c / p]) acc = cfma(Te[(long long)c * m + r], tl[c], acc);
    rhs[slot_partner(n, p, slot)] = acc;
  }
}

// y[b] = alpha A_b x[b] + beta y0[b];  A_b addressed as an Operand (M x K).
__global__ __launch_bounds__(kRows) void zgemv_kernel(GemvArgs a) {
  extern __shared__ cd xs[];
  const int b = blockIdx.y;
  const cd* x = a.x + (long long)b * a.xs;
  for (int k = threadIdx.x; k < a.K; k += kRows) xs[k] = x[k];
  __syncthreads();
  const int r = blockIdx.x * kRows + threadIdx.x;
  if (r >= a.M) return;
  const cd* Ab = a.A.base + (long long)b * a.A.bstride;
  const int row = imap(a.A.r, r);
  cd acc = cmk(0.0, 0.0);
  int k = 0;
  for (; k + 3 < a.K; k += 4) {
    const cd t0 = Ab[(long long)imap(a.A.c, k) * a.A.ld + row];
    const cd t1 = Ab[(long long)imap(a.A.c, k + 1) * a.A.ld + row];
    const cd t2 = Ab[(long long)imap(a.A.c, k + 2) * a.A.ld + row];
    const cd t3 = Ab[(long long)imap(a.A.c, k + 3) * a.A.ld + row];
    acc = cfma(t0, xs[k], acc);
    acc = cfma(t1, xs[k + 1], acc);
    acc = cfma(t2, xs[k + 2], acc);
    acc = cfma(t3, xs[k + 3], acc);
  }
  for (; k < a.K; ++k) acc = cfma(Ab[(long long)imap(a.A.c, k) * a.A.ld + row], xs[k], acc);
  cd out = cmul(a.alpha, acc);
  if (a.y0) out = cfma(a.beta, a.y0[(long long)b * a.y0s + r], out);
  a.y[(long long)b * a.ys + r] = out;
}

// Per pair j (box 2j + which at level g.level): out[j][i] = vec[slot(k_i)]
// (or vec at the partner slot), zero if k_i lies on a physical side.
__global__ void pair_gather_kernel(Geom g, int which, IdxMap local, int len, const cd* vec, cd* out,
                                   long long ostride, int use_partner) {
  const int j = blockIdx.y;
  int bx, by;
  box_xy(g, 2 * j + which, bx, by);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    const int k = imap(local, i);
    const int s = side_of(g, k);
    cd v = cmk(0.0, 0.0);
    if (!side_physical(g, bx, by, s)) {
      int slot = box_slot(g, bx, by, k);
      if (use_partner) slot = slot_partner(g.n, g.p, slot);
      v = vec[slot];
    }
    out[(long long)j * ostride + i] = v;
  }
}

// Inverse of pair_gather: vec[slot] (= or +=) in[j][i]; physical entries skipped.
__global__ void pair_scatter_kernel(Geom g, int which, IdxMap local, int len, const cd* in,
                                    long long istride, cd* vec, int use_partner, int add) {
  const int j = blockIdx.y;
  int bx, by;
  box_xy(g, 2 * j + which, bx, by);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    const int k = imap(local, i);
    const int s = side_of(g, k);
    if (side_physical(g, bx, by, s)) continue;
    int slot = box_slot(g, bx, by, k);
    if (use_partner) slot = slot_partner(g.n, g.p, slot);
    const cd v = in[(long long)j * istride + i];
    vec[slot] = add ? cadd(vec[slot], v) : v;
  }
}

__global__ void index_gather_kernel(const int* idx, int n, const cd* vec, cd* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = vec[idx[i]];
}

__global__ void index_scatter_kernel(const int* idx, int n, const cd* in, cd* vec) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    vec[idx[i]] = in[i];
}

__global__ void fill_kernel(cd* v, long long n, cd val) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    v[i] = val;
}

__global__ void axpby_kernel(cd a, const cd* x, cd b, const cd* y, cd* out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = cadd(cmul(a, x[i]), cmul(b, y[i]));
}

__global__ void copy_kernel(const cd* src, cd* dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---- deterministic reductions -------------------------------------------
// Wave-level sum in a fixed butterfly order.
__device__ inline cd wave_sum(cd v) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

// Block-level sum (256 threads), result valid in thread 0.
__device__ inline cd block_sum(cd v) {
  __shared__ cd ws[4];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) ws[w] = v;
  __syncthreads();
  cd r = cmk(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = cadd(r, ws[i]);
  }
  __syncthreads();
  return r;
}

// Stage 1: partial[v][blk] = sum over chunk blk of conj(V_v) . w   (grid (blocks, nvec))
__global__ __launch_bounds__(256) void dot_stage1_kernel(const cd* V, long long vstride, const cd* w,
                                                         long long n, cd* partial, int nblk) {
  const int v = blockIdx.y;
  const cd* Vv = V + (long long)v * vstride;
  const long long chunk = (n + nblk - 1) / nblk;
  const long long a0 = (long long)blockIdx.x * chunk;
  const long long a1 = a0 + chunk < n ? a0 + chunk : n;
  cd acc = cmk(0.0, 0.0);
  for (long long i = a0 + threadIdx.x; i < a1; i += blockDim.x) acc = cfma(cconj(Vv[i]), w[i], acc);
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[(long long)v * nblk + blockIdx.x] = acc;
}

// Stage 2: out[v] = sum_blk partial[v][blk]; optional: out_norm[v] = sqrt(Re out[v]).
__global__ __launch_bounds__(256) void dot_stage2_kernel(const cd* partial, int nblk, cd* out,
                                                         int accumulate) {
  const int v = blockIdx.x;
  cd acc = cmk(0.0, 0.0);
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc = cadd(acc, partial[(long long)v * nblk + i]);
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[v] = accumulate ? cadd(out[v], acc) : acc;
}

// w -= sum_v h[v] V_v   (h on the device)
__global__ void multi_axpy_kernel(const cd* V, long long vstride, int nvec, const cd* h, cd* w,
                                  long long n, int sign) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    cd acc = w[i];
    for (int v = 0; v < nvec; ++v) {
      const cd t = cmul(h[v], V[(long long)v * vstride + i]);
      acc = sign > 0 ? cadd(acc, t) : csub(acc, t);
    }
    w[i] = acc;
  }
}

// out = w / sqrt(Re nrm2[0]); also stores the norm into hout (complex, im = 0).
__global__ void normalize_kernel(const cd* w, const cd* nrm2, cd* out, long long n, cd* hout) {
  const double nr = sqrt(fmax(nrm2[0].x, 0.0));
  const double s = nr > 0.0 ? 1.0 / nr : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && hout) *hout = cmk(nr, 0.0);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = cscale(w[i], s);
}

// k-step GMRES least squares on the device: minimise |beta e1 - H y| for the
// (k+1) x k Hessenberg H (column-major, ld ldh) by Givens rotations, one thread.
// R: (kMaxCoarse+1) x kMaxCoarse and gv: kMaxCoarse+1 work arrays (LDS).
__device__ void lsq_small(const cd* Hm, int ldh, int k, const cd* beta2, cd* y, int* kused,
                          cd (*R)[kMaxCoarse], cd* gv) {
  const double beta = sqrt(fmax(beta2[0].x, 0.0));
  // the subdiagonal entries H[j+1][j] are the real Arnoldi norms; a (lucky)
  // breakdown h_{j+1,j} <= 1e-14 beta ends the Krylov space at j+1 vectors
  int kk = k;
  for (int j = 0; j < k; ++j) {
    if (!(Hm[(long long)j * ldh + j + 1].x > 1e-14 * beta)) {
      kk = j + 1;
      break;
    }
  }
  for (int j = 0; j <= kk; ++j) gv[j] = cmk(0.0, 0.0);
  gv[0] = cmk(beta, 0.0);
  for (int j = 0; j < kk; ++j)
    for (int i = 0; i <= kk; ++i) R[i][j] = (i <= j + 1) ? Hm[(long long)j * ldh + i] : cmk(0.0, 0.0);
  for (int j = 0; j < kk; ++j) {
    const cd a = R[j][j], b = R[j + 1][j];
    const double den = sqrt(cabs2(a) + cabs2(b));
    const cd c = den > 0 ? cscale(a, 1.0 / den) : cmk(1.0, 0.0);
    const cd s = den > 0 ? cscale(b, 1.0 / den) : cmk(0.0, 0.0);
    for (int q = j; q < kk; ++q) {
      const cd u = R[j][q], v = R[j + 1][q];
      R[j][q] = cadd(cmul(cconj(c), u), cmul(cconj(s), v));
      R[j + 1][q] = csub(cmul(c, v), cmul(s, u));
    }
    const cd gu = gv[j], gw = gv[j + 1];
    gv[j] = cadd(cmul(cconj(c), gu), cmul(cconj(s), gw));
    gv[j + 1] = csub(cmul(c, gw), cmul(s, gu));
  }
  for (int i = kk - 1; i >= 0; --i) {
    cd acc = gv[i];
    for (int q = i + 1; q < kk; ++q) acc = csub(acc, cmul(R[i][q], y[q]));
    y[i] = cabs2(R[i][i]) > 0 ? cmul(acc, cinv(R[i][i])) : cmk(0.0, 0.0);
  }
  for (int i = kk; i < k; ++i) y[i] = cmk(0.0, 0.0);
  if (kused) *kused = kk;
}

// ---- the coarse k-step GMRES, one workgroup per launch ---------------------
constexpr int kCT = 1024;

// Sum over the workgroup (kCT threads) in a fixed order; valid in every thread.
__device__ inline cd wg_sum(cd v, cd* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  cd r = cmk(0.0, 0.0);
  for (int i = 0; i < kCT / 64; ++i) r = cadd(r, red[i]);
  __syncthreads();
  return r;
}

// V_0 = w / |w| with w = vec[idx]; beta2 = |w|^2; H = 0.
__global__ __launch_bounds__(kCT) void coarse_start_kernel(const int* idx, int n, const cd* vec, cd* V, cd* H,
                                                           int hsize, cd* beta2) {
  __shared__ cd red[kCT / 64];
  const int t = threadIdx.x;
  cd acc = cmk(0.0, 0.0);
  for (int i = t; i < n; i += kCT) {
    const cd x = vec[idx[i]];
    V[i] = x;
    acc = cfma(cconj(x), x, acc);
  }
  const cd nr2 = wg_sum(acc, red);
  if (t == 0) beta2[0] = nr2;
  const double nr = sqrt(fmax(nr2.x, 0.0));
  const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = t; i < n; i += kCT) V[i] = cscale(V[i], sc);
  for (int i = t; i < hsize; i += kCT) H[i] = cmk(0.0, 0.0);
}

// Arnoldi step j: w = M v_j (given, or v_j minus the split-K partial sums of
// the pair-form product), two passes of classical Gram-Schmidt against
// V_0..V_j (dots in a fixed order), V_{j+1} = w / |w|, H column j.
__global__ __launch_bounds__(kCT) void coarse_arnoldi_kernel(cd* V, int n, int j, CoarseW src, cd* w, cd* Hcol) {
  __shared__ cd h[kMaxCoarse + 1], h2[kMaxCoarse + 1];
  __shared__ cd red[kCT / 64];
  const int t = threadIdx.x;
  const cd* vj = V + (long long)j * n;
  for (int i = t; i < n; i += kCT) {
    cd x;
    if (src.part) {
      const bool second = i >= src.m;
      const int r = second ? i - src.m : i;
      const long long po = second ? src.poff1 : src.poff0;
      const int ns = second ? src.ns1 : src.ns0;
      cd acc = cmk(0.0, 0.0);
      for (int q = 0; q < ns; ++q) acc = cadd(acc, src.part[po + (long long)q * src.m + r]);
      x = csub(vj[i], acc);
    } else {
      x = src.w[i];
    }
    w[i] = x;
  }
  __syncthreads();
  const int v = t >> 5, l = t & 31;
  for (int pass = 0; pass < 2; ++pass) {
    cd* hv = pass ? h2 : h;
    cd acc = cmk(0.0, 0.0);
    if (v <= j) {
      const cd* Vv = V + (long long)v * n;
      for (int i = l; i < n; i += 32) acc = cfma(cconj(Vv[i]), w[i], acc);
    }
    for (int off = 16; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (l == 0 && v <= j) hv[v] = acc;
    __syncthreads();
    for (int i = t; i < n; i += kCT) {
      cd a = w[i];
      for (int q = 0; q <= j; ++q) a = csub(a, cmul(hv[q], V[(long long)q * n + i]));
      w[i] = a;
    }
    __syncthreads();
  }
  cd acc = cmk(0.0, 0.0);
  for (int i = t; i < n; i += kCT) acc = cfma(cconj(w[i]), w[i], acc);
  const cd nr2 = wg_sum(acc, red);
  const double nr = sqrt(fmax(nr2.x, 0.0));
  const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
  cd* vn = V + (long long)(j + 1) * n;
  for (int i = t; i < n; i += kCT) vn[i] = cscale(w[i], sc);
  if (t <= j) Hcol[t] = cadd(h[t], h2[t]);
  if (t == 0) Hcol[j + 1] = cmk(nr, 0.0);
}

// Arnoldi step j for short coarse vectors (n <= EP * kCT) and few basis vectors
// (j < kFastV): every thread keeps its EP entries of w and of V_0..V_j in
// registers, so global memory is read once and each reduction is one
// workgroup sum of j+1 values.  Same arithmetic as coarse_arnoldi_kernel up to
// the order of the dot-product sums.
constexpr int kFastV = 6;

template <int EP, int NT>
__global__ __launch_bounds__(NT) void coarse_arnoldi_fast_kernel(cd* V, int n, int j, CoarseW src, cd* Hcol) {
  __shared__ cd red[NT / 64][kFastV];
  __shared__ cd hs[kFastV], hsum[kFastV];
  const int t = threadIdx.x;
  const cd zero = cmk(0.0, 0.0);
  cd vv[kFastV][EP];
  cd w[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int i = t + e * NT;
#pragma unroll
    for (int v = 0; v < kFastV; ++v) vv[v][e] = (v <= j && i < n) ? V[(long long)v * n + i] : zero;
  }
  const cd* vj = V + (long long)j * n;
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int i = t + e * NT;
    cd x = zero;
    if (i < n) {
      if (src.part) {
        const bool second = i >= src.m;
        const int r = second ? i - src.m : i;
        const long long po = second ? src.poff1 : src.poff0;
        const int ns = second ? src.ns1 : src.ns0;
        cd acc = zero;
        for (int q0 = 0; q0 < ns; q0 += 8) {
          cd tmp[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tmp[u] = q0 + u < ns ? src.part[po + (long long)(q0 + u) * src.m + r] : zero;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (q0 + u < ns) acc = cadd(acc, tmp[u]);
        }
        x = csub(vj[i], acc);
      } else {
        x = src.w[i];
      }
    }
    w[e] = x;
  }
  for (int pass = 0; pass < 2; ++pass) {
    cd acc[kFastV];
#pragma unroll
    for (int v = 0; v < kFastV; ++v) {
      acc[v] = zero;
#pragma unroll
      for (int e = 0; e < EP; ++e) acc[v] = cfma(cconj(vv[v][e]), w[e], acc[v]);
      acc[v] = wave_sum(acc[v]);
    }
    if ((t & 63) == 0) {
#pragma unroll
      for (int v = 0; v < kFastV; ++v) red[t >> 6][v] = acc[v];
    }
    __syncthreads();
    if (t < kFastV) {
      cd r = zero;
      for (int q = 0; q < NT / 64; ++q) r = cadd(r, red[q][t]);
      hs[t] = r;
      hsum[t] = pass ? cadd(hsum[t], r) : r;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kFastV; ++v) {
      if (v > j) continue;
      const cd hv = hs[v];
#pragma unroll
      for (int e = 0; e < EP; ++e) w[e] = csub(w[e], cmul(hv, vv[v][e]));
    }
    __syncthreads();
  }
  cd acc = zero;
#pragma unroll
  for (int e = 0; e < EP; ++e) acc = cfma(cconj(w[e]), w[e], acc);
  acc = wave_sum(acc);
  if ((t & 63) == 0) red[t >> 6][0] = acc;
  __syncthreads();
  cd nr2 = zero;
  for (int q = 0; q < NT / 64; ++q) nr2 = cadd(nr2, red[q][0]);
  const double nr = sqrt(fmax(nr2.x, 0.0));
  const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
  cd* vn = V + (long long)(j + 1) * n;
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int i = t + e * NT;
    if (i < n) vn[i] = cscale(w[e], sc);
  }
  if (t == 0) {
#pragma unroll
    for (int v = 0; v < kFastV; ++v)
      if (v <= j) Hcol[v] = hsum[v];
    Hcol[j + 1] = cmk(nr, 0.0);
  }
}

// y = argmin |beta e1 - H y|, x = V y, vec[idx] = x.
__global__ __launch_bounds__(kCT) void coarse_finish_kernel(const cd* H, int k, const cd* beta2, const cd* V, int n,
                                                            const int* idx, cd* vec) {
  __shared__ cd y[kMaxCoarse];
  __shared__ cd R[kMaxCoarse + 1][kMaxCoarse];
  __shared__ cd gv[kMaxCoarse + 1];
  if (threadIdx.x == 0) lsq_small(H, k + 1, k, beta2, y, nullptr, R, gv);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kCT) {
    cd acc = cmk(0.0, 0.0);
    for (int v = 0; v < k; ++v) acc = cadd(acc, cmul(y[v], V[(long long)v * n + i]));
    vec[idx[i]] = acc;
  }
}

inline int grid_for(long long n, int block = 256, int cap = 2048) {
  long long g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t skeleton_apply(const Geom& g, const cd* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st) {
  dim3 grid(g.nboxes, (g.b + kRows - 1) / kRows);
  hipError_t e0 = allow_lds(skeleton_apply_kernel, (size_t)g.b * sizeof(cd));
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(skeleton_apply_kernel, grid, dim3(kRows), (size_t)g.b * sizeof(cd), st, g, T, gin,
                     out, zero_physical ? 1 : 0);
  return hipPeekAtLastError();
}

hipError_t rhs_build(const Geom& g, const cd* T, const cd* H, const cd* t, cd* rhs, hipStream_t st) {
  hipLaunchKernelGGL(rhs_kernel, dim3(g.n * g.n), dim3(kRows), 0, st, g, T, H, t, rhs);
  return hipPeekAtLastError();
}

hipError_t zgemv(const GemvArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.batch <= 0) return hipSuccess;
  dim3 grid((a.M + kRows - 1) / kRows, a.batch);
  hipError_t e0 = allow_lds(zgemv_kernel, (size_t)std::max(a.K, 1) * sizeof(cd));
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(zgemv_kernel, grid, dim3(kRows), (size_t)std::max(a.K, 1) * sizeof(cd), st, a);
  return hipPeekAtLastError();
}

hipError_t pair_gather(const Geom& g, int pairs, int which, IdxMap local, int len, const cd* vec,
                       cd* out, long long ostride, bool partner, hipStream_t st) {
  if (len <= 0 || pairs <= 0) return hipSuccess;
  dim3 grid((len + 255) / 256, pairs);
  hipLaunchKernelGGL(pair_gather_kernel, grid, dim3(256), 0, st, g, which, local, len, vec, out, ostride,
                     partner ? 1 : 0);
  return hipPeekAtLastError();
}

hipError_t pair_scatter(const Geom& g, int pairs, int which, IdxMap local, int len, const cd* in,
                        long long istride, cd* vec, bool partner, bool add, hipStream_t st) {
  if (len <= 0 || pairs <= 0) return hipSuccess;
  dim3 grid((len + 255) / 256, pairs);
  hipLaunchKernelGGL(pair_scatter_kernel, grid, dim3(256), 0, st, g, which, local, len, in, istride, vec,
                     partner ? 1 : 0, add ? 1 : 0);
  return hipPeekAtLastError();
}

hipError_t index_gather(const int* idx, int n, const cd* vec, cd* out, hipStream_t st) {
  hipLaunchKernelGGL(index_gather_kernel, dim3(grid_for(n)), dim3(256), 0, st, idx, n, vec, out);
  return hipPeekAtLastError();
}

hipError_t index_scatter(const int* idx, int n, const cd* in, cd* vec, hipStream_t st) {
  hipLaunchKernelGGL(index_scatter_kernel, dim3(grid_for(n)), dim3(256), 0, st, idx, n, in, vec);
  return hipPeekAtLastError();
}

hipError_t vfill(cd* v, long long n, cd val, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, v, n, val);
  return hipPeekAtLastError();
}

hipError_t axpby(cd a, const cd* x, cd b, const cd* y, cd* out, long long n, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, st, a, x, b, y, out, n);
  return hipPeekAtLastError();
}

hipError_t vcopy(const cd* src, cd* dst, long long n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
  return hipPeekAtLastError();
}

int dot_blocks(long long n) {
  long long b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > kMaxDotBlocks ? kMaxDotBlocks : b));
}

hipError_t multi_dot(const cd* V, long long vstride, int nvec, const cd* w, long long n, cd* partial,
                     cd* out, bool accumulate, hipStream_t st) {
  const int nblk = dot_blocks(n);
  hipLaunchKernelGGL(dot_stage1_kernel, dim3(nblk, nvec), dim3(256), 0, st, V, vstride, w, n, partial,
                     nblk);
  hipError_t err = hipPeekAtLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(dot_stage2_kernel, dim3(nvec), dim3(256), 0, st, partial, nblk, out,
                     accumulate ? 1 : 0);
  return hipPeekAtLastError();
}

hipError_t multi_axpy(const cd* V, long long vstride, int nvec, const cd* h, cd* w, long long n, int sign,
                      hipStream_t st) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(256), 0, st, V, vstride, nvec, h, w, n,
                     sign);
  return hipPeekAtLastError();
}

hipError_t normalize(const cd* w, const cd* nrm2, cd* out, long long n, cd* hout, hipStream_t st) {
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n)), dim3(256), 0, st, w, nrm2, out, n, hout);
  return hipPeekAtLastError();
}


hipError_t coarse_start(const int* idx, int n, const cd* vec, cd* V, cd* H, int hsize, cd* beta2,
                        hipStream_t st) {
  hipLaunchKernelGGL(coarse_start_kernel, dim3(1), dim3(kCT), 0, st, idx, n, vec, V, H, hsize, beta2);
  return hipPeekAtLastError();
}

hipError_t coarse_arnoldi(cd* V, int n, int j, const CoarseW& src, cd* wtmp, cd* Hcol, hipStream_t st) {
  if (j < 0 || j + 1 > kMaxCoarse) return hipErrorInvalidValue;
  if (j < kFastV && n <= 4 * 256)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<4, 256>), dim3(1), dim3(256), 0, st, V, n, j, src, Hcol);
  else if (j < kFastV && n <= 8 * 256)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<8, 256>), dim3(1), dim3(256), 0, st, V, n, j, src, Hcol);
  else if (j < kFastV && n <= 16 * 256)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<16, 256>), dim3(1), dim3(256), 0, st, V, n, j, src, Hcol);
  else
    hipLaunchKernelGGL(coarse_arnoldi_kernel, dim3(1), dim3(kCT), 0, st, V, n, j, src, wtmp, Hcol);
  return hipPeekAtLastError();
}

hipError_t coarse_finish(const cd* H, int k, const cd* beta2, const cd* V, int n, const int* idx, cd* vec,
                         hipStream_t st) {
  if (k < 1 || k > kMaxCoarse) return hipErrorInvalidValue;
  hipLaunchKernelGGL(coarse_finish_kernel, dim3(1), dim3(kCT), 0, st, H, k, beta2, V, n, idx, vec);
  return hipPeekAtLastError();
}

}  // namespace hps
