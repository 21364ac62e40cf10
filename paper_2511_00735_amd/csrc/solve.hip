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
// every level-l box B, for each problem of a group (boxes and canonical vectors
// of problem q follow those of problem q-1).  Grid (problems * boxes,
// ceil(b / 64)), 64 threads.  M: the storage type of the box maps (complex
// FP64, or FP32 on the FP32 levels of mixed precision); FP64 arithmetic.
template <class M>
__global__ __launch_bounds__(kRows) void skeleton_apply_kernel(Geom g, const M* T, const cd* gin,
                                                               cd* out, int zero_physical, long long nslots) {
  extern __shared__ cd gB[];
  const int jg = blockIdx.x;
  const int j = jg % g.nboxes;
  const long long so = (long long)(jg / g.nboxes) * nslots;
  gin += so;
  out += so;
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
  const M* Tb = T + (long long)jg * b * b;
  cd acc = cmk(0.0, 0.0);
  for (int s = 0; s < 4; ++s) {
    if (phys_side[s]) continue;
    const int c1 = g.off[s + 1];
    int c = g.off[s];
    for (; c + 3 < c1; c += 4) {
      const cd t0 = to_cd(Tb[(long long)c * b + r]), t1 = to_cd(Tb[(long long)(c + 1) * b + r]);
      const cd t2 = to_cd(Tb[(long long)(c + 2) * b + r]), t3 = to_cd(Tb[(long long)(c + 3) * b + r]);
      acc = cfma(t0, gB[c], acc);
      acc = cfma(t1, gB[c + 1], acc);
      acc = cfma(t2, gB[c + 2], acc);
      acc = cfma(t3, gB[c + 3], acc);
    }
    for (; c < c1; ++c) acc = cfma(to_cd(Tb[(long long)c * b + r]), gB[c], acc);
  }
  const int ps = slot_partner(g.nx, g.ny, g.p, slot);
  out[ps] = csub(gin[ps], acc);
}

// Level-1 right-hand side: rhs[Pi(s)] = (H^e + T^e t_phys)[s]; physical slots 0.
__global__ __launch_bounds__(kRows) void rhs_kernel(Geom g, const cd* T, const cd* H, const cd* t,
                                                    cd* rhs) {
  __shared__ cd tl[256];
  const int e = blockIdx.x;
  const int p = g.p, m = 4 * p;
  const int ix = e % g.nx, iy = e / g.nx;
  const cd* Te = T + (long long)tree_code(g.ax, g.ay, ix, iy) * m * m;
  bool phys[4] = {ix == 0, ix == g.nx - 1, iy == 0, iy == g.ny - 1};
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
    rhs[slot_partner(g.nx, g.ny, p, slot)] = acc;
  }
}

// i in [0, nq * n): problem q = i / n, entry r = i % n.
__global__ void index_gather_kernel(const int* idx, int n, long long ntot, const cd* vec, cd* out,
                                    long long ostride) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ntot;
       i += (long long)gridDim.x * blockDim.x)
    out[(i / n) * ostride + i % n] = vec[idx[i]];
}

__global__ void index_scatter_kernel(const int* idx, int n, long long ntot, const cd* in, long long istride,
                                     cd* vec) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ntot;
       i += (long long)gridDim.x * blockDim.x)
    vec[idx[i]] = in[(i / n) * istride + i % n];
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

// dst = src with either end displaced by a device-held index: src + (*isrc) *
// stride or dst + (*idst) * stride (null: no displacement).
__global__ void copy_at_kernel(const cd* src, cd* dst, long long n, const int* isrc, const int* idst,
                               long long stride) {
  if (isrc) src += (long long)*isrc * stride;
  if (idst) dst += (long long)*idst * stride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void counter_kernel(int* c, int value, int add) {
  if (threadIdx.x == 0) *c = add ? *c + value : value;
}

__global__ void copy_zero_kernel(const cd* src, cd* dst, cd* zero, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    dst[i] = src[i];
    zero[i] = cmk(0.0, 0.0);
  }
}

// ---- deterministic reductions -------------------------------------------
// Wave-level sum in a fixed butterfly order.
// Lane l - s of the same 16-lane row (0 outside the row), by DPP.
template <int kCtrl>
__device__ inline double dpp_shr(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the wavefront, returned to every lane: DPP row shifts by 1, 2, 4, 8
// leave each 16-lane row's sum in its last lane; the four row sums are then
// added in row order (deterministic).
__device__ inline double wave_sum(double v) {
  v += dpp_shr<0x111>(v);
  v += dpp_shr<0x112>(v);
  v += dpp_shr<0x114>(v);
  v += dpp_shr<0x118>(v);
  return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}
__device__ inline cd wave_sum(cd v) { return cmk(wave_sum(v.x), wave_sum(v.y)); }

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

// Stage 1: partial[q][v][blk] = sum over chunk blk of conj(V_v) . w on the
// segment of problem q (grid (blocks, nvec, problems)); with self set, the
// last grid row takes conj(w) . w instead.
__global__ __launch_bounds__(256) void dot_stage1_kernel(const cd* V, long long vstride, const cd* w,
                                                         long long n, cd* partial, int nblk, const int* nvdev,
                                                         int self) {
  const int v = blockIdx.y, q = blockIdx.z;
  const bool selfrow = self && v == (int)gridDim.y - 1;
  if (!selfrow && nvdev && v > *nvdev) return;   // device count (nvdev + 1 vectors; uniform per workgroup)
  const cd* Vv = (selfrow ? w : V + (long long)v * vstride) + (long long)q * n;
  w += (long long)q * n;
  partial += (long long)q * gridDim.y * nblk;
  const long long chunk = (n + nblk - 1) / nblk;
  const long long a0 = (long long)blockIdx.x * chunk;
  const long long a1 = a0 + chunk < n ? a0 + chunk : n;
  cd acc = cmk(0.0, 0.0);
  for (long long i = a0 + threadIdx.x; i < a1; i += blockDim.x) acc = cfma(cconj(Vv[i]), w[i], acc);
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[(long long)v * nblk + blockIdx.x] = acc;
}

// Stage 2: out[q * ostride + v] (+)= sum_blk partial[q][v][blk]  (grid (nvec, problems));
// with selfout set, the last grid row's sum goes to selfout[q * ostride].
__global__ __launch_bounds__(256) void dot_stage2_kernel(const cd* partial, int nblk, cd* out,
                                                         int accumulate, long long ostride, const int* nvdev,
                                                         cd* selfout) {
  const int v = blockIdx.x, q = blockIdx.y;
  const bool selfrow = selfout && v == (int)gridDim.x - 1;
  if (!selfrow && nvdev && v > *nvdev) return;
  partial += (long long)q * gridDim.x * nblk;
  out += (long long)q * ostride;
  cd acc = cmk(0.0, 0.0);
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc = cadd(acc, partial[(long long)v * nblk + i]);
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    if (selfrow)
      selfout[(long long)q * ostride] = acc;
    else
      out[v] = accumulate ? cadd(out[v], acc) : acc;
  }
}

// w += sign * sum_v h[q * hstride + v] V_v on the segment of each problem q
// (h on the device; entries i of [0, nq * n), q = i / n).
__global__ void multi_axpy_kernel(const cd* V, long long vstride, int nvec, const cd* h, long long hstride,
                                  cd* w, long long n, long long ntot, int sign, const int* nvdev) {
  if (nvdev) nvec = *nvdev + 1;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ntot;
       i += (long long)gridDim.x * blockDim.x) {
    const cd* hq = h + (i / n) * hstride;
    cd acc = w[i];
    for (int v = 0; v < nvec; ++v) {
      const cd t = cmul(hq[v], V[(long long)v * vstride + i]);
      acc = sign > 0 ? cadd(acc, t) : csub(acc, t);
    }
    w[i] = acc;
  }
}

// The second Gram-Schmidt pass's update and the normalisation in one pass over
// the vectors, on the segment of problem q (grid.y): w'' = w' - sum_v h[v] V_v
// (v <= *nvdev with nvdev set, else v < nvec, summed in that order), and with
// V orthonormal |w''|^2 = |w'|^2 - sum_v |h[v]|^2 (|w'|^2 in Re nrm2[q *
// nstride]); out = w'' / |w''| (displaced by (*jdev + 1) * jstride with jdev
// set) and hout[q * hstride] = |w''|.
__global__ __launch_bounds__(256) void axpy_normalize_kernel(const cd* V, long long vstride, int nvec, const cd* h,
                                                             long long hstride, const cd* w, long long n,
                                                             const cd* nrm2, long long nstride, cd* out, cd* hout,
                                                             long long houtstride, const int* nvdev,
                                                             const int* jdev, long long jstride) {
  __shared__ double sc_s;
  const int q = blockIdx.y;
  if (nvdev) nvec = *nvdev + 1;
  if (jdev) out += (long long)(*jdev + 1) * jstride;
  const cd* hq = h + (long long)q * hstride;
  if (threadIdx.x < 64) {
    double a = 0.0;
    for (int v = threadIdx.x; v < nvec; v += 64) a += cabs2(hq[v]);
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (threadIdx.x == 0) {
      const double nr = sqrt(fmax(nrm2[(long long)q * nstride].x - a, 0.0));
      sc_s = nr > 0.0 ? 1.0 / nr : 0.0;
      if (blockIdx.x == 0 && hout) hout[(long long)q * houtstride] = cmk(nr, 0.0);
    }
  }
  __syncthreads();
  const double s = sc_s;
  w += (long long)q * n;
  out += (long long)q * n;
  const long long qo = (long long)q * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    cd acc = w[i];
    for (int v = 0; v < nvec; ++v) acc = csub(acc, cmul(hq[v], V[(long long)v * vstride + qo + i]));
    out[i] = cscale(acc, s);
  }
}

// out = w / sqrt(Re nrm2[q * nstride]) on the segment of problem q (grid.y);
// also stores the norm into hout[q * hstride] (complex, im = 0).
__global__ void normalize_kernel(const cd* w, const cd* nrm2, long long nstride, cd* out, long long n, cd* hout,
                                 long long hstride, const int* jdev, long long jstride) {
  const int q = blockIdx.y;
  if (jdev) out += (long long)(*jdev + 1) * jstride;   // V_{j+1} with j on the device
  const double nr = sqrt(fmax(nrm2[(long long)q * nstride].x, 0.0));
  const double s = nr > 0.0 ? 1.0 / nr : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && hout) hout[(long long)q * hstride] = cmk(nr, 0.0);
  w += (long long)q * n;
  out += (long long)q * n;
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
__global__ __launch_bounds__(kCT) void coarse_start_kernel(const int* idx, int n, const cd* vec, cd* V,
                                                           long long vq, cd* H, int hsize, cd* beta2) {
  __shared__ cd red[kCT / 64];
  const int t = threadIdx.x, q = blockIdx.x;
  idx += (long long)q * n;
  V += (long long)q * vq;
  H += (long long)q * hsize;
  beta2 += q;
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
__global__ __launch_bounds__(kCT) void coarse_arnoldi_kernel(cd* V, int n, long long vq, int j, CoarseW src,
                                                             cd* w, cd* Hcol, int hsize) {
  __shared__ cd h[kMaxCoarse + 1], h2[kMaxCoarse + 1];
  __shared__ cd red[kCT / 64];
  const int t = threadIdx.x, qp = blockIdx.x;
  V += (long long)qp * vq;
  w += (long long)qp * n;
  Hcol += (long long)qp * hsize;
  if (src.w) src.w += (long long)qp * n;
  const cd* vj = V + (long long)j * n;
  for (int i = t; i < n; i += kCT) {
    cd x;
    if (src.part) {
      const bool second = i >= src.m;
      const int r = second ? i - src.m : i;
      const long long po = second ? src.poff1 : src.poff0;
      const int ns = second ? src.ns1 : src.ns0;
      cd acc = cmk(0.0, 0.0);
      for (int q = 0; q < ns; ++q) acc = cadd(acc, src.part[po + ((long long)q * src.nb + qp) * src.m + r]);
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
constexpr int kFastSplits = 8;   // split-K partials summed in one round of loads

// The least squares of lsq_small for k <= kFastV in one wavefront (called by
// all 64 lanes of a wave): lane q holds column q of R in registers; rotation j
// is formed in lane j and applied by lanes j..kk-1 (and to the right-hand side
// in every lane); the back substitution sums R[i][q] y_q across the lanes.  The
// same rotations as lsq_small; only the back substitution's sums are added in
// another order.  Hs: (k+1) x k column-major (ld k+1); y[0..k) to LDS.
__device__ void lsq_wave(const cd* Hs, int ldh, int k, double beta, cd* y) {
  const int lane = threadIdx.x & 63;
  int kk = k;
  for (int j = 0; j < k; ++j) {
    if (!(Hs[(long long)j * ldh + j + 1].x > 1e-14 * beta)) {
      kk = j + 1;
      break;
    }
  }
  cd hc[kFastV + 1], g[kFastV + 1];
#pragma unroll
  for (int i = 0; i <= kFastV; ++i) {
    hc[i] = (lane < kk && i <= lane + 1 && i <= kk) ? Hs[(long long)lane * ldh + i] : cmk(0.0, 0.0);
    g[i] = cmk(i == 0 ? beta : 0.0, 0.0);
  }
#pragma unroll
  for (int j = 0; j < kFastV; ++j) {
    if (j < kk) {
      const cd a = hc[j], b = hc[j + 1];   // meaningful in lane j
      const double den = sqrt(cabs2(a) + cabs2(b));
      cd c = den > 0 ? cscale(a, 1.0 / den) : cmk(1.0, 0.0);
      cd s = den > 0 ? cscale(b, 1.0 / den) : cmk(0.0, 0.0);
      c = cmk(lane_value(c.x, j), lane_value(c.y, j));
      s = cmk(lane_value(s.x, j), lane_value(s.y, j));
      if (lane >= j && lane < kk) {
        const cd u = hc[j], v = hc[j + 1];
        hc[j] = cadd(cmul(cconj(c), u), cmul(cconj(s), v));
        hc[j + 1] = csub(cmul(c, v), cmul(s, u));
      }
      const cd gu = g[j], gw = g[j + 1];
      g[j] = cadd(cmul(cconj(c), gu), cmul(cconj(s), gw));
      g[j + 1] = csub(cmul(c, gw), cmul(s, gu));
    }
  }
  cd yq = cmk(0.0, 0.0);   // y of this lane's column
#pragma unroll
  for (int i = kFastV - 1; i >= 0; --i) {
    if (i < kk) {
      const cd sum = wave_sum((lane > i && lane < kk) ? cmul(hc[i], yq) : cmk(0.0, 0.0));
      const cd acc = csub(g[i], sum);
      const cd rii = cmk(lane_value(hc[i].x, i), lane_value(hc[i].y, i));
      const cd yi = cabs2(rii) > 0 ? cmul(acc, cinv(rii)) : cmk(0.0, 0.0);
      if (lane == i) yq = yi;
    }
  }
  if (lane < k) y[lane] = lane < kk ? yq : cmk(0.0, 0.0);
}

template <int EP, int NT>
__global__ __launch_bounds__(NT) void coarse_arnoldi_fast_kernel(cd* V, int n, long long vq, int j, CoarseW src,
                                                                cd* Hcol, int hsize, CoarseEnds ends) {
  __shared__ cd red[NT / 64][kFastV];
  __shared__ cd hs[kFastV], hsum[kFastV];
  const int t = threadIdx.x, qp = blockIdx.x;
  V += (long long)qp * vq;
  Hcol += (long long)qp * hsize;
  if (src.w) src.w += (long long)qp * n;
  const bool first = ends.idx && j == 0, last = ends.idx && j == ends.k - 1;
  // last step: the scatter's slot indices are loaded now, so that their
  // latency passes during the Arnoldi step
  int sidx[EP];
  if (last) {
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
      sidx[e] = i < n ? ends.idx[(long long)qp * n + i] : 0;
    }
  }
  cd vv[kFastV][EP];
  cd w[EP];
  double inv_beta = 1.0;   // first step: w0 = vec[idx] unnormalised, V_0 = w0 / beta
  if (first) {
    // the start of the k-step GMRES in this launch: V_0 = w0 / |w0|, beta^2,
    // H = 0 (the product below was formed from w0 itself)
    const int* idx = ends.idx + (long long)qp * n;
    cd acc = cmk(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
      vv[0][e] = i < n ? ends.vin[idx[i]] : cmk(0.0, 0.0);
      acc = cfma(cconj(vv[0][e]), vv[0][e], acc);
#pragma unroll
      for (int v = 1; v < kFastV; ++v) vv[v][e] = cmk(0.0, 0.0);
    }
    acc = wave_sum(acc);
    if ((t & 63) == 0) red[t >> 6][0] = acc;
    __syncthreads();
    cd b2 = cmk(0.0, 0.0);
    for (int q = 0; q < NT / 64; ++q) b2 = cadd(b2, red[q][0]);
    const double beta = sqrt(fmax(b2.x, 0.0));
    inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
      vv[0][e] = cscale(vv[0][e], inv_beta);
      if (i < n) V[i] = vv[0][e];
    }
    cd* H = Hcol;   // column 0 is the start of the problem's H
    for (int i = t; i < hsize; i += NT) H[i] = cmk(0.0, 0.0);
    if (t == 0) ends.beta2[qp] = b2;
    __syncthreads();   // red is reused below; H is zeroed before column 0 is written
  }
  // later steps load V_0..V_j after the split-K partials below, so that the
  // partials' loads are in flight together without V's registers
  auto load_v = [&]() {
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
#pragma unroll
      for (int v = 0; v < kFastV; ++v) vv[v][e] = (v <= j && i < n) ? V[(long long)v * n + i] : cmk(0.0, 0.0);
    }
  };
  if (src.part) {
    // w = v_j - (sum of the split-K partials, in split order)
    const cd* pp[EP];
    int nse[EP], nsa[EP];
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT, ic = min(i, n - 1);   // ic: a valid address for every lane
      const bool second = ic >= src.m;
      const int r = second ? ic - src.m : ic;
      pp[e] = src.part + (second ? src.poff1 : src.poff0) + (long long)qp * src.m + r;
      nsa[e] = second ? src.ns1 : src.ns0;
      nse[e] = i < n ? nsa[e] : 0;
      w[e] = cmk(0.0, 0.0);
    }
    const long long qs = (long long)src.nb * src.m;
    const int nsmax = max(src.ns0, src.ns1);
    if (nsmax <= kFastSplits) {
      // every split of every entry in one round: unconditional loads (clamped
      // to the entry's last split), so that no branch makes the compiler wait
      // between them
      cd tmp[kFastSplits][EP];
#pragma unroll
      for (int u = 0; u < kFastSplits; ++u)
#pragma unroll
        for (int e = 0; e < EP; ++e) tmp[u][e] = pp[e][(long long)min(u, nsa[e] - 1) * qs];
#pragma unroll
      for (int u = 0; u < kFastSplits; ++u)
#pragma unroll
        for (int e = 0; e < EP; ++e)
          if (u < nse[e]) w[e] = cadd(w[e], tmp[u][e]);
    } else {
      for (int q0 = 0; q0 < nsmax; q0 += 4) {   // four splits at a time
        cd tmp[4][EP];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int e = 0; e < EP; ++e) tmp[u][e] = q0 + u < nse[e] ? pp[e][(q0 + u) * qs] : cmk(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int e = 0; e < EP; ++e)
            if (q0 + u < nse[e]) w[e] = cadd(w[e], tmp[u][e]);
      }
    }
    if (!first) load_v();
    // first step: the product is of w0, so M V_0 = (w0 - partials) / beta;
    // later ones: v_j - partials, v_j from the registers just loaded
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
      cd vje = vv[0][e];
#pragma unroll
      for (int v = 1; v < kFastV; ++v)
        if (v == j) vje = vv[v][e];
      w[e] = i < n ? (first ? csub(vv[0][e], cscale(w[e], inv_beta)) : csub(vje, w[e])) : cmk(0.0, 0.0);
    }
  } else {
    if (!first) load_v();
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int i = t + e * NT;
      w[e] = i < n ? src.w[i] : cmk(0.0, 0.0);
    }
  }
  for (int pass = 0; pass < 2; ++pass) {
    cd acc[kFastV];
#pragma unroll
    for (int v = 0; v < kFastV; ++v) {
      acc[v] = cmk(0.0, 0.0);
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
      cd r = cmk(0.0, 0.0);
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
  cd acc = cmk(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < EP; ++e) acc = cfma(cconj(w[e]), w[e], acc);
  acc = wave_sum(acc);
  if ((t & 63) == 0) red[t >> 6][0] = acc;
  __syncthreads();
  cd nr2 = cmk(0.0, 0.0);
  for (int q = 0; q < NT / 64; ++q) nr2 = cadd(nr2, red[q][0]);
  const double nr = sqrt(fmax(nr2.x, 0.0));
  const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
  if (!last) {
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
    return;
  }
  // last step: the least-squares solve and z = V y, with V_0..V_{k-1} of this
  // thread's entries still in registers (V_k is not needed)
  __shared__ cd Hs[(kFastV + 1) * kFastV];
  __shared__ cd y[kFastV];
  __shared__ cd b2s;
  const int k = ends.k, ldh = k + 1;
  const cd* H = Hcol - (long long)j * ldh;   // the problem's H
  if (t < j * ldh) Hs[t] = H[t];   // columns 0..j-1 (j * ldh <= 30 < NT)
  if (t < ldh) Hs[j * ldh + t] = t <= j ? hsum[t] : (t == j + 1 ? cmk(nr, 0.0) : cmk(0.0, 0.0));
  if (t == 0) b2s = ends.beta2[qp];   // (k = 1: written by this launch, by this thread)
  __syncthreads();
  if (t < 64) lsq_wave(Hs, ldh, k, sqrt(fmax(b2s.x, 0.0)), y);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int i = t + e * NT;
    cd acc = cmk(0.0, 0.0);
#pragma unroll
    for (int v = 0; v < kFastV; ++v)
      if (v < k) acc = cadd(acc, cmul(y[v], vv[v][e]));
    if (i < n) ends.vout[sidx[e]] = acc;
  }
}

// y = argmin |beta e1 - H y|, x = V y, vec[idx] = x.
__global__ __launch_bounds__(kCT) void coarse_finish_kernel(const cd* H, int k, int hsize, const cd* beta2,
                                                            const cd* V, int n, long long vq, const int* idx, cd* vec) {
  __shared__ cd y[kMaxCoarse];
  const int q = blockIdx.x;
  H += (long long)q * hsize;
  beta2 += q;
  V += (long long)q * vq;
  idx += (long long)q * n;
  __shared__ cd R[kMaxCoarse + 1][kMaxCoarse];
  __shared__ cd gv[kMaxCoarse + 1];
  // H and beta^2 staged in LDS by the whole workgroup in one round trip: the
  // serial solve below would otherwise wait on its global loads one by one
  __shared__ cd Hs[(kMaxCoarse + 1) * kMaxCoarse];
  __shared__ cd b2s;
  for (int i = threadIdx.x; i < (k + 1) * k; i += kCT) Hs[i] = H[i];
  if (threadIdx.x == 0) b2s = beta2[0];
  __syncthreads();
  if (threadIdx.x == 0) lsq_small(Hs, k + 1, k, &b2s, y, nullptr, R, gv);
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

namespace {
template <class M>
hipError_t skeleton_apply_t(const Geom& g, const M* T, const cd* gin, cd* out, bool zero_physical,
                            hipStream_t st, int nq) {
  dim3 grid(g.nboxes * nq, (g.b + kRows - 1) / kRows);
  const long long nslots = (long long)g.nx * g.ny * 4 * g.p;
  hipError_t e0 = allow_lds(skeleton_apply_kernel<M>, (size_t)g.b * sizeof(cd));
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(skeleton_apply_kernel<M>, grid, dim3(kRows), (size_t)g.b * sizeof(cd), st, g, T, gin,
                     out, zero_physical ? 1 : 0, nslots);
  return hipPeekAtLastError();
}
}  // namespace

hipError_t skeleton_apply(const Geom& g, const cd* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st, int nq) {
  return skeleton_apply_t(g, T, gin, out, zero_physical, st, nq);
}

hipError_t skeleton_apply(const Geom& g, const cf* T, const cd* gin, cd* out, bool zero_physical,
                          hipStream_t st, int nq) {
  return skeleton_apply_t(g, T, gin, out, zero_physical, st, nq);
}

hipError_t rhs_build(const Geom& g, const cd* T, const cd* H, const cd* t, cd* rhs, hipStream_t st) {
  hipLaunchKernelGGL(rhs_kernel, dim3(g.nx * g.ny), dim3(kRows), 0, st, g, T, H, t, rhs);
  return hipPeekAtLastError();
}




hipError_t index_gather(const int* idx, int n, const cd* vec, cd* out, hipStream_t st, int nq,
                        long long ostride) {
  const long long ntot = (long long)n * nq;
  hipLaunchKernelGGL(index_gather_kernel, dim3(grid_for(ntot)), dim3(256), 0, st, idx, n, ntot, vec, out,
                     ostride ? ostride : n);
  return hipPeekAtLastError();
}

hipError_t index_scatter(const int* idx, int n, const cd* in, cd* vec, hipStream_t st, int nq,
                         long long istride) {
  const long long ntot = (long long)n * nq;
  hipLaunchKernelGGL(index_scatter_kernel, dim3(grid_for(ntot)), dim3(256), 0, st, idx, n, ntot, in,
                     istride ? istride : n, vec);
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

hipError_t vcopy_zero(const cd* src, cd* dst, cd* zero, long long n, hipStream_t st) {
  hipLaunchKernelGGL(copy_zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, zero, n);
  return hipPeekAtLastError();
}

hipError_t vcopy(const cd* src, cd* dst, long long n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
  return hipPeekAtLastError();
}

hipError_t vcopy_at(const cd* src, cd* dst, long long n, const int* isrc, const int* idst, long long stride,
                    hipStream_t st) {
  hipLaunchKernelGGL(copy_at_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n, isrc, idst, stride);
  return hipPeekAtLastError();
}

hipError_t counter_set(int* c, int value, hipStream_t st) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, c, value, 0);
  return hipPeekAtLastError();
}

hipError_t counter_add(int* c, int value, hipStream_t st) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, c, value, 1);
  return hipPeekAtLastError();
}

int dot_blocks(long long n) {
  long long b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > kMaxDotBlocks ? kMaxDotBlocks : b));
}

hipError_t multi_dot(const cd* V, long long vstride, int nvec, const cd* w, long long n, cd* partial,
                     cd* out, bool accumulate, hipStream_t st, int nq, long long ostride, const int* nvdev,
                     cd* selfout) {
  if (nvec <= 0) return hipSuccess;
  const int nblk = dot_blocks(n);
  const int rows = nvec + (selfout ? 1 : 0);
  hipLaunchKernelGGL(dot_stage1_kernel, dim3(nblk, rows, nq), dim3(256), 0, st, V, vstride, w, n, partial,
                     nblk, nvdev, selfout ? 1 : 0);
  hipError_t err = hipPeekAtLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(dot_stage2_kernel, dim3(rows, nq), dim3(256), 0, st, partial, nblk, out,
                     accumulate ? 1 : 0, ostride, nvdev, selfout);
  return hipPeekAtLastError();
}

hipError_t axpy_normalize(const cd* V, long long vstride, int nvec, const cd* h, long long hstride, const cd* w,
                          long long n, const cd* nrm2, long long nstride, cd* out, cd* hout, long long houtstride,
                          hipStream_t st, int nq, const int* nvdev, const int* jdev, long long jstride) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_normalize_kernel, dim3(grid_for(n), nq), dim3(256), 0, st, V, vstride, nvec, h, hstride,
                     w, n, nrm2, nstride, out, hout, houtstride, nvdev, jdev, jstride);
  return hipPeekAtLastError();
}

hipError_t multi_axpy(const cd* V, long long vstride, int nvec, const cd* h, cd* w, long long n, int sign,
                      hipStream_t st, int nq, long long hstride, const int* nvdev) {
  if (nvec <= 0) return hipSuccess;
  const long long ntot = n * nq;
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(ntot)), dim3(256), 0, st, V, vstride, nvec, h, hstride,
                     w, n, ntot, sign, nvdev);
  return hipPeekAtLastError();
}

hipError_t normalize(const cd* w, const cd* nrm2, cd* out, long long n, cd* hout, hipStream_t st, int nq,
                     long long nstride, long long hstride, const int* jdev, long long jstride) {
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n), nq), dim3(256), 0, st, w, nrm2, nstride, out, n, hout,
                     hstride, jdev, jstride);
  return hipPeekAtLastError();
}


hipError_t coarse_start(const int* idx, int n, const cd* vec, cd* V, long long vq, cd* H, int hsize, cd* beta2,
                        int nq, hipStream_t st) {
  hipLaunchKernelGGL(coarse_start_kernel, dim3(nq), dim3(kCT), 0, st, idx, n, vec, V, vq, H, hsize, beta2);
  return hipPeekAtLastError();
}

bool coarse_fast_ok(int n, int k) {
  return k >= 1 && k <= kFastV && n <= 2 * 1024;
}

hipError_t coarse_arnoldi(cd* V, int n, long long vq, int j, const CoarseW& src, cd* wtmp, cd* Hcol, int hsize,
                          int nq, hipStream_t st, const CoarseEnds* ends) {
  if (n < 1 || j < 0 || j + 1 > kMaxCoarse) return hipErrorInvalidValue;
  const CoarseEnds none{};
  if (ends) {
    // the fused start and end exist only on the register kernels
    if (!coarse_fast_ok(n, ends->k) || !ends->idx || !ends->vin || !ends->vout || !ends->beta2 || !src.part)
      return hipErrorInvalidValue;
  }
  const CoarseEnds& ce = ends ? *ends : none;
  if (j < kFastV && n <= 2 * 512)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<2, 512>), dim3(nq), dim3(512), 0, st, V, n, vq, j, src, Hcol,
                       hsize, ce);
  else if (j < kFastV && n <= 2 * 1024)   // more loads in flight on the one CU
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<2, 1024>), dim3(nq), dim3(1024), 0, st, V, n, vq, j, src, Hcol,
                       hsize, ce);
  else if (j < kFastV && n <= 4 * 512)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<4, 512>), dim3(nq), dim3(512), 0, st, V, n, vq, j, src, Hcol,
                       hsize, ce);
  else if (j < kFastV && n <= 4 * 256)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<4, 256>), dim3(nq), dim3(256), 0, st, V, n, vq, j, src, Hcol,
                       hsize, ce);
  else if (j < kFastV && n <= 8 * 256)
    hipLaunchKernelGGL((coarse_arnoldi_fast_kernel<8, 256>), dim3(nq), dim3(256), 0, st, V, n, vq, j, src, Hcol,
                       hsize, ce);
  else   // (16 entries per thread would spill to scratch, which the runtime must allocate at dispatch)
    hipLaunchKernelGGL(coarse_arnoldi_kernel, dim3(nq), dim3(kCT), 0, st, V, n, vq, j, src, wtmp, Hcol, hsize);
  return hipPeekAtLastError();
}

hipError_t coarse_finish(const cd* H, int k, int hsize, const cd* beta2, const cd* V, int n, long long vq,
                         const int* idx, cd* vec, int nq, hipStream_t st) {
  if (k < 1 || k > kMaxCoarse) return hipErrorInvalidValue;
  hipLaunchKernelGGL(coarse_finish_kernel, dim3(nq), dim3(kCT), 0, st, H, k, hsize, beta2, V, n, vq, idx, vec);
  return hipPeekAtLastError();
}

}  // namespace hps
