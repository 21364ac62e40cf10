// Streaming kernels of the multigrid V-cycle (Sec. 4.3): batched split-K complex
// GEMVs with the gathers from / scatters to the canonical skeleton vector fused
// into their load and store paths, and one-workgroup-per-pair kernels that run a
// whole level of the V-cycle for levels with many small pairs.
//
// All of this is HBM-bound: every stored operator is read once per application,
// 16 bytes per complex entry, with column-major tiles read 64 rows at a time so
// that a wavefront loads 1 KB contiguous per column.
#include "common.h"
#include "gemv.h"

namespace hps {

namespace {

constexpr int kRowsT = 64;   // rows per tile (one per lane)
constexpr int kThreads = 256;

__device__ inline cd load_x(const VecIn& x, int b, int k) {
  if (x.p) return x.p[(long long)b * x.stride + k];
  const int s = x.tab[(long long)b * x.tstride + k];
  return s >= 0 ? x.vec[s] : cmk(0.0, 0.0);
}

__device__ inline void store_y(const VecOut& y, int b, int i, cd v) {
  if (y.y0) v = cfma(y.beta, y.y0[(long long)b * y.y0stride + i], v);
  if (y.p) y.p[(long long)b * y.stride + i] = v;
  if (y.vec) {
    const int s = y.tab[(long long)b * y.tstride + i];
    if (s >= 0) y.vec[s] = y.add ? cadd(y.vec[s], v) : v;
  }
}

// grid: x = row tile * nsplit (flattened), y = batch, z = descriptor.
template <class Mt>
__global__ __launch_bounds__(kThreads) void gemv_kernel(GemvBatchT<Mt> gb, cd* partial) {
  __shared__ cd xs[kGemvKChunkMax];
  __shared__ cd red[4][kRowsT];
  const GemvDescT<Mt>& d = gb.d[blockIdx.z];
  const int tiles = (d.M_ + kRowsT - 1) / kRowsT;
  const int nsplit = gb.nsplit[blockIdx.z];
  if ((int)blockIdx.x >= tiles * nsplit) return;
  const int tile = blockIdx.x % tiles, split = blockIdx.x / tiles;
  const int b = blockIdx.y;
  const int kc = (d.K + nsplit - 1) / nsplit;
  const int k0 = split * kc;
  const int k1 = min(d.K, k0 + kc);
  const int t = threadIdx.x, lane = t & 63, grp = t >> 6;
  for (int k = k0 + t; k < k1; k += kThreads) xs[k - k0] = load_x(d.x, b, k);
  __syncthreads();
  const int r = tile * kRowsT + lane;
  cd acc = cmk(0.0, 0.0);
  if (r < d.M_) {
    const Mt* Ab = d.A.base + (long long)b * d.A.bstride;
    const long long row = imap(d.A.r, r);
    int k = k0 + grp;
    constexpr int U = 8;  // independent loads in flight per thread
    for (; k + 4 * (U - 1) < k1; k += 4 * U) {
      Mt a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = Ab[(long long)imap(d.A.c, k + 4 * u) * d.A.ld + row];
#pragma unroll
      for (int u = 0; u < U; ++u) acc = cfma(to_cd(a[u]), xs[k + 4 * u - k0], acc);
    }
    for (; k < k1; k += 4) acc = cfma(to_cd(Ab[(long long)imap(d.A.c, k) * d.A.ld + row]), xs[k - k0], acc);
  }
  red[grp][lane] = acc;
  __syncthreads();
  if (nsplit == 1 && !gb.partials_only) {
    if (grp == 0 && r < d.M_) {
      const cd s = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
      store_y(d.y, b, r, cmul(d.alpha, s));
    }
    return;
  }
  if (grp == 0 && r < d.M_) {
    const cd s = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
    partial[gb.poff[blockIdx.z] + ((long long)split * gb.batch + b) * d.M_ + r] = s;
  }
}

// Sum the split-K partials in split order (deterministic) and apply the epilogue.
// (A device-scope fence per workgroup to let the last split reduce in place
// forces an L2 write-back on this chip and costs more than this launch.)
template <class Mt>
__global__ void gemv_reduce_kernel(GemvBatchT<Mt> gb, const cd* partial) {
  const GemvDescT<Mt>& d = gb.d[blockIdx.z];
  const int nsplit = gb.nsplit[blockIdx.z];
  if (nsplit == 1) return;
  const int b = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.M_; r += gridDim.x * blockDim.x) {
    cd s = cmk(0.0, 0.0);
    for (int q = 0; q < nsplit; ++q)
      s = cadd(s, partial[gb.poff[blockIdx.z] + ((long long)q * gb.batch + b) * d.M_ + r]);
    store_y(d.y, b, r, cmul(d.alpha, s));
  }
}

// ---- one workgroup per pair: a whole V-cycle level ---------------------------
// y[i] = (y0 ? y0[i] : 0) + sum_k A(rm(i), cm(k)) x[k]; x, y0, y in LDS.
template <class Mt, int NT>
__device__ void wg_gemv(const Mt* A, int ld, IdxMap rm, IdxMap cm, int M, int K, const cd* x,
                        const cd* y0, cd* y, cd* red) {
  const int t = threadIdx.x;
  const int RT = M < kRowsT ? M : kRowsT;
  const int G = NT / RT;
  const int r = t % RT, g = t / RT;
  constexpr int U = 8;  // independent loads in flight per thread
  for (int r0 = 0; r0 < M; r0 += RT) {
    const int row = r0 + r;
    cd acc = cmk(0.0, 0.0);
    if (g < G && row < M) {
      const long long ar = imap(rm, row);
      int c = g;
      for (; c + (U - 1) * G < K; c += U * G) {
        Mt a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = A[(long long)imap(cm, c + u * G) * ld + ar];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = cfma(to_cd(a[u]), x[c + u * G], acc);
      }
      for (; c < K; c += G) acc = cfma(to_cd(A[(long long)imap(cm, c) * ld + ar]), x[c], acc);
    }
    if (g < G) red[g * RT + r] = acc;
    __syncthreads();
    if (t < RT && r0 + t < M) {
      cd s = y0 ? y0[r0 + t] : cmk(0.0, 0.0);
      for (int q = 0; q < G; ++q) s = cadd(s, red[q * RT + t]);
      y[r0 + t] = s;
    }
    __syncthreads();
  }
}

// Down sweep of one pair: z0 = A^-1 r_x (kept in Z0), then the exterior
// residual rows across the kept faces receive C~ z0:
// w[dtab(P.E1)] += T^P_{E1,a} z0_P, w[dtab(Q.E2)] += T^Q_{E2,b} z0_Q.
template <class Mt, int NT>
__global__ __launch_bounds__(NT) void vc_down_small_kernel(SmallLevelT<Mt> a, cd* vec) {
  extern __shared__ cd sm[];
  const int m = a.m, e = a.e, m2 = 2 * m;
  cd* r = sm;
  cd* z0 = r + m2;
  cd* dd = z0 + m2;
  cd* red = dd + e;
  const int j = blockIdx.x, t = threadIdx.x;
  const long long bb = (long long)a.g.b * a.g.b;
  const Mt* TP = a.T + (2LL * j) * bb;
  const Mt* TQ = TP + bb;
  const int* xt = a.xtab + (long long)j * m2;
  const int* dt = a.dtab + (long long)j * 2 * e;
  for (int i = t; i < m2; i += NT) r[i] = vec[xt[i]];
  __syncthreads();
  wg_gemv<Mt, NT>(a.Ainv + (long long)j * m2 * m2, m2, im_off(0), im_off(0), m2, m2, r, nullptr, z0, red);
  for (int i = t; i < m2; i += NT) a.Z0[(long long)j * m2 + i] = z0[i];
  wg_gemv<Mt, NT>(TP, a.g.b, a.E1, im_off(a.a0), e, m, z0 + m, nullptr, dd, red);
  for (int i = t; i < e; i += NT) {
    const int s = dt[i];
    if (s >= 0) vec[s] = cadd(vec[s], dd[i]);
  }
  __syncthreads();
  wg_gemv<Mt, NT>(TQ, a.g.b, a.E2, im_off(a.b0), e, m, z0, nullptr, dd, red);
  for (int i = t; i < e; i += NT) {
    const int s = dt[e + i];
    if (s >= 0) vec[s] = cadd(vec[s], dd[i]);
  }
}

// Up sweep of one pair: x = z0 + X y with y the kept-face values of z.
template <class Mt, int NT>
__global__ __launch_bounds__(NT) void vc_up_small_kernel(SmallLevelT<Mt> a, cd* z) {
  extern __shared__ cd sm[];
  const int m = a.m, e = a.e, m2 = 2 * m, e2 = 2 * e;
  cd* y = sm;
  cd* z0 = y + e2;
  cd* x = z0 + m2;
  cd* red = x + m2;
  const int j = blockIdx.x, t = threadIdx.x;
  const int* yt = a.ytab + (long long)j * e2;
  const int* xt = a.xtab + (long long)j * m2;
  for (int i = t; i < e2; i += NT) {
    const int s = yt[i];
    y[i] = s >= 0 ? z[s] : cmk(0.0, 0.0);
  }
  for (int i = t; i < m2; i += NT) z0[i] = a.Z0[(long long)j * m2 + i];
  __syncthreads();
  wg_gemv<Mt, NT>(a.X + (long long)j * m2 * e2, m2, im_off(0), im_off(0), m2, e2, y, z0, x, red);
  for (int i = t; i < m2; i += NT) z[xt[i]] = x[i];
}

}  // namespace

int gemv_nsplit(int M, int K, int batch) {
  const int tiles = (M + kRowsT - 1) / kRowsT;
  int ns = (kGemvTargetBlocks + tiles * batch - 1) / (tiles * batch);
  ns = std::max(1, std::min(ns, (K + 63) / 64));
  while ((K + ns - 1) / ns > kGemvKChunkMax) ++ns;
  return ns;
}

template <class Mt>
hipError_t zgemv_batched(const GemvDescT<Mt>* d, int nd, int batch, cd* partial, hipStream_t st) {
  if (nd <= 0 || nd > kGemvMaxDesc || batch <= 0) return hipErrorInvalidValue;
  GemvBatchT<Mt> gb{};
  gb.batch = batch;
  int gx = 0;
  long long poff = 0;
  bool any_split = false;
  for (int i = 0; i < nd; ++i) {
    gb.d[i] = d[i];
    const int tiles = (d[i].M_ + kRowsT - 1) / kRowsT;
    const int ns = gemv_nsplit(d[i].M_, d[i].K, batch);
    gb.nsplit[i] = ns;
    gb.poff[i] = poff;
    if (ns > 1) { poff += (long long)ns * batch * d[i].M_; any_split = true; }
    gx = std::max(gx, tiles * ns);
  }
  if (any_split && !partial) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gemv_kernel<Mt>, dim3(gx, batch, nd), dim3(kThreads), 0, st, gb, partial);
  hipError_t err = hipPeekAtLastError();
  if (err != hipSuccess || !any_split) return err;
  int maxM = 0;
  for (int i = 0; i < nd; ++i) maxM = std::max(maxM, d[i].M_);
  hipLaunchKernelGGL(gemv_reduce_kernel<Mt>, dim3((maxM + 255) / 256, batch, nd), dim3(256), 0, st, gb, partial);
  return hipPeekAtLastError();
}

template <class Mt>
hipError_t zgemv_partials(const GemvDescT<Mt>* d, int nd, int batch, cd* partial, GemvPartLayout* lay,
                          hipStream_t st, int max_split) {
  if (nd <= 0 || nd > kGemvMaxDesc || batch <= 0 || !partial || !lay) return hipErrorInvalidValue;
  GemvBatchT<Mt> gb{};
  gb.batch = batch;
  gb.partials_only = 1;
  int gx = 0;
  long long poff = 0;
  for (int i = 0; i < nd; ++i) {
    gb.d[i] = d[i];
    const int tiles = (d[i].M_ + kRowsT - 1) / kRowsT;
    int ns = gemv_nsplit(d[i].M_, d[i].K, batch);
    if (max_split > 0 && ns > max_split && (d[i].K + max_split - 1) / max_split <= kGemvKChunkMax) ns = max_split;
    gb.nsplit[i] = ns;
    gb.poff[i] = poff;
    lay->nsplit[i] = ns;
    lay->poff[i] = poff;
    poff += (long long)ns * batch * d[i].M_;
    gx = std::max(gx, tiles * ns);
  }
  hipLaunchKernelGGL(gemv_kernel<Mt>, dim3(gx, batch, nd), dim3(kThreads), 0, st, gb, partial);
  return hipPeekAtLastError();
}

// Threads per pair: 1024 when the level has at most 512 pairs (larger matrices,
// fewer workgroups: more loads in flight per pair), 256 otherwise.
constexpr int kSmallWide = 1024;
inline bool small_wide(int pairs) { return pairs <= 512; }

size_t small_level_lds(int m, int e) {
  return sizeof(cd) * (size_t)(std::max(4 * m + e, 2 * e + 4 * m) + kSmallWide);
}

template <class Mt, int NT>
hipError_t launch_down(const SmallLevelT<Mt>& a, int pairs, cd* vec, hipStream_t st) {
  const size_t lds = small_level_lds(a.m, a.e);
  hipError_t err = allow_lds(vc_down_small_kernel<Mt, NT>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((vc_down_small_kernel<Mt, NT>), dim3(pairs), dim3(NT), lds, st, a, vec);
  return hipPeekAtLastError();
}

template <class Mt, int NT>
hipError_t launch_up(const SmallLevelT<Mt>& a, int pairs, cd* z, hipStream_t st) {
  const size_t lds = small_level_lds(a.m, a.e);
  hipError_t err = allow_lds(vc_up_small_kernel<Mt, NT>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((vc_up_small_kernel<Mt, NT>), dim3(pairs), dim3(NT), lds, st, a, z);
  return hipPeekAtLastError();
}

template <class Mt>
hipError_t vc_down_small(const SmallLevelT<Mt>& a, int pairs, cd* vec, hipStream_t st) {
  return small_wide(pairs) ? launch_down<Mt, kSmallWide>(a, pairs, vec, st) : launch_down<Mt, kThreads>(a, pairs, vec, st);
}

template <class Mt>
hipError_t vc_up_small(const SmallLevelT<Mt>& a, int pairs, cd* z, hipStream_t st) {
  return small_wide(pairs) ? launch_up<Mt, kSmallWide>(a, pairs, z, st) : launch_up<Mt, kThreads>(a, pairs, z, st);
}

template hipError_t zgemv_batched<cd>(const GemvDescT<cd>*, int, int, cd*, hipStream_t);
template hipError_t zgemv_batched<cf>(const GemvDescT<cf>*, int, int, cd*, hipStream_t);
template hipError_t zgemv_partials<cd>(const GemvDescT<cd>*, int, int, cd*, GemvPartLayout*, hipStream_t, int);
template hipError_t vc_down_small<cd>(const SmallLevelT<cd>&, int, cd*, hipStream_t);
template hipError_t vc_down_small<cf>(const SmallLevelT<cf>&, int, cd*, hipStream_t);
template hipError_t vc_up_small<cd>(const SmallLevelT<cd>&, int, cd*, hipStream_t);
template hipError_t vc_up_small<cf>(const SmallLevelT<cf>&, int, cd*, hipStream_t);

}  // namespace hps
