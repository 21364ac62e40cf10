// Batched complex GEMM (FP64 or FP32 storage) on the CDNA4 matrix cores
// (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32) and batched strided copies.  All matrices are column-major; operands are
// addressed through IdxMap row/column selections so that sub-blocks of the
// box maps (a side, all sides but one, a permuted scatter) are read and written
// in place.
//
// Complex product by the 3M scheme on real MFMA tiles (three real products per
// complex one instead of four):
//   t1 += Ar Br,  t2 += Ai Bi,  t3 += (Ar + Ai)(Br + Bi);
//   Re = t1 - t2,  Im = t3 - t1 - t2.
// Tile: BM x BN per workgroup, waves arranged WM x WN, each wave owning
// (BM/WM) x (BN/WN) outputs as 16x16 MFMA tiles; K staged through LDS in
// chunks of KT complex, the next chunk's global loads (FP32: the next two
// chunks') issued into registers before the current chunk is multiplied.
#include "common.h"
#include "host.h"

namespace hps {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KT = 16;

// One 16x16x4 real MFMA per precision, and where its result lands: lane l,
// element v -> row(l, v), column l % 16 (the two layouts differ; both were
// checked on gfx950).
template <class T> struct Mfma;
template <> struct Mfma<cd> {
  typedef d4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mfma<cf> {
  typedef f4 acc;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

// One BM x BN output tile (tile index `tile`, batch entry b) of a GEMM; every
// thread of the workgroup calls it with the same arguments.
template <class T, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void gemm_tile(const GemmArgsT<T>& a, int tile, int b) {
  typedef typename Mfma<T>::acc acc_t;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  // LDS: the K chunk (As, Bs[k] padded: the 16 k-rows of a column land in
  // different banks); after the last chunk the same bytes hold the FP32 output
  // tile (BM x BN, or half its columns per pass at 64 x 64) for the epilogue
  constexpr int kCP = (sizeof(T) == sizeof(cf) && BM == 64) ? BN / 2 : BN;   // columns per epilogue pass
  constexpr size_t kABytes = sizeof(T) * KT * BM, kBBytes = sizeof(T) * KT * (BN + 1);
  constexpr size_t kCBytes = sizeof(T) == sizeof(cf) ? sizeof(T) * kCP * (BM + 1) : 0;
  __shared__ __align__(16) unsigned char smem[(kABytes + kBBytes) > kCBytes ? (kABytes + kBBytes) : kCBytes];
  T (*As)[BM] = reinterpret_cast<T (*)[BM]>(smem);
  T (*Bs)[BN + 1] = reinterpret_cast<T (*)[BN + 1]>(smem + kABytes);
  const int tilesM = (a.M + BM - 1) / BM;
  const int m0 = (tile % tilesM) * BM;
  const int n0 = (tile / tilesM) * BN;
  const int tid = threadIdx.x;
  // Physical rows/columns of a live tile are written as exact zeros: their
  // inputs (skipped entries of earlier products) are never computed, so they
  // must not leak into the stored maps, where they meet zero data.
  __shared__ unsigned char dead_r[BM], dead_c[BN];
  if (a.skip.enabled) {
    __shared__ int live_r, live_c;
    int bx, by;
    box_xy(a.skip.g, b % a.skip.nbox, bx, by);
    if (tid == 0) {
      live_r = a.skip.row_y ? 0 : 1;
      live_c = a.skip.col_y ? 0 : 1;
    }
    __syncthreads();
    if (tid < BM) {
      const bool dead = a.skip.row_y && m0 + tid < a.M &&
                        y_physical(a.skip, bx, by, m0 + tid + a.skip.row_off);
      dead_r[tid] = dead;
      if (a.skip.row_y && m0 + tid < a.M && !dead) live_r = 1;
    }
    if (tid < BN) {
      const bool dead = a.skip.col_y && n0 + tid < a.N &&
                        y_physical(a.skip, bx, by, n0 + tid + a.skip.col_off);
      dead_c[tid] = dead;
      if (a.skip.col_y && n0 + tid < a.N && !dead) live_c = 1;
    }
    __syncthreads();
    if (!live_r || !live_c) return;
  }
  const T* Ab = a.A.base + (long long)b * a.A.bstride;
  const T* Bb = a.B.base + (long long)b * a.B.bstride;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lk = lane >> 4;

  // Fixed per-thread load slots: A(i, k) with i = tid % BM, k = tid / BM + s KSA;
  // B(k, j) with k = tid % KT, j = tid / KT + s JSB.  Row and column maps that
  // do not change along K are resolved once.
  constexpr int SA = BM * KT / NT, SB = BN * KT / NT;
  constexpr int KSA = NT / BM, JSB = NT / KT;
  static_assert(SA * NT == BM * KT && SB * NT == BN * KT, "tile / thread mismatch");
  const int ia = tid % BM, ka = tid / BM;
  const int kb = tid % KT, jb = tid / KT;
  const bool rowok = m0 + ia < a.M;
  const long long rA = rowok ? imap(a.A.r, m0 + ia) : 0;
  long long cB[SB];
  bool colok[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int gj = n0 + jb + s * JSB;
    colok[s] = gj < a.N;
    cB[s] = colok[s] ? (long long)imap(a.B.c, gj) * a.B.ld : 0;
  }
  T ra[SA], rb[SB];
  bool va[SA], vb[SB];
  // The chunk's K-direction map lookups (a table read or an offset) all come
  // before its data loads, and the data loads are unconditional (an entry
  // outside the operand reads offset 0 of the same matrix; its validity is
  // applied when the chunk is stored to LDS): no wait separates the loads of
  // a chunk, and none is needed before the multiply that they overlap.
  auto fetch = [&](int k0) {
    long long offA[SA];
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int gk = k0 + ka + s * KSA;
      va[s] = rowok && gk < a.K;
      offA[s] = va[s] ? (long long)imap_arith(a.A.c, gk) * a.A.ld + rA : 0;
    }
    const int gk = k0 + kb;
    const bool kok = gk < a.K;
    const long long rB = kok ? imap_arith(a.B.r, gk) : 0;
#pragma unroll
    for (int s = 0; s < SA; ++s) ra[s] = Ab[offA[s]];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      vb[s] = kok && colok[s];
      rb[s] = Bb[vb[s] ? cB[s] + rB : 0];
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int s = 0; s < SA; ++s) As[ka + s * KSA][ia] = va[s] ? ra[s] : cx<T>::make(0.0, 0.0);
#pragma unroll
    for (int s = 0; s < SB; ++s) Bs[kb][jb + s * JSB] = vb[s] ? rb[s] : cx<T>::make(0.0, 0.0);
  };

  // complex products by the 3M scheme: t1 = Ar Br, t2 = Ai Bi and
  // t3 = (Ar + Ai)(Br + Bi), then Re = t1 - t2, Im = t3 - t1 - t2 (three real
  // MFMAs per complex product instead of four)
  acc_t t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      t1[i][j] = acc_t{0, 0, 0, 0};
      t2[i][j] = acc_t{0, 0, 0, 0};
      t3[i][j] = acc_t{0, 0, 0, 0};
    }

  // the chunk in LDS times its 3M products
  auto mult = [&]() {
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = As[kk + lk][wm * (BM / WM) + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = Bs[kk + lk][wn * (BN / WN) + j * 16 + lr];
      decltype(av[0].x) as[TM], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) as[i] = av[i].x + av[i].y;
#pragma unroll
      for (int j = 0; j < TN; ++j) bs[j] = bv[j].x + bv[j].y;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          t1[i][j] = Mfma<T>::mma(av[i].x, bv[j].x, t1[i][j]);
          t2[i][j] = Mfma<T>::mma(av[i].y, bv[j].y, t2[i][j]);
          t3[i][j] = Mfma<T>::mma(as[i], bs[j], t3[i][j]);
        }
    }
  };
  if constexpr (sizeof(T) == sizeof(cf)) {
    // FP32: two chunks ahead (chunk c in LDS, chunk c + 1 in the second
    // register set, chunk c + 2 being fetched into the first): a chunk's
    // products take half as long as in FP64, and one chunk of lead left the
    // loads exposed.  (FP64 tiles keep one chunk: a second register set
    // would halve their occupancy.)
    T ra2[SA], rb2[SB];
    bool va2[SA], vb2[SB];
    auto swap_sets = [&]() {
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const T t = ra[s]; ra[s] = ra2[s]; ra2[s] = t;
        const bool v = va[s]; va[s] = va2[s]; va2[s] = v;
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const T t = rb[s]; rb[s] = rb2[s]; rb2[s] = t;
        const bool v = vb[s]; vb[s] = vb2[s]; vb2[s] = v;
      }
    };
    fetch(0);
    stash();
    if (KT < a.K) fetch(KT);
    swap_sets();   // chunk 1 in the second set
    __syncthreads();
    for (int k0 = 0; k0 < a.K; k0 += KT) {
      if (k0 + 2 * KT < a.K) fetch(k0 + 2 * KT);   // into the first set
      mult();
      __syncthreads();
      if (k0 + KT < a.K) {
        swap_sets();   // chunk c + 1 to the first set, chunk c + 2 to the second
        stash();
        __syncthreads();
      }
    }
  } else {
    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < a.K; k0 += KT) {
      // the next chunk's loads are in flight while this one is multiplied
      const bool more = k0 + KT < a.K;
      if (more) fetch(k0 + KT);
      mult();
      __syncthreads();
      if (more) {
        stash();
        __syncthreads();
      }
    }
  }

  acc_t accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      accr[i][j] = t1[i][j] - t2[i][j];
      acci[i][j] = t3[i][j] - t1[i][j] - t2[i][j];
    }
  T* Db = a.D + (long long)b * a.Dstride;
  const T* Cb = a.C.base ? a.C.base + (long long)b * a.C.bstride : nullptr;
  const bool use_c = (a.beta.x != 0.0 || a.beta.y != 0.0);
  // one output entry (tile row r, column c) with its epilogue
  auto emit = [&](int r, int c, T acc) {
    const int gi = m0 + r, gj = n0 + c;
    if (gi >= a.M || gj >= a.N) return;
    T* dst = Db + (long long)imap(a.dc, gj) * a.ldd + imap(a.dr, gi);
    if (a.skip.enabled && (dead_r[r] || dead_c[c])) {
      *dst = cx<T>::make(0.0, 0.0);
      return;
    }
    T out = cmul(a.alpha, acc);
    if (use_c) out = cfma(a.beta, Cb[(long long)imap(a.C.c, gj) * a.C.ld + imap(a.C.r, gi)], out);
    if (a.has_diag && gi == gj) out = cadd(out, a.diag_add);
    *dst = out;
  };
  // FP32 tiles with a short K (where the epilogue weighs most; every small
  // tile) go through LDS (the K-chunk buffers, free after the last chunk's
  // barrier) so that consecutive threads write (and read C at) consecutive
  // rows of a column; in the MFMA layout the 16 lanes of a row group hold 16
  // different columns, one cache line each.  64 x 64 tiles take two passes of
  // 32 columns, written by the waves holding them; with a long K their extra
  // barriers cost more than the coalescing gains.
  bool via_lds = false;
  if constexpr (sizeof(T) == sizeof(cf)) via_lds = BM <= 32 || a.K <= 64;
  if (via_lds) {
    T (*Cs)[BM + 1] = reinterpret_cast<T (*)[BM + 1]>(smem);
#pragma unroll
    for (int h = 0; h < BN / kCP; ++h) {
      if (h) __syncthreads();   // the previous pass's reads are done
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int c = wn * (BN / WN) + j * 16 + lr - h * kCP;
          if (c < 0 || c >= kCP) continue;   // wave-uniform: the column half of this wave
#pragma unroll
          for (int v = 0; v < 4; ++v)
            Cs[c][wm * (BM / WM) + i * 16 + Mfma<T>::row(lk, v)] = cx<T>::make(accr[i][j][v], acci[i][j][v]);
        }
      __syncthreads();
#pragma unroll 4
      for (int idx = tid; idx < BM * kCP; idx += NT)
        emit(idx % BM, h * kCP + idx / BM, Cs[idx / BM][idx % BM]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          emit(wm * (BM / WM) + i * 16 + Mfma<T>::row(lk, v), wn * (BN / WN) + j * 16 + lr,
               cx<T>::make(accr[i][j][v], acci[i][j][v]));
  }
}

template <class T, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void zgemm_kernel(GemmArgsT<T> a) {
  gemm_tile<T, BM, BN, WM, WN>(a, blockIdx.x, blockIdx.y);
}

// Up to kGemmGroup independent GEMMs in one launch: z = GEMM, x = tile, y =
// batch entry; workgroups past a GEMM's tiles or batch leave at once.
template <class T>
struct GemmGroupT {
  GemmArgsT<T> g[kGemmGroup];
};
template <class T, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void zgemm_group_kernel(GemmGroupT<T> grp) {
  const GemmArgsT<T>& a = grp.g[blockIdx.z];
  const int tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  if ((int)blockIdx.x >= tiles || (int)blockIdx.y >= a.batch) return;   // uniform over the workgroup
  gemm_tile<T, BM, BN, WM, WN>(a, blockIdx.x, blockIdx.y);
}

template <class T>
__global__ void zcopy2d_kernel(int M, int N, OperandT<T> S, T alpha, T* D, long long Dstride, int ldd,
                               IdxMap dr, IdxMap dc, PhysSkip skip) {
  const int b = blockIdx.y;
  const long long total = (long long)M * N;
  int bx = 0, by = 0;
  if (skip.enabled) box_xy(skip.g, b % skip.nbox, bx, by);
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M), j = (int)(idx / M);
    if (skip.enabled && ((skip.row_y && y_physical(skip, bx, by, i + skip.row_off)) ||
                         (skip.col_y && y_physical(skip, bx, by, j + skip.col_off))))
      continue;
    T v = cx<T>::make(0.0, 0.0);
    if (S.base) v = cmul(alpha, S.base[(long long)b * S.bstride + (long long)imap(S.c, j) * S.ld + imap(S.r, i)]);
    D[(long long)b * Dstride + (long long)imap(dc, j) * ldd + imap(dr, i)] = v;
  }
}

__global__ void convert_64_32_kernel(const cd* src, cf* dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = to_cf(src[i]);
}

__global__ void convert_32_64_kernel(const cf* src, cd* dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = to_cd(src[i]);
}

template <class T, int BM, int BN, int WM, int WN>
hipError_t launch(const GemmArgsT<T>& a, hipStream_t st) {
  const int tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN>), dim3(tiles, a.batch), dim3(64 * WM * WN), 0,
                     st, a);
  return hipPeekAtLastError();
}

}  // namespace

template <class T, int BM, int BN, int WM, int WN>
hipError_t launch_group(const GemmArgsT<T>* g, int n, hipStream_t st) {
  GemmGroupT<T> grp{};
  int tiles = 0, batch = 0;
  for (int i = 0; i < n; ++i) {
    grp.g[i] = g[i];
    tiles = std::max(tiles, ((g[i].M + BM - 1) / BM) * ((g[i].N + BN - 1) / BN));
    batch = std::max(batch, g[i].batch);
  }
  hipLaunchKernelGGL((zgemm_group_kernel<T, BM, BN, WM, WN>), dim3(tiles, batch, n), dim3(64 * WM * WN), 0, st,
                     grp);
  return hipPeekAtLastError();
}

template <class T>
hipError_t zgemm(const GemmArgsT<T>& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
  if (a.A.c.map || a.B.r.map) return hipErrorInvalidValue;   // K maps are offsets (imap_arith)
  // 64x64 tiles while they still give two workgroups per CU; 32x32 otherwise
  const long long t64 = (long long)((a.M + 63) / 64) * ((a.N + 63) / 64) * a.batch;
  if (a.M >= 48 && a.N >= 48 && t64 >= 512) return launch<T, 64, 64, 2, 2>(a, st);
  if (a.M >= 24 && a.N >= 24) return launch<T, 32, 32, 2, 2>(a, st);
  return launch<T, 16, 16, 1, 1>(a, st);
}

template <class T>
hipError_t zgemm_group(const GemmArgsT<T>* g, int n, hipStream_t st) {
  if (n < 1 || n > kGemmGroup) return hipErrorInvalidValue;
  // drop empty GEMMs; one left: the plain launch
  GemmArgsT<T> live[kGemmGroup];
  int k = 0;
  for (int i = 0; i < n; ++i) {
    if (g[i].A.c.map || g[i].B.r.map) return hipErrorInvalidValue;   // K maps are offsets (imap_arith)
    if (g[i].M > 0 && g[i].N > 0 && g[i].batch > 0) live[k++] = g[i];
  }
  if (k == 0) return hipSuccess;
  if (k == 1) return zgemm(live[0], st);
  // one tile shape for the group, by the same rule as a single GEMM applied to
  // the smallest dimensions and the summed 64 x 64 tile count
  int mn = 1 << 30;
  long long t64 = 0;
  for (int i = 0; i < k; ++i) {
    mn = std::min(mn, std::min(live[i].M, live[i].N));
    t64 += (long long)((live[i].M + 63) / 64) * ((live[i].N + 63) / 64) * live[i].batch;
  }
  if (mn >= 48 && t64 >= 512) return launch_group<T, 64, 64, 2, 2>(live, k, st);
  if (mn >= 24) return launch_group<T, 32, 32, 2, 2>(live, k, st);
  return launch_group<T, 16, 16, 1, 1>(live, k, st);
}

hipError_t convert_c64_c32(const cd* src, cf* dst, long long n, hipStream_t st) {
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(convert_64_32_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, src, dst, n);
  return hipPeekAtLastError();
}

hipError_t convert_c32_c64(const cf* src, cd* dst, long long n, hipStream_t st) {
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(convert_32_64_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, src, dst, n);
  return hipPeekAtLastError();
}

template <class T>
hipError_t zcopy2d(int M, int N, int batch, const OperandT<T>& S, T alpha, T* D, long long Dstride,
                   int ldd, IdxMap dr, IdxMap dc, hipStream_t st, const PhysSkip* skip) {
  PhysSkip none{};
  const PhysSkip sk = skip ? *skip : none;
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const long long total = (long long)M * N;
  int blocks = (int)std::min<long long>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(zcopy2d_kernel<T>, dim3(blocks, batch), dim3(256), 0, st, M, N, S, alpha, D,
                     Dstride, ldd, dr, dc, sk);
  return hipPeekAtLastError();
}

template hipError_t zgemm<cd>(const GemmArgsT<cd>&, hipStream_t);
template hipError_t zgemm<cf>(const GemmArgsT<cf>&, hipStream_t);
template hipError_t zgemm_group<cd>(const GemmArgsT<cd>*, int, hipStream_t);
template hipError_t zgemm_group<cf>(const GemmArgsT<cf>*, int, hipStream_t);
template hipError_t zcopy2d<cd>(int, int, int, const OperandT<cd>&, cd, cd*, long long, int, IdxMap,
                                IdxMap, hipStream_t, const PhysSkip*);
template hipError_t zcopy2d<cf>(int, int, int, const OperandT<cf>&, cf, cf*, long long, int, IdxMap,
                                IdxMap, hipStream_t, const PhysSkip*);

}  // namespace hps
