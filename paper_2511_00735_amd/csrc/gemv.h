// Internal declarations of the V-cycle streaming kernels (gemv.hip).
#pragma once
#include "host.h"

namespace hps {

constexpr int kGemvMaxDesc = 4;          // GEMVs fused into one launch
constexpr int kGemvKChunkMax = 2048;     // K entries staged in LDS per split
constexpr int kGemvTargetBlocks = 1024;  // split-K aims at this many workgroups

// Source of a GEMV's x vector for batch entry (pair) b: a compact array
// p[b*stride + k], the canonical vector gathered through a slot table,
// vec[tab[b*tstride + k]] (negative slot: 0), or the sum in split order of
// another GEMV's split-K partials, sum_s ps[(s*pbatch + b)*pM + proff + k]
// (s < pns), which the workgroups of row tile 0 also store at
// save[b*save_stride + save_off + k].
struct VecIn {
  const cd* p;
  long long stride;
  const cd* vec;
  const int* tab;
  long long tstride;
  const cd* ps;
  int pns, pbatch, pM, proff;
  cd* save;
  long long save_stride;
  int save_off;
};

// Destination of y = alpha A x (+ beta y0): a compact array and/or a scatter into
// the canonical vector through a slot table (assign or add; negative slots
// skipped).
struct VecOut {
  cd* p;
  long long stride;
  const cd* y0;
  long long y0stride;
  cd beta;
  cd* vec;
  const int* tab;
  long long tstride;
  int add;
};

// The matrix may be stored in complex FP64 (M = cd) or FP32 (M = cf); x, y and
// the accumulation are always FP64.  Its column map must be an offset with an
// optional gap, not a table (hipErrorInvalidValue otherwise).
template <class M>
struct GemvDescT {
  int M_, K;
  OperandT<M> A;
  cd alpha;
  VecIn x;
  VecOut y;
};
typedef GemvDescT<cd> GemvDesc;

template <class M>
struct GemvBatchT {
  GemvDescT<M> d[kGemvMaxDesc];
  int nsplit[kGemvMaxDesc];
  long long poff[kGemvMaxDesc];   // partial-sum offsets
  int batch;
  int partials_only;              // every split writes partial sums; no epilogue
};

int gemv_nsplit(int M, int K, int batch);
// nd GEMVs of the same batch size in one launch, plus one reduction launch when
// any of them is split along K (partial sums: at most gemv_nsplit * batch * M each).
template <class M>
hipError_t zgemv_batched(const GemvDescT<M>* d, int nd, int batch, cd* partial, hipStream_t st);
// Partial sums only: descriptor i writes A x (alpha, y0 and y ignored) split
// along K into partial[poff[i] + (s * batch + b) * M + r], s < nsplit[i], for
// a consumer that sums them in split order.  One launch.  max_split > 0 caps
// the split count (a single-workgroup consumer reads fewer partials).
struct GemvPartLayout {
  long long poff[kGemvMaxDesc];
  int nsplit[kGemvMaxDesc];
};
template <class M>
hipError_t zgemv_partials(const GemvDescT<M>* d, int nd, int batch, cd* partial, GemvPartLayout* lay,
                          hipStream_t st, int max_split = 0);

// One V-cycle level of small pairs in one launch per direction: the down sweep
// with two workgroups per pair (one per half of z0), the up sweep with the
// pair's 2m rows split into pieces, one workgroup each.  Per pair j (children P = box 2j, Q = box 2j+1 of level g.level):
//   Ainv  [2m][2m]  inverse of A = [[I, -T^P_aa], [-T^Q_bb, I]] on x = [Q.beta; P.alpha]
//   X     [2m][2e]  A^-1 B, columns y = [P.E1; Q.E2]
//   xtab  [2m]      canonical slots of x;  ytab [2e] slots of y (-1: physical);
//   dtab  [2e]      slots across the face of y (-1: physical)
//   Z0    [2m]      the down sweep's A^-1 r_x, kept for the up sweep.
template <class M>
struct SmallLevelT {
  Geom g;
  int m, e, a0, b0;
  IdxMap E1, E2;
  const M* T;
  const M* Ainv;
  const M* X;
  const int* xtab;
  const int* ytab;
  const int* dtab;
  cd* Z0;
};
// Levels the down-sweep kernel takes (at least 32 pairs, 2m and 2e at most
// 1024), and those the up-sweep kernel takes (any whose row piece and 2e
// values fit its LDS).
bool vc_small_ok(int m, int e, int pairs);
bool vc_up_small_ok(int m, int e, int pairs);
template <class M>
hipError_t vc_down_small(const SmallLevelT<M>& a, int pairs, cd* vec, hipStream_t st);
template <class M>
hipError_t vc_up_small(const SmallLevelT<M>& a, int pairs, cd* z, hipStream_t st);

// Levels 1..K (2 <= K <= kFuseMax) of the V-cycle in one launch, one
// workgroup of 1024 threads per level-(K+1) box (`boxes` of them, problem after
// problem), the box's slot values held in LDS.  Level l's pairs of box B are
// B 2^(K-l) .. (B+1) 2^(K-l) - 1.  Tables hold local slot indices (positions
// in the box's LDS vector); gdown/gup map each local index of box B to its
// canonical slot (the down sweep's set: the box's non-boundary slots and the
// slots across its boundary, -1 unused; the up sweep's: all slots of the
// box's elements).  The operators are those of the per-level kernels.
constexpr int kFuseMax = 4;
struct FusedLevel {
  int m, e, a0, b0, b;
  IdxMap E1, E2;
  const void* T;      // level-l box maps (storage type of the launch)
  const void* Ainv;
  const void* X;
  const int* xl;      // [pairs][2m] local indices of x
  const int* dl;      // [pairs][2e] local indices across y (-1: physical)
  const int* yl;      // [pairs][2e] local indices of y (-1: physical)
  cd* Z0;
};
struct FusedArgs {
  int nloc, nloc_pad;
  const int* gdown;   // [boxes][nloc]
  const int* gup;     // [boxes][nloc]
  FusedLevel lev[kFuseMax];
};
size_t fused_lds_bytes(const FusedArgs& a, int K, bool down);
bool fused_ok(const FusedArgs& a, int K);
template <class M>
hipError_t vc_fused(const FusedArgs& a, int K, int boxes, cd* vec, bool down, hipStream_t st);

}  // namespace hps
