// Internal host-side declarations of the HPS library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.h"

namespace hps {

struct GllTables {
  int N;
  std::vector<double> xi, w, D, Kr;  // D and Kr row-major (N+1)^2
};
GllTables gll_tables(int N);

// ---- leaf kernels (leaf.hip) ------------------------------------------------
constexpr int kLeafMaxQ = 32;  // problems one leaf launch may touch
// Elements G in [G0, G0+count) of a group of problems with E elements each:
// problem q = G / E, element e = G % E (canonical numbering).  Per-problem
// inputs of problems q0 .. q0+kLeafMaxQ-1 travel in the kernel arguments.
struct LeafArgs {
  int nx, ny, ax, ay;  // mesh nx x ny = 2^ax x 2^ay elements (element e = ix + nx iy)
  int N, E, G0, count, q0;
  double h;
  const double* b_nodes[kLeafMaxQ];  // [E][(N+1)^2] per problem
  const double* s_nodes[kLeafMaxQ];  // complex [E][(N+1)^2] per problem, or null
  double kappa[kLeafMaxQ], eta[kLeafMaxQ];
  const double* D;            // (N+1)^2 row-major reference D
  const double* w;            // N+1
  const double* Kr;           // (N+1)^2 reference stiffness
  double* scratch;            // leaf_scratch_doubles(N, count) doubles, 16-byte aligned
  cd* T;                      // level-1 box maps, [q][E][4p][4p], merge-tree order within a problem
  cd* H;                      // [q][E][4p] canonical element order
  int* flag;                  // the problem's error words (common.h)
  int* fb_list;               // [1 + count]: count, then elements G whose interior
                              // block is nearly singular (recomputed by the fallback)
  int linear_out;             // 1: T of element G at T + G*(4p)^2 (no Morton placement)
};
// Leaf maps of elements G0 .. G0+count-1: the leaf kernel, then the complex
// fallback for the elements it lists.
hipError_t leaf_build(const LeafArgs& a, hipStream_t st);
// Field recovery (Sec. 3.1) for elements G in [0, count) of a group of
// problems (q = G / E): u [q][E][(N+1)^2] complex at all nodes from the
// skeleton solution g and boundary data t (canonical vectors per problem).
constexpr int kFieldMaxQ = 64;  // problems of one launch
struct FieldArgs {
  int nx, ny, N, E, count;
  double h;
  const double* b_nodes[kFieldMaxQ];
  const double* s_nodes[kFieldMaxQ];
  const cd* g[kFieldMaxQ];
  const cd* t[kFieldMaxQ];
  cd* u[kFieldMaxQ];
  double kappa[kFieldMaxQ], eta[kFieldMaxQ];
  const double* D;
  const double* w;
  const double* Kr;
  double xl[16], xr[16];       // corner extrapolation weights at xi = -1, +1
  double* scratch;             // field_scratch_doubles(N, blocks)
  int* flag;
};
size_t field_scratch_doubles(int N, int blocks);
hipError_t field_recover(const FieldArgs& a, int blocks, hipStream_t st);
// Clears a problem's device error words (no failure recorded).
hipError_t flag_reset(int* flag, hipStream_t st);
// Scratch doubles of one launch of `count` elements (the leaf kernel's
// bordered matrices, or the fallback's complex element systems).
size_t leaf_scratch_doubles(int N, int count);

// ---- batched complex GEMM and copies (gemm.hip) ---------------------------
// T is cd (complex FP64) or cf (complex FP32).
template <class T>
struct OperandT {
  const T* base;
  long long bstride;  // elements between consecutive batch entries
  int ld;
  IdxMap r, c;
};
typedef OperandT<cd> Operand;
typedef OperandT<cf> OperandF;
// Output tiles of a merge whose rows (or columns) all lie on physical sides of
// the merged box are never needed: the skeleton unknowns are interior
// impedances only.  Batch entry b writes merged box b % nbox of level g.level
// (of problem b / nbox of a group); a y index i (rows: i + row_off when row_y,
// columns: j + col_off when col_y) lands at box-local position ymap[i].
struct PhysSkip {
  int enabled;
  Geom g;
  int nbox;
  const int* ymap;
  int row_y, col_y;
  int row_off, col_off;
};

template <class T>
struct GemmArgsT {
  int M, N, K, batch;
  OperandT<T> A, B;
  T alpha, beta;
  OperandT<T> C;      // read only when beta != 0 (may alias D)
  T* D;
  long long Dstride;
  int ldd;
  IdxMap dr, dc;
  T diag_add;         // added to D(i, i) for i < min(M, N) when has_diag
  int has_diag;
  PhysSkip skip;
};
typedef GemmArgsT<cd> GemmArgs;
// D = alpha * A B + beta * C (+ diag_add I), all column-major; complex MFMA.
// The maps along K (A's columns, B's rows) must be offsets with an optional
// gap (im_off, im_gap), not tables: hipErrorInvalidValue otherwise.
template <class T>
hipError_t zgemm(const GemmArgsT<T>& a, hipStream_t st);
// Up to kGemmGroup independent GEMMs (none reads what another writes) in one
// launch, one tile shape for all of them; GEMMs with an empty M, N or batch
// are skipped.
constexpr int kGemmGroup = 4;
template <class T>
hipError_t zgemm_group(const GemmArgsT<T>* g, int n, hipStream_t st);
// D(dr(i), dc(j)) = alpha * S(sr(i), sc(j)) (S == null: zero), batched.
template <class T>
hipError_t zcopy2d(int M, int N, int batch, const OperandT<T>& S, T alpha, T* D,
                   long long Dstride, int ldd, IdxMap dr, IdxMap dc, hipStream_t st,
                   const PhysSkip* skip = nullptr);
// dst[i] = src[i] converted between complex FP64 and FP32
hipError_t convert_c64_c32(const cd* src, cf* dst, long long n, hipStream_t st);
hipError_t convert_c32_c64(const cf* src, cd* dst, long long n, hipStream_t st);
// true when y index `yi` of merged box (bx, by) lies on a physical side
__host__ __device__ inline bool y_physical(const PhysSkip& s, int bx, int by, int yi) {
  const int k = s.ymap[yi];
  return side_physical(s.g, bx, by, side_of(s.g, k));
}

// ---- batched complex inversion (inverse.hip) -------------------------------
// In-place inverse of `batch` m x m column-major matrices (stride `bstride`),
// Gauss-Jordan.  m <= 32 (and m <= 128 with `pivot`): partial pivoting, in
// registers.  Larger m, blocked in 32-column steps: with `pivot`, partial
// pivoting over all rows; without,
// no row interchanges across blocks (the diagonal blocks inverted as they
// stand) under a threshold test on the multipliers, whose failure records
// `level` in flag[6] (the caller then redoes the inverse with pivoting).
// scratch: see inverse_scratch_bytes.  A zero pivot of matrix b is recorded
// in the problem's error words as flag_where(level, b).
template <class T>
size_t inverse_scratch_bytes(int m, int batch);
template <class T>
hipError_t zinverse(T* A, int m, int lda, long long bstride, int batch, void* scratch,
                    int* flag, int level, bool pivot, hipStream_t st);

}  // namespace hps
