// Pivot selection helpers for the partial-pivoting factorisations: a 64-bit
// key that orders candidates by modulus and then by lowest row, and its
// maximum over a wavefront.
#pragma once
#include <hip/hip_runtime.h>

namespace hps {

// 1 + the FP32 bits of |v|^2 (monotonic for non-negative values; 0 means "no
// candidate") in the high word, the complemented row in the low word: an
// unsigned maximum picks the largest modulus and, among equal ones, the
// lowest row.
template <class R>
__device__ inline unsigned long long pivot_key(R v2, int r) {
  const unsigned hi = __float_as_uint((float)v2) + 1u;
  return ((unsigned long long)hi << 32) | (unsigned int)(0xFFFFFFFFu - (unsigned int)r);
}

__device__ inline int pivot_row(unsigned long long key) {
  return (int)(0xFFFFFFFFu - (unsigned int)(key & 0xFFFFFFFFull));
}

// Largest key of the wavefront (every lane must call): the maximum of the high
// words by DPP row shifts within each 16-lane row and read-lanes across rows;
// among the lanes holding that maximum, the lowest lane's key.
__device__ inline unsigned long long wave_max_key(unsigned long long key) {
  const unsigned hi = (unsigned)(key >> 32);
  unsigned h = hi;
  h = max(h, (unsigned)__builtin_amdgcn_update_dpp((int)h, (int)h, 0x111, 0xF, 0xF, false));
  h = max(h, (unsigned)__builtin_amdgcn_update_dpp((int)h, (int)h, 0x112, 0xF, 0xF, false));
  h = max(h, (unsigned)__builtin_amdgcn_update_dpp((int)h, (int)h, 0x114, 0xF, 0xF, false));
  h = max(h, (unsigned)__builtin_amdgcn_update_dpp((int)h, (int)h, 0x118, 0xF, 0xF, false));
  const unsigned m = max(max((unsigned)__builtin_amdgcn_readlane((int)h, 15), (unsigned)__builtin_amdgcn_readlane((int)h, 31)),
                         max((unsigned)__builtin_amdgcn_readlane((int)h, 47), (unsigned)__builtin_amdgcn_readlane((int)h, 63)));
  const unsigned long long bal = __ballot(hi == m);
  const int l = __ffsll((long long)bal) - 1;
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)key, l);
  return ((unsigned long long)m << 32) | lo;
}

}  // namespace hps
