// Leaf ItI maps with no device allocation: the variant of hps_build_leaves for
// callers that cannot allocate (code under HIP graph capture, serving loops or
// harnesses that forbid hipMalloc).  Everything the leaf kernels need beyond
// the caller's inputs and outputs -- the error words, the fallback's element
// list, the GLL tables and the per-element scratch (bordered matrices, or the
// fallback's complex element systems) -- lives in one file-scope device array
// per GPU, resolved once per device with hipGetSymbolAddress.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hps.h"
#include "host.h"

namespace hps {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU, held until the process ends
constexpr int kMaxList = 4096;                       // largest element list carved below
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

inline size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets inside the array: error words, fallback list, GLL tables, then
// the leaf scratch.
struct Carve {
  size_t flag, list, tables, leaf, leaf_bytes;
};

Carve carve(int N) {
  Carve c;
  const int N1 = N + 1;
  c.flag = 0;
  c.list = up256(sizeof(int) * kFlagWords);
  c.tables = c.list + up256(sizeof(int) * (1 + (size_t)kMaxList));
  c.leaf = c.tables + up256(sizeof(double) * (2 * (size_t)N1 * N1 + N1));
  c.leaf_bytes = kScratchBytes - c.leaf;
  return c;
}

// Largest element count of one call at order N.
int max_count(int N) {
  const Carve c = carve(N);
  int lo = 0;
  for (int k = 1; k <= kMaxList; ++k)
    if (sizeof(double) * leaf_scratch_doubles(N, k) <= c.leaf_bytes) lo = k;
  return lo;
}

}  // namespace
}  // namespace hps

using namespace hps;

// context helpers (api.cpp)
void hps_ctx_set_error(hps_ctx* ctx, const char* msg);
void* hps_ctx_stream(hps_ctx* ctx);

extern "C" hps_status hps_leaf_maps_noalloc(hps_ctx* ctx, int32_t order, double h, double kappa, double eta,
                                            int32_t count, const double* b_nodes, const double* s_nodes,
                                            double* T, double* H) {
  if (!ctx) return HPS_ERR_ARG;
  auto fail = [&](hps_status s, const std::string& m) {
    hps_ctx_set_error(ctx, m.c_str());
    return s;
  };
  if (order < 2 || order > 16) return fail(HPS_ERR_ARG, "order N must be in [2, 16]");
  if (!(std::isfinite(h) && h > 0) || !(std::isfinite(kappa) && kappa > 0) || !(std::isfinite(eta) && eta > 0))
    return fail(HPS_ERR_ARG, "h, kappa and eta must be finite and > 0");
  if (!b_nodes || !T || !H) return fail(HPS_ERR_ARG, "null b_nodes, T or H");
  const int cap = max_count(order);
  if (count < 1 || count > cap)
    return fail(HPS_ERR_ARG, "count must be in [1, " + std::to_string(cap) + "] at order " + std::to_string(order) +
                                 " (the 64 MiB static scratch)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HPS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HPS_ERR_ARG, "device index out of range");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(HPS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    base = static_cast<char*>(g_ptr[dev]);
  }
  hipStream_t st = static_cast<hipStream_t>(hps_ctx_stream(ctx));
  const Carve c = carve(order);
  const int N1 = order + 1;
  // GLL tables into the array; the host copy stays alive until the
  // synchronisation below
  const GllTables t = gll_tables(order);
  std::vector<double> tab;
  tab.insert(tab.end(), t.D.begin(), t.D.end());
  tab.insert(tab.end(), t.w.begin(), t.w.end());
  tab.insert(tab.end(), t.Kr.begin(), t.Kr.end());
  e = hipMemcpyAsync(base + c.tables, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(HPS_ERR_HIP, std::string("upload: ") + hipGetErrorString(e));
  int* flag = reinterpret_cast<int*>(base + c.flag);
  LeafArgs a{};
  a.nx = count;   // elements in call order (the output is linear, so no tree order)
  a.ny = 1;
  a.N = order;
  a.E = count;
  a.G0 = 0;
  a.count = count;
  a.q0 = 0;
  a.h = h;
  a.b_nodes[0] = b_nodes;
  a.s_nodes[0] = s_nodes;
  a.kappa[0] = kappa;
  a.eta[0] = eta;
  const double* tb = reinterpret_cast<const double*>(base + c.tables);
  a.D = tb;
  a.w = tb + N1 * N1;
  a.Kr = tb + N1 * N1 + N1;
  a.scratch = reinterpret_cast<double*>(base + c.leaf);
  a.T = reinterpret_cast<cd*>(T);
  a.H = reinterpret_cast<cd*>(H);
  a.flag = flag;
  a.fb_list = reinterpret_cast<int*>(base + c.list);
  a.linear_out = 1;
  // the array keeps the previous call's contents: the error words start clear
  // (the element list is reset inside leaf_build)
  if ((e = flag_reset(flag, st)) != hipSuccess || (e = leaf_build(a, st)) != hipSuccess) {
    (void)hipStreamSynchronize(st);   // the table upload reads `tab`
    return fail(HPS_ERR_HIP, std::string("leaf launch: ") + hipGetErrorString(e));
  }
  int f[kFlagWords];
  e = hipMemcpyAsync(f, flag, sizeof(f), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HPS_ERR_HIP, std::string("leaf build: ") + hipGetErrorString(e));
  unsigned long long w2, w4;
  std::memcpy(&w2, f + 2, sizeof(w2));
  std::memcpy(&w4, f + 4, sizeof(w4));
  if (f[0] & kFlagNonFinite)
    return fail(HPS_ERR_ARG, "non-finite value in b_nodes or s_nodes of element " + std::to_string(w4));
  if (f[0] & kFlagSingular)
    return fail(HPS_ERR_SINGULAR, "zero pivot in the leaf map of element " +
                                      std::to_string(w2 & ((1ull << 40) - 1)));
  return HPS_OK;
}
