// Allocation-free push-forward for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc.  lag_pushforward_noalloc takes the problem description
// instead of a plan and runs the same kernels as lag_pushforward (eq.
// rhoEndOMT, deterministic binned scatter), with the binning scratch carved
// from one file-scope device array.  The loader gives every GPU the library
// runs on its own copy of that array, held until the process ends; its
// address on a device is resolved once, with that device current.

#include <mutex>

#include "lag_internal.hpp"

namespace lag {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // LAG_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == LAG_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`.  The array's name
// is a host-side stand-in in host code; only this address may reach kernels
// or copies.
int scratch_address(void** out) {
  int dev = 0;
  LAG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LAG_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    LAG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LAG_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LAG_OK;
}

// Lay the binning buffers for np particles out from `base` (256-byte
// aligned pieces); returns the bytes used.  With base == null only sizes.
size_t carve_bins(char* base, long long np, int dim, BinScratch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  const size_t n = (size_t)np;
  BinScratch s;
  s.base = (int*)take(sizeof(int) * n);
  s.vals = (float*)take(sizeof(float) * n * (size_t(1) << dim));
  s.count = (int*)take(sizeof(int) * (n + 1));
  s.start = (int*)take(sizeof(int) * (n + 1));
  s.cursor = (int*)take(sizeof(int) * n);
  s.items = (int*)take(sizeof(int) * n);
  s.scan = (int*)take(sizeof(int) * ((size_t)scan_blocks(np) + 2));
  if (b) *b = s;
  return off;
}

}  // namespace
}  // namespace lag

extern "C" {

int lag_pushforward_noalloc(const lag_problem* prob, const float* T, const float* phi, float* u, void* stream) {
  if (!(prob && T && phi && u)) return LAG_EINVAL;
  int rc = lag_problem_check(prob);
  if (rc) return rc;
  lag::Geo g;
  rc = lag::make_geo(prob, g);
  if (rc) return rc;
  if (lag::carve_bins(nullptr, g.np, g.dim, nullptr) > lag::kScratchBytes) return LAG_ETOOLARGE;
  void* base = nullptr;
  rc = lag::scratch_address(&base);
  if (rc) return rc;
  lag::BinScratch b;
  lag::carve_bins((char*)base, g.np, g.dim, &b);
  return lag::launch_pushforward_bins(g, b, T, phi, u, (hipStream_t)stream);
}

}  // extern "C"
