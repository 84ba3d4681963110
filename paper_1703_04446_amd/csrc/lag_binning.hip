// Deterministic particle-to-grid scatter for the continuity model.
//
// The push-forward u1 = F(y) T (eq. rhoEndOMT, hat width = cell size) and the
// continuity Jacobian product both split a per-particle quantity over the
// 2^d cells around the particle's end point.  Float atomics would make the
// result depend on scheduling, so the scatter is done in gather form:
//   1. every particle records its base cell (corner 0 of the cell containing
//      its end point) and its 2^d corner values; cells count their particles;
//   2. an exclusive scan of the counts gives each cell's bin;
//   3. particles are placed into bins and each bin is sorted by particle id;
//   4. every output cell c sums, for corner o = 0 .. 2^d - 1 in order, the
//      o-th values of the particles in bin(c - o), in ascending particle id.
// The summation order is therefore fixed and the result bit-reproducible.

#include "lag_internal.hpp"

namespace lag {

constexpr int kScanPer = 4;                       // elements per thread
constexpr int kScanTile = kBlock * kScanPer;      // elements per block

__global__ void __launch_bounds__(kBlock) k_zero_i(int* __restrict__ x, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

int launch_zero_i(int* x, long long n, hipStream_t s) {
  if (n <= 0) return LAG_OK;
  hipLaunchKernelGGL(k_zero_i, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, n);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// block-level exclusive scan of `in` (n entries) into `out`; block totals
__global__ void __launch_bounds__(kBlock) k_scan_local(const int* __restrict__ in, int* __restrict__ out,
                                                        int* __restrict__ bsum, long long n) {
  __shared__ int sh[kBlock];
  long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
  int v[kScanPer];
  int t = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    t += v[k];
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  // Hillis-Steele inclusive scan of the thread totals
  for (int off = 1; off < kBlock; off <<= 1) {
    int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - t;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = sh[kBlock - 1];
}

// single block: exclusive scan of the block totals, in place; total at [nb]
__global__ void __launch_bounds__(kBlock) k_scan_blocks(int* __restrict__ bsum, int nb) {
  __shared__ int sh[kBlock];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int start = 0; start < nb; start += kBlock) {
    int i = start + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += x;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry += sh[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_add(int* __restrict__ out, const int* __restrict__ bsum,
                                                      long long n, int nb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / kScanTile];
  if (i == n) out[n] = bsum[nb];
}

__global__ void __launch_bounds__(kBlock) k_bin_fill(const int* __restrict__ base, const int* __restrict__ start,
                                                      int* __restrict__ cursor, int* __restrict__ items, long long n) {
  long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int b = base[j];
  int slot = start[b] + atomicAdd(&cursor[b], 1);
  items[slot] = (int)j;
}

// order every bin by particle id (bins hold a handful of entries)
__global__ void __launch_bounds__(kBlock) k_bin_sort(const int* __restrict__ start, int* __restrict__ items,
                                                      long long n) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int a = start[c], e = start[c + 1];
  for (int i = a + 1; i < e; ++i) {
    int key = items[i];
    int k = i - 1;
    while (k >= a && items[k] > key) {
      items[k + 1] = items[k];
      --k;
    }
    items[k + 1] = key;
  }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_bin_gather(Geo g, const int* __restrict__ start,
                                                        const int* __restrict__ items,
                                                        const float* __restrict__ vals, float* __restrict__ out) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.np) return;
  int ci[3] = {0, 0, 0};
  long long r = c;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    ci[a] = (int)(r % g.mi[a]);
    r /= g.mi[a];
  }
  float acc = 0.f;
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
    long long b = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      int x = ci[a] - ((o >> a) & 1);
      if (x < 0) x += g.mi[a];
      b += (long long)x * stride;
      stride *= g.mi[a];
    }
    int e = start[b + 1];
    for (int k = start[b]; k < e; ++k) acc += vals[(long long)o * g.np + items[k]];
  }
  out[c] = acc;
}

int bin_and_gather(const Geo& g, const BinScratch& b, float* out, hipStream_t s) {
  const long long n = g.np;
  const int nb = (int)((n + kScanTile - 1) / kScanTile);
  const unsigned g1 = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kBlock), 0, s, b.count, b.start, b.scan, n);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, s, b.scan, nb);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b.start,
                     b.scan, n, nb);
  LAG_LAUNCH_CHECK();
  int rc = launch_zero_i(b.cursor, n, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bin_fill, dim3(g1), dim3(kBlock), 0, s, b.base, b.start, b.cursor, b.items, n);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_sort, dim3(g1), dim3(kBlock), 0, s, b.start, b.items, n);
  LAG_LAUNCH_CHECK();
  if (g.dim == 3)
    hipLaunchKernelGGL(k_bin_gather<3>, dim3(g1), dim3(kBlock), 0, s, g, b.start, b.items, b.vals, out);
  else
    hipLaunchKernelGGL(k_bin_gather<2>, dim3(g1), dim3(kBlock), 0, s, g, b.start, b.items, b.vals, out);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

}  // namespace lag
