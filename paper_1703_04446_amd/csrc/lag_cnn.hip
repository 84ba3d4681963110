// 3-D U-Net for the learned Gauss-Newton warm start (gfx950).
//
// Network (channels c0..c3, cubic grid of side S, a multiple of 32):
//   enc0 = relu(conv(relu(conv(x, 2 -> c0)), c0 -> c0))           S
//   enc1 = relu(conv(relu(conv(pool(enc0), c0 -> c1)), c1 -> c1))  S/2
//   enc2 = relu(conv(relu(conv(pool(enc1), c1 -> c2)), c2 -> c2))  S/4
//   mid  = relu(conv(relu(conv(pool(enc2), c2 -> c3)), c3 -> c3))  S/8
//   dec2 = relu(conv([up(mid), enc2], c3 + c2 -> c2))              S/4
//   dec1 = relu(conv([up(dec2), enc1], c2 + c1 -> c1))             S/2
//   dec0 = relu(conv([up(dec1), enc0], c1 + c0 -> c0))             S
//   out  = scale * (dec0 @ Wh + bh)                                 (1x1 head)
// Convolutions are 3x3x3 with periodic padding.  Activations are channel-
// last bfloat16 (a convolution input row of 16 channels is one 32-byte
// segment), gradients float32, master weights float32 with bfloat16 copies
// for the matrix cores.  No pre-activation is kept: the relu backward masks
// with the stored bfloat16 activation, which is non-zero exactly where the
// pre-activation is positive (down to 2^-133).
//
// Every 3x3x3 convolution is an implicit GEMM on the double-K MFMA
// (v_mfma_f32_16x16x32_bf16: A[i][k] in lane i + 16 (k / 8), element k % 8;
// B[k][n] in lane n + 16 (k / 8), element k % 8; C[m][n] in lane n + 16
// (m / 4), element m % 4), with the halo tile and the weights staged in LDS:
//   forward      out[v][co]  = sum_{t,ci} x[v+o_t][ci] W[t][ci][co]     (M=v,  N=co, K=t,ci)
//   backward-in  gx[v][ci]   = sum_{t,co} g[v-o_t][co] W[t][ci][co]     (M=v,  N=ci, K=t,co)
//   backward-W   gW[t][ci][co] = sum_v x[v+o_t][ci] g[v][co]            (M=ci, N=co, K=v)
// Every gradient reduction (weights, biases, head) sums in a fixed order,
// so a training step gives the same bits in every run.
// Concatenation is never materialised by a copy: producers write into
// channel slices of the concatenated buffer ("views": base, channel stride,
// channel offset).

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <random>
#include <vector>

#include <type_traits>

#include "lag_internal.hpp"

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) short i16x4;

namespace lag {
namespace cnn {

constexpr int kLayers = 12;
enum { E0A, E0B, E1A, E1B, E2A, E2B, MA, MB, D2, D1, D0, HEAD };

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even on the 16 high bits (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ int nbr(int v, int s, int dz, int dy, int dx) {
  int x = v % s, y = (v / s) % s, z = v / (s * s);
  x += dx; y += dy; z += dz;
  x = x < 0 ? x + s : (x >= s ? x - s : x);
  y = y < 0 ? y + s : (y >= s ? y - s : y);
  z = z < 0 ? z + s : (z >= s ? z - s : z);
  return (z * s + y) * s + x;
}

// ---------------------------------------------------------------------------
// Convolutions on gfx950's double-K matrix cores, v_mfma_f32_16x16x32_bf16:
// A 16 x 32 with A[i][k] in lane i + 16 (k / 8), element k % 8; B 32 x 16
// with B[k][n] in lane n + 16 (k / 8), element k % 8; C 16 x 16 with C[m][n]
// in lane n + 16 (m / 4), element m % 4.
//
// A block computes an output tile of TX x TY x TZ voxels (x fastest; 8 x 8 x
// 4 on grids of side >= 8, 4 x 4 x 4 on a side of 4), 64 voxels per wave
// (four 16-voxel row tiles), for 16 NT channels.  The contraction runs over
// (tap, channel) in chunks of 16 channels: the chunk's input tile with a
// one-voxel periodic halo, (TX+2)(TY+2)(TZ+2) rows of 16 bf16 (rows padded
// to 24 for the banks), is staged in LDS, and the 27 x 16 = 432 products of
// the chunk take 14 MFMA steps of K = 32: step q, lane group g covers tap
// 2q + g/2 and channels 8 (g % 2) .. +8 (the last half step is tap 27,
// whose weights are zero).  The chunk's weights for the block's 16 NT
// output channels, [28 taps][16 NT][16], are staged in LDS beside the input
// tile (a weight load per K step from L2 would stall every step on its
// latency); the A operand of a row tile and the B operand of a column tile
// are then one 16-byte LDS read per lane each.
//   forward      out[v][co] = sum_{t,ci} x[v + o_t][ci] W[t][ci][co]
//   backward-in  gx[v][ci]  = sum_{t,co} g[v - o_t][co] W[t][ci][co]
// (the backward reads the halo at the mirrored tap and the transposed weights).

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

constexpr int kTaps = 28;      // 27 taps and a zero tap that pads the last K step
constexpr int kRow = 24;       // LDS row of a staged voxel: 16 channels + 8 padding (bf16)

struct ConvTile {
  int lx, ly, lz;              // log2 of the tile extents
};

__host__ __device__ inline ConvTile conv_tile(int s) {
  ConvTile t;
  if (s % 8 == 0) {
    t.lx = 3; t.ly = 3; t.lz = 2;
  } else {
    t.lx = 2; t.ly = 2; t.lz = 2;   // sides that are multiples of 4 only
  }
  return t;
}

// halo offset of tap t (t = 27: offset 0, any valid row)
__device__ __forceinline__ int tap_off(int t, int hx, int hy) {
  if (t >= 27) return 0;
  const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
  return (dz * hy + dy) * hx + dx;
}

// Split over the contraction (small grids, few blocks): blockIdx.z takes
// chunks z, z + gridDim.z, ... and, with gridDim.z > 1, writes its raw sums
// to kpart[z][v][out_cs] for k_conv_finish.
template <bool BWD, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 3))) k_conv_mfma(const unsigned short* __restrict__ in, int in_cs, int in_co,
                                                   int kch, int s, ConvTile T,
                                                   const unsigned short* __restrict__ w, int wn, int wk,
                                                   const float* __restrict__ bias, float* __restrict__ out,
                                                   int out_cs, unsigned short* __restrict__ act, int act_cs,
                                                   int act_co, float* __restrict__ kpart) {
  extern __shared__ uint4 smem[];
  unsigned short* wt = reinterpret_cast<unsigned short*>(smem);         // [kTaps][16 NT][16]
  unsigned short* tile = wt + kTaps * 16 * NT * 16;                     // [H][kRow]
  const int TX = 1 << T.lx, TY = 1 << T.ly, TZ = 1 << T.lz;
  const int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, H = HX * HY * HZ;
  const int ntx = s >> T.lx, nty = s >> T.ly;
  const int b = blockIdx.x;
  const int x0 = (b % ntx) << T.lx, y0 = ((b / ntx) % nty) << T.ly, z0 = (b / (ntx * nty)) << T.lz;
  const int n_base = blockIdx.y * 16 * NT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, grp = lane >> 4;
  // halo row of this lane's voxel in row tile i (tap offset added per step)
  int hb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int u = 64 * wave + 16 * i + m;
    const int x = u & (TX - 1), y = (u >> T.lx) & (TY - 1), z = u >> (T.lx + T.ly);
    hb[i] = (z * HY + y) * HX + x;
  }
  f32x4 acc[4][NT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ci0 = 8 * (grp & 1);
  const int kz = gridDim.z;
  for (int c = 16 * blockIdx.z; c < kch; c += 16 * kz) {
    __syncthreads();   // the previous chunk's reads are done
    // halo and weights, four rows per thread and pass: the four loads go
    // out before the stores (a plain strided loop waits on one global trip
    // per row); past the end a thread loads and stores the last row again,
    // the same value that row's own thread writes
    for (int q0 = threadIdx.x; q0 < 2 * H; q0 += 4 * blockDim.x) {
      uint4 val[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = min(q0 + k * (int)blockDim.x, 2 * H - 1);
        const int r = q >> 1, half = q & 1;
        const int hx = r % HX, hy = (r / HX) % HY, hz = r / (HX * HY);
        int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
        gx = gx < 0 ? gx + s : (gx >= s ? gx - s : gx);
        gy = gy < 0 ? gy + s : (gy >= s ? gy - s : gy);
        gz = gz < 0 ? gz + s : (gz >= s ? gz - s : gz);
        const long long v = ((long long)gz * s + gy) * s + gx;
        val[k] = *reinterpret_cast<const uint4*>(in + v * in_cs + in_co + c + 8 * half);
      }
      __builtin_amdgcn_sched_barrier(0);   // else each load is sunk to its store and waited for alone
#pragma unroll
      for (int k = 0; k < 4; ++k) {   // unconditional: a row past the end stores the last row's value again
        const int q = min(q0 + k * (int)blockDim.x, 2 * H - 1);
        *reinterpret_cast<uint4*>(tile + (q >> 1) * kRow + 8 * (q & 1)) = val[k];
      }
    }
    for (int q0 = threadIdx.x; q0 < kTaps * 16 * NT * 2; q0 += 4 * blockDim.x) {
      uint4 val[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = min(q0 + k * (int)blockDim.x, kTaps * 16 * NT * 2 - 1);
        const int row = q >> 1, half = q & 1;   // row = t * 16 NT + n
        const int t = row / (16 * NT), n = row - t * 16 * NT;
        val[k] = *reinterpret_cast<const uint4*>(w + ((long long)t * wn + n_base + n) * wk + c + 8 * half);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = min(q0 + k * (int)blockDim.x, kTaps * 16 * NT * 2 - 1);
        *reinterpret_cast<uint4*>(wt + (q >> 1) * 16 + 8 * (q & 1)) = val[k];
      }
    }
    __syncthreads();
    // operands of K step q + 1 are read from LDS while step q's MFMAs run
    bf16x8 bv[2][NT], av[2][4];
    auto load_step = [&](int q, bf16x8* b, bf16x8* a) {
      const int t = 2 * q + (grp >> 1);
      const int off = tap_off(BWD ? (t >= 27 ? 27 : 26 - t) : t, HX, HY);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(wt + ((t * 16 * NT) + 16 * nt + m) * 16 + ci0));
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = as_bf16x8(*reinterpret_cast<const uint4*>(tile + (hb[i] + off) * kRow + ci0));
    };
    load_step(0, bv[0], av[0]);
#pragma unroll
    for (int q = 0; q < 14; ++q) {
      const int cur = q & 1;
      if (q + 1 < 14) load_step(q + 1, bv[cur ^ 1], av[cur ^ 1]);
      // left to itself the scheduler sinks each read to its MFMA and waits
      // for it alone (one LDS trip per MFMA)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[cur][i], bv[cur][nt], acc[i][nt], 0, 0, 0);
    }
  }
  // Epilogue: the case is decided once per thread (a branch per output
  // made the compiler wait for every earlier store before the next one).
  // MODE 0: raw split sums to kpart; 1: backward gx to out; 2: forward
  // bias -> relu -> bf16 act, 3: and the pre-activation to out.
  auto epilogue = [&](auto mode_c) {
    constexpr int MODE = decltype(mode_c)::value;
    float bn[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bn[nt] = MODE >= 2 ? bias[n_base + 16 * nt + m] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 64 * wave + 16 * i + 4 * grp + j;
        const int x = x0 + (u & (TX - 1)), y = y0 + ((u >> T.lx) & (TY - 1)), z = z0 + (u >> (T.lx + T.ly));
        const long long v = ((long long)z * s + y) * s + x;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int n = n_base + 16 * nt + m;
          if constexpr (MODE == 0) {
            kpart[((long long)blockIdx.z * s * s * s + v) * out_cs + n] = acc[i][nt][j];
          } else if constexpr (MODE == 1) {
            out[v * out_cs + n] = acc[i][nt][j];
          } else {
            const float val = acc[i][nt][j] + bn[nt];
            if constexpr (MODE == 3) out[v * out_cs + n] = val;
            act[v * act_cs + act_co + n] = f2bf(fmaxf(val, 0.f));
          }
        }
      }
  };
  if (kz > 1) epilogue(std::integral_constant<int, 0>{});
  else if constexpr (BWD) epilogue(std::integral_constant<int, 1>{});
  else if (out) epilogue(std::integral_constant<int, 3>{});
  else epilogue(std::integral_constant<int, 2>{});
}

constexpr int kMaxSplit = 8;   // contraction splits (conv_split: at most 128 input channels / 16)

// Sum of the split contraction in order of z, then the epilogue: forward
// (bias) -> bf16 relu activation (and the pre-activation if out != null);
// backward -> gx.
template <bool BWD, int KZ>
__global__ void k_conv_finish(const float* __restrict__ kpart, long long V, int nch,
                              const float* __restrict__ bias, float* __restrict__ out, unsigned short* __restrict__ act,
                              int act_cs, int act_co) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * nch) return;
  // the KZ parts, all loaded before the sum
  float p[KZ];
#pragma unroll
  for (int z = 0; z < KZ; ++z) p[z] = kpart[z * V * nch + i];
  float sum = 0.f;
#pragma unroll
  for (int z = 0; z < KZ; ++z) sum += p[z];
  if constexpr (BWD) {
    out[i] = sum;
  } else {
    // forward: nch is a layer's output width, 16, 32 or 64 (a power of
    // two: no 64-bit division); i < 2^31
    const int n = (int)((unsigned)i & (unsigned)(nch - 1));
    const long long v = (long long)((unsigned)i >> (__ffs(nch) - 1));
    const float val = sum + bias[n];
    if (out) out[i] = val;
    act[v * act_cs + act_co + n] = f2bf(fmaxf(val, 0.f));
  }
}

// Weight gradient, one block per (voxel range r, 16-channel input slice):
//   part[r][t][ci][co] = sum over the range's tiles of x[v + o_t][ci] g[v][co]
// with M = ci, N = co, K = voxels: the tile's gradient is staged transposed,
// gT[co][u] (u = tile voxel, x fastest), and its input slice with the halo
// transposed, xT[ci][hz][hy][16] (rows of 16 bf16, HX <= 10 used), so that
// 8 voxels consecutive in x are one 16-byte read; the three taps of a tap
// row (dz, dy) share two aligned reads, from which byte alignment takes the
// x shifts dx = 0, 1, 2.  Wave w owns the tap rows w, w + 4, w + 8; a K
// step reads its B operands once for all of them and covers 4 rows of 8 x
// (tile side 8) or 8 rows of 4 x (side 4, element reads).  Fixed-order sum
// over r later.
// Four rows of 8 bf16 (r[k] = row k) written transposed: dst[e * stride + k]
// = r[k][e] for e < 8, as eight 8-byte stores.
__device__ __forceinline__ void transpose_4x8(const uint4 r[4], unsigned short* dst, int stride) {
  const unsigned int* w0 = reinterpret_cast<const unsigned int*>(&r[0]);
  const unsigned int* w1 = reinterpret_cast<const unsigned int*>(&r[1]);
  const unsigned int* w2 = reinterpret_cast<const unsigned int*>(&r[2]);
  const unsigned int* w3 = reinterpret_cast<const unsigned int*>(&r[3]);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    // elements 2d (low halves) and 2d + 1 (high halves) of the four rows
    const unsigned int lo01 = (w0[d] & 0xffffu) | (w1[d] << 16), lo23 = (w2[d] & 0xffffu) | (w3[d] << 16);
    const unsigned int hi01 = (w0[d] >> 16) | (w1[d] & 0xffff0000u), hi23 = (w2[d] >> 16) | (w3[d] & 0xffff0000u);
    *reinterpret_cast<uint2*>(dst + (2 * d) * stride) = make_uint2(lo01, lo23);
    *reinterpret_cast<uint2*>(dst + (2 * d + 1) * stride) = make_uint2(hi01, hi23);
  }
}

template <int NT>
__global__ void __launch_bounds__(256) k_conv_wgrad(const unsigned short* __restrict__ in, int in_cs, int in_co,
                                                    int s, ConvTile T, const unsigned short* __restrict__ g, int cout,
                                                    int tiles_per_range, int cin_pad, float* __restrict__ part) {
  extern __shared__ uint4 smem[];
  const int TX = 1 << T.lx, TY = 1 << T.ly, TZ = 1 << T.lz;
  const int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  const int NV = TX * TY * TZ;
  unsigned short* gT = reinterpret_cast<unsigned short*>(smem);                 // [cout][NV]
  unsigned short* xT = gT + (size_t)cout * NV;                                   // [16][HZ][HY][16]
  const int ntx = s >> T.lx, nty = s >> T.ly, ntiles = ntx * nty * (s >> T.lz);
  const int r = blockIdx.x, cs = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, grp = lane >> 4;
  constexpr int kMaxRows = 3;   // tap rows (dz, dy) per wave: w, w + 4, w + 8 (< 9)
  f32x4 acc[kMaxRows][3][NT];
#pragma unroll
  for (int k = 0; k < kMaxRows; ++k)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[k][dx][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int tb = r * tiles_per_range, te = min(ntiles, tb + tiles_per_range);
  for (int b = tb; b < te; ++b) {
    const int x0 = (b % ntx) << T.lx, y0 = ((b / ntx) % nty) << T.ly, z0 = (b / (ntx * nty)) << T.lz;
    __syncthreads();
    // gT: runs of 4 voxels (consecutive in x) x 8 channels per thread,
    // transposed in registers and written as 8-byte runs of gT[co][u]
    for (int q = threadIdx.x; q < (NV / 4) * (cout / 8); q += blockDim.x) {
      const int u4 = q % (NV / 4), c8 = q / (NV / 4);
      const int u = 4 * u4;
      const int x = x0 + (u & (TX - 1)), y = y0 + ((u >> T.lx) & (TY - 1)), z = z0 + (u >> (T.lx + T.ly));
      const long long v = ((long long)z * s + y) * s + x;
      uint4 r4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) r4[k] = *reinterpret_cast<const uint4*>(g + (v + k) * cout + 8 * c8);
      transpose_4x8(r4, gT + (8 * c8) * NV + u, NV);
    }
    // xT: the 16-channel slice with the halo, runs of 4 halo voxels along x
    // (rows of 16; positions HX .. 15 hold copies, never read)
    const int nrun = (HX + 3) >> 2;   // runs of 4 covering the HX halo positions of a row
    for (int q = threadIdx.x; q < 2 * nrun * HY * HZ; q += blockDim.x) {
      const int half = q & 1, xr = (q >> 1) % nrun, rr = (q >> 1) / nrun;   // rr = hz * HY + hy
      const int hy = rr % HY, hz = rr / HY;
      int gy = y0 + hy - 1, gz = z0 + hz - 1;
      gy = gy < 0 ? gy + s : (gy >= s ? gy - s : gy);
      gz = gz < 0 ? gz + s : (gz >= s ? gz - s : gz);
      const long long vrow = ((long long)gz * s + gy) * s;
      uint4 r4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // positions HX .. 15 of the row are never read: load the last halo
        // voxel there, so that gx stays within one period of the grid
        int gx = x0 + min(4 * xr + k, HX - 1) - 1;
        gx = gx < 0 ? gx + s : (gx >= s ? gx - s : gx);
        r4[k] = *reinterpret_cast<const uint4*>(in + (vrow + gx) * in_cs + in_co + 16 * cs + 8 * half);
      }
      transpose_4x8(r4, xT + ((8 * half) * HZ * HY + rr) * 16 + 4 * xr, HZ * HY * 16);
    }
    __syncthreads();
    if (TX == 8) {
      // tile side 8: every read of a K step (B, and the two row halves of
      // each of the wave's tap rows) is issued before its MFMAs
      for (int q = 0; q < NV / 32; ++q) {
        const int u0 = 32 * q + 8 * grp;
        bf16x8 bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          bv[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(gT + (16 * nt + m) * NV + u0));
        const int y = (u0 >> 3) & (TY - 1), z = u0 >> (3 + T.ly);
        uint4 lo[kMaxRows], hi[kMaxRows];
#pragma unroll
        for (int k = 0; k < kMaxRows; ++k) {
          const int j = min(wave + nw * k, 8);   // rows past 8 read row 8 and are not used
          const unsigned short* row = xT + ((m * HZ + z + j / 3) * HY + y + j % 3) * 16;
          lo[k] = *reinterpret_cast<const uint4*>(row);
          hi[k] = *reinterpret_cast<const uint4*>(row + 8);
        }
        __builtin_amdgcn_sched_barrier(0);   // else each read is sunk to its MFMAs and waited for alone
#pragma unroll
        for (int k = 0; k < kMaxRows; ++k) {
          if (wave + nw * k >= 9) continue;
          const bf16x8 a0 = as_bf16x8(lo[k]);
          const bf16x8 a1 = as_bf16x8(make_uint4(__builtin_amdgcn_alignbyte(lo[k].y, lo[k].x, 2),
                                                 __builtin_amdgcn_alignbyte(lo[k].z, lo[k].y, 2),
                                                 __builtin_amdgcn_alignbyte(lo[k].w, lo[k].z, 2),
                                                 __builtin_amdgcn_alignbyte(hi[k].x, lo[k].w, 2)));
          const bf16x8 a2 = as_bf16x8(make_uint4(lo[k].y, lo[k].z, lo[k].w, hi[k].x));
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            acc[k][0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv[nt], acc[k][0][nt], 0, 0, 0);
            acc[k][1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv[nt], acc[k][1][nt], 0, 0, 0);
            acc[k][2][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bv[nt], acc[k][2][nt], 0, 0, 0);
          }
        }
      }
      continue;                      // next tile
    }
    for (int q = 0; q < NV / 32; ++q) {
      // lane group grp: voxels u = 32 q + 8 grp .. +8; B once per step
      const int u0 = 32 * q + 8 * grp;
      bf16x8 bv[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) bv[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(gT + (16 * nt + m) * NV + u0));
#pragma unroll
      for (int k = 0; k < kMaxRows; ++k) {
        const int j = wave + nw * k;   // tap row (dz, dy); taps 3 j + dx
        if (j >= 9) continue;
        const int dz = j / 3, dy = j % 3;
        if (TX == 8) {
          const int y = (u0 >> 3) & (TY - 1), z = u0 >> (3 + T.ly);
          const unsigned short* row = xT + ((m * HZ + z + dz) * HY + y + dy) * 16;
          const uint4 lo = *reinterpret_cast<const uint4*>(row);
          const uint4 hi = *reinterpret_cast<const uint4*>(row + 8);
          const bf16x8 a0 = as_bf16x8(lo);
          const bf16x8 a1 = as_bf16x8(make_uint4(__builtin_amdgcn_alignbyte(lo.y, lo.x, 2),
                                                 __builtin_amdgcn_alignbyte(lo.z, lo.y, 2),
                                                 __builtin_amdgcn_alignbyte(lo.w, lo.z, 2),
                                                 __builtin_amdgcn_alignbyte(hi.x, lo.w, 2)));
          const bf16x8 a2 = as_bf16x8(make_uint4(lo.y, lo.z, lo.w, hi.x));
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            acc[k][0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv[nt], acc[k][0][nt], 0, 0, 0);
            acc[k][1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv[nt], acc[k][1][nt], 0, 0, 0);
            acc[k][2][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bv[nt], acc[k][2][nt], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            unsigned int w4[4];
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
              unsigned int pair = 0;
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int u = u0 + 2 * k2 + h;
                const int x = u & (TX - 1), y = (u >> T.lx) & (TY - 1), z = u >> (T.lx + T.ly);
                pair |= (unsigned int)xT[((m * HZ + z + dz) * HY + y + dy) * 16 + x + dx] << (16 * h);
              }
              w4[k2] = pair;
            }
            const bf16x8 av = as_bf16x8(make_uint4(w4[0], w4[1], w4[2], w4[3]));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[k][dx][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[k][dx][nt], 0, 0, 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxRows; ++k) {
    const int jr = wave + nw * k;
    if (jr >= 9) continue;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = 3 * jr + dx;
          const int ci = 16 * cs + 4 * grp + j;
          part[(((long long)r * 27 + t) * cin_pad + ci) * cout + 16 * nt + m] = acc[k][dx][nt][j];
        }
  }
}

// G[t][ci][co] += sum over r of part[r][t][ci][co] (ci < cin) and, for the
// outputs after those, gb[co] += sum over the blocks b < nb of
// bpart[b][co], in a fixed order: a block takes OW consecutive outputs
// (32: 128-byte rows for many outputs; 8: more blocks and more rows in
// flight for few); its RW = 256 / OW lane rows sum the rows r = row, row +
// RW, ... (four running sums, taking every fourth of them, added pairwise),
// and the RW row sums are added in order.
template <int OW>
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* __restrict__ part, int nr, int cin, int cin_pad,
                                                      int cout, float* __restrict__ gw, const float* __restrict__ bpart,
                                                      int nb, float* __restrict__ gb) {
  constexpr int RW = 256 / OW;
  __shared__ float sh[RW][OW];
  const long long nw = 27LL * cin * cout;
  const int o = threadIdx.x % OW, row = threadIdx.x / OW;
  const long long i = (long long)blockIdx.x * OW + o;
  float s4[4] = {0.f, 0.f, 0.f, 0.f};
  const float* p = nullptr;
  long long stride = 0;
  int rows = 0;
  if (i < nw) {
    const int co = (int)(i % cout);
    const int ci = (int)((i / cout) % cin);
    const int t = (int)(i / ((long long)cout * cin));
    stride = 27LL * cin_pad * cout;
    p = part + ((long long)t * cin_pad + ci) * cout + co;
    rows = nr;
  } else if (i < nw + cout) {
    stride = cout;
    p = bpart + (i - nw);
    rows = nb;
  }
  int r = row;
  for (; r + 3 * RW < rows; r += 4 * RW) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s4[k] += p[(r + RW * k) * stride];
  }
  for (int k = 0; r < rows; r += RW, ++k) s4[k] += p[r * stride];
  sh[row][o] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  __syncthreads();
  if (row == 0) {
    float tot = 0.f;
    for (int q = 0; q < RW; ++q) tot += sh[q][o];
    if (i < nw) gw[i] += tot;
    else if (i < nw + cout) gb[i - nw] += tot;
  }
}

// out[k] += sum over the rows b < nb of part[b][k]: one block per k, rows
// taken by the threads in a fixed pattern and added in a fixed tree
__global__ void __launch_bounds__(256) k_rows_reduce(const float* __restrict__ part, int nb, int nk,
                                                     float* __restrict__ out) {
  __shared__ float sh[256];
  const int k = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(long long)b * nk + k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] += sh[0];
}

// ---------------------------------------------------------------------------
// elementwise and data-movement kernels

__global__ void k_input(const float* __restrict__ T, const float* __restrict__ R, float scale, int V,
                        unsigned short* __restrict__ x) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
#pragma unroll
  for (int c = 0; c < 16; ++c) x[(long long)v * 16 + c] = 0;
  x[(long long)v * 16] = f2bf(scale * T[v]);
  x[(long long)v * 16 + 1] = f2bf(scale * R[v]);
}

// First convolution (2 input channels: the template and the reference, each
// scaled and rounded to bf16 exactly as k_input stores them).  The general
// kernel would pad the 2 channels to 16; here K runs over (tap, channel)
// pairs, k = 2 tap + ci, 54 of them padded to 64: two double-K MFMA steps.
// A block takes an 8 x 8 x 4 tile (side a multiple of 8); its halo sits in
// LDS as one 32-bit word per voxel (the bf16 pair of T and R), so a lane's
// A operand (taps 16 s + 4 grp .. + 3 of its voxel, both channels) is four
// word reads, and the B operand of each 16-channel output tile stays in
// registers for the whole block.  Writes the bf16 relu activation
// act[v][co] (view act_cs, act_co); wf is the forward weight copy
// [tap][co][wk].
__global__ void __launch_bounds__(256) k_conv_in2(const float* __restrict__ T, const float* __restrict__ R,
                                                  float scale, int s, const unsigned short* __restrict__ wf,
                                                  int wk, int cout, const float* __restrict__ bias,
                                                  unsigned short* __restrict__ act, int act_cs, int act_co) {
  __shared__ unsigned int hx[10 * 10 * 6];
  const int ntx = s >> 3, nty = s >> 3;
  const int b = blockIdx.x;
  const int x0 = (b % ntx) << 3, y0 = ((b / ntx) % nty) << 3, z0 = (b / (ntx * nty)) << 2;
  for (int q = threadIdx.x; q < 600; q += blockDim.x) {
    const int hx_ = q % 10, hy = (q / 10) % 10, hz = q / 100;
    int gx = x0 + hx_ - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
    gx = gx < 0 ? gx + s : (gx >= s ? gx - s : gx);
    gy = gy < 0 ? gy + s : (gy >= s ? gy - s : gy);
    gz = gz < 0 ? gz + s : (gz >= s ? gz - s : gz);
    const long long v = ((long long)gz * s + gy) * s + gx;
    hx[q] = (unsigned int)f2bf(scale * T[v]) | ((unsigned int)f2bf(scale * R[v]) << 16);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, grp = lane >> 4;
  // A operands of the wave's four 16-voxel row tiles, both K steps
  bf16x8 av[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int u = 64 * wave + 16 * i + m;
    const int x = u & 7, y = (u >> 3) & 7, z = u >> 6;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      unsigned int w4[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = 16 * st + 4 * grp + j;
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        w4[j] = t < 27 ? hx[((z + dz) * 10 + y + dy) * 10 + x + dx] : 0u;
      }
      av[i][st] = as_bf16x8(make_uint4(w4[0], w4[1], w4[2], w4[3]));
    }
  }
  for (int nt = 0; nt < cout / 16; ++nt) {
    const int co = 16 * nt + m;
    bf16x8 bw[2];
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      unsigned int w4[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = 16 * st + 4 * grp + j;
        w4[j] = t < 27 ? (unsigned int)wf[((long long)t * cout + co) * wk] |
                             ((unsigned int)wf[((long long)t * cout + co) * wk + 1] << 16)
                       : 0u;
      }
      bw[st] = as_bf16x8(make_uint4(w4[0], w4[1], w4[2], w4[3]));
    }
    const float bco = bias[co];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i][0], bw[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i][1], bw[1], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 64 * wave + 16 * i + 4 * grp + j;
        const long long v = ((long long)(z0 + (u >> 6)) * s + y0 + ((u >> 3) & 7)) * s + x0 + (u & 7);
        act[v * act_cs + act_co + co] = f2bf(fmaxf(acc[j] + bco, 0.f));
      }
    }
  }
}

// Voxel and channel of the flat element i = v c + ch for a channel count c
// that is a power of two (16, 32 or 64 here), and x, y, z of voxel v on a
// grid of side s: 32-bit arithmetic (at most 256^3 x 64 < 2^31 elements;
// 64-bit divisions expand into long branchy sequences).
__device__ __forceinline__ void split_vc(long long i, int c, int& v, int& ch) {
  const unsigned ui = (unsigned)i;
  v = (int)(ui >> (__ffs(c) - 1));
  ch = (int)(ui & (unsigned)(c - 1));
}
__device__ __forceinline__ void split_xyz(int v, int s, int& x, int& y, int& z) {
  const unsigned uv = (unsigned)v, us = (unsigned)s, t = uv / us;
  x = (int)(uv - t * us);
  y = (int)(t % us);
  z = (int)(t / us);
}

// pool: out (size s/2) = mean of the 2x2x2 children of `in` (size s)
__global__ void k_pool(const unsigned short* __restrict__ in, int in_cs, int in_co, int c, int s,
                       unsigned short* __restrict__ out) {
  const int h = s / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)h * h * h * c) return;
  int v, ch, x, y, z;
  split_vc(i, c, v, ch);
  split_xyz(v, h, x, y, z);
  float sum = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int fv = ((2 * z + (o >> 2)) * s + 2 * y + ((o >> 1) & 1)) * s + 2 * x + (o & 1);
    sum += bf2f(in[(long long)fv * in_cs + in_co + ch]);
  }
  out[i] = f2bf(0.125f * sum);
}

// up: out view (size s) channel slice [0, c) = copy of the parent in `in`
// (size s/2); 8 channels (16 bytes) per thread
__global__ void k_up(const unsigned short* __restrict__ in, int c, int s, unsigned short* __restrict__ out,
                     int out_cs) {
  const int c8 = c / 8;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)s * s * s * c8) return;
  int v, ch, x, y, z;
  split_vc(i, c8, v, ch);
  ch *= 8;
  split_xyz(v, s, x, y, z);
  const int h = s / 2;
  const int pv = ((z >> 1) * h + (y >> 1)) * h + (x >> 1);
  *reinterpret_cast<uint4*>(out + (long long)v * out_cs + ch) =
      *reinterpret_cast<const uint4*>(in + (long long)pv * c + ch);
}

// gpre = g (float, view of width gcs at offset goff) masked by the layer's
// relu (its bf16 activation, view of width acs at offset aco, is non-zero
// exactly where the pre-activation is positive); writes the bf16 copy and
// the block's bias-gradient partials part[block][c] (summed in block order
// by k_wgrad_reduce).  8 channels per thread (16-byte loads and stores).
__global__ void k_relu_back(const float* __restrict__ g, int gcs, int goff, const unsigned short* __restrict__ act,
                            int acs, int aco, int c, int V, unsigned short* __restrict__ gb,
                            float* __restrict__ part) {
  __shared__ float sh[256][9];
  // grid-stride over groups of 8 channels: the stride is a multiple of 256
  // and c / 8 divides 256, so a thread keeps its channel group and sums in a
  // fixed order
  const int c8 = c >> 3;
  float val[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const long long n8 = (long long)V * c8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += (long long)gridDim.x * blockDim.x) {
    const int ch = 8 * (int)(i % c8);
    const long long v = i / c8;
    const float4 g0 = *reinterpret_cast<const float4*>(g + v * gcs + goff + ch);
    const float4 g1 = *reinterpret_cast<const float4*>(g + v * gcs + goff + ch + 4);
    const uint4 a = *reinterpret_cast<const uint4*>(act + v * acs + aco + ch);
    const float gi[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
    const unsigned int aw[4] = {a.x, a.y, a.z, a.w};
    unsigned int pk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float lo = (aw[q] & 0x7fffu) != 0u ? gi[2 * q] : 0.f;
      const float hi = (aw[q] & 0x7fff0000u) != 0u ? gi[2 * q + 1] : 0.f;
      val[2 * q] += lo;
      val[2 * q + 1] += hi;
      pk[q] = (unsigned int)f2bf(lo) | ((unsigned int)f2bf(hi) << 16);
    }
    *reinterpret_cast<uint4*>(gb + 8 * i) = make_uint4(pk[0], pk[1], pk[2], pk[3]);
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) sh[threadIdx.x][e] = val[e];
  __syncthreads();
  if ((int)threadIdx.x < c) {
    const int grp = threadIdx.x >> 3, e = threadIdx.x & 7;
    float s = 0.f;
    // rows k = grp, grp + c8, ... (256 / c8 of them, a multiple of 8) added
    // in that order, eight LDS reads in flight at a time
    for (int k0 = grp; k0 < 256; k0 += 8 * c8) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = sh[k0 + u * c8][e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
    part[(long long)blockIdx.x * c + threadIdx.x] = s;
  }
}

// g (size s/2, c channels) += pool-adjoint of gf (size s view): gf / 8 summed? No:
// the gradient of pool at the children is parent / 8 -> add to a full-size buffer
__global__ void k_pool_back(const float* __restrict__ gp, int c, int s, float* __restrict__ gf, int gf_cs,
                            int gf_co) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)s * s * s * c) return;
  int v, ch, x, y, z;
  split_vc(i, c, v, ch);
  split_xyz(v, s, x, y, z);
  const int h = s / 2;
  const int pv = ((z >> 1) * h + (y >> 1)) * h + (x >> 1);
  gf[(long long)v * gf_cs + gf_co + ch] += 0.125f * gp[(long long)pv * c + ch];
}

// gp (size s/2, c) = sum over children of the channel slice [0, c) of g (size s, width gcs)
__global__ void k_up_back(const float* __restrict__ g, int gcs, int c, int s, float* __restrict__ gp) {
  const int h = s / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)h * h * h * c) return;
  int v, ch, x, y, z;
  split_vc(i, c, v, ch);
  split_xyz(v, h, x, y, z);
  float sum = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int fv = ((2 * z + (o >> 2)) * s + 2 * y + ((o >> 1) & 1)) * s + 2 * x + (o & 1);
    sum += g[(long long)fv * gcs + ch];
  }
  gp[i] = sum;
}

// copy channel slice [off, off + c) of g (width gcs) into a compact buffer
__global__ void k_slice(const float* __restrict__ g, int gcs, int off, int c, int V, float* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)V * c) return;
  out[i] = g[(i / c) * gcs + off + i % c];
}

__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

// head: v[k][vox] = scale * (sum_c d0[vox][c] Wh[c][k] + bh[k])
__global__ void k_head_fwd(const unsigned short* __restrict__ d0, int c, int V, const float* __restrict__ wh,
                           const float* __restrict__ bh, float scale, float* __restrict__ vout) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  float o0 = bh[0], o1 = bh[1], o2 = bh[2];
  // the voxel's channels (a multiple of 16) as 16-byte loads, all issued
  // before the sums, which take the channels in order
  for (int c16 = 0; c16 < c; c16 += 16) {
    const uint4 r0 = *reinterpret_cast<const uint4*>(d0 + (long long)v * c + c16);
    const uint4 r1 = *reinterpret_cast<const uint4*>(d0 + (long long)v * c + c16 + 8);
    const unsigned int rw[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int ch = c16 + e;
      const float a = __uint_as_float((e & 1) ? (rw[e >> 1] & 0xffff0000u) : (rw[e >> 1] << 16));
      o0 = fmaf(a, wh[ch * 3 + 0], o0);
      o1 = fmaf(a, wh[ch * 3 + 1], o1);
      o2 = fmaf(a, wh[ch * 3 + 2], o2);
    }
  }
  vout[v] = scale * o0;
  vout[V + v] = scale * o1;
  vout[2 * V + v] = scale * o2;
}

// loss = 1/2 mean (v - target)^2 (FP64 partials), gout = scale (v - target) / n
__global__ void k_mse(const float* __restrict__ v, const float* __restrict__ tgt, long long n, float gscale,
                      float* __restrict__ gout, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float d = v[i] - tgt[i];
    s += (double)d * d;
    gout[i] = gscale * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_mse_final(const double* __restrict__ part, int n, double scale,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * sh[0];
}

// Head backward (1x1, 3 outputs): gd0[v][ch] = sum_k go[k][v] Wh[ch][k]
// (float4 stores), and the block's partials of the head gradients,
// part[block][3 ch + k] = sum_v d0[v][ch] go[k][v] and part[block][3 c + k]
// = sum_v go[k][v].  Grid-stride over voxels with the sums in registers, 16
// channels at a time; a wave adds its lanes in a fixed butterfly and the
// block its four waves in order.
__global__ void __launch_bounds__(256) k_head_bwd(const unsigned short* __restrict__ d0, int c, int V,
                                                  const float* __restrict__ wh, const float* __restrict__ go,
                                                  float* __restrict__ gd0, float* __restrict__ part) {
  __shared__ float sh[4][51];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nk = 3 * c + 3;
  auto wave_sum = [](float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
  };
  for (int c16 = 0; c16 < c; c16 += 16) {
    float acc[16][3], ab[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e][0] = acc[e][1] = acc[e][2] = 0.f;
    float w[16][3];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      w[e][0] = wh[(c16 + e) * 3];
      w[e][1] = wh[(c16 + e) * 3 + 1];
      w[e][2] = wh[(c16 + e) * 3 + 2];
    }
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
      const float g[3] = {go[v], go[V + v], go[2 * V + v]};
      const uint4 r0 = *reinterpret_cast<const uint4*>(d0 + (long long)v * c + c16);
      const uint4 r1 = *reinterpret_cast<const uint4*>(d0 + (long long)v * c + c16 + 8);
      const unsigned int rw[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float a = __uint_as_float((e & 1) ? (rw[e >> 1] & 0xffff0000u) : (rw[e >> 1] << 16));
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[e][k] = fmaf(a, g[k], acc[e][k]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) ab[k] += g[k];
      float4* dst = reinterpret_cast<float4*>(gd0 + (long long)v * c + c16);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float o[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = 4 * q + t;
          o[t] = g[0] * w[e][0] + g[1] * w[e][1] + g[2] * w[e][2];
        }
        dst[q] = make_float4(o[0], o[1], o[2], o[3]);
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float t = wave_sum(acc[e][k]);
        if (lane == 0) sh[wave][e * 3 + k] = t;
      }
    if (c16 == 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float t = wave_sum(ab[k]);
        if (lane == 0) sh[wave][48 + k] = t;
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 51; k += blockDim.x) {
      const float t = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
      if (k < 48) part[(long long)blockIdx.x * nk + 3 * c16 + k] = t;
      else if (c16 == 0) part[(long long)blockIdx.x * nk + 3 * c + (k - 48)] = t;
    }
    __syncthreads();
  }
}

// bf16 weight copies of every convolution in one launch: layer l covers
// threads [start[l], start[l + 1]); wf[t][co][ci_pad], wb[t][ci_pad][co]
// from w[t][ci][co], t < kTaps (tap 27 and the padded channels are zero)
struct WcopyArgs {
  const float* w[kLayers - 1];
  unsigned short* wf[kLayers - 1];
  unsigned short* wb[kLayers - 1];
  int cin[kLayers - 1], cinp[kLayers - 1], cout[kLayers - 1];
  long long start[kLayers];
};

__global__ void k_wcopy(WcopyArgs A) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.start[kLayers - 1]) return;
  int l = 0;
  while (i >= A.start[l + 1]) ++l;
  i -= A.start[l];
  const float* __restrict__ w = A.w[l];
  unsigned short* __restrict__ wf = A.wf[l];
  unsigned short* __restrict__ wb = A.wb[l];
  const int cin = A.cin[l], cin_pad = A.cinp[l], cout = A.cout[l];
  const int co = (int)(i % cout);
  const int ci = (int)((i / cout) % cin_pad);
  const int t = (int)(i / ((long long)cout * cin_pad));
  const unsigned short val =
      (ci < cin && t < 27) ? f2bf(w[((long long)t * cin + ci) * cout + co]) : (unsigned short)0;
  wb[((long long)t * cin_pad + ci) * cout + co] = val;
  wf[((long long)t * cout + co) * cin_pad + ci] = val;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace cnn
}  // namespace lag

// ===========================================================================
// host side

using namespace lag;
using namespace lag::cnn;

struct lag_cnn_s {
  lag_cnn_config cfg;
  int S;
  int c[4];
  int cin[kLayers], cout[kLayers], cinp[kLayers], taps[kLayers];
  int lsize[kLayers];                // grid side of each layer
  long long woff[kLayers], boff[kLayers];
  long long nparams = 0;
  float *P = nullptr, *G = nullptr, *M1 = nullptr, *M2 = nullptr;   // params, grads, Adam moments
  unsigned short* wf[kLayers] = {nullptr};
  unsigned short* wb[kLayers] = {nullptr};
  // activations (bf16); per layer, the view its forward wrote its output to
  unsigned short* x0 = nullptr;      // S^3 x 16
  unsigned short* a[kLayers] = {nullptr};
  unsigned short* actp[kLayers] = {nullptr};
  int acs[kLayers] = {0}, aco[kLayers] = {0};
  unsigned short *p0 = nullptr, *p1 = nullptr, *p2 = nullptr;   // pooled
  unsigned short *cat2 = nullptr, *cat1 = nullptr, *cat0 = nullptr;
  // gradients
  float* gbuf[4] = {nullptr};        // scratch per level (largest widths)
  float* gcat[3] = {nullptr};        // g of cat0 / cat1 / cat2
  float* gtmp[4] = {nullptr};
  // per layer: the bf16 gradient of its pre-activation and its bias
  // partials (the weight gradient reads them on the side stream while the
  // next layers' backward runs on the caller's)
  unsigned short* gbl[kLayers] = {nullptr};
  float* bpl[kLayers] = {nullptr};
  hipStream_t side = nullptr;        // weight gradients (default priority)
  hipEvent_t fork[kLayers] = {nullptr};
  hipEvent_t join = nullptr;
  float* gout = nullptr;             // 3 x S^3
  double* part = nullptr;
  float* wpart = nullptr;            // weight-gradient partials per voxel range
  float* kpart = nullptr;            // split-contraction partials of the convolutions
  float* bpart = nullptr;            // bias / head gradient partials per block
  int adam_t = 0;
  bool wdirty = true;                // master weights changed since the last bf16 copy
};

static int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// output tiles of a grid of side s, and the voxel ranges of the weight gradient
static int conv_tiles(int s) {
  const ConvTile t = conv_tile(s);
  return (s >> t.lx) * (s >> t.ly) * (s >> t.lz);
}
// tiles per voxel range of the weight gradient: about 512 blocks over the
// ranges and the 16-channel input slices (fewer ranges for wide inputs keep
// the partials, ranges x 27 x cin x cout floats, small)
static int wgrad_per_range(int s, int cinp) { return ceil_div((long long)conv_tiles(s) * (cinp / 16), 512); }
static int wgrad_ranges(int s, int cinp) { return ceil_div(conv_tiles(s), wgrad_per_range(s, cinp)); }

// 16-channel output tiles per block: up to 4 on grids of side >= 32, else 1
// (more blocks on the small grids)
static int conv_nt(int s, int n16) {
  if (s < 32) return 1;
  for (int nt = 4; nt > 1; --nt)
    if (n16 % nt == 0) return nt;
  return 1;
}

// Split of the contraction over blockIdx.z when a layer has fewer than 512
// blocks: each block then takes every kz-th 16-channel chunk.
static int conv_split(int s, int nout, int kch) {
  const int blocks = conv_tiles(s) * (nout / (16 * conv_nt(s, nout / 16)));
  if (blocks >= 512) return 1;
  return std::max(1, std::min(std::min(kch / 16, kMaxSplit), ceil_div(512, blocks)));
}

extern "C" {

void lag_cnn_default_config(lag_cnn_config* c) {
  if (!c) return;
  c->size = 64;
  c->channels[0] = 16;
  c->channels[1] = 32;
  c->channels[2] = 64;
  c->channels[3] = 64;
  c->in_scale = 1.f;
  c->out_scale = 0.05f;
  c->seed = 1;
}

int lag_cnn_destroy(lag_cnn n) {
  if (!n) return LAG_OK;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {n->P, n->G, n->M1, n->M2, n->x0, n->p0, n->p1, n->p2, n->cat2, n->cat1, n->cat0,
                  n->gout, n->part, n->wpart, n->bpart, n->kpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int l = 0; l < kLayers; ++l) {
    if (n->wf[l]) (void)hipFree(n->wf[l]);
    if (n->wb[l]) (void)hipFree(n->wb[l]);
    if (n->a[l]) (void)hipFree(n->a[l]);
    if (n->gbl[l]) (void)hipFree(n->gbl[l]);
    if (n->bpl[l]) (void)hipFree(n->bpl[l]);
    if (n->fork[l]) (void)hipEventDestroy(n->fork[l]);
  }
  if (n->join) (void)hipEventDestroy(n->join);
  if (n->side) (void)hipStreamDestroy(n->side);
  for (int i = 0; i < 4; ++i) {
    if (n->gbuf[i]) (void)hipFree(n->gbuf[i]);
    if (n->gtmp[i]) (void)hipFree(n->gtmp[i]);
  }
  for (int i = 0; i < 3; ++i)
    if (n->gcat[i]) (void)hipFree(n->gcat[i]);
  delete n;
  return LAG_OK;
}

#define CNN_ALLOC(ptr, bytes)                                  \
  do {                                                         \
    if (hipMalloc((void**)&(ptr), (bytes)) != hipSuccess) {    \
      (void)hipGetLastError();                                 \
      lag_cnn_destroy(n);                                      \
      return LAG_ENOMEM;                                       \
    }                                                          \
  } while (0)

int lag_cnn_create(const lag_cnn_config* cfg, lag_cnn* out) {
  if (!cfg || !out) return LAG_EINVAL;
  *out = nullptr;
  const int S = cfg->size;
  // every level's voxel count must be a multiple of 64 (one wave tile)
  if (S < 32 || S % 32 || S > 256) return LAG_EINVAL;
  for (int i = 0; i < 4; ++i) {
    const int c = cfg->channels[i];
    if (c != 16 && c != 32 && c != 64) return LAG_EINVAL;
  }
  lag_cnn n = new lag_cnn_s();
  n->cfg = *cfg;
  n->S = S;
  for (int i = 0; i < 4; ++i) n->c[i] = cfg->channels[i];
  const int c0 = n->c[0], c1 = n->c[1], c2 = n->c[2], c3 = n->c[3];
  const int io[kLayers][2] = {{2, c0},  {c0, c0}, {c0, c1}, {c1, c1},      {c1, c2},      {c2, c2},
                              {c2, c3}, {c3, c3}, {c3 + c2, c2}, {c2 + c1, c1}, {c1 + c0, c0}, {c0, 3}};
  const int sz[kLayers] = {S, S, S / 2, S / 2, S / 4, S / 4, S / 8, S / 8, S / 4, S / 2, S, S};
  long long off = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->cin[l] = io[l][0];
    n->cout[l] = io[l][1];
    n->cinp[l] = l == E0A ? 16 : io[l][0];
    n->taps[l] = l == HEAD ? 1 : 27;
    n->lsize[l] = sz[l];
    n->woff[l] = off;
    off += (long long)n->taps[l] * n->cin[l] * n->cout[l];
    n->boff[l] = off;
    off += n->cout[l];
  }
  n->nparams = off;
  CNN_ALLOC(n->P, sizeof(float) * off);
  CNN_ALLOC(n->G, sizeof(float) * off);
  CNN_ALLOC(n->M1, sizeof(float) * off);
  CNN_ALLOC(n->M2, sizeof(float) * off);
  // He-normal initialisation on the host (deterministic from the seed)
  {
    std::vector<float> h(off, 0.f);
    std::mt19937_64 rng(cfg->seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < kLayers; ++l) {
      const double std = l == HEAD ? sqrt(1.0 / n->cin[l]) : sqrt(2.0 / (27.0 * n->cin[l]));
      const long long cnt = (long long)n->taps[l] * n->cin[l] * n->cout[l];
      for (long long i = 0; i < cnt; ++i) h[n->woff[l] + i] = (float)(nd(rng) * std);
    }
    if (hipMemcpy(n->P, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess) {
      lag_cnn_destroy(n);
      return LAG_EHIP;
    }
    (void)hipMemset(n->M1, 0, sizeof(float) * off);
    (void)hipMemset(n->M2, 0, sizeof(float) * off);
  }
  size_t wpart = 0, kpart = 0;
  for (int l = 0; l < HEAD; ++l) {
    const size_t Vl = (size_t)sz[l] * sz[l] * sz[l];
    kpart = std::max(kpart, (size_t)conv_split(sz[l], n->cout[l], n->cinp[l]) * Vl * n->cout[l]);
    kpart = std::max(kpart, (size_t)conv_split(sz[l], n->cinp[l], n->cout[l]) * Vl * n->cinp[l]);
    const size_t wn = (size_t)kTaps * n->cinp[l] * n->cout[l];
    CNN_ALLOC(n->wf[l], 2 * wn);
    CNN_ALLOC(n->wb[l], 2 * wn);
    wpart = std::max(wpart, (size_t)wgrad_ranges(sz[l], n->cinp[l]) * 27 * n->cinp[l] * n->cout[l]);
  }
  const long long V0 = (long long)S * S * S, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  CNN_ALLOC(n->x0, 2 * V0 * 16);
  // activations that are not written into a concatenation buffer
  CNN_ALLOC(n->a[E0A], 2 * V0 * c0);
  CNN_ALLOC(n->a[E1A], 2 * V1 * c1);
  CNN_ALLOC(n->a[E2A], 2 * V2 * c2);
  CNN_ALLOC(n->a[MA], 2 * V3 * c3);
  CNN_ALLOC(n->a[MB], 2 * V3 * c3);
  CNN_ALLOC(n->a[D2], 2 * V2 * c2);
  CNN_ALLOC(n->a[D1], 2 * V1 * c1);
  CNN_ALLOC(n->a[D0], 2 * V0 * c0);
  CNN_ALLOC(n->p0, 2 * V1 * c0);
  CNN_ALLOC(n->p1, 2 * V2 * c1);
  CNN_ALLOC(n->p2, 2 * V3 * c2);
  CNN_ALLOC(n->cat0, 2 * V0 * (c1 + c0));   // [up(dec1) | enc0]
  CNN_ALLOC(n->cat1, 2 * V1 * (c2 + c1));   // [up(dec2) | enc1]
  CNN_ALLOC(n->cat2, 2 * V2 * (c3 + c2));   // [up(mid)  | enc2]
  CNN_ALLOC(n->gcat[0], sizeof(float) * V0 * (c1 + c0));
  CNN_ALLOC(n->gcat[1], sizeof(float) * V1 * (c2 + c1));
  CNN_ALLOC(n->gcat[2], sizeof(float) * V2 * (c3 + c2));
  const long long Vs[4] = {V0, V1, V2, V3};
  for (int i = 0; i < 4; ++i) {
    CNN_ALLOC(n->gbuf[i], sizeof(float) * Vs[i] * 64);
    CNN_ALLOC(n->gtmp[i], sizeof(float) * Vs[i] * 64);
  }
  for (int l = 0; l < HEAD; ++l) {
    const long long Vl = (long long)sz[l] * sz[l] * sz[l];
    CNN_ALLOC(n->gbl[l], 2 * Vl * n->cout[l]);
    CNN_ALLOC(n->bpl[l], sizeof(float) * 1024 * n->cout[l]);
    if (hipEventCreateWithFlags(&n->fork[l], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      lag_cnn_destroy(n);
      return LAG_EHIP;
    }
  }
  if (hipEventCreateWithFlags(&n->join, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&n->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    lag_cnn_destroy(n);
    return LAG_EHIP;
  }
  CNN_ALLOC(n->gout, sizeof(float) * 3 * V0);
  CNN_ALLOC(n->part, sizeof(double) * 1024);
  CNN_ALLOC(n->wpart, sizeof(float) * wpart);
  CNN_ALLOC(n->kpart, sizeof(float) * kpart);
  // bias partials: one row of c per 256 (voxel, channel) pairs; head: 3 c + 3 per 256 voxels
  CNN_ALLOC(n->bpart, sizeof(float) * std::max<long long>(1024 * 64, (V0 / 256 + 1) * (3 * 64 + 3)));
  *out = n;
  return LAG_OK;
}

int lag_cnn_param_count(lag_cnn n, int64_t* count) {
  if (!n || !count) return LAG_EINVAL;
  *count = n->nparams;
  return LAG_OK;
}

int lag_cnn_get_params(lag_cnn n, float* host) {
  if (!n || !host) return LAG_EINVAL;
  LAG_HIP(hipDeviceSynchronize());
  LAG_HIP(hipMemcpy(host, n->P, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  return LAG_OK;
}

int lag_cnn_set_params(lag_cnn n, const float* host) {
  if (!n || !host) return LAG_EINVAL;
  LAG_HIP(hipMemcpy(n->P, host, sizeof(float) * n->nparams, hipMemcpyHostToDevice));
  n->wdirty = true;
  n->adam_t = 0;
  LAG_HIP(hipMemset(n->M1, 0, sizeof(float) * n->nparams));
  LAG_HIP(hipMemset(n->M2, 0, sizeof(float) * n->nparams));
  return LAG_OK;
}

int lag_cnn_get_grads(lag_cnn n, float* host) {
  if (!n || !host) return LAG_EINVAL;
  LAG_HIP(hipDeviceSynchronize());   // every stream's work, the side stream's included
  LAG_HIP(hipMemcpy(host, n->G, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  return LAG_OK;
}

}  // extern "C"

// ---- launch helpers ----------------------------------------------------------

static size_t conv_lds(ConvTile T, int nt);

template <bool BWD>
static int launch_conv(lag_cnn n, int s, int nout, const unsigned short* in, int in_cs, int in_co, int kch,
                       const unsigned short* w, int wn, int wk, const float* bias, float* out, unsigned short* act,
                       int act_cs, int act_co, hipStream_t st) {
  const ConvTile T = conv_tile(s);
  const int nt = conv_nt(s, nout / 16), kz = conv_split(s, nout, kch);
  const dim3 grid(conv_tiles(s), nout / (16 * nt), kz), block(1 << (T.lx + T.ly + T.lz));
  const size_t lds = conv_lds(T, nt);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_conv_mfma<BWD, 1>), grid, block, lds, st, in, in_cs, in_co, kch, s, T, w, wn, wk, bias, out, nout, act, act_cs, act_co, n->kpart); break;
    case 2: hipLaunchKernelGGL((k_conv_mfma<BWD, 2>), grid, block, lds, st, in, in_cs, in_co, kch, s, T, w, wn, wk, bias, out, nout, act, act_cs, act_co, n->kpart); break;
    case 3: hipLaunchKernelGGL((k_conv_mfma<BWD, 3>), grid, block, lds, st, in, in_cs, in_co, kch, s, T, w, wn, wk, bias, out, nout, act, act_cs, act_co, n->kpart); break;
    default: hipLaunchKernelGGL((k_conv_mfma<BWD, 4>), grid, block, lds, st, in, in_cs, in_co, kch, s, T, w, wn, wk, bias, out, nout, act, act_cs, act_co, n->kpart); break;
  }
  LAG_LAUNCH_CHECK();
  if (kz > 1) {
    const long long V = (long long)s * s * s;
    const dim3 fg(ceil_div(V * nout, 256));
#define LAG_FIN(KZ)                                                                                         \
  hipLaunchKernelGGL((k_conv_finish<BWD, KZ>), fg, dim3(256), 0, st, n->kpart, V, nout, bias, out, act, act_cs, \
                     act_co)
    switch (kz) {
      case 2: LAG_FIN(2); break;
      case 3: LAG_FIN(3); break;
      case 4: LAG_FIN(4); break;
      case 5: LAG_FIN(5); break;
      case 6: LAG_FIN(6); break;
      case 7: LAG_FIN(7); break;
      default: LAG_FIN(8); break;   // conv_split never exceeds kMaxSplit = 8
    }
#undef LAG_FIN
    LAG_LAUNCH_CHECK();
  }
  return LAG_OK;
}

static size_t conv_lds(ConvTile T, int nt) {
  return sizeof(unsigned short) * (kRow * (size_t)(((1 << T.lx) + 2) * ((1 << T.ly) + 2) * ((1 << T.lz) + 2)) +
                                   (size_t)kTaps * 16 * nt * 16);
}

static int conv_fwd(lag_cnn n, int l, const unsigned short* in, int in_cs, int in_co, unsigned short* act, int act_cs,
                    int act_co, hipStream_t s) {
  const int sz = n->lsize[l], cout = n->cout[l];
  n->actp[l] = act;   // where the backward finds the relu mask
  n->acs[l] = act_cs;
  n->aco[l] = act_co;
  return launch_conv<false>(n, sz, cout, in, in_cs, in_co, n->cinp[l], n->wf[l], cout, n->cinp[l],
                            n->P + n->boff[l], nullptr, act, act_cs, act_co, s);
}

// backward through relu + conv l: g (float view of the layer output gradient)
// -> bias/weight gradients and, if gx != null, the input gradient gx[V][cin]
static int conv_bwd(lag_cnn n, int l, const float* g, int gcs, int goff, const unsigned short* in, int in_cs,
                    int in_co, float* gx, hipStream_t s) {
  const int sz = n->lsize[l], cout = n->cout[l], cin = n->cinp[l];
  const long long V = (long long)sz * sz * sz;
  const int nb = std::min(ceil_div(V * cout / 8, 256), 1024);
  hipLaunchKernelGGL(k_relu_back, dim3(nb), dim3(256), 0, s, g, gcs, goff, n->actp[l], n->acs[l], n->aco[l], cout,
                     (int)V, n->gbl[l], n->bpl[l]);
  LAG_LAUNCH_CHECK();
  // weight gradient on the side stream, after the relu backward; the input
  // gradient below goes on on the caller's stream meanwhile
  LAG_HIP(hipEventRecord(n->fork[l], s));
  LAG_HIP(hipStreamWaitEvent(n->side, n->fork[l], 0));
  const hipStream_t ws = n->side;
  // weight gradient: partials per voxel range, then their fixed-order sum into G
  const ConvTile T = conv_tile(sz);
  const int NV = 1 << (T.lx + T.ly + T.lz);
  const int tpr = wgrad_per_range(sz, cin), nr = wgrad_ranges(sz, cin);
  const size_t lds = sizeof(unsigned short) * ((size_t)cout * NV +
                                               16 * 16 * (size_t)(((1 << T.ly) + 2) * ((1 << T.lz) + 2)));
  const dim3 wg(nr, cin / 16);
  switch (cout / 16) {
    case 1: hipLaunchKernelGGL(k_conv_wgrad<1>, wg, dim3(256), lds, ws, in, in_cs, in_co, sz, T, n->gbl[l], cout, tpr, cin, n->wpart); break;
    case 2: hipLaunchKernelGGL(k_conv_wgrad<2>, wg, dim3(256), lds, ws, in, in_cs, in_co, sz, T, n->gbl[l], cout, tpr, cin, n->wpart); break;
    default: hipLaunchKernelGGL(k_conv_wgrad<4>, wg, dim3(256), lds, ws, in, in_cs, in_co, sz, T, n->gbl[l], cout, tpr, cin, n->wpart); break;
  }
  LAG_LAUNCH_CHECK();
  // weight and bias gradients: fixed-order sums of the partials
  const long long nout = 27LL * n->cin[l] * cout + cout;
  if (ceil_div(nout, 32) >= 1024)
    hipLaunchKernelGGL(k_wgrad_reduce<32>, dim3(ceil_div(nout, 32)), dim3(256), 0, ws, n->wpart, nr, n->cin[l], cin,
                       cout, n->G + n->woff[l], n->bpl[l], nb, n->G + n->boff[l]);
  else
    hipLaunchKernelGGL(k_wgrad_reduce<8>, dim3(ceil_div(nout, 8)), dim3(256), 0, ws, n->wpart, nr, n->cin[l], cin,
                       cout, n->G + n->woff[l], n->bpl[l], nb, n->G + n->boff[l]);
  LAG_LAUNCH_CHECK();
  if (gx) {
    const int rc = launch_conv<true>(n, sz, cin, n->gbl[l], cout, 0, cout, n->wb[l], cin, cout, nullptr, gx, nullptr, 0,
                                     0, s);
    if (rc) return rc;
  }
  return LAG_OK;
}

static int refresh_weights(lag_cnn n, hipStream_t s) {
  WcopyArgs A;
  A.start[0] = 0;
  for (int l = 0; l < HEAD; ++l) {
    A.w[l] = n->P + n->woff[l];
    A.wf[l] = n->wf[l];
    A.wb[l] = n->wb[l];
    A.cin[l] = n->cin[l];
    A.cinp[l] = n->cinp[l];
    A.cout[l] = n->cout[l];
    A.start[l + 1] = A.start[l] + (long long)kTaps * n->cinp[l] * n->cout[l];
  }
  hipLaunchKernelGGL(k_wcopy, dim3(ceil_div(A.start[HEAD], 256)), dim3(256), 0, s, A);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

static int forward_impl(lag_cnn n, const float* T, const float* R, float* v, hipStream_t s, bool train = false) {
  const int S = n->S, c0 = n->c[0], c1 = n->c[1], c2 = n->c[2], c3 = n->c[3];
  const long long V0 = (long long)S * S * S, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  int rc;
  if (n->wdirty) {  // bf16 copies of the weights, once per change of the master weights
    if ((rc = refresh_weights(n, s))) return rc;
    n->wdirty = false;
  }
  if (train) {  // the first layer's weight gradient reads the stored input
    hipLaunchKernelGGL(k_input, dim3(ceil_div(V0, 256)), dim3(256), 0, s, T, R, n->cfg.in_scale, (int)V0, n->x0);
    LAG_LAUNCH_CHECK();
  }
  const int w0 = c1 + c0, w1 = c2 + c1, w2 = c3 + c2;
  // encoder; enc0/enc1/enc2 are written into their concatenation slices
  // first layer (2 input channels) on the vector ALUs
  n->actp[E0A] = n->a[E0A];
  n->acs[E0A] = c0;
  n->aco[E0A] = 0;
  hipLaunchKernelGGL(k_conv_in2, dim3(conv_tiles(S)), dim3(256), 0, s, T, R, n->cfg.in_scale, S, n->wf[E0A],
                     n->cinp[E0A], c0, n->P + n->boff[E0A], n->a[E0A], c0, 0);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, E0B, n->a[E0A], c0, 0, n->cat0, w0, c1, s))) return rc;
  hipLaunchKernelGGL(k_pool, dim3(ceil_div(V1 * c0, 256)), dim3(256), 0, s, n->cat0, w0, c1, c0, S, n->p0);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, E1A, n->p0, c0, 0, n->a[E1A], c1, 0, s))) return rc;
  if ((rc = conv_fwd(n, E1B, n->a[E1A], c1, 0, n->cat1, w1, c2, s))) return rc;
  hipLaunchKernelGGL(k_pool, dim3(ceil_div(V2 * c1, 256)), dim3(256), 0, s, n->cat1, w1, c2, c1, S / 2, n->p1);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, E2A, n->p1, c1, 0, n->a[E2A], c2, 0, s))) return rc;
  if ((rc = conv_fwd(n, E2B, n->a[E2A], c2, 0, n->cat2, w2, c3, s))) return rc;
  hipLaunchKernelGGL(k_pool, dim3(ceil_div(V3 * c2, 256)), dim3(256), 0, s, n->cat2, w2, c3, c2, S / 4, n->p2);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, MA, n->p2, c2, 0, n->a[MA], c3, 0, s))) return rc;
  if ((rc = conv_fwd(n, MB, n->a[MA], c3, 0, n->a[MB], c3, 0, s))) return rc;
  // decoder
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V2 * c3 / 8, 256)), dim3(256), 0, s, n->a[MB], c3, S / 4, n->cat2, w2);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, D2, n->cat2, w2, 0, n->a[D2], c2, 0, s))) return rc;
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V1 * c2 / 8, 256)), dim3(256), 0, s, n->a[D2], c2, S / 2, n->cat1, w1);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, D1, n->cat1, w1, 0, n->a[D1], c1, 0, s))) return rc;
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V0 * c1 / 8, 256)), dim3(256), 0, s, n->a[D1], c1, S, n->cat0, w0);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, D0, n->cat0, w0, 0, n->a[D0], c0, 0, s))) return rc;
  hipLaunchKernelGGL(k_head_fwd, dim3(ceil_div(V0, 256)), dim3(256), 0, s, n->a[D0], c0, (int)V0,
                     n->P + n->woff[HEAD], n->P + n->boff[HEAD], n->cfg.out_scale, v);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

extern "C" {

int lag_cnn_forward(lag_cnn n, const float* T, const float* R, float* v, void* stream) {
  if (!n || !T || !R || !v) return LAG_EINVAL;
  return forward_impl(n, T, R, v, (hipStream_t)stream);
}

int lag_cnn_backward(lag_cnn n, const float* T, const float* R, const float* target, float* v, double* loss,
                     void* stream) {
  if (!n || !T || !R || !target || !v || !loss) return LAG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = forward_impl(n, T, R, v, s, true);
  if (rc) return rc;
  const int S = n->S, c0 = n->c[0], c1 = n->c[1], c2 = n->c[2], c3 = n->c[3];
  const long long V0 = (long long)S * S * S, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  const int w0 = c1 + c0, w1 = c2 + c1, w2 = c3 + c2;
  if ((rc = launch_fill(n->G, n->nparams, 0.f, s))) return rc;
  // loss and its gradient
  const long long nv = 3 * V0;
  const float gscale = n->cfg.out_scale / (float)nv;
  // gout = d loss / d (head's linear output) = out_scale (v - target) / n
  hipLaunchKernelGGL(k_mse, dim3(1024), dim3(256), 0, s, v, target, nv, gscale, n->gout, n->part);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, n->part, 1024, 0.5 / (double)nv, loss);
  LAG_LAUNCH_CHECK();
  float* gd0 = n->gbuf[0];
  const int hb = std::min(ceil_div(V0, 256), 256);   // head blocks (grid-stride)
  hipLaunchKernelGGL(k_head_bwd, dim3(hb), dim3(256), 0, s, n->a[D0], c0, (int)V0, n->P + n->woff[HEAD], n->gout,
                     gd0, n->bpart);
  LAG_LAUNCH_CHECK();
  // gWh[c][3] and gbh[3] are contiguous in G
  hipLaunchKernelGGL(k_rows_reduce, dim3(3 * c0 + 3), dim3(256), 0, s, n->bpart, hb, 3 * c0 + 3,
                     n->G + n->woff[HEAD]);
  LAG_LAUNCH_CHECK();
  // decoder
  if ((rc = conv_bwd(n, D0, gd0, c0, 0, n->cat0, w0, 0, n->gcat[0], s))) return rc;
  hipLaunchKernelGGL(k_up_back, dim3(ceil_div(V1 * c1, 256)), dim3(256), 0, s, n->gcat[0], w0, c1, S, n->gbuf[1]);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_bwd(n, D1, n->gbuf[1], c1, 0, n->cat1, w1, 0, n->gcat[1], s))) return rc;
  hipLaunchKernelGGL(k_up_back, dim3(ceil_div(V2 * c2, 256)), dim3(256), 0, s, n->gcat[1], w1, c2, S / 2, n->gbuf[2]);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_bwd(n, D2, n->gbuf[2], c2, 0, n->cat2, w2, 0, n->gcat[2], s))) return rc;
  hipLaunchKernelGGL(k_up_back, dim3(ceil_div(V3 * c3, 256)), dim3(256), 0, s, n->gcat[2], w2, c3, S / 4, n->gbuf[3]);
  LAG_LAUNCH_CHECK();
  // bottom
  if ((rc = conv_bwd(n, MB, n->gbuf[3], c3, 0, n->a[MA], c3, 0, n->gtmp[3], s))) return rc;
  if ((rc = conv_bwd(n, MA, n->gtmp[3], c3, 0, n->p2, c2, 0, n->gbuf[3], s))) return rc;
  // g(enc2) = slice of g(cat2) + pool adjoint of g(p2)
  hipLaunchKernelGGL(k_pool_back, dim3(ceil_div(V2 * c2, 256)), dim3(256), 0, s, n->gbuf[3], c2, S / 4,
                     n->gcat[2], w2, c3);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_bwd(n, E2B, n->gcat[2], w2, c3, n->a[E2A], c2, 0, n->gtmp[2], s))) return rc;
  if ((rc = conv_bwd(n, E2A, n->gtmp[2], c2, 0, n->p1, c1, 0, n->gbuf[2], s))) return rc;
  hipLaunchKernelGGL(k_pool_back, dim3(ceil_div(V1 * c1, 256)), dim3(256), 0, s, n->gbuf[2], c1, S / 2,
                     n->gcat[1], w1, c2);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_bwd(n, E1B, n->gcat[1], w1, c2, n->a[E1A], c1, 0, n->gtmp[1], s))) return rc;
  if ((rc = conv_bwd(n, E1A, n->gtmp[1], c1, 0, n->p0, c0, 0, n->gbuf[1], s))) return rc;
  hipLaunchKernelGGL(k_pool_back, dim3(ceil_div(V0 * c0, 256)), dim3(256), 0, s, n->gbuf[1], c0, S, n->gcat[0],
                     w0, c1);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_bwd(n, E0B, n->gcat[0], w0, c1, n->a[E0A], c0, 0, n->gtmp[0], s))) return rc;
  if ((rc = conv_bwd(n, E0A, n->gtmp[0], c0, 0, n->x0, 16, 0, nullptr, s))) return rc;
  // the weight gradients are complete before the caller's stream goes on
  LAG_HIP(hipEventRecord(n->join, n->side));
  LAG_HIP(hipStreamWaitEvent(s, n->join, 0));
  return LAG_OK;
}

int lag_cnn_adam_step(lag_cnn n, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!n || !(lr >= 0.f)) return LAG_EINVAL;
  n->adam_t += 1;
  const float c1 = 1.f - powf(beta1, (float)n->adam_t), c2 = 1.f - powf(beta2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(ceil_div(n->nparams, 256)), dim3(256), 0, (hipStream_t)stream, n->P, n->G, n->M1,
                     n->M2, n->nparams, lr, beta1, beta2, eps, c1, c2);
  LAG_LAUNCH_CHECK();
  n->wdirty = true;
  return LAG_OK;
}

}  // extern "C"
