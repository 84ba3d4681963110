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
// segment), pre-activations and gradients float32, master weights float32
// with bfloat16 copies for the matrix cores.
//
// Every 3x3x3 convolution is an implicit GEMM on the MFMA units
// (v_mfma_f32_16x16x16_bf16: A 16x16 in lanes as A[l%16][4(l/16)+j],
// B as B[4(l/16)+j][l%16], C as C[4(l/16)+j][l%16], j = 0..3):
//   forward      out[v][co]  = sum_{t,ci} x[v+o_t][ci] W[t][ci][co]     (M=v,  N=co, K=t,ci)
//   backward-in  gx[v][ci]   = sum_{t,co} g[v-o_t][co] W[t][ci][co]     (M=v,  N=ci, K=t,co)
//   backward-W   gW[t][ci][co] = sum_v x[v+o_t][ci] g[v][co]            (M=ci, N=co, K=v)
// Concatenation is never materialised by a copy: producers write into
// channel slices of the concatenated buffer ("views": base, channel stride,
// channel offset).

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <random>
#include <vector>

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
// forward convolution: one wave computes 64 voxels x (16*NT) output channels
template <int NT>
__global__ void __launch_bounds__(256) k_conv_fwd(const unsigned short* __restrict__ in, int in_cs, int in_co,
                                                  int cin, int s, const unsigned short* __restrict__ wf,
                                                  const float* __restrict__ bias, int cout,
                                                  float* __restrict__ pre, unsigned short* __restrict__ act,
                                                  int act_cs, int act_co, int co_base) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int V = s * s * s;
  const int v0 = wave * 64;
  if (v0 >= V) return;
  const int r = lane & 15, q = lane >> 4;
  f32x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    int nb[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) nb[mt] = nbr(v0 + 16 * mt + r, s, dz, dy, dx);
    for (int c0 = 0; c0 < cin; c0 += 16) {
      i16x4 a[4], b[NT];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        a[mt] = *(const i16x4*)(in + (long long)nb[mt] * in_cs + in_co + c0 + 4 * q);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = *(const i16x4*)(wf + ((long long)t * cout + co_base + 16 * nt + r) * cin + c0 + 4 * q);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int v = v0 + 16 * mt + 4 * q + j;
        const int co = co_base + 16 * nt + r;
        const float val = acc[mt][nt][j] + bias[co];
        pre[(long long)v * cout + co] = val;
        act[(long long)v * act_cs + act_co + co] = f2bf(fmaxf(val, 0.f));
      }
}

// backward to the input: gx[v][ci] = sum_{t,co} g[v - o_t][co] W[t][ci][co]
template <int NT>
__global__ void __launch_bounds__(256) k_conv_bwd_data(const unsigned short* __restrict__ g, int cout, int s,
                                                       const unsigned short* __restrict__ wb, int cin,
                                                       float* __restrict__ gx, int ci_base) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int V = s * s * s;
  const int v0 = wave * 64;
  if (v0 >= V) return;
  const int r = lane & 15, q = lane >> 4;
  f32x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    int nb[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) nb[mt] = nbr(v0 + 16 * mt + r, s, -dz, -dy, -dx);
    for (int c0 = 0; c0 < cout; c0 += 16) {
      i16x4 a[4], b[NT];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) a[mt] = *(const i16x4*)(g + (long long)nb[mt] * cout + c0 + 4 * q);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = *(const i16x4*)(wb + ((long long)t * cin + ci_base + 16 * nt + r) * cout + c0 + 4 * q);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int v = v0 + 16 * mt + 4 * q + j;
        gx[(long long)v * cin + ci_base + 16 * nt + r] = acc[mt][nt][j];
      }
}

// weight gradient: gW[t][ci][co] += sum over a voxel range of x[v+o_t][ci] g[v][co]
// grid: (voxel ranges, 27 taps, ci tiles * co tiles); one wave per block
__global__ void __launch_bounds__(64) k_conv_bwd_weight(const unsigned short* __restrict__ in, int in_cs, int in_co,
                                                        int cin, int cin_store, int s,
                                                        const unsigned short* __restrict__ g, int cout, int range,
                                                        float* __restrict__ gw) {
  const int lane = threadIdx.x;
  const int r = lane & 15, q = lane >> 4;
  const int t = blockIdx.y;
  const int nco = cout / 16;
  const int ct = blockIdx.z / nco, ot = blockIdx.z % nco;
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  const int V = s * s * s;
  const int vb = blockIdx.x * range, ve = min(V, vb + range);
  const int ci = 16 * ct + r, co = 16 * ot + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = vb; k0 < ve; k0 += 16) {
    i16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int v = k0 + 4 * q + j;   // ve - vb is a multiple of 16
      a[j] = (short)in[(long long)nbr(v, s, dz, dy, dx) * in_cs + in_co + ci];
      b[j] = (short)g[(long long)v * cout + co];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cij = 16 * ct + 4 * q + j;   // padded input channels are not stored
    if (cij < cin_store) unsafeAtomicAdd(&gw[((long long)t * cin_store + cij) * cout + 16 * ot + r], acc[j]);
  }
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

// pool: out (size s/2) = mean of the 2x2x2 children of `in` (size s)
__global__ void k_pool(const unsigned short* __restrict__ in, int in_cs, int in_co, int c, int s,
                       unsigned short* __restrict__ out) {
  const int h = s / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)h * h * h * c) return;
  const int ch = (int)(i % c);
  const int v = (int)(i / c);
  const int x = v % h, y = (v / h) % h, z = v / (h * h);
  float sum = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int fv = ((2 * z + (o >> 2)) * s + 2 * y + ((o >> 1) & 1)) * s + 2 * x + (o & 1);
    sum += bf2f(in[(long long)fv * in_cs + in_co + ch]);
  }
  out[i] = f2bf(0.125f * sum);
}

// up: out view (size s) channel slice [0, c) = copy of the parent in `in` (size s/2)
__global__ void k_up(const unsigned short* __restrict__ in, int c, int s, unsigned short* __restrict__ out,
                     int out_cs) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)s * s * s * c) return;
  const int ch = (int)(i % c);
  const int v = (int)(i / c);
  const int x = v % s, y = (v / s) % s, z = v / (s * s);
  const int h = s / 2;
  const int pv = ((z >> 1) * h + (y >> 1)) * h + (x >> 1);
  out[(long long)v * out_cs + ch] = in[(long long)pv * c + ch];
}

// gpre = g (float, view of width gcs at offset goff) masked by pre > 0;
// writes the bf16 copy and accumulates the bias gradient
__global__ void k_relu_back(const float* __restrict__ g, int gcs, int goff, const float* __restrict__ pre, int c,
                            int V, unsigned short* __restrict__ gb, float* __restrict__ gbias) {
  __shared__ float sh[256];
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float val = 0.f;
  int ch = 0;
  if (i < (long long)V * c) {
    ch = (int)(i % c);
    const long long v = i / c;
    val = pre[i] > 0.f ? g[v * gcs + goff + ch] : 0.f;
    gb[i] = f2bf(val);
  }
  // block partial sums per channel (c divides 256 for c in {16, 32, 64})
  sh[threadIdx.x] = val;
  __syncthreads();
  if ((int)threadIdx.x < c) {
    float s = 0.f;
    for (int k = threadIdx.x; k < 256; k += c) s += sh[k];
    unsafeAtomicAdd(&gbias[threadIdx.x], s);
  }
}

// g (size s/2, c channels) += pool-adjoint of gf (size s view): gf / 8 summed? No:
// the gradient of pool at the children is parent / 8 -> add to a full-size buffer
__global__ void k_pool_back(const float* __restrict__ gp, int c, int s, float* __restrict__ gf, int gf_cs,
                            int gf_co) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)s * s * s * c) return;
  const int ch = (int)(i % c);
  const int v = (int)(i / c);
  const int x = v % s, y = (v / s) % s, z = v / (s * s);
  const int h = s / 2;
  const int pv = ((z >> 1) * h + (y >> 1)) * h + (x >> 1);
  gf[(long long)v * gf_cs + gf_co + ch] += 0.125f * gp[(long long)pv * c + ch];
}

// gp (size s/2, c) = sum over children of the channel slice [0, c) of g (size s, width gcs)
__global__ void k_up_back(const float* __restrict__ g, int gcs, int c, int s, float* __restrict__ gp) {
  const int h = s / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)h * h * h * c) return;
  const int ch = (int)(i % c);
  const int v = (int)(i / c);
  const int x = v % h, y = (v / h) % h, z = v / (h * h);
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
  for (int ch = 0; ch < c; ++ch) {
    float a = bf2f(d0[(long long)v * c + ch]);
    o0 = fmaf(a, wh[ch * 3 + 0], o0);
    o1 = fmaf(a, wh[ch * 3 + 1], o1);
    o2 = fmaf(a, wh[ch * 3 + 2], o2);
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

__global__ void k_mse_final(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = scale * s;
  }
}

// head backward: gd0[vox][c] = sum_k go[k][vox] Wh[c][k]; gWh, gbh by block partial sums
__global__ void k_head_bwd(const unsigned short* __restrict__ d0, int c, int V, const float* __restrict__ wh,
                           const float* __restrict__ go, float* __restrict__ gd0, float* __restrict__ gwh,
                           float* __restrict__ gbh) {
  __shared__ float sh[256];
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (v < V) {
    g0 = go[v];
    g1 = go[V + v];
    g2 = go[2 * V + v];
    for (int ch = 0; ch < c; ++ch)
      gd0[(long long)v * c + ch] = g0 * wh[ch * 3] + g1 * wh[ch * 3 + 1] + g2 * wh[ch * 3 + 2];
  }
  // weight gradient: gwh[ch][k] += sum_v d0[v][ch] g_k[v]
  for (int ch = 0; ch < c; ++ch) {
    float a = v < V ? bf2f(d0[(long long)v * c + ch]) : 0.f;
    for (int k = 0; k < 3; ++k) {
      sh[threadIdx.x] = a * (k == 0 ? g0 : (k == 1 ? g1 : g2));
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) unsafeAtomicAdd(&gwh[ch * 3 + k], sh[0]);
      __syncthreads();
    }
  }
  for (int k = 0; k < 3; ++k) {
    sh[threadIdx.x] = k == 0 ? g0 : (k == 1 ? g1 : g2);
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(&gbh[k], sh[0]);
    __syncthreads();
  }
}

// bf16 weight copies: wf[t][co][ci_pad], wb[t][ci_pad][co] from w[t][ci][co]
__global__ void k_wcopy(const float* __restrict__ w, int taps, int cin, int cin_pad, int cout,
                        unsigned short* __restrict__ wf, unsigned short* __restrict__ wb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)taps * cin_pad * cout) return;
  const int co = (int)(i % cout);
  const int ci = (int)((i / cout) % cin_pad);
  const int t = (int)(i / ((long long)cout * cin_pad));
  const unsigned short val = ci < cin ? f2bf(w[((long long)t * cin + ci) * cout + co]) : (unsigned short)0;
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
  // activations (bf16) and pre-activations (fp32)
  unsigned short* x0 = nullptr;      // S^3 x 16
  unsigned short* a[kLayers] = {nullptr};
  float* pre[kLayers] = {nullptr};
  unsigned short *p0 = nullptr, *p1 = nullptr, *p2 = nullptr;   // pooled
  unsigned short *cat2 = nullptr, *cat1 = nullptr, *cat0 = nullptr;
  // gradients
  float* gbuf[4] = {nullptr};        // scratch per level (largest widths)
  float* gcat[3] = {nullptr};        // g of cat0 / cat1 / cat2
  float* gtmp[4] = {nullptr};
  unsigned short* gb16 = nullptr;    // bf16 gradient of a pre-activation (largest)
  float* gout = nullptr;             // 3 x S^3
  double* part = nullptr;
  int adam_t = 0;
};

static int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

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
                  n->gb16, n->gout, n->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int l = 0; l < kLayers; ++l) {
    if (n->wf[l]) (void)hipFree(n->wf[l]);
    if (n->wb[l]) (void)hipFree(n->wb[l]);
    if (n->a[l]) (void)hipFree(n->a[l]);
    if (n->pre[l]) (void)hipFree(n->pre[l]);
  }
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
  for (int l = 0; l < HEAD; ++l) {
    const size_t wn = (size_t)27 * n->cinp[l] * n->cout[l];
    CNN_ALLOC(n->wf[l], 2 * wn);
    CNN_ALLOC(n->wb[l], 2 * wn);
    const long long V = (long long)sz[l] * sz[l] * sz[l];
    CNN_ALLOC(n->pre[l], sizeof(float) * V * n->cout[l]);
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
  CNN_ALLOC(n->gb16, 2 * V0 * 64);
  CNN_ALLOC(n->gout, sizeof(float) * 3 * V0);
  CNN_ALLOC(n->part, sizeof(double) * 1024);
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
  LAG_HIP(hipMemcpy(host, n->P, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  return LAG_OK;
}

int lag_cnn_set_params(lag_cnn n, const float* host) {
  if (!n || !host) return LAG_EINVAL;
  LAG_HIP(hipMemcpy(n->P, host, sizeof(float) * n->nparams, hipMemcpyHostToDevice));
  n->adam_t = 0;
  LAG_HIP(hipMemset(n->M1, 0, sizeof(float) * n->nparams));
  LAG_HIP(hipMemset(n->M2, 0, sizeof(float) * n->nparams));
  return LAG_OK;
}

int lag_cnn_get_grads(lag_cnn n, float* host) {
  if (!n || !host) return LAG_EINVAL;
  LAG_HIP(hipMemcpy(host, n->G, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  return LAG_OK;
}

}  // extern "C"

// ---- launch helpers ----------------------------------------------------------

static int conv_fwd(lag_cnn n, int l, const unsigned short* in, int in_cs, int in_co, unsigned short* act, int act_cs,
                    int act_co, hipStream_t s) {
  const int sz = n->lsize[l], cout = n->cout[l];
  const long long V = (long long)sz * sz * sz;
  const int waves = ceil_div(V, 64);
  const dim3 grid(ceil_div(waves, 4));
  const float* bias = n->P + n->boff[l];
  // output channels in groups of up to 64 (NT = 4 tiles of 16)
  for (int cb = 0; cb < cout; cb += 64) {
    const int nt = std::min(4, (cout - cb) / 16);
    switch (nt) {
      case 1: hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), 0, s, in, in_cs, in_co, n->cinp[l], sz, n->wf[l], bias, cout, n->pre[l], act, act_cs, act_co, cb); break;
      case 2: hipLaunchKernelGGL(k_conv_fwd<2>, grid, dim3(256), 0, s, in, in_cs, in_co, n->cinp[l], sz, n->wf[l], bias, cout, n->pre[l], act, act_cs, act_co, cb); break;
      case 3: hipLaunchKernelGGL(k_conv_fwd<3>, grid, dim3(256), 0, s, in, in_cs, in_co, n->cinp[l], sz, n->wf[l], bias, cout, n->pre[l], act, act_cs, act_co, cb); break;
      default: hipLaunchKernelGGL(k_conv_fwd<4>, grid, dim3(256), 0, s, in, in_cs, in_co, n->cinp[l], sz, n->wf[l], bias, cout, n->pre[l], act, act_cs, act_co, cb); break;
    }
    LAG_LAUNCH_CHECK();
  }
  return LAG_OK;
}

// backward through relu + conv l: g (float view of the layer output gradient)
// -> bias/weight gradients and, if gx != null, the input gradient gx[V][cin]
static int conv_bwd(lag_cnn n, int l, const float* g, int gcs, int goff, const unsigned short* in, int in_cs,
                    int in_co, float* gx, hipStream_t s) {
  const int sz = n->lsize[l], cout = n->cout[l], cin = n->cinp[l];
  const long long V = (long long)sz * sz * sz;
  hipLaunchKernelGGL(k_relu_back, dim3(ceil_div(V * cout, 256)), dim3(256), 0, s, g, gcs, goff, n->pre[l], cout,
                     (int)V, n->gb16, n->G + n->boff[l]);
  LAG_LAUNCH_CHECK();
  // weight gradient (accumulated into G, which the caller zeroes)
  const int range = V >= 4096 ? 4096 : (int)V;
  dim3 grid(ceil_div(V, range), 27, (cin / 16) * (cout / 16));
  hipLaunchKernelGGL(k_conv_bwd_weight, grid, dim3(64), 0, s, in, in_cs, in_co, cin, n->cin[l], sz, n->gb16, cout,
                     range, n->G + n->woff[l]);
  LAG_LAUNCH_CHECK();
  if (gx) {
    const int waves = ceil_div(V, 64);
    const dim3 g2(ceil_div(waves, 4));
    for (int cb = 0; cb < cin; cb += 64) {
      const int nt = std::min(4, (cin - cb) / 16);
      switch (nt) {
        case 1: hipLaunchKernelGGL(k_conv_bwd_data<1>, g2, dim3(256), 0, s, n->gb16, cout, sz, n->wb[l], cin, gx, cb); break;
        case 2: hipLaunchKernelGGL(k_conv_bwd_data<2>, g2, dim3(256), 0, s, n->gb16, cout, sz, n->wb[l], cin, gx, cb); break;
        case 3: hipLaunchKernelGGL(k_conv_bwd_data<3>, g2, dim3(256), 0, s, n->gb16, cout, sz, n->wb[l], cin, gx, cb); break;
        default: hipLaunchKernelGGL(k_conv_bwd_data<4>, g2, dim3(256), 0, s, n->gb16, cout, sz, n->wb[l], cin, gx, cb); break;
      }
      LAG_LAUNCH_CHECK();
    }
  }
  return LAG_OK;
}

static int refresh_weights(lag_cnn n, hipStream_t s) {
  for (int l = 0; l < HEAD; ++l) {
    const long long cnt = 27LL * n->cinp[l] * n->cout[l];
    hipLaunchKernelGGL(k_wcopy, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, n->P + n->woff[l], 27, n->cin[l],
                       n->cinp[l], n->cout[l], n->wf[l], n->wb[l]);
    LAG_LAUNCH_CHECK();
  }
  return LAG_OK;
}

static int forward_impl(lag_cnn n, const float* T, const float* R, float* v, hipStream_t s) {
  const int S = n->S, c0 = n->c[0], c1 = n->c[1], c2 = n->c[2], c3 = n->c[3];
  const long long V0 = (long long)S * S * S, V1 = V0 / 8, V2 = V1 / 8, V3 = V2 / 8;
  int rc;
  if ((rc = refresh_weights(n, s))) return rc;
  hipLaunchKernelGGL(k_input, dim3(ceil_div(V0, 256)), dim3(256), 0, s, T, R, n->cfg.in_scale, (int)V0, n->x0);
  LAG_LAUNCH_CHECK();
  const int w0 = c1 + c0, w1 = c2 + c1, w2 = c3 + c2;
  // encoder; enc0/enc1/enc2 are written into their concatenation slices
  if ((rc = conv_fwd(n, E0A, n->x0, 16, 0, n->a[E0A], c0, 0, s))) return rc;
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
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V2 * c3, 256)), dim3(256), 0, s, n->a[MB], c3, S / 4, n->cat2, w2);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, D2, n->cat2, w2, 0, n->a[D2], c2, 0, s))) return rc;
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V1 * c2, 256)), dim3(256), 0, s, n->a[D2], c2, S / 2, n->cat1, w1);
  LAG_LAUNCH_CHECK();
  if ((rc = conv_fwd(n, D1, n->cat1, w1, 0, n->a[D1], c1, 0, s))) return rc;
  hipLaunchKernelGGL(k_up, dim3(ceil_div(V0 * c1, 256)), dim3(256), 0, s, n->a[D1], c1, S, n->cat0, w0);
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
  int rc = forward_impl(n, T, R, v, s);
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
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, n->part, 1024, 0.5 / (double)nv, loss);
  LAG_LAUNCH_CHECK();
  float* gd0 = n->gbuf[0];
  hipLaunchKernelGGL(k_head_bwd, dim3(ceil_div(V0, 256)), dim3(256), 0, s, n->a[D0], c0, (int)V0,
                     n->P + n->woff[HEAD], n->gout, gd0, n->G + n->woff[HEAD], n->G + n->boff[HEAD]);
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
  return LAG_OK;
}

int lag_cnn_adam_step(lag_cnn n, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!n || !(lr >= 0.f)) return LAG_EINVAL;
  n->adam_t += 1;
  const float c1 = 1.f - powf(beta1, (float)n->adam_t), c2 = 1.f - powf(beta2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(ceil_div(n->nparams, 256)), dim3(256), 0, (hipStream_t)stream, n->P, n->G, n->M1,
                     n->M2, n->nparams, lr, beta1, beta2, eps, c1, c2);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

}  // extern "C"
