// Regulariser stencil and spectral preconditioner (gfx950).
//
// Regulariser (Sec. 2.1; derivative and Hessian term in Sec. 3.2): per time
// node j and component c, out = s_j A p_{j,c} (+ gamma p) with
// A = -Laplace_h (diffusion) or Laplace_h^2 (curvature) on the periodic
// velocity grid and s_j a per-node scale (alpha h_v^d w_j).  Differences are
// formed before scaling so smooth fields lose little to cancellation.
//
// Preconditioner (Sec. 3.2, PCG paragraph): the regulariser block of the
// Gauss-Newton matrix is circulant on the periodic grid, so it is inverted
// in Fourier space: z = F^-1[F(r) / mu(k)], mu(k) = s_j lambda_A(k) + gamma.
// The transform is a hand-written Stockham autosort FFT of radix 4/2/3/5
// performed line by line in LDS; r is real and mu(k) real and even, so only
// the half spectrum along x is formed (two real rows per complex line), and
// the forward and inverse transforms along the last axis are fused with the
// division.  Twiddles and eigenvalue tables are computed on the host in
// double precision at plan creation.

#include <math.h>

#include <vector>

#include "lag_internal.hpp"

namespace lag {

// ---------------------------------------------------------------------------
// regulariser

template <int D, bool CURV>
__global__ void __launch_bounds__(kBlock) k_reg(Geo g, const float* __restrict__ p, float* __restrict__ out,
                                                const float* __restrict__ scale, float gamma, int accumulate,
                                                float ih2x, float ih2y, float ih2z) {
  if (halted(g.halt)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nv * g.nodes * D) return;
  const float ih2[3] = {ih2x, ih2y, ih2z};
  float val = reg_value<D, CURV>(g, p, scale, gamma, ih2, i);
  if (accumulate) val += out[i];
  out[i] = val;
}

RegTail reg_tail(lag_plan P, const float* p, int with_gamma, float extra_scale, double* part) {
  RegTail r;
  r.p = p;
  r.scale = P->reg_scale + (extra_scale != 0.f ? 0 : P->geo.nodes);
  r.gamma = with_gamma ? (float)P->prob.gamma : 0.f;
  for (int a = 0; a < 3; ++a) {
    double h = P->prob.extent[a] / P->prob.vel_m[a];
    r.ih2[a] = (float)(1.0 / (h * h));
  }
  r.curv = P->prob.reg == LAG_CURVATURE;
  r.part = part;
  return r;
}

int launch_reg(lag_plan P, const float* p, float* out, int accumulate, int with_gamma, float extra_scale,
               hipStream_t s) {
  // extra_scale selects the table: 1 -> alpha h_v^d w_j, 0 -> h_v^d w_j
  const float* scale = P->reg_scale + (extra_scale != 0.f ? 0 : P->geo.nodes);
  const float gamma = with_gamma ? (float)P->prob.gamma : 0.f;
  float ih2[3];
  for (int a = 0; a < 3; ++a) {
    double h = P->prob.extent[a] / P->prob.vel_m[a];
    ih2[a] = (float)(1.0 / (h * h));
  }
  const long long tot = P->geo.nv * P->fields;
  unsigned grid = (unsigned)((tot + kBlock - 1) / kBlock);
  const bool curv = P->prob.reg == LAG_CURVATURE;
  if (P->geo.dim == 3) {
    if (curv)
      hipLaunchKernelGGL((k_reg<3, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, p, out, scale, gamma, accumulate,
                         ih2[0], ih2[1], ih2[2]);
    else
      hipLaunchKernelGGL((k_reg<3, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, p, out, scale, gamma, accumulate,
                         ih2[0], ih2[1], ih2[2]);
  } else {
    if (curv)
      hipLaunchKernelGGL((k_reg<2, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, p, out, scale, gamma, accumulate,
                         ih2[0], ih2[1], ih2[2]);
    else
      hipLaunchKernelGGL((k_reg<2, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, p, out, scale, gamma, accumulate,
                         ih2[0], ih2[1], ih2[2]);
  }
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// ---------------------------------------------------------------------------
// FFT

struct FftLine {
  int n;            // line length
  int nrad;         // number of radix stages
  int rad[16];      // radices in application order
  const float2* tw; // tw[q] = exp(-2 pi i q / n)
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Quotient by a divisor that is fixed for the kernel, for the per-element
// index loops (a runtime integer division costs tens of instructions).  With
// m = floor((2^32 - 1) / d) + 1, m d = 2^32 + delta with 0 <= delta < d, so
// floor(e m / 2^32) = floor(e / d) whenever e delta < 2^32: every e below
// 2^32 / d (here e < 2^20, d <= 1024).
struct DivBy {
  unsigned d, m;
  __device__ __forceinline__ explicit DivBy(int dd)
      : d((unsigned)dd), m(dd > 1 ? 0xFFFFFFFFu / (unsigned)dd + 1u : 0u) {}
  __device__ __forceinline__ int operator()(int e) const {
    return d > 1 ? (int)__umulhi((unsigned)e, m) : e;
  }
};

// Power-of-two lengths (radices 4 and 2 only): the same Stockham stages as
// lds_fft with every index division a shift and every remainder a mask.  The
// butterflies, twiddles and output positions are those of the general
// routine, so the result is bitwise the same; the runtime divisions of the
// general index arithmetic made a stage about five times as expensive.
template <bool INV>
__device__ float2* lds_fft_pow2(const FftLine& L, const float2* tw, int lines, int ls, float2* b0, float2* b1) {
  const int ln = __ffs(L.n) - 1;  // log2 n
  int lNs = 0;                     // log2 of the finished sub-transform length
  for (int st = 0; st < L.nrad; ++st) {
    const int R = L.rad[st];
    const int lR = R == 4 ? 2 : 1;
    const int lnb = ln - lR;            // n / R butterflies per line
    const int lspan = ln - lNs - lR;    // twiddle stride n / (Ns R)
    const int nbm = (1 << lnb) - 1, nsm = (1 << lNs) - 1;
    for (int b = threadIdx.x; b < (lines << lnb); b += blockDim.x) {
      const int line = b >> lnb, j = b & nbm;
      const float2* src = b0 + line * ls;
      float2* dst = b1 + line * ls;
      const int k = j & nsm;
      float2 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r < R) {
          float2 x = src[j + (r << lnb)];
          float2 t = tw[(r * k) << lspan];
          if (INV) t.y = -t.y;
          v[r] = r ? cmul(x, t) : x;
        }
      }
      float2 w[4];
      if (R == 2) {
        w[0] = make_float2(v[0].x + v[1].x, v[0].y + v[1].y);
        w[1] = make_float2(v[0].x - v[1].x, v[0].y - v[1].y);
      } else {
        float2 a = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        float2 bq = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        float2 c = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        float2 dj = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
        w[0] = make_float2(a.x + c.x, a.y + c.y);
        w[2] = make_float2(a.x - c.x, a.y - c.y);
        w[1] = make_float2(bq.x + dj.x, bq.y + dj.y);
        w[3] = make_float2(bq.x - dj.x, bq.y - dj.y);
      }
      const int d0 = ((j >> lNs) << (lNs + lR)) + k;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < R) dst[d0 + (r << lNs)] = w[r];
    }
    __syncthreads();
    float2* t = b0;
    b0 = b1;
    b1 = t;
    lNs += lR;
  }
  return b0;
}

// In-LDS Stockham FFT of `lines` lines of length n (buffers [lines][ls],
// line stride ls >= n), twiddles tw (the table of L staged in LDS).  Returns
// the buffer holding the result.  INV selects exp(+2 pi i ...).
template <bool INV>
__device__ float2* lds_fft(const FftLine& L, const float2* tw, int lines, int ls, float2* b0, float2* b1) {
  const int n = L.n;
  if ((n & (n - 1)) == 0) return lds_fft_pow2<INV>(L, tw, lines, ls, b0, b1);
  int Ns = 1;
  for (int st = 0; st < L.nrad; ++st) {
    const int R = L.rad[st];
    const int nb = n / R;
    const int span = n / (Ns * R);      // twiddle stride
    const int step = n / R;             // small-DFT root stride
    for (int b = threadIdx.x; b < lines * nb; b += blockDim.x) {
      const int line = b / nb, j = b - (b / nb) * nb;
      const float2* src = b0 + line * ls;
      float2* dst = b1 + line * ls;
      const int k = j % Ns;
      float2 v[5];
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        if (r < R) {
          float2 x = src[j + r * nb];
          float2 t = tw[r * k * span];
          if (INV) t.y = -t.y;
          v[r] = r ? cmul(x, t) : x;
        }
      }
      float2 w[5];
      if (R == 2) {
        w[0] = make_float2(v[0].x + v[1].x, v[0].y + v[1].y);
        w[1] = make_float2(v[0].x - v[1].x, v[0].y - v[1].y);
      } else if (R == 4) {
        float2 a = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        float2 bq = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        float2 c = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        // multiply d by -i (forward) or +i (inverse)
        float2 dj = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
        w[0] = make_float2(a.x + c.x, a.y + c.y);
        w[2] = make_float2(a.x - c.x, a.y - c.y);
        w[1] = make_float2(bq.x + dj.x, bq.y + dj.y);
        w[3] = make_float2(bq.x - dj.x, bq.y - dj.y);
      } else {
        // generic small DFT with roots from the twiddle table
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          if (s < R) {
            float2 acc = v[0];
#pragma unroll
            for (int r = 1; r < 5; ++r) {
              if (r < R) {
                float2 t = tw[((r * s) % R) * step];
                if (INV) t.y = -t.y;
                float2 m = cmul(v[r], t);
                acc.x += m.x;
                acc.y += m.y;
              }
            }
            w[s] = acc;
          }
        }
      }
      const int d0 = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < 5; ++r)
        if (r < R) dst[d0 + r * Ns] = w[r];
    }
    __syncthreads();
    float2* t = b0;
    b0 = b1;
    b1 = t;
    Ns *= R;
  }
  return b0;
}

// Spectral symbol of the regulariser block (with the zero-mode rule) times
// the number of grid points (to normalise the unscaled inverse transform).
struct Symbol {
  const float* lam[3];
  const float* scale;  // per node s_j
  const float* mu1;    // per node replacement for mu = 0
  float gamma;
  int curv;
  float nv;
};

// One pass along y (axis 1) or z (axis 2) for all lines of all fields of the
// half spectrum along x (cx = m_x / 2 + 1 columns; layout [field][z][y][cx]).
// MODE 0: forward; 1: inverse; 2: forward, divide by mu, inverse (the last
// axis).  A block takes lpb neighbouring x columns of one (field, z or y).
template <int D, int MODE>
__global__ void __launch_bounds__(kBlock) k_fft_axis(Geo g, int axis, int lpb, FftLine L, Symbol sym,
                                                     const float2* __restrict__ in, float2* __restrict__ out, int cx) {
  if (halted(g.halt)) return;
  extern __shared__ float2 sh[];
  const int n = L.n;
  const int ls = n | 1;     // odd line stride: writes across lines hit distinct banks
  float2* b0 = sh;
  float2* b1 = sh + lpb * ls;
  float2* twl = sh + 2 * lpb * ls;  // twiddles, staged with the first load
  // the thread's first twiddle is stored after the data loads below (both
  // trips overlap; a thread past the end stores the last twiddle again)
  const int tq = min((int)threadIdx.x, n - 1);
  const float2 twv = L.tw[tq];
  for (int q = threadIdx.x + blockDim.x; q < n; q += blockDim.x) twl[q] = L.tw[q];
  const int m0 = cx, m1 = g.mv[1], m2 = D == 3 ? g.mv[2] : 1;
  const long long fstride = (long long)m0 * m1 * m2;
  const int fields = g.nodes * D;
  const long long group = blockIdx.x;
  const int xg = (int)(group % ((m0 + lpb - 1) / lpb));
  const long long rest = group / ((m0 + lpb - 1) / lpb);
  const int other = axis == 1 ? m2 : m1;
  const int o = (int)(rest % other);
  const int f = (int)(rest / other);  // field
  if (f >= fields) return;
  const int x0 = xg * lpb;
  const int nlines = min(lpb, m0 - x0);
  // element 0 of line 0, step along the line; lines are neighbouring columns
  const long long base = axis == 1 ? (long long)f * fstride + (long long)o * m0 * m1 + x0
                                   : (long long)f * fstride + (long long)o * m0 + x0;
  const long long estride = axis == 1 ? (long long)m0 : (long long)m0 * m1;
  const int c1 = axis == 1 ? 0 : o;  // y of the lines (z pass)
  // load across lines (neighbouring x columns): contiguous runs of nlines
  const DivBy by_lines(nlines), by_n(n);
  // two elements per thread and pass, both loads issued before the stores
  // (past the end the last element is loaded and stored again)
  for (int e0 = threadIdx.x; e0 < nlines * n; e0 += 2 * blockDim.x) {
    float2 v[2];
    int at[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + u * (int)blockDim.x, nlines * n - 1);
      const int i = by_lines(e), l = e - i * nlines;
      v[u] = in[base + l + (long long)i * estride];
      at[u] = l * ls + i;
    }
    __builtin_amdgcn_sched_barrier(0);   // else the second load is issued after the first store's wait
#pragma unroll
    for (int u = 0; u < 2; ++u) b0[at[u]] = v[u];
  }
  twl[tq] = twv;
  __syncthreads();
  float2* res;
  if (MODE == 1) {
    res = lds_fft<true>(L, twl, nlines, ls, b0, b1);
  } else {
    res = lds_fft<false>(L, twl, nlines, ls, b0, b1);
  }
  if (MODE == 2) {
    // divide by the symbol; the fused axis is the last one
    float2* other = (res == b0) ? b1 : b0;
    for (int e = threadIdx.x; e < nlines * n; e += blockDim.x) {
      const int l = by_n(e), i = e - l * n;
      // x frequency across lines; in 2-D the fused axis is y, in 3-D z
      const int kx = x0 + l;
      const int ky = D == 2 ? i : c1;
      const int kz = D == 2 ? 0 : i;
      float lam = sym.lam[0][kx] + sym.lam[1][ky] + (D == 3 ? sym.lam[2][kz] : 0.f);
      if (sym.curv) lam = lam * lam;
      const int j = f / D;
      float mu = fmaf(sym.scale[j], lam, sym.gamma);
      if (mu == 0.f) mu = sym.mu1[j];
      float inv = 1.f / (mu * sym.nv);
      float2 v = res[l * ls + i];
      res[l * ls + i] = make_float2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    res = lds_fft<true>(L, twl, nlines, ls, res, other);
  }
  for (int e = threadIdx.x; e < nlines * n; e += blockDim.x) {
    const int i = by_lines(e), l = e - i * nlines;
    out[base + l + (long long)i * estride] = res[l * ls + i];
  }
}

// x pass, forward, real input: rows 2p and 2p + 1 of the real field form one
// complex line a + i b; after its FFT Z the half spectra of the two rows are
// A(k) = (Z(k) + conj Z(n-k)) / 2 and B(k) = (Z(k) - conj Z(n-k)) / 2i,
// stored for k = 0 .. n/2 (the rest follows from Hermitian symmetry).
template <int D>
__global__ void __launch_bounds__(kBlock) k_fft_x_r2c(Geo g, int lpb, FftLine L, const float* __restrict__ in,
                                                      float2* __restrict__ out, long long rows, int cx) {
  if (halted(g.halt)) return;
  extern __shared__ float2 sh[];
  const int n = L.n, ls = n | 1;
  float2* b0 = sh;
  float2* b1 = sh + lpb * ls;
  float2* twl = sh + 2 * lpb * ls;  // twiddles, staged with the first load
  for (int q = threadIdx.x; q < n; q += blockDim.x) twl[q] = L.tw[q];
  const long long pairs = (rows + 1) / 2;
  const long long pr0 = (long long)blockIdx.x * lpb;
  if (pr0 >= pairs) return;
  const int nlines = (int)min((long long)lpb, pairs - pr0);
  const DivBy by_n(n), by_cx(cx);
  for (int e = threadIdx.x; e < nlines * n; e += blockDim.x) {
    const int l = by_n(e), i = e - l * n;
    const long long ra = 2 * (pr0 + l);
    const float a = in[ra * n + i];
    const float b = ra + 1 < rows ? in[(ra + 1) * n + i] : 0.f;
    b0[l * ls + i] = make_float2(a, b);
  }
  __syncthreads();
  const float2* res = lds_fft<false>(L, twl, nlines, ls, b0, b1);
  for (int e = threadIdx.x; e < nlines * cx; e += blockDim.x) {
    const int l = by_cx(e), k = e - l * cx;
    const long long ra = 2 * (pr0 + l);
    const float2 z = res[l * ls + k], zm = res[l * ls + (k == 0 ? 0 : n - k)];
    out[ra * cx + k] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    if (ra + 1 < rows) out[(ra + 1) * cx + k] = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
  }
}

// x pass, inverse, real output: the inverse of k_fft_x_r2c.  The two rows'
// half spectra A, B are extended by Hermitian symmetry, the line A + i B is
// transformed back, and its real and imaginary parts are the two rows.
template <int D>
__global__ void __launch_bounds__(kBlock) k_fft_x_c2r(Geo g, int lpb, FftLine L, const float2* __restrict__ in,
                                                      float* __restrict__ out, long long rows, int cx) {
  if (halted(g.halt)) return;
  extern __shared__ float2 sh[];
  const int n = L.n, ls = n | 1;
  float2* b0 = sh;
  float2* b1 = sh + lpb * ls;
  float2* twl = sh + 2 * lpb * ls;  // twiddles, staged with the first load
  for (int q = threadIdx.x; q < n; q += blockDim.x) twl[q] = L.tw[q];
  const long long pairs = (rows + 1) / 2;
  const long long pr0 = (long long)blockIdx.x * lpb;
  if (pr0 >= pairs) return;
  const int nlines = (int)min((long long)lpb, pairs - pr0);
  const DivBy by_n(n);
  for (int e = threadIdx.x; e < nlines * n; e += blockDim.x) {
    const int l = by_n(e), i = e - l * n;
    const long long ra = 2 * (pr0 + l);
    const bool direct = i < cx;
    const int k = direct ? i : n - i;
    float2 a = in[ra * cx + k];
    float2 b = ra + 1 < rows ? in[(ra + 1) * cx + k] : make_float2(0.f, 0.f);
    if (!direct) {
      a.y = -a.y;
      b.y = -b.y;
    }
    b0[l * ls + i] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  const float2* res = lds_fft<true>(L, twl, nlines, ls, b0, b1);
  for (int e = threadIdx.x; e < nlines * n; e += blockDim.x) {
    const int l = by_n(e), i = e - l * n;
    const long long ra = 2 * (pr0 + l);
    const float2 v = res[l * ls + i];
    out[ra * n + i] = v.x;
    if (ra + 1 < rows) out[(ra + 1) * n + i] = v.y;
  }
}

// The plane kernels run one block per plane (3 x 64 blocks at 64^3): 1024
// threads per block overlap more of each block's chain of load, FFT stages
// and store than 256 (54.5 -> 44.9 us per preconditioner application).
constexpr int kPlaneBlock = 1024;

// 3-D: x and y transforms of one z-plane of one field in LDS.  Forward: the
// plane's real rows, two per complex line, are transformed along x and split
// into their half spectra (as in k_fft_x_r2c), written transposed
// ([kx][y], odd stride) into the other buffer, transformed along y, and
// stored as [field][z][y][cx].  One block per (field, z).
__global__ void __launch_bounds__(kPlaneBlock) k_fft_xy_fwd(Geo g, FftLine Lx, FftLine Ly, const float* __restrict__ in,
                                                       float2* __restrict__ out, int cx) {
  if (halted(g.halt)) return;
  extern __shared__ float2 sh[];
  const int nx = Lx.n, ny = Ly.n, lsx = nx | 1, lsy = ny | 1;
  const int pairs = (ny + 1) / 2;
  const int cap = max(pairs * lsx, cx * lsy);
  const DivBy by_nx(nx), by_cx(cx);
  float2* b0 = sh;
  float2* b1 = sh + cap;
  float2* twx = sh + 2 * cap;
  float2* twy = twx + nx;
  // twiddles (twy follows twx): the thread's first one is loaded here and
  // stored after the data loads below, so both trips overlap (a thread past
  // the end stores the last twiddle again)
  const int tq = min((int)threadIdx.x, nx + ny - 1);
  const float2 twv = tq < nx ? Lx.tw[tq] : Ly.tw[tq - nx];
  for (int q = threadIdx.x + blockDim.x; q < nx + ny; q += blockDim.x) twx[q] = q < nx ? Lx.tw[q] : Ly.tw[q - nx];
  const long long plane = blockIdx.x;
  const float* src = in + plane * nx * ny;
  for (int e0 = threadIdx.x; e0 < pairs * nx; e0 += 2 * blockDim.x) {   // two per pass, loads first
    float2 v[2];
    int at[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + u * (int)blockDim.x, pairs * nx - 1);
      const int l = by_nx(e), i = e - l * nx;
      const int y = 2 * l;
      const float a = src[y * nx + i];
      const float b = src[min(y + 1, ny - 1) * nx + i];
      v[u] = make_float2(a, y + 1 < ny ? b : 0.f);
      at[u] = l * lsx + i;
    }
    __builtin_amdgcn_sched_barrier(0);   // else the second load is issued after the first store's wait
#pragma unroll
    for (int u = 0; u < 2; ++u) b0[at[u]] = v[u];
  }
  twx[tq] = twv;
  __syncthreads();
  float2* rx = lds_fft<false>(Lx, twx, pairs, lsx, b0, b1);
  float2* t = rx == b0 ? b1 : b0;
  for (int e = threadIdx.x; e < pairs * cx; e += blockDim.x) {
    const int l = by_cx(e), k = e - l * cx;
    const float2 z = rx[l * lsx + k], zm = rx[l * lsx + (k == 0 ? 0 : nx - k)];
    t[k * lsy + 2 * l] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    if (2 * l + 1 < ny) t[k * lsy + 2 * l + 1] = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
  }
  __syncthreads();
  const float2* ry = lds_fft<false>(Ly, twy, cx, lsy, t, rx);
  float2* dst = out + plane * ny * cx;
  for (int e = threadIdx.x; e < ny * cx; e += blockDim.x) {
    const int y = by_cx(e), k = e - y * cx;
    dst[y * cx + k] = ry[k * lsy + y];
  }
}

// Inverse of k_fft_xy_fwd: y transform of the plane's half spectrum, then
// the row pairs' lines A + i B rebuilt by Hermitian symmetry (as in
// k_fft_x_c2r), transformed along x and written as real rows.
__global__ void __launch_bounds__(kPlaneBlock) k_fft_xy_inv(Geo g, FftLine Lx, FftLine Ly, const float2* __restrict__ in,
                                                       float* __restrict__ out, int cx, const float* __restrict__ r,
                                                       double* __restrict__ rz) {
  if (halted(g.halt)) return;
  extern __shared__ float2 sh[];
  const int nx = Lx.n, ny = Ly.n, lsx = nx | 1, lsy = ny | 1;
  const int pairs = (ny + 1) / 2;
  const int cap = max(pairs * lsx, cx * lsy);
  const DivBy by_nx(nx), by_cx(cx);
  float2* b0 = sh;
  float2* b1 = sh + cap;
  float2* twx = sh + 2 * cap;
  float2* twy = twx + nx;
  // twiddles (twy follows twx): the thread's first one is loaded here and
  // stored after the data loads below, so both trips overlap (a thread past
  // the end stores the last twiddle again)
  const int tq = min((int)threadIdx.x, nx + ny - 1);
  const float2 twv = tq < nx ? Lx.tw[tq] : Ly.tw[tq - nx];
  for (int q = threadIdx.x + blockDim.x; q < nx + ny; q += blockDim.x) twx[q] = q < nx ? Lx.tw[q] : Ly.tw[q - nx];
  const long long plane = blockIdx.x;
  const float2* src = in + plane * ny * cx;
  for (int e0 = threadIdx.x; e0 < ny * cx; e0 += 2 * blockDim.x) {   // two per pass, loads first
    float2 v[2];
    int at[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + u * (int)blockDim.x, ny * cx - 1);
      const int y = by_cx(e), k = e - y * cx;
      v[u] = src[y * cx + k];
      at[u] = k * lsy + y;
    }
    __builtin_amdgcn_sched_barrier(0);   // else the second load is issued after the first store's wait
#pragma unroll
    for (int u = 0; u < 2; ++u) b0[at[u]] = v[u];
  }
  twx[tq] = twv;
  __syncthreads();
  float2* ry = lds_fft<true>(Ly, twy, cx, lsy, b0, b1);
  float2* t = ry == b0 ? b1 : b0;
  for (int e = threadIdx.x; e < pairs * nx; e += blockDim.x) {
    const int l = by_nx(e), i = e - l * nx;
    const bool direct = i < cx;
    const int k = direct ? i : nx - i;
    float2 a = ry[k * lsy + 2 * l];
    float2 b = 2 * l + 1 < ny ? ry[k * lsy + 2 * l + 1] : make_float2(0.f, 0.f);
    if (!direct) {
      a.y = -a.y;
      b.y = -b.y;
    }
    t[l * lsx + i] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  const float2* rx = lds_fft<true>(Lx, twx, pairs, lsx, t, ry);
  float* dst = out + plane * nx * ny;
  const float* rp = r ? r + plane * nx * ny : nullptr;
  double acc = 0.0;
  for (int e = threadIdx.x; e < pairs * nx; e += blockDim.x) {
    const int l = by_nx(e), i = e - l * nx;
    const float2 v = rx[l * lsx + i];
    dst[2 * l * nx + i] = v.x;
    if (rp) acc += (double)rp[2 * l * nx + i] * (double)v.x;
    if (2 * l + 1 < ny) {
      dst[(2 * l + 1) * nx + i] = v.y;
      if (rp) acc += (double)rp[(2 * l + 1) * nx + i] * (double)v.y;
    }
  }
  if (rz) {  // r . z partial of this plane (kernel argument: the whole block)
    __shared__ double sh[kPlaneBlock];
    const double tb = block_sum(acc, sh);
    if (threadIdx.x == 0) rz[blockIdx.x] = tb;
  }
}

static bool factor_radices(int n, int* rad, int* nrad) {
  int k = 0;
  int m = n;
  while (m % 4 == 0 && k < 16) { rad[k++] = 4; m /= 4; }
  while (m % 2 == 0 && k < 16) { rad[k++] = 2; m /= 2; }
  while (m % 3 == 0 && k < 16) { rad[k++] = 3; m /= 3; }
  while (m % 5 == 0 && k < 16) { rad[k++] = 5; m /= 5; }
  *nrad = k;
  return m == 1;
}

int precond_setup(lag_plan P) {
  const int D = P->geo.dim;
  P->fft_ok = 1;
  for (int a = 0; a < D; ++a) {
    int n = P->prob.vel_m[a];
    if (n > 1024 || !factor_radices(n, P->fft_rad[a], &P->fft_nrad[a])) P->fft_ok = 0;
  }
  if (!P->fft_ok) return LAG_OK;  // spectral_precond_apply reports LAG_EUNSUPPORTED
  LAG_HIP(hipMalloc(&P->fft_buf, sizeof(float2) * P->geo.nv * P->fields));
  for (int a = 0; a < D; ++a) {
    const int n = P->prob.vel_m[a];
    std::vector<float2> tw(n);
    for (int q = 0; q < n; ++q) {
      double ang = -2.0 * M_PI * (double)q / (double)n;
      tw[q] = make_float2((float)cos(ang), (float)sin(ang));
    }
    LAG_HIP(hipMalloc(&P->fft_tw[a], sizeof(float2) * n));
    LAG_HIP(hipMemcpy(P->fft_tw[a], tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
    std::vector<float> lam(n);
    const double h = P->prob.extent[a] / n;
    for (int k = 0; k < n; ++k) {
      double sn = sin(M_PI * (double)k / (double)n);
      lam[k] = (float)(4.0 / (h * h) * sn * sn);
    }
    LAG_HIP(hipMalloc(&P->fft_lam[a], sizeof(float) * n));
    LAG_HIP(hipMemcpy(P->fft_lam[a], lam.data(), sizeof(float) * n, hipMemcpyHostToDevice));
  }
  // smallest nonzero eigenvalue of each node's block (replaces a zero mode)
  double lmin = 1e300;
  for (int a = 0; a < D; ++a) {
    const int n = P->prob.vel_m[a];
    const double h = P->prob.extent[a] / n;
    double sn = sin(M_PI / (double)n);
    lmin = fmin(lmin, 4.0 / (h * h) * sn * sn);
  }
  if (P->prob.reg == LAG_CURVATURE) lmin = lmin * lmin;
  std::vector<float> mu1(P->geo.nodes);
  double hv = 1.0;
  for (int a = 0; a < D; ++a) hv *= P->prob.extent[a] / P->prob.vel_m[a];
  for (int j = 0; j < P->geo.nodes; ++j)
    mu1[j] = (float)(P->prob.alpha * hv * P->node_w[j] * lmin + P->prob.gamma);
  LAG_HIP(hipMalloc(&P->fft_mu1, sizeof(float) * P->geo.nodes));
  LAG_HIP(hipMemcpy(P->fft_mu1, mu1.data(), sizeof(float) * P->geo.nodes, hipMemcpyHostToDevice));
  return LAG_OK;
}

// About 1024 elements (4 per thread) and at most 16 lines per block, so that
// a 64^3 field splits into enough blocks to fill the chip; the lines of the
// y and z passes are neighbouring x columns, read as runs of lpb values
// (16 complex values: 128-byte runs; 8 measured 7 % slower in the z pass).
static int lines_per_block(int n, int axis, int m0) {
  int lpb = 1024 / n;
  if (lpb < 1) lpb = 1;
  if (lpb > 16) lpb = 16;
  if (axis != 0 && lpb > m0) lpb = m0;
  return lpb;
}

static FftLine fft_line(lag_plan P, int axis) {
  FftLine L;
  L.n = P->prob.vel_m[axis];
  L.nrad = P->fft_nrad[axis];
  for (int i = 0; i < 16; ++i) L.rad[i] = P->fft_rad[axis][i];
  L.tw = P->fft_tw[axis];
  return L;
}

template <int D, int MODE>
static int fft_pass(lag_plan P, int axis, const float2* in, float2* out, hipStream_t s) {
  FftLine L;
  L.n = P->prob.vel_m[axis];
  L.nrad = P->fft_nrad[axis];
  for (int i = 0; i < 16; ++i) L.rad[i] = P->fft_rad[axis][i];
  L.tw = P->fft_tw[axis];
  Symbol sym;
  for (int a = 0; a < 3; ++a) sym.lam[a] = P->fft_lam[a];
  sym.scale = P->reg_scale;
  sym.mu1 = P->fft_mu1;
  sym.gamma = (float)P->prob.gamma;
  sym.curv = P->prob.reg == LAG_CURVATURE;
  sym.nv = (float)P->geo.nv;
  const int m1 = P->prob.vel_m[1], m2 = D == 3 ? P->prob.vel_m[2] : 1;
  const int cx = P->prob.vel_m[0] / 2 + 1;  // half spectrum along x
  const int lpb = lines_per_block(L.n, axis, cx);
  const long long xg = (cx + lpb - 1) / lpb;
  const long long groups = xg * (axis == 1 ? m2 : m1) * P->fields;
  size_t lds = sizeof(float2) * (2 * (size_t)lpb * (L.n | 1) + L.n);
  hipLaunchKernelGGL((k_fft_axis<D, MODE>), dim3((unsigned)groups), dim3(kBlock), lds, s, P->geo, axis, lpb, L,
                     sym, in, out, cx);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// x pass of the real field (forward: real rows -> half spectra; inverse:
// half spectra -> real rows), two rows per complex line
template <int D>
static int fft_x(lag_plan P, bool inverse, const void* in, void* out, hipStream_t s) {
  FftLine L;
  L.n = P->prob.vel_m[0];
  L.nrad = P->fft_nrad[0];
  for (int i = 0; i < 16; ++i) L.rad[i] = P->fft_rad[0][i];
  L.tw = P->fft_tw[0];
  const int m1 = P->prob.vel_m[1], m2 = D == 3 ? P->prob.vel_m[2] : 1;
  const int cx = L.n / 2 + 1;
  const long long rows = (long long)P->fields * m1 * m2;
  const long long pairs = (rows + 1) / 2;
  const int lpb = lines_per_block(L.n, 0, cx);
  const unsigned groups = (unsigned)((pairs + lpb - 1) / lpb);
  const size_t lds = sizeof(float2) * (2 * (size_t)lpb * (L.n | 1) + L.n);
  if (inverse)
    hipLaunchKernelGGL(k_fft_x_c2r<D>, dim3(groups), dim3(kBlock), lds, s, P->geo, lpb, L, (const float2*)in,
                       (float*)out, rows, cx);
  else
    hipLaunchKernelGGL(k_fft_x_r2c<D>, dim3(groups), dim3(kBlock), lds, s, P->geo, lpb, L, (const float*)in,
                       (float2*)out, rows, cx);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_precond(lag_plan P, const float* r, float* z, hipStream_t s, double* rz, int* nrz) {
  if (!P->fft_ok) return LAG_EUNSUPPORTED;
  if (!(P->prob.alpha > 0.0) && !(P->prob.gamma > 0.0)) return LAG_EINVAL;
  float2* buf = P->fft_buf;
  int rc;
  if (P->geo.dim == 3) {
    const int nx = P->prob.vel_m[0], ny = P->prob.vel_m[1], cx = nx / 2 + 1;
    const size_t cap = std::max<size_t>((size_t)((ny + 1) / 2) * (nx | 1), (size_t)cx * (ny | 1));
    const size_t lds = sizeof(float2) * (2 * cap + nx + ny);
    if (lds <= 64 * 1024) {  // x and y of a plane together, then z
      FftLine Lx = fft_line(P, 0), Ly = fft_line(P, 1);
      const unsigned planes = (unsigned)(P->fields * P->prob.vel_m[2]);
      hipLaunchKernelGGL(k_fft_xy_fwd, dim3(planes), dim3(kPlaneBlock), lds, s, P->geo, Lx, Ly, r, buf, cx);
      LAG_LAUNCH_CHECK();
      if ((rc = fft_pass<3, 2>(P, 2, buf, buf, s))) return rc;
      hipLaunchKernelGGL(k_fft_xy_inv, dim3(planes), dim3(kPlaneBlock), lds, s, P->geo, Lx, Ly, buf, z, cx,
                         rz ? r : nullptr, rz);
      LAG_LAUNCH_CHECK();
      if (rz) *nrz = (int)planes;
      return LAG_OK;
    }
    if ((rc = fft_x<3>(P, false, r, buf, s))) return rc;
    if ((rc = fft_pass<3, 0>(P, 1, buf, buf, s))) return rc;
    if ((rc = fft_pass<3, 2>(P, 2, buf, buf, s))) return rc;
    if ((rc = fft_pass<3, 1>(P, 1, buf, buf, s))) return rc;
    if ((rc = fft_x<3>(P, true, buf, z, s))) return rc;
  } else {
    if ((rc = fft_x<2>(P, false, r, buf, s))) return rc;
    if ((rc = fft_pass<2, 2>(P, 1, buf, buf, s))) return rc;
    if ((rc = fft_x<2>(P, true, buf, z, s))) return rc;
  }
  if (rz) {  // the separate passes: a separate inner product
    if ((rc = launch_dot_partial(P, P->n_unknowns, r, z, rz, s))) return rc;
    *nrz = (int)std::min<long long>(kRedBlocks, std::max<long long>(1, (P->n_unknowns + kBlock - 1) / kBlock));
  }
  return LAG_OK;
}

}  // namespace lag
