// Reductions and vector updates for the Gauss-Newton-Krylov driver.
//
// Inner products and the SSD distance (eq. SSD) accumulate in float64 with a
// fixed grid and a fixed reduction tree, so their results do not depend on
// scheduling.  PCG scalars stay on the device: the update kernels read
// alpha = (r.z)/(p.Hp) and beta = (r.z)_new/(r.z)_old from device memory.

#include "lag_internal.hpp"

namespace lag {

__global__ void __launch_bounds__(kBlock) k_dot_partial(const float* __restrict__ x, const float* __restrict__ y,
                                                         long long n, double* __restrict__ part,
                                                         const int* __restrict__ halt) {
  if (halted(halt)) return;
  __shared__ double sh[kBlock];
  double s = 0.0;
  const long long st = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += 4 * st) {   // four elements' loads in flight (clamped), terms added in index order
    float xa[4], ya[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long k = min(i + u * st, n - 1);
      xa[u] = x[k];
      ya[u] = y[k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * st < n) s += (double)xa[u] * (double)ya[u];
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// SSD partials; also writes wres = scale * (u - R) when wres != null
__global__ void __launch_bounds__(kBlock) k_ssd_partial(const float* __restrict__ u, const float* __restrict__ R,
                                                         float* __restrict__ wres, float scale, long long n,
                                                         double* __restrict__ part) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 4 * st) {
    float ua[4], ra[4];              // four elements' loads in flight (clamped), terms added in index order
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long k = min(i + q * st, n - 1);
      ua[q] = u[k];
      ra[q] = R[k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i + q * st >= n) break;
      const float r = ua[q] - ra[q];
      s += (double)r * (double)r;
      if (wres) wres[i + q * st] = scale * r;
    }
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Sum of the block partials of a reduction, in the same order in every block
// of kBlock threads (so consumers can take it without a separate launch).
// Four loads are issued before the first add, in the same order of addition
// as a plain strided loop.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nparts, double* sh) {
  double s = 0.0;
  const int bs = blockDim.x;
  int i = threadIdx.x;
  for (; i + 3 * bs < nparts; i += 4 * bs) {
    const double a = part[i], b = part[i + bs], c = part[i + 2 * bs], d = part[i + 3 * bs];
    s += a;
    s += b;
    s += c;
    s += d;
  }
  for (; i < nparts; i += bs) s += part[i];
  return block_sum(s, sh);
}

__global__ void __launch_bounds__(kBlock) k_final_sum(const double* __restrict__ part, int nparts, double scale,
                                                       double* __restrict__ dst, const int* __restrict__ halt) {
  if (halted(halt)) return;
  __shared__ double sh[kBlock];
  double t = sum_partials(part, nparts, sh);
  if (threadIdx.x == 0) *dst = scale * t;
}

static int reduce_launch(long long n, unsigned& blocks) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  blocks = (unsigned)b;
  return 0;
}

int launch_dot(lag_plan P, long long n, const float* x, const float* y, double* dst, hipStream_t s) {
  unsigned blocks;
  reduce_launch(n, blocks);
  hipLaunchKernelGGL(k_dot_partial, dim3(blocks), dim3(kBlock), 0, s, x, y, n, P->red_partial, P->geo.halt);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, s, P->red_partial, (int)blocks, 1.0, dst, P->geo.halt);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_dot_partial(lag_plan P, long long n, const float* x, const float* y, double* part, hipStream_t s) {
  unsigned blocks;
  reduce_launch(n, blocks);
  hipLaunchKernelGGL(k_dot_partial, dim3(blocks), dim3(kBlock), 0, s, x, y, n, part, P->geo.halt);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// Regulariser energy 0.5 v . (s_j A v), s_j = h_v^d w_j: block partials of
// v_i reg_value(v)_i on the grid of k_dot_partial, then the fixed-order final
// sum times 1/2: the terms and order of a regulariser pass, an inner product
// and a halving, in two launches.
template <int D, bool CURV>
__global__ void __launch_bounds__(kBlock) k_reg_energy(Geo g, const float* __restrict__ v,
                                                        const float* __restrict__ scale, float ih2x, float ih2y,
                                                        float ih2z, long long n, double* __restrict__ part) {
  if (halted(g.halt)) return;
  __shared__ double sh[kBlock];
  const float ih2[3] = {ih2x, ih2y, ih2z};
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s += (double)v[i] * (double)reg_value<D, CURV>(g, v, scale, 0.f, ih2, i);
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

int launch_reg_energy(lag_plan P, const float* v, double* dst, hipStream_t s) {
  const long long n = P->n_unknowns;
  unsigned blocks;
  reduce_launch(n, blocks);
  const RegTail r = reg_tail(P, v, 0, 0.f, nullptr);
#define LAG_RE(DD, CV)                                                                                      \
  hipLaunchKernelGGL((k_reg_energy<DD, CV>), dim3(blocks), dim3(kBlock), 0, s, P->geo, v, r.scale, r.ih2[0], \
                     r.ih2[1], r.ih2[2], n, P->red_partial)
  if (P->geo.dim == 3) {
    if (r.curv) LAG_RE(3, true);
    else LAG_RE(3, false);
  } else {
    if (r.curv) LAG_RE(2, true);
    else LAG_RE(2, false);
  }
#undef LAG_RE
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, s, P->red_partial, (int)blocks, 0.5, dst, P->geo.halt);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_ssd(lag_plan P, const float* u, const float* R, float* wres, float scale, double* dst, hipStream_t s) {
  unsigned blocks;
  const long long n = P->geo.np;
  reduce_launch(n, blocks);
  hipLaunchKernelGGL(k_ssd_partial, dim3(blocks), dim3(kBlock), 0, s, u, R, wres, scale, n, P->red_partial);
  LAG_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, s, P->red_partial, (int)blocks,
                     0.5 * (double)P->geo.cell_img, dst, P->geo.halt);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

__global__ void __launch_bounds__(kBlock) k_axpy(long long n, float a, const float* __restrict__ x,
                                                  float* __restrict__ y) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fmaf(a, x[i], y[i]);
}

int launch_axpy(long long n, float a, const float* x, float* y, hipStream_t s) {
  if (n <= 0) return LAG_OK;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, a, x, y);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

__global__ void k_combine_J(double* s3, double alpha) {
  if (threadIdx.x == 0 && blockIdx.x == 0) s3[0] = s3[1] + alpha * s3[2];
}

int launch_combine_J(double* s3, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_combine_J, dim3(1), dim3(64), 0, s, s3, alpha);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// ---- PCG updates with device scalars --------------------------------------
// sc[0] = r.z (current), sc[1] = p.Hp, sc[2] = r.z (new), sc[3] = r.r,
// sc[4] = breakdown flag (p.Hp <= 0).  The update kernels finish the inner
// products they need from the block partials of k_dot_partial themselves.

// x += alpha p, r -= alpha Hp with alpha = sc[0] / p.Hp (p.Hp from `php`
// partials; no update when p.Hp <= 0), and the block partials of the new
// r.r into `rr` (the grid and order of k_dot_partial over r, r).
__global__ void __launch_bounds__(kBlock) k_pcg_xr(long long n, float* __restrict__ x, float* __restrict__ r,
                                                    const float* __restrict__ p, const float* __restrict__ Hp,
                                                    double* __restrict__ sc, const double* __restrict__ php,
                                                    int nphp, double* __restrict__ rr, const int* __restrict__ halt) {
  if (halted(halt)) return;
  __shared__ double sh[kBlock];
  const long long st = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // four elements' loads in flight (clamped), terms added in index order;
  // the first four go out before the p.Hp partials are summed, so both
  // trips overlap
  float ra[4], pa[4], xa[4], ha[4];
  auto load4 = [&](long long i0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long k = min(i0 + u * st, n - 1);
      ra[u] = r[k];
      pa[u] = p[k];
      xa[u] = x[k];
      ha[u] = Hp[k];
    }
  };
  if (i < n) load4(i);
  const double pHp = sum_partials(php, nphp, sh);
  const bool ok = pHp > 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[1] = pHp;
    if (!ok) sc[4] = 1.0;
  }
  const float a = ok ? (float)(sc[0] / pHp) : 0.f;
  double s = 0.0;
  for (; i < n; i += 4 * st) {
    if (i != (long long)blockIdx.x * blockDim.x + threadIdx.x) load4(i);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i + u * st >= n) break;
      float ri = ra[u];
      if (ok) {
        x[i + u * st] = fmaf(a, pa[u], xa[u]);
        ri = fmaf(-a, ha[u], ri);
        r[i + u * st] = ri;
      }
      s += (double)ri * (double)ri;
    }
  }
  __syncthreads();  // every thread has read sh[0] of the first sum
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) rr[blockIdx.x] = t;
}

// p = z + beta p with beta = r.z (from `rz` partials, stored to sc[2]) / sc[0],
// one thread per grid node (all D components), which also writes the packed
// copy of p that the next matvec gathers from: the node and its periodic
// ghost images (index + m on the axes where it is 0), the layout of k_pack.
template <int D>
__global__ void __launch_bounds__(kBlock) k_pcg_p_pack(Geo g, float* __restrict__ p, const float* __restrict__ z,
                                                        double* __restrict__ sc, const double* __restrict__ rz,
                                                        int nrz, const int* __restrict__ halt,
                                                        typename VecT<D>::T* __restrict__ pk) {
  if (halted(halt)) return;
  __shared__ double sh[kBlock];
  const long long nv = g.nv, tot = nv * g.nodes;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // the first node's p and z are loaded before the r.z partials are summed
  // (both trips overlap)
  float p0[D], z0[D];
  if (t0 < tot) {
    const long long j = t0 / nv, q = t0 - j * nv;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const long long i = (j * D + c) * nv + q;
      p0[c] = p[i];
      z0[c] = z[i];
    }
  }
  const double rznew = sum_partials(rz, nrz, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[2] = rznew;
  const float beta = (float)(rznew / sc[0]);
  for (long long t = t0; t < tot; t += (long long)gridDim.x * blockDim.x) {
    long long j, q;
    int x, y, zc;
    split_index(g, t, j, q, x, y, zc);
    if (D != 3) zc = 0;
    float v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const long long i = (j * D + c) * nv + q;
      v[c] = fmaf(beta, t == t0 ? p0[c] : p[i], t == t0 ? z0[c] : z[i]);
      p[i] = v[c];
    }
    typename VecT<D>::T val;
    if constexpr (D == 3) val = make_float4(v[0], v[1], v[2], 0.f);
    else val = make_float2(v[0], v[1]);
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      if (((o & 1) && x != 0) || ((o & 2) && y != 0) || ((o & 4) && zc != 0)) continue;
      const int X = (o & 1) ? g.mv[0] : x, Y = (o & 2) ? g.mv[1] : y, Z = (o & 4) ? g.mv[2] : zc;
      pk[j * g.nvp + ((long long)Z * g.pv[1] + Y) * g.pv[0] + X] = val;
    }
  }
}

// Device-side PCG control for graph-captured iterations.  ctl[0] = halt
// (0 running, 1 converged, 2 breakdown, 3 iteration cap), ctl[1] =
// completed iterations, ctl[2] = iteration cap; sc[3] = r.r, sc[4] =
// breakdown flag, sc[6] = tol^2 b.b.  Init evaluates the test before the
// first iteration; check runs after each iteration.
__global__ void k_pcg_ctl_init(int* ctl, const double* sc, int maxit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl[1] = 0;
  ctl[2] = maxit;
  ctl[0] = sc[4] != 0.0 ? 2 : (sc[3] <= sc[6] ? 1 : (maxit <= 0 ? 3 : 0));
}

// After an iteration: sc[3] = r.r from the `rr` partials (mirrored into the
// control block for the host), sc[0] = sc[2] (the new r.z becomes current),
// then the stopping test.
__global__ void __launch_bounds__(kBlock) k_pcg_check(int* ctl, double* sc, const double* __restrict__ rr, int nrr,
                                                       int* mirror) {
  // mirror != null: the control block's first six ints are also written to
  // pinned host memory (visible once the kernel has completed), which
  // spares a separate device-to-host copy per iteration
  auto publish = [&]() {
    if (mirror) {
#pragma unroll
      for (int k = 0; k < 6; ++k) mirror[k] = ctl[k];
      __threadfence_system();
    }
  };
  if (ctl[0] != 0) {
    if (threadIdx.x == 0) publish();
    return;
  }
  __shared__ double sh[kBlock];
  const double t = sum_partials(rr, nrr, sh);
  if (threadIdx.x != 0) return;
  sc[3] = t;
  reinterpret_cast<double*>(ctl)[2] = t;
  sc[0] = sc[2];
  const int it = ctl[1] + 1;
  if (sc[4] != 0.0) {     // this iteration broke down: it does not count
    ctl[0] = 2;
    publish();
    return;
  }
  ctl[1] = it;
  if (t <= sc[6]) ctl[0] = 1;
  else if (it >= ctl[2]) ctl[0] = 3;
  publish();
}

int launch_pcg_ctl_init(int* ctl, const double* sc, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_ctl_init, dim3(1), dim3(64), 0, s, ctl, sc, maxit);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_pcg_check(lag_plan P, hipStream_t s) {
  unsigned blocks;
  reduce_launch(P->n_unknowns, blocks);
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(kBlock), 0, s, P->ctl, P->scalars, P->red_partial2, (int)blocks,
                     P->ctl_mirror);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// x, r update with the p.Hp partials in red_partial (P->php_n of them, from
// the matvec); new r.r partials go to red_partial2 (consumed by
// launch_pcg_check)
int launch_pcg_xr(lag_plan P, float* x, float* r, const float* p, const float* Hp, hipStream_t s) {
  const long long n = P->n_unknowns;
  unsigned blocks;
  reduce_launch(n, blocks);
  hipLaunchKernelGGL(k_pcg_xr, dim3(blocks), dim3(kBlock), 0, s, n, x, r, p, Hp, P->scalars, P->red_partial,
                     P->php_n, P->red_partial2, P->ctl);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

// p update with the r.z partials in red_partial (P->rz_n of them, from the
// preconditioner)
int launch_pcg_p(lag_plan P, float* p, const float* z, hipStream_t s) {
  const long long n = P->n_unknowns;
  unsigned blocks;
  reduce_launch(n, blocks);
  if (P->geo.dim == 3)
    hipLaunchKernelGGL(k_pcg_p_pack<3>, dim3(blocks), dim3(kBlock), 0, s, P->geo, p, z, P->scalars, P->red_partial,
                       P->rz_n, P->ctl, (float4*)P->pack_p);
  else
    hipLaunchKernelGGL(k_pcg_p_pack<2>, dim3(blocks), dim3(kBlock), 0, s, P->geo, p, z, P->scalars, P->red_partial,
                       P->rz_n, P->ctl, (float2*)P->pack_p);
  LAG_LAUNCH_CHECK();
  P->packed_by_pcg = p;  // the next matvec of the solve needs no pack
  return LAG_OK;
}

__global__ void __launch_bounds__(kBlock) k_scale_mul(long long n, float c, const float* __restrict__ a,
                                                       const float* __restrict__ w, float* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = c * a[i];
  if (w) v *= w[i];
  out[i] = v;
}

int launch_scale_mul(long long n, float c, const float* a, const float* w, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_mul, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, c, a, w, out);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

__global__ void __launch_bounds__(kBlock) k_copy_axpby(long long n, float a, const float* __restrict__ x, float b,
                                                        const float* __restrict__ y, float* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + (y ? b * y[i] : 0.f);
}

int launch_axpby(long long n, float a, const float* x, float b, const float* y, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_axpby, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, a, x, b, y,
                     out);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

}  // namespace lag
