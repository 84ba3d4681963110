// Multilevel continuation (Sec. 3.2, last paragraph): restriction of images
// to a grid with half the cells per axis (mean of the 2^d children, the
// midpoint-rule integral over the coarse cell) and cell-centred linear
// refinement of velocities (weights 3/4 and 1/4 per axis, periodic).  Also
// the cell average onto the velocity grid at any ratio, which feeds the
// warm-start network.

#include <vector>

#include "lag_internal.hpp"

namespace lag {

template <int D>
__global__ void __launch_bounds__(kBlock) k_restrict(const float* __restrict__ f, float* __restrict__ out, int cx,
                                                     int cy, int cz) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nc = (long long)cx * cy * cz;
  if (i >= nc) return;
  const int x = (int)(i % cx), y = (int)((i / cx) % cy), z = (int)(i / ((long long)cx * cy));
  const int fx = 2 * cx, fy = 2 * cy;
  float s = 0.f;
  if (D == 2) {
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) s += f[(long long)(2 * y + dy) * fx + 2 * x + dx];
    out[i] = 0.25f * s;
  } else {
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
          s += f[((long long)(2 * z + dz) * fy + 2 * y + dy) * fx + 2 * x + dx];
    out[i] = 0.125f * s;
  }
}

// one fine-grid value per thread, over all fields (components x nodes)
template <int D>
__global__ void __launch_bounds__(kBlock) k_prolong(const float* __restrict__ c, float* __restrict__ out, int cx,
                                                    int cy, int cz, int fields) {
  const int fx = 2 * cx, fy = 2 * cy, fz = D == 3 ? 2 * cz : 1;
  const long long nf = (long long)fx * fy * fz;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * fields) return;
  const long long fld = i / nf, r = i - fld * nf;
  const int x = (int)(r % fx), y = (int)((r / fx) % fy), z = (int)(r / ((long long)fx * fy));
  // neighbour coarse cells and weights along each axis
  int i0[3], i1[3];
  float w1[3];
  const int fi[3] = {x, y, z}, cm[3] = {cx, cy, cz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      i0[a] = i1[a] = 0;
      w1[a] = 0.f;
      continue;
    }
    const int k = fi[a] >> 1;
    if (fi[a] & 1) {                 // at coarse coordinate k + 1/4
      i0[a] = k;
      i1[a] = k + 1 == cm[a] ? 0 : k + 1;
    } else {                         // at coarse coordinate k - 1/4
      i0[a] = k;
      i1[a] = k == 0 ? cm[a] - 1 : k - 1;
    }
    w1[a] = 0.25f;
  }
  const float* src = c + fld * (long long)cx * cy * cz;
  float s = 0.f;
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
    float w = 1.f;
    int idx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < D) {
        const bool b = (o >> a) & 1;
        idx[a] = b ? i1[a] : i0[a];
        w *= b ? w1[a] : 1.f - w1[a];
      } else {
        idx[a] = 0;
      }
    }
    s = fmaf(w, src[((long long)idx[2] * cy + idx[1]) * cx + idx[0]], s);
  }
  out[i] = s;
}

// Cell average over a coarser grid with any ratio: along axis a, in units of
// 1 / (img_m * vel_m) of the domain, fine cell i spans [i vm, (i + 1) vm) and
// coarse cell I spans [I im, (I + 1) im); the weight of i in I is their
// integer overlap divided by im.  One coarse value per thread.
template <int D>
__global__ void __launch_bounds__(kBlock) k_resample(const float* __restrict__ f, float* __restrict__ out, int fx,
                                                     int fy, int fz, int cx, int cy, int cz) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nc = (long long)cx * cy * cz;
  if (i >= nc) return;
  const int X = (int)(i % cx), Y = (int)((i / cx) % cy), Z = (int)(i / ((long long)cx * cy));
  const int fm[3] = {fx, fy, fz}, cm[3] = {cx, cy, cz}, C[3] = {X, Y, Z};
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // fine cells overlapping [C im, (C + 1) im) (fine cell i covers [i vm, (i + 1) vm))
    const long long b0 = (long long)C[a] * fm[a], b1 = b0 + fm[a];
    lo[a] = (int)(b0 / cm[a]);
    hi[a] = (int)((b1 + cm[a] - 1) / cm[a]);  // exclusive
  }
  if (D == 2) {
    lo[2] = 0;
    hi[2] = 1;
  }
  float s = 0.f;
  for (int z = lo[2]; z < hi[2]; ++z) {
    float wz = 1.f;
    if (D == 3) {
      const long long a0 = (long long)z * cm[2], a1 = a0 + cm[2];
      const long long b0 = (long long)Z * fm[2], b1 = b0 + fm[2];
      wz = (float)(min(a1, b1) - max(a0, b0)) / (float)fm[2];
    }
    for (int y = lo[1]; y < hi[1]; ++y) {
      const long long a0 = (long long)y * cm[1], a1 = a0 + cm[1];
      const long long b0 = (long long)Y * fm[1], b1 = b0 + fm[1];
      const float wy = wz * (float)(min(a1, b1) - max(a0, b0)) / (float)fm[1];
      for (int x = lo[0]; x < hi[0]; ++x) {
        const long long c0 = (long long)x * cm[0], c1 = c0 + cm[0];
        const long long d0 = (long long)X * fm[0], d1 = d0 + fm[0];
        const float w = wy * (float)(min(c1, d1) - max(c0, d0)) / (float)fm[0];
        s = fmaf(w, f[((long long)z * fy + y) * fx + x], s);
      }
    }
  }
  out[i] = s;
}

int launch_restrict(int dim, const int fine_m[3], const float* f, float* out, hipStream_t s) {
  const int cx = fine_m[0] / 2, cy = fine_m[1] / 2, cz = dim == 3 ? fine_m[2] / 2 : 1;
  const long long nc = (long long)cx * cy * cz;
  unsigned grid = (unsigned)((nc + kBlock - 1) / kBlock);
  if (dim == 3)
    hipLaunchKernelGGL(k_restrict<3>, dim3(grid), dim3(kBlock), 0, s, f, out, cx, cy, cz);
  else
    hipLaunchKernelGGL(k_restrict<2>, dim3(grid), dim3(kBlock), 0, s, f, out, cx, cy, cz);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_prolong(int dim, const int fine_m[3], int fields, const float* c, float* out, hipStream_t s) {
  const int cx = fine_m[0] / 2, cy = fine_m[1] / 2, cz = dim == 3 ? fine_m[2] / 2 : 1;
  const long long nf = (long long)fine_m[0] * fine_m[1] * (dim == 3 ? fine_m[2] : 1) * fields;
  unsigned grid = (unsigned)((nf + kBlock - 1) / kBlock);
  if (dim == 3)
    hipLaunchKernelGGL(k_prolong<3>, dim3(grid), dim3(kBlock), 0, s, c, out, cx, cy, cz, fields);
  else
    hipLaunchKernelGGL(k_prolong<2>, dim3(grid), dim3(kBlock), 0, s, c, out, cx, cy, cz, fields);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

}  // namespace lag

using namespace lag;

static bool even_grids(const lag_problem* p) {
  for (int a = 0; a < p->dim; ++a)
    if (p->img_m[a] % 2 || p->vel_m[a] % 2 || p->img_m[a] < 4 || p->vel_m[a] < 4) return false;
  return true;
}

static lag_problem coarser(const lag_problem* p) {
  lag_problem c = *p;
  for (int a = 0; a < p->dim; ++a) {
    c.img_m[a] /= 2;
    c.vel_m[a] /= 2;
  }
  return c;
}

extern "C" {

int lag_restrict_image(lag_plan P, const float* f, float* coarse, void* stream) {
  if (!P || !f || !coarse) return LAG_EINVAL;
  if (!even_grids(&P->prob)) return LAG_EINVAL;
  return launch_restrict(P->prob.dim, P->prob.img_m, f, coarse, (hipStream_t)stream);
}

int lag_prolong_velocity(lag_plan P, const float* v_coarse, float* v_fine, void* stream) {
  if (!P || !v_coarse || !v_fine) return LAG_EINVAL;
  if (!even_grids(&P->prob)) return LAG_EINVAL;
  return launch_prolong(P->prob.dim, P->prob.vel_m, P->fields, v_coarse, v_fine, (hipStream_t)stream);
}

int lag_resample_to_velocity_grid(lag_plan P, const float* f, float* out, void* stream) {
  if (!P || !f || !out) return LAG_EINVAL;
  const lag_problem& p = P->prob;
  for (int a = 0; a < p.dim; ++a)
    if (p.img_m[a] < p.vel_m[a]) return LAG_EINVAL;
  const int fz = p.dim == 3 ? p.img_m[2] : 1, cz = p.dim == 3 ? p.vel_m[2] : 1;
  const long long nc = (long long)p.vel_m[0] * p.vel_m[1] * cz;
  const unsigned grid = (unsigned)((nc + kBlock - 1) / kBlock);
  hipStream_t s = (hipStream_t)stream;
  if (p.dim == 3)
    hipLaunchKernelGGL(k_resample<3>, dim3(grid), dim3(kBlock), 0, s, f, out, p.img_m[0], p.img_m[1], fz,
                       p.vel_m[0], p.vel_m[1], cz);
  else
    hipLaunchKernelGGL(k_resample<2>, dim3(grid), dim3(kBlock), 0, s, f, out, p.img_m[0], p.img_m[1], fz,
                       p.vel_m[0], p.vel_m[1], cz);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int lag_multilevel_solve(const lag_problem* finest, int32_t levels, const float* T, const float* R, float* v,
                         const lag_gn_options* opt, lag_gn_info* infos, void* stream) {
  if (!finest || !T || !R || !v || levels < 1 || levels > 8) return LAG_EINVAL;
  int rc = lag_problem_check(finest);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::vector<lag_problem> probs(levels);
  probs[0] = *finest;  // index 0 = finest
  for (int l = 1; l < levels; ++l) {
    if (!even_grids(&probs[l - 1])) return LAG_EINVAL;
    probs[l] = coarser(&probs[l - 1]);
  }
  std::vector<lag_plan> plans(levels, nullptr);
  std::vector<float*> bufs;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (float* b : bufs) (void)hipFree(b);
    for (lag_plan p : plans)
      if (p) lag_plan_destroy(p);
  };
  auto alloc = [&](size_t n, float** out) -> int {
    if (hipMalloc((void**)out, n * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return LAG_ENOMEM;
    }
    bufs.push_back(*out);
    return LAG_OK;
  };
  std::vector<const float*> Ts(levels), Rs(levels);
  std::vector<float*> vs(levels);
  Ts[0] = T;
  Rs[0] = R;
  vs[0] = v;
  for (int l = 0; l < levels && rc == LAG_OK; ++l) {
    rc = lag_plan_create(&probs[l], &plans[l]);
    if (rc) break;
    if (l == 0) continue;
    int64_t np = 0, nu = 0;
    lag_problem_sizes(&probs[l], &np, &nu);
    float *t, *r, *vv;
    if ((rc = alloc(np, &t)) || (rc = alloc(np, &r)) || (rc = alloc(nu, &vv))) break;
    if ((rc = lag_restrict_image(plans[l - 1], Ts[l - 1], t, stream))) break;
    if ((rc = lag_restrict_image(plans[l - 1], Rs[l - 1], r, stream))) break;
    Ts[l] = t;
    Rs[l] = r;
    vs[l] = vv;
  }
  if (rc) {
    cleanup();
    return rc;
  }
  // coarse to fine
  int status = LAG_OK;
  for (int l = levels - 1; l >= 0; --l) {
    if (l == levels - 1) {
      if (l > 0) rc = launch_fill(vs[l], plans[l]->n_unknowns, 0.f, s);
    } else {
      rc = lag_prolong_velocity(plans[l], vs[l + 1], vs[l], stream);
    }
    if (rc) break;
    lag_gn_info info;
    rc = lag_gn_solve(plans[l], Ts[l], Rs[l], vs[l], opt, &info, stream);
    if (infos) infos[levels - 1 - l] = info;
    // a coarse level only provides the starting guess of the next one: a
    // stalled line search there hands over its last accepted iterate
    if (rc == LAG_ELINESEARCH) {
      if (l == 0) status = rc;
      rc = LAG_OK;
    }
    if (rc) break;
  }
  cleanup();
  return rc ? rc : status;
}

}  // extern "C"
