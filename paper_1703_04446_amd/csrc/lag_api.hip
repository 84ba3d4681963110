// C ABI of liblaglddmm: argument validation, plan management, the hot-path
// entry points and the native PCG / Gauss-Newton driver.

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "lag_internal.hpp"

namespace lag {

static thread_local std::string g_hip_error;

// Serialises the calls that must not overlap a stream capture on another
// thread: plan creation and destruction (allocations, synchronous copies)
// and the capture and instantiation of a graph.
std::mutex& api_lock() {
  static std::mutex m;
  return m;
}

int set_hip_error(hipError_t e) {
  g_hip_error = hipGetErrorString(e);
  return LAG_EHIP;
}

void set_hip_error_text(const char* msg) { g_hip_error = msg ? msg : ""; }

int launch_scale_mul(long long n, float c, const float* a, const float* w, float* out, hipStream_t s);
int launch_axpby(long long n, float a, const float* x, float b, const float* y, float* out, hipStream_t s);

// Lanes of one wave sit on a 4x4x4 (3-D) or 8x8 (2-D) lattice.
static void choose_bricks(lag_plan P, const int32_t* want) {
  const int D = P->geo.dim;
  lag::Bricks& B = P->bricks;
  // 16 x 16 x 12 bricks at the usual 2:1 image-to-velocity ratio keep the
  // fixed-point tile at 52 KB (three blocks per CU) and give few enough
  // bricks for one resident generation on 256 CUs at 128^3.
  int target[3] = {16, 16, D == 3 ? 12 : 1};
  if (want)
    for (int a = 0; a < D; ++a) target[a] = want[a];
  const size_t budget = 64 * 1024;
  int halo = D == 3 ? 3 : 4;
  for (int a = 0; a < 3; ++a) {
    if (a < D) {
      double r = (double)P->prob.img_m[a] / P->prob.vel_m[a];
      B.stride[a] = std::max(1, (int)lround(r));
    } else {
      B.stride[a] = 1;
    }
  }
  // Lane lattice of a wave (log2 extents, 64 lanes): 2-D 8 x 8; 3-D 4 x 4 x 4
  // or 8 x 4 x 2, the first whose regions divide the target on most axes.
  {
    const int lat3[2][3] = {{2, 2, 2}, {3, 2, 1}};
    const int lat2[3] = {3, 3, 0};
    int best = -1, best_fit = -1;
    for (int c = 0; c < (D == 3 ? 2 : 1); ++c) {
      const int* ls = D == 3 ? lat3[c] : lat2;
      int fit = 0;
      for (int a = 0; a < D; ++a) {
        const int rd = (1 << ls[a]) * B.stride[a];
        fit += target[a] >= rd && target[a] % rd == 0;
      }
      if (fit > best_fit) {
        best_fit = fit;
        best = c;
      }
    }
    for (int a = 0; a < 3; ++a) B.lsh[a] = D == 3 ? lat3[best][a] : lat2[a];
  }
  int lane[3], nreg[3];
  for (int a = 0; a < 3; ++a) {
    lane[a] = 1 << B.lsh[a];
    B.rdim[a] = lane[a] * B.stride[a];
    nreg[a] = a < D ? std::max(1, target[a] / B.rdim[a]) : 1;
  }
  for (;;) {
    int tvol = 1;
    for (int a = 0; a < 3; ++a) {
      B.bdim[a] = nreg[a] * B.rdim[a];
      if (a < D) {
        double ext = ceil((B.bdim[a] - 1) * P->geo.ratio[a]);
        B.tdim[a] = (int)ext + 3 + 2 * halo;
      } else {
        B.tdim[a] = 1;
      }
      tvol *= B.tdim[a];
    }
    // tile plus a few reduction slots
    size_t bytes = sizeof(float) * ((size_t)P->fields * tvol + 8);
    if (bytes <= budget) {
      B.tvol = tvol;
      break;
    }
    int amax = 0;
    for (int a = 1; a < D; ++a)
      if (nreg[a] > nreg[amax]) amax = a;
    if (nreg[amax] > 1) {
      nreg[amax] = (nreg[amax] + 1) / 2;
    } else if (halo > 1) {
      --halo;
    } else {
      B.tvol = tvol;  // smallest possible tile; exceeds the budget only for huge node counts
      break;
    }
  }
  // Pad the tile's row and plane strides so that the 64 lanes of a wave,
  // which start one velocity cell apart on the lane lattice, fall into
  // distinct LDS banks for the same corner/component (fewest lanes per bank
  // for 32 and for 64 banks, then smallest tile).
  {
    const int lat[3] = {lane[0], lane[1], lane[2]};
    auto worst = [&](int t0, int t1, int nb) {
      int cnt[64] = {0};
      int w = 0;
      for (int z = 0; z < lat[2]; ++z)
        for (int y = 0; y < lat[1]; ++y)
          for (int x = 0; x < lat[0]; ++x) {
            int b = (x + t0 * y + t0 * t1 * z) % nb;
            w = std::max(w, ++cnt[b]);
          }
      return w;
    };
    int best0 = B.tdim[0], best1 = B.tdim[1];
    long long bestkey = -1;
    const int span1 = D == 3 ? 32 : 1;
    // padding must not lower the number of blocks an LDS of 160 KB holds
    auto lds_bytes = [&](long long vol) { return sizeof(float) * ((size_t)P->fields * vol + 8); };
    const size_t cu_lds = 160 * 1024;
    const size_t fit0 = cu_lds / lds_bytes((long long)B.tdim[0] * B.tdim[1] * B.tdim[2]);
    for (int t0 = B.tdim[0]; t0 < B.tdim[0] + 32; ++t0)
      for (int t1 = B.tdim[1]; t1 < B.tdim[1] + span1; ++t1) {
        long long vol = (long long)t0 * t1 * B.tdim[2];
        const size_t bytes = lds_bytes(vol);
        if ((bytes > budget || cu_lds / bytes < fit0) && !(t0 == B.tdim[0] && t1 == B.tdim[1])) continue;
        long long key = ((long long)worst(t0, t1, 32) * 65 + worst(t0, t1, 64)) * (1LL << 32) + vol;
        if (bestkey < 0 || key < bestkey) {
          bestkey = key;
          best0 = t0;
          best1 = t1;
        }
      }
    B.tdim[0] = best0;
    B.tdim[1] = best1;
    B.tvol = B.tdim[0] * B.tdim[1] * B.tdim[2];
  }
  B.halo = halo;
  B.nbricks = 1;
  for (int a = 0; a < 3; ++a) {
    B.nreg[a] = nreg[a];
    B.nb[a] = a < D ? (P->prob.img_m[a] + B.bdim[a] - 1) / B.bdim[a] : 1;
    B.nbricks *= B.nb[a];
  }
}

static void free_plan(lag_plan P) {
  if (!P) return;
  void* ptrs[] = {P->pack_v, P->pack_p, P->st_j0[0], P->st_j0[1], P->st_th[0], P->st_th[1], P->reg_scale,
                  P->img_a, P->img_b, P->phi, P->bin_count, P->bin_start, P->bin_cursor, P->bin_items,
                  P->part_base, P->part_vals, P->scan_blocks, P->red_partial, P->red_partial2, P->scalars, P->fft_buf,
                  P->fft_tw[0], P->fft_tw[1], P->fft_tw[2], P->fft_lam[0], P->fft_lam[1], P->fft_lam[2],
                  P->fft_mu1, P->flags, P->tile_part, P->cover_start[0], P->cover_start[1],
                  P->cover_start[2], P->cover_ent[0], P->cover_ent[1], P->cover_ent[2], P->jac_vals,
                  P->jac_cell, P->jac_cnt, P->jac_max, P->jac_fb, P->pg_vals, P->pg_cells, P->pg_rows,
                  P->pg_npages, P->pg_order, P->pg_redo, P->dfr_list, P->dfr_hdr, P->dfr_acc, P->pg_axbox,
                  P->pgc_start[0], P->pgc_start[1], P->pgc_start[2], P->pgc_ent[0], P->pgc_ent[1],
                  P->pgc_ent[2]};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (P->ctl) (void)hipFree(P->ctl);
  if (P->ctl_host) (void)hipHostFree(P->ctl_host);
  if (P->sc_host) (void)hipHostFree(P->sc_host);
  if (P->pcg_exec) (void)hipGraphExecDestroy(P->pcg_exec);
  if (P->gstream) (void)hipStreamDestroy(P->gstream);
  for (hipEvent_t e : P->ctl_ev)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < 10; ++i)
    if (P->vec[i]) (void)hipFree(P->vec[i]);
  if (P->prof_on)
    for (int i = 0; i < 2 * 256; ++i) (void)hipEventDestroy(P->prof_ev[i]);
  delete P;
}

}  // namespace lag

using namespace lag;

#define LAG_CHECK(cond)          \
  do {                           \
    if (!(cond)) return LAG_EINVAL; \
  } while (0)

namespace lag {
int make_geo(const lag_problem* prob, Geo& g) {
  const int D = prob->dim;
  g = Geo{};
  g.dim = D;
  g.nodes = prob->nt_nodes;
  g.nsteps = prob->nsteps;
  g.np = 1;
  g.nv = 1;
  double cell = 1.0;
  for (int a = 0; a < 3; ++a) {
    g.mi[a] = a < D ? prob->img_m[a] : 1;
    g.mv[a] = a < D ? prob->vel_m[a] : 1;
    double L = a < D ? prob->extent[a] : 1.0;
    g.inv_hi[a] = (float)(g.mi[a] / L);
    g.inv_hv[a] = (float)(g.mv[a] / L);
    g.ratio[a] = (double)g.mv[a] / (double)g.mi[a];
    if (a < D) {
      g.np *= g.mi[a];
      g.nv *= g.mv[a];
      cell *= L / g.mi[a];
    }
  }
  g.cell_img = (float)cell;
  g.nvp = 1;
  for (int a = 0; a < 3; ++a) {
    g.pv[a] = a < D ? g.mv[a] + 1 : 1;
    g.nvp *= g.pv[a];
  }
  if (g.nvp >= (1LL << 31)) return LAG_EUNSUPPORTED;  // packed-field offsets are 32-bit
  return LAG_OK;
}
}  // namespace lag

static inline hipStream_t S(void* s) { return (hipStream_t)s; }

extern "C" {

const char* lag_strerror(int status) {
  switch (status) {
    case LAG_OK: return "ok";
    case LAG_EINVAL: return "invalid argument";
    case LAG_EUNSUPPORTED: return "unsupported problem or size";
    case LAG_EHIP: return "HIP runtime error";
    case LAG_ENOMEM: return "device allocation failed";
    case LAG_EBREAKDOWN: return "PCG breakdown (p^T H p <= 0)";
    case LAG_ELINESEARCH: return "Armijo line search failed";
    case LAG_ETOOLARGE: return "problem exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

const char* lag_last_hip_error(void) { return g_hip_error.c_str(); }

int lag_problem_check(const lag_problem* p) {
  LAG_CHECK(p);
  LAG_CHECK(p->dim == 2 || p->dim == 3);
  long long np = 1, nv = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < p->dim) {
      LAG_CHECK(p->img_m[a] >= 2 && p->img_m[a] <= (1 << 20));
      LAG_CHECK(p->vel_m[a] >= 2 && p->vel_m[a] <= (1 << 20));
      LAG_CHECK(p->extent[a] > 0.0 && isfinite(p->extent[a]));
      np *= p->img_m[a];
      nv *= p->vel_m[a];
    } else {
      LAG_CHECK(p->img_m[a] == 1 && p->vel_m[a] == 1);
    }
  }
  LAG_CHECK(p->nt_nodes >= 1 && p->nt_nodes <= 64);
  LAG_CHECK(p->model == LAG_TRANSPORT || p->model == LAG_CONTINUITY);
  LAG_CHECK(p->reg == LAG_DIFFUSION || p->reg == LAG_CURVATURE);
  LAG_CHECK(p->nsteps >= 1 && p->nsteps <= (1 << 16));
  LAG_CHECK(p->alpha >= 0.0 && isfinite(p->alpha));
  LAG_CHECK(p->gamma >= 0.0 && isfinite(p->gamma));
  LAG_CHECK(p->jac_blocks >= 0 && p->jac_blocks <= 255);
  LAG_CHECK(np <= 0x7fffffffLL);
  LAG_CHECK(nv * p->nt_nodes * p->dim <= 0x7fffffffLL);
  return LAG_OK;
}

int lag_problem_sizes(const lag_problem* p, int64_t* n_points, int64_t* n_unknowns) {
  int rc = lag_problem_check(p);
  if (rc) return rc;
  int64_t np = 1, nv = 1;
  for (int a = 0; a < p->dim; ++a) {
    np *= p->img_m[a];
    nv *= p->vel_m[a];
  }
  if (n_points) *n_points = np;
  if (n_unknowns) *n_unknowns = nv * p->dim * p->nt_nodes;
  return LAG_OK;
}

#define ALLOC(ptr, bytes)                                         \
  do {                                                            \
    if (hipMalloc((void**)&(ptr), (bytes)) != hipSuccess) {       \
      (void)hipGetLastError();                                    \
      lag::free_plan(P);                                          \
      return LAG_ENOMEM;                                          \
    }                                                             \
  } while (0)

#define HIPC(call)                                                \
  do {                                                            \
    hipError_t _e = (call);                                       \
    if (_e != hipSuccess) {                                       \
      lag::free_plan(P);                                          \
      return lag::set_hip_error(_e);                              \
    }                                                             \
  } while (0)

int lag_plan_create(const lag_problem* prob, lag_plan* out) { return lag_plan_create_tuned(prob, nullptr, out); }

static int plan_create_locked(const lag_problem* prob, const int32_t* brick_target, lag_plan* out);

int lag_plan_create_tuned(const lag_problem* prob, const int32_t* brick_target, lag_plan* out) {
  std::lock_guard<std::mutex> lk(api_lock());
  return plan_create_locked(prob, brick_target, out);
}

static int plan_create_locked(const lag_problem* prob, const int32_t* brick_target, lag_plan* out) {
  LAG_CHECK(out);
  *out = nullptr;
  if (brick_target && prob)
    for (int a = 0; a < prob->dim && a < 3; ++a) LAG_CHECK(brick_target[a] >= 1 && brick_target[a] <= 1024);
  int rc = lag_problem_check(prob);
  if (rc) return rc;
  lag_plan P = new lag_plan_s();
  P->prob = *prob;
  HIPC(hipGetDevice(&P->device));
  const int D = prob->dim;
  Geo& g = P->geo;
  rc = make_geo(prob, g);
  if (rc) {
    free_plan(P);
    return rc;
  }
  double cellv = 1.0;
  for (int a = 0; a < D; ++a) cellv *= prob->extent[a] / g.mv[a];
  P->fields = g.nodes * D;
  P->n_unknowns = (long long)P->fields * g.nv;
  choose_bricks(P, brick_target);
  {
    // the matrix-free adjoint kernels hold a 64-bit tile of the brick in LDS
    int max_lds = 0;
    HIPC(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device));
    if (adjoint_lds_bytes(P) > (size_t)max_lds) {
      free_plan(P);
      return LAG_EUNSUPPORTED;
    }
  }

  // time-node quadrature weights (trapezoid; 1 for a stationary field)
  const int nt = g.nodes - 1;
  for (int j = 0; j < g.nodes; ++j)
    P->node_w[j] = nt == 0 ? 1.0 : ((j == 0 || j == nt) ? 0.5 / nt : 1.0 / nt);
  std::vector<float> scale(2 * g.nodes);
  for (int j = 0; j < g.nodes; ++j) {
    scale[j] = (float)(prob->alpha * cellv * P->node_w[j]);
    scale[g.nodes + j] = (float)(cellv * P->node_w[j]);
  }
  ALLOC(P->reg_scale, sizeof(float) * 2 * g.nodes);
  HIPC(hipMemcpy(P->reg_scale, scale.data(), sizeof(float) * 2 * g.nodes, hipMemcpyHostToDevice));

  // RK4 stage tables (Algorithm 1: stage times t_k, t_k + dt/2, t_k + dt/2, t_k + dt)
  const int N = prob->nsteps;
  for (int k2 = 0; k2 < 2; ++k2) {
    const int dir = k2 == 0 ? -1 : 1;
    const double dt = (double)dir / N;
    const double t0 = dir > 0 ? 0.0 : 1.0;
    std::vector<int> j0(4 * N);
    std::vector<float> th(4 * N);
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    for (int k = 0; k < N; ++k) {
      const double tk = t0 + k * dt;
      for (int s = 0; s < 4; ++s) {
        double t = tk + cst[s] * dt;
        int jj = 0;
        double theta = 0.0;
        if (nt > 0) {
          jj = std::min((int)floor(t * nt), nt - 1);
          jj = std::max(jj, 0);
          theta = t * nt - jj;
        }
        j0[4 * k + s] = jj;
        th[4 * k + s] = (float)theta;
      }
    }
    ALLOC(P->st_j0[k2], sizeof(int) * 4 * N);
    ALLOC(P->st_th[k2], sizeof(float) * 4 * N);
    HIPC(hipMemcpy(P->st_j0[k2], j0.data(), sizeof(int) * 4 * N, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->st_th[k2], th.data(), sizeof(float) * 4 * N, hipMemcpyHostToDevice));
  }

  const size_t vec = D == 3 ? sizeof(float4) : sizeof(float2);
  ALLOC(P->pack_v, vec * g.nvp * g.nodes);
  ALLOC(P->pack_p, vec * g.nvp * g.nodes);
  ALLOC(P->img_a, sizeof(float) * g.np);
  ALLOC(P->img_b, sizeof(float) * g.np);
  ALLOC(P->phi, sizeof(float) * g.np * D);
  ALLOC(P->bin_count, sizeof(int) * (g.np + 1));
  ALLOC(P->bin_start, sizeof(int) * (g.np + 1));
  ALLOC(P->bin_cursor, sizeof(int) * g.np);
  ALLOC(P->bin_items, sizeof(int) * g.np);
  ALLOC(P->part_base, sizeof(int) * g.np);
  ALLOC(P->part_vals, sizeof(float) * g.np * (1 << D));
  ALLOC(P->scan_blocks, sizeof(int) * ((g.np + 1023) / 1024 + 2));
  ALLOC(P->red_partial, sizeof(double) * std::max<long long>(kRedBlocks, (P->n_unknowns + kBlock - 1) / kBlock));
  ALLOC(P->red_partial2, sizeof(double) * kRedBlocks);
  ALLOC(P->scalars, sizeof(double) * 32);
  HIPC(hipMemset(P->scalars, 0, sizeof(double) * 32));
  for (int i = 0; i < 10; ++i) ALLOC(P->vec[i], sizeof(float) * P->n_unknowns);
  ALLOC(P->flags, sizeof(int) * 4);
  HIPC(hipMemset(P->flags, 0, sizeof(int) * 4));
  ALLOC(P->dfr_list, sizeof(int) * g.np);
  ALLOC(P->dfr_hdr, sizeof(int) * 4);
  HIPC(hipMemset(P->dfr_hdr, 0, sizeof(int) * 4));
  ALLOC(P->dfr_acc, sizeof(unsigned long long) * (size_t)P->n_unknowns);
  HIPC(hipMemset(P->dfr_acc, 0, sizeof(unsigned long long) * (size_t)P->n_unknowns));
  if (prob->jac_blocks > 0 && prob->model == LAG_TRANSPORT && g.nodes == 1) {
    const lag::Bricks& B = P->bricks;
    P->jac_k = prob->jac_blocks;
    P->jac_slots = (long long)B.nbricks * B.bdim[0] * B.bdim[1] * B.bdim[2];
    const int nv4 = D == 3 ? 6 : 2;
    ALLOC(P->jac_vals, sizeof(float4) * (size_t)P->jac_k * nv4 * P->jac_slots);
    ALLOC(P->jac_cell, sizeof(int) * (size_t)P->jac_k * P->jac_slots);
    ALLOC(P->jac_cnt, (size_t)P->jac_slots);
    ALLOC(P->jac_max, sizeof(int) * 2);
    ALLOC(P->jac_fb, sizeof(float) * (size_t)P->n_unknowns);
    HIPC(hipMemset(P->jac_fb, 0, sizeof(float) * (size_t)P->n_unknowns));
    P->pg_cap = jac_pages_per_brick(P, P->jac_k);
    if (P->pg_cap > 0) {
      const size_t chunks = (size_t)B.nbricks * (size_t)P->pg_cap;
      ALLOC(P->pg_vals, sizeof(float4) * chunks * nv4 * 64);
      ALLOC(P->pg_cells, sizeof(int) * chunks * 64);
      ALLOC(P->pg_rows, sizeof(int) * chunks * 64);
      ALLOC(P->pg_npages, sizeof(int) * (size_t)B.nbricks);
      ALLOC(P->pg_order, sizeof(int) * pg_order_len(B.nbricks));
      ALLOC(P->pg_redo, sizeof(int));
      HIPC(hipMemset(P->pg_redo, 0, sizeof(int)));
    }
  }
  rc = tiles_setup(P);
  if (rc) {
    lag::free_plan(P);
    return rc;
  }
  rc = precond_setup(P);
  if (rc) {
    lag::free_plan(P);
    return rc;
  }
  HIPC(hipDeviceSynchronize());
  *out = P;
  return LAG_OK;
}

int lag_plan_destroy(lag_plan plan) {
  if (!plan) return LAG_OK;
  std::lock_guard<std::mutex> lk(api_lock());   // no capture runs while the device synchronises
  (void)hipDeviceSynchronize();
  lag::free_plan(plan);
  return LAG_OK;
}

int lag_profile_enable(lag_plan P, int32_t enable) {
  LAG_CHECK(P);
  if (enable && !P->prof_on) {
    for (int i = 0; i < 2 * 256; ++i) LAG_HIP(hipEventCreate(&P->prof_ev[i]));
    P->prof_on = 1;
  }
  P->prof_n = 0;
  return LAG_OK;
}

int lag_profile_read(lag_plan P, double* ms_total, int32_t* launches) {
  LAG_CHECK(P && ms_total && launches);
  *ms_total = 0.0;
  *launches = 0;
  if (!P->prof_on) return LAG_OK;
  for (int i = 0; i < P->prof_n; ++i) {
    LAG_HIP(hipEventSynchronize(P->prof_ev[2 * i + 1]));
    float ms = 0.f;
    LAG_HIP(hipEventElapsedTime(&ms, P->prof_ev[2 * i], P->prof_ev[2 * i + 1]));
    *ms_total += ms;
  }
  *launches = P->prof_n;
  P->prof_n = 0;
  return LAG_OK;
}

int lag_plan_problem(lag_plan plan, lag_problem* out) {
  LAG_CHECK(plan && out);
  *out = plan->prob;
  return LAG_OK;
}

int lag_adjoint_stats(lag_plan P, int32_t* deferred, int32_t* redone, void* stream) {
  LAG_CHECK(P);
  hipStream_t s = S(stream);
  int host[4] = {0, 0, 0, 0};
  LAG_HIP(hipMemcpyAsync(host, P->dfr_hdr, sizeof(host), hipMemcpyDeviceToHost, s));
  LAG_HIP(hipStreamSynchronize(s));
  if (deferred) *deferred = host[0];
  if (redone) *redone = host[2];
  return LAG_OK;
}

int lag_plan_flags(lag_plan P, int32_t* flags, int32_t clear, void* stream) {
  LAG_CHECK(P && flags);
  const hipStream_t s = S(stream);
  int host = 0;
  LAG_HIP(hipMemcpyAsync(&host, P->flags, sizeof(int), hipMemcpyDeviceToHost, s));
  LAG_HIP(hipStreamSynchronize(s));
  if (clear) LAG_HIP(hipMemsetAsync(P->flags, 0, sizeof(int), s));
  *flags = host;
  return LAG_OK;
}

int lag_trace(lag_plan P, const float* v, int32_t dir, float* phi, void* stream) {
  LAG_CHECK(P && v && phi && (dir == 1 || dir == -1));
  int rc = launch_pack(P, v, P->pack_v, S(stream));
  if (rc) return rc;
  return launch_trace(P, P->pack_v, dir, phi, S(stream));
}

int lag_transport(lag_plan P, const float* T, const float* phi, float* u, void* stream) {
  LAG_CHECK(P && T && phi && u);
  return launch_transport(P, T, phi, u, S(stream));
}

int lag_pushforward(lag_plan P, const float* T, const float* phi, float* u, void* stream) {
  LAG_CHECK(P && T && phi && u);
  return launch_pushforward(P, T, phi, u, S(stream));
}

int lag_jvp(lag_plan P, const float* v, const float* T, const float* dv, float* Jdv, void* stream) {
  LAG_CHECK(P && v && T && dv && Jdv);
  int rc = launch_pack(P, v, P->pack_v, S(stream));
  if (rc) return rc;
  P->packed_by_pcg = nullptr;
  if ((rc = launch_pack(P, dv, P->pack_p, S(stream)))) return rc;
  return launch_jvp(P, P->pack_v, P->pack_p, T, Jdv, S(stream));
}

int lag_vjp(lag_plan P, const float* v, const float* T, const float* w, float* JTw, void* stream) {
  LAG_CHECK(P && v && T && w && JTw);
  int rc = launch_pack(P, v, P->pack_v, S(stream));
  if (rc) return rc;
  return launch_vjp(P, P->pack_v, T, w, JTw, S(stream));
}

int gn_hessmat(lag_plan P, const float* v, const float* T, const float* wvox, const float* p, float* Hp,
               void* stream) {
  LAG_CHECK(P && v && T && p && Hp);
  hipStream_t s = S(stream);
  int rc = launch_pack(P, v, P->pack_v, s);
  if (rc) return rc;
  P->packed_by_pcg = nullptr;
  if ((rc = launch_pack(P, p, P->pack_p, s))) return rc;
  if (P->prob.model == LAG_TRANSPORT) {
    if ((rc = launch_fill(Hp, P->n_unknowns, 0.f, s))) return rc;
    if ((rc = launch_hess_transport(P, P->pack_v, P->pack_p, T, wvox, Hp, s))) return rc;
  } else {
    // J p on the image grid, weight by h^d W, then J^T
    if ((rc = launch_jvp(P, P->pack_v, P->pack_p, T, P->img_a, s))) return rc;
    if ((rc = launch_scale_mul(P->geo.np, P->geo.cell_img, P->img_a, wvox, P->img_b, s))) return rc;
    if ((rc = launch_vjp(P, P->pack_v, T, P->img_b, Hp, s))) return rc;
  }
  return launch_reg(P, p, Hp, /*accumulate=*/1, /*gamma=*/1, 1.f, s);
}

int spectral_precond_apply(lag_plan P, const float* r, float* z, void* stream) {
  LAG_CHECK(P && r && z);
  return launch_precond(P, r, z, S(stream));
}

int lag_reg_apply(lag_plan P, const float* p, float* out, void* stream) {
  LAG_CHECK(P && p && out);
  return launch_reg(P, p, out, 0, 1, 1.f, S(stream));
}

int lag_dot(lag_plan P, int64_t n, const float* x, const float* y, double* out, void* stream) {
  LAG_CHECK(P && x && y && out && n >= 0 && n <= 0x7fffffffLL);
  return launch_dot(P, n, x, y, out, S(stream));
}

}  // extern "C"

namespace lag {
__global__ void k_set(double* x, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *x = v;
}
}  // namespace lag

extern "C" {

// Objective (eq. SSD plus the regulariser) from the deformed template uu:
// out3 = {J, distance, regulariser}; wres = cell volume * (uu - R) when not
// null.
static int objective_from_image(lag_plan P, const float* v, const float* uu, const float* R, float* wres,
                                double* out3, hipStream_t s) {
  int rc;
  if ((rc = launch_ssd(P, uu, R, wres, P->geo.cell_img, out3 + 1, s))) return rc;
  if ((rc = launch_reg_energy(P, v, out3 + 2, s))) return rc;
  return launch_combine_J(out3, P->prob.alpha, s);
}

static int objective_full(lag_plan P, const float* v, const float* T, const float* R, float* u, float* wres,
                          double* out3, hipStream_t s) {
  const int dir = P->prob.model == LAG_TRANSPORT ? -1 : 1;
  int rc = launch_pack(P, v, P->pack_v, s);
  if (rc) return rc;
  if ((rc = launch_trace(P, P->pack_v, dir, P->phi, s))) return rc;
  float* uu = u ? u : P->img_a;
  if (P->prob.model == LAG_TRANSPORT) rc = launch_transport(P, T, P->phi, uu, s);
  else rc = launch_pushforward(P, T, P->phi, uu, s);
  if (rc) return rc;
  return objective_from_image(P, v, uu, R, wres, out3, s);
}

int lag_objective(lag_plan P, const float* v, const float* T, const float* R, float* u, double* out3,
                  void* stream) {
  LAG_CHECK(P && v && T && R);
  return objective_full(P, v, T, R, u, nullptr, out3 ? out3 : P->scalars + 8, S(stream));
}

int lag_gradient(lag_plan P, const float* v, const float* T, const float* R, float* g, double* out3,
                 void* stream) {
  LAG_CHECK(P && v && T && R && g);
  hipStream_t s = S(stream);
  int rc = objective_full(P, v, T, R, nullptr, P->img_b, out3 ? out3 : P->scalars + 8, s);
  if (rc) return rc;
  // pack_v still holds v
  if ((rc = launch_vjp(P, P->pack_v, T, P->img_b, g, s))) return rc;
  return launch_reg(P, v, g, 1, 0, 1.f, s);
}

// Gradient at v = 0: the characteristics do not move (the RK4 map of a zero
// field is the identity, phi = 0), so the trace is a fill and the adjoint
// sweep a sum of the RK4 weights at the start points; the regulariser of
// v = 0 adds nothing.
static int gradient_at_zero(lag_plan P, const float* T, const float* R, float* g, double* out3, hipStream_t s) {
  float* zero = P->vec[8];
  int rc = launch_fill(zero, P->n_unknowns, 0.f, s);
  if (rc) return rc;
  if ((rc = launch_fill(P->phi, P->geo.np * P->geo.dim, 0.f, s))) return rc;
  if (P->prob.model == LAG_TRANSPORT) rc = launch_transport(P, T, P->phi, P->img_a, s);
  else rc = launch_pushforward(P, T, P->phi, P->img_a, s);
  if (rc) return rc;
  if ((rc = objective_from_image(P, zero, P->img_a, R, P->img_b, out3, s))) return rc;
  return launch_vjp(P, nullptr, T, P->img_b, g, s, true);
}

int lag_gradient_at_zero(lag_plan P, const float* T, const float* R, float* g, double* out3, void* stream) {
  LAG_CHECK(P && T && R && g);
  return gradient_at_zero(P, T, R, g, out3 ? out3 : P->scalars + 8, S(stream));
}

// ---- assembled Jacobian ------------------------------------------------------

// Assemble J at v (launch only); with u != null also write the transported
// image T(phi).  jacobian_assembled() completes it from the block counts
// {largest per row, total} read back from P->jac_max.
static int jacobian_assemble_launch(lag_plan P, const float* v, const float* T, float* u, hipStream_t s) {
  P->jac_ready = 0;
  if (P->jac_k == 0) return LAG_EUNSUPPORTED;
  int rc = launch_pack(P, v, P->pack_v, s);
  if (rc) return rc;
  return launch_jac_assemble(P, P->pack_v, T, u, s);
}

static int32_t jacobian_assembled(lag_plan P, const int mx[2]) {
  P->jac_ready = mx[0] <= P->jac_k;
  P->jac_blocks_stored = mx[1];
  P->jac_max_seen = mx[0];
  return P->jac_ready;
}

static int jacobian_assemble(lag_plan P, const float* v, const float* T, float* u, int32_t* stored, hipStream_t s) {
  *stored = 0;
  int rc = jacobian_assemble_launch(P, v, T, u, s);
  if (rc) return rc;
  int mx[2] = {0, 0};
  LAG_HIP(hipMemcpyAsync(mx, P->jac_max, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  LAG_HIP(hipStreamSynchronize(s));
  *stored = jacobian_assembled(P, mx);
  return LAG_OK;
}

// Raise the capacity to hold rows of `need` blocks (plus a quarter of
// headroom, at most 255: a slot's count is one byte) when the new arrays fit
// in half of the free device memory beside the old ones.  Block k of a row
// lives at [k][...][slot] whatever the capacity, so only the value and cell
// arrays are replaced; a captured PCG graph holding their old addresses is
// dropped.  The caller's stream must be idle (hipFree waits for the device);
// the API lock keeps the allocation clear of another thread's graph capture.
// Returns true if the capacity grew; on an allocation failure the old arrays
// stay and the error is cleared.
static bool jacobian_grow(lag_plan P, int need) {
  if (P->jac_k == 0 || need <= P->jac_k || need > 255) return false;
  std::lock_guard<std::mutex> lk(api_lock());
  const int k = std::min(255, std::max(need, P->jac_k + (P->jac_k + 3) / 4));
  const int nv4 = P->geo.dim == 3 ? 6 : 2;
  const size_t vb = sizeof(float4) * (size_t)k * nv4 * (size_t)P->jac_slots;
  const size_t cb = sizeof(int) * (size_t)k * (size_t)P->jac_slots;
  size_t fr = 0, total = 0;
  if (hipMemGetInfo(&fr, &total) != hipSuccess || vb + cb > fr / 2) {
    (void)hipGetLastError();
    return false;
  }
  // the paged copy grows with the capacity (or is given up beyond 64 blocks
  // per row, where the products read the [k][slot] layout directly)
  const int pcap = jac_pages_per_brick(P, k);
  const size_t chunks = (size_t)P->bricks.nbricks * (size_t)pcap;
  const size_t pvb = sizeof(float4) * chunks * nv4 * 64, pcb = sizeof(int) * chunks * 64;
  if (vb + cb + pvb + 2 * pcb > fr / 2) return false;
  float4* nvals = nullptr;
  int* ncell = nullptr;
  float4* npv = nullptr;
  int *npc = nullptr, *npr = nullptr;
  bool ok = hipMalloc(&nvals, vb) == hipSuccess && hipMalloc(&ncell, cb) == hipSuccess;
  if (ok && pcap > 0)
    ok = hipMalloc(&npv, pvb) == hipSuccess && hipMalloc(&npc, pcb) == hipSuccess && hipMalloc(&npr, pcb) == hipSuccess;
  if (!ok) {
    for (void* q : {(void*)nvals, (void*)ncell, (void*)npv, (void*)npc, (void*)npr})
      if (q) (void)hipFree(q);
    (void)hipGetLastError();
    return false;
  }
  (void)hipFree(P->jac_vals);
  (void)hipFree(P->jac_cell);
  for (void* q : {(void*)P->pg_vals, (void*)P->pg_cells, (void*)P->pg_rows})
    if (q) (void)hipFree(q);
  P->jac_vals = nvals;
  P->jac_cell = ncell;
  P->pg_vals = npv;
  P->pg_cells = npc;
  P->pg_rows = npr;
  P->pg_cap = pcap;
  if (pcap > 0 && (!P->pg_npages || !P->pg_order || !P->pg_redo)) {
    const size_t nb = sizeof(int) * (size_t)P->bricks.nbricks;
    if ((!P->pg_npages && hipMalloc(&P->pg_npages, nb) != hipSuccess) ||
        (!P->pg_order && hipMalloc(&P->pg_order, sizeof(int) * pg_order_len(P->bricks.nbricks)) != hipSuccess) ||
        (!P->pg_redo && (hipMalloc(&P->pg_redo, sizeof(int)) != hipSuccess ||
                         hipMemset(P->pg_redo, 0, sizeof(int)) != hipSuccess))) {
      (void)hipGetLastError();
      P->pg_cap = 0;
    }
  }
  P->jac_k = k;
  if (P->pcg_exec) {
    (void)hipGraphExecDestroy(P->pcg_exec);
    P->pcg_exec = nullptr;
  }
  return true;
}

int lag_jacobian_assemble(lag_plan P, const float* v, const float* T, int32_t* stored, void* stream) {
  LAG_CHECK(P && v && T && stored);
  return jacobian_assemble(P, v, T, nullptr, stored, S(stream));
}

int lag_jacobian_info(lag_plan P, int64_t* blocks, int32_t* max_blocks, int32_t* bytes_per_block) {
  LAG_CHECK(P && blocks && max_blocks && bytes_per_block);
  *blocks = P->jac_ready ? P->jac_blocks_stored : 0;
  *max_blocks = P->jac_max_seen;
  *bytes_per_block = P->geo.dim == 3 ? 6 * 16 + 4 : 2 * 16 + 4;
  return LAG_OK;
}

// Assembled Gauss-Newton matvec; with part != null also the block partials
// of p . Hp (count in P->php_n), for PCG.
// Pack a direction into P->pack_p (clears the PCG's already-packed mark).
static int pack_direction(lag_plan P, const float* p, hipStream_t s) {
  P->packed_by_pcg = nullptr;
  return launch_pack(P, p, P->pack_p, s);
}

static int hessmat_assembled(lag_plan P, const float* wvox, const float* p, float* Hp, double* part, hipStream_t s) {
  int rc = LAG_OK;
  // the PCG update leaves its direction packed (k_pcg_p_pack); others pack here
  if (P->packed_by_pcg != p && (rc = pack_direction(P, p, s))) return rc;
  const RegTail rt = reg_tail(P, p, 1, 1.f, part);  // + alpha A p + gamma p, fused into the tile reduction
  return launch_jac_apply(P, P->pack_p, wvox, nullptr, P->geo.cell_img, Hp, s, &rt);
}

int gn_hessmat_assembled(lag_plan P, const float* wvox, const float* p, float* Hp, void* stream) {
  LAG_CHECK(P && p && Hp && P->jac_ready);
  return hessmat_assembled(P, wvox, p, Hp, nullptr, S(stream));
}

// Matrix-free Gauss-Newton matvec; with part != null also the block
// partials of p . Hp (count in P->php_n), for PCG.
static int hessmat_free(lag_plan P, const float* v, const float* T, const float* wvox, const float* p, float* Hp,
                        double* part, hipStream_t s) {
  int rc = gn_hessmat(P, v, T, wvox, p, Hp, s);
  if (rc || !part) return rc;
  const long long n = P->n_unknowns;
  if ((rc = launch_dot_partial(P, n, p, Hp, part, s))) return rc;
  P->php_n = (int)std::min<long long>(kRedBlocks, std::max<long long>(1, (n + kBlock - 1) / kBlock));
  return LAG_OK;
}

int lag_vjp_assembled(lag_plan P, const float* w, float* JTw, void* stream) {
  LAG_CHECK(P && w && JTw && P->jac_ready);
  return launch_jac_apply(P, P->pack_p, nullptr, w, 1.f, JTw, S(stream), nullptr);
}

// Objective and gradient with the stored Jacobian; u = T(phi) at v when the
// assembly already produced it, else traced here.
static int gradient_assembled(lag_plan P, const float* v, const float* T, const float* R, const float* u, float* g,
                              double* out3, hipStream_t s) {
  int rc = u ? objective_from_image(P, v, u, R, P->img_b, out3, s)
             : objective_full(P, v, T, R, nullptr, P->img_b, out3, s);
  if (rc) return rc;
  const RegTail rt = reg_tail(P, v, 0, 1.f, nullptr);  // + alpha A v, fused into the tile reduction
  return launch_jac_apply(P, P->pack_p, nullptr, P->img_b, 1.f, g, s, &rt);
}

int lag_gradient_assembled(lag_plan P, const float* v, const float* T, const float* R, float* g, double* out3,
                           void* stream) {
  LAG_CHECK(P && v && T && R && g && P->jac_ready);
  hipStream_t s = S(stream);
  return gradient_assembled(P, v, T, R, nullptr, g, out3 ? out3 : P->scalars + 8, s);
}

// ---- PCG / Gauss-Newton ------------------------------------------------------

static int read_scalars(lag_plan P, double* host, int off, int cnt, hipStream_t s) {
  LAG_HIP(hipMemcpyAsync(host, P->scalars + off, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  LAG_HIP(hipStreamSynchronize(s));
  return LAG_OK;
}

}  // extern "C"

// PCG control block (device flags, pinned host mirrors, capture stream, copy
// events), allocated on a plan's first PCG call.
static int ensure_pcg_ctl(lag_plan P) {
  if (P->ctl && P->ctl_ev[1]) return LAG_OK;
  std::lock_guard<std::mutex> lk(api_lock());
  if (!P->ctl_host) LAG_HIP(hipHostMalloc((void**)&P->ctl_host, sizeof(int) * 16, hipHostMallocDefault));
  if (!P->sc_host) LAG_HIP(hipHostMalloc((void**)&P->sc_host, sizeof(double) * 16, hipHostMallocDefault));
  if (!P->gstream) LAG_HIP(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
  for (int k = 0; k < 2; ++k)
    if (!P->ctl_ev[k]) LAG_HIP(hipEventCreateWithFlags(&P->ctl_ev[k], hipEventDisableTiming));
  if (!P->ctl) LAG_HIP(hipMalloc((void**)&P->ctl, sizeof(int) * 8));
  return LAG_OK;
}

// Options of an internal PCG call: bb >= 0 is b.b, known to the caller (no
// synchronisation for it); with gdot != null the final read also returns
// gdx = gdot . x.
struct PcgExtra {
  double bb = -1.0;
  const float* gdot = nullptr;
  double gdx = 0.0;
  // enqueued after the solve and before its last read (which then returns
  // scalars 0..15); set to true when it ran
  std::function<int(hipStream_t)> before_read;
  bool ran = false;
};

// PCG start: x = 0, r = b, z = M r, p = z, device scalars and control block
// (sc[0] = r.z, sc[3] = r.r, sc[4] = breakdown flag, sc[5] = b.b, sc[6] =
// tol^2 b.b).  Synchronises once for |b| unless the caller knows it; *nb = 0
// means b = 0 (nothing else launched).
static int pcg_start(lag_plan P, const float* b, float* x, double tol, int32_t maxit, double* nb, hipStream_t s,
                     const PcgExtra* ex) {
  const long long n = P->n_unknowns;
  float *r = P->vec[3], *z = P->vec[4], *p = P->vec[5];
  double* sc = P->scalars;
  int rc;
  P->packed_by_pcg = nullptr;  // p is rewritten below
  if ((rc = launch_fill(x, n, 0.f, s))) return rc;
  if ((rc = launch_axpby(n, 1.f, b, 0.f, nullptr, r, s))) return rc;
  hipLaunchKernelGGL(lag::k_set, dim3(1), dim3(64), 0, s, sc + 4, 0.0);
  LAG_LAUNCH_CHECK();
  double bb;
  if (ex && ex->bb >= 0.0) {
    bb = ex->bb;
  } else {
    if ((rc = launch_dot(P, n, b, b, sc + 5, s))) return rc;
    LAG_HIP(hipMemcpyAsync(P->sc_host, sc, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
    LAG_HIP(hipStreamSynchronize(s));
    bb = P->sc_host[5];
  }
  *nb = sqrt(bb);
  if (*nb == 0.0) return LAG_OK;
  if ((rc = launch_precond(P, r, z, s))) return rc;
  if ((rc = launch_dot(P, n, r, z, sc + 0, s))) return rc;
  if ((rc = launch_axpby(n, 1.f, z, 0.f, nullptr, p, s))) return rc;
  if (ex && ex->bb >= 0.0) {  // r = b: r.r is the caller's b.b
    hipLaunchKernelGGL(lag::k_set, dim3(1), dim3(64), 0, s, sc + 3, bb);
    LAG_LAUNCH_CHECK();
  } else if ((rc = launch_dot(P, n, r, r, sc + 3, s))) {
    return rc;
  }
  hipLaunchKernelGGL(lag::k_set, dim3(1), dim3(64), 0, s, sc + 6, tol * tol * bb);
  LAG_LAUNCH_CHECK();
  return launch_pcg_ctl_init(P->ctl, sc, maxit, s);
}

// One PCG iteration on stream g (alpha, beta and the stopping test on the
// device; every kernel returns at entry once ctl[0] is set).
template <class Op>
static int pcg_iteration(lag_plan P, Op& H, float* x, hipStream_t g) {
  float *r = P->vec[3], *z = P->vec[4], *p = P->vec[5], *Hp = P->vec[6];
  int rc;
  if ((rc = H(p, Hp, g, P->red_partial))) return rc;      // also the p.Hp partials (P->php_n)
  if ((rc = launch_pcg_xr(P, x, r, p, Hp, g))) return rc;   // also r.r partials
  if ((rc = launch_precond(P, r, z, g, P->red_partial, &P->rz_n))) return rc;  // also the r.z partials
  if ((rc = launch_pcg_p(P, p, z, g))) return rc;
  return launch_pcg_check(P, g);
}

// Read the control block and scalars after the last iteration (and, with
// ex->gdot, gdot . x into ex->gdx in the same read).
static int pcg_finish(lag_plan P, double nb, const float* x, lag_pcg_info* info, hipStream_t s, PcgExtra* ex) {
  int nsc = 6;
  if (ex && ex->gdot) {
    const int rc = launch_dot(P, P->n_unknowns, ex->gdot, x, P->scalars + 12, s);
    if (rc) return rc;
    nsc = 13;
  }
  if (ex && ex->before_read) {
    const int rc = ex->before_read(s);
    if (rc) return rc;
    ex->ran = true;
    nsc = 16;
  }
  LAG_HIP(hipMemcpyAsync(P->ctl_host, P->ctl, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
  LAG_HIP(hipMemcpyAsync(P->sc_host, P->scalars, sizeof(double) * nsc, hipMemcpyDeviceToHost, s));
  LAG_HIP(hipStreamSynchronize(s));
  if (ex && ex->gdot) ex->gdx = P->sc_host[12];
  lag_pcg_info loc;
  loc.iters = P->ctl_host[1];
  loc.breakdown = P->ctl_host[0] == 2;
  loc.matvecs = loc.iters + (loc.breakdown ? 1 : 0);
  loc.relres = sqrt(P->sc_host[3]) / nb;
  if (info) *info = loc;
  return loc.breakdown ? LAG_EBREAKDOWN : LAG_OK;
}

// Preconditioned CG with the Gauss-Newton operator `H` (a callable
// H(p, Hp, stream) -> status), launched eagerly.  The stopping test runs on
// the device, so the host enqueues iteration k + 1 before it reads the
// control block of iteration k: the GPU does not wait for the host between
// iterations, and at most one enqueued iteration finds the halt flag set and
// does nothing.  When the residual trend says iteration k will meet the
// tolerance, the host waits for it instead of enqueuing k + 1 (scheduling
// only; the arithmetic is the same).  Timed matvec launches of an iteration
// that found the halt flag set are dropped.
template <class Op>
static int pcg_impl(lag_plan P, Op H, const float* b, float* x, double tol, int32_t maxit, lag_pcg_info* info,
                    hipStream_t s, PcgExtra* ex = nullptr) {
  int rc;
  if ((rc = ensure_pcg_ctl(P))) return rc;
  double nb = 0.0;
  if ((rc = pcg_start(P, b, x, tol, maxit, &nb, s, ex))) return rc;
  if (nb == 0.0) {  // x = 0
    if (info) *info = lag_pcg_info{0, 0, 0, 0.0};
    if (ex) ex->gdx = 0.0;
    return LAG_OK;
  }
  std::vector<int> prof_at;
  prof_at.reserve(maxit > 0 ? maxit : 0);
  int enq = 0;
  const double thresh = tol * tol * nb * nb;
  double rr_prev = nb * nb;  // r.r after iteration it - 2 (b.b before the first)
  auto wait_slot = [&](int slot, bool* stop, double* rr) {
    const hipError_t e = hipEventSynchronize(P->ctl_ev[slot]);
    if (e != hipSuccess) return set_hip_error(e);
    const int* c = P->ctl_host + 8 * slot;
    *stop = c[0] != 0;
    *rr = reinterpret_cast<const double*>(c)[2];
    return (int)LAG_OK;
  };
  P->geo.halt = P->ctl;
  for (int it = 0; it < maxit; ++it) {
    prof_at.push_back(P->prof_n);
    const int slot = it & 1;
    P->ctl_mirror = P->ctl_host + 8 * slot;   // the check writes this iteration's control block there
    rc = pcg_iteration(P, H, x, s);
    P->ctl_mirror = nullptr;
    if (rc) break;
    ++enq;
    if (hipEventRecord(P->ctl_ev[slot], s) != hipSuccess) {
      rc = set_hip_error(hipGetLastError());
      break;
    }
    if (it == 0) continue;
    bool stop = false;
    double rr = 0.0;
    if ((rc = wait_slot(slot ^ 1, &stop, &rr)) || stop) break;
    // r.r after iteration it, extrapolated from the last ratio: when it
    // comes within a factor 2 of the tolerance (residuals fall unevenly),
    // wait for iteration it instead of enqueuing it + 1
    const bool likely = rr_prev > 0.0 && rr * (rr / rr_prev) <= 4.0 * thresh;
    rr_prev = rr;
    if (likely && ((rc = wait_slot(slot, &stop, &rr)) || stop)) break;
  }
  P->geo.halt = nullptr;
  if (rc) return rc;
  rc = pcg_finish(P, nb, x, info, s, ex);
  const int ran = P->ctl_host[1] + (P->ctl_host[0] == 2 ? 1 : 0);
  if (ran < enq && P->prof_n > prof_at[ran]) P->prof_n = prof_at[ran];
  return rc;
}

// Graph-captured PCG: the iteration of pcg_impl, `per_graph` iterations per
// graph, built once per plan and argument set (key) and replayed; the host
// reads the control block after each replay, i.e. once per `per_graph`
// iterations.  The captured kernels take only the plan's buffers and the
// pointers in `key`, so a replay is valid while those are unchanged.
template <class Op>
static int pcg_graph_impl(lag_plan P, Op H, const void* const key[6], int mode, const float* b, float* x,
                          double tol, int32_t maxit, int32_t per_graph, lag_pcg_info* info, hipStream_t s,
                          PcgExtra* ex = nullptr) {
  int rc;
  if ((rc = ensure_pcg_ctl(P))) return rc;
  double nb = 0.0;
  if ((rc = pcg_start(P, b, x, tol, maxit, &nb, s, ex))) return rc;
  if (nb == 0.0) {  // x = 0
    if (info) *info = lag_pcg_info{0, 0, 0, 0.0};
    if (ex) ex->gdx = 0.0;
    return LAG_OK;
  }
  // (re)capture when the arguments differ from the cached graph's
  bool same = P->pcg_exec && P->pcg_key_i[0] == mode && P->pcg_key_i[1] == per_graph;
  for (int k = 0; k < 6 && same; ++k) same = P->pcg_key[k] == key[k];
  if (!same) {
    std::lock_guard<std::mutex> lk(api_lock());
    if (P->pcg_exec) {
      (void)hipGraphExecDestroy(P->pcg_exec);
      P->pcg_exec = nullptr;
    }
    hipStream_t g = P->gstream;
    LAG_HIP(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal));
    P->geo.halt = P->ctl;
    P->capturing = 1;
    int crc = LAG_OK;
    for (int u = 0; u < per_graph && crc == LAG_OK; ++u) crc = pcg_iteration(P, H, x, g);
    P->geo.halt = nullptr;
    P->capturing = 0;
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(g, &graph);
    if (crc != LAG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return crc;
    }
    if (ce != hipSuccess) return set_hip_error(ce);
    const hipError_t ie = hipGraphInstantiate(&P->pcg_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      P->pcg_exec = nullptr;
      return set_hip_error(ie);
    }
    for (int k = 0; k < 6; ++k) P->pcg_key[k] = key[k];
    P->pcg_key_i[0] = mode;
    P->pcg_key_i[1] = per_graph;
  }
  // replay until the device says stop (bounded by the iteration cap); as in
  // pcg_impl, replay l + 1 is enqueued before the control block of replay l
  // is read
  const int launches = (maxit + per_graph - 1) / per_graph;
  for (int l = 0; l < launches; ++l) {
    const int slot = l & 1;
    LAG_HIP(hipGraphLaunch(P->pcg_exec, s));
    LAG_HIP(hipMemcpyAsync(P->ctl_host + 8 * slot, P->ctl, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    LAG_HIP(hipEventRecord(P->ctl_ev[slot], s));
    if (l > 0) {
      LAG_HIP(hipEventSynchronize(P->ctl_ev[slot ^ 1]));
      if (P->ctl_host[8 * (slot ^ 1)] != 0) break;
    }
  }
  return pcg_finish(P, nb, x, info, s, ex);
}

extern "C" {

int lag_pcg(lag_plan P, const float* v, const float* T, const float* wvox, const float* b, float* x, double tol,
            int32_t maxit, lag_pcg_info* info, void* stream) {
  LAG_CHECK(P && v && T && b && x && maxit >= 0 && tol >= 0.0);
  auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
    return hessmat_free(P, v, T, wvox, p, Hp, part, st);
  };
  return pcg_impl(P, H, b, x, tol, maxit, info, S(stream));
}

int lag_pcg_graph(lag_plan P, const float* v, const float* T, const float* wvox, const float* b, float* x,
                  double tol, int32_t maxit, int32_t iters_per_graph, lag_pcg_info* info, void* stream) {
  LAG_CHECK(P && v && T && b && x && maxit >= 0 && tol >= 0.0 && iters_per_graph >= 1 && iters_per_graph <= 64);
  auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
    return hessmat_free(P, v, T, wvox, p, Hp, part, st);
  };
  const void* key[6] = {v, T, wvox, b, x, nullptr};
  return pcg_graph_impl(P, H, key, 0, b, x, tol, maxit, iters_per_graph, info, S(stream));
}

int lag_pcg_assembled(lag_plan P, const float* wvox, const float* b, float* x, double tol, int32_t maxit,
                      lag_pcg_info* info, void* stream) {
  LAG_CHECK(P && b && x && maxit >= 0 && tol >= 0.0 && P->jac_ready);
  auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
    return hessmat_assembled(P, wvox, p, Hp, part, st);
  };
  return pcg_impl(P, H, b, x, tol, maxit, info, S(stream));
}

int lag_pcg_assembled_graph(lag_plan P, const float* wvox, const float* b, float* x, double tol, int32_t maxit,
                            int32_t iters_per_graph, lag_pcg_info* info, void* stream) {
  LAG_CHECK(P && b && x && maxit >= 0 && tol >= 0.0 && P->jac_ready && iters_per_graph >= 1 &&
            iters_per_graph <= 64);
  auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
    return hessmat_assembled(P, wvox, p, Hp, part, st);
  };
  const void* key[6] = {nullptr, nullptr, wvox, b, x, nullptr};
  return pcg_graph_impl(P, H, key, 1, b, x, tol, maxit, iters_per_graph, info, S(stream));
}

void lag_gn_default_options(lag_gn_options* o) {
  if (!o) return;
  o->gtol = 1e-2;
  o->max_gn = 50;
  o->pcg_tol = 0.1;
  o->pcg_maxit = 50;
  o->armijo_c1 = 1e-4;
  o->max_halvings = 10;
  o->graph_iters = 0;
}

// The Gauss-Newton step's PCG solve (assembled or matrix-free, eager or
// graph-replayed) with the step's extras (known b.b, g . dv in the last read).
static int gn_pcg(lag_plan P, bool stored, const float* v, const float* T, const float* b, float* x,
                  const lag_gn_options& o, lag_pcg_info* pi, hipStream_t s, PcgExtra* ex) {
  if (stored) {
    auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
      return hessmat_assembled(P, nullptr, p, Hp, part, st);
    };
    if (o.graph_iters > 0) {
      const void* key[6] = {nullptr, nullptr, nullptr, b, x, nullptr};
      return pcg_graph_impl(P, H, key, 1, b, x, o.pcg_tol, o.pcg_maxit, o.graph_iters, pi, s, ex);
    }
    return pcg_impl(P, H, b, x, o.pcg_tol, o.pcg_maxit, pi, s, ex);
  }
  auto H = [&](const float* p, float* Hp, hipStream_t st, double* part) {
    return hessmat_free(P, v, T, nullptr, p, Hp, part, st);
  };
  if (o.graph_iters > 0) {
    const void* key[6] = {v, T, nullptr, b, x, nullptr};
    return pcg_graph_impl(P, H, key, 0, b, x, o.pcg_tol, o.pcg_maxit, o.graph_iters, pi, s, ex);
  }
  return pcg_impl(P, H, b, x, o.pcg_tol, o.pcg_maxit, pi, s, ex);
}

int lag_gn_step(lag_plan P, const float* T, const float* R, const float* v, float* v_next,
                const lag_gn_options* opt, double gstop, lag_gn_step_info* info, void* stream) {
  LAG_CHECK(P && T && R && v && v_next && v != v_next);
  lag_gn_options o;
  lag_gn_default_options(&o);
  if (opt) o = *opt;
  LAG_CHECK(o.pcg_maxit >= 0 && o.max_halvings >= 0 && o.graph_iters >= 0 && o.graph_iters <= 64);
  hipStream_t s = S(stream);
  const long long n = P->n_unknowns;
  float *g = P->vec[0], *rhs = P->vec[1], *dv = P->vec[2];
  double* sc = P->scalars;
  double h[8];
  lag_gn_step_info loc;
  memset(&loc, 0, sizeof(loc));
  int rc;
  int32_t stored = 0;
  if (P->jac_k > 0) {
    // Assemble J and take the gradient from it without waiting for the
    // overflow check, which is read back with the objective (the stored
    // counts never exceed the capacity, so the speculative product stays in
    // bounds); on overflow the gradient is redone matrix-free.  The
    // assembly's forward pass leaves T(phi) at v in img_a: no second trace.
    // After an overflow the capacity grows once to the largest row seen and
    // the assembly is repeated; without room the step runs matrix-free.
    for (int attempt = 0; attempt < 2 && !stored; ++attempt) {
      int mx[2] = {0, 0};
      if ((rc = jacobian_assemble_launch(P, v, T, P->img_a, s))) return rc;
      if ((rc = gradient_assembled(P, v, T, R, P->img_a, g, sc + 8, s))) return rc;
      if ((rc = launch_dot(P, n, g, g, sc + 11, s))) return rc;
      LAG_HIP(hipMemcpyAsync(mx, P->jac_max, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
      if ((rc = read_scalars(P, h, 8, 4, s))) return rc;
      stored = jacobian_assembled(P, mx);
      if (!stored && (attempt > 0 || !jacobian_grow(P, mx[0]))) break;
    }
  }
  if (!stored) {
    if ((rc = lag_gradient(P, v, T, R, g, sc + 8, stream))) return rc;
    if ((rc = launch_dot(P, n, g, g, sc + 11, s))) return rc;
    if ((rc = read_scalars(P, h, 8, 4, s))) return rc;
  }
  loc.assembled = stored;
  loc.J = h[0];
  loc.gnorm = sqrt(h[3]);
  loc.J_next = loc.J;
  if (loc.gnorm <= gstop) {
    loc.stopped = 1;
    if (info) *info = loc;
    return launch_axpby(n, 1.f, v, 0.f, nullptr, v_next, s);
  }
  if ((rc = launch_axpby(n, -1.f, g, 0.f, nullptr, rhs, s))) return rc;
  lag_pcg_info pi;
  PcgExtra ex;
  ex.bb = h[3];   // rhs = -g: rhs . rhs = g . g exactly
  ex.gdot = g;    // slope g . dv, read with the solver's last scalars
  // the line search's first trial (mu = 1) is enqueued before that read too
  ex.before_read = [&](hipStream_t st) {
    int r2 = launch_axpby(n, 1.f, v, 1.f, dv, v_next, st);
    if (r2) return r2;
    return objective_full(P, v_next, T, R, nullptr, nullptr, sc + 13, st);
  };
  rc = gn_pcg(P, stored != 0, v, T, rhs, dv, o, &pi, s, &ex);
  if (rc != LAG_OK && rc != LAG_EBREAKDOWN) return rc;
  loc.pcg_iters = pi.iters;
  loc.matvecs = pi.matvecs;
  const double slope = ex.gdx;
  double mu = 1.0;
  for (int k = 0; k <= o.max_halvings; ++k) {
    if (k == 0 && ex.ran) {
      h[5] = P->sc_host[13];
    } else {
      if ((rc = launch_axpby(n, 1.f, v, (float)mu, dv, v_next, s))) return rc;
      if ((rc = objective_full(P, v_next, T, R, nullptr, nullptr, sc + 13, s))) return rc;
      if ((rc = read_scalars(P, h + 5, 13, 1, s))) return rc;
    }
    if (h[5] <= loc.J + o.armijo_c1 * mu * slope) {
      loc.accepted = 1;
      loc.J_next = h[5];
      loc.mu = mu;
      break;
    }
    loc.halvings = k + 1;
    mu *= 0.5;
  }
  if (!loc.accepted) {
    if (info) *info = loc;
    if ((rc = launch_axpby(n, 1.f, v, 0.f, nullptr, v_next, s))) return rc;
    return LAG_ELINESEARCH;
  }
  if (info) *info = loc;
  return LAG_OK;
}

int lag_gn_solve(lag_plan P, const float* T, const float* R, float* v, const lag_gn_options* opt,
                 lag_gn_info* info, void* stream) {
  LAG_CHECK(P && T && R && v);
  lag_gn_options o;
  lag_gn_default_options(&o);
  if (opt) o = *opt;
  LAG_CHECK(o.max_gn >= 0 && o.pcg_maxit >= 0 && o.max_halvings >= 0 && o.gtol >= 0.0 && o.graph_iters >= 0 &&
            o.graph_iters <= 64);
  hipStream_t s = S(stream);
  const long long n = P->n_unknowns;
  float *g = P->vec[0], *vn = P->vec[7];
  double* sc = P->scalars;
  double h[8];
  lag_gn_info loc;
  memset(&loc, 0, sizeof(loc));
  int rc;
  // reference gradient norm at v = 0; a start at v = 0 takes it from the
  // first step's own gradient (the step then stops only if g = 0, or
  // always if gtol >= 1, as |g| <= gtol |g| would)
  if ((rc = launch_dot(P, n, v, v, sc + 16, s))) return rc;
  if ((rc = read_scalars(P, h, 16, 1, s))) return rc;
  const bool from_zero = h[0] == 0.0;
  if (!from_zero) {
    if ((rc = gradient_at_zero(P, T, R, g, sc + 8, s))) return rc;
    if ((rc = launch_dot(P, n, g, g, sc + 11, s))) return rc;
    if ((rc = read_scalars(P, h, 8, 4, s))) return rc;
    loc.g0 = sqrt(h[3]);
  }
  double gstop = o.gtol * loc.g0;
  int status = LAG_OK;
  for (int it = 0; it <= o.max_gn; ++it) {
    lag_gn_step_info si;
    // the last pass only evaluates the gradient (gstop = +inf)
    double stop_here = it == o.max_gn ? 1e300 : gstop;
    if (it == 0 && from_zero && it != o.max_gn) stop_here = o.gtol >= 1.0 ? 1e300 : 0.0;
    rc = lag_gn_step(P, T, R, v, vn, &o, stop_here, &si, stream);
    if (rc != LAG_OK && rc != LAG_ELINESEARCH) return rc;
    if (it == 0 && from_zero) {
      loc.g0 = si.gnorm;
      gstop = o.gtol * loc.g0;
    }
    if (it == 0) loc.J0 = si.J;
    loc.J = si.J;
    loc.gnorm = si.gnorm;
    if (si.stopped) {
      loc.converged = si.gnorm <= gstop;
      break;
    }
    loc.iters = it + 1;
    loc.pcg_iters += si.pcg_iters;
    loc.matvecs += si.matvecs;
    if (rc == LAG_ELINESEARCH) {
      status = LAG_ELINESEARCH;
      break;
    }
    if ((rc = launch_axpby(n, 1.f, vn, 0.f, nullptr, v, s))) return rc;
    loc.J = si.J_next;
  }
  if (info) *info = loc;
  return status;
}

}  // extern "C"

// ---- many pairs in lockstep, PCG of the whole batch as one graph ----------

namespace lag {

// Word 0 (the halt flag) of many plans' PCG control blocks, gathered.
__global__ void k_gather_ctl(const int* const* ctl, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ctl[i][0];
}

// Halt a plan's PCG: its iterations in a replayed graph return at entry.
__global__ void k_halt_ctl(int* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl[0] = 3;
}

}  // namespace lag

namespace {

constexpr int kBatchStreams = 4;  // hardware queues HIP gives one process

// The Gauss-Newton operator of one pair, assembled or matrix-free.
struct BatchOp {
  lag_plan P;
  const float* v;
  const float* T;
  int assembled;
  int operator()(const float* p, float* Hp, hipStream_t s, double* part) const {
    return assembled ? hessmat_assembled(P, nullptr, p, Hp, part, s) : hessmat_free(P, v, T, nullptr, p, Hp, part, s);
  }
};

struct BatchPair {
  lag_plan P = nullptr;
  int active = 1;
  int in_graph = 0;      // has iterations in the current batch graph
  int stored = 0;        // this step's gradient and operator use the assembled Jacobian
  int graph_mode = -1;   // operator captured in the batch graph (-1: none)
  int graph_gen = -1;    // Jacobian storage generation captured
  int gen = 0;           // bumped when the Jacobian storage is reallocated
  bool from_zero = true;
  double gstop = 0.0, slope = 0.0, mu = 1.0;
  int status = LAG_OK;
  lag_gn_info info{};
};

}  // namespace

extern "C" {

int lag_batch_solve_graph(int32_t npairs, const lag_problem* probs, const float* const* T, const float* const* R,
                          float* const* v, const lag_gn_options* opt, const int32_t* bricks, lag_gn_info* infos,
                          int32_t* status) {
  if (npairs < 0 || (npairs > 0 && (!probs || !T || !R || !v || !status))) return LAG_EINVAL;
  lag_gn_options o;
  lag_gn_default_options(&o);
  if (opt) o = *opt;
  if (o.max_gn < 0 || o.pcg_maxit < 0 || o.max_halvings < 0 || o.gtol < 0.0 || o.graph_iters < 0 ||
      o.graph_iters > 64)
    return LAG_EINVAL;
  for (int i = 0; i < npairs; ++i) {
    const int rc = lag_problem_check(&probs[i]);
    if (rc) return rc;
    if (!T[i] || !R[i] || !v[i]) return LAG_EINVAL;
    status[i] = LAG_OK;
  }
  if (npairs == 0) return LAG_OK;
  constexpr int kSc = 24;  // host copy of scalars 0..23 per pair
  const int per_graph = o.graph_iters > 0 ? o.graph_iters : 4;
  std::vector<BatchPair> pr(npairs);
  hipStream_t es[kBatchStreams] = {};
  hipEvent_t ev_es[kBatchStreams] = {};
  hipStream_t s0 = nullptr;
  hipEvent_t ev0 = nullptr, ev_state[2] = {nullptr, nullptr};
  int** d_ctl = nullptr;
  int* d_state = nullptr;
  int* h_state = nullptr;   // pinned, 2 x npairs halt flags
  double* h_sc = nullptr;   // pinned, kSc per pair
  int* h_ctl = nullptr;     // pinned, 4 per pair (PCG control block)
  int* h_mx = nullptr;      // pinned, 2 per pair (longest row, blocks stored)
  hipGraphExec_t exec = nullptr;
  int ng = 0;                    // pairs in the current graph
  int captures = 0, replays = 0;
  auto cleanup = [&]() {
    if (s0) (void)hipStreamSynchronize(s0);
    for (hipStream_t s : es)
      if (s) (void)hipStreamSynchronize(s);
    if (exec) (void)hipGraphExecDestroy(exec);
    for (auto& p : pr)
      if (p.P) lag_plan_destroy(p.P);
    for (int k = 0; k < kBatchStreams; ++k) {
      if (es[k]) (void)hipStreamDestroy(es[k]);
      if (ev_es[k]) (void)hipEventDestroy(ev_es[k]);
    }
    if (s0) (void)hipStreamDestroy(s0);
    for (hipEvent_t e : {ev0, ev_state[0], ev_state[1]})
      if (e) (void)hipEventDestroy(e);
    for (void* q : {(void*)d_ctl, (void*)d_state})
      if (q) (void)hipFree(q);
    for (void* q : {(void*)h_state, (void*)h_sc, (void*)h_ctl, (void*)h_mx})
      if (q) (void)hipHostFree(q);
  };
  auto fail = [&](int rc) {
    const std::string msg = lag_last_hip_error();
    cleanup();
    if (!msg.empty()) set_hip_error_text(msg.c_str());
    return rc;
  };
#define BTRY(expr)               \
  do {                           \
    const int _r = (expr);       \
    if (_r) return fail(_r);     \
  } while (0)
#define BHIP(call)                                          \
  do {                                                      \
    const hipError_t _e = (call);                           \
    if (_e != hipSuccess) return fail(set_hip_error(_e));   \
  } while (0)
  for (int i = 0; i < npairs; ++i) {
    BTRY(lag_plan_create_tuned(&probs[i], bricks ? bricks + 3 * i : nullptr, &pr[i].P));
    BTRY(ensure_pcg_ctl(pr[i].P));
  }
  for (int k = 0; k < kBatchStreams; ++k) {
    BHIP(hipStreamCreateWithFlags(&es[k], hipStreamNonBlocking));
    BHIP(hipEventCreateWithFlags(&ev_es[k], hipEventDisableTiming));
  }
  BHIP(hipStreamCreateWithFlags(&s0, hipStreamNonBlocking));
  BHIP(hipEventCreateWithFlags(&ev0, hipEventDisableTiming));
  for (auto& e : ev_state) BHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  BHIP(hipMalloc((void**)&d_ctl, sizeof(int*) * npairs));
  BHIP(hipMalloc((void**)&d_state, sizeof(int) * npairs));
  BHIP(hipHostMalloc((void**)&h_state, sizeof(int) * 2 * npairs, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_sc, sizeof(double) * kSc * npairs, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_ctl, sizeof(int) * 4 * npairs, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_mx, sizeof(int) * 2 * npairs, hipHostMallocDefault));
  {
    std::vector<int*> ctl(npairs);
    for (int i = 0; i < npairs; ++i) ctl[i] = pr[i].P->ctl;
    BHIP(hipMemcpy(d_ctl, ctl.data(), sizeof(int*) * npairs, hipMemcpyHostToDevice));
  }
  auto st = [&](int i) { return es[i % kBatchStreams]; };
  auto sync_all = [&]() -> int {
    for (hipStream_t s : es) LAG_HIP(hipStreamSynchronize(s));
    return LAG_OK;
  };
  auto sc = [&](int i, int k) { return h_sc[(size_t)kSc * i + k]; };
  auto copy_sc = [&](int i, int off, int cnt) -> int {
    LAG_HIP(hipMemcpyAsync(h_sc + (size_t)kSc * i + off, pr[i].P->scalars + off, sizeof(double) * cnt,
                           hipMemcpyDeviceToHost, st(i)));
    return LAG_OK;
  };
  // gradient of pair i at v[i] into vec[0]; J, D, S and |g|^2 into scalars 8..11
  auto gradient = [&](int i, bool assembled) -> int {
    lag_plan P = pr[i].P;
    hipStream_t s = st(i);
    int r;
    if (assembled) {
      if ((r = jacobian_assemble_launch(P, v[i], T[i], P->img_a, s))) return r;
      if ((r = gradient_assembled(P, v[i], T[i], R[i], P->img_a, P->vec[0], P->scalars + 8, s))) return r;
      LAG_HIP(hipMemcpyAsync(h_mx + 2 * i, P->jac_max, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
    } else if ((r = lag_gradient(P, v[i], T[i], R[i], P->vec[0], P->scalars + 8, s))) {
      return r;
    }
    if ((r = launch_dot(P, P->n_unknowns, P->vec[0], P->vec[0], P->scalars + 11, s))) return r;
    return copy_sc(i, 8, 4);
  };
  // objective of pair i at v + mu dv (into vec[7]), J into scalar 13
  auto trial = [&](int i, double mu) -> int {
    lag_plan P = pr[i].P;
    hipStream_t s = st(i);
    int r;
    if ((r = launch_axpby(P->n_unknowns, 1.f, v[i], (float)mu, P->vec[2], P->vec[7], s))) return r;
    if ((r = objective_full(P, P->vec[7], T[i], R[i], nullptr, nullptr, P->scalars + 13, s))) return r;
    return copy_sc(i, 12, 2);
  };

  // reference gradient norm: |g(v = 0)| for a start away from zero, else
  // the first gradient's (as lag_gn_solve)
  for (int i = 0; i < npairs; ++i) {
    lag_plan P = pr[i].P;
    BTRY(launch_dot(P, P->n_unknowns, v[i], v[i], P->scalars + 16, st(i)));
    BTRY(copy_sc(i, 16, 1));
  }
  BTRY(sync_all());
  bool any_start = false;
  for (int i = 0; i < npairs; ++i) {
    pr[i].from_zero = sc(i, 16) == 0.0;
    if (pr[i].from_zero) continue;
    any_start = true;
    lag_plan P = pr[i].P;
    BTRY(gradient_at_zero(P, T[i], R[i], P->vec[0], P->scalars + 8, st(i)));
    BTRY(launch_dot(P, P->n_unknowns, P->vec[0], P->vec[0], P->scalars + 11, st(i)));
    BTRY(copy_sc(i, 8, 4));
  }
  if (any_start) BTRY(sync_all());
  for (int i = 0; i < npairs; ++i)
    if (!pr[i].from_zero) {
      pr[i].info.g0 = sqrt(sc(i, 11));
      pr[i].gstop = o.gtol * pr[i].info.g0;
    }

  for (int it = 0; it <= o.max_gn; ++it) {
    // ---- gradients (assembled where the plan stores J), all pairs at once
    int nact = 0;
    for (int i = 0; i < npairs; ++i)
      if (pr[i].active) BTRY(gradient(i, pr[i].P->jac_k > 0));
    BTRY(sync_all());
    for (int i = 0; i < npairs; ++i) {
      BatchPair& b = pr[i];
      if (!b.active) continue;
      lag_plan P = b.P;
      b.stored = 0;
      if (P->jac_k > 0) {
        b.stored = jacobian_assembled(P, h_mx + 2 * i);
        if (!b.stored) {  // over capacity: grow once and assemble again, else matrix-free
          if (jacobian_grow(P, h_mx[2 * i])) {
            ++b.gen;
            BTRY(gradient(i, true));
            BTRY(sync_all());
            b.stored = jacobian_assembled(P, h_mx + 2 * i);
          }
          if (!b.stored) {
            BTRY(gradient(i, false));
            BTRY(sync_all());
          }
        }
      }
      const double J = sc(i, 8), gn = sqrt(sc(i, 11));
      if (it == 0) {
        b.info.J0 = J;
        if (b.from_zero) {
          b.info.g0 = gn;
          b.gstop = o.gtol * gn;
        }
      }
      b.info.J = J;
      b.info.gnorm = gn;
      if (gn <= b.gstop) {
        b.info.converged = 1;
        b.active = 0;
      } else if (it == o.max_gn) {
        b.active = 0;
      } else {
        ++nact;
      }
    }
    if (nact == 0) break;

    // ---- PCG: starts on the pairs' streams, iterations in one graph
    for (int i = 0; i < npairs; ++i) {
      BatchPair& b = pr[i];
      lag_plan P = b.P;
      if (!b.active) {
        if (b.in_graph) {
          hipLaunchKernelGGL(lag::k_halt_ctl, dim3(1), dim3(64), 0, st(i), P->ctl);
          BHIP(hipGetLastError());
        }
        continue;
      }
      BTRY(launch_axpby(P->n_unknowns, -1.f, P->vec[0], 0.f, nullptr, P->vec[1], st(i)));
      PcgExtra ex;
      ex.bb = sc(i, 11);  // rhs = -g: rhs . rhs = g . g
      double nb = 0.0;
      BTRY(pcg_start(P, P->vec[1], P->vec[2], o.pcg_tol, o.pcg_maxit, &nb, st(i), &ex));
    }
    // the graph holds the pairs running when it was captured; it is captured
    // again when a running pair changes its operator or storage, or once
    // half of the pairs in it have stopped (their halted iterations still
    // cost a dispatch each)
    int in_graph = 0;
    bool same = exec != nullptr;
    for (int i = 0; i < npairs; ++i) {
      in_graph += pr[i].in_graph;
      if (pr[i].active)
        same = same && pr[i].in_graph && pr[i].graph_mode == pr[i].stored && pr[i].graph_gen == pr[i].gen;
    }
    same = same && 2 * nact > in_graph;
    if (!same) {
      // capture the running pairs' `per_graph` PCG iterations, the k-th
      // of them on branch k mod kBatchStreams
      BTRY(sync_all());
      std::lock_guard<std::mutex> lk(api_lock());
      if (exec) {
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
      }
      BHIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
      int crc = hipEventRecord(ev0, s0) == hipSuccess ? LAG_OK : LAG_EHIP;
      for (int k = 0; k < kBatchStreams && crc == LAG_OK; ++k)
        if (hipStreamWaitEvent(es[k], ev0, 0) != hipSuccess) crc = LAG_EHIP;
      std::vector<int*> ctl;
      for (int i = 0; i < npairs && crc == LAG_OK; ++i) {
        BatchPair& b = pr[i];
        b.in_graph = b.active;
        if (!b.active) continue;
        lag_plan P = b.P;
        b.graph_mode = b.stored;
        b.graph_gen = b.gen;
        BatchOp H{P, v[i], T[i], b.graph_mode == 1};
        const hipStream_t br = es[ctl.size() % kBatchStreams];
        ctl.push_back(P->ctl);
        P->geo.halt = P->ctl;
        P->capturing = 1;
        for (int u = 0; u < per_graph && crc == LAG_OK; ++u) crc = pcg_iteration(P, H, P->vec[2], br);
        P->geo.halt = nullptr;
        P->capturing = 0;
      }
      ng = (int)ctl.size();
      for (int k = 0; k < kBatchStreams && crc == LAG_OK; ++k)
        if (hipEventRecord(ev_es[k], es[k]) != hipSuccess || hipStreamWaitEvent(s0, ev_es[k], 0) != hipSuccess)
          crc = LAG_EHIP;
      hipGraph_t graph = nullptr;
      const hipError_t ce = hipStreamEndCapture(s0, &graph);
      if (crc != LAG_OK || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(crc != LAG_OK ? crc : set_hip_error(ce));
      }
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        exec = nullptr;
        return fail(set_hip_error(ie));
      }
      BHIP(hipMemcpy(d_ctl, ctl.data(), sizeof(int*) * ng, hipMemcpyHostToDevice));
      ++captures;
    }
    // the starts must be done before the graph runs
    for (int k = 0; k < kBatchStreams; ++k) {
      BHIP(hipEventRecord(ev_es[k], es[k]));
      BHIP(hipStreamWaitEvent(s0, ev_es[k], 0));
    }
    // replay until every pair's PCG has stopped; as in pcg_graph_impl the
    // flags of replay l are read after replay l + 1 is enqueued
    const int launches = (o.pcg_maxit + per_graph - 1) / per_graph;
    for (int l = 0; l < launches; ++l) {
      const int slot = l & 1;
      BHIP(hipGraphLaunch(exec, s0));
      hipLaunchKernelGGL(lag::k_gather_ctl, dim3((ng + 255) / 256), dim3(256), 0, s0, d_ctl, ng, d_state);
      BHIP(hipGetLastError());
      BHIP(hipMemcpyAsync(h_state + slot * npairs, d_state, sizeof(int) * ng, hipMemcpyDeviceToHost, s0));
      BHIP(hipEventRecord(ev_state[slot], s0));
      ++replays;
      if (l > 0) {
        BHIP(hipEventSynchronize(ev_state[slot ^ 1]));
        bool all = true;
        for (int k = 0; k < ng && all; ++k) all = h_state[(slot ^ 1) * npairs + k] != 0;
        if (all) break;
      }
    }
    BHIP(hipEventRecord(ev0, s0));
    for (int k = 0; k < kBatchStreams; ++k) BHIP(hipStreamWaitEvent(es[k], ev0, 0));

    // ---- PCG results, slope g . dv and the first trial (mu = 1)
    for (int i = 0; i < npairs; ++i) {
      BatchPair& b = pr[i];
      if (!b.active) continue;
      lag_plan P = b.P;
      BHIP(hipMemcpyAsync(h_ctl + 4 * i, P->ctl, sizeof(int) * 4, hipMemcpyDeviceToHost, st(i)));
      BTRY(launch_dot(P, P->n_unknowns, P->vec[0], P->vec[2], P->scalars + 12, st(i)));
      b.mu = 1.0;
      BTRY(trial(i, 1.0));
    }
    BTRY(sync_all());
    std::vector<int> pending;
    for (int i = 0; i < npairs; ++i) {
      BatchPair& b = pr[i];
      if (!b.active) continue;
      const int iters = h_ctl[4 * i + 1];
      b.info.iters += 1;
      b.info.pcg_iters += iters;
      b.info.matvecs += iters + (h_ctl[4 * i] == 2 ? 1 : 0);
      b.slope = sc(i, 12);
      pending.push_back(i);
    }
    // ---- Armijo backtracking by halving, all pending pairs per round
    for (int k = 0;; ++k) {
      std::vector<int> next;
      for (int i : pending) {
        BatchPair& b = pr[i];
        const double Jt = sc(i, 13);
        if (Jt <= b.info.J + o.armijo_c1 * b.mu * b.slope) {
          b.info.J = Jt;
          BTRY(launch_axpby(b.P->n_unknowns, 1.f, b.P->vec[7], 0.f, nullptr, v[i], st(i)));
        } else if (k < o.max_halvings) {
          b.mu *= 0.5;
          next.push_back(i);
        } else {
          b.status = LAG_ELINESEARCH;
          b.active = 0;
        }
      }
      if (next.empty()) break;
      for (int i : next) BTRY(trial(i, pr[i].mu));
      BTRY(sync_all());
      pending.swap(next);
    }
  }
  BTRY(sync_all());
#undef BTRY
#undef BHIP
  (void)captures;
  (void)replays;
  for (int i = 0; i < npairs; ++i) {
    status[i] = pr[i].status;
    if (infos) infos[i] = pr[i].info;
  }
  cleanup();
  return LAG_OK;
}

}  // extern "C"
