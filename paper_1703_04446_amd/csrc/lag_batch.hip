// Many independent registration problems of uneven sizes and both models:
// a brick-shape autotuner and a batched Gauss-Newton driver.
//
// Batching here means keeping the GPU busy with many small solves at once:
// worker threads, each with its own HIP stream and its own plan per distinct
// problem (plans own scratch, so one plan serves one stream), take pairs
// from a shared queue in order of decreasing size and run lag_gn_solve;
// with lag_gn_options.graph_iters > 0 every PCG loop runs as a replayed
// graph with its stopping test on the device, which removes most host
// round trips of a small solve.

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lag_internal.hpp"

namespace lag {

// smooth periodic test field for timing: v_c(x) = A sin(2 pi (x_{c+1} + c/7))
// (cell centres; a displacement of a few cells, so characteristics move)
__global__ void k_tune_velocity(float* v, int dim, int mx, int my, int mz, float amp) {
  const long long nv = (long long)mx * my * mz;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * dim) return;
  const int c = (int)(i / nv);
  const long long r = i - c * nv;
  const int x = (int)(r % mx), y = (int)((r / mx) % my), z = (int)(r / ((long long)mx * my));
  const float pos[3] = {(x + 0.5f) / mx, (y + 0.5f) / my, (z + 0.5f) / mz};
  const int a = (c + 1) % dim;
  v[i] = amp * sinpif(2.f * (pos[a] + c / 7.f));
}

// smooth test image: product of cosines (non-zero gradient almost everywhere)
__global__ void k_tune_image(float* T, int mx, int my, int mz) {
  const long long n = (long long)mx * my * mz;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % mx), y = (int)((i / mx) % my), z = (int)(i / ((long long)mx * my));
  T[i] = 1.f + 0.5f * cospif(2.f * (x + 0.5f) / mx) * cospif(2.f * (y + 0.5f) / my) *
                   cospif(2.f * (z + 0.5f) / mz);
}

}  // namespace lag

using namespace lag;

namespace {

bool same_problem(const lag_problem& a, const lag_problem& b) { return memcmp(&a, &b, sizeof(a)) == 0; }

// Candidate brick targets (image cells per axis) for the autotuner.
std::vector<std::array<int32_t, 3>> candidates(int dim) {
  if (dim == 3)
    return {{16, 16, 12}, {16, 16, 8}, {8, 16, 8}, {16, 16, 16}, {8, 8, 8}, {32, 16, 8}, {16, 8, 8}};
  return {{16, 16, 1}, {32, 16, 1}, {32, 32, 1}, {64, 32, 1}, {16, 8, 1}, {64, 64, 1}};
}

}  // namespace

extern "C" {

int lag_autotune_bricks(const lag_problem* prob, int32_t* best_target, double* best_ms, void* stream) {
  if (!prob || !best_target) return LAG_EINVAL;
  int rc = lag_problem_check(prob);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int64_t np = 0, nu = 0;
  lag_problem_sizes(prob, &np, &nu);
  float *v = nullptr, *T = nullptr, *p = nullptr, *Hp = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (float* b : {v, T, p, Hp})
      if (b) (void)hipFree(b);
  };
  if (hipMalloc((void**)&v, sizeof(float) * nu) != hipSuccess || hipMalloc((void**)&T, sizeof(float) * np) ||
      hipMalloc((void**)&p, sizeof(float) * nu) || hipMalloc((void**)&Hp, sizeof(float) * nu)) {
    (void)hipGetLastError();
    cleanup();
    return LAG_ENOMEM;
  }
  const int D = prob->dim;
  const int mx = prob->vel_m[0], my = prob->vel_m[1], mz = D == 3 ? prob->vel_m[2] : 1;
  const long long nvel = (long long)mx * my * mz;
  // amplitude: about two velocity cells of displacement over the unit time
  const float amp = 2.f * (float)prob->extent[0] / (float)mx;
  for (int j = 0; j < prob->nt_nodes; ++j)
    hipLaunchKernelGGL(k_tune_velocity, dim3((unsigned)((nvel * D + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       v + (long long)j * D * nvel, D, mx, my, mz, amp);
  hipLaunchKernelGGL(k_tune_velocity, dim3((unsigned)((nvel * D + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, D,
                     mx, my, mz, 1.f);
  for (int j = 1; j < prob->nt_nodes; ++j)
    (void)hipMemcpyAsync(p + (long long)j * D * nvel, p, sizeof(float) * D * nvel, hipMemcpyDeviceToDevice, s);
  hipLaunchKernelGGL(k_tune_image, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, T,
                     prob->img_m[0], prob->img_m[1], D == 3 ? prob->img_m[2] : 1);
  if (hipGetLastError() != hipSuccess) {
    cleanup();
    return LAG_EHIP;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e300;
  std::vector<std::array<int, 3>> seen;
  for (const auto& c : candidates(D)) {
    lag_plan P = nullptr;
    if (lag_plan_create_tuned(prob, c.data(), &P) != LAG_OK) continue;
    std::array<int, 3> eff = {P->bricks.bdim[0], P->bricks.bdim[1], P->bricks.bdim[2]};
    if (std::find(seen.begin(), seen.end(), eff) != seen.end()) {
      lag_plan_destroy(P);
      continue;
    }
    seen.push_back(eff);
    int32_t stored = 0;
    const bool assembled = P->jac_k > 0 && lag_jacobian_assemble(P, v, T, &stored, s) == LAG_OK && stored;
    auto matvec = [&]() {
      return assembled ? gn_hessmat_assembled(P, nullptr, p, Hp, s) : gn_hessmat(P, v, T, nullptr, p, Hp, s);
    };
    int ok = matvec() == LAG_OK;  // warm-up
    const int reps = 5;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && ok; ++r) ok = matvec() == LAG_OK;
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    lag_plan_destroy(P);
    if (!ok) continue;
    const double per = ms / reps;
    if (per < best) {
      best = per;
      for (int a = 0; a < 3; ++a) best_target[a] = c[a];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  if (best >= 1e300) return LAG_EHIP;
  if (best_ms) *best_ms = best;
  return LAG_OK;
}

int lag_batch_solve(int32_t npairs, const lag_problem* probs, const float* const* T, const float* const* R,
                    float* const* v, const lag_gn_options* opt, int32_t workers, const int32_t* bricks_in,
                    int32_t autotune, lag_gn_info* infos, int32_t* status) {
  if (npairs < 0 || (npairs > 0 && (!probs || !T || !R || !v || !status)) || workers < 1 || workers > 16)
    return LAG_EINVAL;
  for (int i = 0; i < npairs; ++i) {
    int rc = lag_problem_check(&probs[i]);
    if (rc) return rc;
    if (!T[i] || !R[i] || !v[i]) return LAG_EINVAL;
  }
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return LAG_EHIP;
  for (int i = 0; i < npairs; ++i) status[i] = LAG_OK;
  // distinct problems (shape, model, parameters) and their brick shapes
  std::vector<lag_problem> kinds;
  std::vector<int> kind_of(npairs);
  for (int i = 0; i < npairs; ++i) {
    int k = 0;
    while (k < (int)kinds.size() && !same_problem(kinds[k], probs[i])) ++k;
    if (k == (int)kinds.size()) kinds.push_back(probs[i]);
    kind_of[i] = k;
  }
  std::vector<std::array<int32_t, 3>> bricks(kinds.size());
  std::vector<int> tuned(kinds.size(), 0);
  if (bricks_in) {
    // the first pair of each distinct problem names its shape
    for (int i = npairs - 1; i >= 0; --i) {
      for (int a = 0; a < 3; ++a) bricks[kind_of[i]][a] = bricks_in[3 * i + a];
      tuned[kind_of[i]] = 1;
    }
  } else if (autotune) {
    for (size_t k = 0; k < kinds.size(); ++k) {
      double ms = 0.0;
      if (lag_autotune_bricks(&kinds[k], bricks[k].data(), &ms, nullptr) == LAG_OK) tuned[k] = 1;
    }
  }
  // largest problems first (cost ~ characteristics x steps)
  std::vector<int> order(npairs);
  for (int i = 0; i < npairs; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    int64_t na = 0, nb = 0, u = 0;
    lag_problem_sizes(&probs[a], &na, &u);
    lag_problem_sizes(&probs[b], &nb, &u);
    return na * probs[a].nsteps > nb * probs[b].nsteps;
  });
  std::atomic<int> next(0);
  std::atomic<int> fatal(LAG_OK);
  std::mutex err_mu;
  std::string err_text;   // first HIP error message of any worker
  auto note = [&](int rc) {
    if (rc != LAG_EHIP) return;
    std::lock_guard<std::mutex> lk(err_mu);
    if (err_text.empty()) err_text = lag_last_hip_error();
  };
  auto work = [&]() {
    if (hipSetDevice(device) != hipSuccess) {
      fatal = LAG_EHIP;
      return;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      fatal = LAG_EHIP;
      return;
    }
    std::vector<lag_plan> plans(kinds.size(), nullptr);
    for (;;) {
      const int q = next.fetch_add(1);
      if (q >= npairs || fatal.load() != LAG_OK) break;
      const int i = order[q];
      const int k = kind_of[i];
      if (!plans[k]) {
        const int rc = lag_plan_create_tuned(&kinds[k], tuned[k] ? bricks[k].data() : nullptr, &plans[k]);
        if (rc != LAG_OK) {
          status[i] = rc;
          note(rc);
          continue;
        }
      }
      lag_gn_info info;
      memset(&info, 0, sizeof(info));
      status[i] = lag_gn_solve(plans[k], T[i], R[i], v[i], opt, &info, s);
      note(status[i]);
      if (infos) infos[i] = info;
    }
    (void)hipStreamSynchronize(s);
    for (lag_plan P : plans)
      if (P) lag_plan_destroy(P);
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) pool.emplace_back(work);
  for (auto& t : pool) t.join();
  if (!err_text.empty()) set_hip_error_text(err_text.c_str());
  if (fatal.load() != LAG_OK) return fatal.load();
  for (int i = 0; i < npairs; ++i)
    if (status[i] != LAG_OK && status[i] != LAG_ELINESEARCH) return status[i];
  return LAG_OK;
}

}  // extern "C"
