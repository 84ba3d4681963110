// Host-side internals of liblaglddmm: the plan object, status helpers and
// the launchers each translation unit exports to the C-ABI layer.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>

#include "laglddmm.h"
#include "lag_device.hpp"

struct lag_plan_s {
  lag_problem prob;
  int device = 0;
  lag::Geo geo{};
  lag::Bricks bricks{};
  int fields = 0;              // nodes * dim velocity fields
  long long n_unknowns = 0;

  // packed copies of velocity-shaped inputs (float2/float4 per node)
  void* pack_v = nullptr;
  void* pack_p = nullptr;
  // RK4 stage tables, [0] for dir = -1 and [1] for dir = +1 (4N entries)
  int* st_j0[2] = {nullptr, nullptr};
  float* st_th[2] = {nullptr, nullptr};
  // time-node weights of the regulariser (host copy and device scale table)
  double node_w[64];
  float* reg_scale = nullptr;  // per node: alpha h_v^d w_j
  // image-sized scratch
  float* img_a = nullptr;
  float* img_b = nullptr;
  float* phi = nullptr;        // dim * np
  // deterministic binning (continuity)
  int* bin_count = nullptr;    // np + 1
  int* bin_start = nullptr;    // np + 1
  int* bin_cursor = nullptr;   // np
  int* bin_items = nullptr;    // np
  int* part_base = nullptr;    // np
  float* part_vals = nullptr;  // 2^d * np
  int* scan_blocks = nullptr;  // block sums for the scan
  // reductions
  double* red_partial = nullptr;  // max(kRedBlocks, one per kBlock unknowns)
  double* red_partial2 = nullptr; // kRedBlocks (PCG: r.r partials)
  int php_n = 0;                  // p.Hp partials in red_partial from the last PCG matvec
  int rz_n = 0;                   // r.z partials in red_partial from the last PCG preconditioning
  const float* packed_by_pcg = nullptr;  // PCG direction whose packed copy pack_p holds (set by its update)
  double* scalars = nullptr;      // 16 device scalars
  // velocity-sized scratch (PCG / GN vectors)
  float* vec[10] = {nullptr};
  // spectral preconditioner
  int fft_ok = 0;
  float2* fft_buf = nullptr;   // fields * nv complex
  float2* fft_tw[3] = {nullptr, nullptr, nullptr};
  float* fft_lam[3] = {nullptr, nullptr, nullptr};
  float* fft_mu1 = nullptr;    // per node replacement for a zero mode
  int fft_rad[3][16];
  int fft_nrad[3];
  // assembled Jacobian (transport, stationary): capacity jac_k blocks per
  // characteristic slot; jac_ready once a complete assembly is stored
  int jac_k = 0;
  long long jac_slots = 0;
  float4* jac_vals = nullptr;
  int* jac_cell = nullptr;
  unsigned char* jac_cnt = nullptr;
  int* jac_max = nullptr;
  int jac_ready = 0;
  long long jac_blocks_stored = 0;
  int jac_max_seen = 0;
  // paged copy of the assembled Jacobian (k_jac_pack): pg_cap pages of 128
  // positions per brick; 0 = not used (the products read the [k][slot]
  // layout directly)
  int pg_cap = 0;
  float4* pg_vals = nullptr;
  int* pg_cells = nullptr;
  int* pg_rows = nullptr;
  int* pg_npages = nullptr;
  int* pg_order = nullptr;     // [XCD][slot] launch order of the bricks, -1 past a range (k_brick_order)
  int* pg_redo = nullptr;      // count of bricks whose product pass was redone at the exact scale
  // per-brick partial velocity tiles and, per axis, the list of (brick,
  // tile offset) pairs covering each velocity index (fixed-order reduction)
  float* tile_part = nullptr;
  int* cover_start[3] = {nullptr, nullptr, nullptr};
  int2* cover_ent[3] = {nullptr, nullptr, nullptr};
  int cover_max = 0;  // most covering bricks of a node along one axis
  // the paged product writes, per brick, only the tile nodes that the bricks
  // sharing its index along each axis touch: per axis and brick index the
  // lowest and highest tile node (lo at [off[a] + i], hi at [nb_sum + off[a]
  // + i], off = 0, nb[0], nb[0] + nb[1]), and the cover lists restricted to
  // those nodes (k_jac_pack, k_cover_filter, once per assembly)
  int* pg_axbox = nullptr;
  int* pgc_start[3] = {nullptr, nullptr, nullptr};
  int2* pgc_ent[3] = {nullptr, nullptr, nullptr};
  // assembled matvec: out-of-tile contributions (float atomics), added and
  // cleared by the tile reduction, so outputs need no fill beforehand
  float* jac_fb = nullptr;
  // matrix-free adjoint products: characteristics whose cells leave their
  // brick's tile, handled apart in a 64-bit fixed-point buffer
  int* dfr_list = nullptr;               // np image cell indices
  int* dfr_hdr = nullptr;                // [0] count, [1] largest magnitude sum (float bits), [2] bricks redone
  unsigned long long* dfr_acc = nullptr; // fields * nv, zero between calls
  // status flags written by kernels (kFlag* bits)
  int* flags = nullptr;
  // PCG control: device control block, pinned host mirrors (two slots, read
  // one iteration late), their copy events, the capture stream and the
  // cached graph executable with the arguments it was captured for
  int* ctl = nullptr;          // device int[8]: status, iterations, cap, -, r.r (double at [4])
  int* ctl_host = nullptr;     // pinned host int[2][8]
  int* ctl_mirror = nullptr;   // set around an eager PCG iteration: k_pcg_check writes the control block there
  double* sc_host = nullptr;   // pinned host double[8]
  hipEvent_t ctl_ev[2] = {nullptr, nullptr};
  hipStream_t gstream = nullptr;
  hipGraphExec_t pcg_exec = nullptr;
  const void* pcg_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int pcg_key_i[2] = {-1, -1};
  int capturing = 0;
  // optional HIP-event timing of the dominant Gauss-Newton matvec kernel
  int prof_on = 0;
  int prof_n = 0;
  hipEvent_t prof_ev[2 * 256];
};

namespace lag {

constexpr int kRedBlocks = 1024;

int set_hip_error(hipError_t e);   // records the message, returns LAG_EHIP
void set_hip_error_text(const char* msg);  // records a message from another thread
#define LAG_HIP(call)                                    \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return ::lag::set_hip_error(_e); \
  } while (0)
#define LAG_LAUNCH_CHECK() LAG_HIP(hipGetLastError())

// ---- launchers (each returns a LAG_* status) -----------------------------
int launch_pack(lag_plan P, const float* v, void* dst, hipStream_t s);
int launch_fill(float* x, long long n, float val, hipStream_t s);
int launch_zero_i(int* x, long long n, hipStream_t s);
// Scratch of the deterministic binned scatter: per particle its base cell
// and 2^d corner values, per image cell a count, a bin start and a fill
// cursor, the binned particle ids, and the scan's block sums.
struct BinScratch {
  int* base = nullptr;     // np
  float* vals = nullptr;   // 2^d * np
  int* count = nullptr;    // np + 1
  int* start = nullptr;    // np + 1
  int* cursor = nullptr;   // np
  int* items = nullptr;    // np
  int* scan = nullptr;     // scan_blocks(np) + 2
};
inline long long scan_blocks(long long np) { return (np + 1023) / 1024; }
inline BinScratch plan_bins(lag_plan P) {
  BinScratch b;
  b.base = P->part_base;
  b.vals = P->part_vals;
  b.count = P->bin_count;
  b.start = P->bin_start;
  b.cursor = P->bin_cursor;
  b.items = P->bin_items;
  b.scan = P->scan_blocks;
  return b;
}
// Launch geometry of a validated problem (host only); LAG_EUNSUPPORTED if
// the packed velocity field needs offsets beyond 32 bits.
int make_geo(const lag_problem* prob, Geo& g);
// deterministic binned scatter of per-particle corner values (b.base/b.vals)
int bin_and_gather(const Geo& g, const BinScratch& b, float* out, hipStream_t s);
// push-forward through explicit binning scratch (the plan's, or a caller's)
int launch_pushforward_bins(const Geo& g, const BinScratch& b, const float* T, const float* phi, float* u,
                            hipStream_t s);
int launch_trace(lag_plan P, const void* vpack, int dir, float* phi, hipStream_t s);
int launch_transport(lag_plan P, const float* T, const float* phi, float* u, hipStream_t s);
int launch_pushforward(lag_plan P, const float* T, const float* phi, float* u, hipStream_t s);
int launch_jvp(lag_plan P, const void* vpack, const void* dpack, const float* T, float* out,
               hipStream_t s);
// seed: transport -> per-characteristic weights w (image-shaped);
//       continuity -> image-shaped field w whose interpolant gradient is taken.
int launch_vjp(lag_plan P, const void* vpack, const float* T, const float* w, float* out,
               hipStream_t s, bool zero = false);
int launch_hess_transport(lag_plan P, const void* vpack, const void* ppack, const float* T,
                          const float* wvox, float* out, hipStream_t s);
// paged: the partial tiles of the paged product, read through the
// restricted cover lists (the nodes they leave out count as zero)
int launch_tile_reduce(lag_plan P, float* out, float* fb, hipStream_t s, const RegTail* rt, bool deferred = false,
                       bool paged = false);
// LDS of the matrix-free adjoint kernel (64-bit tile of the plan's bricks)
size_t adjoint_lds_bytes(lag_plan P);
int launch_jac_assemble(lag_plan P, const void* vpack, const float* T, float* u, hipStream_t s);
// pages per brick of the paged copy for capacity kmax (0: layout not used)
int jac_pages_per_brick(lag_plan P, int kmax);
// Launch slots per XCD of the paged product (room for a brick range of up to
// twice the even share; k_brick_order), and the length of the order array.
__host__ __device__ inline int pg_xcd_slots(long long nbricks) { return (int)(2 * ((nbricks + kXcds - 1) / kXcds)); }
__host__ __device__ inline size_t pg_order_len(long long nbricks) { return (size_t)kXcds * (size_t)pg_xcd_slots(nbricks); }
int launch_jac_apply(lag_plan P, const void* ppack, const float* wvox, const float* wseed, float scale, float* out,
                     hipStream_t s, const RegTail* rt);
int tiles_setup(lag_plan P);       // partial-tile buffer + cover tables (plan creation)
int launch_reg(lag_plan P, const float* p, float* out, int accumulate, int with_gamma,
               float extra_scale, hipStream_t s);
// Regulariser parameters for the tile reduction (same tables as launch_reg).
RegTail reg_tail(lag_plan P, const float* p, int with_gamma, float extra_scale, double* part);
// z = M r; with rz != null also the block partials of r . z (count in *nrz)
int launch_precond(lag_plan P, const float* r, float* z, hipStream_t s, double* rz = nullptr, int* nrz = nullptr);
int precond_setup(lag_plan P);     // host tables + allocations (plan creation)

// reductions: result written to dst (device double)
int launch_dot(lag_plan P, long long n, const float* x, const float* y, double* dst, hipStream_t s);
// D = h^d/2 |u - R|^2 -> dst; wres = scale * (u - R) if wres != null
int launch_ssd(lag_plan P, const float* u, const float* R, float* wres, float scale, double* dst,
               hipStream_t s);
int launch_axpy(long long n, float a, const float* x, float* y, hipStream_t s);
int launch_combine_J(double* s3, double alpha, hipStream_t s);
int launch_dot_partial(lag_plan P, long long n, const float* x, const float* y, double* part, hipStream_t s);
// *dst = 0.5 v . (h_v^d w_j A v), the regulariser energy
int launch_reg_energy(lag_plan P, const float* v, double* dst, hipStream_t s);
int launch_pcg_xr(lag_plan P, float* x, float* r, const float* p, const float* Hp, hipStream_t s);
int launch_pcg_p(lag_plan P, float* p, const float* z, hipStream_t s);
int launch_pcg_ctl_init(int* ctl, const double* sc, int maxit, hipStream_t s);
int launch_pcg_check(lag_plan P, hipStream_t s);

// Timing of the dominant matvec kernel (off unless enabled): the next pair
// of events, which the launch itself stamps at the kernel's start and end
// (hipExtLaunchKernelGGL), so the time excludes the gap before the dispatch;
// both null when not timing (or while a graph is captured).
inline void prof_events(lag_plan P, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (P->prof_on && !P->capturing && P->prof_n < 256) {
    *start = P->prof_ev[2 * P->prof_n];
    *stop = P->prof_ev[2 * P->prof_n + 1];
    ++P->prof_n;
  }
}

}  // namespace lag
