// RK4 characteristics, transport, Jacobian products and the fused
// Gauss-Newton matvec (transport model) for gfx950.
//
// Algorithm 1 (RK4 with the derivative recursion) is evaluated per
// characteristic, one thread per characteristic, in float32 with the
// position kept as a displacement from the start cell centre.
//
// Jacobian-transpose products need the adjoint of the RK4 map.  Instead of
// storing the trajectory (which would make memory grow with N) the kernels
// make two forward sweeps:
//   pass 1: positions, the tangent (for J p) and the flow Jacobian
//           F = d y_N / d y_0 = M_{N-1} ... M_0, M_k the RK4 step Jacobian;
//   seed:   ybar_N from the image side, ybar_0 = F^T ybar_N;
//   pass 2: recompute each step's stages, recover ybar_{k+1} = M_k^{-T}
//           ybar_k by a d x d solve, form the stage adjoints and scatter
//           them onto the velocity grid.
// This is the exact discrete adjoint (up to rounding) with O(1) state per
// characteristic, the memory property the paper stresses for its forward
// recursion.  Positions are formed with explicit fmaf so both passes select
// bit-identical interpolation cells.
//
// Velocity-grid accumulation goes through an LDS tile per brick of image
// cells (float atomics in LDS, then one atomic per touched tile node into
// global memory); points whose stencil leaves the tile fall back to global
// atomics, so results never depend on the tile margin.

#include <math.h>

#include <vector>

#include "lag_internal.hpp"

namespace lag {

// ---------------------------------------------------------------------------
// small dense helpers
template <int D>
__device__ __forceinline__ void matmul(const float A[D][D], const float B[D][D], float C[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < D; ++k) s = fmaf(A[i][k], B[k][j], s);
      C[i][j] = s;
    }
}

// Jacobian of one RK4 step, M = I + dt/6 (K1 + 2 K2 + 2 K3 + K4) with
// K1 = G1, K2 = G2 (I + dt/2 K1), K3 = G3 (I + dt/2 K2), K4 = G4 (I + dt K3).
template <int D>
__device__ __forceinline__ void step_jacobian(float dt, const float G1[D][D], const float G2[D][D],
                                              const float G3[D][D], const float G4[D][D], float M[D][D]) {
  float A[D][D], K2[D][D], K3[D][D], K4[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A[i][j] = (i == j ? 1.f : 0.f) + 0.5f * dt * G1[i][j];
  matmul<D>(G2, A, K2);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A[i][j] = (i == j ? 1.f : 0.f) + 0.5f * dt * K2[i][j];
  matmul<D>(G3, A, K3);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A[i][j] = (i == j ? 1.f : 0.f) + dt * K3[i][j];
  matmul<D>(G4, A, K4);
  const float c = dt / 6.f;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
      M[i][j] = (i == j ? 1.f : 0.f) + c * (G1[i][j] + 2.f * K2[i][j] + 2.f * K3[i][j] + K4[i][j]);
}

// Solve M^T x = b; returns false if M is (numerically) singular.
__device__ __forceinline__ bool solveT(const float M[3][3], const float b[3], float x[3]) {
  // rows of M^T are the columns of M
  float a00 = M[0][0], a01 = M[1][0], a02 = M[2][0];
  float a10 = M[0][1], a11 = M[1][1], a12 = M[2][1];
  float a20 = M[0][2], a21 = M[1][2], a22 = M[2][2];
  float c00 = a11 * a22 - a12 * a21, c01 = a12 * a20 - a10 * a22, c02 = a10 * a21 - a11 * a20;
  float det = a00 * c00 + a01 * c01 + a02 * c02;
  if (!(fabsf(det) > 1e-20f)) return false;
  float inv = 1.f / det;
  float c10 = a02 * a21 - a01 * a22, c11 = a00 * a22 - a02 * a20, c12 = a01 * a20 - a00 * a21;
  float c20 = a01 * a12 - a02 * a11, c21 = a02 * a10 - a00 * a12, c22 = a00 * a11 - a01 * a10;
  x[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) * inv;
  x[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) * inv;
  x[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * inv;
  return true;
}
__device__ __forceinline__ bool solveT(const float M[2][2], const float b[2], float x[2]) {
  float det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  if (!(fabsf(det) > 1e-20f)) return false;
  float inv = 1.f / det;
  // M^T = [[M00, M10], [M01, M11]]
  x[0] = (M[1][1] * b[0] - M[1][0] * b[1]) * inv;
  x[1] = (-M[0][1] * b[0] + M[0][0] * b[1]) * inv;
  return true;
}

// Frobenius condition number of a step Jacobian divided by the dimension:
// 1 for a scaled rotation (the identity included), growing without bound as
// M approaches a singular matrix (infinite when det M = 0).  Its product over
// the steps bounds how much forward recovery (pass 2) can amplify rounding.
__device__ __forceinline__ float step_cond(const float M[3][3]) {
  float n2 = 0.f, a2 = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) n2 = fmaf(M[i][j], M[i][j], n2);
  const float c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1], c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  const float c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0], c10 = M[0][2] * M[2][1] - M[0][1] * M[2][2];
  const float c11 = M[0][0] * M[2][2] - M[0][2] * M[2][0], c12 = M[0][1] * M[2][0] - M[0][0] * M[2][1];
  const float c20 = M[0][1] * M[1][2] - M[0][2] * M[1][1], c21 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  const float c22 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  a2 = c00 * c00 + c01 * c01 + c02 * c02 + c10 * c10 + c11 * c11 + c12 * c12 + c20 * c20 + c21 * c21 + c22 * c22;
  const float det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
  return sqrtf(n2 * a2) / (3.f * fabsf(det));
}
__device__ __forceinline__ float step_cond(const float M[2][2]) {
  // the adjugate of a 2 x 2 matrix has the same Frobenius norm as M
  const float n2 = M[0][0] * M[0][0] + M[0][1] * M[0][1] + M[1][0] * M[1][0] + M[1][1] * M[1][1];
  const float det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  return n2 / (2.f * fabsf(det));
}

// Forward recovery is used while the product of the step condition numbers
// stays below this bound; beyond it (or if it is not finite) a characteristic
// takes the recomputed reverse sweep instead, which inverts nothing.
constexpr float kMaxRecoveryGrowth = 100.f;

__device__ __forceinline__ bool recovery_ok(float growth) { return growth <= kMaxRecoveryGrowth; }

// Stage positions and the state update, with explicit fmaf so that every
// sweep rounds identically.
template <int D>
__device__ __forceinline__ void stage_pos(const float phi[D], float c, const float k[D], float P[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) P[a] = fmaf(c, k[a], phi[a]);
}
template <int D>
__device__ __forceinline__ void rk4_update(float phi[D], float dt, const float k1[D], const float k2[D],
                                           const float k3[D], const float k4[D]) {
  const float c = dt * (1.f / 6.f);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float s = fmaf(2.f, k2[a], k1[a]);
    s = fmaf(2.f, k3[a], s);
    s = s + k4[a];
    phi[a] = fmaf(c, s, phi[a]);
  }
}

template <int D>
__device__ __forceinline__ void matvec_acc(const float G[D][D], const float x[D], const float e[D], float y[D]) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    float s = e[c];
#pragma unroll
    for (int a = 0; a < D; ++a) s = fmaf(G[c][a], x[a], s);
    y[c] = s;
  }
}

// Plan status bits written by the adjoint kernels (read by lag_plan_flags).
constexpr int kFlagRecompute = 1;  // some characteristic took the recomputed reverse sweep
constexpr int kFlagSingular = 2;   // forward recovery met a singular step (not expected: guarded)
constexpr int kFlagSpill = 4;      // an adjoint value left its tile: added by float atomics (order not fixed)

// Whether every sample of one characteristic falls in a brick's tile (with
// the cell's upper corners): origin and last usable cell offset are uniform
// across the block, so only the flag takes a register per lane.
template <int D>
struct CellBox {
  int org[D];
  int last[D];   // tile size - 2
  bool in;
  __device__ __forceinline__ void reset(const int o[3], const int td[3]) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      org[a] = o[a];
      last[a] = td[a] - 2;
    }
    in = true;
  }
  __device__ __forceinline__ void take(const Loc<D>& L) {
#pragma unroll
    for (int a = 0; a < D; ++a) in = in && (unsigned)(L.c[a] - org[a]) <= (unsigned)last[a];
  }
};

// ---------------------------------------------------------------------------
// pass 1: positions, optional tangent (direction field dp) and flow Jacobian.
template <int D, bool NS, bool TAN, bool FJ>
__device__ __forceinline__ void forward_pass(const Geo& g, const Stages& st,
                                             const typename VecT<D>::T* __restrict__ vp,
                                             const typename VecT<D>::T* __restrict__ dp,
                                             const Start<D>& S, float phi[D], float dphi[D],
                                             float F[D][D], float* growth = nullptr,
                                             CellBox<D>* box = nullptr) {
  constexpr bool GR = TAN || FJ;
  if (FJ && growth) *growth = 1.f;
  const float dt = st.dt, hdt = 0.5f * dt;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    phi[a] = 0.f;
    dphi[a] = 0.f;
#pragma unroll
    for (int b = 0; b < D; ++b) F[a][b] = (a == b) ? 1.f : 0.f;
  }
  for (int k = 0; k < g.nsteps; ++k) {
    const int q = 4 * k;
    float k1[D], k2[D], k3[D], k4[D], P[D];
    float G1[D][D], G2[D][D], G3[D][D], G4[D][D];
    float e[D], Dk[D], Dsum[D], X[D], dummy[D][D];
    Loc<D> L;
    // stage 1 at phi
    locate_v<D>(g, S, phi, L);
    if (box) box->take(L);
    sample_vel<D, NS, GR>(vp, g, st, q, L, k1, G1);
    if (TAN) {
      sample_vel<D, NS, false>(dp, g, st, q, L, e, dummy);
      matvec_acc<D>(G1, dphi, e, Dk);
#pragma unroll
      for (int a = 0; a < D; ++a) { Dsum[a] = Dk[a]; X[a] = fmaf(hdt, Dk[a], dphi[a]); }
    }
    // stage 2 at phi + dt/2 k1
    stage_pos<D>(phi, hdt, k1, P);
    locate_v<D>(g, S, P, L);
    if (box) box->take(L);
    sample_vel<D, NS, GR>(vp, g, st, q + 1, L, k2, G2);
    if (TAN) {
      sample_vel<D, NS, false>(dp, g, st, q + 1, L, e, dummy);
      matvec_acc<D>(G2, X, e, Dk);
#pragma unroll
      for (int a = 0; a < D; ++a) { Dsum[a] = fmaf(2.f, Dk[a], Dsum[a]); X[a] = fmaf(hdt, Dk[a], dphi[a]); }
    }
    // stage 3 at phi + dt/2 k2
    stage_pos<D>(phi, hdt, k2, P);
    locate_v<D>(g, S, P, L);
    if (box) box->take(L);
    sample_vel<D, NS, GR>(vp, g, st, q + 2, L, k3, G3);
    if (TAN) {
      sample_vel<D, NS, false>(dp, g, st, q + 2, L, e, dummy);
      matvec_acc<D>(G3, X, e, Dk);
#pragma unroll
      for (int a = 0; a < D; ++a) { Dsum[a] = fmaf(2.f, Dk[a], Dsum[a]); X[a] = fmaf(dt, Dk[a], dphi[a]); }
    }
    // stage 4 at phi + dt k3
    stage_pos<D>(phi, dt, k3, P);
    locate_v<D>(g, S, P, L);
    if (box) box->take(L);
    sample_vel<D, NS, GR>(vp, g, st, q + 3, L, k4, G4);
    if (TAN) {
      sample_vel<D, NS, false>(dp, g, st, q + 3, L, e, dummy);
      matvec_acc<D>(G4, X, e, Dk);
#pragma unroll
      for (int a = 0; a < D; ++a) dphi[a] = fmaf(dt * (1.f / 6.f), Dsum[a] + Dk[a], dphi[a]);
    }
    if (FJ) {
      float M[D][D], Fn[D][D];
      step_jacobian<D>(dt, G1, G2, G3, G4, M);
      if (growth) *growth *= step_cond(M);
      matmul<D>(M, F, Fn);
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) F[a][b] = Fn[a][b];
    }
    rk4_update<D>(phi, dt, k1, k2, k3, k4);
  }
}

// ---------------------------------------------------------------------------
// v 2^e rounded to the nearest integer, as a two's-complement 64-bit word,
// for |v| 2^e < 2^62, in float arithmetic: t = v 2^(e-32) splits exactly
// into floor(t) (an int32) and the fraction t - floor(t), whose scaling by
// 2^32 is exact and is rounded to the nearest integer (at most 2^32 - 256).
__device__ __forceinline__ unsigned long long fix64(float v, int e) {
  const float t = ldexpf(v, e - 32);
  const float hi = floorf(t);
  const unsigned lo = __float2uint_rn(ldexpf(t - hi, 32));
  return ((unsigned long long)(long long)(int)hi << 32) + lo;
}

// ---------------------------------------------------------------------------
// Velocity-grid accumulators of the matrix-free adjoint products.  A scatter
// hands over one sample (add: corner weights times a stage adjoint, split
// between two time nodes for a time-dependent field) or one register-merged
// cell (add_block: 2^d corners x d components per time slot); the three
// accumulators differ only in where the values go.
//
// AdjTile: the brick's LDS tile in 64-bit fixed point with unit 2^-e.  An
// integer sum does not depend on the order of its additions, so the tile is
// the same bit for bit on every run; sabs sums the magnitudes the thread
// added (their block-wide sum bounds every partial sum of the tile).  Cells
// outside the tile do not occur for a characteristic whose forward cells
// passed CellBox::inside (the adjoint replay samples the same cells); should
// one occur, its values go to the output by float atomics and `spill` is set.
template <int D, bool NS>
struct AdjTile {
  unsigned long long* tile;
  float* gout;
  const int* j0;
  const float* th;
  int org[3];
  int td[3];
  int mv[3];
  int tvol;
  long long nv;
  int e;
  float sabs;
  bool spill;

  __device__ __forceinline__ bool base_of(const int c[D], int& base) const {
    bool in = true;
    int t[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      t[a] = c[a] - org[a];
      in = in && (t[a] >= 0) && (t[a] + 1 < td[a]);
    }
    base = (t[2] * td[1] + t[1]) * td[0] + t[0];
    return in;
  }
  __device__ __forceinline__ int corner_off(int base, int o) const {
    int off = base + (o & 1) + ((o >> 1) & 1) * td[0];
    if (D == 3) off += ((o >> 2) & 1) * td[0] * td[1];
    return off;
  }
  __device__ __forceinline__ void put(int i, float v) {
    atomicAdd(&tile[i], fix64(v, e));
    sabs += fabsf(v);
  }
  __device__ __forceinline__ void spill_put(const int c[D], int o, int field, float v) {
    Loc<D> L;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      L.c[a] = c[a];
      L.f[a] = 0.f;
    }
    unsafeAtomicAdd(&gout[(long long)field * nv + corner_index<D>(L, mv, o)], v);
    spill = true;
  }

  __device__ __forceinline__ void add(const Loc<D>& L, int q, const float kb[D]) {
    float w[1 << D];
    corner_weights<D>(L, w);
    int jA = 0;
    float wA = 1.f, wB = 0.f;
    if (NS) {
      jA = j0[q];
      wB = th[q];
      wA = 1.f - wB;
    }
    int base;
    if (base_of(L.c, base)) {
#pragma unroll
      for (int o = 0; o < (1 << D); ++o) {
        const int off = corner_off(base, o);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float val = w[o] * kb[c];
          put((jA * D + c) * tvol + off, wA * val);
          if (NS) put(((jA + 1) * D + c) * tvol + off, wB * val);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int o = 0; o < (1 << D); ++o)
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float val = w[o] * kb[c];
          spill_put(L.c, o, jA * D + c, wA * val);
          if (NS) spill_put(L.c, o, (jA + 1) * D + c, wB * val);
        }
    }
  }

  template <int NSLOT>
  __device__ __forceinline__ void add_block(const int cell[D], int jA, const float a[NSLOT][1 << D][D]) {
    int base;
    if (base_of(cell, base)) {
#pragma unroll
      for (int o = 0; o < (1 << D); ++o) {
        const int off = corner_off(base, o);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s)
#pragma unroll
          for (int c = 0; c < D; ++c) put(((jA + s) * D + c) * tvol + off, a[s][o][c]);
        // one corner's conversions at a time (they would otherwise be
        // hoisted ahead of the atomics, each holding a register)
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int o = 0; o < (1 << D); ++o)
#pragma unroll
        for (int s = 0; s < NSLOT; ++s)
#pragma unroll
          for (int c = 0; c < D; ++c) spill_put(cell, o, (jA + s) * D + c, a[s][o][c]);
    }
  }
};

// AdjBound: the magnitude sum of what a characteristic scatters, with no
// memory traffic (the same values as the other accumulators).
template <int D, bool NS>
struct AdjBound {
  const int* j0;
  const float* th;
  float sabs;

  __device__ __forceinline__ void add(const Loc<D>& L, int q, const float kb[D]) {
    float w[1 << D];
    corner_weights<D>(L, w);
    float wA = 1.f, wB = 0.f;
    if (NS) {
      wB = th[q];
      wA = 1.f - wB;
    }
#pragma unroll
    for (int o = 0; o < (1 << D); ++o)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const float val = w[o] * kb[c];
        sabs += fabsf(wA * val);
        if (NS) sabs += fabsf(wB * val);
      }
  }

  template <int NSLOT>
  __device__ __forceinline__ void add_block(const int*, int, const float a[NSLOT][1 << D][D]) {
#pragma unroll
    for (int o = 0; o < (1 << D); ++o)
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) sabs += fabsf(a[s][o][c]);
  }
};

// AdjWide: 64-bit fixed point with unit 2^-e in a grid-sized buffer (the
// characteristics that leave their tile); integer atomics, so the sum does
// not depend on the order either.
template <int D, bool NS>
struct AdjWide {
  unsigned long long* acc;
  const int* j0;
  const float* th;
  int mv[3];
  long long nv;
  int e;

  __device__ __forceinline__ void put(long long gi, int field, float v) {
    const long long q = __double2ll_rn(ldexp((double)v, e));
    atomicAdd(&acc[(long long)field * nv + gi], (unsigned long long)q);
  }

  __device__ __forceinline__ void add(const Loc<D>& L, int q, const float kb[D]) {
    float w[1 << D];
    corner_weights<D>(L, w);
    int jA = 0;
    float wA = 1.f, wB = 0.f;
    if (NS) {
      jA = j0[q];
      wB = th[q];
      wA = 1.f - wB;
    }
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      const long long gi = corner_index<D>(L, mv, o);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const float val = w[o] * kb[c];
        put(gi, jA * D + c, wA * val);
        if (NS) put(gi, (jA + 1) * D + c, wB * val);
      }
    }
  }

  template <int NSLOT>
  __device__ __forceinline__ void add_block(const int cell[D], int jA, const float a[NSLOT][1 << D][D]) {
    Loc<D> L;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      L.c[ax] = cell[ax];
      L.f[ax] = 0.f;
    }
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      const long long gi = corner_index<D>(L, mv, o);
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) put(gi, (jA + s) * D + c, a[s][o][c]);
    }
  }
};

// Register accumulator that merges the scatter of consecutive samples
// falling in the same velocity cell (and time interval); it is flushed to
// the tile only when the cell changes, which cuts LDS atomics by the number
// of RK4 stages spent inside one cell.
template <int D, bool NS>
struct Merge {
  static constexpr int NSLOT = NS ? 2 : 1;
  int cell[D];
  int j0;
  bool active;
  float a[NSLOT][1 << D][D];

  __device__ __forceinline__ void reset() { active = false; }

  template <class Acc>
  __device__ __forceinline__ void flush(Acc& acc) {
    if (active) acc.template add_block<NSLOT>(cell, j0, a);
    active = false;
  }

  template <class Acc>
  __device__ __forceinline__ void add(Acc& acc, const Stages& st, const Loc<D>& L, int q, const float kb[D]) {
    int jA = NS ? st.j0[q] : 0;
    float th = NS ? st.th[q] : 0.f;
    bool same = active && (jA == j0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) same = same && (L.c[ax] == cell[ax]);
    if (!same) {
      flush(acc);
      active = true;
      j0 = jA;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) cell[ax] = L.c[ax];
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
#pragma unroll
        for (int o = 0; o < (1 << D); ++o)
#pragma unroll
          for (int c = 0; c < D; ++c) a[s][o][c] = 0.f;
    }
    float w[1 << D];
    corner_weights<D>(L, w);
#pragma unroll
    for (int o = 0; o < (1 << D); ++o)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        float val = w[o] * kb[c];
        if (NS) {
          a[0][o][c] = fmaf(1.f - th, val, a[0][o][c]);
          a[1][o][c] = fmaf(th, val, a[1][o][c]);
        } else {
          a[0][o][c] += val;
        }
      }
  }
};

// 3-D time-dependent fields would need 48 merge registers; they scatter
// every sample directly instead.
template <int D, bool NS>
struct UseMerge {
  static constexpr bool value = !(NS && D == 3);
};

// pass 2: replay the sweep, recover the step adjoints and scatter them.
// The four stage adjoints of a step are formed last-to-first (each depends
// on the next) and then scattered first-to-last, so that consecutive
// scatters move monotonically along the characteristic and the register
// merge sees each crossed cell once.
template <int D, bool NS, class Acc>
__device__ __forceinline__ bool adjoint_pass(const Geo& g, const Stages& st,
                                             const typename VecT<D>::T* __restrict__ vp,
                                             const Start<D>& S, float ybar[D], Acc& acc) {
  const float dt = st.dt, hdt = 0.5f * dt;
  float phi[D];
  bool ok = true;
  constexpr bool MERGE = UseMerge<D, NS>::value;
  Merge<D, NS> mg;
  mg.reset();
  auto scat = [&](const Loc<D>& L, int q, const float kb[D]) {
    if constexpr (MERGE) mg.add(acc, st, L, q, kb);
    else acc.add(L, q, kb);
  };
#pragma unroll
  for (int a = 0; a < D; ++a) phi[a] = 0.f;
  for (int k = 0; k < g.nsteps; ++k) {
    const int q = 4 * k;
    float k1[D], k2[D], k3[D], k4[D], P[D];
    float G1[D][D], G2[D][D], G3[D][D], G4[D][D];
    Loc<D> L1, L2, L3, L4;
    locate_v<D>(g, S, phi, L1);
    sample_vel<D, NS, true>(vp, g, st, q, L1, k1, G1);
    stage_pos<D>(phi, hdt, k1, P);
    locate_v<D>(g, S, P, L2);
    sample_vel<D, NS, true>(vp, g, st, q + 1, L2, k2, G2);
    stage_pos<D>(phi, hdt, k2, P);
    locate_v<D>(g, S, P, L3);
    sample_vel<D, NS, true>(vp, g, st, q + 2, L3, k3, G3);
    stage_pos<D>(phi, dt, k3, P);
    locate_v<D>(g, S, P, L4);
    sample_vel<D, NS, true>(vp, g, st, q + 3, L4, k4, G4);

    float M[D][D], yn[D];
    step_jacobian<D>(dt, G1, G2, G3, G4, M);
    if (!solveT(M, ybar, yn)) {
      ok = false;
#pragma unroll
      for (int a = 0; a < D; ++a) yn[a] = ybar[a];
    }
    // adjoints of the stage velocities, last stage first
    float kb1[D], kb2[D], kb3[D], kb4[D], pb[D];
    const float c6 = dt * (1.f / 6.f), c3 = dt * (1.f / 3.f);
#pragma unroll
    for (int a = 0; a < D; ++a) kb4[a] = c6 * yn[a];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float t = 0.f;
#pragma unroll
      for (int c = 0; c < D; ++c) t = fmaf(G4[c][a], kb4[c], t);
      pb[a] = t;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) kb3[a] = fmaf(dt, pb[a], c3 * yn[a]);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float t = 0.f;
#pragma unroll
      for (int c = 0; c < D; ++c) t = fmaf(G3[c][a], kb3[c], t);
      pb[a] = t;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) kb2[a] = fmaf(hdt, pb[a], c3 * yn[a]);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float t = 0.f;
#pragma unroll
      for (int c = 0; c < D; ++c) t = fmaf(G2[c][a], kb2[c], t);
      pb[a] = t;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) kb1[a] = fmaf(hdt, pb[a], c6 * yn[a]);
    scat(L1, q, kb1);
    scat(L2, q + 1, kb2);
    scat(L3, q + 2, kb3);
    scat(L4, q + 3, kb4);
#pragma unroll
    for (int a = 0; a < D; ++a) ybar[a] = yn[a];
    rk4_update<D>(phi, dt, k1, k2, k3, k4);
  }
  if constexpr (MERGE) mg.flush(acc);
  return ok;
}

// adjoint_pass at v = 0: no characteristic moves, every stage point is the
// start point and every step Jacobian the identity, so each step's stage
// adjoints are the RK4 weights dt/6, dt/3, dt/3, dt/6 times the constant
// adjoint, all scattered at the start point.  For a stationary field they
// are one contribution with the summed weights (zero_add: the same terms up
// to the order of the float additions), merged in the caller's register
// accumulator across the thread's characteristics, which start in the same
// velocity cell for all phases of a region; a time-dependent field splits
// every stage between its two nodes and keeps one scatter per stage.
template <int D, class Acc>
__device__ __forceinline__ void zero_add(const Geo& g, const Stages& st, const Start<D>& S, const float ybar[D],
                                         Acc& acc, Merge<D, false>& mg) {
  const float dt = st.dt;
  const float c6 = dt * (1.f / 6.f), c3 = dt * (1.f / 3.f);
  float wsum = 0.f;
  for (int k = 0; k < g.nsteps; ++k) wsum += (c6 + c3) + (c3 + c6);
  float phi[D], kb[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    phi[a] = 0.f;
    kb[a] = wsum * ybar[a];
  }
  Loc<D> L;
  locate_v<D>(g, S, phi, L);
  mg.add(acc, st, L, 0, kb);
}

template <int D, bool NS, class Acc>
__device__ __forceinline__ void zero_adjoint(const Geo& g, const Stages& st, const Start<D>& S, const float ybar[D],
                                             Acc& acc) {
  const float dt = st.dt;
  float phi[D], k6[D], k3[D];
  const float c6 = dt * (1.f / 6.f), c3 = dt * (1.f / 3.f);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    phi[a] = 0.f;
    k6[a] = c6 * ybar[a];
    k3[a] = c3 * ybar[a];
  }
  Loc<D> L;
  locate_v<D>(g, S, phi, L);
  constexpr bool MERGE = UseMerge<D, NS>::value;
  Merge<D, NS> mg;
  mg.reset();
  auto scat = [&](const Loc<D>& L, int q, const float kb[D]) {
    if constexpr (MERGE) mg.add(acc, st, L, q, kb);
    else acc.add(L, q, kb);
  };
  for (int k = 0; k < g.nsteps; ++k) {
    const int q = 4 * k;
    scat(L, q, k6);
    scat(L, q + 1, k3);
    scat(L, q + 2, k3);
    scat(L, q + 3, k6);
  }
  if constexpr (MERGE) mg.flush(acc);
}

// Stored-trajectory variant for the assembly.  Pass 1 records the step start
// points phi_k (k = 0..N-1) of the characteristic, with the same operations
// as forward_pass without tangents; pass 2 runs the exact reverse sweep of
// the discrete RK4 map (eq. phiRK4): from lambda_N = grad T(phi_N), each step
// back forms the stage adjoints and lambda_k = lambda_{k+1} + sum_i G_i^T kb_i,
// and scatters kb_i at the stage points (last stage first).  No flow
// Jacobian and no 3x3 solves: fewer operations than forward recovery, and
// no failure when a step Jacobian is singular.  `traj` is this thread's
// slice of an LDS array with stride `ts` floats between entries.
template <int D>
__device__ __forceinline__ void forward_record(const Geo& g, const Stages& st,
                                               const typename VecT<D>::T* __restrict__ vp, const Start<D>& S,
                                               float phi[D], float* traj, int ts) {
  const float dt = st.dt, hdt = 0.5f * dt;
  float G[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a) phi[a] = 0.f;
  for (int k = 0; k < g.nsteps; ++k) {
    const int q = 4 * k;
#pragma unroll
    for (int a = 0; a < D; ++a) traj[(k * D + a) * ts] = phi[a];
    float k1[D], k2[D], k3[D], k4[D], P[D];
    Loc<D> L;
    locate_v<D>(g, S, phi, L);
    sample_vel<D, false, false>(vp, g, st, q, L, k1, G);
    stage_pos<D>(phi, hdt, k1, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, false, false>(vp, g, st, q + 1, L, k2, G);
    stage_pos<D>(phi, hdt, k2, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, false, false>(vp, g, st, q + 2, L, k3, G);
    stage_pos<D>(phi, dt, k3, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, false, false>(vp, g, st, q + 3, L, k4, G);
    rk4_update<D>(phi, dt, k1, k2, k3, k4);
  }
}

// One step back of the exact reverse sweep of the RK4 map (eq. phiRK4): from
// the step start point phi_k and lam = lambda_{k+1}, recompute the four
// stages, form the stage adjoints (last to first), hand them to
// scat(L, q, kb) last stage first, and return lambda_k in lam.
template <int D, bool NS, class Scat>
__device__ __forceinline__ void reverse_step(const Geo& g, const Stages& st,
                                             const typename VecT<D>::T* __restrict__ vp, const Start<D>& S,
                                             int k, const float phi[D], float lam[D], Scat scat) {
  const float dt = st.dt, hdt = 0.5f * dt;
  const float c6 = dt * (1.f / 6.f), c3 = dt * (1.f / 3.f);
  const int q = 4 * k;
  float k1[D], k2[D], k3[D], k4[D], P[D];
  float G1[D][D], G2[D][D], G3[D][D], G4[D][D];
  Loc<D> L1, L2, L3, L4;
  locate_v<D>(g, S, phi, L1);
  sample_vel<D, NS, true>(vp, g, st, q, L1, k1, G1);
  stage_pos<D>(phi, hdt, k1, P);
  locate_v<D>(g, S, P, L2);
  sample_vel<D, NS, true>(vp, g, st, q + 1, L2, k2, G2);
  stage_pos<D>(phi, hdt, k2, P);
  locate_v<D>(g, S, P, L3);
  sample_vel<D, NS, true>(vp, g, st, q + 2, L3, k3, G3);
  stage_pos<D>(phi, dt, k3, P);
  locate_v<D>(g, S, P, L4);
  sample_vel<D, NS, true>(vp, g, st, q + 3, L4, k4, G4);
  (void)k4;
  float kb1[D], kb2[D], kb3[D], kb4[D], pb[D], sum[D];
#pragma unroll
  for (int a = 0; a < D; ++a) kb4[a] = c6 * lam[a];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < D; ++c) t = fmaf(G4[c][a], kb4[c], t);
    pb[a] = t;
    sum[a] = t;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) kb3[a] = fmaf(dt, pb[a], c3 * lam[a]);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < D; ++c) t = fmaf(G3[c][a], kb3[c], t);
    pb[a] = t;
    sum[a] += t;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) kb2[a] = fmaf(hdt, pb[a], c3 * lam[a]);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < D; ++c) t = fmaf(G2[c][a], kb2[c], t);
    pb[a] = t;
    sum[a] += t;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) kb1[a] = fmaf(hdt, pb[a], c6 * lam[a]);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < D; ++c) t = fmaf(G1[c][a], kb1[c], t);
    sum[a] += t;
  }
  scat(L4, q + 3, kb4);
  scat(L3, q + 2, kb3);
  scat(L2, q + 1, kb2);
  scat(L1, q, kb1);
#pragma unroll
  for (int a = 0; a < D; ++a) lam[a] += sum[a];
}

template <int D, class Acc>
__device__ __forceinline__ void reverse_sweep(const Geo& g, const Stages& st,
                                              const typename VecT<D>::T* __restrict__ vp, const Start<D>& S,
                                              const float* traj, int ts, float lam[D], Acc& acc) {
  Merge<D, false> mg;
  mg.reset();
  for (int k = g.nsteps - 1; k >= 0; --k) {
    float phi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) phi[a] = traj[(k * D + a) * ts];
    reverse_step<D, false>(g, st, vp, S, k, phi, lam,
                           [&](const Loc<D>& L, int q, const float kb[D]) { mg.add(acc, st, L, q, kb); });
  }
  mg.flush(acc);
}

// The same reverse sweep without stored step start points: phi_k is traced
// again from the start point for every k (the operations of forward_pass,
// so the cells are bitwise those of the forward pass).  O(N^2) samples and
// O(1) state, no step Jacobian is inverted: the fallback of forward recovery
// for characteristics whose step Jacobians are (nearly) singular.  lam is
// lambda_N on entry.
template <int D, bool NS>
__device__ __forceinline__ void retrace(const Geo& g, const Stages& st,
                                        const typename VecT<D>::T* __restrict__ vp, const Start<D>& S,
                                        int ksteps, float phi[D]) {
  const float dt = st.dt, hdt = 0.5f * dt;
  float G[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a) phi[a] = 0.f;
  for (int k = 0; k < ksteps; ++k) {
    const int q = 4 * k;
    float k1[D], k2[D], k3[D], k4[D], P[D];
    Loc<D> L;
    locate_v<D>(g, S, phi, L);
    sample_vel<D, NS, false>(vp, g, st, q, L, k1, G);
    stage_pos<D>(phi, hdt, k1, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, NS, false>(vp, g, st, q + 1, L, k2, G);
    stage_pos<D>(phi, hdt, k2, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, NS, false>(vp, g, st, q + 2, L, k3, G);
    stage_pos<D>(phi, dt, k3, P);
    locate_v<D>(g, S, P, L);
    sample_vel<D, NS, false>(vp, g, st, q + 3, L, k4, G);
    rk4_update<D>(phi, dt, k1, k2, k3, k4);
  }
}

template <int D, bool NS, class Acc>
__device__ __forceinline__ void reverse_recompute(const Geo& g, const Stages& st,
                                                  const typename VecT<D>::T* __restrict__ vp, const Start<D>& S,
                                                  float lam[D], Acc& acc) {
  constexpr bool MERGE = UseMerge<D, NS>::value;
  Merge<D, NS> mg;
  mg.reset();
  for (int k = g.nsteps - 1; k >= 0; --k) {
    float phi[D];
    retrace<D, NS>(g, st, vp, S, k, phi);
    reverse_step<D, NS>(g, st, vp, S, k, phi, lam, [&](const Loc<D>& L, int q, const float kb[D]) {
      if constexpr (MERGE) mg.add(acc, st, L, q, kb);
      else acc.add(L, q, kb);
    });
  }
  if constexpr (MERGE) mg.flush(acc);
}

// ---------------------------------------------------------------------------
// kernels

// Interleave the D components of each node (per time node) and add the
// periodic ghost layer: packed node (X, Y, Z), X <= mv[0] etc., holds grid
// node (X mod mv[0], Y mod mv[1], Z mod mv[2]).
template <int D>
__global__ void __launch_bounds__(kBlock) k_pack(const float* __restrict__ v, typename VecT<D>::T* __restrict__ out,
                                                 Geo g, const int* __restrict__ halt) {
  if (halted(halt)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = g.nvp * g.nodes;
  if (i >= tot) return;
  const long long j = i / g.nvp, q = i - j * g.nvp;
  const int X = (int)(q % g.pv[0]), Y = (int)((q / g.pv[0]) % g.pv[1]), Z = (int)(q / ((long long)g.pv[0] * g.pv[1]));
  const int x = X == g.mv[0] ? 0 : X, y = Y == g.mv[1] ? 0 : Y, z = Z == g.mv[2] ? 0 : Z;
  const long long nv = g.nv;
  const float* b = v + j * D * nv + ((long long)z * g.mv[1] + y) * g.mv[0] + x;
  if constexpr (D == 3) {
    out[i] = make_float4(b[0], b[nv], b[2 * nv], 0.f);
  } else {
    out[i] = make_float2(b[0], b[nv]);
  }
}

__global__ void __launch_bounds__(kBlock) k_fill(float* __restrict__ x, long long n, float val) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = val;
}

template <int D, bool NS>
__global__ void __launch_bounds__(kBlock) k_trace(Geo g, Stages st, const typename VecT<D>::T* __restrict__ vp,
                                                  float* __restrict__ phi_out) {
  long long blk = xcd_block((g.np + kBlock - 1) / kBlock);
  if (blk < 0) return;
  long long p = blk * kBlock + threadIdx.x;
  if (p >= g.np) return;
  Start<D> S;
  make_start<D>(g, p, S);
  float phi[D], dphi[D], F[D][D];
  forward_pass<D, NS, false, false>(g, st, vp, nullptr, S, phi, dphi, F);
#pragma unroll
  for (int a = 0; a < D; ++a) phi_out[a * g.np + p] = phi[a];
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_transport(Geo g, const float* __restrict__ T, const float* __restrict__ phi,
                                                      float* __restrict__ u) {
  long long blk = xcd_block((g.np + kBlock - 1) / kBlock);
  if (blk < 0) return;
  long long p = blk * kBlock + threadIdx.x;
  if (p >= g.np) return;
  Start<D> S;
  long long r = p;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S.i[a] = (int)(r % g.mi[a]);
    r /= g.mi[a];
  }
  float ph[D];
#pragma unroll
  for (int a = 0; a < D; ++a) ph[a] = phi[a * g.np + p];
  Loc<D> L;
  locate_i<D>(g, S, ph, L);
  float val, grad[D];
  sample_img<D, true, false>(T, g, L, val, grad);
  u[p] = val;
}

// transport JVP: Jdv_i = grad T(y_i) . dy_i
template <int D, bool NS>
__global__ void __launch_bounds__(kBlock) k_jvp_transport(Geo g, Stages st, const typename VecT<D>::T* __restrict__ vp,
                                                          const typename VecT<D>::T* __restrict__ dp,
                                                          const float* __restrict__ T, float* __restrict__ out) {
  long long blk = xcd_block((g.np + kBlock - 1) / kBlock);
  if (blk < 0) return;
  long long p = blk * kBlock + threadIdx.x;
  if (p >= g.np) return;
  Start<D> S;
  make_start<D>(g, p, S);
  float phi[D], dphi[D], F[D][D];
  forward_pass<D, NS, true, false>(g, st, vp, dp, S, phi, dphi, F);
  Loc<D> L;
  locate_i<D>(g, S, phi, L);
  float val, gT[D];
  sample_img<D, false, true>(T, g, L, val, gT);
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < D; ++a) s = fmaf(gT[a], dphi[a], s);
  out[p] = s;
}

// continuity JVP, first half: per particle, the 2^d corner contributions
// T_j grad w_o(y_j) . dy_j and the base cell, plus the bin count.
template <int D, bool NS>
__global__ void __launch_bounds__(kBlock) k_jvp_cont_prep(Geo g, Stages st, const typename VecT<D>::T* __restrict__ vp,
                                                          const typename VecT<D>::T* __restrict__ dp,
                                                          const float* __restrict__ T, int* __restrict__ base,
                                                          float* __restrict__ vals, int* __restrict__ count) {
  if (halted(g.halt)) return;
  long long blk = xcd_block((g.np + kBlock - 1) / kBlock);
  if (blk < 0) return;
  long long p = blk * kBlock + threadIdx.x;
  if (p >= g.np) return;
  Start<D> S;
  make_start<D>(g, p, S);
  float phi[D], dphi[D], F[D][D];
  forward_pass<D, NS, true, false>(g, st, vp, dp, S, phi, dphi, F);
  Loc<D> L;
  locate_i<D>(g, S, phi, L);
  float dw[1 << D][D];
  corner_dweights<D>(L, g.inv_hi, dw);
  const float m = T[p];
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) s = fmaf(dw[o][a], dphi[a], s);
    vals[(long long)o * g.np + p] = m * s;
  }
  int b = (int)corner_index<D>(L, g.mi, 0);
  base[p] = b;
  atomicAdd(&count[b], 1);
}

// push-forward, first half: corner weights times the particle mass.
template <int D>
__global__ void __launch_bounds__(kBlock) k_push_prep(Geo g, const float* __restrict__ T, const float* __restrict__ phi,
                                                      int* __restrict__ base, float* __restrict__ vals,
                                                      int* __restrict__ count) {
  long long blk = xcd_block((g.np + kBlock - 1) / kBlock);
  if (blk < 0) return;
  long long p = blk * kBlock + threadIdx.x;
  if (p >= g.np) return;
  Start<D> S;
  long long r = p;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S.i[a] = (int)(r % g.mi[a]);
    r /= g.mi[a];
  }
  float ph[D];
#pragma unroll
  for (int a = 0; a < D; ++a) ph[a] = phi[a * g.np + p];
  Loc<D> L;
  locate_i<D>(g, S, ph, L);
  float w[1 << D];
  corner_weights<D>(L, w);
  const float m = T[p];
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) vals[(long long)o * g.np + p] = m * w[o];
  int b = (int)corner_index<D>(L, g.mi, 0);
  base[p] = b;
  atomicAdd(&count[b], 1);
}

// ---------------------------------------------------------------------------
// brick kernels with an LDS accumulation tile

template <int D>
__device__ __forceinline__ void brick_origin(const Geo& g, const Bricks& B, long long bid, int O[3], int org[3]) {
  int b0 = (int)(bid % B.nb[0]);
  int b1 = (int)((bid / B.nb[0]) % B.nb[1]);
  int b2 = (int)(bid / ((long long)B.nb[0] * B.nb[1]));
  int bb[3] = {b0, b1, b2};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    O[a] = bb[a] * B.bdim[a];
    if (a < D) {
      double s = ((double)O[a] + 0.5) * g.ratio[a] - 0.5;
      org[a] = (int)floor(s) - B.halo;
    } else {
      org[a] = 0;
    }
  }
}

// A brick is split into 64-row items, (region, phase) pairs: within an item
// the 64 lanes sit `stride` image cells apart on the lane lattice, so that
// they start in distinct velocity cells (few LDS atomic collisions).
__device__ __forceinline__ int brick_items(const Bricks& B) {
  return B.nreg[0] * B.nreg[1] * B.nreg[2] * B.stride[0] * B.stride[1] * B.stride[2];
}

// Image cell of the row that lattice position l takes in item w of the brick
// with origin O; false when that cell lies outside the image.
template <int D>
__device__ __forceinline__ bool item_cell(const Geo& g, const Bricks& B, const int O[3], int w, const int l[3],
                                          int idx[3]) {
  const int P = B.stride[0] * B.stride[1] * B.stride[2];
  const int reg = w / P, ph = w - reg * P;
  const int r0 = reg % B.nreg[0], r1 = (reg / B.nreg[0]) % B.nreg[1], r2 = reg / (B.nreg[0] * B.nreg[1]);
  const int p0 = ph % B.stride[0], p1 = (ph / B.stride[0]) % B.stride[1], p2 = ph / (B.stride[0] * B.stride[1]);
  idx[0] = O[0] + r0 * B.rdim[0] + l[0] * B.stride[0] + p0;
  idx[1] = O[1] + r1 * B.rdim[1] + l[1] * B.stride[1] + p1;
  idx[2] = O[2] + r2 * B.rdim[2] + l[2] * B.stride[2] + p2;
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) in = in && idx[a] < g.mi[a];
  return in;
}

// Iterate over the characteristics of a brick, one item per wave at a time.
template <int D, class Body>
__device__ __forceinline__ void for_brick_points(const Geo& g, const Bricks& B, const int O[3], Body body) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int l[3];
  lane_lattice(B, lane, l);
  const int items = brick_items(B);
  for (int w = wave; w < items; w += nw) {
    int idx[3];
    if (item_cell<D>(g, B, O, w, l, idx)) body(idx);
  }
}

// ---------------------------------------------------------------------------
// RK4 trace through an LDS-staged velocity tile (stationary fields).  One
// block per brick stages the brick's velocity footprint (the same tile
// geometry as the accumulation tiles: brick plus halo, padded strides) as
// D planes of floats, then traces the brick's characteristics reading the
// eight corners of every sample from LDS; a sample whose cell leaves the
// tile reads the packed field in HBM instead.  The interpolation performs
// the same operations in the same order as sample_vec, so the result is
// bitwise that of k_trace.
template <int D>
struct VelTile {
  const float* lds;  // [D][tvol]
  int org[3];
  int td[3];
  int tvol;
};

template <int D>
__device__ __forceinline__ void sample_tile(const typename VecT<D>::T* __restrict__ vp, const Geo& g,
                                            const VelTile<D>& T, const Loc<D>& L, float val[D]) {
  bool in = true;
  int t[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    t[a] = L.c[a] - T.org[a];
    in = in && (t[a] >= 0) && (t[a] + 1 < T.td[a]);
  }
  if (!in) {
    float G[D][D];
    sample_vec<false>(vp, g, L, val, G);
    return;
  }
  const int sy = T.td[0];
  if constexpr (D == 3) {
    const int sz = T.td[0] * T.td[1];
    const int b = (t[2] * T.td[1] + t[1]) * T.td[0] + t[0];
    const float fx = L.f[0], fy = L.f[1], fz = L.f[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* f = T.lds + c * T.tvol + b;
      const float a000 = f[0], a100 = f[1], a010 = f[sy], a110 = f[sy + 1];
      const float a001 = f[sz], a101 = f[sz + 1], a011 = f[sz + sy], a111 = f[sz + sy + 1];
      const float e00 = lerpf(a000, a100, fx), e10 = lerpf(a010, a110, fx);
      const float e01 = lerpf(a001, a101, fx), e11 = lerpf(a011, a111, fx);
      const float g0 = lerpf(e00, e10, fy), g1 = lerpf(e01, e11, fy);
      val[c] = lerpf(g0, g1, fz);
    }
  } else {
    const int b = t[1] * T.td[0] + t[0];
    const float fx = L.f[0], fy = L.f[1];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float* f = T.lds + c * T.tvol + b;
      const float e0 = lerpf(f[0], f[1], fx), e1 = lerpf(f[sy], f[sy + 1], fx);
      val[c] = lerpf(e0, e1, fy);
    }
  }
}

// 512 threads (8 waves) share a brick's tile: the 52 KB tile lets three
// blocks onto a CU, so the waves per CU are set by the block size.
constexpr int kTraceBlock = 512;

template <int D>
__global__ void __launch_bounds__(kTraceBlock) k_trace_tile(Geo g, Stages st, Bricks B,
                                                       const typename VecT<D>::T* __restrict__ vp,
                                                       float* __restrict__ phi_out) {
  extern __shared__ float vtile[];
  const long long bid = xcd_block(B.nbricks);
  if (bid < 0) return;
  int O[3], org[3];
  brick_origin<D>(g, B, bid, O, org);
  VelTile<D> T;
  T.lds = vtile;
  T.tvol = B.tvol;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T.org[a] = org[a];
    T.td[a] = B.tdim[a];
  }
  // stage the footprint: node (org + t) of the periodic grid, one packed
  // vector load per node
  for (int i = threadIdx.x; i < B.tvol; i += blockDim.x) {
    const int t0 = i % B.tdim[0], t1 = (i / B.tdim[0]) % B.tdim[1], t2 = i / (B.tdim[0] * B.tdim[1]);
    const int x = wrapi(org[0] + t0, g.mv[0]), y = wrapi(org[1] + t1, g.mv[1]);
    const int z = D == 3 ? wrapi(org[2] + t2, g.mv[2]) : 0;
    const auto q = vp[packed_corner(g, x, y, z)];
    vtile[i] = q.x;
    vtile[B.tvol + i] = q.y;
    if constexpr (D == 3) vtile[2 * B.tvol + i] = q.z;
  }
  __syncthreads();
  const float dt = st.dt, hdt = 0.5f * dt;
  for_brick_points<D>(g, B, O, [&](const int idx[3]) {
    Start<D> S;
    make_start_idx<D>(g, idx, S);
    float phi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) phi[a] = 0.f;
    for (int k = 0; k < g.nsteps; ++k) {
      float k1[D], k2[D], k3[D], k4[D], P[D];
      Loc<D> L;
      locate_v<D>(g, S, phi, L);
      sample_tile<D>(vp, g, T, L, k1);
      stage_pos<D>(phi, hdt, k1, P);
      locate_v<D>(g, S, P, L);
      sample_tile<D>(vp, g, T, L, k2);
      stage_pos<D>(phi, hdt, k2, P);
      locate_v<D>(g, S, P, L);
      sample_tile<D>(vp, g, T, L, k3);
      stage_pos<D>(phi, dt, k3, P);
      locate_v<D>(g, S, P, L);
      sample_tile<D>(vp, g, T, L, k4);
      rk4_update<D>(phi, dt, k1, k2, k3, k4);
    }
    long long p = idx[0] + (long long)g.mi[0] * idx[1];
    if (D == 3) p += (long long)g.mi[0] * g.mi[1] * idx[2];
#pragma unroll
    for (int a = 0; a < D; ++a) phi_out[a * g.np + p] = phi[a];
  });
}

// ---------------------------------------------------------------------------
// Matrix-free adjoint products (J^T w and the transport Gauss-Newton data
// term), one characteristic at a time, seeded at its end point y_N:
//   MODE 0  transport, J^T w:   seed w_i grad T(y_i)
//   MODE 1  continuity, J^T w:  seed T_j grad I(w)(y_j)
//   MODE 2  transport, h^d J^T W J p:  seed h^d W_i (grad T(y_i) . dy_i) grad T(y_i)
// ZERO: at v = 0 (vp unused), y = x and a unit flow Jacobian.
struct AdjArgs {
  const void* vp;      // packed velocity
  const void* pp;      // packed direction (MODE 2)
  const float* T;      // template (MODE 0, 2), masses (MODE 1)
  const float* w;      // image-grid weights (MODE 0, 1)
  const float* wvox;   // per-voxel weights or null (MODE 2)
};

template <int D>
struct AdjItem {
  Start<D> S;
  float yN[D];    // seed at t = 1
  float y0[D];    // F^T yN, the forward-recovery start at t = 0
  float growth;   // conditioning product of the step Jacobians
};

// Trace and seed the characteristic of image cell idx; false for a zero seed.
template <int D, bool NS, int MODE, bool ZERO>
__device__ __forceinline__ bool adj_prepare(const Geo& g, const Stages& st, const AdjArgs& A, const int idx[3],
                                            AdjItem<D>& it, CellBox<D>* box) {
  using VT = typename VecT<D>::T;
  make_start_idx<D>(g, idx, it.S);
  long long p = idx[0] + (long long)g.mi[0] * idx[1];
  if (D == 3) p += (long long)g.mi[0] * g.mi[1] * idx[2];
  float phi[D], dphi[D], F[D][D];
  it.growth = 1.f;
  Loc<D> L;
  if constexpr (MODE == 2) {
    const float W = A.wvox ? A.wvox[p] : 1.f;
    if (W == 0.f) return false;
    forward_pass<D, NS, true, true>(g, st, (const VT*)A.vp, (const VT*)A.pp, it.S, phi, dphi, F, &it.growth, box);
    locate_i<D>(g, it.S, phi, L);
    float gT[D], val;
    sample_img<D, false, true>(A.T, g, L, val, gT);
    float Jp = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) Jp = fmaf(gT[a], dphi[a], Jp);
    const float s = g.cell_img * W * Jp;
    if (s == 0.f) return false;
#pragma unroll
    for (int a = 0; a < D; ++a) it.yN[a] = s * gT[a];
  } else {
    if constexpr (ZERO) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        phi[a] = 0.f;
#pragma unroll
        for (int b = 0; b < D; ++b) F[a][b] = a == b ? 1.f : 0.f;
      }
    } else {
      forward_pass<D, NS, false, true>(g, st, (const VT*)A.vp, nullptr, it.S, phi, dphi, F, &it.growth, box);
    }
    locate_i<D>(g, it.S, phi, L);
    float gr[D], val;
    if (MODE == 0) {
      sample_img<D, false, true>(A.T, g, L, val, gr);
      const float wi = A.w[p];
#pragma unroll
      for (int a = 0; a < D; ++a) it.yN[a] = wi * gr[a];
    } else {
      sample_img<D, false, true>(A.w, g, L, val, gr);
      const float m = A.T[p];
#pragma unroll
      for (int a = 0; a < D; ++a) it.yN[a] = m * gr[a];
    }
    bool nz = false;
#pragma unroll
    for (int a = 0; a < D; ++a) nz = nz || (it.yN[a] != 0.f);
    if (!nz) return false;
  }
#pragma unroll
  for (int b = 0; b < D; ++b) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) s = fmaf(F[a][b], it.yN[a], s);
    it.y0[b] = s;
  }
  return true;
}

// Magnitude estimate of a characteristic's scatter, without tracing it: the
// seed formed at the start point x (as if v were 0, with dy = p(x) for
// MODE 2), times the time span; the stage adjoints of a step sum to about
// |dt| times the step's adjoint, which runs from y_0 = F^T y_N to y_N.
template <int D, bool NS, int MODE>
__device__ __forceinline__ float adj_guess(const Geo& g, const Stages& st, const AdjArgs& A, const int idx[3]) {
  using VT = typename VecT<D>::T;
  Start<D> S;
  make_start_idx<D>(g, idx, S);
  long long p = idx[0] + (long long)g.mi[0] * idx[1];
  if (D == 3) p += (long long)g.mi[0] * g.mi[1] * idx[2];
  float zero[D];
#pragma unroll
  for (int a = 0; a < D; ++a) zero[a] = 0.f;
  Loc<D> L;
  locate_i<D>(g, S, zero, L);
  float gr[D], val;
  sample_img<D, false, true>(MODE == 1 ? A.w : A.T, g, L, val, gr);
  float n1 = 0.f;
#pragma unroll
  for (int a = 0; a < D; ++a) n1 += fabsf(gr[a]);
  float s;
  if constexpr (MODE == 0) {
    s = fabsf(A.w[p]);
  } else if constexpr (MODE == 1) {
    s = fabsf(A.T[p]);
  } else {
    const float W = A.wvox ? A.wvox[p] : 1.f;
    Loc<D> Lv;
    locate_v<D>(g, S, zero, Lv);
    float pv[D], dummy[D][D];
    sample_vel<D, NS, false>((const VT*)A.pp, g, st, 0, Lv, pv, dummy);
    float Jp = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) Jp = fmaf(gr[a], pv[a], Jp);
    s = fabsf(g.cell_img * W * Jp);
  }
  return fabsf((float)g.nsteps * st.dt) * s * n1;
}

// The reverse sweep of a prepared characteristic into acc; returns kFlag*
// bits.  Forward recovery unless the step Jacobians are ill-conditioned.
template <int D, bool NS, bool ZERO, class Acc>
__device__ __forceinline__ int adj_scatter(const Geo& g, const Stages& st, const void* vpv, AdjItem<D>& it, Acc& acc,
                                           Merge<D, false>& zmg) {
  using VT = typename VecT<D>::T;
  const VT* vp = (const VT*)vpv;
  if constexpr (ZERO) {
    if constexpr (!NS) zero_add<D>(g, st, it.S, it.y0, acc, zmg);
    else zero_adjoint<D, NS>(g, st, it.S, it.y0, acc);
    return 0;
  } else {
    if (!recovery_ok(it.growth)) {
      reverse_recompute<D, NS>(g, st, vp, it.S, it.yN, acc);
      return kFlagRecompute;
    }
    return adjoint_pass<D, NS>(g, st, vp, it.S, it.y0, acc) ? 0 : kFlagSingular;
  }
}

// Block-wide float sum in a fixed order (butterflies within each wave, then
// the wave totals in wave order); every thread calls it and gets the total.
// red holds one float per wave.
__device__ __forceinline__ float block_sum_fixed(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// Exponent e with bound 2^e in [2^(top-1), 2^top), bound > 0.
__device__ __forceinline__ int fix_unit(float bound, int top) {
  int x;
  frexpf(bound, &x);
  return top - x;
}

// Unit of the deferred buffer: n characteristics, each scattering at most
// smax in magnitude, keep every partial sum below 2^61 units.
__device__ __forceinline__ int deferred_unit(int n, float smax) {
  int x;
  frexp((double)n * (double)smax, &x);
  return 61 - x;
}

// Adjoint products through the brick's LDS tile; the brick's tile goes to
// its slot of `part` (k_tile_reduce sums the overlapping tiles per node in a
// fixed order).  The tile is 64-bit fixed point with a per-brick unit 2^-e,
// so the brick's sums do not depend on the order of the additions.  Each
// wave takes a contiguous run of the brick's items, and before anything is
// scattered the magnitude estimates (adj_guess) of the waves' first items,
// scaled by items / first items, set e so that the estimate is about 2^45
// units.  The exact magnitude sum S of the pass then decides: the pass
// stands if every partial sum provably stays below 2^62 units (S < 2^62
// units) and the unit is fine enough (S >= 2^36 units: a unit of at most
// 2^-36 S, far below float rounding of the sums), otherwise the whole block
// redoes the brick at the unit S sets (S about 2^60 units).  32 bits would
// not do: with weights of both signs S can exceed the largest output entry a
// thousandfold, and a unit of S 2^-28 is then visible at 1e-5.  A
// characteristic whose forward cells leave the tile is not scattered here
// but appended to the deferred list (once, on the first pass) for
// k_adjoint_deferred.
struct Deferred {
  int* list;                // deferred characteristics (image cell index); room for every point
  int* hdr;                 // [0] count, [1] largest magnitude sum (float bits), [2] bricks redone (this call)
  unsigned long long* acc;  // fields * nv, 64-bit fixed point, cleared by k_tile_reduce
};

// Stationary 3-D bricks hold 32 or more 64-row items: eight waves share the
// brick's tile (two per SIMD on one LDS tile of up to 104 KB).  2-D bricks
// hold few items, and time-dependent 3-D fields need more registers than two
// waves per SIMD leave: four waves.
template <int D, bool NS>
struct AdjBlock {
  static constexpr int threads = (D == 3 && !NS) ? 512 : 256;
};

template <int D, bool NS, int MODE, bool ZERO>
__global__ void __launch_bounds__((AdjBlock<D, NS>::threads)) k_adjoint(Geo g, Stages st, Bricks B, AdjArgs A, float* __restrict__ out,
                                                    float* __restrict__ part, int* __restrict__ flags, Deferred dq) {
  if (halted(g.halt)) return;
  extern __shared__ unsigned long long ldsq[];
  const long long bid = xcd_block(B.nbricks);
  if (bid < 0) return;
  int O[3], org[3];
  brick_origin<D>(g, B, bid, O, org);
  const int tot = g.nodes * D * B.tvol;
  float* red = reinterpret_cast<float*>(ldsq + tot);
  AdjTile<D, NS> acc;
  acc.tile = ldsq;
  acc.gout = out;
  acc.j0 = st.j0;
  acc.th = st.th;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.org[a] = org[a];
    acc.td[a] = B.tdim[a];
    acc.mv[a] = g.mv[a];
  }
  acc.tvol = B.tvol;
  acc.nv = g.nv;
  acc.e = 0;
  acc.sabs = 0.f;
  acc.spill = false;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) ldsq[i] = 0ull;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int l[3];
  lane_lattice(B, lane, l);
  const int items = brick_items(B);
  const int run = (items + nw - 1) / nw;
  const int w0 = wave * run, w1 = min(items, w0 + run);
  int status = 0;
  Merge<D, false> zmg;  // ZERO with a stationary field: kept across the thread's points
  zmg.reset();
  // trace item w's characteristic; false when it scatters nothing here
  auto prepare = [&](int w, AdjItem<D>& it, bool first) -> bool {
    int idx[3];
    if (!item_cell<D>(g, B, O, w, l, idx)) return false;
    if constexpr (ZERO) {
      return adj_prepare<D, NS, MODE, true>(g, st, A, idx, it, nullptr);
    } else {
      CellBox<D> box;
      box.reset(org, B.tdim);
      if (!adj_prepare<D, NS, MODE, false>(g, st, A, idx, it, &box)) return false;
      if (box.in) return true;
      if (first) {
        long long p = idx[0] + (long long)g.mi[0] * idx[1];
        if (D == 3) p += (long long)g.mi[0] * g.mi[1] * idx[2];
        dq.list[atomicAdd(dq.hdr, 1)] = (int)p;
      }
      return false;
    }
  };
  // pass 0 at the estimated unit; pass 1 (rare) redoes the brick at the exact one
  for (int pass = 0;; ++pass) {
    const bool first = pass == 0;
    if (first) {
      int idx[3];
      const bool cur = w0 < w1 && item_cell<D>(g, B, O, w0, l, idx);
      float est = block_sum_fixed(cur ? adj_guess<D, NS, MODE>(g, st, A, idx) : 0.f, red);  // also orders the tile clear
      est *= (float)items / (float)((items + run - 1) / run);
      acc.e = est > 0.f ? fix_unit(est, 46) : 0;
    }
    for (int w = w0; w < w1; ++w) {
      AdjItem<D> it;
      if (prepare(w, it, first)) status |= adj_scatter<D, NS, ZERO>(g, st, A.vp, it, acc, zmg);
    }
    if constexpr (ZERO && !NS) zmg.flush(acc);
    const float sb = block_sum_fixed(acc.sabs, red);
    const double m = ldexp((double)sb, acc.e);
    if (!first || !(sb > 0.f) || (m < 0x1p62 && m >= 0x1p36)) break;  // the same in every thread
    for (int i = threadIdx.x; i < tot; i += blockDim.x) ldsq[i] = 0ull;
    __syncthreads();
    acc.e = fix_unit(sb, 61);
    acc.sabs = 0.f;
    zmg.reset();
    if (threadIdx.x == 0) atomicAdd(dq.hdr + 2, 1);
  }
  if (acc.spill) status |= kFlagSpill;
  if (status) atomicOr(flags, status);
  __syncthreads();
  float* dst = part + bid * (long long)tot;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) dst[i] = (float)ldexp((double)(long long)ldsq[i], -acc.e);
}

// The deferred characteristics, grid-stride: PASS 0 finds the largest
// magnitude sum of one characteristic's scatter (an order-free maximum),
// PASS 1 scatters them into the 64-bit buffer at the unit that bound fixes.
template <int D, bool NS, int MODE, int PASS>
__global__ void __launch_bounds__(kBlock) k_adjoint_deferred(Geo g, Stages st, AdjArgs A, Deferred dq,
                                                             int* __restrict__ flags) {
  if (halted(g.halt)) return;
  const int n = dq.hdr[0];
  if (n == 0) return;
  const float smax = __int_as_float(dq.hdr[1]);
  if (PASS == 1 && !(smax > 0.f)) return;
  const int e = PASS == 1 ? deferred_unit(n, smax) : 0;
  int status = 0;
  Merge<D, false> zmg;
  zmg.reset();
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long p = dq.list[i];
    int idx[3];
    idx[0] = (int)(p % g.mi[0]);
    idx[1] = (int)((p / g.mi[0]) % g.mi[1]);
    idx[2] = D == 3 ? (int)(p / ((long long)g.mi[0] * g.mi[1])) : 0;
    AdjItem<D> it;
    if (!adj_prepare<D, NS, MODE, false>(g, st, A, idx, it, nullptr)) continue;
    if constexpr (PASS == 0) {
      AdjBound<D, NS> acc{st.j0, st.th, 0.f};
      adj_scatter<D, NS, false>(g, st, A.vp, it, acc, zmg);
      atomicMax(reinterpret_cast<unsigned*>(dq.hdr + 1), __float_as_uint(acc.sabs));
    } else {
      AdjWide<D, NS> acc;
      acc.acc = dq.acc;
      acc.j0 = st.j0;
      acc.th = st.th;
#pragma unroll
      for (int a = 0; a < 3; ++a) acc.mv[a] = g.mv[a];
      acc.nv = g.nv;
      acc.e = e;
      status |= adj_scatter<D, NS, false>(g, st, A.vp, it, acc, zmg);
    }
  }
  if (status) atomicOr(flags, status);
}

// ---------------------------------------------------------------------------
// Assembled Jacobian (transport model, stationary velocity).
//
// Row i of J = d u1 / d v is grad T(y_i)^T d y_i / d v; by the adjoint
// replay above it is a sum over RK4 samples of corner-weight x stage-adjoint
// products, which the register merge already groups into one block of
// 2^d x d values per velocity cell the characteristic crosses.  Storing
// those blocks (cell + values) once per Gauss-Newton iteration turns every
// following matvec into a stream over J: s_i = h^d W_i J_i p, then
// s_i J_i^T scattered through the LDS tile.  Blocks are stored in the
// brick-processing order (slot = brick, wave item, lane) so each wave reads
// its 64 rows with coalesced loads.  A cell is stored as three 10-bit
// offsets from the brick's tile origin.

template <int D>
struct JacLayout {
  static constexpr int NV = (1 << D) * D;      // values per block
  static constexpr int NV4 = (NV + 3) / 4;     // float4 per block
};

template <int D>
struct JacWriter {
  float4* __restrict__ vals;   // [k][NV4][nslots]
  int* __restrict__ cells;     // [k][nslots]
  long long nslots;
  long long slot;
  int kmax;
  int count;
  int org[3];

  template <int NSLOT>
  __device__ __forceinline__ void add_block(const int cell[D], int /*jA*/, const float a[NSLOT][1 << D][D]) {
    if (count < kmax) {
      int packed = 0;
      bool fits = true;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        int t = cell[ax] - org[ax] + 512;
        fits = fits && t >= 0 && t < 1024;
        packed |= (t & 1023) << (10 * ax);
      }
      if (!fits) {
        count = 256;  // out of the packed cell's reach: no capacity (<= 255) can store this row
      } else {
        cells[(long long)count * nslots + slot] = packed;
        const float* f = &a[0][0][0];
#pragma unroll
        for (int j = 0; j < JacLayout<D>::NV4; ++j)
          vals[((long long)count * JacLayout<D>::NV4 + j) * nslots + slot] =
              make_float4(f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3]);
      }
    }
    ++count;
  }
};

// Assemble the stored Jacobian, one wave per 64-row item over all bricks
// (rows are independent here, so the launch is not tied to one block per
// brick).  Slot of a row: brick, item, lane, as the matvec reads them.  With
// u != null also writes the transported image u = T(phi) (eq. rhoEndIR),
// which the forward pass samples anyway.
template <int D, bool STORED>
__global__ void __launch_bounds__(kBlock) k_jac_assemble(Geo g, Stages st, Bricks B,
                                                         const typename VecT<D>::T* __restrict__ vp,
                                                         const float* __restrict__ T, float4* __restrict__ vals,
                                                         int* __restrict__ cells, unsigned char* __restrict__ cnt,
                                                         long long nslots, int kmax, int* __restrict__ maxcount,
                                                         int* __restrict__ flags, float* __restrict__ u) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int items = brick_items(B);
  const long long nitems = (long long)B.nbricks * items;
  // blocks in launch order (dealt round-robin over the XCDs): every XCD gets
  // the same mix of full and short bricks (the top slab of bricks holds
  // fewer image rows)
  const long long blk = blockIdx.x;
  if (blk >= (nitems + nw - 1) / nw) return;
  const long long item = blk * nw + wave;
  if (item >= nitems) return;  // whole wave
  const long long bid = item / items;
  const int w = (int)(item - bid * items);
  int O[3], org[3];
  brick_origin<D>(g, B, bid, O, org);
  int l[3], idx[3];
  lane_lattice(B, lane, l);
  const bool in = item_cell<D>(g, B, O, w, l, idx);
  const long long slot = bid * (long long)B.bdim[0] * B.bdim[1] * B.bdim[2] + (long long)w * 64 + lane;
  int count = 0;
  bool bad = false, fallback = false;
  extern __shared__ float traj_lds[];  // STORED: [step][axis][thread]
  float* traj = traj_lds + threadIdx.x;
  if (in) {
    Start<D> S;
    make_start_idx<D>(g, idx, S);
    float phi[D], dphi[D], F[D][D];
    float growth = 1.f;
    if constexpr (STORED) forward_record<D>(g, st, vp, S, phi, traj, kBlock);
    else forward_pass<D, false, false, true>(g, st, vp, nullptr, S, phi, dphi, F, &growth);
    Loc<D> L;
    locate_i<D>(g, S, phi, L);
    float gT[D], val;
    sample_img<D, true, true>(T, g, L, val, gT);
    if (u) {  // the transported image T(phi(x)) comes for free
      long long pi = idx[0] + (long long)g.mi[0] * idx[1];
      if (D == 3) pi += (long long)g.mi[0] * g.mi[1] * idx[2];
      u[pi] = val;
    }
    bool nz = false;
#pragma unroll
    for (int a = 0; a < D; ++a) nz = nz || (gT[a] != 0.f);
    if (nz) {
      float y0[D];
      if constexpr (STORED) {
#pragma unroll
        for (int b = 0; b < D; ++b) y0[b] = gT[b];  // adjoint at t = 1
      } else {
#pragma unroll
        for (int b = 0; b < D; ++b) {  // adjoint at t = 0 (forward recovery)
          float t = 0.f;
#pragma unroll
          for (int a = 0; a < D; ++a) t = fmaf(F[a][b], gT[a], t);
          y0[b] = t;
        }
      }
      JacWriter<D> jw;
      jw.vals = vals;
      jw.cells = cells;
      jw.nslots = nslots;
      jw.slot = slot;
      jw.kmax = kmax;
      jw.count = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) jw.org[a] = org[a];
      if constexpr (STORED) {
        reverse_sweep<D>(g, st, vp, S, traj, kBlock, y0, jw);
      } else if (!recovery_ok(growth)) {  // (nearly) singular step Jacobians
#pragma unroll
        for (int b = 0; b < D; ++b) y0[b] = gT[b];
        reverse_recompute<D, false>(g, st, vp, S, y0, jw);
        fallback = true;
      } else if (!adjoint_pass<D, false>(g, st, vp, S, y0, jw)) {
        bad = true;
      }
      count = jw.count;
    }
  }
  cnt[slot] = (unsigned char)min(count, kmax);  // never more than stored (an overflow shows in maxcount)
  // one set of atomics per wave
  int wmax = count, wsum = min(count, kmax);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    wmax = max(wmax, __shfl_xor(wmax, off, 64));
    wsum += __shfl_xor(wsum, off, 64);
  }
  const int wflags = (__ballot(fallback) != 0 ? kFlagRecompute : 0) | (__ballot(bad) != 0 ? kFlagSingular : 0);
  if (lane == 0) {
    if (wmax > 0) atomicMax(maxcount, wmax);
    if (wsum > 0) atomicAdd(maxcount + 1, wsum);
    if (wflags) atomicOr(flags, wflags);
  }
}

// Corner values of one stored block: dot with p (gather) or scale.
template <int D>
__device__ __forceinline__ void jac_block_cell(int packed, const int org[3], int cell[D]) {
#pragma unroll
  for (int ax = 0; ax < D; ++ax) cell[ax] = org[ax] + ((packed >> (10 * ax)) & 1023) - 512;
}

template <int D>
__device__ __forceinline__ float jac_block_dot(const Geo& g, const int cell[D], const float* f,
                                               const typename VecT<D>::T* __restrict__ pp) {
  float s = 0.f;
  if constexpr (D == 3) {
    const int x0 = wrapi(cell[0], g.mv[0]), y0 = wrapi(cell[1], g.mv[1]), z0 = wrapi(cell[2], g.mv[2]);
    const unsigned sy = (unsigned)g.pv[0], sz = (unsigned)g.pv[0] * (unsigned)g.pv[1];
    const float4* c0 = pp + packed_corner(g, x0, y0, z0);
    const unsigned off[8] = {0u, 1u, sy, sy + 1u, sz, sz + 1u, sz + sy, sz + sy + 1u};
    float4 q[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) q[o] = c0[off[o]];
    // keep the eight gathers ahead of their first use: left to itself the
    // scheduler sinks each load to its FMAs and waits for it alone, which
    // makes the eight L2 trips of a block serial
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      s = fmaf(f[3 * o], q[o].x, s);
      s = fmaf(f[3 * o + 1], q[o].y, s);
      s = fmaf(f[3 * o + 2], q[o].z, s);
    }
  } else {
    const int x0 = wrapi(cell[0], g.mv[0]), y0 = wrapi(cell[1], g.mv[1]);
    const unsigned sy = (unsigned)g.pv[0];
    const float2* c0 = pp + packed_corner(g, x0, y0, 0);
    const unsigned off[4] = {0u, 1u, sy, sy + 1u};
    float2 q[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) q[o] = c0[off[o]];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      s = fmaf(f[2 * o], q[o].x, s);
      s = fmaf(f[2 * o + 1], q[o].y, s);
    }
  }
  return s;
}

// jac_block_dot in two halves, so that other loads can be issued between
// the gathers of p and their use.
template <int D> struct PGather;
template <> struct PGather<3> { float4 q[8]; };
template <> struct PGather<2> { float2 q[4]; };

template <int D>
__device__ __forceinline__ void jac_block_gather(const Geo& g, const int cell[D],
                                                 const typename VecT<D>::T* __restrict__ pp, PGather<D>& G) {
  if constexpr (D == 3) {
    const int x0 = wrapi(cell[0], g.mv[0]), y0 = wrapi(cell[1], g.mv[1]), z0 = wrapi(cell[2], g.mv[2]);
    const unsigned sy = (unsigned)g.pv[0], sz = (unsigned)g.pv[0] * (unsigned)g.pv[1];
    const float4* c0 = pp + packed_corner(g, x0, y0, z0);
    const unsigned off[8] = {0u, 1u, sy, sy + 1u, sz, sz + 1u, sz + sy, sz + sy + 1u};
#pragma unroll
    for (int o = 0; o < 8; ++o) G.q[o] = c0[off[o]];
  } else {
    const int x0 = wrapi(cell[0], g.mv[0]), y0 = wrapi(cell[1], g.mv[1]);
    const unsigned sy = (unsigned)g.pv[0];
    const float2* c0 = pp + packed_corner(g, x0, y0, 0);
    const unsigned off[4] = {0u, 1u, sy, sy + 1u};
#pragma unroll
    for (int o = 0; o < 4; ++o) G.q[o] = c0[off[o]];
  }
}

template <int D>
__device__ __forceinline__ float jac_block_finish(const float* f, const PGather<D>& G) {
  float s = 0.f;
  if constexpr (D == 3) {
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      s = fmaf(f[3 * o], G.q[o].x, s);
      s = fmaf(f[3 * o + 1], G.q[o].y, s);
      s = fmaf(f[3 * o + 2], G.q[o].z, s);
    }
  } else {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      s = fmaf(f[2 * o], G.q[o].x, s);
      s = fmaf(f[2 * o + 1], G.q[o].y, s);
    }
  }
  return s;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int D>
__device__ __forceinline__ void jac_load(const float4* __restrict__ vals, const int* __restrict__ cells,
                                         long long nslots, long long slot, int k, const int org[3], int cell[D],
                                         float f[4 * JacLayout<D>::NV4]) {
  constexpr int NV4 = JacLayout<D>::NV4;
  jac_block_cell<D>(cells[(long long)k * nslots + slot], org, cell);
#pragma unroll
  for (int j = 0; j < NV4; ++j) {
    float4 q = vals[((long long)k * NV4 + j) * nslots + slot];
    f[4 * j] = q.x; f[4 * j + 1] = q.y; f[4 * j + 2] = q.z; f[4 * j + 3] = q.w;
  }
}

template <int D>
__device__ __forceinline__ void jac_scatter(const Geo& g, const Bricks& B, const int org[3], int* tile,
                                            float* __restrict__ out, const int cell[D],
                                            const float f[4 * JacLayout<D>::NV4], float s, int e) {
  bool tin = true;
  int t[3] = {0, 0, 0};
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    t[ax] = cell[ax] - org[ax];
    tin = tin && (t[ax] >= 0) && (t[ax] + 1 < B.tdim[ax]);
  }
  if (tin) {
    const int tb0 = (t[2] * B.tdim[1] + t[1]) * B.tdim[0] + t[0];
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      int off = tb0 + (o & 1) + ((o >> 1) & 1) * B.tdim[0];
      if (D == 3) off += ((o >> 2) & 1) * B.tdim[0] * B.tdim[1];
#pragma unroll
      for (int c = 0; c < D; ++c) atomicAdd(&tile[c * B.tvol + off], __float2int_rn(ldexpf(s * f[o * D + c], e)));
    }
  } else {
    // outside the tile: direct float atomics into the output
    Loc<D> L;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) L.c[ax] = cell[ax];
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      long long gi = corner_index<D>(L, g.mv, o);
#pragma unroll
      for (int c = 0; c < D; ++c) unsafeAtomicAdd(&out[(long long)c * g.nv + gi], s * f[o * D + c]);
    }
  }
}

// Apply the stored Jacobian: with wseed == null, s_i = scale W_i J_i p
// (Gauss-Newton data term); otherwise s_i = scale wseed_i (transpose
// product J^T w).  Then scatter s_i J_i^T into the brick's tile.
//
// The tile accumulates in 32-bit fixed point: integer LDS atomics are several
// times faster than float ones, and an integer sum does not depend on the
// order of the additions, so the result is reproducible bit for bit.  A
// stored block adds at most one entry to each (node, component), so no
// partial sum of the tile exceeds sum_i |s_i| R_i, R_i = sum_k max |J_ik|
// (max over the entries of block k of row i).  The brick is processed in
// rounds of one 64-row item per wave: each round forms its s_i (keeping the
// first two blocks of a row in registers, so the blocks are read once), adds
// its rows' share to that bound, and, when the bound needs a smaller power of
// two to stay below 2^30, first rescales the tile by a rounding right shift;
// then it scatters.  Every wave passes every round's barrier.
template <int D>
__global__ void __launch_bounds__(kBlock) k_jac_apply(Geo g, Bricks B, const float4* __restrict__ vals,
                                                      const int* __restrict__ cells,
                                                      const unsigned char* __restrict__ cnt, long long nslots,
                                                      const typename VecT<D>::T* __restrict__ pp,
                                                      const float* __restrict__ wvox, const float* __restrict__ wseed,
                                                      float scale, float* __restrict__ out, float* __restrict__ part) {
  if (halted(g.halt)) return;
  extern __shared__ float lds[];
  long long bid = xcd_block(B.nbricks);
  if (bid < 0) return;
  int O[3], org[3];
  brick_origin<D>(g, B, bid, O, org);
  const int tot = D * B.tvol;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int* tile = (int*)lds;             // [D][tvol] fixed-point sums
  float* red = lds + tot;            // [2][waves] per-round bounds
  for (int i = threadIdx.x; i < tot; i += blockDim.x) tile[i] = 0;
  const long long base = bid * (long long)B.bdim[0] * B.bdim[1] * B.bdim[2];
  constexpr int NV4 = JacLayout<D>::NV4;
  int l[3];
  lane_lattice(B, lane, l);
  const int nitems = brick_items(B);
  const int rounds = (nitems + nw - 1) / nw;
  float btot = 0.f;                  // bound of all rows so far (same in every thread)
  int e = 0;                         // current scale 2^e (valid once btot > 0)
  bool finite = true;
  const bool need_p = wvox || wseed;
  unsigned long long pk = 0;
  for (int r = 0; r < rounds; ++r) {
    const int w = wave + r * nw;
    if ((r & 7) == 0) {  // counts of rounds r .. r + 7 in one trip (0 outside the image)
      pk = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int wj = wave + (r + j) * nw;
        if (r + j < rounds && wj < nitems) pk |= (unsigned long long)cnt[base + (long long)wj * 64 + lane] << (8 * j);
      }
    }
    int n = (int)((pk >> (8 * (r & 7))) & 0xff);
    long long slot = 0, p = 0;
    if (w < nitems) {
      slot = base + w * 64 + lane;
      if (need_p && n > 0) {
        int idx[3];
        (void)item_cell<D>(g, B, O, w, l, idx);
        p = idx[0] + (long long)g.mi[0] * idx[1];
        if (D == 3) p += (long long)g.mi[0] * g.mi[1] * idx[2];
      }
    }
    float f0[4 * NV4], f1[4 * NV4];
    int c0[D], c1[D];
    float s = 0.f, rb = 0.f;
    if (n > 0) {
      jac_load<D>(vals, cells, nslots, slot, 0, org, c0, f0);
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < 4 * NV4; ++j) m = fmaxf(m, fabsf(f0[j]));
      rb = m;
      if (!wseed) s = jac_block_dot<D>(g, c0, f0, pp);
    }
    if (n > 1) {
      jac_load<D>(vals, cells, nslots, slot, 1, org, c1, f1);
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < 4 * NV4; ++j) m = fmaxf(m, fabsf(f1[j]));
      rb += m;
      if (!wseed) s += jac_block_dot<D>(g, c1, f1, pp);
    }
    for (int k = 2; k < n; ++k) {
      int cell[D];
      float f[4 * NV4];
      jac_load<D>(vals, cells, nslots, slot, k, org, cell, f);
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < 4 * NV4; ++j) m = fmaxf(m, fabsf(f[j]));
      rb += m;
      if (!wseed) s += jac_block_dot<D>(g, cell, f, pp);
    }
    if (n > 0) s = wseed ? scale * wseed[p] : s * scale * (wvox ? wvox[p] : 1.f);
    // this round's share of the bound, summed in a fixed order
    const float bw = wave_sum(fabsf(s) * rb);
    float* rr = red + (r & 1) * nw;  // a wave runs at most one round ahead
    if (lane == 0) rr[wave] = bw;
    __syncthreads();
    float bs = 0.f;
    for (int q = 0; q < nw; ++q) bs += rr[q];
    const float prev = btot;
    btot += bs;
    finite = finite && btot <= 3.0e38f;  // false for inf and NaN
    if (!finite || btot == 0.f) continue;
    int ex = 0;
    (void)frexpf(btot, &ex);
    const int enew = 30 - ex;        // btot * 2^enew < 2^30
    if (prev == 0.f) {
      e = enew;                      // tile still zero
    } else if (enew < e) {
      const int d = e - enew;        // rescale the sums of earlier rounds
      for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int x = tile[i];
        tile[i] = d >= 31 ? 0 : (int)(((long long)x + (1LL << (d - 1))) >> d);
      }
      e = enew;
      __syncthreads();
    }
    if (s != 0.f) {
      jac_scatter<D>(g, B, org, tile, out, c0, f0, s, e);
      if (n > 1) jac_scatter<D>(g, B, org, tile, out, c1, f1, s, e);
      for (int k = 2; k < n; ++k) {
        int cell[D];
        float f[4 * NV4];
        jac_load<D>(vals, cells, nslots, slot, k, org, cell, f);
        jac_scatter<D>(g, B, org, tile, out, cell, f, s, e);
      }
    }
  }
  __syncthreads();
  float* dst = part + bid * (long long)tot;
  const float nan = __int_as_float(0x7fc00000);
  for (int i = threadIdx.x; i < tot; i += blockDim.x) dst[i] = finite ? ldexpf((float)tile[i], -e) : nan;
}

// ---------------------------------------------------------------------------
// Paged layout of the assembled Jacobian.
//
// The assembly writes block k of a row at [k][...][slot]; rows carry 1, 2, 3
// or more blocks, so a product that walks that layout level by level leaves
// lanes idle at the higher levels and makes one dependent memory trip per
// level.  After the assembly, k_jac_pack lays each brick's blocks out
// densely, rows in slot order, in pages of 64 positions (one per lane): a
// row never straddles a page (a row that does not fit the rest of a page
// starts the next one), the first block of a row carries kJacHead in its
// cell word, and unused positions hold the cell word -1, so a page's valid
// positions are a prefix of it.  Layout: values [page][float4 j][64], cells
// [page][64], and at a row's first position the row's slot within its brick
// (for voxel weights and seeds).  Brick b owns pages [b * cap, (b + 1) * cap).
constexpr int kJacHead = int(0x80000000u);
constexpr int kPagePos = 64;

// Pages a brick needs at most: every full page holds at least 65 - kmax
// blocks (a row of at most kmax blocks that does not fit leaves fewer than
// kmax positions unused), plus a partial last page.
inline int jac_page_cap(long long brick_rows, int kmax) {
  return (int)((brick_rows * kmax + (kPagePos + 1 - kmax) - 1) / (kPagePos + 1 - kmax)) + 1;
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active) on
// DPP: shifts by 1, 2, 4 and 8 within each row of 16 lanes (zero from
// outside the row), then each row's total broadcast into the rows above.
__device__ __forceinline__ int wave_incl_scan(int x) {
  int v = x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);    // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);    // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);    // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);    // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2 and 3
  return v;
}

// A brick's block counts into LDS, zero past its rows (16-byte loads when
// the brick's counts are 16-byte aligned; a byte loop would wait on one HBM
// trip per iteration).
__device__ __forceinline__ void load_counts(const unsigned char* __restrict__ cnt, long long base, int rows,
                                            unsigned char* cl) {
  const int rows64 = (rows + 63) & ~63;
  int done = 0;
  if (((base | (long long)(size_t)cnt) & 15) == 0) {
    const uint4* src = reinterpret_cast<const uint4*>(cnt + base);
    uint4* dst = reinterpret_cast<uint4*>(cl);
    const int full = rows >> 4;      // 16-byte groups inside the brick
#pragma unroll 4
    for (int i = threadIdx.x; i < full; i += blockDim.x) dst[i] = src[i];
    done = 16 * full;
  }
  for (int i = done + threadIdx.x; i < rows64; i += blockDim.x) cl[i] = i < rows ? cnt[base + i] : 0;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_jac_pack(Bricks B, const float4* __restrict__ vals,
                                                     const int* __restrict__ cells,
                                                     const unsigned char* __restrict__ cnt, long long nslots,
                                                     int cap, float4* __restrict__ pv, int* __restrict__ pc,
                                                     int* __restrict__ prow, int* __restrict__ npages,
                                                     int* __restrict__ axbox) {
  constexpr int NV4 = JacLayout<D>::NV4;
  // LDS: the rows that hold blocks (slot within the brick) and their first
  // positions (increasing), then the counts of all rows
  extern __shared__ int sh[];
  __shared__ int s_rows, s_pos;
  __shared__ int s_box[6];           // per axis: lowest and highest tile node touched
  // bricks dealt round-robin over the XCDs (brick b on XCD b mod 8): the
  // copy streams every byte once, so no XCD needs a compact brick set, and
  // interleaving evens out their page totals (contiguous ranges left the
  // fullest XCD about 8 % above the mean at 128^3)
  const long long bid = blockIdx.x;
  if (bid >= B.nbricks) return;
  if (threadIdx.x < 6) s_box[threadIdx.x] = threadIdx.x < 3 ? 0x7fff : -1;
  const int rows = B.bdim[0] * B.bdim[1] * B.bdim[2];
  const long long base = bid * (long long)rows;
  const int r4 = (rows + 3) & ~3;
  int* rl = sh;                      // [rows]
  int* rs = sh + r4;                 // [rows]
  unsigned char* cl = (unsigned char*)(sh + 2 * r4);   // [rows rounded up to 64], 16-byte aligned
  const int rows64 = (rows + 63) & ~63;
  load_counts(cnt, base, rows, cl);
  __syncthreads();
  if (threadIdx.x < 64) {
    // Greedy placement in slot order by wave 0, 64 rows at a time: a prefix
    // sum places the rows as if none straddled a page; the rows before the
    // first one that would straddle stand, that row starts the next page,
    // and the scan resumes after it (about one straddling row per page).
    const int lane = threadIdx.x;
    int at = 0, nr = 0;
    for (int i0 = 0; i0 < rows; i0 += 64) {
      const int n = cl[i0 + lane];
      int start = 0;
      while (start < 64) {
        const int x = lane >= start ? n : 0;
        const int incl = wave_incl_scan(x);
        const int p = at + incl - x;
        const bool straddle = lane >= start && n > 0 && (p & (kPagePos - 1)) + n > kPagePos;
        const unsigned long long sm = __ballot(straddle);
        const int first = sm ? __ffsll((long long)sm) - 1 : 64;
        // rows start .. first - 1 are placed; compact the ones with blocks
        const bool keep = lane >= start && lane < first && n > 0;
        const unsigned long long km = __ballot(keep);
        const int rank = __popcll(km & ((1ull << lane) - 1));
        if (keep) {
          rl[nr + rank] = i0 + lane;
          rs[nr + rank] = p;
        }
        nr += __popcll(km);
        if (first == 64) {
          at += __builtin_amdgcn_readlane(incl, 63);
          break;
        }
        // the straddling row opens the next page
        const int pf = __builtin_amdgcn_readlane(p, first), nf = __builtin_amdgcn_readlane(n, first);
        const int page_at = (pf + kPagePos - 1) & ~(kPagePos - 1);
        if (lane == 0) {
          rl[nr] = i0 + first;
          rs[nr] = page_at;
        }
        nr += 1;
        at = page_at + nf;
        start = first + 1;
      }
    }
    if (lane == 0) {
      s_rows = nr;
      s_pos = at;
      npages[bid] = (at + kPagePos - 1) / kPagePos;
    }
  }
  __syncthreads();
  const int nr = s_rows;
  const int used = ((s_pos + kPagePos - 1) / kPagePos) * kPagePos;
  const long long q0 = bid * (long long)cap * kPagePos;   // first position of the brick
  // tile nodes touched by the blocks that scatter into the tile (their cell
  // and the next node along each axis)
  int blo[3] = {0x7fff, 0x7fff, 0x7fff}, bhi[3] = {-1, -1, -1};
  // one thread per destination position: coalesced writes; the source row
  // is the last row whose first position is at or before it
  for (int q = threadIdx.x; q < used; q += blockDim.x) {
    int lo = 0, hi = nr - 1;         // rs[lo] <= q (rs[0] = 0)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rs[mid] <= q) lo = mid;
      else hi = mid - 1;
    }
    const int row = nr > 0 ? rl[lo] : 0;
    const int k = q - (nr > 0 ? rs[lo] : 0);
    const bool valid = nr > 0 && k < (int)cl[row];
    const long long qq = q0 + q;     // = page * 64 + lane
    const long long pg = qq >> 6;
    const int j = (int)(qq & 63);
    if (valid) {
      const long long slot = base + row;
      int cw = cells[(long long)k * nslots + slot];
      {
        int t[3] = {0, 0, 0};
        bool tin = true;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          t[ax] = ((cw >> (10 * ax)) & 1023) - 512;
          tin = tin && t[ax] >= 0 && t[ax] + 1 < B.tdim[ax];
        }
        if (tin) {
#pragma unroll
          for (int ax = 0; ax < D; ++ax) {
            blo[ax] = min(blo[ax], t[ax]);
            bhi[ax] = max(bhi[ax], t[ax] + 1);
          }
        }
      }
      if (k == 0) cw |= kJacHead;
      pc[qq] = cw;
      prow[qq] = k == 0 ? row : -1;
#pragma unroll
      for (int v = 0; v < NV4; ++v) pv[(pg * NV4 + v) * 64 + j] = vals[((long long)k * NV4 + v) * nslots + slot];
    } else {
      pc[qq] = -1;
      prow[qq] = -1;
    }
  }
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      blo[ax] = min(blo[ax], __shfl_xor(blo[ax], off, 64));
      bhi[ax] = max(bhi[ax], __shfl_xor(bhi[ax], off, 64));
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      atomicMin(&s_box[ax], blo[ax]);
      atomicMax(&s_box[3 + ax], bhi[ax]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_box[0] <= s_box[3]) {
    // into the box of every brick index of this brick along each axis
    const int bi[3] = {(int)(bid % B.nb[0]), (int)((bid / B.nb[0]) % B.nb[1]), (int)(bid / ((long long)B.nb[0] * B.nb[1]))};
    const int off[3] = {0, B.nb[0], B.nb[0] + B.nb[1]}, nbs = B.nb[0] + B.nb[1] + B.nb[2];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      atomicMin(&axbox[off[ax] + bi[ax]], s_box[ax]);
      atomicMax(&axbox[nbs + off[ax] + bi[ax]], s_box[3 + ax]);
    }
  }
}

// Empty axis boxes (lo above hi) before the pack fills them.
__global__ void k_axbox_init(int* __restrict__ axbox, int nbs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * nbs) axbox[i] = i < nbs ? 0x7fff : -1;
}

// The cover lists of the paged product: per axis a and velocity index X,
// the (brick index, tile node) entries of the full lists whose node lies in
// that brick index's axis box, in the same order.  One block per axis
// (axes beyond the dimension keep their lists); a block-wide scan in chunks
// of blockDim places them.
__global__ void __launch_bounds__(1024) k_cover_filter(int D, int3 mv, int3 nb, const int* __restrict__ axbox,
                                                      const int* __restrict__ cs0, const int2* __restrict__ ce0,
                                                      const int* __restrict__ cs1, const int2* __restrict__ ce1,
                                                      const int* __restrict__ cs2, const int2* __restrict__ ce2,
                                                      int* __restrict__ os0, int2* __restrict__ oe0,
                                                      int* __restrict__ os1, int2* __restrict__ oe1,
                                                      int* __restrict__ os2, int2* __restrict__ oe2) {
  __shared__ int sh[1024];
  __shared__ int carry;
  const int a = blockIdx.x;
  const int m = a == 0 ? mv.x : (a == 1 ? mv.y : mv.z);
  const int* cs = a == 0 ? cs0 : (a == 1 ? cs1 : cs2);
  const int2* ce = a == 0 ? ce0 : (a == 1 ? ce1 : ce2);
  int* os = a == 0 ? os0 : (a == 1 ? os1 : os2);
  int2* oe = a == 0 ? oe0 : (a == 1 ? oe1 : oe2);
  const int off = a == 0 ? 0 : (a == 1 ? nb.x : nb.x + nb.y), nbs = nb.x + nb.y + nb.z;
  auto keep = [&](int2 e) {
    return a >= D || (e.y >= axbox[off + e.x] && e.y <= axbox[nbs + off + e.x]);
  };
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int X0 = 0; X0 < m; X0 += blockDim.x) {
    const int X = X0 + threadIdx.x;
    int n = 0;
    if (X < m)
      for (int e = cs[X]; e < cs[X + 1]; ++e) n += keep(ce[e]);
    sh[threadIdx.x] = n;
    __syncthreads();
    for (int d = 1; d < (int)blockDim.x; d <<= 1) {   // inclusive scan
      const int t = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    const int base = carry + sh[threadIdx.x] - n;
    if (X < m) {
      os[X] = base;
      int k = base;
      for (int e = cs[X]; e < cs[X + 1]; ++e)
        if (keep(ce[e])) oe[k++] = ce[e];
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry = base + n;
    __syncthreads();
  }
  if (threadIdx.x == 0) os[m] = carry;
}

// Launch order of the bricks for the paged product.  Each XCD takes a
// contiguous range of bricks (a compact set, so its L2 holds its part of p
// and of the tiles), the ranges cut where the running sum of page counts
// crosses each eighth of the total (even ranges of bricks left the fullest
// XCD about 8 % above the mean at 128^3), each at most `cap` bricks long;
// within a range the bricks go in decreasing order of their page counts
// (ties by brick index), so the heaviest start in the first generation of
// resident blocks and the lightest fill the slots that free up.
// order[x * cap + j] is the j-th brick of XCD x, -1 past its range.  With
// balance == 0 (more bricks than the LDS prefix holds) the ranges are even.
// One block; every brick's thread counts the bricks of its range that go
// first.
__global__ void __launch_bounds__(1024) k_brick_order(const int* __restrict__ npages, int nbricks, int cap,
                                                      int balance, int* __restrict__ order) {
  extern __shared__ int pre[];       // [nbricks + 1] page counts before each brick
  __shared__ int sc[1024];
  __shared__ int s_lo[kXcds + 1];
  __shared__ int carry;
  if (balance) {
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nbricks; c0 += blockDim.x) {   // inclusive scan in chunks of blockDim
      const int b = c0 + threadIdx.x;
      sc[threadIdx.x] = b < nbricks ? npages[b] : 0;
      __syncthreads();
      for (int d = 1; d < (int)blockDim.x; d <<= 1) {
        const int t = (int)threadIdx.x >= d ? sc[threadIdx.x - d] : 0;
        __syncthreads();
        sc[threadIdx.x] += t;
        __syncthreads();
      }
      if (b < nbricks) pre[b + 1] = carry + sc[threadIdx.x];
      __syncthreads();
      if (threadIdx.x == blockDim.x - 1) carry += sc[threadIdx.x];
      __syncthreads();
    }
    if (threadIdx.x == 0) pre[0] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int even = (nbricks + kXcds - 1) / kXcds;
    s_lo[0] = 0;
    for (int x = 0; x < kXcds - 1; ++x) {
      int bnd;
      if (balance) {                 // first brick with at least (x + 1) / 8 of the pages before it
        const long long target = (long long)pre[nbricks] * (x + 1) / kXcds;
        int lo = 0, hi = nbricks;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (pre[mid] >= target) hi = mid;
          else lo = mid + 1;
        }
        bnd = lo;
      } else {
        bnd = min(nbricks, (x + 1) * even);
      }
      // every range within cap bricks, and room for the rest
      bnd = max(bnd, max(s_lo[x], nbricks - (kXcds - 1 - x) * cap));
      bnd = min(bnd, min(s_lo[x] + cap, nbricks));
      s_lo[x + 1] = bnd;
    }
    s_lo[kXcds] = nbricks;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbricks; b += blockDim.x) {
    int x = 0;
    while (x < kXcds - 1 && b >= s_lo[x + 1]) ++x;
    const int lo = s_lo[x], hi = s_lo[x + 1];
    const int key = npages[b];
    int rank = 0;                    // bricks of the range that go first
    for (int c = lo; c < hi; ++c) {
      const int kc = npages[c];
      rank += kc > key || (kc == key && c < b);
    }
    order[x * cap + rank] = b;
  }
  for (int q = threadIdx.x; q < kXcds * cap; q += blockDim.x) {
    const int x = q / cap, j = q - x * cap;
    if (j >= s_lo[x + 1] - s_lo[x]) order[q] = -1;
  }
}

// The same pointer with its origin hidden from the compiler: loads through
// it may alias any memory, so an empty asm with a memory clobber orders
// them (loads through __restrict__ read-only arguments may be moved across
// such an asm).
template <class T>
__device__ __forceinline__ T* opaque(T* p) {
  using G = __attribute__((address_space(1))) T*;   // global memory (kernel arguments point there)
  G q = (G)p;
  asm volatile("" : "+s"(q));
  return (T*)q;
}

constexpr int kPgBlock = 512;   // 8 waves share a brick's tile (two blocks per CU)

// Fixed-point scale of a brick's tile.  A stored block adds at most one
// entry to each (node, component) of the tile, so no partial sum of the tile
// exceeds Bt = sum_i |s_i| R_i (R_i = sum over the row's blocks of max
// |J_ik|); a scale 2^e with Bt 2^e < 2^30 therefore never overflows 32-bit
// integers, and integer sums do not depend on the order of the additions.
// Bt is only known once every s_i is.  Each wave takes a contiguous run of
// the brick's pages; after the first page of every wave (spread over the
// brick) one barrier sums their exact share of Bt, which, scaled to the
// brick's page count with 4x headroom, sets e; the waves then stream their
// pages without synchronising, scattering round(s_i J_ik 2^e) and adding up
// their exact shares of Bt.  At the end the exact Bt decides: if 2^e Bt
// could have overflowed, or e lies more than three bits below the exact
// scale, the brick is redone at the exact scale (a second pass over its
// pages).  Every choice depends on the data only, so the result is the same
// in every run.  With wseed == null, s_i = scale W_i J_i p (a row's blocks
// are summed in position order, identically in every lane of the row);
// otherwise s_i = scale wseed_i.
template <int D, bool WS, bool WV>
__global__ void __launch_bounds__(kPgBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_jac_apply_pg(Geo g, Bricks B, const float4* __restrict__ pv, const int* __restrict__ pc,
               const int* __restrict__ prow, const int* __restrict__ npages, const int* __restrict__ order,
               int cap, const typename VecT<D>::T* __restrict__ pp,
               const float* __restrict__ wvox, const float* __restrict__ wseed, float scale,
               float* __restrict__ out, float* __restrict__ part, int* __restrict__ redo,
               const int* __restrict__ axbox) {
  if (halted(g.halt)) return;
  extern __shared__ float lds[];
  const long long lb = xcd_block((long long)kXcds * pg_xcd_slots(B.nbricks));   // XCD x's slots x * cap + j
  if (lb < 0) return;
  const long long bid = order[lb];   // heaviest bricks of each XCD first
  if (bid < 0) return;               // past this XCD's range
  int O[3], org[3];
  brick_origin<D>(g, B, bid, O, org);
  const int tot = D * B.tvol;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int* tile = (int*)lds;             // [D][tvol] fixed-point sums
  float* red = lds + tot;            // [2 * waves] bound shares
  float* stage = red + 2 * nw + 64 * wave;   // this wave's 64 staging slots
  auto zero_tile = [&]() {           // 16-byte LDS writes (the tile starts the LDS block)
    int4* t4 = (int4*)tile;
    for (int i = threadIdx.x; i < tot / 4; i += blockDim.x) t4[i] = make_int4(0, 0, 0, 0);
    for (int i = 4 * (tot / 4) + threadIdx.x; i < tot; i += blockDim.x) tile[i] = 0;
  };
  zero_tile();
  constexpr int NV4 = JacLayout<D>::NV4;
  constexpr bool ROW = WS || WV;     // the row's image index is needed
  auto row_image = [&](int row) {
    int l[3], idx[3];
    lane_lattice(B, row & 63, l);
    (void)item_cell<D>(g, B, O, row >> 6, l, idx);
    long long pi = idx[0] + (long long)g.mi[0] * idx[1];
    if (D == 3) pi += (long long)g.mi[0] * g.mi[1] * idx[2];
    return pi;
  };
  // the lanes' terms summed in a fixed order: by eight lanes in groups of
  // eight, then by lane 0 (through the wave's staging slots)
  auto wave_total = [&](float x) {
    __builtin_amdgcn_wave_barrier();
    stage[lane] = x;
    __builtin_amdgcn_wave_barrier();
    float q = 0.f;
    if (lane < 8) {
      float y[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) y[k] = stage[8 * lane + k];
#pragma unroll
      for (int k = 0; k < 8; ++k) q += y[k];
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 8) stage[lane] = q;
    __builtin_amdgcn_wave_barrier();
    float tsum = 0.f;
    if (lane == 0) {
      float y[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) y[k] = stage[k];
#pragma unroll
      for (int k = 0; k < 8; ++k) tsum += y[k];
    }
    __builtin_amdgcn_wave_barrier();
    return tsum;                     // valid in lane 0
  };
  const int np = npages[bid];
  const int per = (np + nw - 1) / nw;            // pages of each wave
  const int p0 = min(np, wave * per), p1 = min(np, p0 + per);
  const long long pg0 = bid * (long long)cap;
  pv = opaque(pv);
  pc = opaque(pc);
  prow = opaque(prow);
  pp = opaque(pp);
  // Pages are double-buffered: while a page is gathered, summed and
  // scattered, the next one is in flight.  Loads complete in issue order,
  // so within a page everything it consumes (the row's weight or seed, the
  // gathers of p) is issued before the next page's loads, and all of them are
  // issued without branches (a page index past the wave's last page reads
  // that last page and is marked empty).
  auto load_page = [&](int page, float* ff, int& ww, int& rr) {
    const long long pg = pg0 + min(page, max(p1 - 1, 0));
    const int w0 = pc[pg * 64 + lane];
    if (ROW) rr = prow[pg * 64 + lane];
#pragma unroll
    for (int j = 0; j < NV4; ++j) {
      const float4 a = pv[(pg * NV4 + j) * 64 + lane];
      ff[4 * j] = a.x; ff[4 * j + 1] = a.y; ff[4 * j + 2] = a.z; ff[4 * j + 3] = a.w;
    }
    ww = page < p1 ? w0 : -1;
  };
  // s of this lane's position (and the cell of its block); the next page's
  // loads go out in between
  auto page_s = [&](int page, const float* f, int w, int rw, float* fn, int& wn, int& rwn, int* cl) {
    const bool v = w != -1;
    jac_block_cell<D>(w & ~kJacHead, org, cl);   // in range for any word (wrapped on use)
    // segment [a, z) of this lane's position: rows are contiguous, heads mark
    // their first positions, valid positions are a prefix of the page
    const unsigned long long hm = __ballot(v && (w & kJacHead));
    const int nvalid = __popcll(__ballot(v));
    int a = 0, z = 0;
    if (v) {
      const unsigned long long below = hm & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
      a = 63 - __clzll((long long)below);
      const unsigned long long above = lane == 63 ? 0ull : (hm & ~((2ull << lane) - 1));
      z = above ? __ffsll((long long)above) - 1 : nvalid;
    }
    float sv = 0.f;
    if constexpr (ROW) {
      const int row = __shfl(rw, a, 64);   // the row's slot, from its first position
      sv = WS ? wseed[v ? row_image(row) : 0] : wvox[v ? row_image(row) : 0];
    }
    PGather<D> G;
    if constexpr (!WS) jac_block_gather<D>(g, cl, pp, G);
    // gathers (and the weight) first, then the next page, then the use; an
    // empty asm with a memory clobber keeps the compiler's passes from
    // moving loads across these points, the scheduling barrier keeps the
    // machine scheduler from doing so
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    load_page(page + 1, fn, wn, rwn);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    float t = 0.f;
    if constexpr (!WS) {
      // row sums through the wave's LDS staging slots (a wave's LDS accesses
      // complete in order): every lane reads its row's products and adds
      // them in position order, eight reads in flight at a time
      stage[lane] = jac_block_finish<D>(f, G);
      __builtin_amdgcn_wave_barrier();
      for (int k0 = a; k0 < z; k0 += 8) {
        float x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = k0 + k < z ? stage[k0 + k] : 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k0 + k < z) t += x[k];
      }
      __builtin_amdgcn_wave_barrier();
    }
    return v ? (WS ? scale * sv : t * scale * (WV ? sv : 1.f)) : 0.f;
  };
  auto block_max = [&](const float* f) {
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < 4 * NV4; ++j) m = fmaxf(m, fabsf(f[j]));
    return m;
  };
  // one pass over the wave's pages at scale e; the first page's products
  // arrive already formed (s0, cl0, f0) when `first` is set
  float fa[4 * NV4], fb[4 * NV4];
  int wa = -1, wb = -1, ra = -1, rb = -1;
  float bshare = 0.f;                // this lane's exact share of Bt
  auto stream = [&](int from, int e, bool fin) {
    for (int page = from; page < p1; page += 2) {
      int cl[D];
      float s = page_s(page, fa, wa, ra, fb, wb, rb, cl);
      bshare += fabsf(s) * (wa != -1 ? block_max(fa) : 0.f);
      if (fin && s != 0.f) jac_scatter<D>(g, B, org, tile, out, cl, fa, s, e);
      if (page + 1 < p1) {
        s = page_s(page + 1, fb, wb, rb, fa, wa, ra, cl);
        bshare += fabsf(s) * (wb != -1 ? block_max(fb) : 0.f);
        if (fin && s != 0.f) jac_scatter<D>(g, B, org, tile, out, cl, fb, s, e);
      }
    }
  };
  // ---- first page of every wave: the estimate of Bt
  int cl0[D];
  float s0 = 0.f;
  if (p0 < p1) {
    load_page(p0, fb, wb, rb);
    s0 = page_s(p0, fb, wb, rb, fa, wa, ra, cl0);
    bshare = fabsf(s0) * (wb != -1 ? block_max(fb) : 0.f);
  }
  {
    const float bw = wave_total(bshare);
    if (lane == 0) red[wave] = bw;
  }
  __syncthreads();
  float b1 = 0.f;
  int n1 = 0;
  for (int q = 0; q < nw; ++q) {
    b1 += red[q];
    n1 += min(np, q * per) < min(np, q * per + per);
  }
  const float est = n1 > 0 ? 4.f * b1 * ((float)np / (float)n1) : 0.f;
  int e = 0;
  bool ok = est <= 3.0e38f;          // false for inf and NaN
  if (ok && est > 0.f) {
    int ex = 0;
    (void)frexpf(est, &ex);
    e = 30 - ex;                     // est * 2^e < 2^30
  }
  if (ok && s0 != 0.f) jac_scatter<D>(g, B, org, tile, out, cl0, fb, s0, e);
  stream(p0 + 1, e, ok);
  // ---- the exact bound decides whether the pass stands
  {
    const float bw = wave_total(bshare);
    __syncthreads();                 // every wave has read red[] above
    if (lane == 0) red[nw + wave] = bw;
  }
  __syncthreads();
  float bt = 0.f;
  for (int q = 0; q < nw; ++q) bt += red[nw + q];
  const bool finite = bt <= 3.0e38f;
  int ee = 0;
  if (finite && bt > 0.f) {
    int ex = 0;
    (void)frexpf(bt, &ex);
    ee = 30 - ex;                    // the exact scale
  }
  const bool again = finite && bt > 0.f && (!ok || e > ee || e < ee - 3);
  if (again) {
    if (threadIdx.x == 0) atomicAdd(redo, 1);
    zero_tile();
    __syncthreads();
    bshare = 0.f;
    if (p0 < p1) load_page(p0, fa, wa, ra);
    stream(p0, ee, true);
    e = ee;
  }
  __syncthreads();
  // The tile reduction reads only the nodes inside the axis boxes of the
  // brick's indices (k_jac_pack, k_cover_filter): write the planes z0 .. z1
  // of those, each as the contiguous run of its rows y0 .. y1 (whole rows
  // along x).
  float* dst = part + bid * (long long)tot;
  const float nan = __int_as_float(0x7fc00000);
  const int nbs = B.nb[0] + B.nb[1] + B.nb[2];
  const int by = (int)((bid / B.nb[0]) % B.nb[1]), bz = (int)(bid / ((long long)B.nb[0] * B.nb[1]));
  const int y0 = axbox[B.nb[0] + by], y1 = axbox[nbs + B.nb[0] + by];
  const int z0 = D == 3 ? axbox[B.nb[0] + B.nb[1] + bz] : 0;
  const int z1 = D == 3 ? axbox[nbs + B.nb[0] + B.nb[1] + bz] : 0;
  const int run = (y1 - y0 + 1) * B.tdim[0];     // values per plane
  const int nz = z1 - z0 + 1;
  if (run > 0 && nz > 0) {
    // a wave per plane, the plane's run across the lanes with four LDS
    // reads in flight (no index division per value)
    for (int f = 0; f < D; ++f)
      for (int z = wave; z < nz; z += nw) {
        const int base = f * B.tvol + ((z0 + z) * B.tdim[1] + y0) * B.tdim[0];
        for (int j0 = 0; j0 < run; j0 += 256) {
          int v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            v[k] = tile[base + min(j0 + 64 * k + lane, run - 1)];   // unconditional: in flight together
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int j = j0 + 64 * k + lane;
            if (j < run) dst[base + j] = finite ? ldexpf((float)v[k], -e) : nan;
          }
        }
      }
  }
}

// Sum the partial tiles into the velocity-grid output in a fixed order:
// out[f][node] += sum over covering bricks (z, then y, then x order), or,
// with fb != null, out = sum + fb and fb = 0 (fb holds the kernel's
// out-of-tile atomics, so out needs no fill beforehand).  With
// K > 0 (at most K covering bricks per axis) all loads are issued before the
// sum, which adds the same terms in the same order as the generic loops.
template <int D, int K>
__device__ __forceinline__ float tile_sum(const Geo& g, const Bricks& B, int fields, const float* __restrict__ part,
                                          const int* __restrict__ cs0, const int2* __restrict__ ce0,
                                          const int* __restrict__ cs1, const int2* __restrict__ ce1,
                                          const int* __restrict__ cs2, const int2* __restrict__ ce2, long long f,
                                          int X, int Y, int Z) {
  if (D != 3) Z = 0;
  const long long tsz = (long long)fields * B.tvol;
  const float* pf = part + f * B.tvol;
  float sum = 0.f;
  if constexpr (K > 0) {
    const int sx = cs0[X], nx = cs0[X + 1] - sx;
    const int sy = cs1[Y], ny = cs1[Y + 1] - sy;
    const int sz = cs2[Z], nz = cs2[Z + 1] - sz;
    // The first two entries of each list and their 2x2x2 tile values are
    // loaded unconditionally, at indices that are always in range (a
    // conditional load becomes a branch that waits for it alone): entries
    // past a list's end read a valid slot and are replaced by (0, 0), whose
    // tile value is read and left out of the sum.  Third and later entries
    // (rarer) load under their conditions.
    int2 cx[K], cy[K], cz[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < 2) {
        const int2 ex = ce0[nx > 0 ? sx + min(k, nx - 1) : 0];
        const int2 ey = ce1[ny > 0 ? sy + min(k, ny - 1) : 0];
        const int2 ez = ce2[nz > 0 ? sz + min(k, nz - 1) : 0];
        cx[k] = k < nx ? ex : make_int2(0, 0);
        cy[k] = k < ny ? ey : make_int2(0, 0);
        cz[k] = k < nz ? ez : make_int2(0, 0);
      } else {
        cx[k] = k < nx ? ce0[sx + k] : make_int2(0, 0);
        cy[k] = k < ny ? ce1[sy + k] : make_int2(0, 0);
        cz[k] = k < nz ? ce2[sz + k] : make_int2(0, 0);
      }
    }
    float v[K][K][K];
#pragma unroll
    for (int kz = 0; kz < K; ++kz)
#pragma unroll
      for (int ky = 0; ky < K; ++ky)
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
          const long long b = cx[kx].x + (long long)B.nb[0] * (cy[ky].x + B.nb[1] * cz[kz].x);
          const int t = cx[kx].y + B.tdim[0] * (cy[ky].y + B.tdim[1] * cz[kz].y);
          if (kz < 2 && ky < 2 && kx < 2) v[kz][ky][kx] = pf[b * tsz + t];
          else v[kz][ky][kx] = (kz < nz && ky < ny && kx < nx) ? pf[b * tsz + t] : 0.f;
        }
    // the first term unconditionally and the others through selects, so no
    // load is sunk into a branch of its own (adding +0 leaves the sum as is;
    // a node without covering tiles takes 0 at the end)
    sum = v[0][0][0];
#pragma unroll
    for (int kz = 0; kz < K; ++kz)
#pragma unroll
      for (int ky = 0; ky < K; ++ky)
#pragma unroll
        for (int kx = 0; kx < K; ++kx)
          if (kz + ky + kx > 0) sum += (kz < nz && ky < ny && kx < nx) ? v[kz][ky][kx] : 0.f;
    if (nx == 0 || ny == 0 || nz == 0) sum = 0.f;
  } else {
    for (int ez = cs2[Z]; ez < cs2[Z + 1]; ++ez) {
      const int2 cz = ce2[ez];
      for (int ey = cs1[Y]; ey < cs1[Y + 1]; ++ey) {
        const int2 cy = ce1[ey];
        const int bzy = cy.x + B.nb[1] * cz.x;
        const int tzy = cy.y + B.tdim[1] * cz.y;
        for (int ex = cs0[X]; ex < cs0[X + 1]; ++ex) {
          const int2 cx = ce0[ex];
          const long long b = cx.x + (long long)B.nb[0] * bzy;
          const int t = cx.y + B.tdim[0] * tzy;
          sum += pf[b * tsz + t];
        }
      }
    }
  }
  return sum;
}

// REG = 1 (diffusion) or 2 (curvature): out = reg_value(rt.p) + (tile sum
// + fb), the operation order of the separate regulariser kernel, and with
// rt.part the block partials of rt.p . out.
template <int D, int K, int REG>
__global__ void __launch_bounds__(kBlock) k_tile_reduce(Geo g, Bricks B, int fields, const float* __restrict__ part,
                                                        const int* __restrict__ cs0, const int2* __restrict__ ce0,
                                                        const int* __restrict__ cs1, const int2* __restrict__ ce1,
                                                        const int* __restrict__ cs2, const int2* __restrict__ ce2,
                                                        float* __restrict__ fb, float* __restrict__ out, RegTail rt,
                                                        Deferred dq) {
  if (halted(g.halt)) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < g.nv * fields;
  float val = 0.f;
  if (valid) {
    // one index split and no branch between the tile sum's chain of
    // cover-list and tile loads and the regulariser's loads, which the
    // compiler then issues before it waits for the tile values
    long long f, r;
    int X, Y, Z;
    split_index(g, i, f, r, X, Y, Z);
    const float sum = tile_sum<D, K>(g, B, fields, part, cs0, ce0, cs1, ce1, cs2, ce2, f, X, Y, Z);
    float rv = 0.f;
    if constexpr (REG != 0) rv = reg_value_at<D, REG == 2>(g, rt.p, rt.scale, rt.gamma, rt.ih2, f, r, X, Y, Z);
    float t;
    if (fb) {
      t = sum + fb[i];
      fb[i] = 0.f;
    } else {
      t = out[i] + sum;
    }
    if (dq.hdr) {  // the deferred characteristics' 64-bit sums (uniform branch)
      const int n = dq.hdr[0];
      const float smax = __int_as_float(dq.hdr[1]);
      if (n > 0 && smax > 0.f) {
        t += (float)ldexp((double)(long long)dq.acc[i], -deferred_unit(n, smax));
        dq.acc[i] = 0ull;
      }
    }
    if constexpr (REG != 0) {
      val = rv + t;
    } else {
      val = t;
    }
    out[i] = val;
  }
  if constexpr (REG != 0) {
    if (rt.part) {  // kernel argument: the whole block takes this branch
      __shared__ double sh[kBlock];
      const double d = valid ? (double)rt.p[i] * (double)val : 0.0;
      const double tb = block_sum(d, sh);
      if (threadIdx.x == 0) rt.part[blockIdx.x] = tb;
    }
  }
}

int launch_tile_reduce(lag_plan P, float* out, float* fb, hipStream_t s, const RegTail* rt, bool deferred,
                       bool paged) {
  const long long tot = P->geo.nv * P->fields;
  unsigned grid = (unsigned)((tot + kBlock - 1) / kBlock);
  const RegTail none;
  const RegTail& r = rt ? *rt : none;
  Deferred dq{nullptr, nullptr, nullptr};
  if (deferred) dq = Deferred{P->dfr_list, P->dfr_hdr, P->dfr_acc};
  const int reg = r.p ? (r.curv ? 2 : 1) : 0;
  int* const* cs = paged ? P->pgc_start : P->cover_start;
  int2* const* ce = paged ? P->pgc_ent : P->cover_ent;
#define LAG_REDUCE(DIM, K, RG)                                                                                   \
  hipLaunchKernelGGL((k_tile_reduce<DIM, K, RG>), dim3(grid), dim3(kBlock), 0, s, P->geo, P->bricks, P->fields,  \
                     P->tile_part, cs[0], ce[0], cs[1], ce[1], cs[2], ce[2], fb, out, r, dq)
#define LAG_REDUCE_K(DIM, RG)          \
  do {                                 \
    if (P->cover_max <= 3)             \
      LAG_REDUCE(DIM, 3, RG);          \
    else if (P->cover_max <= 4)        \
      LAG_REDUCE(DIM, 4, RG);          \
    else                               \
      LAG_REDUCE(DIM, 0, RG);          \
  } while (0)
  if (P->geo.dim == 3) {
    if (reg == 0) LAG_REDUCE_K(3, 0);
    else if (reg == 1) LAG_REDUCE_K(3, 1);
    else LAG_REDUCE_K(3, 2);
  } else {
    if (reg == 0) LAG_REDUCE_K(2, 0);
    else if (reg == 1) LAG_REDUCE_K(2, 1);
    else LAG_REDUCE_K(2, 2);
  }
#undef LAG_REDUCE_K
#undef LAG_REDUCE
  LAG_LAUNCH_CHECK();
  if (r.part) P->php_n = (int)grid;
  return LAG_OK;
}

int tiles_setup(lag_plan P) {
  const Geo& g = P->geo;
  const Bricks& B = P->bricks;
  LAG_HIP(hipMalloc(&P->tile_part, sizeof(float) * (size_t)B.nbricks * P->fields * B.tvol));
  for (int a = 0; a < 3; ++a) {
    const int m = g.mv[a];
    std::vector<std::vector<int2>> lists(m);
    for (int b = 0; b < B.nb[a]; ++b) {
      int org = 0;
      if (a < g.dim) {
        double sv = ((double)(b * B.bdim[a]) + 0.5) * g.ratio[a] - 0.5;
        org = (int)floor(sv) - B.halo;
      }
      for (int t = 0; t < B.tdim[a]; ++t) {
        int X = ((org + t) % m + m) % m;
        lists[X].push_back(make_int2(b, t));
      }
    }
    std::vector<int> start(m + 1, 0);
    std::vector<int2> ent;
    for (int X = 0; X < m; ++X) {
      start[X] = (int)ent.size();
      ent.insert(ent.end(), lists[X].begin(), lists[X].end());
    }
    start[m] = (int)ent.size();
    for (int X = 0; X < m; ++X) P->cover_max = std::max(P->cover_max, (int)lists[X].size());
    LAG_HIP(hipMalloc(&P->cover_start[a], sizeof(int) * (m + 1)));
    LAG_HIP(hipMalloc(&P->cover_ent[a], sizeof(int2) * std::max<size_t>(ent.size(), 1)));
    LAG_HIP(hipMemcpy(P->cover_start[a], start.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice));
    LAG_HIP(hipMemcpy(P->cover_ent[a], ent.data(), sizeof(int2) * ent.size(), hipMemcpyHostToDevice));
    // the paged product's restricted lists (filled after each assembly)
    LAG_HIP(hipMalloc(&P->pgc_start[a], sizeof(int) * (m + 1)));
    LAG_HIP(hipMalloc(&P->pgc_ent[a], sizeof(int2) * std::max<size_t>(ent.size(), 1)));
  }
  LAG_HIP(hipMalloc(&P->pg_axbox, sizeof(int) * 2 * (size_t)(B.nb[0] + B.nb[1] + B.nb[2])));
  return LAG_OK;
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned grid_for(long long nlogical) {
  long long per = (nlogical + kXcds - 1) / kXcds;
  return (unsigned)(per * kXcds);
}

static inline Stages stages_for(lag_plan P, int dir) {
  Stages st;
  int k = dir < 0 ? 0 : 1;
  st.j0 = P->st_j0[k];
  st.th = P->st_th[k];
  st.dt = (float)((double)dir / (double)P->prob.nsteps);
  return st;
}

static inline int model_dir(lag_plan P) { return P->prob.model == LAG_TRANSPORT ? -1 : 1; }

int launch_pack(lag_plan P, const float* v, void* dst, hipStream_t s) {
  long long tot = P->geo.nvp * P->geo.nodes;
  unsigned grid = (unsigned)((tot + kBlock - 1) / kBlock);
  if (P->geo.dim == 3)
    hipLaunchKernelGGL(k_pack<3>, dim3(grid), dim3(kBlock), 0, s, v, (float4*)dst, P->geo, P->geo.halt);
  else
    hipLaunchKernelGGL(k_pack<2>, dim3(grid), dim3(kBlock), 0, s, v, (float2*)dst, P->geo, P->geo.halt);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_fill(float* x, long long n, float val, hipStream_t s) {
  if (n <= 0) return LAG_OK;
  unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, s, x, n, val);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

#define LAG_DISPATCH_DNS(KERNEL, ...)                                              \
  do {                                                                             \
    const bool ns_ = P->geo.nodes > 1;                                             \
    if (P->geo.dim == 3) {                                                         \
      if (ns_) hipLaunchKernelGGL((KERNEL<3, true>), __VA_ARGS__);                 \
      else hipLaunchKernelGGL((KERNEL<3, false>), __VA_ARGS__);                    \
    } else {                                                                       \
      if (ns_) hipLaunchKernelGGL((KERNEL<2, true>), __VA_ARGS__);                 \
      else hipLaunchKernelGGL((KERNEL<2, false>), __VA_ARGS__);                    \
    }                                                                              \
  } while (0)

int launch_trace(lag_plan P, const void* vpack, int dir, float* phi, hipStream_t s) {
  Stages st = stages_for(P, dir);
  const lag::Bricks& B = P->bricks;
  const size_t tile = sizeof(float) * (size_t)P->geo.dim * B.tvol;
  if (P->geo.nodes == 1 && tile <= 64 * 1024) {  // LDS-staged velocity tile per brick
    unsigned grid = grid_for(B.nbricks);
    if (P->geo.dim == 3)
      hipLaunchKernelGGL(k_trace_tile<3>, dim3(grid), dim3(kTraceBlock), tile, s, P->geo, st, B, (const float4*)vpack,
                         phi);
    else
      hipLaunchKernelGGL(k_trace_tile<2>, dim3(grid), dim3(kTraceBlock), tile, s, P->geo, st, B, (const float2*)vpack,
                         phi);
    LAG_LAUNCH_CHECK();
    return LAG_OK;
  }
  unsigned grid = grid_for((P->geo.np + kBlock - 1) / kBlock);
  if (P->geo.dim == 3) {
    if (P->geo.nodes > 1)
      hipLaunchKernelGGL((k_trace<3, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st, (const float4*)vpack, phi);
    else
      hipLaunchKernelGGL((k_trace<3, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st, (const float4*)vpack, phi);
  } else {
    if (P->geo.nodes > 1)
      hipLaunchKernelGGL((k_trace<2, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st, (const float2*)vpack, phi);
    else
      hipLaunchKernelGGL((k_trace<2, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st, (const float2*)vpack, phi);
  }
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}

int launch_transport(lag_plan P, const float* T, const float* phi, float* u, hipStream_t s) {
  unsigned grid = grid_for((P->geo.np + kBlock - 1) / kBlock);
  if (P->geo.dim == 3)
    hipLaunchKernelGGL(k_transport<3>, dim3(grid), dim3(kBlock), 0, s, P->geo, T, phi, u);
  else
    hipLaunchKernelGGL(k_transport<2>, dim3(grid), dim3(kBlock), 0, s, P->geo, T, phi, u);
  LAG_LAUNCH_CHECK();
  return LAG_OK;
}


int launch_pushforward_bins(const Geo& g, const BinScratch& b, const float* T, const float* phi, float* u,
                            hipStream_t s) {
  int rc = launch_zero_i(b.count, g.np + 1, s);
  if (rc) return rc;
  const unsigned grid = grid_for((g.np + kBlock - 1) / kBlock);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_push_prep<3>, dim3(grid), dim3(kBlock), 0, s, g, T, phi, b.base, b.vals, b.count);
  else
    hipLaunchKernelGGL(k_push_prep<2>, dim3(grid), dim3(kBlock), 0, s, g, T, phi, b.base, b.vals, b.count);
  LAG_LAUNCH_CHECK();
  return bin_and_gather(g, b, u, s);
}

int launch_pushforward(lag_plan P, const float* T, const float* phi, float* u, hipStream_t s) {
  return launch_pushforward_bins(P->geo, plan_bins(P), T, phi, u, s);
}

int launch_jvp(lag_plan P, const void* vpack, const void* dpack, const float* T, float* out, hipStream_t s) {
  const int dir = model_dir(P);
  Stages st = stages_for(P, dir);
  unsigned grid = grid_for((P->geo.np + kBlock - 1) / kBlock);
  if (P->prob.model == LAG_TRANSPORT) {
    if (P->geo.dim == 3) {
      if (P->geo.nodes > 1)
        hipLaunchKernelGGL((k_jvp_transport<3, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                           (const float4*)vpack, (const float4*)dpack, T, out);
      else
        hipLaunchKernelGGL((k_jvp_transport<3, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                           (const float4*)vpack, (const float4*)dpack, T, out);
    } else {
      if (P->geo.nodes > 1)
        hipLaunchKernelGGL((k_jvp_transport<2, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                           (const float2*)vpack, (const float2*)dpack, T, out);
      else
        hipLaunchKernelGGL((k_jvp_transport<2, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                           (const float2*)vpack, (const float2*)dpack, T, out);
    }
    LAG_LAUNCH_CHECK();
    return LAG_OK;
  }
  int rc = launch_zero_i(P->bin_count, P->geo.np + 1, s);
  if (rc) return rc;
  if (P->geo.dim == 3) {
    if (P->geo.nodes > 1)
      hipLaunchKernelGGL((k_jvp_cont_prep<3, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                         (const float4*)vpack, (const float4*)dpack, T, P->part_base, P->part_vals, P->bin_count);
    else
      hipLaunchKernelGGL((k_jvp_cont_prep<3, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                         (const float4*)vpack, (const float4*)dpack, T, P->part_base, P->part_vals, P->bin_count);
  } else {
    if (P->geo.nodes > 1)
      hipLaunchKernelGGL((k_jvp_cont_prep<2, true>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                         (const float2*)vpack, (const float2*)dpack, T, P->part_base, P->part_vals, P->bin_count);
    else
      hipLaunchKernelGGL((k_jvp_cont_prep<2, false>), dim3(grid), dim3(kBlock), 0, s, P->geo, st,
                         (const float2*)vpack, (const float2*)dpack, T, P->part_base, P->part_vals, P->bin_count);
  }
  LAG_LAUNCH_CHECK();
  return bin_and_gather(P->geo, plan_bins(P), out, s);
}

size_t adjoint_lds_bytes(lag_plan P) {
  return sizeof(unsigned long long) * (size_t)P->fields * P->bricks.tvol + sizeof(float) * (512 / 64);
}

// Matrix-free adjoint product: the tile pass, then (when some characteristic
// left its tile) the two passes over the deferred list, then the fixed-order
// reduction of the tiles plus the deferred sums.  out must hold zeros (the
// tile pass's float fallback adds into it).
template <int D, bool NS, int MODE, bool ZERO>
static int launch_adjoint_t(lag_plan P, const AdjArgs& A, const Stages& st, float* out, hipStream_t s, bool prof) {
  const lag::Bricks& B = P->bricks;
  const Deferred dq{P->dfr_list, P->dfr_hdr, P->dfr_acc};
  int rc = launch_zero_i(P->dfr_hdr, 3, s);
  if (rc) return rc;
  const size_t lds = adjoint_lds_bytes(P);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) prof_events(P, &e0, &e1);
  if (e0)
    hipExtLaunchKernelGGL((k_adjoint<D, NS, MODE, ZERO>), dim3(grid_for(B.nbricks)), dim3(AdjBlock<D, NS>::threads),
                          lds, s, e0, e1, 0, P->geo, st, B, A, out, P->tile_part, P->flags, dq);
  else
    hipLaunchKernelGGL((k_adjoint<D, NS, MODE, ZERO>), dim3(grid_for(B.nbricks)), dim3(AdjBlock<D, NS>::threads), lds,
                       s, P->geo, st, B, A, out, P->tile_part, P->flags, dq);
  LAG_LAUNCH_CHECK();
  if constexpr (!ZERO) {
    const unsigned dgrid = (unsigned)std::min<long long>((P->geo.np + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL((k_adjoint_deferred<D, NS, MODE, 0>), dim3(dgrid), dim3(kBlock), 0, s, P->geo, st, A, dq,
                       P->flags);
    hipLaunchKernelGGL((k_adjoint_deferred<D, NS, MODE, 1>), dim3(dgrid), dim3(kBlock), 0, s, P->geo, st, A, dq,
                       P->flags);
    LAG_LAUNCH_CHECK();
  }
  return launch_tile_reduce(P, out, nullptr, s, nullptr, !ZERO);
}

template <int MODE, bool ZERO>
static int launch_adjoint(lag_plan P, const AdjArgs& A, const Stages& st, float* out, hipStream_t s, bool prof) {
  const bool ns = P->geo.nodes > 1;
  if (P->geo.dim == 3)
    return ns ? launch_adjoint_t<3, true, MODE, ZERO>(P, A, st, out, s, prof)
              : launch_adjoint_t<3, false, MODE, ZERO>(P, A, st, out, s, prof);
  return ns ? launch_adjoint_t<2, true, MODE, ZERO>(P, A, st, out, s, prof)
            : launch_adjoint_t<2, false, MODE, ZERO>(P, A, st, out, s, prof);
}

int launch_vjp(lag_plan P, const void* vpack, const float* T, const float* w, float* out, hipStream_t s,
               bool zero) {
  int rc = launch_fill(out, P->n_unknowns, 0.f, s);
  if (rc) return rc;
  const Stages st = stages_for(P, model_dir(P));
  const AdjArgs A{zero ? nullptr : vpack, nullptr, T, w, nullptr};
  if (P->prob.model == LAG_TRANSPORT)
    return zero ? launch_adjoint<0, true>(P, A, st, out, s, false) : launch_adjoint<0, false>(P, A, st, out, s, false);
  return zero ? launch_adjoint<1, true>(P, A, st, out, s, false) : launch_adjoint<1, false>(P, A, st, out, s, false);
}

int launch_hess_transport(lag_plan P, const void* vpack, const void* ppack, const float* T, const float* wvox,
                          float* out, hipStream_t s) {
  const Stages st = stages_for(P, -1);
  const AdjArgs A{vpack, ppack, T, nullptr, wvox};
  return launch_adjoint<2, false>(P, A, st, out, s, true);
}

int launch_jac_assemble(lag_plan P, const void* vpack, const float* T, float* u, hipStream_t s) {
  Stages st = stages_for(P, -1);
  const lag::Bricks& B = P->bricks;
  const long long items = (long long)B.nbricks * B.nreg[0] * B.nreg[1] * B.nreg[2] * B.stride[0] * B.stride[1] *
                          B.stride[2];
  unsigned grid = grid_for((items + kBlock / 64 - 1) / (kBlock / 64));
  int rc = launch_zero_i(P->jac_max, 2, s);
  if (rc) return rc;
  // the stored-trajectory sweep keeps N step start points per thread in LDS
  const size_t traj = sizeof(float) * (size_t)P->geo.nsteps * P->geo.dim * kBlock;
  const bool stored = traj <= 64 * 1024;
  const size_t lds = stored ? traj : 0;
#define LAG_ASM(DIM, ST, VT)                                                                                     \
  hipLaunchKernelGGL((k_jac_assemble<DIM, ST>), dim3(grid), dim3(kBlock), lds, s, P->geo, st, B, (const VT*)vpack, \
                     T, P->jac_vals, P->jac_cell, P->jac_cnt, P->jac_slots, P->jac_k, P->jac_max, P->flags, u)
  if (P->geo.dim == 3) {
    if (stored) LAG_ASM(3, true, float4);
    else LAG_ASM(3, false, float4);
  } else {
    if (stored) LAG_ASM(2, true, float2);
    else LAG_ASM(2, false, float2);
  }
#undef LAG_ASM
  LAG_LAUNCH_CHECK();
  if (P->pg_cap > 0) {  // the paged copy the products read
    const size_t prows = (size_t)B.bdim[0] * B.bdim[1] * B.bdim[2];
    const size_t plds = 2 * sizeof(int) * ((prows + 3) & ~(size_t)3) + ((prows + 63) & ~(size_t)63);
    unsigned pgrid = grid_for(B.nbricks);
    const int nbs = B.nb[0] + B.nb[1] + B.nb[2];
    hipLaunchKernelGGL(k_axbox_init, dim3((2 * nbs + 255) / 256), dim3(256), 0, s, P->pg_axbox, nbs);
    LAG_LAUNCH_CHECK();
    if (P->geo.dim == 3)
      hipLaunchKernelGGL(k_jac_pack<3>, dim3(pgrid), dim3(kBlock), plds, s, B, P->jac_vals, P->jac_cell, P->jac_cnt,
                         P->jac_slots, P->pg_cap, P->pg_vals, P->pg_cells, P->pg_rows, P->pg_npages, P->pg_axbox);
    else
      hipLaunchKernelGGL(k_jac_pack<2>, dim3(pgrid), dim3(kBlock), plds, s, B, P->jac_vals, P->jac_cell, P->jac_cnt,
                         P->jac_slots, P->pg_cap, P->pg_vals, P->pg_cells, P->pg_rows, P->pg_npages, P->pg_axbox);
    LAG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cover_filter, dim3(3), dim3(1024), 0, s, P->geo.dim,
                       make_int3(P->geo.mv[0], P->geo.mv[1], P->geo.mv[2]), make_int3(B.nb[0], B.nb[1], B.nb[2]),
                       P->pg_axbox, P->cover_start[0], P->cover_ent[0], P->cover_start[1], P->cover_ent[1],
                       P->cover_start[2], P->cover_ent[2], P->pgc_start[0], P->pgc_ent[0], P->pgc_start[1],
                       P->pgc_ent[1], P->pgc_start[2], P->pgc_ent[2]);
    LAG_LAUNCH_CHECK();
    const int balance = B.nbricks < 16000;   // the page-count prefix fits 64 KB of LDS
    hipLaunchKernelGGL(k_brick_order, dim3(1), dim3(1024), balance ? sizeof(int) * (B.nbricks + 1) : 0, s,
                       P->pg_npages, (int)B.nbricks, pg_xcd_slots(B.nbricks), balance, P->pg_order);
    LAG_LAUNCH_CHECK();
  }
  return LAG_OK;
}

int jac_pages_per_brick(lag_plan P, int kmax) {
  const lag::Bricks& B = P->bricks;
  const long long rows = (long long)B.bdim[0] * B.bdim[1] * B.bdim[2];
  if (kmax < 1 || kmax > 64 || rows * (long long)(2 * sizeof(int) + 1) + 128 > 64 * 1024) return 0;
  return jac_page_cap(rows, kmax);
}

int launch_jac_apply(lag_plan P, const void* ppack, const float* wvox, const float* wseed, float scale, float* out,
                     hipStream_t s, const RegTail* rt) {
  const lag::Bricks& B = P->bricks;
  unsigned grid = grid_for(B.nbricks);
  const size_t lds = sizeof(float) * ((size_t)P->geo.dim * B.tvol + 2 * (kBlock / 64));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!wseed) prof_events(P, &e0, &e1);
  if (P->pg_cap > 0) {
    grid = (unsigned)pg_order_len(B.nbricks);   // the order array's slots (k_brick_order)
    const size_t plds = sizeof(float) * ((size_t)P->geo.dim * B.tvol + 2 * (kPgBlock / 64) + kPgBlock);
#define LAG_PG(DD, WS, WV, VT)                                                                                    \
  do {                                                                                                            \
    if (e0)                                                                                                       \
      hipExtLaunchKernelGGL((k_jac_apply_pg<DD, WS, WV>), dim3(grid), dim3(kPgBlock), plds, s, e0, e1, 0, P->geo,  \
                            B, P->pg_vals, P->pg_cells, P->pg_rows, P->pg_npages, P->pg_order, P->pg_cap,          \
                            (const VT*)ppack, wvox, wseed, scale, P->jac_fb, P->tile_part, P->pg_redo,             \
                            P->pg_axbox);                                                                         \
    else                                                                                                          \
      hipLaunchKernelGGL((k_jac_apply_pg<DD, WS, WV>), dim3(grid), dim3(kPgBlock), plds, s, P->geo, B, P->pg_vals, \
                         P->pg_cells, P->pg_rows, P->pg_npages, P->pg_order, P->pg_cap, (const VT*)ppack, wvox,    \
                         wseed, scale, P->jac_fb, P->tile_part, P->pg_redo, P->pg_axbox);                          \
  } while (0)
    if (P->geo.dim == 3) {
      if (wseed) LAG_PG(3, true, false, float4);
      else if (wvox) LAG_PG(3, false, true, float4);
      else LAG_PG(3, false, false, float4);
    } else {
      if (wseed) LAG_PG(2, true, false, float2);
      else if (wvox) LAG_PG(2, false, true, float2);
      else LAG_PG(2, false, false, float2);
    }
#undef LAG_PG
  } else if (P->geo.dim == 3) {
    if (e0)
      hipExtLaunchKernelGGL(k_jac_apply<3>, dim3(grid), dim3(kBlock), lds, s, e0, e1, 0, P->geo, B, P->jac_vals,
                            P->jac_cell, P->jac_cnt, P->jac_slots, (const float4*)ppack, wvox, wseed, scale,
                            P->jac_fb, P->tile_part);
    else
      hipLaunchKernelGGL(k_jac_apply<3>, dim3(grid), dim3(kBlock), lds, s, P->geo, B, P->jac_vals, P->jac_cell,
                         P->jac_cnt, P->jac_slots, (const float4*)ppack, wvox, wseed, scale, P->jac_fb,
                         P->tile_part);
  } else {
    if (e0)
      hipExtLaunchKernelGGL(k_jac_apply<2>, dim3(grid), dim3(kBlock), lds, s, e0, e1, 0, P->geo, B, P->jac_vals,
                            P->jac_cell, P->jac_cnt, P->jac_slots, (const float2*)ppack, wvox, wseed, scale,
                            P->jac_fb, P->tile_part);
    else
      hipLaunchKernelGGL(k_jac_apply<2>, dim3(grid), dim3(kBlock), lds, s, P->geo, B, P->jac_vals, P->jac_cell,
                         P->jac_cnt, P->jac_slots, (const float2*)ppack, wvox, wseed, scale, P->jac_fb,
                         P->tile_part);
  }
  LAG_LAUNCH_CHECK();
  // assigns out; the paged product wrote only the nodes its cover lists read
  return launch_tile_reduce(P, out, P->jac_fb, s, rt, false, P->pg_cap > 0);
}

}  // namespace lag
