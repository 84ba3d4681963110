// Device-side building blocks shared by the laglddmm kernels (gfx950).
//
// Geometry: periodic cell-centred grids.  A characteristic is identified by
// its start image cell (integer multi-index) and carries its displacement
// phi from that cell centre.  Its fractional cell coordinate on a grid with
// m_G cells per axis is s = (i + 1/2) m_G/m_img - 1/2 + phi m_G/L; the
// integer part of the constant term is kept as an int and only the small
// fractional remainder is added to phi m_G/L in float32, so cell selection
// loses no precision to large absolute coordinates.
//
// Interpolation (Sec. 3.1): trilinear (bilinear) in space per velocity
// component, linear in time between velocity nodes.  Velocities are packed
// per node as float4 {vx, vy, vz, 0} (3-D) or float2 {vx, vy} (2-D) so one
// corner of one sample is one vector load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lag {

constexpr int kBlock = 256;        // threads per block for point kernels
constexpr int kXcds = 8;           // MI355X: 8 XCDs, blocks dispatched round-robin

template <int D> struct VecT;
template <> struct VecT<2> { using T = float2; };
template <> struct VecT<3> { using T = float4; };

// Launch-time geometry of one problem (passed by value).
struct Geo {
  int dim;
  int nodes;
  int nsteps;
  int mi[3];            // image cells per axis (unused axes 1)
  int mv[3];            // velocity cells per axis
  float inv_hi[3];      // m_img / L
  float inv_hv[3];      // m_vel / L
  double ratio[3];      // m_vel / m_img
  long long np;         // image cells = characteristics
  long long nv;         // velocity cells per field
  int pv[3];            // packed-field extents: mv + 1 on used axes (periodic ghost layer), else 1
  long long nvp;        // packed-field nodes per time node
  float cell_img;       // image cell volume h^d
  // device flag of a graph-captured PCG loop: once non-zero, the kernels of
  // the loop return at entry (null outside captured graphs)
  const int* halt;
};

__device__ __forceinline__ bool halted(const int* h) { return h != nullptr && *h != 0; }

// Per-call RK4 stage-time table: for stage q = 4k + s the lower node j0 and
// the weight theta of node j0 + 1 (linear interpolation in time).
struct Stages {
  const int* j0;
  const float* th;
  float dt;
};

// Brick decomposition used by kernels that accumulate into the velocity
// grid through an LDS tile.
struct Bricks {
  int bdim[3];        // brick size in image cells
  int nb[3];          // bricks per axis
  int nbricks;        // total
  int stride[3];      // lane stride in image cells (about m_img / m_vel)
  int lsh[3];         // log2 of the wave's lane lattice per axis (lane bits x, then y, then z)
  int rdim[3];        // wave region = lattice extent * stride per axis
  int nreg[3];        // regions per brick per axis
  int tdim[3];        // LDS tile size in velocity cells
  int halo;           // tile margin in velocity cells
  int tvol;           // tdim product
};

// A lane's position on the wave's lane lattice.
__device__ __forceinline__ void lane_lattice(const Bricks& B, int lane, int l[3]) {
  l[0] = lane & ((1 << B.lsh[0]) - 1);
  l[1] = (lane >> B.lsh[0]) & ((1 << B.lsh[1]) - 1);
  l[2] = lane >> (B.lsh[0] + B.lsh[1]);
}

__device__ __forceinline__ int wrapi(int c, int m) {
  if ((unsigned)c < (unsigned)m) return c;
  int r = c % m;
  return r < 0 ? r + m : r;
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

// XCD-aware block remap: consecutive logical blocks land on the same XCD so
// each XCD's L2 sees a compact part of the grid.  Launch kXcds*ceil(n/kXcds)
// blocks; returns -1 for the padding blocks.
__device__ __forceinline__ long long xcd_block(long long nlogical) {
  long long b = blockIdx.x;
  long long per = (nlogical + kXcds - 1) / kXcds;
  long long id = (b % kXcds) * per + b / kXcds;
  return id < nlogical ? id : -1;
}

template <int D>
struct Start {
  int i[D];          // image cell multi-index
  int cv[D];         // integer part of the start coordinate on the velocity grid
  float fv[D];       // fractional part (exact for power-of-two ratios)
};

template <int D>
__device__ __forceinline__ void make_start(const Geo& g, long long p, Start<D>& S) {
  long long r = p;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S.i[a] = (int)(r % g.mi[a]);
    r /= g.mi[a];
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s = ((double)S.i[a] + 0.5) * g.ratio[a] - 0.5;
    double fl = floor(s);
    S.cv[a] = (int)fl;
    S.fv[a] = (float)(s - fl);
  }
}

template <int D>
__device__ __forceinline__ void make_start_idx(const Geo& g, const int idx[D], Start<D>& S) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S.i[a] = idx[a];
    double s = ((double)idx[a] + 0.5) * g.ratio[a] - 0.5;
    double fl = floor(s);
    S.cv[a] = (int)fl;
    S.fv[a] = (float)(s - fl);
  }
}

template <int D> struct Loc { int c[D]; float f[D]; };

// Point on the velocity grid.
template <int D>
__device__ __forceinline__ void locate_v(const Geo& g, const Start<D>& S, const float phi[D], Loc<D>& L) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = fmaf(phi[a], g.inv_hv[a], S.fv[a]);
    float fl = floorf(t);
    L.c[a] = S.cv[a] + (int)fl;
    L.f[a] = t - fl;
  }
}

// Point on the image grid (start coordinate is the integer cell itself).
template <int D>
__device__ __forceinline__ void locate_i(const Geo& g, const Start<D>& S, const float phi[D], Loc<D>& L) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = phi[a] * g.inv_hi[a];
    float fl = floorf(t);
    L.c[a] = S.i[a] + (int)fl;
    L.f[a] = t - fl;
  }
}

// ---------------------------------------------------------------------------
// Vector field sampling: value and (optionally) spatial Jacobian G[c][a] =
// d v_c / d y_a of the trilinear interpolant.  One-sided on grid lines
// (the floor-selected cell), consistent with the oracle.
// Regulariser value at entry i of a velocity-shaped field p (Sec. 2.1):
// s_j A p_{j,c} (+ gamma p) with A = -Laplace_h (diffusion) or Laplace_h^2
// (curvature) on the periodic grid, s_j = scale[node]; differences are
// formed before scaling so smooth fields lose little to cancellation.
template <int D>
__device__ __forceinline__ float lap_at(const float* __restrict__ f, const int m[3], const float ih2[3],
                                        int x, int y, int z) {
  // -Laplace_h f at (x, y, z); arguments already wrapped
  const float c = f[((long long)z * m[1] + y) * m[0] + x];
  float s = 0.f;
  {
    int xp = x + 1 == m[0] ? 0 : x + 1, xm = x == 0 ? m[0] - 1 : x - 1;
    float a = f[((long long)z * m[1] + y) * m[0] + xp] - c;
    float b = f[((long long)z * m[1] + y) * m[0] + xm] - c;
    s = fmaf(-(a + b), ih2[0], s);
  }
  {
    int yp = y + 1 == m[1] ? 0 : y + 1, ym = y == 0 ? m[1] - 1 : y - 1;
    float a = f[((long long)z * m[1] + yp) * m[0] + x] - c;
    float b = f[((long long)z * m[1] + ym) * m[0] + x] - c;
    s = fmaf(-(a + b), ih2[1], s);
  }
  if (D == 3) {
    int zp = z + 1 == m[2] ? 0 : z + 1, zm = z == 0 ? m[2] - 1 : z - 1;
    float a = f[((long long)zp * m[1] + y) * m[0] + x] - c;
    float b = f[((long long)zm * m[1] + y) * m[0] + x] - c;
    s = fmaf(-(a + b), ih2[2], s);
  }
  return s;
}

// Field f and node r (with its x, y, z on the velocity grid) of the flat
// index i = f nv + r: 32-bit divisions where the indices fit (the 64-bit
// ones expand into long branchy sequences), else 64-bit.
__device__ __forceinline__ void split_index(const Geo& g, long long i, long long& f, long long& r, int& x, int& y,
                                            int& z) {
  if (i < 0x7fffffffLL && g.nv < 0x7fffffffLL) {
    const unsigned ui = (unsigned)i, nv = (unsigned)g.nv, m0 = (unsigned)g.mv[0], m1 = (unsigned)g.mv[1];
    const unsigned uf = ui / nv, ur = ui - uf * nv, t = ur / m0;
    f = uf;
    r = ur;
    x = (int)(ur - t * m0);
    y = (int)(t % m1);
    z = (int)(t / m1);
  } else {
    f = i / g.nv;
    r = i - f * g.nv;
    x = (int)(r % g.mv[0]);
    y = (int)((r / g.mv[0]) % g.mv[1]);
    z = (int)(r / ((long long)g.mv[0] * g.mv[1]));
  }
}

// The regulariser at field f, node r = (x, y, z) (split_index).
template <int D, bool CURV>
__device__ __forceinline__ float reg_value_at(const Geo& g, const float* __restrict__ p,
                                              const float* __restrict__ scale, float gamma, const float ih2[3],
                                              long long f, long long r, int x, int y, int z) {
  const int j = (int)(f / D);
  const float* fld = p + f * g.nv;
  const int m[3] = {g.mv[0], g.mv[1], D == 3 ? g.mv[2] : 1};
  float a;
  if (!CURV) {
    a = lap_at<D>(fld, m, ih2, x, y, z);
  } else {
    // (-Laplace)(-Laplace p) by differences of the inner Laplacian
    const float c = lap_at<D>(fld, m, ih2, x, y, z);
    float s = 0.f;
    {
      int xp = x + 1 == m[0] ? 0 : x + 1, xm = x == 0 ? m[0] - 1 : x - 1;
      float u = lap_at<D>(fld, m, ih2, xp, y, z) - c, w = lap_at<D>(fld, m, ih2, xm, y, z) - c;
      s = fmaf(-(u + w), ih2[0], s);
    }
    {
      int yp = y + 1 == m[1] ? 0 : y + 1, ym = y == 0 ? m[1] - 1 : y - 1;
      float u = lap_at<D>(fld, m, ih2, x, yp, z) - c, w = lap_at<D>(fld, m, ih2, x, ym, z) - c;
      s = fmaf(-(u + w), ih2[1], s);
    }
    if (D == 3) {
      int zp = z + 1 == m[2] ? 0 : z + 1, zm = z == 0 ? m[2] - 1 : z - 1;
      float u = lap_at<D>(fld, m, ih2, x, y, zp) - c, w = lap_at<D>(fld, m, ih2, x, y, zm) - c;
      s = fmaf(-(u + w), ih2[2], s);
    }
    a = s;
  }
  float val = scale[j] * a;
  const float cr = fld[r];           // loaded either way: no branch around a load
  if (gamma != 0.f) val = fmaf(gamma, cr, val);
  return val;
}

template <int D, bool CURV>
__device__ __forceinline__ float reg_value(const Geo& g, const float* __restrict__ p, const float* __restrict__ scale,
                                           float gamma, const float ih2[3], long long i) {
  long long f, r;
  int x, y, z;
  split_index(g, i, f, r, x, y, z);   // z = 0 in 2-D (a node lies below mv[0] mv[1])
  return reg_value_at<D, CURV>(g, p, scale, gamma, ih2, f, r, x, y, z);
}

// Block-wide float64 sum in a fixed tree (every thread of the block calls
// it; all get the total).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return sh[0];
}

// Regulariser term fused into the tile reduction of the assembled products:
// out = reg_value(p) + (tile sum); with part != null also the block partials
// of p . out (float64).
struct RegTail {
  const float* p = nullptr;
  const float* scale = nullptr;
  float gamma = 0.f;
  float ih2[3] = {0.f, 0.f, 0.f};
  int curv = 0;
  double* part = nullptr;
};

// Packed fields carry a periodic ghost layer (k_pack), so the eight corners
// of a cell sit at fixed offsets from its lower corner: +1 along x, +pv[0]
// along y, +pv[0] pv[1] along z.
__device__ __forceinline__ unsigned packed_corner(const Geo& g, int x0, int y0, int z0) {
  return ((unsigned)z0 * (unsigned)g.pv[1] + (unsigned)y0) * (unsigned)g.pv[0] + (unsigned)x0;
}

template <bool GRAD>
__device__ __forceinline__ void sample_vec(const float4* __restrict__ f, const Geo& g, const Loc<3>& L,
                                           float val[3], float G[3][3]) {
  const int x0 = wrapi(L.c[0], g.mv[0]), y0 = wrapi(L.c[1], g.mv[1]), z0 = wrapi(L.c[2], g.mv[2]);
  const unsigned sy = (unsigned)g.pv[0], sz = (unsigned)g.pv[0] * (unsigned)g.pv[1];
  const float4* c0 = f + packed_corner(g, x0, y0, z0);
  const float4* c1 = c0 + sz;
  float4 a000 = c0[0], a100 = c0[1];
  float4 a010 = c0[sy], a110 = c0[sy + 1];
  float4 a001 = c1[0], a101 = c1[1];
  float4 a011 = c1[sy], a111 = c1[sy + 1];
  const float fx = L.f[0], fy = L.f[1], fz = L.f[2];
#define LAG_COMP(c, FLD)                                                         \
  {                                                                             \
    float e00 = lerpf(a000.FLD, a100.FLD, fx), e10 = lerpf(a010.FLD, a110.FLD, fx); \
    float e01 = lerpf(a001.FLD, a101.FLD, fx), e11 = lerpf(a011.FLD, a111.FLD, fx); \
    float g0 = lerpf(e00, e10, fy), g1 = lerpf(e01, e11, fy);                   \
    val[c] = lerpf(g0, g1, fz);                                                 \
    if (GRAD) {                                                                 \
      G[c][2] = (g1 - g0) * g.inv_hv[2];                                        \
      G[c][1] = lerpf(e10 - e00, e11 - e01, fz) * g.inv_hv[1];                  \
      float d0 = lerpf(a100.FLD - a000.FLD, a110.FLD - a010.FLD, fy);           \
      float d1 = lerpf(a101.FLD - a001.FLD, a111.FLD - a011.FLD, fy);           \
      G[c][0] = lerpf(d0, d1, fz) * g.inv_hv[0];                                \
    }                                                                           \
  }
  LAG_COMP(0, x)
  LAG_COMP(1, y)
  LAG_COMP(2, z)
#undef LAG_COMP
}

template <bool GRAD>
__device__ __forceinline__ void sample_vec(const float2* __restrict__ f, const Geo& g, const Loc<2>& L,
                                           float val[2], float G[2][2]) {
  const int x0 = wrapi(L.c[0], g.mv[0]), y0 = wrapi(L.c[1], g.mv[1]);
  const unsigned sy = (unsigned)g.pv[0];
  const float2* c0 = f + packed_corner(g, x0, y0, 0);
  float2 a00 = c0[0], a10 = c0[1];
  float2 a01 = c0[sy], a11 = c0[sy + 1];
  const float fx = L.f[0], fy = L.f[1];
#define LAG_COMP(c, FLD)                                                   \
  {                                                                       \
    float e0 = lerpf(a00.FLD, a10.FLD, fx), e1 = lerpf(a01.FLD, a11.FLD, fx); \
    val[c] = lerpf(e0, e1, fy);                                           \
    if (GRAD) {                                                           \
      G[c][1] = (e1 - e0) * g.inv_hv[1];                                  \
      G[c][0] = lerpf(a10.FLD - a00.FLD, a11.FLD - a01.FLD, fy) * g.inv_hv[0]; \
    }                                                                     \
  }
  LAG_COMP(0, x)
  LAG_COMP(1, y)
#undef LAG_COMP
}

// Velocity (and Jacobian) at stage q of the current sweep: stationary fields
// have one node; otherwise blend nodes j0 and j0+1 with weight theta.
template <int D, bool NS, bool GRAD>
__device__ __forceinline__ void sample_vel(const typename VecT<D>::T* __restrict__ f, const Geo& g,
                                           const Stages& st, int q, const Loc<D>& L,
                                           float val[D], float G[D][D]) {
  if (!NS) {
    sample_vec<GRAD>(f, g, L, val, G);
  } else {
    int j0 = st.j0[q];
    float th = st.th[q];
    float v0[D], v1[D], G0[D][D], G1[D][D];
    sample_vec<GRAD>(f + (long long)j0 * g.nvp, g, L, v0, G0);
    sample_vec<GRAD>(f + (long long)(j0 + 1) * g.nvp, g, L, v1, G1);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      val[c] = lerpf(v0[c], v1[c], th);
      if (GRAD) {
#pragma unroll
        for (int a = 0; a < D; ++a) G[c][a] = lerpf(G0[c][a], G1[c][a], th);
      }
    }
  }
}

// Scalar image sampling: value and gradient of the (bi/tri)linear interpolant.
template <int D, bool VAL, bool GRAD>
__device__ __forceinline__ void sample_img(const float* __restrict__ T, const Geo& g, const Loc<D>& L,
                                           float& val, float grad[D]) {
  if constexpr (D == 3) {
    const int mx = g.mi[0], my = g.mi[1], mz = g.mi[2];
    int x0 = wrapi(L.c[0], mx), y0 = wrapi(L.c[1], my), z0 = wrapi(L.c[2], mz);
    int x1 = (x0 + 1 == mx) ? 0 : x0 + 1;
    int y1 = (y0 + 1 == my) ? 0 : y0 + 1;
    int z1 = (z0 + 1 == mz) ? 0 : z0 + 1;
    long long r00 = ((long long)z0 * my + y0) * mx, r01 = ((long long)z0 * my + y1) * mx;
    long long r10 = ((long long)z1 * my + y0) * mx, r11 = ((long long)z1 * my + y1) * mx;
    float a000 = T[r00 + x0], a100 = T[r00 + x1], a010 = T[r01 + x0], a110 = T[r01 + x1];
    float a001 = T[r10 + x0], a101 = T[r10 + x1], a011 = T[r11 + x0], a111 = T[r11 + x1];
    const float fx = L.f[0], fy = L.f[1], fz = L.f[2];
    float e00 = lerpf(a000, a100, fx), e10 = lerpf(a010, a110, fx);
    float e01 = lerpf(a001, a101, fx), e11 = lerpf(a011, a111, fx);
    float g0 = lerpf(e00, e10, fy), g1 = lerpf(e01, e11, fy);
    if (VAL) val = lerpf(g0, g1, fz);
    if (GRAD) {
      grad[2] = (g1 - g0) * g.inv_hi[2];
      grad[1] = lerpf(e10 - e00, e11 - e01, fz) * g.inv_hi[1];
      float d0 = lerpf(a100 - a000, a110 - a010, fy);
      float d1 = lerpf(a101 - a001, a111 - a011, fy);
      grad[0] = lerpf(d0, d1, fz) * g.inv_hi[0];
    }
  } else {
    const int mx = g.mi[0], my = g.mi[1];
    int x0 = wrapi(L.c[0], mx), y0 = wrapi(L.c[1], my);
    int x1 = (x0 + 1 == mx) ? 0 : x0 + 1;
    int y1 = (y0 + 1 == my) ? 0 : y0 + 1;
    float a00 = T[(long long)y0 * mx + x0], a10 = T[(long long)y0 * mx + x1];
    float a01 = T[(long long)y1 * mx + x0], a11 = T[(long long)y1 * mx + x1];
    const float fx = L.f[0], fy = L.f[1];
    float e0 = lerpf(a00, a10, fx), e1 = lerpf(a01, a11, fx);
    if (VAL) val = lerpf(e0, e1, fy);
    if (GRAD) {
      grad[1] = (e1 - e0) * g.inv_hi[1];
      grad[0] = lerpf(a10 - a00, a11 - a01, fy) * g.inv_hi[0];
    }
  }
}

// Corner weights of a linear stencil, corner code bit a = offset along axis a.
template <int D>
__device__ __forceinline__ void corner_weights(const Loc<D>& L, float w[1 << D]) {
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
    float p = 1.f;
#pragma unroll
    for (int a = 0; a < D; ++a) p *= ((o >> a) & 1) ? L.f[a] : 1.f - L.f[a];
    w[o] = p;
  }
}

// Derivatives of the corner weights with respect to the physical position.
template <int D>
__device__ __forceinline__ void corner_dweights(const Loc<D>& L, const float inv_h[3], float dw[1 << D][D]) {
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float p = ((o >> a) & 1) ? inv_h[a] : -inv_h[a];
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (b != a) p *= ((o >> b) & 1) ? L.f[b] : 1.f - L.f[b];
      dw[o][a] = p;
    }
  }
}

// Flat index (x fastest) of corner o of the cell at L on a grid of size m.
template <int D>
__device__ __forceinline__ long long corner_index(const Loc<D>& L, const int m[3], int o) {
  long long idx = 0, stride = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int c = wrapi(L.c[a] + ((o >> a) & 1), m[a]);
    idx += (long long)c * stride;
    stride *= m[a];
  }
  return idx;
}

}  // namespace lag
