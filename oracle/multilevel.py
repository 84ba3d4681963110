"""Multilevel continuation (oracle; test infrastructure only).

Sec. 3.2, last paragraph: the problem is first solved with a coarse
discretisation of distance, regulariser and velocity; the solution is then
refined and used as the starting guess on the next finer level, up to the
finest level.

Readings:

* Level l halves every grid of level l+1 along every axis (sizes must be
  even); images are restricted by averaging the 2^d fine cells of a coarse
  cell (the midpoint-rule integral of the fine image over the coarse cell);
* the velocity is refined by cell-centred (bi/tri)linear interpolation on
  the periodic coarse grid, per component and time node: a fine centre lies
  a quarter coarse cell from the nearest coarse centre, so the weights along
  each axis are 3/4 and 1/4;
* every level uses the same N, alpha, gamma and time nodes; each level's
  Gauss-Newton solve uses that level's own |g(v = 0)| as the reference.
"""

from __future__ import annotations

from dataclasses import replace

import numpy as np

from .gn import gn_solve
from .grid import Problem


def coarsen_problem(prob: Problem) -> Problem:
    for a in range(prob.dim):
        if prob.img_m[a] % 2 or prob.vel_m[a] % 2:
            raise ValueError("multilevel needs even grid sizes on every level")
    img = tuple(m // 2 for m in prob.img_m[: prob.dim]) + tuple(prob.img_m[prob.dim:])
    vel = tuple(m // 2 for m in prob.vel_m[: prob.dim]) + tuple(prob.vel_m[prob.dim:])
    return replace(prob, img_m=img, vel_m=vel)


def restrict_image(prob: Problem, f):
    """Average of the 2^d fine cells of each coarse cell (prob = fine level)."""
    f = np.asarray(f, dtype=np.float64).reshape(prob.img_shape)
    if prob.dim == 2:
        return 0.25 * (f[0::2, 0::2] + f[0::2, 1::2] + f[1::2, 0::2] + f[1::2, 1::2])
    out = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out = out + f[dz::2, dy::2, dx::2]
    return out / 8.0


def cell_average_matrix(fine_m, coarse_m):
    """Dense (coarse_m, fine_m) matrix of the cell average along one axis:
    entry (I, i) = |fine cell i  intersect  coarse cell I| / |coarse cell I|
    on [0, 1) with fine cells of width 1/fine_m and coarse cells 1/coarse_m."""
    W = np.zeros((coarse_m, fine_m))
    for I in range(coarse_m):
        a, b = I / coarse_m, (I + 1) / coarse_m
        for i in range(fine_m):
            lo, hi = max(a, i / fine_m), min(b, (i + 1) / fine_m)
            if hi > lo:
                W[I, i] = (hi - lo) * coarse_m
    return W


def resample_to_velocity_grid(prob: Problem, f):
    """Average of the piecewise-constant image over each velocity cell (any
    ratio img_m / vel_m >= 1): the per-axis cell-average matrices applied
    along every axis of the image array."""
    f = np.asarray(f, dtype=np.float64).reshape(prob.img_shape)
    out = f
    for a in range(prob.dim):
        W = cell_average_matrix(prob.img_m[a], prob.vel_m[a])
        axis = prob.dim - 1 - a          # storage order is reversed (x last)
        out = np.moveaxis(np.tensordot(W, out, axes=([1], [axis])), 0, axis)
    return out


def _prolong_axis(c, axis):
    """Cell-centred linear refinement of a periodic array along one axis."""
    left = np.roll(c, 1, axis=axis)    # c[i-1]
    right = np.roll(c, -1, axis=axis)  # c[i+1]
    even = 0.75 * c + 0.25 * left      # fine cell 2i   at coarse coordinate i - 1/4
    odd = 0.75 * c + 0.25 * right      # fine cell 2i+1 at coarse coordinate i + 1/4
    shape = list(c.shape)
    shape[axis] *= 2
    out = np.empty(shape)
    idx_e = [slice(None)] * c.ndim
    idx_o = [slice(None)] * c.ndim
    idx_e[axis] = slice(0, None, 2)
    idx_o[axis] = slice(1, None, 2)
    out[tuple(idx_e)] = even
    out[tuple(idx_o)] = odd
    return out


def prolong_velocity(coarse: Problem, v):
    """Refine a coarse velocity (coarse-level shape) to the next finer grid."""
    v = np.asarray(v, dtype=np.float64).reshape(coarse.vel_shape)
    out = v
    for a in range(coarse.dim):
        out = _prolong_axis(out, axis=2 + coarse.dim - 1 - a)
    return out


def multilevel_solve(prob: Problem, T, R, levels, **gn_kw):
    """Coarse-to-fine Gauss-Newton; returns (v on the finest grid, per-level histories)."""
    probs = [prob]
    Ts = [np.asarray(T, dtype=np.float64).ravel()]
    Rs = [np.asarray(R, dtype=np.float64).ravel()]
    for _ in range(levels - 1):
        Ts.append(restrict_image(probs[-1], Ts[-1]).ravel())
        Rs.append(restrict_image(probs[-1], Rs[-1]).ravel())
        probs.append(coarsen_problem(probs[-1]))
    v = None
    hists = []
    for lev in range(levels - 1, -1, -1):
        P = probs[lev]
        v0 = None if v is None else prolong_velocity(probs[lev + 1], v)
        v, h = gn_solve(P, Ts[lev], Rs[lev], v0=v0, **gn_kw)
        hists.append(h)
    return v, hists
