"""Grids and interpolation for the oracle (test infrastructure only).

Discretisation (Sec. 3, first paragraphs): the domain is divided into a
regular mesh of cells, integrals use the midpoint rule at cell centres, the
velocity lives at cell centres in space and at the nodes of a regular time
grid with n_t cells, so there are n = (n_t + 1) d m^d unknowns.  The velocity
grid may differ from the image grid.

Readings taken here:

* Boundary: periodic box [0, L)^d for images and velocities (the paper pads
  its velocity domain instead); this is what makes the FFT preconditioner
  exact.
* Interpolation I(v, y, t) (Sec. 3.1, text after eq. forwardEuler): bi/tri-
  linear in space and linear in time, per velocity component.  Time nodes sit
  at t_j = j/n_t; a time t uses nodes j0 = min(floor(t n_t), n_t - 1) and
  j0 + 1 with weights (1 - theta, theta), theta = t n_t - j0.
* Positions are carried as (start cell index, displacement phi).  The
  fractional cell coordinate of a point on a grid with m_G cells per axis is
  s_a = (i_a + 1/2) m_G,a / m_img,a - 1/2 + phi_a m_G,a / L_a; its cell is
  c = floor(s) and its in-cell offset f = s - c (so exactly on a grid line the
  right-hand cell is chosen, and one-sided derivatives are taken there).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Problem:
    """One registration problem on periodic cell-centred grids (x first)."""
    dim: int
    img_m: tuple
    vel_m: tuple
    nodes: int = 1                 # 1 = stationary; else n_t + 1 time nodes
    model: str = "transport"       # "transport" (eq. transport) | "continuity"
    reg: str = "diffusion"         # "diffusion" (H1) | "curvature" (H2)
    nsteps: int = 5                # N, RK4 steps over the unit time interval
    alpha: float = 1e-2
    gamma: float = 0.0
    extent: tuple = field(default=(1.0, 1.0, 1.0))

    @property
    def d(self):
        return self.dim

    @property
    def n_points(self):
        return int(np.prod(self.img_m[: self.dim]))

    @property
    def n_vel(self):
        return int(np.prod(self.vel_m[: self.dim]))

    @property
    def n_unknowns(self):
        # n = (n_t + 1) * d * m^d  (Sec. 3)
        return self.nodes * self.dim * self.n_vel

    @property
    def h_img(self):
        return np.array([self.extent[a] / self.img_m[a] for a in range(self.dim)])

    @property
    def h_vel(self):
        return np.array([self.extent[a] / self.vel_m[a] for a in range(self.dim)])

    @property
    def cell_img(self):
        """h^d of the image grid (midpoint-rule cell volume)."""
        return float(np.prod(self.h_img))

    @property
    def cell_vel(self):
        return float(np.prod(self.h_vel))

    @property
    def vel_shape(self):
        return (self.nodes, self.dim) + tuple(reversed(self.vel_m[: self.dim]))

    @property
    def img_shape(self):
        return tuple(reversed(self.img_m[: self.dim]))


def start_indices(prob, points=None):
    """Integer image-cell multi-indices (x first), shape (d, n), of flat ids."""
    if points is None:
        points = np.arange(prob.n_points)
    points = np.asarray(points, dtype=np.int64)
    idx = np.empty((prob.dim, points.size), dtype=np.int64)
    rem = points.copy()
    for a in range(prob.dim):
        idx[a] = rem % prob.img_m[a]
        rem //= prob.img_m[a]
    return idx


def grid_coords(prob, grid_m, idx, phi):
    """Fractional cell coordinates s (d, n) on a grid with grid_m cells/axis."""
    s = np.empty(phi.shape, dtype=np.float64)
    for a in range(prob.dim):
        ratio = grid_m[a] / prob.img_m[a]
        s[a] = (idx[a] + 0.5) * ratio - 0.5 + phi[a] * (grid_m[a] / prob.extent[a])
    return s


def grid_margin(s):
    """Distance (in cells) from each point to the nearest grid line, min over axes."""
    f = s - np.floor(s)
    return np.min(np.minimum(f, 1.0 - f), axis=0)


def _corner(code, dim):
    return [(code >> a) & 1 for a in range(dim)]


def _flat(grid_m, cells):
    """Flat x-fastest index of integer cell multi-indices, wrapped periodically."""
    flat = np.zeros(cells.shape[1], dtype=np.int64)
    stride = 1
    for a in range(len(cells)):
        flat += np.mod(cells[a], grid_m[a]) * stride
        stride *= grid_m[a]
    return flat


def corner_stencil(grid_m, h, s):
    """Linear-interpolation stencil at fractional coordinates s (d, n).

    Returns a list over the 2^d corners of (flat index, weight, dweight) where
    dweight[a] is the derivative of the weight with respect to the physical
    coordinate y_a (one-sided on grid lines, per the floor rule).
    """
    dim = s.shape[0]
    c = np.floor(s).astype(np.int64)
    f = s - c
    out = []
    for code in range(1 << dim):
        o = _corner(code, dim)
        fac = [f[a] if o[a] else 1.0 - f[a] for a in range(dim)]
        dfac = [(1.0 if o[a] else -1.0) / h[a] for a in range(dim)]
        w = np.ones(s.shape[1])
        for a in range(dim):
            w = w * fac[a]
        dw = np.empty(s.shape)
        for a in range(dim):
            g = np.full(s.shape[1], dfac[a])
            for b in range(dim):
                if b != a:
                    g = g * fac[b]
            dw[a] = g
        cells = c + np.array(o, dtype=np.int64)[:, None]
        out.append((_flat(grid_m, cells), w, dw))
    return out


def interp(field, stencil):
    """Interpolate fields (ncomp, ngrid) with a stencil -> (ncomp, n)."""
    val = 0.0
    for flat, w, _ in stencil:
        val = val + w * field[:, flat]
    return val


def interp_grad(field, stencil):
    """Spatial gradient of the interpolant: (ncomp, d, n)."""
    g = 0.0
    for flat, _, dw in stencil:
        g = g + field[:, None, flat] * dw[None, :, :]
    return g


def scatter(out, stencil, values):
    """Adjoint of ``interp``: out (ncomp, ngrid) += sum_corners w * values."""
    for flat, w, _ in stencil:
        for c in range(values.shape[0]):
            np.add.at(out[c], flat, w * values[c])


def node_weights(prob):
    """Time-quadrature weights w_j of the velocity nodes (regulariser).

    Reading of the factor written as Delta t in the regulariser derivative
    (Sec. 3.2): the time integral of the regulariser is approximated by the
    trapezoidal rule over the nodes, w = (1/(2 n_t), 1/n_t, ..., 1/(2 n_t));
    a stationary velocity has the single weight 1.
    """
    if prob.nodes == 1:
        return np.ones(1)
    nt = prob.nodes - 1
    w = np.full(prob.nodes, 1.0 / nt)
    w[0] = w[-1] = 0.5 / nt
    return w


def time_weights(prob, t):
    """Nodes and weights of the linear-in-time interpolation at time t."""
    if prob.nodes == 1:
        return [(0, 1.0)]
    nt = prob.nodes - 1
    j0 = min(int(np.floor(t * nt)), nt - 1)
    theta = t * nt - j0
    return [(j0, 1.0 - theta), (j0 + 1, theta)]
