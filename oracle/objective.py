"""Objective, gradient and Gauss-Newton Hessian (oracle; test infrastructure).

Sec. 3.2 of the paper: J(v) = D(u1(v), R) + alpha S(v) with the midpoint-rule
SSD distance D = h^d/2 |res|^2, res = u1 - R (eq. SSD), gradient
d_v J = (d_v u1)^T h^d res + alpha d_v S, and the Gauss-Newton approximation
H = (d_v u1)^T (h^d I) (d_v u1) + alpha (quadrature) h^d B^T B + gamma I.

Regularisers (Sec. 2.1): diffusion S = 1/2 int sum_k |grad v^k|^2 and
curvature S = 1/2 int sum_k |Laplace v^k|^2, i.e. B^T B = -Laplace_h or
(Laplace_h)^2 with the periodic (2d+1)-point Laplacian.

Readings:

* h^d in the data term is the image cell volume; in the regulariser it is the
  velocity cell volume (the two grids may differ).
* The factor written as Delta t in the regulariser terms is the time
  quadrature weight of each velocity node (trapezoidal rule; weight 1 for a
  stationary velocity).
* gamma I is added to the Hessian as printed, unscaled.
* An optional voxel weight W (default 1) multiplies the data term of the
  Hessian: H = h^d J^T W J + ...; it is used to mask characteristics.
"""

from __future__ import annotations

import numpy as np

from .grid import node_weights
from .lagrangian import trace, transport, pushforward, jvp, vjp


def laplacian_apply(prob, f):
    """-Laplace_h f on the periodic velocity grid, for one scalar field."""
    f = np.asarray(f, dtype=np.float64).reshape(tuple(reversed(prob.vel_m[: prob.dim])))
    h = prob.h_vel
    out = np.zeros_like(f)
    for a in range(prob.dim):
        ax = prob.dim - 1 - a          # storage axis of coordinate a
        out += (2.0 * f - np.roll(f, 1, axis=ax) - np.roll(f, -1, axis=ax)) / (h[a] * h[a])
    return out


def _A(prob, f):
    if prob.reg == "diffusion":
        return laplacian_apply(prob, f)
    return laplacian_apply(prob, laplacian_apply(prob, f))


def regularizer_apply(prob, p):
    """alpha * h_v^d * w_j * A p_{j,c} for every node j and component c."""
    p = np.asarray(p, dtype=np.float64).reshape(prob.vel_shape)
    w = node_weights(prob)
    out = np.empty_like(p)
    for j in range(prob.nodes):
        for c in range(prob.dim):
            out[j, c] = prob.alpha * prob.cell_vel * w[j] * _A(prob, p[j, c])
    return out


def regularizer_energy(prob, v):
    """S(v) = 1/2 sum_j w_j h_v^d sum_c <v_jc, A v_jc> (without alpha)."""
    v = np.asarray(v, dtype=np.float64).reshape(prob.vel_shape)
    w = node_weights(prob)
    s = 0.0
    for j in range(prob.nodes):
        for c in range(prob.dim):
            s += 0.5 * w[j] * prob.cell_vel * float(np.sum(v[j, c] * _A(prob, v[j, c])))
    return s


def ssd(prob, u, R):
    """D = h^d / 2 * res^T res with res = u - R (eq. SSD)."""
    res = np.asarray(u, dtype=np.float64).reshape(-1) - np.asarray(R, dtype=np.float64).reshape(-1)
    return 0.5 * prob.cell_img * float(res @ res), res


def final_state(prob, v, T):
    """u1(v): transport (eq. rhoEndIR) or push-forward (eq. rhoEndOMT)."""
    phi = trace(prob, v)
    if prob.model == "transport":
        return transport(prob, T, phi)
    return pushforward(prob, T, phi)


def objective(prob, v, T, R):
    """Returns dict(J, D, S, u, res) with J = D + alpha S (eq. discOpti)."""
    u = final_state(prob, v, T)
    D, res = ssd(prob, u, R)
    S = regularizer_energy(prob, v)
    return {"J": D + prob.alpha * S, "D": D, "S": S, "u": u, "res": res}


def gradient(prob, v, T, R):
    """d_v J = (d_v u1)^T h^d res + alpha d_v S; also returns the objective."""
    obj = objective(prob, v, T, R)
    g = vjp(prob, v, T, prob.cell_img * obj["res"]) + regularizer_apply(prob, v)
    return g, obj


def hessmat(prob, v, T, p, wvox=None, points=None):
    """Gauss-Newton matvec H p = h^d J^T (W (J p)) + alpha h_v^d w_j A p + gamma p.

    ``points`` restricts the data term to a subset of characteristics
    (transport) or particles (continuity); ``wvox`` is W on those
    characteristics (transport) or on the image grid (continuity).
    """
    Jp = jvp(prob, v, T, p, points=points)
    if wvox is not None:
        Jp = Jp * np.asarray(wvox, dtype=np.float64).reshape(-1)
    Hp = prob.cell_img * vjp(prob, v, T, Jp, points=points)
    Hp = Hp + regularizer_apply(prob, p)
    return Hp + prob.gamma * np.asarray(p, dtype=np.float64).reshape(prob.vel_shape)
