"""Lagrangian solver and its derivatives (oracle; test infrastructure only).

Follows Sec. 3.1 and Algorithm 1 of the paper:

* characteristics are integrated by RK4 with N equal steps of size +-1/N
  (forward from t = 0 for the continuity equation, backward from t = 1 for
  the transport equation);
* the transport solve is one interpolation of the template at the end points
  of the backward characteristics (eq. rhoEndIR);
* the continuity solve is the particle-in-cell push-forward (eq. rhoEndOMT)
  with hat width equal to the cell size, i.e. the transpose of linear
  interpolation at the forward end points (the special case the paper states
  right after eq. ukOMT, and the one its experiments use);
* RK4 is written as an explicit Runge-Kutta method given by its Butcher
  tableau (stage offsets A, weights B, nodes C); the Jacobian-vector product
  is the tangent-linear map of that discrete scheme (Sec. 3.2: the derivative
  of the final state is obtained by differentiating the RK4 recursion), and
  the vector-Jacobian product is the exact reverse-mode adjoint of the same
  map (this oracle keeps the whole trajectory in memory for it; the memory-
  lean recursion of the paper is what the GPU path implements).

Readings:

* Algorithm 1 as printed puts the fourth RK4 stage at y + (dt/2) v3 while its
  derivative line uses the full step; the classical RK4 stage y + dt v3 is
  used (the printed variant is only first-order accurate).
* Positions are stored as displacements from the start cell centre.
* The transport end point is y(v, x_c, 1, 0) and the continuity end point is
  y(v, x_c, 0, 1).
"""

from __future__ import annotations

import numpy as np

from .grid import (start_indices, grid_coords, grid_margin, corner_stencil,
                   interp, interp_grad, scatter, time_weights)


def _direction(prob):
    # transport: backward characteristics; continuity: forward (Sec. 3.1)
    return -1 if prob.model == "transport" else +1


# Classical fourth-order Runge-Kutta method as a Butcher tableau: stage i is
# evaluated at phi + dt * sum_j A[i][j] k_j and time t + C[i] dt; the step adds
# dt * sum_i B[i] k_i.  (Algorithm 1 prints the last stage point with dt/2;
# the classical full step dt is used, see the module readings.)
RK4_A = ((), (0.5,), (0.0, 0.5), (0.0, 0.0, 1.0))
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
RK4_C = (0.0, 0.5, 0.5, 1.0)


def _stage_point(phi, dt, row, ks):
    """phi + dt * sum_j row[j] ks[j] (the stage offsets of one tableau row)."""
    out = phi
    for a, k in zip(row, ks):
        if a != 0.0:
            out = out + (dt * a) * k
    return out


class _GridVelocity:
    """I(v, y, t) and its derivatives for points given as (start idx, phi)."""

    def __init__(self, prob, v, idx):
        self.prob = prob
        self.v = np.asarray(v, dtype=np.float64).reshape(prob.nodes, prob.dim, prob.n_vel)
        self.idx = idx
        self.margin = np.full(idx.shape[1], np.inf)

    def stencil(self, phi, track=True):
        s = grid_coords(self.prob, self.prob.vel_m, self.idx, phi)
        if track:
            self.margin = np.minimum(self.margin, grid_margin(s))
        return corner_stencil(self.prob.vel_m, self.prob.h_vel, s)

    def sample(self, phi, t, grad=False, dv=None, track=True):
        """Velocity (and optionally its spatial gradient and the sample of a
        direction dv) at the points.  ``track`` records the distance to the
        nearest grid line; the very first sample sits at the fixed start
        point, which does not depend on v, and is not tracked."""
        st = self.stencil(phi, track)
        val, g, dval = 0.0, 0.0, 0.0
        for j, wt in time_weights(self.prob, t):
            val = val + wt * interp(self.v[j], st)
            if grad:
                g = g + wt * interp_grad(self.v[j], st)
            if dv is not None:
                dval = dval + wt * interp(dv[j], st)
        return val, (g if grad else None), (dval if dv is not None else None)

    def scatter(self, out, phi, t, lam):
        """out (nodes, d, n_vel) += d_v I(v, y, t)^T lam."""
        st = corner_stencil(self.prob.vel_m, self.prob.h_vel,
                            grid_coords(self.prob, self.prob.vel_m, self.idx, phi))
        for j, wt in time_weights(self.prob, t):
            scatter(out[j], st, wt * lam)


def _matvec(g, x):
    """(comp, axis, n) times (axis, n) -> (comp, n)."""
    return np.einsum("can,an->cn", g, x)


def _matTvec(g, x):
    """(comp, axis, n)^T times (comp, n) -> (axis, n)."""
    return np.einsum("can,cn->an", g, x)


def rk4_characteristics(sample, phi0, direction, nsteps, keep_path=False):
    """RK4 for dy/dt = v(y, t) on [0, 1] (Algorithm 1 without the derivative).

    ``sample(phi, t)`` returns the velocity at the current points.  Returns
    the final displacement and, optionally, the list of states phi_k.
    """
    dt = direction / nsteps
    t0 = 0.0 if direction > 0 else 1.0
    phi = phi0.copy()
    path = [phi.copy()] if keep_path else None
    for k in range(nsteps):
        tk = t0 + k * dt
        ks = []
        for row, c in zip(RK4_A, RK4_C):
            ks.append(sample(_stage_point(phi, dt, row, ks), tk + c * dt))
        phi = _stage_point(phi, dt, RK4_B, ks)
        if keep_path:
            path.append(phi.copy())
    return phi, path


def trace_analytic(velocity, y0, direction, nsteps):
    """RK4 characteristics of an analytic velocity ``velocity(y, t)``.

    Runs the same RK4 routine as ``trace`` (with absolute positions), so the
    order of the scheme can be checked against exact ODE solutions.
    """
    y0 = np.asarray(y0, dtype=np.float64)
    phi, _ = rk4_characteristics(lambda phi, t: velocity(y0 + phi, t),
                                 np.zeros_like(y0), direction, nsteps)
    return y0 + phi


def trace(prob, v, direction=None, points=None, return_margin=False, phi0=None):
    """End-point displacements phi (d, n) of the characteristics.

    direction -1 gives y(v, x_c, 1, 0), +1 gives y(v, x_c, 0, 1) (Sec. 3.1).
    ``phi0`` optionally moves the start points off the cell centres (start at
    x_c + phi0); the result is still measured from x_c.
    """
    direction = _direction(prob) if direction is None else direction
    idx = start_indices(prob, points)
    vel = _GridVelocity(prob, v, idx)
    start = np.zeros((prob.dim, idx.shape[1])) if phi0 is None else np.array(phi0, dtype=np.float64)
    first = [phi0 is None]

    def sample(p, t):
        track = not first[0]
        first[0] = False
        return vel.sample(p, t, track=track)[0]
    phi, _ = rk4_characteristics(sample, start, direction, prob.nsteps)
    if return_margin:
        return phi, vel.margin
    return phi


def _image_stencil(prob, idx, phi):
    s = grid_coords(prob, prob.img_m, idx, phi)
    return corner_stencil(prob.img_m, prob.h_img, s), grid_margin(s)


def transport(prob, T, phi, points=None):
    """u1(x_c) = T(y(v, x_c, 1, 0)) by linear interpolation (eq. rhoEndIR)."""
    idx = start_indices(prob, points)
    st, _ = _image_stencil(prob, idx, phi)
    return interp(np.asarray(T, dtype=np.float64).reshape(1, -1), st)[0]


def pushforward(prob, T, phi, points=None):
    """u1 = F(y(v, x_c, 0, 1)) T(x_c) with F the transpose of linear
    interpolation (eq. rhoEndOMT, hat width = cell size).

    Particles sit at the image cell centres listed in ``points`` (all by
    default) and carry mass T(x_j); the result is a full image.
    """
    idx = start_indices(prob, points)
    Tf = np.asarray(T, dtype=np.float64).reshape(-1)
    mass = Tf if points is None else Tf[np.asarray(points)]
    st, _ = _image_stencil(prob, idx, phi)
    u = np.zeros((1, prob.n_points))
    scatter(u, st, mass[None, :])
    return u[0]


def _tangent(prob, vel, dv, direction):
    """Tangent-linear RK4 map: the derivative of the discrete characteristic
    along the velocity direction dv (Sec. 3.2, the derivative recursion that
    accompanies Algorithm 1).

    Differentiating a stage k_i = V(P_i, t_i) with P_i = phi + dt sum_j
    A_ij k_j gives dk_i = V(dv; P_i, t_i) + grad_y V(P_i, t_i) dP_i with
    dP_i = dphi + dt sum_j A_ij dk_j; the step gives dphi + dt sum_i B_i dk_i.
    Returns (phi_N, dphi_N) where dphi_N = (d_v y) dv.
    """
    n = vel.idx.shape[1]
    dt = direction / prob.nsteps
    t0 = 0.0 if direction > 0 else 1.0
    phi = np.zeros((prob.dim, n))
    dphi = np.zeros((prob.dim, n))
    for k in range(prob.nsteps):
        tk = t0 + k * dt
        ks, dks = [], []
        for i, (row, c) in enumerate(zip(RK4_A, RK4_C)):
            P = _stage_point(phi, dt, row, ks)
            dP = _stage_point(dphi, dt, row, dks)
            # the first sample of the first step sits at the fixed start point
            val, grad, dval = vel.sample(P, tk + c * dt, grad=True, dv=dv,
                                         track=not (k == 0 and i == 0))
            ks.append(val)
            dks.append(dval + _matvec(grad, dP))
        phi = _stage_point(phi, dt, RK4_B, ks)
        dphi = _stage_point(dphi, dt, RK4_B, dks)
    return phi, dphi


def jvp(prob, v, T, dv, points=None, return_margin=False):
    """(d_v u1) dv (Sec. 3.2, derivative of the final state).

    transport:  grad T(y) . (d_v y) dv per characteristic (shape (n,));
    continuity: sum_j T_j grad_y F(y_j) . (d_v y_j) dv, a full image.
    ``return_margin`` also returns each characteristic's smallest distance
    (in cells) to a grid line over every velocity sample and the final
    interpolation, which locates the kinks of the piecewise-linear model.
    """
    idx = start_indices(prob, points)
    vel = _GridVelocity(prob, v, idx)
    dvf = np.asarray(dv, dtype=np.float64).reshape(prob.nodes, prob.dim, prob.n_vel)
    phi, dphi = _tangent(prob, vel, dvf, _direction(prob))
    st, m_img = _image_stencil(prob, idx, phi)
    Tf = np.asarray(T, dtype=np.float64).reshape(-1)
    if prob.model == "transport":
        gT = interp_grad(Tf[None, :], st)[0]          # (d, n)
        out = np.sum(gT * dphi, axis=0)
    else:
        mass = Tf if points is None else Tf[np.asarray(points)]
        out = np.zeros(prob.n_points)
        for flat, _, dw in st:
            np.add.at(out, flat, mass * np.sum(dw * dphi, axis=0))
    if return_margin:
        return out, np.minimum(vel.margin, m_img)
    return out


def vjp(prob, v, T, w, points=None):
    """(d_v u1)^T w, the adjoint of ``jvp`` (used by the gradient, Sec. 3.2).

    transport: w holds one weight per listed characteristic;
    continuity: w is a full image and the listed points are the particles.
    Returns an array shaped like v.
    """
    idx = start_indices(prob, points)
    vel = _GridVelocity(prob, v, idx)
    direction = _direction(prob)
    phiN, path = rk4_characteristics(lambda p, t: vel.sample(p, t)[0],
                                     np.zeros((prob.dim, idx.shape[1])), direction,
                                     prob.nsteps, keep_path=True)
    st, _ = _image_stencil(prob, idx, phiN)
    Tf = np.asarray(T, dtype=np.float64).reshape(-1)
    wf = np.asarray(w, dtype=np.float64).reshape(-1)
    if prob.model == "transport":
        ybar = wf[None, :] * interp_grad(Tf[None, :], st)[0]
    else:
        mass = Tf if points is None else Tf[np.asarray(points)]
        ybar = mass[None, :] * interp_grad(wf[None, :], st)[0]

    out = np.zeros((prob.nodes, prob.dim, prob.n_vel))
    dt = direction / prob.nsteps
    t0 = 0.0 if direction > 0 else 1.0
    ns = len(RK4_B)
    for k in range(prob.nsteps - 1, -1, -1):
        phi = path[k]
        tk = t0 + k * dt
        # recompute the stage points, velocities and gradients of step k
        P, ks, gs = [], [], []
        for row, c in zip(RK4_A, RK4_C):
            P.append(_stage_point(phi, dt, row, ks))
            val, grad, _ = vel.sample(P[-1], tk + c * dt, grad=True)
            ks.append(val)
            gs.append(grad)
        # adjoint of phi_{k+1} = phi_k + dt sum_i B_i k_i, stages in reverse:
        # kbar_i collects dt B_i ybar and dt A_ji Pbar_j from later stages j;
        # Pbar_i = grad_y V(P_i)^T kbar_i feeds phibar and the earlier stages,
        # and kbar_i itself is scattered onto the velocity grid at P_i.
        kbar = [(dt * b) * ybar for b in RK4_B]
        phib = ybar.copy()
        for i in range(ns - 1, -1, -1):
            vel.scatter(out, P[i], tk + RK4_C[i] * dt, kbar[i])
            pb = _matTvec(gs[i], kbar[i])
            phib = phib + pb
            for j, a in enumerate(RK4_A[i]):
                if a != 0.0:
                    kbar[j] = kbar[j] + (dt * a) * pb
        ybar = phib
    return out.reshape(prob.vel_shape)
