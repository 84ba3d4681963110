"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an invariant, brute force, a library routine, or a number the
paper prints.  They run on the CPU.
"""

import os

import numpy as np
import pytest

import oracle as O
from synthetic import blob_image, fourier_velocity, random_direction

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def prob2(m=(12, 10), vm=None, **kw):
    vm = m if vm is None else vm
    base = dict(dim=2, img_m=m, vel_m=vm, nodes=1, model="transport", reg="diffusion",
                nsteps=4, alpha=1e-2, gamma=0.0)
    base.update(kw)
    return O.Problem(**base)


def prob3(m=(6, 5, 4), vm=None, **kw):
    vm = m if vm is None else vm
    base = dict(dim=3, img_m=m, vel_m=vm, nodes=1, model="transport", reg="diffusion",
                nsteps=3, alpha=1e-2, gamma=0.0)
    base.update(kw)
    return O.Problem(**base)


def const_velocity(P, c):
    v = np.zeros(P.vel_shape)
    for a in range(P.dim):
        v[:, a] = c[a]
    return v


# --------------------------------------------------------------------- P0
def test_unknown_counts_match_paper():
    """n = (n_t+1) d m^d against the unknown counts the paper prints."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "unknown_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        dim, mx, my, mz, nodes, n, tol = (int(x) for x in r[:7])
        P = O.Problem(dim=dim, img_m=(mx, my, mz), vel_m=(mx, my, mz), nodes=nodes)
        assert abs(P.n_unknowns - n) <= tol, r


# --------------------------------------------------------------------- P1
@pytest.mark.parametrize("model", ["transport", "continuity"])
def test_constant_velocity_integer_shift(model):
    """Constant v = k h translates by whole cells: transport and push-forward
    reduce to np.roll, and phi = -+c exactly (RK4 is exact for constant v)."""
    P = prob2(m=(12, 10), model=model, nsteps=3)
    h = P.h_img
    c = np.array([3 * h[0], -2 * h[1]])
    v = const_velocity(P, c)
    T = blob_image(P.img_m, 3, 7).ravel()
    sign = -1 if model == "transport" else 1
    phi = O.trace(P, v)
    np.testing.assert_allclose(phi, sign * c[:, None] * np.ones((1, P.n_points)), atol=1e-14)
    Ti = T.reshape(P.img_shape)
    if model == "transport":
        u = O.transport(P, T, phi).reshape(P.img_shape)
        # u(x) = T(x - c)  -> roll by +k along each axis
        ref = np.roll(np.roll(Ti, 3, axis=1), -2, axis=0)
    else:
        u = O.pushforward(P, T, phi).reshape(P.img_shape)
        ref = np.roll(np.roll(Ti, 3, axis=1), -2, axis=0)
    np.testing.assert_allclose(u, ref, atol=1e-13)


@pytest.mark.parametrize("model", ["transport", "continuity"])
def test_constant_velocity_fractional_shift(model):
    """A fractional shift (k + f) h along x gives (1-f) roll(k) + f roll(k+1)."""
    P = prob2(m=(9, 7), model=model, nsteps=2)
    f = 0.3
    c = np.array([(2 + f) * P.h_img[0], 0.0])
    v = const_velocity(P, c)
    T = blob_image(P.img_m, 2, 3).ravel()
    Ti = T.reshape(P.img_shape)
    phi = O.trace(P, v)
    if model == "transport":
        u = O.transport(P, T, phi).reshape(P.img_shape)
        # T(x_i - (2+f)h) = (1-f) T[i-2] + f T[i-3]
        ref = (1 - f) * np.roll(Ti, 2, axis=1) + f * np.roll(Ti, 3, axis=1)
    else:
        u = O.pushforward(P, T, phi).reshape(P.img_shape)
        # particle j lands at x_j + (2+f)h: cell j+2 gets 1-f, cell j+3 gets f
        ref = (1 - f) * np.roll(Ti, 2, axis=1) + f * np.roll(Ti, 3, axis=1)
    np.testing.assert_allclose(u, ref, atol=1e-13)


def test_constant_velocity_3d_and_coarse_velocity_grid():
    """Constant v on a coarser velocity grid (ratio 1/2) still translates exactly."""
    P = prob3(m=(8, 6, 4), vm=(4, 3, 2), nsteps=2)
    h = P.h_img
    c = np.array([h[0], 2 * h[1], -h[2]])
    v = const_velocity(P, c)
    T = blob_image(P.img_m, 3, 11).ravel()
    u = O.transport(P, T, O.trace(P, v)).reshape(P.img_shape)
    ref = np.roll(np.roll(np.roll(T.reshape(P.img_shape), 1, axis=2), 2, axis=1), -1, axis=0)
    np.testing.assert_allclose(u, ref, atol=1e-13)


# --------------------------------------------------------------------- P2
def test_constant_image_invariant_under_transport():
    P = prob2(m=(10, 8), nsteps=3)
    v = fourier_velocity(P.vel_m, 3, 0.2, 5)
    T = np.full(P.n_points, 2.5)
    u = O.transport(P, T, O.trace(P, v))
    np.testing.assert_allclose(u, 2.5, rtol=0, atol=1e-14)
    dv = random_direction(P.vel_shape, 9)
    np.testing.assert_allclose(O.jvp(P, v, T, dv), 0.0, atol=1e-12)


# --------------------------------------------------------------------- P3
@pytest.mark.parametrize("nodes", [1, 3])
def test_mass_conservation(nodes):
    """Columns of the push-forward sum to one (Sec. 3.1): mass is conserved,
    every J dv has zero total mass, and J^T 1 = 0."""
    P = prob2(m=(12, 10), vm=(6, 5), model="continuity", nodes=nodes, nsteps=4)
    v = fourier_velocity(P.vel_m, 3, 0.15, 21, nodes=nodes)
    T = blob_image(P.img_m, 3, 4, density=True).ravel()
    u = O.pushforward(P, T, O.trace(P, v))
    assert abs(u.sum() - T.sum()) <= 1e-13 * T.sum()
    dv = random_direction(P.vel_shape, 3)
    assert abs(O.jvp(P, v, T, dv).sum()) <= 1e-12 * np.abs(O.jvp(P, v, T, dv)).sum()
    JT1 = O.vjp(P, v, T, np.ones(P.n_points))
    assert np.abs(JT1).max() <= 1e-12


# --------------------------------------------------------------------- P4
@pytest.mark.parametrize("direction", [-1, 1])
def test_nonstationary_spatially_constant_is_trapezoid(direction):
    """Spatially constant, piecewise-linear-in-time v: RK4 is Simpson's rule on
    each step, exact when steps do not straddle nodes, so phi = +-int v dt =
    +-(1/n_t)(c_0/2 + c_1 + ... + c_nt/2)."""
    nodes = 4
    P = prob2(m=(6, 5), nodes=nodes, nsteps=6)
    rng = np.random.default_rng(1)
    cs = rng.uniform(-0.3, 0.3, size=(nodes, 2))
    v = np.zeros(P.vel_shape)
    for j in range(nodes):
        for a in range(2):
            v[j, a] = cs[j, a]
    nt = nodes - 1
    integral = (0.5 * cs[0] + cs[1:-1].sum(axis=0) + 0.5 * cs[-1]) / nt
    phi = O.trace(P, v, direction=direction)
    np.testing.assert_allclose(phi, direction * integral[:, None] * np.ones((1, P.n_points)),
                               atol=1e-14)


# --------------------------------------------------------------------- P5
def test_rk4_fourth_order_rotation():
    """The shared RK4 routine is fourth order on an exact rotation."""
    omega = 2.0

    def vel(y, t):
        return np.stack([-omega * y[1], omega * y[0]])

    y0 = np.array([[0.7], [0.2]])
    exact = np.array([[np.cos(omega) * 0.7 - np.sin(omega) * 0.2],
                      [np.sin(omega) * 0.7 + np.cos(omega) * 0.2]])
    errs = [np.abs(O.trace_analytic(vel, y0, +1, n) - exact).max() for n in (4, 8, 16, 32)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.25), slopes
    # backward direction returns to the start point to RK4 accuracy
    back = O.trace_analytic(vel, exact, -1, 64)
    assert np.abs(back - y0).max() < 1e-7


def test_rk4_fourth_order_time_dependent():
    """y' = t y (exact y0 exp(t^2/2)) checks the stage times."""
    def vel(y, t):
        return t * y
    y0 = np.array([[1.0]])
    errs = [abs(O.trace_analytic(vel, y0, +1, n)[0, 0] - np.exp(0.5)) for n in (4, 8, 16)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.3), slopes


def test_printed_stage_would_fail_order_pin(monkeypatch):
    """Planting the printed fourth-stage point (y + dt/2 v3) in the oracle
    makes the order pin fail: the pin catches that reading error."""
    import oracle.lagrangian as L

    def bad_rk4(sample, phi0, direction, nsteps, keep_path=False):
        dt = direction / nsteps
        t0 = 0.0 if direction > 0 else 1.0
        phi = phi0.copy()
        for k in range(nsteps):
            t = t0 + k * dt
            k1 = sample(phi, t)
            k2 = sample(phi + 0.5 * dt * k1, t + 0.5 * dt)
            k3 = sample(phi + 0.5 * dt * k2, t + 0.5 * dt)
            k4 = sample(phi + 0.5 * dt * k3, t + dt)
            phi = phi + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        return phi, None

    monkeypatch.setattr(L, "rk4_characteristics", bad_rk4)

    def vel(y, t):
        return np.stack([-2.0 * y[1], 2.0 * y[0]])
    y0 = np.array([[0.7], [0.2]])
    exact = np.array([[np.cos(2.0) * 0.7 - np.sin(2.0) * 0.2],
                      [np.sin(2.0) * 0.7 + np.cos(2.0) * 0.2]])
    errs = [np.abs(L.trace_analytic(vel, y0, +1, n) - exact).max() for n in (8, 16, 32)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes < 2.0), slopes


# --------------------------------------------------------------------- P6
def test_pushforward_is_transpose_of_interpolation():
    """F = P^T for hat width h (Sec. 3.1): <F(phi) a, b> = <a, P(phi) b>."""
    P = prob2(m=(11, 9), vm=(6, 5), model="continuity", nodes=2, nsteps=3)
    v = fourier_velocity(P.vel_m, 3, 0.2, 8, nodes=2)
    phi = O.trace(P, v)
    rng = np.random.default_rng(3)
    a = rng.standard_normal(P.n_points)
    b = rng.standard_normal(P.n_points)
    lhs = O.pushforward(P, a, phi) @ b
    rhs = a @ O.transport(P, b, phi)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)


def test_pushforward_columns_brute_force():
    """Each column of F (one particle of unit mass) is the bilinear hat split."""
    P = prob2(m=(5, 4), model="continuity", nsteps=1)
    rng = np.random.default_rng(0)
    phi = rng.uniform(-0.5, 0.5, size=(2, P.n_points)) * P.h_img[:, None] * 3
    for j in [0, 7, 19]:
        e = np.zeros(P.n_points)
        e[j] = 1.0
        col = O.pushforward(P, e, phi).reshape(P.img_shape)
        ix, iy = j % 5, j // 5
        x = (ix + 0.5) * P.h_img[0] + phi[0, j]
        y = (iy + 0.5) * P.h_img[1] + phi[1, j]
        ref = np.zeros(P.img_shape)
        for cy in range(4):
            for cx in range(5):
                # periodic tent distance from cell centre in cells
                dx = ((x / P.h_img[0] - (cx + 0.5)) + 2.5) % 5 - 2.5
                dy = ((y / P.h_img[1] - (cy + 0.5)) + 2.0) % 4 - 2.0
                ref[cy, cx] = max(0.0, 1 - abs(dx)) * max(0.0, 1 - abs(dy))
        np.testing.assert_allclose(col, ref, atol=1e-14)
        assert abs(col.sum() - 1.0) < 1e-14


# --------------------------------------------------------------------- P7
@pytest.mark.parametrize("model,nodes,dim", [("transport", 1, 2), ("transport", 3, 2),
                                             ("continuity", 1, 2), ("continuity", 2, 2),
                                             ("transport", 1, 3), ("continuity", 2, 3)])
def test_dot_test(model, nodes, dim):
    """<q, J p> = <J^T q, p>: the VJP is the adjoint of the JVP."""
    if dim == 2:
        P = prob2(m=(10, 8), vm=(5, 4), model=model, nodes=nodes, nsteps=3)
    else:
        P = prob3(m=(6, 6, 4), vm=(3, 3, 2), model=model, nodes=nodes, nsteps=2)
    v = fourier_velocity(P.vel_m, 2, 0.15, 31, nodes=nodes)
    T = blob_image(P.img_m, 3, 2, density=(model == "continuity")).ravel()
    p = random_direction(P.vel_shape, 5)
    q = random_direction((P.n_points,), 6)
    lhs = q @ O.jvp(P, v, T, p)
    rhs = np.sum(O.vjp(P, v, T, q) * p)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


# --------------------------------------------------------------------- P8
def test_taylor_objective_second_order():
    """J(v + e dv) - J(v) - e g^T dv decays like e^2 (scalar objective)."""
    P = prob2(m=(16, 16), vm=(8, 8), nsteps=3, alpha=1e-3)
    T = blob_image(P.img_m, 4, 12).ravel()
    vt = fourier_velocity(P.vel_m, 3, 0.08, 13)
    R = O.transport(P, T, O.trace(P, vt))
    v = 0.4 * vt
    dv = fourier_velocity(P.vel_m, 3, 0.05, 14)
    g, obj = O.gradient(P, v, T, R)
    J0 = obj["J"]
    eps = np.array([1e-1, 5e-2, 2.5e-2, 1.25e-2])
    rem = np.array([abs(O.objective(P, v + e * dv, T, R)["J"] - J0 - e * np.sum(g * dv))
                    for e in eps])
    slopes = np.log2(rem[:-1] / rem[1:])
    assert np.all(slopes > 1.8), slopes
    # zeroth order remainder decays only linearly
    rem0 = np.array([abs(O.objective(P, v + e * dv, T, R)["J"] - J0) for e in eps])
    assert np.all(np.log2(rem0[:-1] / rem0[1:]) < 1.3)


def test_taylor_state_l1():
    """u1(v + e dv) - u1(v) - e J dv: l1 remainder O(e^2) for the transport state."""
    P = prob2(m=(24, 24), vm=(12, 12), nsteps=3)
    T = blob_image(P.img_m, 5, 15).ravel()
    v = fourier_velocity(P.vel_m, 3, 0.06, 16)
    dv = fourier_velocity(P.vel_m, 3, 0.04, 17)
    u0 = O.transport(P, T, O.trace(P, v))
    Jdv = O.jvp(P, v, T, dv)
    eps = np.array([4e-2, 2e-2, 1e-2])
    rem = np.array([np.abs(O.transport(P, T, O.trace(P, v + e * dv)) - u0 - e * Jdv).sum()
                    for e in eps])
    slopes = np.log2(rem[:-1] / rem[1:])
    assert np.all(slopes > 1.7), slopes


# --------------------------------------------------------------------- P9
@pytest.mark.parametrize("model,nodes", [("transport", 1), ("transport", 2),
                                         ("continuity", 1), ("continuity", 2)])
def test_jvp_matches_finite_differences(model, nodes):
    """Brute force on a tiny grid: central-difference Jacobian columns of
    u1(v) equal the JVP columns (away from kinks of the linear model)."""
    P = prob2(m=(8, 8), vm=(4, 4), model=model, nodes=nodes, nsteps=3)
    v = fourier_velocity(P.vel_m, 2, 0.12, 41, nodes=nodes)
    T = blob_image(P.img_m, 3, 42, density=(model == "continuity")).ravel()

    def u1(vv):
        phi = O.trace(P, vv)
        return O.transport(P, T, phi) if model == "transport" else O.pushforward(P, T, phi)

    _, margin = O.jvp(P, v, T, np.zeros(P.vel_shape), return_margin=True)
    ok = margin > 1e-4
    assert ok.mean() > 0.8
    eps = 1e-7
    n = P.n_unknowns
    worst = 0.0
    for col in range(0, n, 3):
        e = np.zeros(n)
        e[col] = 1.0
        e = e.reshape(P.vel_shape)
        fd = (u1(v + eps * e) - u1(v - eps * e)) / (2 * eps)
        jv = O.jvp(P, v, T, e)
        if model == "transport":
            diff = np.abs(fd - jv)[ok]
            scale = np.abs(jv).max() + 1e-30
        else:
            # a masked particle spreads into 4 cells; compare the full image
            # only when no particle of the problem is near a kink
            if not ok.all():
                continue
            diff = np.abs(fd - jv)
            scale = np.abs(jv).max() + 1e-30
        worst = max(worst, diff.max() / scale)
    assert worst < 1e-6, worst


def test_jvp_continuity_finite_differences_smooth_case():
    """Continuity JVP vs central differences where no particle nears a kink."""
    P2 = prob2(m=(6, 6), vm=(6, 6), model="continuity", nsteps=2)
    rng = np.random.default_rng(5)
    # a constant offset of 0.3 cells plus a small random field keeps every
    # sample after the first, and every end point, away from the grid lines
    vshift = 0.3 * P2.h_img[0] + 0.01 * P2.h_img[0] * rng.standard_normal(P2.vel_shape)
    T = rng.uniform(0.5, 1.5, P2.n_points)
    _, margin = O.jvp(P2, vshift, T, np.zeros(P2.vel_shape), return_margin=True)
    assert margin.min() > 1e-3
    eps = 1e-6

    def u1(vv):
        return O.pushforward(P2, T, O.trace(P2, vv))
    for col in range(P2.n_unknowns):
        e = np.zeros(P2.n_unknowns)
        e[col] = 1
        e = e.reshape(P2.vel_shape)
        fd = (u1(vshift + eps * e) - u1(vshift - eps * e)) / (2 * eps)
        jv = O.jvp(P2, vshift, T, e)
        assert np.abs(jv).max() > 1.0
        assert np.abs(fd - jv).max() <= 1e-7 * np.abs(jv).max()


# --------------------------------------------------------------------- P10
@pytest.mark.parametrize("model,gamma", [("transport", 0.0), ("transport", 1e-3),
                                         ("continuity", 1e-3)])
def test_dense_hessian(model, gamma):
    """H from n matvecs is symmetric, PSD (eigenvalues >= gamma) and equals
    h^d J^T W J + reg with J assembled once from JVP columns and once from
    VJP rows."""
    P = prob2(m=(6, 6), vm=(3, 3), model=model, nodes=2, nsteps=2, gamma=gamma,
              reg="curvature" if model == "continuity" else "diffusion")
    v = fourier_velocity(P.vel_m, 1, 0.1, 51, nodes=2)
    T = blob_image(P.img_m, 2, 52, density=(model == "continuity")).ravel()
    W = np.random.default_rng(2).uniform(0.5, 1.5, P.n_points)
    n = P.n_unknowns
    E = np.eye(n)
    H = np.stack([O.hessmat(P, v, T, E[i].reshape(P.vel_shape), wvox=W).ravel()
                  for i in range(n)], axis=1)
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev.min() >= gamma - 1e-12 * np.abs(ev).max()
    Jc = np.stack([O.jvp(P, v, T, E[i].reshape(P.vel_shape)) for i in range(n)], axis=1)
    Jr = np.stack([O.vjp(P, v, T, np.eye(P.n_points)[k]).ravel() for k in range(P.n_points)])
    np.testing.assert_allclose(Jc, Jr, atol=1e-12 * np.abs(Jc).max())
    Reg = np.stack([O.regularizer_apply(P, E[i].reshape(P.vel_shape)).ravel()
                    for i in range(n)], axis=1)
    Href = P.cell_img * Jc.T @ (W[:, None] * Jc) + Reg + gamma * np.eye(n)
    np.testing.assert_allclose(H, Href, atol=1e-12 * np.abs(H).max())


# --------------------------------------------------------------------- P11
@pytest.mark.parametrize("dims,reg,gamma,nodes", [((5, 4), "diffusion", 0.0, 1),
                                                  ((6, 6), "curvature", 0.0, 3),
                                                  ((5, 4), "curvature", 1e-2, 2),
                                                  ((4, 3, 5), "diffusion", 1e-3, 1),
                                                  ((4, 3, 5), "curvature", 0.0, 2)])
def test_preconditioner_matches_dense_inverse(dims, reg, gamma, nodes):
    """The FFT preconditioner equals the dense inverse of the regulariser block
    (gamma > 0), or of M + mu_1 P_0 with P_0 the projector on constants and
    mu_1 the smallest nonzero eigenvalue of M (gamma = 0)."""
    d = len(dims)
    P = O.Problem(dim=d, img_m=dims, vel_m=dims, nodes=nodes, reg=reg, alpha=0.37,
                  gamma=gamma, extent=(1.0, 1.3, 0.8)[:d] + (1.0,) * (3 - d))
    n = P.n_unknowns
    E = np.eye(n)
    M = np.stack([(O.regularizer_apply(P, E[i].reshape(P.vel_shape)) +
                   gamma * E[i].reshape(P.vel_shape)).ravel() for i in range(n)], axis=1)
    nb = P.n_vel
    Minv = np.zeros_like(M)
    for b in range(nodes * d):
        sl = slice(b * nb, (b + 1) * nb)
        blk = M[sl, sl]
        if gamma == 0.0:
            ev = np.linalg.eigvalsh(blk)
            mu1 = ev[ev > 1e-9 * ev.max()].min()
            blk = blk + mu1 * np.full((nb, nb), 1.0 / nb)
        Minv[sl, sl] = np.linalg.inv(blk)
    Z = np.stack([O.spectral_precond_apply(P, E[i].reshape(P.vel_shape)).ravel()
                  for i in range(n)], axis=1)
    np.testing.assert_allclose(Z, Minv, atol=1e-11 * np.abs(Minv).max())


# --------------------------------------------------------------------- P12
def test_laplacian_stencil_vs_fourier_symbol():
    """-Laplace_h applied to a Fourier mode returns the mode times the symbol
    sum_a 4/h_a^2 sin^2(pi k_a/m_a); constants are in the null space."""
    P = O.Problem(dim=3, img_m=(6, 5, 4), vel_m=(6, 5, 4), extent=(1.0, 2.0, 0.5))
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    for k in [(1, 0, 0), (2, 3, 1), (5, 4, 3)]:
        mode = np.cos(2 * np.pi * (k[0] * x / 6 + k[1] * y / 5 + k[2] * z / 4))
        lam = sum(4.0 / P.h_vel[a] ** 2 * np.sin(np.pi * k[a] / P.vel_m[a]) ** 2 for a in range(3))
        np.testing.assert_allclose(O.laplacian_apply(P, mode), lam * mode, atol=1e-10 * lam)
    np.testing.assert_allclose(O.laplacian_apply(P, np.ones((4, 5, 6))), 0.0, atol=1e-12)


def test_laplacian_smooth_function_second_order():
    """-Laplace_h sin(2 pi x) cos(2 pi y) -> 8 pi^2 * it, second order in h."""
    errs = []
    for m in (16, 32, 64):
        P = O.Problem(dim=2, img_m=(m, m), vel_m=(m, m))
        x = (np.arange(m) + 0.5) / m
        f = np.outer(np.cos(2 * np.pi * x), np.sin(2 * np.pi * x))  # (y, x)
        errs.append(np.abs(O.laplacian_apply(P, f) - 8 * np.pi ** 2 * f).max())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.1), slopes


def test_regularizer_energy_matches_gradient():
    """alpha d_v S equals regularizer_apply; S(v) = 1/2 v^T (dS/dv) exactly
    for the quadratic form (checked by central differences)."""
    P = prob2(m=(6, 5), nodes=3, reg="curvature", alpha=0.7)
    v = random_direction(P.vel_shape, 77)
    g = O.regularizer_apply(P, v)
    rng = np.random.default_rng(4)
    for _ in range(5):
        e = rng.standard_normal(P.vel_shape)
        fd = (O.regularizer_energy(P, v + 1e-4 * e) - O.regularizer_energy(P, v - 1e-4 * e)) / 2e-4
        assert abs(P.alpha * fd - np.sum(g * e)) <= 1e-8 * abs(P.alpha * fd)


def _seminorm_form(P, x, y):
    """h_v^d sum_c <x_c, A y_c> for stationary fields, computed without the
    oracle's stencil: diffusion by summation by parts, h^d sum_a D_a^+ x . D_a^+ y
    with forward differences; curvature through the DFT symbol of the
    Laplacian, h^d sum_k lambda(k)^2 conj(x^) y^ / n (Parseval)."""
    x = np.asarray(x, dtype=np.float64).reshape((P.dim,) + tuple(reversed(P.vel_m[: P.dim])))
    y = np.asarray(y, dtype=np.float64).reshape(x.shape)
    hv = P.h_vel
    total = 0.0
    for c in range(P.dim):
        if P.reg == "diffusion":
            for a in range(P.dim):
                ax = P.dim - 1 - a
                dx = (np.roll(x[c], -1, axis=ax) - x[c]) / hv[a]
                dy = (np.roll(y[c], -1, axis=ax) - y[c]) / hv[a]
                total += float(np.sum(dx * dy))
        else:
            shape = x[c].shape
            lam = np.zeros(shape)
            for a in range(P.dim):
                ax = P.dim - 1 - a
                k = np.arange(shape[ax]).reshape([-1 if i == ax else 1 for i in range(len(shape))])
                lam = lam + 4.0 / hv[a] ** 2 * np.sin(np.pi * k / shape[ax]) ** 2
            X, Y = np.fft.fftn(x[c]), np.fft.fftn(y[c])
            total += float(np.real(np.sum(np.conj(X) * lam ** 2 * Y))) / x[c].size
    return P.cell_vel * total


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
@pytest.mark.parametrize("nt", [1, 2, 3, 5])
def test_time_quadrature_weights_trapezoid_error(reg, nt):
    """The regulariser's time weights (node_weights) integrate a velocity that
    is linear in time, v(t) = a + b t sampled at the n_t + 1 nodes, with the
    composite trapezoid rule.  The integrand 1/2 <v(t), A v(t)> is quadratic
    in t, so the exact integral is S = 1/2 (<a,a> + <a,b> + <b,b>/3) and the
    trapezoid rule exceeds it by exactly <b,b> / (12 n_t^2).  Equal weights
    1/n_t, or end weights that are not halved, miss this by O(1/n_t)."""
    P = O.Problem(dim=2, img_m=(6, 5), vel_m=(6, 5), nodes=nt + 1, reg=reg, alpha=1.0,
                  extent=(1.0, 1.3, 1.0))
    Ps = O.Problem(dim=2, img_m=(6, 5), vel_m=(6, 5), nodes=1, reg=reg, alpha=1.0,
                   extent=(1.0, 1.3, 1.0))
    a = random_direction(Ps.vel_shape, 501)[0]
    b = random_direction(Ps.vel_shape, 502)[0]
    v = np.stack([a + b * (j / nt) for j in range(nt + 1)])
    q = lambda x, y: _seminorm_form(Ps, x, y)  # noqa: E731
    exact = 0.5 * (q(a, a) + q(a, b) + q(b, b) / 3.0)
    expected = exact + q(b, b) / (12.0 * nt * nt)
    got = O.regularizer_energy(P, v)
    assert abs(got - expected) <= 1e-11 * abs(expected), (got, expected, exact)
    # the pin has teeth: the two plausible misreadings miss it
    assert abs(got - exact) > 1e-3 * abs(exact)
    # a velocity constant in time gives the stationary energy 1/2 <a,a>
    vc = np.stack([a] * (nt + 1))
    assert abs(O.regularizer_energy(P, vc) - 0.5 * q(a, a)) <= 1e-11 * q(a, a)
    assert abs(O.regularizer_energy(Ps, a[None]) - 0.5 * q(a, a)) <= 1e-11 * q(a, a)


@pytest.mark.parametrize("plant", ["equal", "mean"])
def test_time_quadrature_pin_rejects_misread_weights(plant, monkeypatch):
    """Planting a misreading of the time weights in the oracle (every node
    1/n_t, i.e. end weights not halved; or equal weights 1/(n_t + 1)) makes
    the trapezoid pin fail."""
    import importlib
    OBJ = importlib.import_module("oracle.objective")

    def bad(prob):
        nt = prob.nodes - 1
        if plant == "equal":       # every node weighted 1/n_t (ends not halved)
            return np.full(prob.nodes, 1.0 / nt)
        return np.full(prob.nodes, 1.0 / prob.nodes)   # equal weights summing to 1
    monkeypatch.setattr(OBJ, "node_weights", bad)
    with pytest.raises(AssertionError):
        test_time_quadrature_weights_trapezoid_error("diffusion", 3)


# --------------------------------------------------------------------- P13
def test_pcg_solves_spd_system_like_cholesky():
    import scipy.linalg as sla
    rng = np.random.default_rng(9)
    n = 30
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    b = rng.standard_normal(n)
    Dinv = 1.0 / np.diag(A)
    x, info = O.pcg(lambda p: A @ p, b, lambda r: Dinv * r, tol=1e-14, maxit=n * 3)
    ref = sla.cho_solve(sla.cho_factor(A), b)
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    assert not info["breakdown"]


def test_pcg_breakdown_on_indefinite():
    A = np.diag([1.0, -1.0, 2.0])
    b = np.array([0.0, 1.0, 0.0])
    _, info = O.pcg(lambda p: A @ p, b, tol=1e-12, maxit=10)
    assert info["breakdown"]


def test_pcg_hessian_system_with_spectral_preconditioner():
    """PCG on the GN system converges to the dense solution."""
    P = prob2(m=(6, 6), vm=(3, 3), nsteps=2, gamma=1e-4)
    v = fourier_velocity(P.vel_m, 1, 0.1, 61)
    T = blob_image(P.img_m, 2, 62).ravel()
    n = P.n_unknowns
    E = np.eye(n)
    H = np.stack([O.hessmat(P, v, T, E[i].reshape(P.vel_shape)).ravel() for i in range(n)], axis=1)
    b = random_direction(P.vel_shape, 63)
    x, info = O.pcg(lambda p: O.hessmat(P, v, T, p), b,
                    lambda r: O.spectral_precond_apply(P, r), tol=1e-13, maxit=200)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(H, b.ravel()), rtol=1e-8,
                               atol=1e-8 * np.abs(x).max())


# --------------------------------------------------------------------- P14
def test_zero_velocity_closed_forms():
    """v = 0: phi = 0, u1 = T, and for transport on equal grids
    J p = -sum_a D+_a T * p_a (forward difference: the right-hand cell is
    taken exactly on grid lines)."""
    P = prob2(m=(9, 7), nsteps=3)
    T = blob_image(P.img_m, 3, 71).ravel()
    v = np.zeros(P.vel_shape)
    phi = O.trace(P, v)
    assert np.all(phi == 0)
    np.testing.assert_array_equal(O.transport(P, T, phi), T)
    p = random_direction(P.vel_shape, 72)
    Ti = T.reshape(P.img_shape)
    dTx = (np.roll(Ti, -1, axis=1) - Ti) / P.h_img[0]
    dTy = (np.roll(Ti, -1, axis=0) - Ti) / P.h_img[1]
    ref = -(dTx * p[0, 0] + dTy * p[0, 1]).ravel()
    np.testing.assert_allclose(O.jvp(P, v, T, p), ref, atol=1e-12 * np.abs(ref).max())
    # continuity at v = 0: push-forward is the identity
    Pc = prob2(m=(9, 7), model="continuity", nsteps=3)
    np.testing.assert_array_equal(O.pushforward(Pc, T, phi), T)


# --------------------------------------------------------------------- P15
def test_round_trip_converges():
    """y(v, y(v, x, 0, 1), 1, 0) -> x as N grows (Sec. 2, inverse maps)."""
    errs = []
    for N in (2, 4, 8, 16):
        P = prob2(m=(16, 16), vm=(8, 8), nsteps=N, nodes=3)
        v = fourier_velocity(P.vel_m, 2, 0.1, 81, nodes=3)
        fwd = O.trace(P, v, direction=+1)
        back = O.trace(P, v, direction=-1, phi0=fwd)
        errs.append(np.abs(back).max())
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 0.05 * errs[0]


# --------------------------------------------------------------------- P16
def test_gn_solve_converges_2d():
    P = O.Problem(dim=2, img_m=(32, 32), vel_m=(32, 32), nsteps=5, alpha=1e-2)
    T = blob_image(P.img_m, 8, 1000).ravel()
    vt = fourier_velocity(P.vel_m, 4, 0.05, 1001)
    R = O.transport(P, T, O.trace(P, vt))
    v, hist = O.gn_solve(P, T, R, pcg_maxit=20)
    assert hist["status"] == "converged"
    J = np.array(hist["J"])
    assert np.all(np.diff(J) <= 0)
    assert hist["gnorm"][-1] <= 1e-2 * hist["g0"]
    assert J[-1] < 0.2 * J[0]


# --------------------------------------------------------------------- multilevel
def test_restriction_is_cell_average():
    """Restriction keeps constants and the integral; on a separable image it is
    the product of the 1-D pair averages."""
    P = O.Problem(dim=2, img_m=(8, 6), vel_m=(4, 4))
    np.testing.assert_allclose(O.restrict_image(P, np.full(48, 3.0)), 3.0, atol=1e-15)
    rng = np.random.default_rng(0)
    f, g = rng.standard_normal(8), rng.standard_normal(6)
    img = np.outer(g, f)                      # (y, x)
    ref = np.outer(0.5 * (g[0::2] + g[1::2]), 0.5 * (f[0::2] + f[1::2]))
    np.testing.assert_allclose(O.restrict_image(P, img.ravel()), ref, atol=1e-14)
    P3 = O.Problem(dim=3, img_m=(4, 6, 2), vel_m=(2, 2, 2))
    x = rng.standard_normal(48)
    assert abs(O.restrict_image(P3, x).sum() * 8 - x.sum()) < 1e-12


def test_prolongation_brute_force_and_linear_exactness():
    """Refinement equals periodic tent-weight interpolation written out point by
    point, keeps constants, and reproduces linear functions away from the wrap."""
    C = O.Problem(dim=2, img_m=(6, 4), vel_m=(6, 4))
    rng = np.random.default_rng(1)
    vc = rng.standard_normal(C.vel_shape)
    vf = O.prolong_velocity(C, vc)
    H = 1.0 / np.array([6, 4])
    for jf in range(8):
        for i_f in range(12):
            xf = np.array([(i_f + 0.5) * H[0] / 2, (jf + 0.5) * H[1] / 2])
            acc = np.zeros(2)
            for jc in range(4):
                for ic in range(6):
                    xc = np.array([(ic + 0.5) * H[0], (jc + 0.5) * H[1]])
                    d = np.abs(xf - xc)
                    d = np.minimum(d, 1.0 - d)            # periodic distance
                    wgt = np.prod(np.maximum(0.0, 1.0 - d / H))
                    acc += wgt * vc[0, :, jc, ic]
            np.testing.assert_allclose(vf[0, :, jf, i_f], acc, atol=1e-14)
    np.testing.assert_allclose(O.prolong_velocity(C, np.full(C.vel_shape, 2.0)), 2.0, atol=1e-15)
    # linear in x on the coarse centres: interior fine centres are exact
    C3 = O.Problem(dim=3, img_m=(8, 4, 4), vel_m=(8, 4, 4))
    xc = (np.arange(8) + 0.5) / 8
    lin = np.broadcast_to(2.0 + 3.0 * xc, (4, 4, 8))
    vc3 = np.zeros(C3.vel_shape)
    vc3[0, 0] = lin
    vf3 = O.prolong_velocity(C3, vc3)
    xf = (np.arange(16) + 0.5) / 16
    np.testing.assert_allclose(vf3[0, 0, 3, 5, 1:15], 2.0 + 3.0 * xf[1:15], atol=1e-14)


def test_multilevel_solve_converges_2d():
    P = O.Problem(dim=2, img_m=(32, 32), vel_m=(32, 32), nsteps=4, alpha=1e-2)
    T = blob_image(P.img_m, 6, 2000).ravel()
    vt = fourier_velocity(P.vel_m, 3, 0.05, 2001)
    R = O.transport(P, T, O.trace(P, vt))
    v, hists = O.multilevel_solve(P, T, R, levels=2, pcg_maxit=20)
    assert [h["status"] for h in hists] == ["converged", "converged"]
    assert v.shape == P.vel_shape
    J_final = O.objective(P, v, T, R)["J"]
    assert J_final < 0.2 * O.objective(P, np.zeros(P.vel_shape), T, R)["J"]


def test_resample_to_velocity_grid_pins():
    """Cell average onto the velocity grid: ratio 2 is the 2^d mean, constants
    and the integral are kept, and a non-integer ratio (7 -> 2, 5 -> 3)
    equals the mean over a common refinement (each fine cell split into
    coarse_m equal parts, each coarse cell then owning fine_m of them)."""
    P2 = O.Problem(dim=3, img_m=(8, 6, 4), vel_m=(4, 3, 2))
    x = np.random.default_rng(5).standard_normal(P2.n_points)
    np.testing.assert_allclose(O.resample_to_velocity_grid(P2, x), O.restrict_image(P2, x), atol=1e-14)
    P = O.Problem(dim=2, img_m=(7, 5), vel_m=(2, 3))
    np.testing.assert_allclose(O.resample_to_velocity_grid(P, np.full(35, 2.5)), 2.5, atol=1e-14)
    f = np.random.default_rng(6).standard_normal((5, 7))      # (y, x)
    out = O.resample_to_velocity_grid(P, f.ravel())
    assert abs(out.sum() * (1 / 6) - f.sum() * (1 / 35)) < 1e-13
    # common refinement: x split 7*2 = 14 sub-cells, y split 5*3 = 15
    fine = np.repeat(np.repeat(f, 3, axis=0), 2, axis=1)     # (15, 14)
    ref = fine.reshape(3, 5, 2, 7).mean(axis=(1, 3))          # (vel y, vel x)
    np.testing.assert_allclose(out, ref, atol=1e-14)
