"""Characteristics whose RK4 step Jacobians are close to singular.

The GPU's matrix-free adjoint (lag_vjp, gn_hessmat) recovers the adjoint of
each step from the next by a d x d solve with the step Jacobian (forward
recovery).  For a velocity with large gradients and a single RK4 step, some
step Jacobians come close to singular; those characteristics must take the
recomputed reverse sweep (no inversion) so that the products stay exact.
The oracle stores the whole trajectory and inverts nothing, so it is the
reference; the cases are checked to contain such characteristics first.
"""

import numpy as np
import pytest

import oracle as O
from cases import Case, gpu_problem, oracle_problem, relerr
from oracle.grid import start_indices
from oracle.lagrangian import RK4_A, RK4_B, RK4_C, _GridVelocity, _stage_point
from synthetic import fourier_velocity, random_direction
from test_gpu_parity import MASK_CELLS, Dev, f32

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return _t


@pytest.fixture(scope="module")
def L():
    import paper_1703_04446_amd as _L
    _L.load()
    return _L


def recovery_growth(P, v):
    """Per characteristic, the product over steps of the Frobenius condition
    number of the RK4 step Jacobian divided by d (FP64, from the oracle's
    velocity samples)."""
    idx = start_indices(P, None)
    vel = _GridVelocity(P, v, idx)
    dt = (-1.0 if P.model == "transport" else 1.0) / P.nsteps
    t0 = 1.0 if dt < 0 else 0.0
    d = P.dim
    phi = np.zeros((d, idx.shape[1]))
    g = np.ones(idx.shape[1])
    eye = np.eye(d)[:, :, None]
    for k in range(P.nsteps):
        ks, Gs = [], []
        for row, c in zip(RK4_A, RK4_C):
            val, G, _ = vel.sample(_stage_point(phi, dt, row, ks), t0 + (k + c) * dt, grad=True)
            ks.append(val)
            Gs.append(G)
        # M = d phi_{k+1} / d phi_k by the chain rule through the stages
        dP = [eye]
        dK = []
        for i, row in enumerate(RK4_A):
            Pi = eye + sum(dt * a * dK[j] for j, a in enumerate(row) if a != 0.0) if i else eye
            dK.append(np.einsum("abn,bcn->acn", Gs[i], Pi))
        M = eye + sum(dt * b * dK[i] for i, b in enumerate(RK4_B))
        Mt = np.moveaxis(M, 2, 0)
        kap = np.linalg.norm(Mt, axis=(1, 2)) * np.linalg.norm(np.linalg.inv(Mt), axis=(1, 2)) / d
        g = g * kap
        phi = _stage_point(phi, dt, RK4_B, ks)
    return g


CASES = [
    (Case("2d_transport_singular", 2, (24, 20), (12, 10), nsteps=1, seed=7950), 2, 0.5, 9),
    (Case("2d_continuity_singular", 2, (24, 20), (12, 10), nsteps=1, model="continuity", seed=7960), 2, 0.5, 6),
    (Case("3d_transport_singular", 3, (12, 10, 8), (6, 5, 4), nsteps=1, seed=7970), 2, 0.8, 1),
]


@pytest.mark.parametrize("case,kmax,amp,vseed", CASES, ids=[c[0].name for c in CASES])
def test_near_singular_step_jacobians(case, kmax, amp, vseed, torch, L):
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    n, nu = plan.n_points, plan.n_unknowns
    T = f32(case.template())
    v = f32(fourier_velocity(case.vel_m, kmax, amp, vseed))
    p = f32(random_direction(case.vel_shape, vseed + 100))
    w = f32(random_direction((n,), vseed + 200))
    growth = recovery_growth(OP, v)
    print(case.name, "characteristics with growth > 100:", int((growth > 100).sum()), "of", n,
          "max", float(growth.max()), flush=True)
    assert (growth > 300).sum() >= 1, "case does not exercise the fallback"
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    keep = margin >= MASK_CELLS
    assert L.lag_plan_flags(plan) == 0
    JTw = dev.empty(nu)
    H = dev.empty(nu)
    if case.model == "transport":
        wm = w * keep
        L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(wm), JTw)
        JTw_o = O.vjp(OP, v, T, wm)
        W = f32(keep.astype(np.float64))
        L.gn_hessmat(plan, dev.put(v), dev.put(T), dev.put(W), dev.put(p), H)
        H_o = O.hessmat(OP, v, T, p, wvox=W)
    else:
        Tm = T * keep
        L.lag_vjp(plan, dev.put(v), dev.put(Tm), dev.put(w), JTw)
        JTw_o = O.vjp(OP, v, Tm, w)
        L.gn_hessmat(plan, dev.put(v), dev.put(Tm), None, dev.put(p), H)
        H_o = O.hessmat(OP, v, Tm, p)
    flags = L.lag_plan_flags(plan)
    e_vjp, e_h = relerr(dev.get(JTw), JTw_o), relerr(dev.get(H), H_o)
    print(case.name, f"flags {flags} vjp {e_vjp:.2e} hessmat {e_h:.2e} masked {1 - keep.mean():.3f}", flush=True)
    assert flags == 1, flags          # the recomputed sweep ran; forward recovery never met a singular step
    assert e_vjp < TOL and e_h < TOL
    plan.close()
