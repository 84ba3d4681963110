"""Parity at the workloads' full sizes, in the benchmark's launch configuration.

At 128^3 and 256x256x224 the oracle cannot evaluate every characteristic in
seconds, so the GPU runs the full problem while the oracle evaluates a random
sample of characteristics one by one:

* per-characteristic outputs (phi, transported state, J p) are compared on
  the sample;
* sums over characteristics (J^T w, the Gauss-Newton data term) are compared
  with weights supported on the sample (zero elsewhere), which the oracle
  evaluates exactly with ``points=sample``;
* the regulariser and the preconditioner act on the velocity grid only and
  are compared in full;
* with every characteristic weighted, identities that hold at any size (dot
  test, energy, symmetry) and the agreement of the assembled and matrix-free
  products cover the rows the sample leaves out.

The 2-D 256^2 continuity workload (5 time nodes, N = 32) is small enough for
a full comparison.
"""

import numpy as np
import pytest

import oracle as O
from cases import relerr
from synthetic import workload
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


def oprob(w, **kw):
    d = dict(dim=w.dim, img_m=w.img_m, vel_m=w.vel_m, nodes=w.nodes, model=w.model, reg=w.reg,
             nsteps=w.nsteps, alpha=w.alpha, gamma=w.gamma)
    d.update(kw)
    return O.Problem(**d)


def gplan(L, w, jac_blocks=8, **kw):
    d = dict(nt_nodes=w.nodes, model=w.model, reg=w.reg, nsteps=w.nsteps, alpha=w.alpha, gamma=w.gamma,
             jac_blocks=jac_blocks)
    d.update(kw)
    return L.Plan(L.make_problem(w.dim, w.img_m, w.vel_m, **d))


@pytest.mark.parametrize("name,nsample", [("3d128_transport", 4096), ("3d256_transport", 2048)])
def test_transport_fullsize_sampled(name, nsample, torch, L):
    w = workload(name)
    dev = Dev(torch)
    print(f"[{name}] setting up", flush=True)
    T = f32(w.template().ravel())
    v = f32(0.5 * w.velocity_true())          # the benchmark's iterate
    p = f32(w.direction(0))
    OP = oprob(w)
    plan = gplan(L, w)
    n, nu = plan.n_points, plan.n_unknowns
    rng = np.random.default_rng(4242)
    S = np.sort(rng.choice(n, nsample, replace=False))
    Td, vd, pd = dev.put(T), dev.put(v), dev.put(p)

    # characteristics and transported state
    phi = dev.empty(3 * n)
    L.lag_trace(plan, vd, -1, phi)
    u = dev.empty(n)
    L.lag_transport(plan, Td, phi, u)
    phi_o = O.trace(OP, v, points=S)
    phig = dev.get(phi).reshape(3, n)[:, S]
    e_phi = relerr(phig, phi_o)
    e_u = relerr(dev.get(u)[S], O.transport(OP, T, phi_o, points=S))

    # J p on the sample, kink-masked
    Jp = dev.empty(n)
    L.lag_jvp(plan, vd, Td, pd, Jp)
    Jp_o, margin = O.jvp(OP, v, T, p, points=S, return_margin=True)
    keep = margin >= MASK_CELLS
    e_jvp = relerr(dev.get(Jp)[S][keep], Jp_o[keep])

    # sums over the sample: J^T w and the Gauss-Newton data term
    wS = np.zeros(n)
    wS[S] = f32(w.image_direction(0).ravel())[S] * keep
    JTw = dev.empty(nu)
    L.lag_vjp(plan, vd, Td, dev.put(wS), JTw)
    e_vjp = relerr(dev.get(JTw), O.vjp(OP, v, T, wS[S], points=S))

    planD = gplan(L, w, alpha=0.0, gamma=0.0)
    OPD = oprob(w, alpha=0.0, gamma=0.0)
    W = np.zeros(n)
    W[S] = keep.astype(np.float64)
    Hm = dev.empty(nu)
    L.gn_hessmat(planD, vd, Td, dev.put(W), pd, Hm)
    Ho = O.hessmat(OPD, v, T, p, wvox=W[S], points=S)
    e_hm = relerr(dev.get(Hm), Ho)
    assert L.lag_jacobian_assemble(planD, vd, Td)
    Ha = dev.empty(nu)
    L.gn_hessmat_assembled(planD, dev.put(W), pd, Ha)
    e_ha = relerr(dev.get(Ha), Ho)

    # velocity-grid operators in full
    R = dev.empty(nu)
    L.lag_reg_apply(plan, pd, R)
    e_reg = relerr(dev.get(R), O.regularizer_apply(OP, p) + w.gamma * p)
    z = dev.empty(nu)
    L.spectral_precond_apply(plan, pd, z)
    e_pc = relerr(dev.get(z), O.spectral_precond_apply(OP, p))
    res = dict(phi=e_phi, u=e_u, jvp=e_jvp, vjp=e_vjp, hess_matfree=e_hm, hess_assembled=e_ha, reg=e_reg,
               precond=e_pc, masked=1 - keep.mean())
    print(name, {k: f"{x:.2e}" for k, x in res.items()}, flush=True)
    for k in ("phi", "u", "jvp", "vjp", "hess_matfree", "hess_assembled", "reg", "precond"):
        assert res[k] < TOL, (k, res[k])
    planD.close()
    plan.close()


@pytest.mark.parametrize("name", ["3d128_transport", "3d256_transport"])
def test_transport_fullsize_all_rows(name, torch, L):
    """Every characteristic weighted (W = 1, no sample): properties that hold
    at any size tie the full products to the sampled parity above.

    * dot test <w, J p> = <J^T w, p> with w over all rows;
    * energy identity <p, H_D p> = h^d |J p|^2 for the data term H_D;
    * symmetry <q, H_D p> = <H_D q, p>;
    * the assembled and the matrix-free Gauss-Newton products agree entry by
      entry (two kernels with different accumulation structures)."""
    w = workload(name)
    dev = Dev(torch)
    T = f32(w.template().ravel())
    v = f32(0.5 * w.velocity_true())
    p = f32(w.direction(0))
    q = f32(w.direction(1))
    planD = gplan(L, w, alpha=0.0, gamma=0.0)
    n, nu = planD.n_points, planD.n_unknowns
    hd = float(np.prod(1.0 / np.array(w.img_m, dtype=np.float64)))
    Td, vd, pd, qd = dev.put(T), dev.put(v), dev.put(p), dev.put(q)
    wimg = f32(w.image_direction(0).ravel())
    Jp = dev.empty(n)
    L.lag_jvp(planD, vd, Td, pd, Jp)
    JTw = dev.empty(nu)
    L.lag_vjp(planD, vd, Td, dev.put(wimg), JTw)
    Jpg, JTwg = dev.get(Jp), dev.get(JTw)
    lhs, rhs = float(wimg @ Jpg), float(JTwg.ravel() @ p.ravel())
    scale = float(np.abs(wimg) @ np.abs(Jpg))
    e_dot = abs(lhs - rhs) / scale
    Hm = dev.empty(nu)
    L.gn_hessmat(planD, vd, Td, None, pd, Hm)
    Hq = dev.empty(nu)
    L.gn_hessmat(planD, vd, Td, None, qd, Hq)
    Hmg, Hqg = dev.get(Hm), dev.get(Hq)
    energy = hd * float(Jpg @ Jpg)
    e_energy = abs(float(p.ravel() @ Hmg.ravel()) - energy) / energy
    a, b = float(q.ravel() @ Hmg.ravel()), float(Hqg.ravel() @ p.ravel())
    e_sym = abs(a - b) / (float(np.abs(q.ravel()) @ np.abs(Hmg.ravel())) + 1e-300)
    assert L.lag_jacobian_assemble(planD, vd, Td)
    Ha = dev.empty(nu)
    L.gn_hessmat_assembled(planD, None, pd, Ha)
    e_am = relerr(dev.get(Ha), Hmg)
    res = dict(dot=e_dot, energy=e_energy, symmetry=e_sym, assembled_vs_matfree=e_am)
    print(name, "all rows", {k: f"{x:.2e}" for k, x in res.items()}, flush=True)
    for k, x in res.items():
        assert x < TOL, (k, x)
    planD.close()


def test_continuity_2d256_full(torch, L):
    """The 2-D 256^2 mass-preserving workload, compared in full."""
    w = workload("2d256_continuity")
    dev = Dev(torch)
    OP = oprob(w)
    plan = gplan(L, w, jac_blocks=0)
    n, nu = plan.n_points, plan.n_unknowns
    T = f32(w.template().ravel())
    v = f32(0.5 * w.velocity_true())
    p = f32(w.direction(0))
    q = f32(w.image_direction(0).ravel())
    Td, vd, pd = dev.put(T), dev.put(v), dev.put(p)
    phi = dev.empty(2 * n)
    L.lag_trace(plan, vd, 1, phi)
    phi_o = O.trace(OP, v)
    e_phi = relerr(dev.get(phi), phi_o)
    phi32 = f32(phi_o)
    u = dev.empty(n)
    L.lag_pushforward(plan, Td, dev.put(phi32), u)
    ug = dev.get(u)
    e_u = relerr(ug, O.pushforward(OP, T, phi32.reshape(2, n)))
    mass = abs(ug.sum() - T.sum()) / T.sum()
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    Tm = T * (margin >= MASK_CELLS)
    Jp = dev.empty(n)
    L.lag_jvp(plan, vd, dev.put(Tm), pd, Jp)
    e_jvp = relerr(dev.get(Jp), O.jvp(OP, v, Tm, p))
    JTq = dev.empty(nu)
    L.lag_vjp(plan, vd, dev.put(Tm), dev.put(q), JTq)
    e_vjp = relerr(dev.get(JTq), O.vjp(OP, v, Tm, q))
    H = dev.empty(nu)
    L.gn_hessmat(plan, vd, dev.put(Tm), None, pd, H)
    e_h = relerr(dev.get(H), O.hessmat(OP, v, Tm, p))
    z = dev.empty(nu)
    L.spectral_precond_apply(plan, pd, z)
    e_pc = relerr(dev.get(z), O.spectral_precond_apply(OP, p))
    res = dict(phi=e_phi, u=e_u, jvp=e_jvp, vjp=e_vjp, hess=e_h, precond=e_pc, mass=mass)
    print("2d256_continuity", {k: f"{x:.2e}" for k, x in res.items()}, flush=True)
    for k in ("phi", "u", "jvp", "vjp", "hess", "precond"):
        assert res[k] < TOL, (k, res[k])
    assert mass < 1e-6
