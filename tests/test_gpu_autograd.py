"""torch.autograd wrapper of the Lagrangian transport (hand-written J^T backward).

Loss L(v, T) = 1/2 sum_i m_i (u1_i - R_i)^2 with a kink mask m.  Checked:
* dL/dv and dL/dT against the oracle's J^T and P^T of the same weights;
* directional derivatives along 10 seeded directions against the oracle's
  J dv and against central differences of the oracle's loss;
* a Taylor test of the GPU's own forward: the remainder
  L(v + e dv) - L(v) - e <grad, dv> decays like e^2;
* the same at 128^3 with the loss restricted to a sample of characteristics.
"""

import numpy as np
import pytest

import oracle as O
from cases import SMALL_CASES, oracle_problem, gpu_problem, relerr
from synthetic import workload
from test_gpu_parity import MASK_CELLS, Dev, f32

pytestmark = pytest.mark.gpu


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


def check_grad(OP, plan, T, v, R, m, dirs, torch, L, sample=None):
    from paper_1703_04446_amd.autograd import lagrangian_transport
    dev = Dev(torch)
    vt = dev.put(v).requires_grad_(True)
    Tt = dev.put(T).requires_grad_(True)
    Rt, mt = dev.put(R), dev.put(m)
    u = lagrangian_transport(vt, Tt, plan)
    loss = 0.5 * (mt.double() * (u.double() - Rt.double()) ** 2).sum()
    loss.backward()
    gv, gT = dev.get(vt.grad), dev.get(Tt.grad)
    pts = sample
    phi_o = O.trace(OP, v, points=pts)
    uo = O.transport(OP, T, phi_o, points=pts)
    Rs = R if pts is None else R[pts]
    ms = m if pts is None else m[pts]
    res = ms * (uo - Rs)
    gv_o = O.vjp(OP, v, T, res, points=pts).ravel()
    out = {"grad_v": relerr(gv, gv_o)}
    if pts is None:
        # dL/dT = P(phi)^T res, the push-forward of the weights along phi
        out["grad_T"] = relerr(gT, O.pushforward(OP, res, phi_o))
    # directional derivatives: backward vs oracle J dv vs oracle central differences
    dd_err, fd_err = 0.0, 0.0
    for dv in dirs:
        a = float(gv @ dv.ravel())
        Jdv = O.jvp(OP, v, T, dv, points=pts)
        b = float(res @ Jdv)
        eps = 1e-6

        def loss_o(vv):
            uu = O.transport(OP, T, O.trace(OP, vv, points=pts), points=pts)
            return 0.5 * float(np.sum(ms * (uu - Rs) ** 2))
        fd = (loss_o(v + eps * dv) - loss_o(v - eps * dv)) / (2 * eps)
        dd_err = max(dd_err, abs(a - b) / (abs(b) + 1e-30))
        fd_err = max(fd_err, abs(b - fd) / (abs(fd) + 1e-30))
    out["dir_vs_oracle"] = dd_err
    out["oracle_vs_fd"] = fd_err
    return out, gv


def test_autograd_small_3d(torch, L):
    case = SMALL_CASES[4]
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    T = f32(case.template())
    v = f32(case.velocity())
    R = f32(O.objective(OP, case.velocity(seed_off=2), T, np.zeros(plan.n_points))["u"])
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    m = (margin >= MASK_CELLS).astype(np.float64)
    dirs = [f32(case.direction(10 + i)) for i in range(10)]
    r, gv = check_grad(OP, plan, T, v, R, m, dirs, torch, L)
    print("autograd small", {k: f"{x:.2e}" for k, x in r.items()}, flush=True)
    assert r["grad_v"] < 1e-5 and r["grad_T"] < 1e-5
    assert r["dir_vs_oracle"] < 1e-4
    assert r["oracle_vs_fd"] < 1e-5

    # Taylor test of the GPU forward with its own gradient
    from paper_1703_04446_amd.autograd import lagrangian_transport
    dev = Dev(torch)
    Rt, mt, Tt = dev.put(R), dev.put(m), dev.put(T)

    def loss_gpu(vv):
        u = lagrangian_transport(dev.put(vv), Tt, plan)
        return 0.5 * float((mt.double() * (u.double() - Rt.double()) ** 2).sum())
    L0 = loss_gpu(v)
    dv = f32(case.velocity(seed_off=30))
    gdv = float(gv @ dv.ravel())
    eps = np.array([0.4, 0.2, 0.1, 0.05])
    rem = np.array([abs(loss_gpu(v + e * dv) - L0 - e * gdv) for e in eps])
    slopes = np.log2(rem[:-1] / rem[1:])
    print("taylor remainders", rem, "slopes", slopes, flush=True)
    assert np.all(slopes > 1.6), slopes


def test_autograd_128_sampled(torch, L):
    """The 128^3 workload: full GPU forward/backward, loss on a sample."""
    w = workload("3d128_transport")
    OP = O.Problem(dim=3, img_m=w.img_m, vel_m=w.vel_m, nsteps=w.nsteps, alpha=w.alpha)
    plan = L.Plan(L.make_problem(3, w.img_m, w.vel_m, nsteps=w.nsteps, alpha=w.alpha))
    T = f32(w.template().ravel())
    v = f32(0.5 * w.velocity_true())
    n = plan.n_points
    rng = np.random.default_rng(77)
    S = np.sort(rng.choice(n, 2048, replace=False))
    R = f32(0.9 * T)
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), points=S, return_margin=True)
    m = np.zeros(n)
    m[S] = margin >= MASK_CELLS
    dirs = [f32(w.direction(10 + i)) for i in range(10)]
    r, _ = check_grad(OP, plan, T, v, R, m, dirs, torch, L, sample=S)
    print("autograd 128^3", {k: f"{x:.2e}" for k, x in r.items()}, flush=True)
    assert r["grad_v"] < 1e-5
    assert r["dir_vs_oracle"] < 1e-4
    assert r["oracle_vs_fd"] < 1e-5
