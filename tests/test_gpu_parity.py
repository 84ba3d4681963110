"""GPU (HIP, gfx950) vs FP64 oracle parity through the C-ABI.

Inputs are rounded to float32 once and both sides consume the same rounded
values.  Tolerances (relative: the larger of the 2-norm error and the
largest entry error, both relative to the reference; see cases.relerr):

* characteristics phi, transported / pushed-forward states, matvecs,
  regulariser and preconditioner: 1e-5;
* mass: sum(u1) matches sum(T) to 1e-6 relative.

Kinks: linear interpolation makes Jacobians piecewise constant, so float32
and float64 may pick different cells for a point within rounding distance
of a grid line.  The oracle reports, per characteristic, the smallest
distance (in cells) from any of its samples to a grid line; characteristics
closer than MASK_CELLS are excluded from Jacobian comparisons (their output
entries are skipped for J p, and their weights are zeroed for J^T w and the
Hessian so both sides sum the same terms).
"""

import numpy as np
import pytest

import oracle as O
from cases import MIN_CASES, SMALL_CASES, Case, gpu_problem, oracle_problem, relerr

pytestmark = pytest.mark.gpu

MASK_CELLS = 2e-5
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
    _L.load()  # fail loudly if the HIP library is missing
    return _L


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


class Dev:
    def __init__(self, torch):
        self.t = torch

    def put(self, a):
        return self.t.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()

    def empty(self, n):
        return self.t.empty(int(n), dtype=self.t.float32, device="cuda")

    def get(self, x):
        self.t.cuda.synchronize()
        return x.detach().cpu().numpy().astype(np.float64)


def run_case(case: Case, torch, L):
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    n, nu, d = plan.n_points, plan.n_unknowns, case.dim
    T = f32(case.template())
    v = f32(case.velocity())
    p = f32(case.direction(0))
    w = f32(case.image_field(0))
    direction = -1 if case.model == "transport" else 1
    out = {}

    # --- characteristics (Algorithm 1) ---------------------------------
    phi_o = O.trace(OP, v)
    phi_g = dev.empty(d * n)
    L.lag_trace(plan, dev.put(v), direction, phi_g)
    out["trace"] = relerr(dev.get(phi_g), phi_o)

    # --- state: transport or push-forward ------------------------------
    phi32 = f32(phi_o)   # same end points on both sides
    u_g = dev.empty(n)
    if case.model == "transport":
        L.lag_transport(plan, dev.put(T), dev.put(phi32), u_g)
        u_o = O.transport(OP, T, phi32.reshape(d, n))
    else:
        L.lag_pushforward(plan, dev.put(T), dev.put(phi32), u_g)
        u_o = O.pushforward(OP, T, phi32.reshape(d, n))
        ug = dev.get(u_g)
        out["mass"] = abs(ug.sum() - T.sum()) / T.sum()
        # bitwise reproducible
        u_g2 = dev.empty(n)
        L.lag_pushforward(plan, dev.put(T), dev.put(phi32), u_g2)
        out["push_bitwise"] = bool(np.array_equal(dev.get(u_g2), ug))
    out["state"] = relerr(dev.get(u_g), u_o)

    # --- kink mask -------------------------------------------------------
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    keep = margin >= MASK_CELLS
    out["masked_fraction"] = 1.0 - keep.mean()

    # --- J p -------------------------------------------------------------
    Jp_g = dev.empty(n)
    if case.model == "transport":
        L.lag_jvp(plan, dev.put(v), dev.put(T), dev.put(p), Jp_g)
        Jp_o = O.jvp(OP, v, T, p)
        out["jvp"] = relerr(dev.get(Jp_g)[keep], Jp_o[keep])
        out["jvp_unmasked"] = relerr(dev.get(Jp_g), Jp_o)
    else:
        Tm = T * keep
        L.lag_jvp(plan, dev.put(v), dev.put(Tm), dev.put(p), Jp_g)
        Jp_o = O.jvp(OP, v, Tm, p)
        out["jvp"] = relerr(dev.get(Jp_g), Jp_o)
        out["jvp_mass"] = abs(dev.get(Jp_g).sum()) / (np.abs(Jp_o).sum() + 1e-300)

    # --- J^T w -----------------------------------------------------------
    JTw_g = dev.empty(nu)
    if case.model == "transport":
        wm = w * keep
        L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(wm), JTw_g)
        JTw_o = O.vjp(OP, v, T, wm)
    else:
        Tm = T * keep
        L.lag_vjp(plan, dev.put(v), dev.put(Tm), dev.put(w), JTw_g)
        JTw_o = O.vjp(OP, v, Tm, w)
    out["vjp"] = relerr(dev.get(JTw_g), JTw_o)

    # --- Gauss-Newton matvec -------------------------------------------
    Hp_g = dev.empty(nu)
    if case.model == "transport":
        W = keep.astype(np.float64) * np.random.default_rng(case.seed).uniform(0.5, 1.5, n)
        W = f32(W)
        L.gn_hessmat(plan, dev.put(v), dev.put(T), dev.put(W), dev.put(p), Hp_g)
        Hp_o = O.hessmat(OP, v, T, p, wvox=W)
    else:
        Tm = T * keep
        L.gn_hessmat(plan, dev.put(v), dev.put(Tm), None, dev.put(p), Hp_g)
        Hp_o = O.hessmat(OP, v, Tm, p)
    out["hessmat"] = relerr(dev.get(Hp_g), Hp_o)
    out["flags"] = L.lag_plan_flags(plan)
    # data term alone (alpha = gamma = 0), which the regulariser could hide
    cD = case.with_(alpha=0.0, gamma=0.0)
    planD = L.Plan(gpu_problem(cD))
    OPD = oracle_problem(cD)
    HD_g = dev.empty(nu)
    if case.model == "transport":
        L.gn_hessmat(planD, dev.put(v), dev.put(T), dev.put(W), dev.put(p), HD_g)
        HD_o = O.hessmat(OPD, v, T, p, wvox=W)
    else:
        L.gn_hessmat(planD, dev.put(v), dev.put(Tm), None, dev.put(p), HD_g)
        HD_o = O.hessmat(OPD, v, Tm, p)
    out["hessmat_data"] = relerr(dev.get(HD_g), HD_o)
    planD.close()
    reg_o = O.regularizer_apply(OP, p) + case.gamma * p

    # --- regulariser and spectral preconditioner ----------------------------
    R_g = dev.empty(nu)
    L.lag_reg_apply(plan, dev.put(p), R_g)
    out["reg"] = relerr(dev.get(R_g), reg_o)
    z_g = dev.empty(nu)
    L.spectral_precond_apply(plan, dev.put(p), z_g)
    out["precond"] = relerr(dev.get(z_g), O.spectral_precond_apply(OP, p))

    # --- objective ----------------------------------------------------------
    vt = f32(case.velocity(seed_off=2))
    R = f32(O.objective(OP, vt, T, np.zeros(n))["u"])
    obj_o = O.objective(OP, v, T, R)
    out3 = torch.zeros(3, dtype=torch.float64, device="cuda")
    uo_g = dev.empty(n)
    L.lag_objective(plan, dev.put(v), dev.put(T), dev.put(R), uo_g, out3)
    J3 = dev.get(out3)
    out["obj_J"] = abs(J3[0] - obj_o["J"]) / abs(obj_o["J"])
    out["obj_D"] = abs(J3[1] - obj_o["D"]) / abs(obj_o["D"])
    out["obj_S"] = abs(J3[2] - obj_o["S"]) / abs(obj_o["S"])
    g_g = dev.empty(nu)
    L.lag_gradient(plan, dev.put(v), dev.put(T), dev.put(R), g_g, out3)
    g_o, _ = O.gradient(OP, v, T, R)
    out["grad_unmasked"] = relerr(dev.get(g_g), g_o)
    plan.close()
    return out


@pytest.mark.parametrize("case", SMALL_CASES, ids=[c.name for c in SMALL_CASES])
def test_small_case_parity(case, torch, L):
    r = run_case(case, torch, L)
    print(case.name, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    assert r["masked_fraction"] < 0.05
    for key in ("trace", "state", "jvp", "vjp", "hessmat", "hessmat_data", "reg", "precond",
                "obj_J", "obj_D", "obj_S"):
        assert r[key] < TOL, (key, r[key])
    assert r["flags"] & 2 == 0     # forward recovery never met a singular step
    if case.model == "continuity":
        assert r["mass"] < 1e-6
        assert r["push_bitwise"]
        assert r["jvp_mass"] < 1e-5
    # the unmasked gradient includes kink characteristics on both sides
    assert r["grad_unmasked"] < 1e-3


@pytest.mark.parametrize("case", MIN_CASES, ids=[c.name for c in MIN_CASES])
def test_minimum_size_parity(case, torch, L):
    """Smallest accepted grids: tiles wrap the domain, FFT sizes 2 and 3."""
    r = run_case(case, torch, L)
    print(case.name, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    for key in ("trace", "state", "jvp", "vjp", "hessmat", "hessmat_data", "reg", "precond",
                "obj_J", "obj_D", "obj_S"):
        assert r[key] < TOL, (key, r[key])
    if case.model == "continuity":
        assert r["mass"] < 1e-6 and r["push_bitwise"]


def test_zero_velocity_closed_form(torch, L):
    """v = 0: phi = 0 exactly, u1 = T exactly, and the transport J p equals
    the one-sided difference closed form of the oracle."""
    case = Case("zero", 2, (32, 24), (32, 24), nsteps=3, seed=8100)
    dev = Dev(torch)
    plan = L.Plan(gpu_problem(case))
    T = f32(case.template())
    v = np.zeros(case.vel_shape)
    phi = dev.empty(2 * plan.n_points)
    L.lag_trace(plan, dev.put(v), -1, phi)
    assert np.all(dev.get(phi) == 0)
    u = dev.empty(plan.n_points)
    L.lag_transport(plan, dev.put(T), phi, u)
    assert np.array_equal(dev.get(u), T)
    p = f32(case.direction(1))
    Jp = dev.empty(plan.n_points)
    L.lag_jvp(plan, dev.put(v), dev.put(T), dev.put(p), Jp)
    ref = O.jvp(oracle_problem(case), v, T, p)
    assert relerr(dev.get(Jp), ref) < TOL


def test_constant_velocity_translation(torch, L):
    """A whole-cell constant velocity translates the image exactly (np.roll)."""
    case = Case("shift", 3, (16, 12, 8), (8, 6, 4), nsteps=2, seed=8200)
    dev = Dev(torch)
    plan = L.Plan(gpu_problem(case))
    T = f32(case.template())
    v = np.zeros(case.vel_shape)
    h = 1.0 / np.array(case.img_m)
    v[0, 0], v[0, 1], v[0, 2] = 2 * h[0], -h[1], 3 * h[2]
    phi = dev.empty(3 * plan.n_points)
    L.lag_trace(plan, dev.put(v), -1, phi)
    u = dev.empty(plan.n_points)
    L.lag_transport(plan, dev.put(T), phi, u)
    ref = np.roll(np.roll(np.roll(T.reshape(8, 12, 16), 2, axis=2), -1, axis=1), 3, axis=0)
    np.testing.assert_allclose(dev.get(u).reshape(8, 12, 16), ref, atol=1e-6 * np.abs(T).max())


def test_constant_image_stays_constant(torch, L):
    case = SMALL_CASES[4]
    dev = Dev(torch)
    plan = L.Plan(gpu_problem(case))
    v = f32(case.velocity(scale=3.0))
    T = np.full(plan.n_points, 1.75)
    phi = dev.empty(3 * plan.n_points)
    L.lag_trace(plan, dev.put(v), -1, phi)
    u = dev.empty(plan.n_points)
    L.lag_transport(plan, dev.put(T), phi, u)
    assert np.abs(dev.get(u) - 1.75).max() < 1e-6
    Jp = dev.empty(plan.n_points)
    L.lag_jvp(plan, dev.put(v), dev.put(T), dev.put(f32(case.direction(2))), Jp)
    assert np.abs(dev.get(Jp)).max() < 1e-4


def test_dot_test_gpu(torch, L):
    """<q, J p> = <J^T q, p> between the GPU's own JVP and VJP kernels."""
    for case in (SMALL_CASES[1], SMALL_CASES[2], SMALL_CASES[5]):
        dev = Dev(torch)
        plan = L.Plan(gpu_problem(case))
        T, v = f32(case.template()), f32(case.velocity())
        p, q = f32(case.direction(3)), f32(case.image_field(3))
        Jp, JTq = dev.empty(plan.n_points), dev.empty(plan.n_unknowns)
        L.lag_jvp(plan, dev.put(v), dev.put(T), dev.put(p), Jp)
        L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(q), JTq)
        a = float(dev.get(Jp) @ q)
        b = float(dev.get(JTq).ravel() @ p.ravel())
        assert abs(a - b) <= 1e-5 * (abs(a) + abs(b)), (case.name, a, b)


def test_hessmat_equals_composition(torch, L):
    """gn_hessmat = h^d J^T (W J p) + reg(p) + gamma p, built from the GPU's
    own lag_jvp, lag_vjp and lag_reg_apply."""
    for case in (SMALL_CASES[0], SMALL_CASES[2]):
        dev = Dev(torch)
        plan = L.Plan(gpu_problem(case))
        T, v, p = f32(case.template()), f32(case.velocity()), f32(case.direction(4))
        Hp = dev.empty(plan.n_unknowns)
        L.gn_hessmat(plan, dev.put(v), dev.put(T), None, dev.put(p), Hp)
        Jp = dev.empty(plan.n_points)
        L.lag_jvp(plan, dev.put(v), dev.put(T), dev.put(p), Jp)
        hd = float(np.prod(1.0 / np.array(case.img_m)))
        JTJp = dev.empty(plan.n_unknowns)
        L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(hd * dev.get(Jp)), JTJp)
        R = dev.empty(plan.n_unknowns)
        L.lag_reg_apply(plan, dev.put(p), R)
        comp = dev.get(JTJp) + dev.get(R)
        assert relerr(dev.get(Hp), comp) < 1e-5, case.name


@pytest.mark.parametrize("case", [
    SMALL_CASES[4].with_(name="3d_far", amplitude=1.2),
    SMALL_CASES[0].with_(name="2d_far", amplitude=0.5, nsteps=8),
], ids=lambda c: c.name)
def test_trace_far_displacement(case, torch, L):
    """Characteristics that travel several velocity cells beyond a brick's
    staged velocity tile read the field from HBM: the trace still matches
    the oracle."""
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    v = f32(case.velocity())
    phi_o = O.trace(OP, v)
    phi_g = dev.empty(case.dim * plan.n_points)
    L.lag_trace(plan, dev.put(v), -1, phi_g)
    cells = np.abs(phi_o.reshape(case.dim, -1)).max(axis=1) * np.array(case.vel_m)
    print("trace far", case.name, "max displacement in velocity cells", cells, flush=True)
    assert cells.max() > 4
    assert relerr(dev.get(phi_g), phi_o) < TOL
