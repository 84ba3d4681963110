"""The matrix-free adjoint products repeat bit for bit.

lag_vjp, gn_hessmat and lag_gradient sum their velocity-grid contributions
in integer fixed point (a 32-bit tile per brick, and a 64-bit grid buffer
for the characteristics that leave their brick's tile), whose values do not
depend on the order of the additions, and then combine the tiles in a fixed
order.  Each case below calls every product three times on the same inputs
and requires identical bits.  The far-displacement cases move
characteristics several velocity cells beyond their tiles, so the deferred
64-bit pass runs; their products must also match the oracle (1e-5, the
kink-masked comparison of the parity tests).  A weight field with a single
non-zero entry at a point that no wave traces first makes the brick's
magnitude estimate zero, so the brick is redone at the exact unit; that
product must match the oracle too.
"""

import numpy as np
import pytest

import oracle as O
from cases import SMALL_CASES, Case, gpu_problem, oracle_problem, relerr
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


# velocity grids several tiles wide (a tile spans its brick plus a halo of
# 3 (3-D) or 4 (2-D) velocity cells), velocities that move characteristics
# farther than that
FAR_CASES = [
    SMALL_CASES[4].with_(name="3d_transport_far", amplitude=1.2),
    SMALL_CASES[0].with_(name="2d_transport_far", amplitude=0.5, nsteps=8),
    Case("2d_continuity_ns_far", 2, (96, 96), (48, 48), nodes=2, model="continuity", reg="curvature",
         alpha=1e-3, nsteps=8, amplitude=0.3, seed=7210),
    Case("3d_continuity_ns_far", 3, (40, 36, 32), (20, 18, 16), nodes=2, model="continuity", nsteps=6,
         amplitude=0.5, seed=7510),
]


def products(case, plan, dev, L, T, v, w, p, W):
    """J^T w, the Gauss-Newton product and the gradient, on fresh outputs."""
    nu = plan.n_unknowns
    JTw, Hp, g = dev.empty(nu), dev.empty(nu), dev.empty(nu)
    L.lag_vjp(plan, v, T, w, JTw)
    stats = L.lag_adjoint_stats(plan)
    L.gn_hessmat(plan, v, T, W, p, Hp)
    out3 = dev.torch.zeros(3, dtype=dev.torch.float64, device="cuda")
    L.lag_gradient(plan, v, T, w, g, out3)
    return JTw, Hp, g, stats


@pytest.mark.parametrize("case", SMALL_CASES + FAR_CASES, ids=[c.name for c in SMALL_CASES + FAR_CASES])
def test_adjoint_products_repeat_bitwise(case, torch, L):
    dev = Dev(torch)
    dev.torch = torch
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    n = plan.n_points
    T = f32(case.template())
    v = f32(case.velocity())
    p = f32(case.direction(0))
    w = f32(case.image_field(0))
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    keep = margin >= MASK_CELLS
    if case.model == "transport":
        Tin, win = T, f32(w * keep)
        W = f32(keep.astype(np.float64) * np.random.default_rng(case.seed).uniform(0.5, 1.5, n))
        Wd = dev.put(W)
    else:
        Tin, win, W, Wd = f32(T * keep), w, None, None
    dv, dT, dw, dp = dev.put(v), dev.put(Tin), dev.put(win), dev.put(p)
    first = products(case, plan, dev, L, dT, dv, dw, dp, Wd)
    for rep in range(2):
        again = products(case, plan, dev, L, dT, dv, dw, dp, Wd)
        for name, a, b in zip(("vjp", "hessmat", "gradient"), first[:3], again[:3]):
            assert torch.equal(a, b), (case.name, name, rep, relerr(dev.get(a), dev.get(b)))
        assert again[3] == first[3]
    deferred, redone = first[3]
    flags = L.lag_plan_flags(plan)
    print(case.name, "deferred", deferred, "redone", redone, "flags", flags, flush=True)
    assert flags & 4 == 0   # no value took the order-dependent float fallback
    if case in FAR_CASES:
        cells = np.abs(O.trace(OP, v).reshape(case.dim, -1)).max(axis=1) * np.array(case.vel_m)
        print(case.name, "max displacement in velocity cells", cells, flush=True)
        assert deferred > 0
        JTw_o = O.vjp(OP, v, Tin, win)
        Hp_o = O.hessmat(OP, v, Tin, p, wvox=W)
        e_vjp, e_hp = relerr(dev.get(first[0]), JTw_o), relerr(dev.get(first[1]), Hp_o)
        print(case.name, f"vjp {e_vjp:.2e} hessmat {e_hp:.2e} masked {1 - keep.mean():.3f}", flush=True)
        assert e_vjp < TOL and e_hp < TOL
    plan.close()


def test_brick_redone_at_exact_unit(torch, L):
    """A single non-zero weight at an odd x cell: the waves' first items (the
    phase-0 cells of each region) see zero weight, the brick's estimate is
    zero, and the brick is redone at the unit its exact magnitude sum sets."""
    case = SMALL_CASES[4]   # 3-D, image 24 x 20 x 16 on a 12 x 10 x 8 velocity grid
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    T, v = f32(case.template()), f32(case.velocity())
    _, margin = O.jvp(OP, v, T, np.zeros(OP.vel_shape), return_margin=True)
    w = np.zeros(case.img_m[::-1], dtype=np.float32)
    w[7, 9, 11] = 3.0    # z, y, x: x = 11 is odd
    w = w.ravel()
    assert margin[np.flatnonzero(w)[0]] >= MASK_CELLS
    out = dev.empty(plan.n_unknowns)
    L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(w), out)
    deferred, redone = L.lag_adjoint_stats(plan)
    e = relerr(dev.get(out), O.vjp(OP, v, T, w))
    print("single weight: redone", redone, "deferred", deferred, f"err {e:.2e}", flush=True)
    assert redone >= 1
    assert e < TOL
    out2 = dev.empty(plan.n_unknowns)
    L.lag_vjp(plan, dev.put(v), dev.put(T), dev.put(w), out2)
    assert torch.equal(out, out2)
    plan.close()
