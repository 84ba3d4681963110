"""Multilevel continuation on the GPU: restriction and refinement kernels
against the oracle, and the coarse-to-fine solve checked iterate-wise."""

import numpy as np
import pytest

import oracle as O
from cases import Case, gpu_problem, oracle_problem, relerr
from test_gpu_parity import Dev, f32

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


@pytest.mark.parametrize("case", [
    Case("ml2d", 2, (24, 20), (12, 10), nodes=3, seed=8300),
    Case("ml3d", 3, (16, 12, 8), (8, 6, 4), seed=8400),
], ids=lambda c: c.name)
def test_restrict_and_prolong(case, torch, L):
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    f = f32(case.template())
    c = dev.empty(plan.n_points >> case.dim)
    L.lag_restrict_image(plan, dev.put(f), c)
    assert relerr(dev.get(c), O.restrict_image(OP, f)) < 1e-6
    coarse = O.coarsen_problem(OP)
    vc = f32(np.random.default_rng(case.seed).standard_normal(coarse.vel_shape))
    vf = dev.empty(plan.n_unknowns)
    L.lag_prolong_velocity(plan, dev.put(vc), vf)
    assert relerr(dev.get(vf), O.prolong_velocity(coarse, vc)) < 1e-6


def test_multilevel_solve(torch, L):
    """Three levels (16^2, 32^2, 64^2) on the 2-D 64^2 workload."""
    case = Case("ml_solve", 2, (64, 64), (64, 64), nsteps=5, nblobs=8, kmax=4, amplitude=0.05, seed=1000)
    dev = Dev(torch)
    OP = oracle_problem(case)
    T = f32(case.template())
    R = f32(O.objective(OP, case.velocity(), T, np.zeros(OP.n_points))["u"])
    v = torch.zeros(OP.n_unknowns, device="cuda")
    opt = L.lag_gn_default_options()
    opt.pcg_maxit = 20
    infos, st = L.lag_multilevel_solve(gpu_problem(case), 3, dev.put(T), dev.put(R), v, opt)
    print("multilevel", infos, flush=True)
    assert st == L.LAG_OK
    assert infos[-1]["converged"]
    # every level reduces its own objective
    assert all(i["J"] < i["J0"] for i in infos)
    vg = dev.get(v).reshape(OP.vel_shape)
    Jo = O.objective(OP, vg, T, R)["J"]
    assert abs(Jo - infos[-1]["J"]) <= 1e-5 * abs(Jo)
    assert infos[-1]["J"] < 0.2 * O.objective(OP, np.zeros(OP.vel_shape), T, R)["J"]
    # the finest level starts from the refined coarse solution, so it needs
    # fewer Gauss-Newton iterations than the coarsest level
    assert infos[-1]["iters"] <= infos[0]["iters"]


@pytest.mark.parametrize("img,vel", [((28, 20, 24), (8, 8, 8)), ((256, 256, 224), (64, 64, 64)),
                                     ((45, 36), (15, 18))], ids=["3d_ragged", "3d_256x256x224", "2d"])
def test_resample_to_velocity_grid(img, vel, torch, L):
    """Cell average onto the velocity grid at non-integer ratios (224 / 64)."""
    dim = len(img)
    OP = O.Problem(dim=dim, img_m=img, vel_m=vel)
    plan = L.Plan(L.make_problem(dim, img, vel, nsteps=2))
    f = f32(np.random.default_rng(sum(img)).uniform(0.0, 1.0, OP.n_points))
    out = torch.empty(int(np.prod(vel)), device="cuda")
    L.lag_resample_to_velocity_grid(plan, torch.from_numpy(f.astype(np.float32)).cuda(), out)
    assert relerr(out.cpu().numpy(), O.resample_to_velocity_grid(OP, f)) < 1e-6
    plan.close()
