"""PCG with the stopping test on the device, replayed as a captured HIP graph.

The graph variant runs the same kernels in the same order as the
host-driven PCG, and every operator sums in integer fixed point with fixed
reduction trees (assembled and matrix-free alike), so its iterates are
identical bit for bit to the eager ones.  Every graph is replayed several
times with the program's own eager work and synchronisations in between,
and each replay is checked against the eager result.
"""

import numpy as np
import pytest

import oracle as O
from cases import SMALL_CASES, gpu_problem, oracle_problem, relerr
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


def rhs(case, OP, T, v, seed):
    """A Gauss-Newton right-hand side: minus the gradient at v (oracle)."""
    vt = case.velocity(seed_off=seed)
    R = O.objective(OP, vt, T, np.zeros(OP.n_points))["u"]
    g, _ = O.gradient(OP, v, T, R)
    return f32(-np.asarray(g))


@pytest.mark.parametrize("per_graph", [1, 3, 4])
def test_assembled_graph_pcg_is_bitwise_eager(per_graph, torch, L):
    case = SMALL_CASES[0]
    dev = Dev(torch)
    OP = oracle_problem(case)
    prob = gpu_problem(case)
    prob.jac_blocks = 16
    plan = L.Plan(prob)
    T, v = f32(case.template()), f32(case.velocity())
    b = rhs(case, OP, T, v, 3)
    assert L.lag_jacobian_assemble(plan, dev.put(v), dev.put(T))
    db = dev.put(b)
    xe = dev.empty(plan.n_unknowns)
    ie = L.lag_pcg_assembled(plan, None, db, xe, tol=1e-3, maxit=40)
    ref = xe.clone()
    for rep in range(3):
        xg = dev.empty(plan.n_unknowns)
        ig = L.lag_pcg_assembled_graph(plan, None, db, xg, tol=1e-3, maxit=40, iters_per_graph=per_graph)
        torch.cuda.synchronize()
        assert ig["iters"] == ie["iters"] and ig["matvecs"] == ie["matvecs"], (ig, ie)
        assert abs(ig["relres"] - ie["relres"]) <= 1e-12 * max(ie["relres"], 1e-30)
        assert torch.equal(xg, ref), f"replay {rep}"
        # eager work between replays: an eager solve of another right-hand side
        xo = dev.empty(plan.n_unknowns)
        L.lag_pcg_assembled(plan, None, dev.put(rhs(case, OP, T, v, 4 + rep)), xo, tol=1e-3, maxit=40)
        torch.cuda.synchronize()
    plan.close()


def test_graph_pcg_iteration_cap(torch, L):
    """A cap that is not a multiple of the captured iterations is honoured."""
    case = SMALL_CASES[0]
    dev = Dev(torch)
    OP = oracle_problem(case)
    prob = gpu_problem(case)
    prob.jac_blocks = 16
    plan = L.Plan(prob)
    T, v = f32(case.template()), f32(case.velocity())
    assert L.lag_jacobian_assemble(plan, dev.put(v), dev.put(T))
    db = dev.put(rhs(case, OP, T, v, 3))
    xe, xg = dev.empty(plan.n_unknowns), dev.empty(plan.n_unknowns)
    ie = L.lag_pcg_assembled(plan, None, db, xe, tol=1e-12, maxit=5)
    ig = L.lag_pcg_assembled_graph(plan, None, db, xg, tol=1e-12, maxit=5, iters_per_graph=2)
    assert ie["iters"] == ig["iters"] == 5
    assert torch.equal(xe, xg)
    ig0 = L.lag_pcg_assembled_graph(plan, None, db, xg, tol=0.5, maxit=0, iters_per_graph=4)
    assert ig0["iters"] == 0 and float(xg.abs().max()) == 0.0
    plan.close()


@pytest.mark.parametrize("case", [SMALL_CASES[4], SMALL_CASES[3], SMALL_CASES[6]],
                         ids=[SMALL_CASES[i].name for i in (4, 3, 6)])
def test_matrix_free_graph_pcg(case, torch, L):
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    T, v = f32(case.template()), f32(case.velocity())
    b = rhs(case, OP, T, v, 3)
    dv, dT, db = dev.put(v), dev.put(T), dev.put(b)
    xe = dev.empty(plan.n_unknowns)
    ie = L.lag_pcg(plan, dv, dT, None, db, xe, tol=0.1, maxit=30)
    # the eager solve itself repeats bit for bit
    xr = dev.empty(plan.n_unknowns)
    ir = L.lag_pcg(plan, dv, dT, None, db, xr, tol=0.1, maxit=30)
    assert ir["iters"] == ie["iters"] and torch.equal(xr, xe)
    for rep in range(2):
        xg = dev.empty(plan.n_unknowns)
        ig = L.lag_pcg_graph(plan, dv, dT, None, db, xg, tol=0.1, maxit=30, iters_per_graph=3)
        torch.cuda.synchronize()
        print(case.name, ie, ig, flush=True)
        assert ig["iters"] == ie["iters"], (ig, ie)
        assert torch.equal(xg, xe), f"replay {rep}: {relerr(dev.get(xg), dev.get(xe)):.2e}"
        L.lag_pcg(plan, dv, dT, None, db, dev.empty(plan.n_unknowns), tol=1e-1, maxit=5)
        torch.cuda.synchronize()
    plan.close()


def test_gn_solve_with_graph_pcg(torch, L):
    case = SMALL_CASES[0]
    dev = Dev(torch)
    OP = oracle_problem(case)
    prob = gpu_problem(case)
    prob.jac_blocks = 16
    T = f32(case.template())
    R = f32(O.objective(OP, case.velocity(), T, np.zeros(OP.n_points))["u"])
    out = []
    for gi in (0, 4):
        plan = L.Plan(prob)
        o = L.lag_gn_default_options()
        o.pcg_maxit, o.graph_iters = 20, gi
        v = torch.zeros(plan.n_unknowns, device="cuda")
        info = L.lag_gn_solve(plan, dev.put(T), dev.put(R), v, o)
        out.append((info, v.clone()))
        plan.close()
    (i0, v0), (i4, v4) = out
    print(i0, i4, flush=True)
    assert i0["converged"] and i4["converged"]
    assert i0["iters"] == i4["iters"] and i0["pcg_iters"] == i4["pcg_iters"]
    assert torch.equal(v0, v4)
