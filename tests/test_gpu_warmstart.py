"""Learned warm start: training on the solver's own solutions, then
prediction + Gauss-Newton refinement (64^3 images on a 32^3 velocity grid).

The network's benefit is a measurement (the benchmark reports solve times);
what is asserted here is the contract: training lowers the loss on the
solver's solutions, a warm-started solve meets the same stopping test as a
solve from zero (|g| <= gtol |g(v = 0)|), and the prediction itself moves
the objective below its value at v = 0 on held-out pairs.
"""

import numpy as np
import pytest

from synthetic import blob_image, fourier_velocity

pytestmark = pytest.mark.gpu

IMG, VEL, N = (64, 64, 64), (32, 32, 32), 5


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


def make_pairs(torch, L, plan, templates, seeds):
    pairs = []
    n = plan.n_points
    phi = torch.empty(3 * n, device="cuda")
    for j, T in enumerate(templates):
        for s in seeds:
            vt = torch.from_numpy(fourier_velocity(VEL, 3, 0.05, s).astype(np.float32).ravel()).cuda()
            L.lag_trace(plan, vt, -1, phi)
            R = torch.empty(n, device="cuda")
            L.lag_transport(plan, T, phi, R)
            pairs.append((T, R))
    return pairs


def test_train_predict_refine(torch, L):
    from paper_1703_04446_amd import warmstart as WS
    prob = L.make_problem(3, IMG, VEL, nsteps=N, alpha=1e-2, jac_blocks=8)
    plan = L.Plan(prob)
    templates = [torch.from_numpy(blob_image(IMG, 8, 7000 + j).astype(np.float32).ravel()).cuda()
                 for j in range(2)]
    train_pairs = make_pairs(torch, L, plan, templates, range(7100, 7106))
    test_pairs = make_pairs(torch, L, plan, templates, range(7200, 7202))
    opts = L.lag_gn_default_options()
    data = WS.solve_targets(plan, train_pairs, opts)
    assert all(d[3]["converged"] for d in data)
    cfg = L.lag_cnn_default_config()
    cfg.size = VEL[0]
    for i, c in enumerate((16, 16, 32, 32)):
        cfg.channels[i] = c
    net = L.Cnn(cfg)
    losses = WS.train(net, data, steps=120, lr=2e-3, seed=1)
    print("loss", losses[:3], "...", losses[-3:], flush=True)
    assert np.all(np.isfinite(losses))
    assert losses[-12:].mean() < 0.7 * losses[:6].mean()
    out3 = torch.zeros(3, dtype=torch.float64, device="cuda")
    u = torch.empty(plan.n_points, device="cuda")
    for T, R in test_pairs:
        v0 = torch.zeros(plan.n_unknowns, device="cuda")
        vp = torch.empty_like(v0)
        plain = WS.plain_solve(plan, T, R, v0, opts)
        Tc, Rc = WS.velocity_grid_inputs(plan, T, R)
        WS.predict(net, Tc, Rc, vp)
        L.lag_objective(plan, vp, T, R, u, out3)
        J_pred = out3[0].item()
        warm = WS.warm_solve(plan, net, T, R, vp, opts)
        print(f"plain iters {plain['iters']} J {plain['J']:.4e}; warm iters {warm['iters']} "
              f"J0 {warm['J0']:.4e} (J(0) {plain['J0']:.4e}) J {warm['J']:.4e}", flush=True)
        assert warm["converged"] and plain["converged"]
        assert warm["gnorm"] <= opts.gtol * warm["g0"] * (1 + 1e-12)
        assert abs(warm["g0"] - plain["g0"]) <= 1e-6 * plain["g0"]
        assert abs(J_pred - warm["J0"]) <= 1e-6 * abs(J_pred)
        assert J_pred < plain["J0"]
    net.close()
    plan.close()
