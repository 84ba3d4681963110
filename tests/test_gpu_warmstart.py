"""Learned warm start: training on the solver's own solutions, then
prediction + Gauss-Newton refinement (64^3 images on a 32^3 velocity grid).

Asserted: training lowers the loss on the solver's solutions; a
warm-started solve meets the same stopping test as a solve from zero
(|g| <= gtol |g(v = 0)|); the objective the solver starts from is the
objective of the prediction; and the warm start pays off on held-out pairs
(new velocities): the prediction's objective is well below J(0) and the
refinement needs fewer Gauss-Newton iterations than the solve from zero.
Recipe and bars from GPU runs of this configuration (4 templates x 12
velocities, 3000 Adam steps at lr 5e-4): prediction objective 0.38 J(0)
on average, iterations 3.1 -> 2.1; bars: 0.6 J(0) and fewer iterations.
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
    for T in templates:
        for s in seeds:
            vt = torch.from_numpy(fourier_velocity(VEL, 4, 0.05, s).astype(np.float32).ravel()).cuda()
            L.lag_trace(plan, vt, -1, phi)
            R = torch.empty(n, device="cuda")
            L.lag_transport(plan, T, phi, R)
            pairs.append((T, R))
    return pairs


def test_train_predict_refine(torch, L):
    from paper_1703_04446_amd import warmstart as WS
    prob = L.make_problem(3, IMG, VEL, nsteps=N, alpha=1e-2, jac_blocks=8)
    plan = L.Plan(prob)
    templates = [torch.from_numpy(blob_image(IMG, 8, 9000 + j).astype(np.float32).ravel()).cuda()
                 for j in range(4)]
    train_pairs = make_pairs(torch, L, plan, templates, range(9100, 9112))
    test_pairs = make_pairs(torch, L, plan, templates, range(9500, 9503))
    opts = L.lag_gn_default_options()
    data = WS.solve_targets(plan, train_pairs, opts)
    assert all(d[3]["converged"] for d in data)
    cfg = L.lag_cnn_default_config()
    cfg.size = VEL[0]
    for i, c in enumerate((16, 16, 32, 32)):
        cfg.channels[i] = c
    net = L.Cnn(cfg)
    losses = WS.train(net, data, steps=3000, lr=5e-4, seed=1)
    print("loss", losses[:50].mean(), "->", losses[-50:].mean(), flush=True)
    assert np.all(np.isfinite(losses))
    assert losses[-50:].mean() < 0.5 * losses[:50].mean()
    out3 = torch.zeros(3, dtype=torch.float64, device="cuda")
    u = torch.empty(plan.n_points, device="cuda")
    ratios, it_plain, it_warm = [], [], []
    for T, R in test_pairs:
        v0 = torch.zeros(plan.n_unknowns, device="cuda")
        vp = torch.empty_like(v0)
        plain = WS.plain_solve(plan, T, R, v0, opts)
        Tc, Rc = WS.velocity_grid_inputs(plan, T, R)
        WS.predict(net, Tc, Rc, vp)
        L.lag_objective(plan, vp, T, R, u, out3)
        J_pred = out3[0].item()
        warm = WS.warm_solve(plan, net, T, R, vp, opts)
        assert warm["converged"] and plain["converged"]
        assert warm["gnorm"] <= opts.gtol * warm["g0"] * (1 + 1e-12)
        assert abs(warm["g0"] - plain["g0"]) <= 1e-6 * plain["g0"]
        assert abs(J_pred - warm["J0"]) <= 1e-6 * abs(J_pred)
        ratios.append(J_pred / plain["J0"])
        it_plain.append(plain["iters"])
        it_warm.append(warm["iters"])
    print(f"J_pred / J(0) {np.mean(ratios):.3f}; GN iterations plain {np.mean(it_plain):.2f} "
          f"warm {np.mean(it_warm):.2f}", flush=True)
    assert np.mean(ratios) < 0.6
    assert np.mean(it_warm) < np.mean(it_plain)
    net.close()
    plan.close()
