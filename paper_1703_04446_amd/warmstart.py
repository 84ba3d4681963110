"""Learned warm start for the Gauss-Newton solve.

A 3-D U-Net (``lag_cnn_*``, bf16 MFMA kernels) maps the template and the
reference, averaged over the cells of the velocity grid, to a stationary
velocity.  It is
trained on image pairs and the Gauss-Newton solutions that the solver itself
produces for them (``lag_gn_solve`` from v = 0); at solve time its
prediction is the starting value that ``lag_gn_solve`` refines.  The
stopping test is unchanged (|g| <= gtol |g(v = 0)|), so the refined solution
meets the same tolerance as a solve from zero and the network only changes
how many iterations that takes.

Everything here is orchestration of C-ABI calls on torch's current stream;
images and velocities are float32 device tensors in the layouts of the
C-ABI (x fastest; velocities component-major).
"""

from __future__ import annotations

import time

import numpy as np

from . import _lib as L


def velocity_grid_inputs(plan, T, R):
    """T and R averaged over the cells of the velocity grid (any ratio of
    image to velocity cells >= 1, lag_resample_to_velocity_grid).  The
    velocity grid must be a cube: it is the network's domain."""
    import torch
    p = plan.prob
    vel = [p.vel_m[a] for a in range(p.dim)]
    if p.dim != 3 or len(set(vel)) != 1:
        raise ValueError("the warm-start network needs a cubic 3-D velocity grid")
    n = vel[0] ** 3
    Tc = torch.empty(n, device=T.device, dtype=torch.float32)
    Rc = torch.empty(n, device=T.device, dtype=torch.float32)
    L.lag_resample_to_velocity_grid(plan, T, Tc)
    L.lag_resample_to_velocity_grid(plan, R, Rc)
    return Tc, Rc


def solve_targets(plan, pairs, options=None):
    """Gauss-Newton solutions from v = 0 for each (T, R): the training set.

    Returns a list of (Tc, Rc, v_star, info) with Tc, Rc on the velocity grid.
    """
    import torch
    out = []
    for T, R in pairs:
        v = torch.zeros(plan.n_unknowns, device=T.device, dtype=torch.float32)
        info = L.lag_gn_solve(plan, T, R, v, options)
        Tc, Rc = velocity_grid_inputs(plan, T, R)
        out.append((Tc, Rc, v, info))
    return out


def train(net, data, steps, lr=2e-3, seed=0, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam on (Tc, Rc, v_star) samples, one sample per step in shuffled
    epochs.  Returns the per-step losses (read once at the end)."""
    import torch
    rng = np.random.default_rng(seed)
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda")
    v = torch.empty(3 * net.n_voxels, device="cuda", dtype=torch.float32)
    order = []
    for i in range(steps):
        if not order:
            order = list(rng.permutation(len(data)))
        Tc, Rc, vs = data[order.pop()][:3]
        L.lag_cnn_backward(net, Tc, Rc, vs, v, losses[i:i + 1])
        L.lag_cnn_adam_step(net, lr, beta1, beta2, eps)
    return losses.cpu().numpy()


def predict(net, Tc, Rc, v):
    L.lag_cnn_forward(net, Tc, Rc, v)


def warm_solve(plan, net, T, R, v, options=None):
    """Predict a starting velocity with the network, then refine it with
    lag_gn_solve.  Returns the solver's info plus the wall time of both
    stages (seconds, synchronised)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tc, Rc = velocity_grid_inputs(plan, T, R)
    predict(net, Tc, Rc, v)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = L.lag_gn_solve(plan, T, R, v, options)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info["predict_s"] = t1 - t0
    info["solve_s"] = t2 - t1
    return info


def plain_solve(plan, T, R, v, options=None):
    """lag_gn_solve from v = 0, timed like warm_solve."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v.zero_()
    info = L.lag_gn_solve(plan, T, R, v, options)
    torch.cuda.synchronize()
    info["predict_s"] = 0.0
    info["solve_s"] = time.perf_counter() - t0
    return info
