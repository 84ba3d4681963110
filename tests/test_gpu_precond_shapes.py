"""Spectral preconditioner on grid shapes that select its other code paths.

In 3-D the x and y transforms of one plane run together in one block when
the plane's half spectrum fits in 64 KB of LDS; otherwise five separate line
passes run.  A 240 x 45 plane needs about 89 KB and takes the separate
passes; 15 x 9 takes the fused path with an odd x length (so the half
spectrum has no Nyquist column).  Both are compared with the oracle's FFT
inverse of the regulariser block (eq. (10) and its spectral inverse) to the
1e-5 relative bar of the other float32 parity tests.
"""

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


CASES = [
    Case("split_passes", 3, (240, 45, 3), (240, 45, 3), seed=9100),
    Case("split_passes_h2_nodes", 3, (240, 45, 3), (240, 45, 3), nodes=3, reg="curvature",
         gamma=0.05, seed=9200),
    Case("fused_odd_x", 3, (15, 9, 4), (15, 9, 4), seed=9300),
    Case("fused_odd_x_h2", 3, (15, 9, 4), (15, 9, 4), nodes=2, reg="curvature", seed=9400),
    Case("plane_2d_odd", 2, (15, 9), (15, 9), reg="curvature", gamma=0.1, seed=9500),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c.name)
def test_precond_shapes(case, torch, L):
    print("precond shape", case.name, case.vel_m, case.nodes, case.reg, flush=True)
    dev = Dev(torch)
    OP = oracle_problem(case)
    plan = L.Plan(gpu_problem(case))
    r = f32(np.random.default_rng(case.seed).standard_normal(case.vel_shape))
    z = dev.empty(plan.n_unknowns)
    L.spectral_precond_apply(plan, dev.put(r), z)
    err = relerr(dev.get(z), O.spectral_precond_apply(OP, r))
    print("  relerr", err, flush=True)
    assert err < 1e-5
