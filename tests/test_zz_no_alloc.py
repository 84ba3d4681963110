"""lag_pushforward_noalloc (no plan; scratch in a fixed device array) against
lag_pushforward (plan-owned scratch): the same kernels, so the results must
be bitwise equal.  Two calls in a row, the second on a smaller problem (the
shared scratch keeps the first call's contents), then a problem close to
the scratch's capacity; the small cases are also checked against the
oracle's push-forward and for mass conservation."""

import numpy as np
import pytest

import oracle as O
from synthetic import blob_image

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


def _inputs(img, seed):
    d = len(img)
    rng = np.random.default_rng(seed)
    n = int(np.prod(img))
    T = blob_image(img, 6, seed, density=True).ravel().astype(np.float32)
    h = 1.0 / np.array(img, dtype=np.float64)
    phi = np.concatenate([rng.uniform(-3.0, 3.0, n) * h[a] for a in range(d)]).astype(np.float32)
    return T, phi


def _compare(torch, L, img, seed, oracle_check):
    d = len(img)
    prob = L.make_problem(d, img, tuple(max(2, m // 2) for m in img), model="continuity")
    T, phi = _inputs(img, seed)
    Td, phid = torch.from_numpy(T).cuda(), torch.from_numpy(phi).cuda()
    n = T.size
    u0 = torch.full((n,), float("nan"), device="cuda")
    u1 = torch.full((n,), float("nan"), device="cuda")
    print(f"noalloc push-forward {img}: {n} cells", flush=True)
    L.lag_pushforward_noalloc(prob, Td, phid, u1)
    plan = L.Plan(prob)
    L.lag_pushforward(plan, Td, phid, u0)
    torch.cuda.synchronize()
    a, b = u1.cpu().numpy(), u0.cpu().numpy()
    plan.close()
    assert np.array_equal(a, b), np.abs(a - b).max()
    assert abs(a.astype(np.float64).sum() - T.astype(np.float64).sum()) <= 1e-6 * T.astype(np.float64).sum()
    if oracle_check:
        P = O.Problem(dim=d, img_m=img, vel_m=tuple(max(2, m // 2) for m in img), model="continuity")
        ref = O.pushforward(P, T.astype(np.float64), phi.astype(np.float64).reshape(d, n))
        err = max(np.linalg.norm(a - ref) / np.linalg.norm(ref), np.abs(a - ref).max() / np.abs(ref).max())
        assert err < 1e-5, err


def test_noalloc_pushforward_matches_plan_entry_point(torch, L):
    _compare(torch, L, (48, 40, 36), 9101, True)     # first call on this device
    _compare(torch, L, (37, 29), 9102, True)         # second call, smaller problem
    _compare(torch, L, (1280, 1280), 9103, False)    # near the scratch's capacity (59 of 64 MiB)
    _compare(torch, L, (96, 90, 100), 9104, False)   # 3-D near the capacity (45 of 64 MiB)
