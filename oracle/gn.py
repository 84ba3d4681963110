"""PCG and inexact Gauss-Newton with Armijo line search (oracle; tests only).

Sec. 3.2: the search direction solves H(v_i) dv = -d_v J(v_i) (eq. solveGN)
by preconditioned conjugate gradients; the update v_{i+1} = v_i + mu dv takes
mu from an Armijo backtracking line search.  Sec. 4.1 sets PCG to at most 50
iterations with relative residual tolerance 0.1.

Readings (the paper defers the stopping rules to FAIR's defaults, which it
does not list):

* PCG starts at x0 = 0 and stops when |r_k|_2 <= tol |b|_2 or after maxit
  iterations; p^T H p <= 0 is reported as a breakdown.
* Gauss-Newton stops when |g_k| <= gtol |g(v = 0)| (gtol = 1e-2) or after
  max_gn iterations; Armijo uses c1 = 1e-4, step halving, at most 10
  halvings, after which the solve stops with a line-search failure.
"""

from __future__ import annotations

import numpy as np

from .grid import Problem
from .objective import objective, gradient, hessmat
from .precond import spectral_precond_apply


def pcg(apply_H, b, apply_M=None, tol=0.1, maxit=50):
    """Preconditioned CG for H x = b.  Returns (x, info dict)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = float(np.linalg.norm(b.ravel()))
    info = {"iters": 0, "relres": 1.0, "breakdown": False, "matvecs": 0}
    if nb == 0.0:
        info["relres"] = 0.0
        return x, info
    z = apply_M(r) if apply_M is not None else r.copy()
    p = z.copy()
    rz = float(np.vdot(r, z))
    for it in range(maxit):
        if np.linalg.norm(r.ravel()) <= tol * nb:
            break
        Hp = apply_H(p)
        info["matvecs"] += 1
        pHp = float(np.vdot(p, Hp))
        if pHp <= 0.0:
            info["breakdown"] = True
            break
        a = rz / pHp
        x = x + a * p
        r = r - a * Hp
        info["iters"] = it + 1
        z = apply_M(r) if apply_M is not None else r.copy()
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    info["relres"] = float(np.linalg.norm(r.ravel())) / nb
    return x, info


def gn_solve(prob: Problem, T, R, v0=None, gtol=1e-2, max_gn=50, c1=1e-4,
             max_halvings=10, pcg_tol=0.1, pcg_maxit=50, callback=None):
    """Inexact Gauss-Newton-Krylov solve of min_v J(v).  Returns (v, history)."""
    v = np.zeros(prob.vel_shape) if v0 is None else np.array(v0, dtype=np.float64).reshape(prob.vel_shape)
    g_zero, _ = gradient(prob, np.zeros(prob.vel_shape), T, R)
    g0 = float(np.linalg.norm(g_zero.ravel()))
    hist = {"J": [], "gnorm": [], "pcg_iters": [], "mu": [], "status": "maxit"}
    for it in range(max_gn):
        g, obj = gradient(prob, v, T, R)
        gn = float(np.linalg.norm(g.ravel()))
        hist["J"].append(obj["J"])
        hist["gnorm"].append(gn)
        if callback is not None:
            callback(it, v, obj, g)
        if gn <= gtol * g0:
            hist["status"] = "converged"
            break
        dv, info = pcg(lambda p: hessmat(prob, v, T, p), -g,
                       lambda r: spectral_precond_apply(prob, r),
                       tol=pcg_tol, maxit=pcg_maxit)
        hist["pcg_iters"].append(info["iters"])
        slope = float(np.vdot(g, dv))
        mu = 1.0
        accepted = False
        for _ in range(max_halvings + 1):
            Jt = objective(prob, v + mu * dv, T, R)["J"]
            if Jt <= obj["J"] + c1 * mu * slope:
                accepted = True
                break
            mu *= 0.5
        if not accepted:
            hist["status"] = "linesearch_failed"
            break
        hist["mu"].append(mu)
        v = v + mu * dv
    hist["g0"] = g0
    return v, hist
