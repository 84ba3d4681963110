"""Spectral preconditioner (oracle; test infrastructure only).

Sec. 3.2 (PCG paragraph): the Hessian of the regulariser is block diagonal,
one block per velocity component (and time node), each a structured
discretised differential operator; the preconditioner applies its
(pseudo-)inverse by a fast transform, optionally shifted by gamma I.

Readings:

* On the periodic grid used here the blocks are circulant, so the transform
  is the DFT (the paper's padded, Neumann-type grid needs a DCT).  The block
  of node j is M_j = alpha h_v^d w_j A + gamma I with A = -Laplace_h or
  (Laplace_h)^2; its symbol is mu(k) = alpha h_v^d w_j lambda_A(k) + gamma,
  lambda_{-Laplace}(k) = sum_a (4 / h_a^2) sin^2(pi k_a / m_a).
* Pseudo-inverse: when gamma = 0 the constant mode has mu(0) = 0; it is
  given the smallest nonzero eigenvalue of the same block instead, so the
  preconditioner stays symmetric positive definite.
"""

from __future__ import annotations

import numpy as np

from .grid import node_weights


def _lambda_A(prob):
    """Eigenvalues of A on the periodic velocity grid, storage-order shape."""
    shape = tuple(reversed(prob.vel_m[: prob.dim]))
    lam = np.zeros(shape)
    h = prob.h_vel
    for a in range(prob.dim):
        ax = prob.dim - 1 - a
        k = np.arange(prob.vel_m[a])
        la = (4.0 / h[a] ** 2) * np.sin(np.pi * k / prob.vel_m[a]) ** 2
        sh = [1] * prob.dim
        sh[ax] = prob.vel_m[a]
        lam = lam + la.reshape(sh)
    if prob.reg == "curvature":
        lam = lam * lam
    return lam


def spectral_symbol(prob):
    """mu_j(k) for every node j, after the pseudo-inverse rule for mu = 0."""
    lam = _lambda_A(prob)
    w = node_weights(prob)
    mus = []
    for j in range(prob.nodes):
        mu = prob.alpha * prob.cell_vel * w[j] * lam + prob.gamma
        if mu.flat[0] == 0.0:
            nz = mu[mu > 0]
            if nz.size == 0:
                raise ValueError("regulariser block is identically zero")
            mu = mu.copy()
            mu.flat[0] = nz.min()
        mus.append(mu)
    return np.stack(mus)


def spectral_precond_apply(prob, r):
    """z = F^-1 [ F(r) / mu(k) ] per velocity component and time node."""
    r = np.asarray(r, dtype=np.float64).reshape(prob.vel_shape)
    mu = spectral_symbol(prob)
    z = np.empty_like(r)
    for j in range(prob.nodes):
        for c in range(prob.dim):
            z[j, c] = np.real(np.fft.ifftn(np.fft.fftn(r[j, c]) / mu[j]))
    return z
