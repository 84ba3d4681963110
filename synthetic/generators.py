"""Seeded generators for synthetic registration inputs.

Conventions used everywhere in this repository:

* grid sizes are given x first: ``m = (mx, my)`` or ``(mx, my, mz)``;
* arrays are stored x fastest, i.e. NumPy C-order shape ``(my, mx)`` or
  ``(mz, my, mx)`` (the reverse of ``m``);
* velocity-shaped arrays have shape ``(nodes, d) + reversed(m)``, component 0
  being the x component;
* the domain is the periodic box ``[0, L_0) x ... x [0, L_{d-1})`` and cells
  are centred at ``(i + 1/2) h`` with ``h = L / m``.

The image model follows the workload description of Gaussian-blob phantoms
(centres uniform in the inner 70% of the box, widths sigma in [0.03, 0.1],
amplitudes in [0.5, 1]); the velocity model draws complex Gaussian Fourier
coefficients on the integer wave vectors with 0 < |k| <= K and rescales the
real field so that its largest pointwise Euclidean norm equals the requested
amplitude.  Both are input recipes only.
"""

from __future__ import annotations

import numpy as np


def _shape(m):
    return tuple(int(x) for x in reversed(m))


def cell_centres(m, extent=None):
    """Per-axis cell-centre coordinates ``[(i + 1/2) L_a / m_a]`` (x first)."""
    d = len(m)
    extent = (1.0,) * d if extent is None else tuple(extent[:d])
    return [(np.arange(m[a]) + 0.5) * (extent[a] / m[a]) for a in range(d)]


def blob_image(m, nblobs, seed, extent=None, density=False):
    """Sum of periodic isotropic Gaussian blobs sampled at cell centres.

    Returns a float64 array of shape ``reversed(m)``.  With ``density=True``
    the result is scaled to unit mass, ``sum(T) * prod(h) = 1``.
    """
    d = len(m)
    extent = (1.0,) * d if extent is None else tuple(float(e) for e in extent[:d])
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15, 0.85, size=(nblobs, d))
    sigmas = rng.uniform(0.03, 0.1, size=nblobs)
    amps = rng.uniform(0.5, 1.0, size=nblobs)
    xs = cell_centres(m, extent)
    # Separable periodic profiles: per blob and axis, the sum over the image
    # copies at offsets -L, 0, +L of the 1-D Gaussian factor.
    prof = []
    for a in range(d):
        c = centres[:, a, None] * extent[a]
        s = sigmas[:, None] * extent[a]
        g = np.zeros((nblobs, m[a]))
        for o in (-1.0, 0.0, 1.0):
            g += np.exp(-((xs[a][None, :] - c - o * extent[a]) ** 2) / (2.0 * s * s))
        prof.append(g)
    # sum over blobs of the outer products, in storage order (last axis = x)
    if d == 2:
        out = np.einsum("b,by,bx->yx", amps, prof[1], prof[0], optimize=True)
    else:
        out = np.einsum("b,bz,by,bx->zyx", amps, prof[2], prof[1], prof[0], optimize=True)
    if density:
        cell = float(np.prod([extent[a] / m[a] for a in range(d)]))
        out /= out.sum() * cell
    return out


def fourier_velocity(m, kmax, amplitude, seed, nodes=1):
    """Smooth periodic random velocity of shape ``(nodes, d) + reversed(m)``.

    Each time node is drawn independently: complex Gaussian coefficients on
    every integer wave vector with ``0 < |k|_2 <= kmax`` (per component), the
    real part of the inverse DFT, then one common scale per node so that
    ``max_x |v(x)|_2 = amplitude``.
    """
    d = len(m)
    rng = np.random.default_rng(seed)
    shape = _shape(m)
    # signed integer frequencies along each storage axis
    freqs = [np.fft.fftfreq(n, 1.0 / n) for n in shape]
    grids = np.meshgrid(*freqs, indexing="ij")
    k2 = sum(g * g for g in grids)
    support = (k2 > 0) & (k2 <= kmax * kmax)
    v = np.zeros((nodes, d) + shape, dtype=np.float64)
    for j in range(nodes):
        for c in range(d):
            coef = np.zeros(shape, dtype=np.complex128)
            nsup = int(support.sum())
            coef[support] = rng.standard_normal(nsup) + 1j * rng.standard_normal(nsup)
            v[j, c] = np.real(np.fft.ifftn(coef))
        peak = np.sqrt((v[j] ** 2).sum(axis=0)).max()
        if peak > 0:
            v[j] *= amplitude / peak
    return v


def random_direction(shape, seed, scale=1.0):
    """Standard-normal direction of the given shape, scaled to unit RMS * scale."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    return x * (scale / np.sqrt(np.mean(x * x)))

