"""Shared parity-case descriptions for the GPU tests.

A case is a workload (grid sizes, model, regulariser, steps) plus seeded
inputs from ``synthetic``.  ``oracle_problem`` and ``gpu_problem`` build the
two independent problem objects from the same description.
"""

from dataclasses import dataclass, replace

import numpy as np

import oracle as O
from synthetic import blob_image, fourier_velocity, random_direction


@dataclass(frozen=True)
class Case:
    name: str
    dim: int
    img_m: tuple
    vel_m: tuple
    nodes: int = 1
    model: str = "transport"
    reg: str = "diffusion"
    nsteps: int = 4
    alpha: float = 1e-2
    gamma: float = 0.0
    nblobs: int = 6
    kmax: int = 3
    amplitude: float = 0.06
    seed: int = 7000
    extent: tuple = (1.0, 1.0, 1.0)

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def vel_shape(self):
        return (self.nodes, self.dim) + tuple(reversed(self.vel_m))

    @property
    def n_points(self):
        return int(np.prod(self.img_m))

    def template(self):
        return blob_image(self.img_m, self.nblobs, self.seed, extent=self.extent,
                          density=(self.model == "continuity")).ravel()

    def velocity(self, scale=1.0, seed_off=1):
        return scale * fourier_velocity(self.vel_m, self.kmax, self.amplitude,
                                        self.seed + seed_off, nodes=self.nodes)

    def direction(self, i=0):
        return random_direction(self.vel_shape, self.seed + 100 + i)

    def image_field(self, i=0):
        return random_direction((self.n_points,), self.seed + 200 + i)


def oracle_problem(c: Case):
    return O.Problem(dim=c.dim, img_m=c.img_m, vel_m=c.vel_m, nodes=c.nodes, model=c.model,
                     reg=c.reg, nsteps=c.nsteps, alpha=c.alpha, gamma=c.gamma,
                     extent=tuple(c.extent) + (1.0,) * (3 - len(c.extent)))


def gpu_problem(c: Case):
    import paper_1703_04446_amd as L
    return L.make_problem(c.dim, c.img_m, c.vel_m, nt_nodes=c.nodes, model=c.model, reg=c.reg,
                          nsteps=c.nsteps, alpha=c.alpha, gamma=c.gamma, extent=c.extent)


def relerr(a, b):
    """Parity error of ``a`` against the reference ``b``: the larger of the
    relative 2-norm error |a - b| / |b| and the largest entry error
    max|a - b| / max|b|.  The entry bound keeps a wrong entry in a small
    region (a brick edge, a tile halo) from hiding under the norm."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    e2 = np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
    einf = (np.abs(a - b).max() if b.size else 0.0) / (mb if mb > 0 else 1.0)
    return float(max(e2, einf))


# Cases small enough for the oracle to finish in seconds, chosen to cover
# 2-D/3-D, stationary/time-dependent, transport/continuity, equal and
# coarser velocity grids, bricks with ragged edges and FFT sizes with prime
# factors 2, 3 and 5.
SMALL_CASES = [
    Case("2d_transport_64", 2, (64, 64), (64, 64), nsteps=5, nblobs=8, kmax=4, amplitude=0.05, seed=1000),
    Case("2d_transport_ns_ragged", 2, (45, 36), (15, 18), nodes=3, nsteps=6, reg="curvature",
         alpha=1e-3, gamma=1e-3, amplitude=0.08, seed=7100),
    Case("2d_continuity_ns", 2, (40, 36), (20, 18), nodes=3, model="continuity", reg="curvature",
         nsteps=6, alpha=1e-3, amplitude=0.08, seed=7200),
    Case("2d_continuity_stat", 2, (30, 50), (30, 25), model="continuity", nsteps=3, amplitude=0.07,
         seed=7250),
    Case("3d_transport", 3, (24, 20, 16), (12, 10, 8), nsteps=4, nblobs=10, seed=7300),
    Case("3d_transport_ns", 3, (20, 18, 12), (10, 9, 6), nodes=2, nsteps=4, reg="curvature",
         alpha=1e-3, gamma=1e-4, seed=7400),
    Case("3d_continuity_ns", 3, (16, 12, 10), (8, 6, 5), nodes=2, model="continuity", nsteps=4,
         amplitude=0.07, seed=7500),
    Case("3d_transport_equal_grids", 3, (16, 16, 16), (16, 16, 16), nsteps=3, extent=(1.0, 1.2, 0.9),
         seed=7600),
]

# Smallest grids the ABI accepts: bricks and LDS tiles are larger than the
# whole grid (every tile wraps the periodic domain several times), FFT sizes
# 2 and 3, a single RK4 step.
MIN_CASES = [
    Case("2d_min_transport", 2, (2, 2), (2, 2), nsteps=1, nblobs=1, kmax=1, amplitude=0.3, seed=7700),
    Case("3d_min_transport", 3, (4, 2, 2), (2, 2, 2), nsteps=2, nblobs=1, kmax=1, amplitude=0.3, seed=7800),
    Case("2d_min_continuity", 2, (3, 2), (3, 2), model="continuity", nsteps=1, nblobs=1, kmax=1,
         amplitude=0.3, seed=7900, gamma=1e-3),
]
