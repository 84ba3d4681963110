"""Workload descriptions: grid sizes, step counts, weights and seeds.

Each workload names the synthetic phantom recipe it is drawn from.  The
reference image R is *not* produced here: it is the template transported (or
pushed forward) by the ground-truth velocity, which needs the method itself,
so the oracle computes it for tests and the GPU path computes it for the
benchmark.

Sizes are x first.  ``nodes`` is the number of velocity time nodes (1 means a
stationary velocity; otherwise the nodes sit at t_j = j/(nodes-1)).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .generators import blob_image, fourier_velocity, random_direction


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    img_m: tuple
    vel_m: tuple
    nodes: int
    model: str          # "transport" | "continuity"
    reg: str            # "diffusion" | "curvature"
    nsteps: int
    alpha: float
    gamma: float
    nblobs: int
    kmax: int
    amplitude: float
    seed_base: int
    pcg_maxit: int = 50
    pcg_tol: float = 0.1
    extent: tuple = field(default=(1.0, 1.0, 1.0))

    # --- seeded inputs -------------------------------------------------
    def template(self):
        return blob_image(self.img_m, self.nblobs, self.seed_base,
                          extent=self.extent, density=(self.model == "continuity"))

    def velocity_true(self):
        return fourier_velocity(self.vel_m, self.kmax, self.amplitude,
                                self.seed_base + 1, nodes=self.nodes)

    def direction(self, i):
        return random_direction(self.vel_shape, self.seed_base + 100 + i)

    def image_direction(self, i):
        return random_direction(tuple(reversed(self.img_m)), self.seed_base + 200 + i)

    # --- sizes -----------------------------------------------------------
    @property
    def vel_shape(self):
        return (self.nodes, self.dim) + tuple(reversed(self.vel_m))

    @property
    def img_shape(self):
        return tuple(reversed(self.img_m))

    @property
    def n_points(self):
        return int(np.prod(self.img_m))

    @property
    def n_unknowns(self):
        return int(self.nodes * self.dim * np.prod(self.vel_m))


# The five workload recipes (the first three and the last are single-pair
# registration problems; "batched" is described for completeness only).
WORKLOADS = {
    # 2-D 64^2, stationary, transport, RK4 N=5, 8 blobs, |k|<=4, A=0.05,
    # diffusion alpha=1e-2, PCG at most 20 iterations.
    "2d64_transport": Workload(
        name="2d64_transport", dim=2, img_m=(64, 64), vel_m=(64, 64), nodes=1,
        model="transport", reg="diffusion", nsteps=5, alpha=1e-2, gamma=0.0,
        nblobs=8, kmax=4, amplitude=0.05, seed_base=1000, pcg_maxit=20),
    # 2-D 256^2 densities, continuity, 4 time intervals (5 nodes) on 128^2,
    # 8 RK4 steps per interval, |k|<=6, A=0.08, curvature alpha=1e-3.
    "2d256_continuity": Workload(
        name="2d256_continuity", dim=2, img_m=(256, 256), vel_m=(128, 128), nodes=5,
        model="continuity", reg="curvature", nsteps=32, alpha=1e-3, gamma=0.0,
        nblobs=8, kmax=6, amplitude=0.08, seed_base=2000),
    # 3-D 128^3 images, stationary 64^3 velocity, transport, RK4 N=10,
    # 24 blobs, |k|<=4, A=0.05 (regulariser unstated: diffusion 1e-2).
    "3d128_transport": Workload(
        name="3d128_transport", dim=3, img_m=(128, 128, 128), vel_m=(64, 64, 64), nodes=1,
        model="transport", reg="diffusion", nsteps=10, alpha=1e-2, gamma=0.0,
        nblobs=24, kmax=4, amplitude=0.05, seed_base=3000),
    # 3-D 256x256x224 transport on a 64^3 stationary velocity (N unstated: 10).
    "3d256_transport": Workload(
        name="3d256_transport", dim=3, img_m=(256, 256, 224), vel_m=(64, 64, 64), nodes=1,
        model="transport", reg="diffusion", nsteps=10, alpha=1e-2, gamma=0.0,
        nblobs=24, kmax=4, amplitude=0.05, seed_base=5000),
}


def workload(name, **overrides):
    """Look up a workload by name, optionally replacing some fields."""
    w = WORKLOADS[name]
    if overrides:
        d = dict(w.__dict__)
        d.update(overrides)
        w = Workload(**d)
    return w
