"""FP64 CPU oracle for the Lagrangian Gauss-Newton-Krylov registration path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference against which the GPU library is checked.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the two
share no code: the only common dependency is the seeded input generator
package ``synthetic``, which holds none of the method's arithmetic.

Everything is float64 NumPy, vectorised over characteristics with explicit
Python loops over RK4 steps and stages, so that each step can be read against
the paper (Mang & Ruthotto, "A Lagrangian Gauss-Newton-Krylov solver for mass-
and intensity-preserving diffeomorphic image registration"):

* ``grid``        - cell-centred periodic grids, (bi/tri)linear interpolation
                    in space and linear interpolation in time (Sec. 3, the
                    space-time discretisation; Sec. 3.1, the interpolation I).
* ``lagrangian``  - RK4 characteristics with the forward derivative recursion
                    (Algorithm 1), the transport solve (eq. rhoEndIR), the
                    particle push-forward (eq. rhoEndOMT with delta = h), and
                    their Jacobian products (Sec. 3.2, derivative of u1).
* ``objective``   - SSD distance (eq. SSD), diffusion / curvature
                    regularisers (Sec. 2.1), gradient and Gauss-Newton
                    Hessian (Sec. 3.2).
* ``precond``     - the spectral preconditioner (Sec. 3.2, PCG paragraph).
* ``gn``          - PCG and inexact Gauss-Newton with Armijo line search
                    (eq. solveGN).
* ``multilevel``  - coarse-to-fine continuation (Sec. 3.2, last paragraph) and
                    the cell average onto the velocity grid.
* ``cnn``         - the warm-start U-Net (not in the paper; forward and
                    backward in FP64).

Readings of passages that are silent, ambiguous or garbled are listed in the
module docstrings where they are used.  Functions pinned only by
self-consistency are marked "parity unpinned" (none at present).
"""

from .grid import Problem, time_weights, node_weights
from .lagrangian import (trace, transport, pushforward, jvp, vjp,
                         trace_analytic)
from .objective import (ssd, regularizer_apply, regularizer_energy, objective,
                        gradient, hessmat, laplacian_apply)
from .precond import spectral_precond_apply, spectral_symbol
from .gn import pcg, gn_solve
from .multilevel import (restrict_image, prolong_velocity, coarsen_problem, multilevel_solve,
                         resample_to_velocity_grid)

__all__ = [
    "Problem", "time_weights", "node_weights",
    "trace", "transport", "pushforward", "jvp", "vjp", "trace_analytic",
    "ssd", "regularizer_apply", "regularizer_energy", "objective", "gradient",
    "hessmat", "laplacian_apply",
    "spectral_precond_apply", "spectral_symbol",
    "pcg", "gn_solve",
    "restrict_image", "prolong_velocity", "coarsen_problem", "multilevel_solve",
    "resample_to_velocity_grid",
]
