"""FP64 CPU reference for differentiable XPBD.

TEST INFRASTRUCTURE ONLY: the checker of the GPU library.  Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import it; the product package never does.

Every function here follows the paper step by step (forward: Sec. 3.1
Eq. xpbd / xpbdUpdateRule; exact adjoint: the chain rule per projection with
the partials of Sec. 4.3 and the adjoint recurrence of supplemental Sec. A;
implicit adjoint: Eq. adjointXPBD).  Constraint derivatives are exact
forward-mode automatic differentiation of each constraint's definition.

Pins (tests/test_oracle_*.py):
  * one distance constraint at zero compliance is satisfied after one
    projection; a two-particle spring matches its closed-form implicit-Euler
    recurrence and derivative; free fall matches its closed form;
  * constraint gradients and Hessian-vector products against central finite
    differences; the element invariants of Sec. 4.3.1 (zero force sum, zero
    torque, symmetric Hessian with zero block-row sums); dihedral geometry;
  * momentum conservation and rigid equivariance of whole rollouts;
  * the exact adjoint against central finite differences of whole rollouts
    on tiny meshes (every parameter group);
  * the exact adjoint converges to the implicit adjoint of Eq. adjointXPBD
    as the iteration count grows.
"""
from .oracle import (  # noqa: F401
    OracleScene, build_library, library_path, forward, adjoint, adjoint_implicit, psd_project, point_triangle_d2,
    constraint, rest_data, goal_l2, max_threads,
)
