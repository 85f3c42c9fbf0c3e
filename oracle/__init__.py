"""CPU FP64 oracle of the DDM-GNN preconditioned Krylov solve.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
calls it, links it or reads anything it writes.

Plain, slow, obviously correct numpy code in float64, written from the paper:

* ``decomp``  - overlapping sub-meshes (Sec. II.A: R_i, k_i), partition-of-unity
  weights, the Nicolaides coarse basis (Sec. II.A, eq. (7)), and the local DSS
  graphs with geometric edge features (Sec. III.B).
* ``dss``     - the DSS_theta forward pass (Sec. III.B, eqs. (14)-(18)).
* ``schwarz`` - the coarse problem and the DDM-GNN apply (Sec. III.A, eqs.
  (11)-(13) and the gluing step); the DDM-LU and one-level variants (eqs. (6)-(7)).
* ``krylov``  - PCG as Algorithm 1, flexible CG (truncated FCG(m)), restarted flexible
  GMRES, plain CG.
* ``train``   - the training loss of DSS_theta (the residual loss of Sec. II.B summed over
  the blocks, Sec. III.B) with its gradient by float64 autograd, and the Adam step.

Parity status of each function is stated in its docstring; every function is
pinned by tests except where a docstring says "parity unpinned".
"""
from . import decomp, dss, schwarz, krylov, train  # noqa: F401
