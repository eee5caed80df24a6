"""CPU FP64 reference ("oracle") for the ph-AFQMC walker two-body local energy.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, calls or links
anything here; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP path: the two sides meet
only through arrays produced by the seeded input generator.

The reference follows Weber et al., "A Localized-Orbital Energy Evaluation for
Auxiliary-Field Quantum Monte Carlo" (arXiv 2202.00832):

* ``fock``    - second-quantised brute force of <Psi_T|H2|phi>/<Psi_T|phi>
                (Sec. 2.1.1, Eq. 9) on tiny Fock spaces; pins everything else.
* ``energy``  - Green's function (Eq. 11, 14, 15), generalised Wick E2 (Eq. 10),
                half-rotated Cholesky route (Sec. 2.2, Eq. 16), HR-ERI route
                (Eq. 17), pair SVD compression (Sec. 2.3.1, Eq. 18) and the LO
                energy (Sec. 2.3.2, Eq. 19 and Eq. 22), plus the a-priori error
                bound of the truncation.
* ``multidet`` - multi-determinant (CAS-type) trials: the weighted sum of
                Eq. 12 by its definition, and the LO energy by the
                Sherman-Morrison-Woodbury steps of Eq. 20-23.

Every function is plain numpy in float64 / complex128, without blocking,
fusion or reordering beyond what the equations state.
"""
from . import energy, fock, multidet  # noqa: F401
