"""Plain FP64 CPU oracle for Schwarz-preconditioned CG on finite cell systems.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
library's product path never does.  It shares no code with the GPU library:
the two meet only at the seeded problem descriptions of ``fcgen``.

Everything here is written for a reader to check against the paper by eye:
no blocking, fusion or reordering beyond what the definitions state.

Modules
-------
basis     integrated Legendre shape functions and Gauss-Legendre rules
geometry  physical-domain indicator, exact box classification, octree leaves
assemble  finite cell weak form (Eq. 1 with the indicator alpha), assembly
schwarz   additive Schwarz blocks (Eq. 6), pseudo-inverses (Eqs. 9-11),
          Algorithm 1 with its diagonal-scaling fallback
pcg       preconditioned CG, the stopping criterion (Eq. 12), the energy
          error (Eq. 13) and a direct reference solve
ebe       element-by-element forms of A and S (no global matrix), for the
          CPU timing of the full benchmark problem
"""
