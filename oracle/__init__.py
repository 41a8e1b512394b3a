"""FP64 CPU oracle for the twisted-mass Wilson Dslash, CG, fermion force and HMC.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import this package.  It shares no
code with the HIP library (no kernels, headers, tables or helpers); the only
module both sides read is the seeded input generator
``paper_1209_5942_amd.synth``, which draws random fields and holds none of the
method's arithmetic.

Every function is a plain, slow transcription of a definition in the paper
(Bach, Lindenstruth, Philipsen, Pinke, "Lattice QCD based on OpenCL",
arXiv:1209.5942), in FP64; each module header cites the passage it follows and
the reading taken where the paper is silent or garbled.  It is pinned by the
CPU tests in ``tests/test_oracle_*.py`` against closed forms, invariants and
brute force.
"""
from . import dirac, force, hmc  # noqa: F401
