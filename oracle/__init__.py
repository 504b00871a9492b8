"""CPU FP64 oracle for the stochastic multiscale FEM (test infrastructure only).

This package is the slow, plainly written reference that the GPU path is
checked against.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product package never does, and the
two share no code.  See ``stomsfem_oracle.c`` for the plain path and
``rb.py`` / ``ri.py`` / ``mlp.py`` for the accelerations, ``sc.py`` for
sparse-grid collocation with dictionaries, ``twolevel.py`` for the
two-level Monte Carlo estimator, ``gauss.py`` for the Gaussian medium
and its local KL parametrization and ``loads.py`` for the element loads of
a bilinear source.
"""
from .core import *  # noqa: F401,F403
