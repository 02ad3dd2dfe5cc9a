"""CPU FP64 oracle for the INLA hyperparameter objective (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never
imports, links or executes anything in here.
"""
from .inla_oracle import *  # noqa: F401,F403
