"""MI355X (gfx950) library for the INLA hyperparameter objective on
block-tridiagonal-with-arrowhead precision matrices: assembly, block Cholesky
and log-determinants, substitution, selected inversion, batched f(theta) and
its exact gradient.  The compute runs in libinla_bta.so (hand-written HIP);
this package only marshals arguments.
"""
from .binding import (  # noqa: F401
    Bta,
    BtaTensors,
    EvalState,
    InlaError,
    InlaObjective,
    Model,
    assemble,
    build_id,
    eval_f,
    eval_f_grad,
    eval_f_grad_poisson,
    factor_logdet,
    factor_logdet_noalloc,
    header_functions,
    integrate,
    lib,
    minimize,
    objective,
    profile_begin,
    profile_end,
    release_workspace,
    selinv,
    solve,
)
