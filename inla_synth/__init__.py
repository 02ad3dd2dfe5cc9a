"""Seeded synthetic inputs for the spatio-temporal latent Gaussian model.

This package only draws random numbers and lays out the observation design
(observation matrix A in CSR form, responses y, hyperparameter points).  It
contains none of the inference arithmetic: no precision matrices, no
factorizations, no objective.  Both the CPU oracle and the GPU library consume
what it returns.
"""
from .generate import (  # noqa: F401
    ModelData,
    THETA0,
    config_model,
    config_theta_batch,
    make_model,
    poisson_counts,
    uneven_batch,
    line_search_points,
    fd_stencil,
)
