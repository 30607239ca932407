"""Seeded synthetic inputs for the GMF hot path.

This package generates data and starting values only.  It holds none of the
estimator's arithmetic (no link derivatives, no gradients, no updates), so the
oracle and the HIP path can both consume its output without sharing code.
"""
from .generate import (Problem, make_problem, gen_poisson_small, gen_nb,
                       gen_gaussian_lowrank, gen_tiny, gen_nb_rows, mlp_init, holdout,
                       CONFIGS)

__all__ = ["Problem", "make_problem", "gen_poisson_small", "gen_nb",
           "gen_gaussian_lowrank", "gen_tiny", "gen_nb_rows", "mlp_init", "holdout",
           "CONFIGS"]
