"""Seeded synthetic inputs shared by the oracle tests and the GPU path."""
from .problems import (CONFIGS, GAUGE_WORKLOAD, Problem, haar_orthogonal, make_config,
                       make_general, make_near_degenerate, make_problem,
                       make_serving_request, nonorthogonal_gauge, redundant_gauge,
                       poisson_arrivals, random_amplitudes,
                       serving_request_shapes)

__all__ = ["CONFIGS", "GAUGE_WORKLOAD", "Problem", "haar_orthogonal", "make_config", "make_general",
           "make_near_degenerate", "make_problem", "make_serving_request", "nonorthogonal_gauge", "redundant_gauge",
           "poisson_arrivals", "random_amplitudes", "serving_request_shapes"]
