"""MI355X (gfx950) implementation of the data-parallel hot path of
mutation-guided quadratic optimisation (arXiv 2605.06921): batched projected
gradient ascent on the relaxed MIS and MaxCut objectives with exact integer
rounding, evaluation, 1-flip local search and the mutation reset, behind the
C-ABI library libmqo (include/mqo.h).

``paper_2605_06921_amd.mqo`` is the ctypes binding; it fails on import when
libmqo.so has not been built (``paper_2605_06921_amd.build.build()``).
"""
from . import mqo  # noqa: F401
from .mqo import (DeviceGraph, MqoError, Objective, UnrolledPGA, Workspace, init_iterate,  # noqa: F401
                  local_search, objective, objective_grad, pair_search, pga_steps, reset, round_evaluate, solve,
                  solve_maxcut, solve_mis, toy_reset, unrolled_backward, unrolled_forward, unrolled_pga,
                  validate_graph_host)
