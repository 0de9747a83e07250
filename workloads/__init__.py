"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package holds input generation only: network weights, the L-inf box,
root pre-activation bounds by interval arithmetic, BaB split domains and
LP-implied cutting planes.  It contains none of the bound-propagation
arithmetic of GCP-CROWN (Theorem 3.1 of arXiv 2208.05740); each side
implements that independently.
"""
from .gen import (  # noqa: F401
    Edge, Node, Net, Splits, Cuts, Problem,
    make_workload, WORKLOAD_NAMES, make_problem, make_tiny, mlp_net, cnn_net, cnn_wide_net, resnet_net,
    crown_alpha_init,
    forward, ibp_bounds, unstable_index, num_relu_neurons,
)
