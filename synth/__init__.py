"""Seeded synthetic instances for domain propagation (inputs only).

Nothing here computes activities, candidates or any other step of the
propagation method; the module only draws matrices, bounds and sides.
Both the GPU library's tests/benchmarks and the oracle take their inputs
from here.
"""
from .instances import (  # noqa: F401
    BASE_SEED,
    Instance,
    cached,
    config0,
    config1,
    config2,
    config3_matrix,
    config3_nodes,
    config4_pool,
    config4_requests,
    from_rows,
    branch_children,
    code_edges,
    hard_sums,
    layout_mix,
    request_bounds,
    node_bounds,
    random_small,
)
