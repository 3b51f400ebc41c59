"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This package draws the random inputs of the benchmark workloads (orbital
centres, well depths, column-block sizes, orbital values) and evaluates the
synthetic potential field at points that the caller supplies.  It holds none
of the method's arithmetic: no quadrature, no shape functions, no BCSR
layout, no operator application.  The one piece of geometry it contains is the
a-priori support rule that decides which nodes of an orbital carry non-zero
values; this is part of the definition of the synthetic input (the paper's
orbitals are localised around atoms, Sec. 3.3), not of the operator.
"""

from .workloads import (  # noqa: F401
    ALL_FACES,
    CONFIGS,
    MeshSpec,
    Workload,
    custom_workload,
    support_nodes,
    make_workload,
    potential_at,
    orbital_values,
    orbital_values_generic,
    request_inputs,
)
