"""Seeded synthetic workloads for filtered nearest-neighbour search.

This package only draws random inputs (vectors, per-item attributes, query
vectors and query filters).  It holds none of the search method's arithmetic:
no distances, no filter evaluation, no graph logic.  Both the CPU oracle and
the GPU library consume what it produces.
"""
from .gen import (  # noqa: F401
    FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_BOOLEAN, FILTER_TABLE,
    Workload, mixture, zipf_label_sets, range_filters, make_config,
    encode_filters, CONFIG_NAMES,
)
