"""Seeded synthetic galaxy / random catalogs (inputs only; no estimator arithmetic).

Shared by the tests, the oracle timing leg of the bench and the GPU bench; it
holds none of the method's arithmetic (no painting, no harmonics, no binning).
"""
from .catalogs import (WORKLOADS, Workload, make_workload_catalog, uniform_cube,  # noqa: F401
                       cone_shell_uniform, lognormal_catalog, tiny_node_catalog,
                       serving_stream, to_xyzw)
