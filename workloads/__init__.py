"""Seeded synthetic graph generators shared by the tests, the benchmark and the
smoke check.

This module only builds graphs (vertex count, edge list, edge lengths) and
draws random parameters.  It holds none of the sampler's arithmetic: no mesh,
no matrices, no quadrature, no noise.  Both the CPU oracle and the GPU path
receive its output as plain arrays.
"""

from .graphs import (  # noqa: F401
    Graph,
    lattice,
    preferential_attachment,
    random_geometric,
    interval,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_c5_eval,
    config_c5_train,
    config_paper_ba,
)
