"""CPU oracle: test infrastructure, not part of the product.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the HIP library.
"""
from .fe_oracle import (  # noqa: F401
    Oracle, gauss_legendre, gll_nodes, lagrange_values, lagrange_derivatives,
    cell_dof_map, constrained_mask, nodes_per_dir, chebyshev_filter,
)
