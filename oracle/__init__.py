"""FP64 CPU oracle of the coupled three-population phase-change LBM step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that
the HIP path is checked against.  Only the test-suite, the package's smoke
check and the benchmark's CPU-baseline leg may import it; the product path
(the C-ABI library and its Python binding) never imports, links or calls
anything here, and this package imports nothing from the product.

Parity unpinned: the oracle functions are pinned by closed forms and exact
invariants (see tests/test_oracle_*.py); the parts listed under "parity
unpinned" in the module docstring of :mod:`oracle.lbm_oracle` have no such
pin beyond self-consistency.
"""
from .lbm_oracle import (Lattice, lattice, Model, State, Macros)  # noqa: F401
