"""FP64 CPU oracle for the bond-based PMB peridynamics step (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and this
package never imports the product.  The arithmetic lives in ``pd_oracle.c`` (plain
C, built with ``gcc -O2 -ffp-contract=off``); this module only marshals arguments,
plus ``cstep.py``, an independent NumPy re-statement used for complex-step
derivatives.
"""
from .oracle import (OracleSim, build, family, bc_arrays, damage, force,  # noqa: F401
                     apply_jt, adjoint_ec, lib_path)
