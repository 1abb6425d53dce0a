"""CPU oracle for the multigrid curvature-energy minimisation (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

``liboracle.so`` is compiled from ``mgc_oracle.c`` (exact minimisation of the
discretised local energy) and ``fbs_oracle.c`` (the paper's forward-backward
splitting step with tangent-plane estimates) with gcc (FP64, optional OpenMP
across the blocks of one colour); see :func:`build`.
"""
from .oracle import (  # noqa: F401
    build, lib_path, OracleParams, SolveInfo, Oracle, default_levels, FbsParams, FbsOracle,
)
