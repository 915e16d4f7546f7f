"""Plain FP64 CPU oracle for one KCM iteration (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It loads ``liboracle.so`` built from ``kcm_oracle.c`` with gcc
and shares nothing with the HIP library except the seeded inputs of
``synth``.
"""
from .oracle import (  # noqa: F401
    OracleChain,
    PairParams,
    SasaParams,
    StepRule,
    build,
    fk,
    fk_extend,
    fk_prefix,
    iterate,
    pair_forces,
    samples,
    sasa_atoms,
    sasa_definitional,
    sasa_events,
    sasa_forces,
    step,
    threads,
    torques,
)
from .mc import mc_minimize  # noqa: F401,E402
