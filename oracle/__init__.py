"""Plain CPU reference (the oracle) of the world step of arXiv 2302.09334.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The product package never imports it.
"""
from .oracle import (  # noqa: F401
    OracleConfig,
    OracleWorld,
    build,
    gauss_pair,
    gru_eval,
    ln_unit,
    n_inputs,
    n_params,
    philox,
    sincos_2pi,
    threshold_table,
)
