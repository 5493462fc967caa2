"""Plain CPU reference (the oracle) of the world step of arXiv 2302.09334.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The product package never imports it.
"""
from .oracle import (  # noqa: F401
    CTRL_CNN_LSTM,
    CTRL_GRU,
    DYN_BENCH,
    DYN_PAPER,
    NO_ACTION,
    OracleConfig,
    OracleWorld,
    build,
    cnn_eval,
    cnn_n_features,
    cnn_n_params,
    gauss_pair,
    gumbel,
    gru_eval,
    ln_unit,
    n_inputs,
    n_params,
    philox,
    sample_action,
    sincos_2pi,
    threshold_table,
)
