"""CPU FP64 oracle -- test infrastructure only (see oracle/oracle.py)."""
from .oracle import *  # noqa: F401,F403
from .oracle import build, lib, cpqr, id_coefficients, compress, error_norms  # noqa: F401
