"""MI355X-native stiff chemistry hot path: per-cell constant-volume reactor
integration (matrix-form rates, implicit BDF, bulk-sparse split) behind the
C ABI of libchem.so; this package is its thin ctypes binding."""
from .chem import (CHEM_OK, CHEM_W_INCOMPLETE, ChemError, Context, Mechanism, ST_DONE, ST_FAIL,  # noqa: F401
                   ST_KMAX, ST_SKIPPED, ST_SURR_OK, ST_SURR_REJ, ST_TINV, MLP, lib)
