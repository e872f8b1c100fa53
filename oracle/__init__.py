"""CPU oracle (test infrastructure only; never imported by the product path)."""
from .ttice_oracle import (TTICE, tt_svd, tt_full, truncation_rank, tail_energies,
                           compression_ratio, relative_error)
