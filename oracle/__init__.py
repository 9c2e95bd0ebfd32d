"""CPU oracle for block classical Gram-Schmidt economic QR (Carson & Ma,
"The Performance of Low-Synchronization Variants of Reorthogonalized Block
Classical Gram-Schmidt", arXiv 2507.21791).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The GPU library never calls it and shares no code
with it: the two meet only on seeded inputs.

Layout
  linalg   -- the handful of dense primitives the algorithms use, written out
              plainly, for two number systems: IEEE binary64 (numpy float64)
              and 50-digit mpmath (numpy object arrays of mpf).
  variants -- BCGSI+, BCGSI+P-2S, BCGSI+P-1S and BCGS-PIPI+, step by step in
              the paper's order and notation (section 2).
  checks   -- loss of orthogonality, relative residual, Householder reference.

Every function states which passage of the paper it follows.
"""

from .linalg import Breakdown, FP64, MP, make_mp
from .variants import (VARIANTS, bcgs_i_plus, bcgs_p_2s, bcgs_p_1s,
                       bcgs_pipi_plus, qr, tsqr_slot)
from .checks import (loss_of_orthogonality, relative_residual,
                     householder_reference, chunked_gram)

__all__ = [
    "Breakdown", "FP64", "MP", "make_mp", "VARIANTS", "bcgs_i_plus",
    "bcgs_p_2s", "bcgs_p_1s", "bcgs_pipi_plus", "qr", "tsqr_slot",
    "loss_of_orthogonality", "relative_residual", "householder_reference",
    "chunked_gram",
]
