"""MI355X (gfx950) tensor-ring ALS: Python binding of libtrals.so.

The package only marshals arguments; the mode-n update (X-streaming MTTSP,
Gram ring, FP64 solve) runs in the HIP library.  PyTorch provides device memory
and the stream.
"""
from ._lib import (PREC, TR_BF16, TR_F32, TR_F64, TR_FP8, TR_NE, TR_QR, TR_QRNE, VARIANT, TRError,  # noqa: F401
                   header_symbols, lib)
from .api import TRContext, TRServer, gen_planted, tr_inner, tr_norm  # noqa: F401
