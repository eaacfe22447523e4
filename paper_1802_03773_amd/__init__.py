"""MI355X (gfx950) structured-QR Levenberg-Marquardt step solver.

The hot path lives in libqrkit.so (HIP kernels behind the C ABI of include/qrkit.h);
`qrkit` is its ctypes binding.
"""
from . import qrkit  # noqa: F401
from .qrkit import (BandedSolver, BlockAngularBatch, BlockAngularCamSolver, BlockAngularNcolSolver,  # noqa: F401
                    BlockAngularSolver,
                    LMDriver, QRKError, discover_banded, discover_blockangular, factor_banded,
                    factor_blockangular)
