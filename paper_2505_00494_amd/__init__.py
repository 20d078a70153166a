"""QR-CTMRG on MI355X: HIP kernels behind a C ABI (libqrctm.so) and a thin binding."""
from .qrctm import (CTMError, ConvergenceWarning, Context, GRAD_CHECKPOINT, GRAD_FIXED_POINT,
                    PREC_BF16X6_MFMA, PREC_FP32_MFMA, PREC_FP64, QR_AUTO, QR_HOUSEHOLDER, energy,
                    gemm, header_functions, lib, qr, qr_noalloc)

__all__ = ["CTMError", "ConvergenceWarning", "Context", "GRAD_CHECKPOINT", "GRAD_FIXED_POINT",
           "PREC_BF16X6_MFMA", "PREC_FP32_MFMA", "PREC_FP64", "QR_AUTO", "QR_HOUSEHOLDER", "energy",
           "gemm", "header_functions", "lib", "qr", "qr_noalloc"]
