// Corner spectrum and convergence measure (spectrum.hip).
#pragma once
#include "common.h"

namespace qrctm {

size_t spectrum_scratch_bytes(int n);
// s_out = sort(|eig(sym C)|) descending / sum; delta_out = ||s_out - s_prev||_2
// (zero padded).  S is n x n scratch; s_out must not alias s_prev.
Status corner_spectrum(const double* C, int n, double* S, const double* s_prev, int n_prev,
                       double* s_out, double* delta_out, hipStream_t st);

}  // namespace qrctm
