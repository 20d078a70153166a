// Warm-up eigensolver (eigh.hip).
#pragma once
#include "common.h"

namespace qrctm {

size_t eigh_scratch_bytes(int n);
// Z: n x n (symmetrised inside).  U (n x k): eigenvectors of the k largest
// |lambda|, sign-fixed; Cd (k x k) = diag(lambda).  Blocks the host once per sweep.
Status eigh_select(const double* Z, int n, int k, double* U, double* Cd, void* ws, size_t ws_bytes,
                   hipStream_t st);

}  // namespace qrctm
