// Householder QR with diag(R) >= 0 (qr.hip).
#pragma once
#include "common.h"

namespace qrctm {

struct QrScratch {
    size_t off_A, off_part, off_rowbuf, off_red, off_redsum, off_xend, off_ratio, off_err;
    size_t total;
};

QrScratch qr_scratch_layout(int m, int n);
bool qr_fits(int m, int n);
// Workgroups of the cooperative launch for an m x n factorisation (all of them
// must be resident at once).
int qr_grid(int m, int n);
// Q (m x n) and R (n x n) from M (m x n), all device, row-major.  diag_ratio_dev
// (device, may be null) receives min|R_ii| / max|R_ii|; err_dev (device int, may
// be null) is or-ed with 2 if a grid barrier timed out.  Q may alias M.  One cooperative
// kernel; no scratch but ws.  epoch numbers the launches on one ws: 0 (always
// allowed) clears the exchange buffers first; a caller that passes 0, 1, 2, ...
// to consecutive launches on the same ws (in stream order) has them cleared
// only when the count passes a multiple of 2^21.
Status qr_pos(const double* M, double* Q, double* R, int m, int n, void* ws, size_t ws_bytes,
              hipStream_t st, double* diag_ratio_dev, int* err_dev, unsigned long long epoch = 0);

}  // namespace qrctm
