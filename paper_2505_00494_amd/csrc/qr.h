// Householder QR with diag(R) >= 0 (qr.hip).
#pragma once
#include "common.h"

namespace qrctm {

struct QrScratch {
    size_t off_A, off_part, off_rowbuf, off_red, off_redsum, off_xend, off_ratio, off_err;
    size_t off_chol, off_fallbacks;  // Cholesky-QR2 scratch (qr_chol.hip), fallback counter
    size_t total;
};

// Cholesky-QR2 (qr_chol.hip): scratch layout relative to QrScratch::off_chol.
struct CholQrScratch {
    size_t off_Q1, off_part, off_G, off_R1, off_R2, off_Ri, off_work, off_stats, off_state,
        off_dev, off_splitk;
    size_t splitk_bytes, total;
};
bool cholqr_supported(int m, int n);
CholQrScratch cholqr_scratch_layout(int m, int n);
// Q, R of M by Cholesky-QR2 into Q (may alias M) and R; *state_out receives the
// device word that is 0 when the factorisation was accepted (otherwise Q, R
// were not written and the caller must run the Householder kernel).
Status cholqr2(const double* M, double* Q, double* R, int m, int n, char* base,
               const CholQrScratch& L, double* diag_ratio_dev, int** state_out, hipStream_t st);

// QR methods of qr_pos
constexpr int kQrAuto = 0;         // Cholesky-QR2, Householder where it is rejected
constexpr int kQrHouseholder = 1;  // Householder only

QrScratch qr_scratch_layout(int m, int n);
bool qr_fits(int m, int n);
// Workgroups of the Householder kernel for an m x n factorisation (all of them
// must be resident at once).
int qr_grid(int m, int n);
// Q (m x n) and R (n x n) from M (m x n), all device, row-major.  diag_ratio_dev
// (device, may be null) receives min|R_ii| / max|R_ii|; err_dev (device int, may
// be null) is or-ed with 2 if a grid barrier timed out.  Q may alias M.  No
// scratch but ws.  method kQrAuto: Cholesky-QR2 where supported, the
// Householder kernel (an ordinary launch behind it, idle unless needed) where
// it rejects the factorisation; kQrHouseholder: the Householder kernel only
// (a cooperative launch).
// epoch numbers the launches on one ws: 0 (always allowed) clears the
// exchange buffers first; a caller that passes 0, 1, 2, ... to consecutive
// launches on the same ws (in stream order) has them cleared only when the
// count passes a multiple of 2^21.
Status qr_pos(const double* M, double* Q, double* R, int m, int n, void* ws, size_t ws_bytes,
              hipStream_t st, double* diag_ratio_dev, int* err_dev, unsigned long long epoch = 0,
              int method = kQrAuto);
// Householder fallbacks taken on ws since its last clearing (epoch 0), read
// from the device (synchronises st).
Status qr_fallback_count(const void* ws, int m, int n, hipStream_t st, unsigned long long* out);

}  // namespace qrctm
