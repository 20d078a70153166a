// Edge contraction 3b with the double layer applied as its two single layers
// (edge_split.hip).
//
// 3b of the QR-CTMRG step (the middle product of T' = Q^T (T a) Q, Fig. 1e) is
//   Z[al][r][f][dd] = sum_{u,l} Y[al][f][u][l] a[u][l][r][dd],
// with a = sum_s A_s (x) A_s (Fig. 1b) and every double-layer leg ket-major
// (u = u_k D + u_b).  As one GEMM it costs 2 chio chi D^8 flops.  Applying the
// ket layer and then the bra layer costs 4 d chio chi D^6 and never forms a:
//   X_s[u_b l_b][r_k d_k] = sum_{u_k l_k} Y[al][f][u_k u_b][l_k l_b] A_s[u_k][l_k][d_k][r_k]
//   Z[al][r_k r_b][f][d_k d_b] = sum_s sum_{u_b l_b} X_s[u_b l_b][r_k d_k] A_s[u_b][l_b][d_b][r_b]
// The result equals the double-layer product up to the order of rounding.
#pragma once
#include "common.h"

namespace qrctm {

// (d, D) for which the fused kernel is built: d = 2, 1 <= D <= 8.
bool edge_split_supported(int d, int D);
// Doubles in the prepared operand, including the launch counters that follow
// it (0 when unsupported).
size_t edge_split_operand_size(int d, int D);
// Bk[s][k][n] = As[s][u][l][dd][r] for k = u D + l, n = r D + dd (zero outside
// k, n < D^2; rows padded to a multiple of 4, columns to a multiple of 16),
// its transpose in the same shape after it, and the launch counters cleared.  As is the prepared site tensor, layout
// [s][u][l][dd][r].
Status edge_split_prepare(const double* As, int d, int D, double* Bk, hipStream_t st);
// Z (chio x D^2 x chi x D^2, layout [al][r][f][dd]) from Y (chio x chi x D^2 x
// D^2, layout [al][f][u][l]) and the prepared operand, whose counters the launch
// uses (launches on one Bk must be ordered, e.g. on one stream).  Y and Z must
// not overlap.  fp32: products on the FP32 matrix cores (Y and Bk rounded to
// FP32, FP32 accumulation; Y and Z stay double in memory), for the mixed forms.
Status edge_split_3b(const double* Y, double* Bk, int d, int D, int chi, int chio, double* Z,
                     hipStream_t st, bool fp32 = false);
// (d, D) for which the fused reverse is built: d = 2, 1 <= D <= 8.
bool edge_split_bw_supported(int d, int D);
// Doubles of the partial-sum scratch edge_split_3b_backward needs.
size_t edge_split_bw_part_size(int d, int D);
// Reverse of edge_split_3b: from Zb (the cotangent of Z, layout [al][f][r][dd])
// and the forward input Y, write Yb (layout [u][al][f][l]) and add the site
// tensor's cotangent from both layers into Asb (layout [s][u][l][dd][r]).
// Y, Zb and Yb must not overlap; part is scratch of edge_split_bw_part_size.
Status edge_split_3b_backward(const double* Y, const double* Zb, double* Bk, int d, int D, int chi,
                              int chio, double* Yb, double* part, size_t part_doubles, double* Asb,
                              hipStream_t st);

}  // namespace qrctm
