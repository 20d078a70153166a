// Non-GEMM kernels of the reverse pass (adjoint.hip).
#pragma once
#include "common.h"

namespace qrctm {

size_t sym_norm_backward_scratch_bytes();
// (Cn, Tn) = sym_norm(Cp, Tp) with norms = (||sym Cp||, ||sym Tp||); given the
// cotangents (Cb, Tb) of (Cn, Tn), write those of (Cp, Tp).
Status sym_norm_backward(const double* Cn, const double* Tn, const double* Cb, const double* Tb,
                         const double* norms, int chi, int Dab, double* Cpb, double* Tpb,
                         double* part, hipStream_t st);
Status copyltu(const double* M, int n, double* Ms, hipStream_t st);
// *out (host) = |Cb|^2 + |Tb|^2 (nC, nT entries); part: sym_norm_backward scratch.
// Synchronises the stream.
Status sq_norm(const double* Cb, const double* Tb, long long nC, long long nT, double* part,
               double* out, hipStream_t st);
// *out (host) = |C1 - C0|^2 + |T1 - T0|^2; synchronises the stream.
Status sq_diff(const double* C1, const double* C0, const double* T1, const double* T0,
               long long nC, long long nT, double* part, double* out, hipStream_t st);
// Ri = R^{-1} for the upper-triangular n x n R (row-major).  scratch (n x n
// doubles, overwritten; may be null) holds R^T when R's triangle does not fit
// in LDS.  dinv (device, n, may be null): the back substitution multiplies by
// dinv[i] in place of dividing by R_ii (a regularised inverse).
Status tri_inv_upper(const double* R, int n, double* Ri, double* scratch, hipStream_t st,
                     const double* dinv = nullptr);
// dinv[i] = R_ii / (R_ii^2 + eps^2), eps = eps_rel * max_i |R_ii| (Tikhonov form of
// 1 / R_ii; exactly 0 where R_ii = 0)
Status reg_recip_diag(const double* R, int n, double eps_rel, double* dinv, hipStream_t st);
// Asb += reverse of a_int = sum_s As (x) As (a_int layout [U][L][R][Dn])
Status double_layer_backward(const double* abar, const double* As, int d, int D, double* Asb,
                             hipStream_t st);
// Asb += reverse of a_open = As[s] (x) As[t] (ket s, bra t; a_int layout [U][L][R][Dn])
Status open_layer_backward(const double* aob, const double* As, int D, int s, int t, double* Asb,
                           hipStream_t st);
// dA from the cotangent of As = P(A)/max|P(A)|
Status c4v_backward(const double* Asb, const double* As, const double* scale, const int* imax,
                    int d, int D, double* dA, hipStream_t st);
Status ratio_min(const double* r, double* acc, bool reset, hipStream_t st);

}  // namespace qrctm
