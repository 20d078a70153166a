// a1/a2/a3/a9 kernels (tensor_ops.hip).
#pragma once
#include "common.h"

namespace qrctm {

// As = P(A) / max|P(A)|; scale_out (device, may be null) receives max|P(A)| and
// imax_out (device, may be null) the first flat index attaining it; bad (device
// int) is or-ed with 1 on a non-finite or all-zero tensor.
Status c4v_prepare(const double* A, int d, int D, double* As, double* scale_out, int* bad,
                   int* imax_out, hipStream_t st);
// a_int[U][L][R][Dn] = sum_s As[s,u,l,d,r] As[s,u',l',d',r'], bond D^2.
Status double_layer(const double* As, int d, int D, double* a_int, hipStream_t st);
// user layout a[U][L][Dn][R] -> a_int[U][L][R][Dn]
Status dl_to_internal(const double* a, int Dab, double* a_int, hipStream_t st);
// b = vec(I_D) (length D^2)
Status eye_vec(double* b, int D, hipStream_t st);
// C0 (Dab x Dab), T0 (Dab x Dab x Dab) from a_int and the boundary vector b.
Status init_env(const double* a_int, const double* b, int Dab, double* C, double* T,
                hipStream_t st);
size_t sym_norm_scratch_bytes();
// Cn = sym(Cp)/||.||, Tn = sym(Tp)/||.||; norms (device, 2 doubles, may be null).
Status sym_norm(const double* Cp, const double* Tp, int chi, int Dab, double* Cn, double* Tn,
                double* part, double* norms, int* bad, hipStream_t st);

}  // namespace qrctm
