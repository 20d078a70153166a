// GEMM descriptors of the contractions of one CTMRG renormalisation step
// (shared by the step driver and the observables).  Layouts (row-major):
//   C[x,y], T[x,m,y], a[U][L][R][Dn], Q[(e,u),alpha] (chi*Dab x chio),
//   Y[alpha][f][u][l], Z[alpha][r][f][d] (chio*chi*Dab^2 each).
#pragma once
#include "common.h"

namespace qrctm {

struct StepPtrs {
    const double *C, *T, *a;
    double *Q, *R, *Y, *Z, *Tp, *W, *Cp;
};

inline GemmDesc g_reduced_corner(const StepPtrs& p, int chi, int Dab) {
    GemmDesc g;  // ct[(y,m), c] = sum_x C[y,x] T[x,m,c]
    g.M = chi; g.N = (long long)Dab * chi; g.K = chi;
    g.A = p.C; g.lda = chi; g.B = p.T; g.ldb = (long long)Dab * chi;
    g.C = p.Q; g.map = OutMap::plain(g.M, g.N, g.N);
    return g;
}
inline GemmDesc g_edge_a(const StepPtrs& p, const double* Q, int chi, int chio, int Dab) {
    GemmDesc g;  // Y[al,f,u,l] = sum_e Q[(e,u),al] T[f,l,e]   (T[x,m,y] = T[y,m,x])
    g.trans_a = 1; g.trans_b = 1;
    g.M = (long long)Dab * chio; g.N = (long long)chi * Dab; g.K = chi;
    g.A = Q; g.lda = (long long)Dab * chio;
    g.B = p.T; g.ldb = chi;
    g.C = p.Y;
    const long long D2 = (long long)Dab * Dab;
    g.map = OutMap{chio, Dab, (long long)chi * D2, Dab, D2, 1};
    return g;
}
inline GemmDesc g_edge_b(const StepPtrs& p, int chi, int chio, int Dab) {
    GemmDesc g;  // Z[al,r,f,d] = sum_{u,l} Y[al,f,u,l] a[u,l,r,d]
    const long long D2 = (long long)Dab * Dab;
    g.M = (long long)chio * chi; g.N = D2; g.K = D2;
    g.A = p.Y; g.lda = D2; g.B = p.a; g.ldb = D2;
    g.C = p.Z;
    g.map = OutMap{chi, (long long)chi * D2, Dab, Dab, (long long)chi * Dab, 1};
    return g;
}
inline GemmDesc g_edge_c(const StepPtrs& p, const double* Q, int chi, int chio, int Dab) {
    GemmDesc g;  // T'[al,r,be] = sum_{f,d} Z[al,r,f,d] Q[(f,d),be]
    g.M = (long long)chio * Dab; g.N = chio; g.K = (long long)chi * Dab;
    g.A = p.Z; g.lda = (long long)chi * Dab; g.B = Q; g.ldb = chio;
    g.C = p.Tp; g.map = OutMap::plain(g.M, g.N, g.N);
    return g;
}
inline GemmDesc g_corner_w(const StepPtrs& p, int chi, int Dab) {
    GemmDesc g;  // W[g,r,b] = sum_c R[g,c] Q[(c,r),b]
    g.M = chi; g.N = (long long)Dab * chi; g.K = chi;
    g.A = p.R; g.lda = chi; g.B = p.Q; g.ldb = (long long)Dab * chi;
    g.C = p.W; g.map = OutMap::plain(g.M, g.N, g.N);
    return g;
}
inline GemmDesc g_corner_c(const StepPtrs& p, int chi, int Dab) {
    GemmDesc g;  // C'[a,b] = sum_{g,r} T'[g,r,a] W[g,r,b]
    g.trans_a = 1;
    g.M = chi; g.N = chi; g.K = (long long)chi * Dab;
    g.A = p.Tp; g.lda = chi; g.B = p.W; g.ldb = chi;
    g.C = p.Cp; g.map = OutMap::plain(chi, chi, chi);
    return g;
}

}  // namespace qrctm
