// Observables (energy.hip).
#pragma once
#include "common.h"

namespace qrctm {

struct EnergyArgs {
    int d, D, chi;
    const double *C, *T, *As;  // As: C4v-averaged, max-normalised site tensor
    const double* a;           // double layer a[U][L][R][Dn] (next-nearest-neighbour term)
    double *Qbuf, *Ybuf, *Zbuf;  // step buffers reused by the next-nearest-neighbour term
    char* ws;
    size_t ws_bytes;
    void* splitk;
    size_t splitk_bytes;
};
size_t energy_scratch_bytes(int d, int D, int chi);
// E = 2 <h_nn> (+ 2 J2 <h_nnn>); h_* are host d^2 x d^2 matrices.
Status energy_eval(const EnergyArgs& ea, const double* h_nn, const double* h_nnn, double J2,
                   double* E, hipStream_t st);

// E (host) and its cotangents with respect to C, T (device, chi x chi and
// chi x Dab x chi, overwritten) and As (device, d D^4, overwritten); h_nnn
// (nullable) with J2 adds the plaquette term, which needs a, Qbuf, Ybuf, Zbuf.
Status energy_grad_eval(const EnergyArgs& ea, const double* h_nn, const double* h_nnn, double J2,
                        double* E, double* Cb, double* Tb, double* Asb, hipStream_t st);

struct ClassicalArgs {
    int Dab, chi;
    const double *C, *T, *a;  // a in the internal layout a[U][L][R][Dn]
    char* ws;
    size_t ws_bytes;
};
size_t classical_scratch_bytes(int Dab, int chi);
Status classical_lnz(const ClassicalArgs& ca, double* lnk, hipStream_t st);
// imp in the user layout imp[U][L][Dn][R]
Status classical_expect(const ClassicalArgs& ca, const double* imp, double* v, hipStream_t st);

}  // namespace qrctm
