// Observables from a converged environment.
//
// Quantum (Heisenberg paragraph; energy per site from the environment): the
// two-site reduced density matrix of a nearest-neighbour pair from the 2x1
// cluster (4 corners, 6 edges, two open sites).  The open site is never formed
// as a double-layer tensor with open physical legs (d^2 D^8 entries); the ket
// and the bra layer are contracted one after the other instead:
//   E1[q,L,t]   = C T C                               (left column)
//   E2[U,w,L,t] = sum_q T[q,U,w] E1[q,L,t]            (top edge)
//   ket:  sum_{u,l} E2 . A[s,u,l,d,r]                 (K = D^2)
//   bra:  sum_{u',l'} (...) . A[s',u',l',d',r']       (K = D^2)
//   Left[w,s,s',R,v] = sum_{t,Dn} (...) T[t,Dn,v]     (bottom edge)
//   rho[(s1 s1'),(s2 s2')] = sum Left[..,s1,s1',..] Left[..,s2,s2',..]
// (the right half equals the left half by the mirror symmetry of the C4v
// network).  The J1-J2 paragraph adds a diagonal pair from the 2x2 plaquette
// (nnn_rho).  Each contraction is one FP64 MFMA GEMM; the index reorders between
// them are HBM-bound permutes or are folded into the GEMM output map.
//
// Classical (Discussion paragraph: classical partition functions): ln kappa =
// ln Z33 + ln Z22 - 2 ln Z32 and <O> = Z33(impurity) / Z33(a).
#include "adjoint.h"
#include "common.h"
#include "energy.h"
#include "step_gemms.h"
#include "tensor_ops.h"

namespace qrctm {
namespace {

constexpr int kMaxDims = 8;

struct PermArgs {
    int nd;
    long long out_dims[kMaxDims];    // output shape
    long long in_strides[kMaxDims];  // input stride of each OUTPUT axis
    long long total;
};

// One output element per thread, written in order; its source offset from the
// output index, axis by axis.  I = unsigned when every offset fits in 32 bits
// (32-bit division is several times cheaper than 64-bit).
template <class I>
__global__ void permute_kernel(const double* __restrict__ in, double* out, PermArgs p) {
    I dims[kMaxDims], strides[kMaxDims];
    for (int q = 0; q < p.nd; ++q) {
        dims[q] = (I)p.out_dims[q];
        strides[q] = (I)p.in_strides[q];
    }
    const I total = (I)p.total;
    for (I e = (I)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (I)gridDim.x * blockDim.x) {
        I rem = e, src = 0;
        for (int q = p.nd - 1; q >= 0; --q) {
            const I i = rem % dims[q];
            rem /= dims[q];
            src += i * strides[q];
        }
        out[e] = in[src];
    }
}

// out = in.transpose(axes) for a row-major tensor of shape dims
Status permute(const double* in, double* out, int nd, const long long* dims, const int* axes,
               hipStream_t st) {
    PermArgs p{};
    p.nd = nd;
    long long stride[kMaxDims];
    long long s = 1;
    for (int q = nd - 1; q >= 0; --q) {
        stride[q] = s;
        s *= dims[q];
    }
    p.total = s;
    for (int q = 0; q < nd; ++q) {
        p.out_dims[q] = dims[axes[q]];
        p.in_strides[q] = stride[axes[q]];
    }
    const int blocks = (int)std::min<long long>(ceil_div(p.total, 256), 65536);
    if (p.total < (1LL << 31)) {
        hipLaunchKernelGGL(permute_kernel<unsigned>, dim3(blocks), dim3(256), 0, st, in, out, p);
    } else {
        hipLaunchKernelGGL(permute_kernel<long long>, dim3(blocks), dim3(256), 0, st, in, out, p);
    }
    return launch_check("permute_kernel");
}

constexpr int kRedBlocks = 512;

// partial sums of sum_i x[i] * y[ (i / ny) + (i % ny) * nx ] (transposed y when tr)
__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                   long long n, long long rows, long long cols, int tr,
                                   double* part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const long long j = tr ? (e % cols) * rows + e / cols : e;
        acc += x[e] * y[j];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(const double* __restrict__ part, int n, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

Status dot(const double* x, const double* y, long long n, long long rows, long long cols, int tr,
           double* part, double* out, hipStream_t st) {
    const int blocks = (int)std::max<long long>(1, std::min<long long>(ceil_div(n, 256), kRedBlocks));
    hipLaunchKernelGGL(dot_partial_kernel, dim3(blocks), dim3(256), 0, st, x, y, n, rows, cols, tr,
                       part);
    QRCTM_TRY(launch_check("dot_partial_kernel"));
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, st, part, blocks, out);
    return launch_check("sum_kernel");
}

// e = 2 Tr(rm h)/Tr(rm) (+ 2 J2 Tr(rm2 h2)/Tr(rm2)) from rho[(s1 s1'),(s2 s2')]
__global__ void bond_energy_kernel(const double* __restrict__ rho, const double* __restrict__ h,
                                   int d, double scale, double* out, int accumulate) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    const int d2 = d * d;
    for (int s1 = 0; s1 < d; ++s1)
        for (int t1 = 0; t1 < d; ++t1)
            for (int s2 = 0; s2 < d; ++s2)
                for (int t2 = 0; t2 < d; ++t2) {
                    const double r = rho[(size_t)(s1 * d + t1) * d2 + (s2 * d + t2)];
                    num += r * h[(size_t)(t1 * d + t2) * d2 + (s1 * d + s2)];
                    if (s1 == t1 && s2 == t2) den += r;
                }
    const double v = scale * num / den;
    *out = accumulate ? *out + v : v;
}

struct ELayout {
    size_t E1, F, E2, Yb, E3, E4, E4p, Left, Lp, Ak, rho, h, scal;
    size_t Lpb, Leftb, E1b, Fb, Akb, rhob, rho2, rhob2, red;
    size_t splitk, total;
    size_t splitk_bytes;
};

ELayout e_layout(int d, int D, int chi) {
    ELayout L{};
    size_t off = 0;
    auto take = [&](size_t count) {
        const size_t o = off;
        off += (count * sizeof(double) + 255) / 256 * 256;
        return o;
    };
    const size_t c = chi, D2 = (size_t)D * D, D4 = D2 * D2, dd = d;
    L.E1 = take(c * D2 * c);
    L.F = take(c * D2 * c);
    L.E2 = take(c * c * D4);
    L.Yb = take(c * c * D4);
    L.E3 = take(dd * c * c * D4);
    L.E4 = take(dd * dd * c * c * D4);
    L.E4p = take(dd * dd * c * c * D4);
    L.Left = take(c * dd * dd * D2 * c);
    L.Lp = take(c * dd * dd * D2 * c);
    L.Ak = take(dd * D4);
    L.rho = take(dd * dd * dd * dd);
    L.h = take(2 * dd * dd * dd * dd);
    L.scal = take(16);
    L.Lpb = take(c * dd * dd * D2 * c);
    L.Leftb = take(c * dd * dd * D2 * c);
    L.E1b = take(c * D2 * c);
    L.Fb = take(c * D2 * c);
    L.Akb = take(dd * D4);
    L.rhob = take(dd * dd * dd * dd);
    L.rho2 = take(dd * dd * dd * dd);
    L.rhob2 = take(dd * dd * dd * dd);
    L.red = take(kRedBlocks);
    // split-K partials: the largest over every product of the forward and reverse
    // energy contractions (M, N, K as in nn_rho_forward, energy_grad_eval, nnn_rho)
    size_t sk = 0;
    {
        auto add = [&](long long M, long long N, long long K) {
            GemmDesc g;
            g.M = M; g.N = N; g.K = K;
            sk = std::max(sk, gemm_splitk_bytes(g));
        };
        const long long cc = (long long)c, q = (long long)D2, e = (long long)dd;
        const long long K = cc * q * cc, Mleft = cc * e * e * q, n = cc * q;
        // forward
        add(q * cc, q * cc, cc);
        add(cc * cc * q, e * q, q);
        add(cc * cc * e * q, e * q, q);
        add(cc * e * e * q, cc, cc * q);
        add(e * e, e * e, K);
        // reverse
        add(e * e, K, e * e);
        add(Mleft, cc * q, cc);
        add(cc * q, cc, Mleft);
        add(cc * cc * e * q, q, e * q);
        add(q, e * q, cc * cc * e * q);
        add(cc * cc * q, q, e * q);
        add(q, e * q, cc * cc * q);
        add(cc, q * cc, q * cc);
        add(cc * q, cc, cc);
        add(cc, cc, cc * q);
        add(cc, q * cc, cc);
        // next-nearest-neighbour term (Dab = D^2)
        add(cc, q * cc, cc);
        add(q * cc, q * cc, cc);
        add(cc * cc, q * q, q * q);
        add(n, n, n);
        // its reverse (plaquette cotangents, 3b and 3a reversed)
        add(q * q, q * q, cc * cc);
        add(q * cc, cc, cc * q);
    }
    L.splitk_bytes = sk + 256;
    L.splitk = take(L.splitk_bytes / sizeof(double) + 1);
    L.total = off;
    return L;
}

struct CLayout {
    size_t F, E1, X1, X2, imp, part, scal, splitk, total;
    size_t splitk_bytes;
};

CLayout c_layout(int Dab, int chi) {
    CLayout L{};
    size_t off = 0;
    auto take = [&](size_t count) {
        const size_t o = off;
        off += (count * sizeof(double) + 255) / 256 * 256;
        return o;
    };
    const size_t c = chi, D = Dab;
    L.F = take(c * D * c);
    L.E1 = take(c * D * c);
    L.X1 = take(c * c * D * D);
    L.X2 = take(c * c * D * D);
    L.imp = take(D * D * D * D);
    L.part = take(kRedBlocks);
    L.scal = take(16);
    // split-K partials of the products below (left_column, z33, C C)
    size_t sk = 0;
    {
        auto add = [&](long long M, long long N, long long K) {
            GemmDesc g;
            g.M = M; g.N = N; g.K = K;
            sk = std::max(sk, gemm_splitk_bytes(g));
        };
        const long long cc = (long long)c, q = (long long)D, q2 = q * q;
        add(cc, q * cc, cc);
        add(cc * q, cc, cc);
        add(q * cc, q * cc, cc);
        add(cc * cc, q2, q2);
        add(cc, cc, cc);
    }
    L.splitk_bytes = sk + 256;
    L.splitk = take(L.splitk_bytes / sizeof(double) + 1);
    L.total = off;
    return L;
}

// E1[q,L,t] = sum C[q,p] T[p,L,r] C[r,t]; sk: split-K scratch of skb bytes
Status left_column(const double* C, const double* T, int chi, int Dab, double* F, double* E1,
                   void* sk, size_t skb, hipStream_t st) {
    GemmDesc g;
    g.M = chi; g.N = (long long)Dab * chi; g.K = chi;
    g.A = C; g.lda = chi; g.B = T; g.ldb = (long long)Dab * chi;
    g.C = F; g.map = OutMap::plain(g.M, g.N, g.N);
    QRCTM_TRY(gemm_f64(g, sk, skb, st));
    GemmDesc h;
    h.M = (long long)chi * Dab; h.N = chi; h.K = chi;
    h.A = F; h.lda = chi; h.B = C; h.ldb = chi;
    h.C = E1; h.map = OutMap::plain(h.M, h.N, h.N);
    return gemm_f64(h, sk, skb, st);
}

// Z33 of the 3x3 network with centre tensor ct (internal layout a[U][L][R][Dn])
Status z33(const ClassicalArgs& ca, const CLayout& L, const double* ct, double* out,
           hipStream_t st) {
    char* b = ca.ws;
    const int chi = ca.chi, Dab = ca.Dab;
    const long long D2 = (long long)Dab * Dab;
    double* E1 = reinterpret_cast<double*>(b + L.E1);
    double* X1 = reinterpret_cast<double*>(b + L.X1);
    double* X2 = reinterpret_cast<double*>(b + L.X2);
    void* sk = b + L.splitk;
    const size_t skb = L.splitk_bytes;
    // X1[w][t][U][L] = sum_q T[q,U,w] E1[q,L,t]
    GemmDesc g;
    g.trans_a = 1;
    g.M = (long long)Dab * chi; g.N = (long long)Dab * chi; g.K = chi;
    g.A = ca.T; g.lda = (long long)Dab * chi; g.B = E1; g.ldb = (long long)Dab * chi;
    g.C = X1;
    g.map = OutMap{chi, Dab, (long long)chi * D2, chi, 1, D2};
    QRCTM_TRY(gemm_f64(g, sk, skb, st));
    // X2[w][t][R][Dn] = X1[(w,t),(U,L)] ct[(U,L),(R,Dn)]
    GemmDesc h;
    h.M = (long long)chi * chi; h.N = D2; h.K = D2;
    h.A = X1; h.lda = D2; h.B = ct; h.ldb = D2;
    h.C = X2; h.map = OutMap::plain(h.M, h.N, h.N);
    QRCTM_TRY(gemm_f64(h, sk, skb, st));
    // Y3[w][t][R][Dn] = sum_v E1[w,R,v] T[t,Dn,v]   (into X1)
    GemmDesc k;
    k.trans_b = 1;
    k.M = (long long)chi * Dab; k.N = (long long)chi * Dab; k.K = chi;
    k.A = E1; k.lda = chi; k.B = ca.T; k.ldb = chi;
    k.C = X1;
    k.map = OutMap{Dab, (long long)chi * D2, Dab, Dab, D2, 1};
    QRCTM_TRY(gemm_f64(k, sk, skb, st));
    return dot(X2, X1, (long long)chi * chi * D2, 0, 1, 0, reinterpret_cast<double*>(b + L.part),
               out, st);
}

Status classical_parts(const ClassicalArgs& ca, double* z33v, double* z22v, double* z32v,
                       const double* imp_dev, hipStream_t st) {
    const CLayout L = c_layout(ca.Dab, ca.chi);
    Status s;
    if (ca.ws_bytes < L.total) {
        s.code = -2;
        s.msg = "classical observables: scratch too small";
        return s;
    }
    char* b = ca.ws;
    const int chi = ca.chi, Dab = ca.Dab;
    double* F = reinterpret_cast<double*>(b + L.F);
    double* E1 = reinterpret_cast<double*>(b + L.E1);
    double* part = reinterpret_cast<double*>(b + L.part);
    double* sc = reinterpret_cast<double*>(b + L.scal);
    QRCTM_TRY(left_column(ca.C, ca.T, chi, Dab, F, E1, b + L.splitk, L.splitk_bytes, st));
    if (z32v) QRCTM_TRY(dot(E1, E1, (long long)chi * Dab * chi, 0, 1, 0, part, sc + 0, st));
    if (z22v) {
        GemmDesc g;  // C2 = C C into F
        g.M = chi; g.N = chi; g.K = chi;
        g.A = ca.C; g.lda = chi; g.B = ca.C; g.ldb = chi;
        g.C = F; g.map = OutMap::plain(chi, chi, chi);
        QRCTM_TRY(gemm_f64(g, b + L.splitk, L.splitk_bytes, st));
        QRCTM_TRY(dot(F, F, (long long)chi * chi, chi, chi, 1, part, sc + 1, st));
    }
    const double* ct = ca.a;
    if (imp_dev) {
        double* imp = reinterpret_cast<double*>(b + L.imp);
        QRCTM_TRY(dl_to_internal(imp_dev, Dab, imp, st));
        QRCTM_TRY(z33(ca, L, imp, sc + 3, st));
    }
    QRCTM_TRY(z33(ca, L, ct, sc + 2, st));
    double h[4] = {0, 0, 0, 0};
    QRCTM_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st));
    QRCTM_HIP(hipStreamSynchronize(st));
    if (z32v) *z32v = h[0];
    if (z22v) *z22v = h[1];
    if (z33v) *z33v = imp_dev ? h[3] / h[2] : h[2];
    return s;
}

}  // namespace

size_t energy_scratch_bytes(int d, int D, int chi) { return e_layout(d, D, chi).total; }
size_t classical_scratch_bytes(int Dab, int chi) { return c_layout(Dab, chi).total; }

Status classical_lnz(const ClassicalArgs& ca, double* lnk, hipStream_t st) {
    double a = 0, b = 0, c = 0;
    QRCTM_TRY(classical_parts(ca, &a, &b, &c, nullptr, st));
    *lnk = std::log(a) + std::log(b) - 2.0 * std::log(c);
    return Status{};
}

Status classical_expect(const ClassicalArgs& ca, const double* imp, double* v, hipStream_t st) {
    return classical_parts(ca, v, nullptr, nullptr, imp, st);
}

namespace {

GemmDesc gd(int ta, int tb, long long M, long long N, long long K, const double* A, long long lda,
            const double* B, long long ldb, double* C, OutMap mp, double beta = 0.0) {
    GemmDesc g;
    g.trans_a = ta; g.trans_b = tb;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
    g.C = C; g.map = mp; g.beta = beta;
    return g;
}

OutMap plain(long long M, long long N) { return OutMap::plain(M, N, N); }

// rho[(s1 s1'),(s2 s2')] of the nearest-neighbour pair; keeps every
// intermediate in the tape for the reverse pass.
Status nn_rho_forward(const EnergyArgs& ea, const ELayout& L, hipStream_t st) {
    char* b = ea.ws;
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    const int d = ea.d, D = ea.D, chi = ea.chi;
    const long long c = chi, DD = D, D2 = (long long)D * D, dd = d;
    void* sk = b + L.splitk;
    const size_t skb = L.splitk_bytes;
    QRCTM_TRY(left_column(ea.C, ea.T, chi, (int)D2, P(L.F), P(L.E1), sk, skb, st));
    // E2[(U,w),(L,t)] = sum_q T[q,U,w] E1[q,L,t]   ([u][u'][w][l][l'][t])
    QRCTM_TRY(gemm_f64(gd(1, 0, D2 * c, D2 * c, c, ea.T, D2 * c, P(L.E1), D2 * c, P(L.E2),
                          plain(D2 * c, D2 * c)), sk, skb, st));
    {   // Yb[w][t][u'][l'][u][l]
        const long long dims[6] = {DD, DD, c, DD, DD, c};
        const int axes[6] = {2, 5, 1, 4, 0, 3};
        QRCTM_TRY(permute(P(L.E2), P(L.Yb), 6, dims, axes, st));
    }
    {   // Ak[u][l][s][d][r] from As[s][u][l][d][r]
        const long long dims[5] = {dd, DD, DD, DD, DD};
        const int axes[5] = {1, 2, 0, 3, 4};
        QRCTM_TRY(permute(ea.As, P(L.Ak), 5, dims, axes, st));
    }
    // ket: rows (w,t,u',l'), K (u,l), cols (s,d,r) -> E3 [w][t][s][d][r][u'][l']
    QRCTM_TRY(gemm_f64(gd(0, 0, c * c * D2, dd * D2, D2, P(L.Yb), D2, P(L.Ak), dd * D2, P(L.E3),
                          OutMap{D2, dd * D2 * D2, 1, dd * D2, 0, D2}), sk, skb, st));
    // bra: rows (w,t,s,d,r), K (u',l'), cols (s',d',r') -> E4
    QRCTM_TRY(gemm_f64(gd(0, 0, c * c * dd * D2, dd * D2, D2, P(L.E3), D2, P(L.Ak), dd * D2,
                          P(L.E4), plain(c * c * dd * D2, dd * D2)), sk, skb, st));
    {   // E4p [w][s][s'][r][r'][t][d][d']
        const long long dims[8] = {c, c, dd, DD, DD, dd, DD, DD};
        const int axes[8] = {0, 2, 5, 4, 7, 1, 3, 6};
        QRCTM_TRY(permute(P(L.E4), P(L.E4p), 8, dims, axes, st));
    }
    // Left[(w,s,s',R), v] = sum_{(t,Dn)} E4p[(w,s,s',R),(t,Dn)] T[(t,Dn), v]
    QRCTM_TRY(gemm_f64(gd(0, 0, c * dd * dd * D2, c, c * D2, P(L.E4p), c * D2, ea.T, c, P(L.Left),
                          plain(c * dd * dd * D2, c)), sk, skb, st));
    {   // Lp[(s,s'), (w,R,v)]
        const long long dims[5] = {c, dd, dd, D2, c};
        const int axes[5] = {1, 2, 0, 3, 4};
        QRCTM_TRY(permute(P(L.Left), P(L.Lp), 5, dims, axes, st));
    }
    // rho = Lp Lp^T
    const long long K = c * D2 * c;
    QRCTM_TRY(gemm_f64(gd(0, 1, dd * dd, dd * dd, K, P(L.Lp), K, P(L.Lp), K, P(L.rho),
                          plain(dd * dd, dd * dd)), sk, skb, st));
    return Status{};
}

// rhob = dE/drho + (dE/drho)^T for E = scale Tr(rm h)/Tr(rm) (rho layout
// [(s1 s1'),(s2 s2')]); the symmetrised form is what both densities need:
// rho = Lp Lp^T (nearest neighbours) and rho[q1][q2] = Tr(X_q1 X_q2) (plaquette)
// are symmetric functions of their two factors.
__global__ void rho_bar_kernel(const double* __restrict__ rho, const double* __restrict__ h, int d,
                               double scale, double* rhob) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int d2 = d * d;
    double num = 0.0, den = 0.0;
    for (int s1 = 0; s1 < d; ++s1)
        for (int t1 = 0; t1 < d; ++t1)
            for (int s2 = 0; s2 < d; ++s2)
                for (int t2 = 0; t2 < d; ++t2) {
                    const double r = rho[(size_t)(s1 * d + t1) * d2 + (s2 * d + t2)];
                    num += r * h[(size_t)(t1 * d + t2) * d2 + (s1 * d + s2)];
                    if (s1 == t1 && s2 == t2) den += r;
                }
    const double ratio = num / den;
    for (int s1 = 0; s1 < d; ++s1)
        for (int t1 = 0; t1 < d; ++t1)
            for (int s2 = 0; s2 < d; ++s2)
                for (int t2 = 0; t2 < d; ++t2) {
                    const double g = (scale / den) * (h[(size_t)(t1 * d + t2) * d2 + (s1 * d + s2)] -
                                                      ((s1 == t1 && s2 == t2) ? ratio : 0.0));
                    rhob[(size_t)(s1 * d + t1) * d2 + (s2 * d + t2)] = g;
                }
    for (int i = 0; i < d2; ++i)
        for (int j = i; j < d2; ++j) {
            const double v = rhob[(size_t)i * d2 + j] + rhob[(size_t)j * d2 + i];
            rhob[(size_t)i * d2 + j] = v;
            rhob[(size_t)j * d2 + i] = v;
        }
}

// a_open[U][L][R][Dn] = As[s,u,l,d,r] As[t,u',l',d',r'] (ket s, bra t)
__global__ void open_layer_kernel(const double* __restrict__ As, int D, int s, int t, double* a) {
    const long long D2 = (long long)D * D;
    const long long n = D2 * D2 * D2 * D2;
    const int D4 = D * D * D * D;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        long long rem = e;
        const int Dn = (int)(rem % D2); rem /= D2;
        const int R = (int)(rem % D2); rem /= D2;
        const int L = (int)(rem % D2); rem /= D2;
        const int U = (int)rem;
        const int ik = (((U / D) * D + L / D) * D + Dn / D) * D + R / D;
        const int ib = (((U % D) * D + L % D) * D + Dn % D) * D + R % D;
        a[e] = As[(size_t)s * D4 + ik] * As[(size_t)t * D4 + ib];
    }
}

__global__ void sym_square_kernel(const double* __restrict__ Z, long long n, double* out) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n * n;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, j = e % n;
        out[e] = 0.5 * (Z[e] + Z[j * n + i]);
    }
}

// In place over the d^2 matrices X_q (n^2 entries each, q = s d + t):
// X_q <- sum_q2 S[q][q2] X_q2, S = rhob of the plaquette density (d^2 <= 16).
__global__ void mix_planes_kernel(double* X, long long nn, int d2, const double* __restrict__ S) {
    double v[16];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        for (int q = 0; q < d2; ++q) v[q] = X[(size_t)q * nn + e];
        for (int q = 0; q < d2; ++q) {
            double a = 0.0;
            for (int q2 = 0; q2 < d2; ++q2) a += S[q * d2 + q2] * v[q2];
            X[(size_t)q * nn + e] = a;
        }
    }
}

// out[al][f][r][d] = (S[(al,r),(f,d)] + S[(f,d),(al,r)]) / 2 for the n x n
// matrix S (n = chi Dab): the cotangent of an enlarged corner sym(Z), Z in the
// layout of the step's 3b output, brought to the row order (al,f) x (r,d) of
// the 3b GEMM.  32 x 32 tiles of S and of its transpose through LDS.
constexpr int kSpTile = 32;
__global__ __launch_bounds__(256) void sym_perm_kernel(const double* __restrict__ S, int chi,
                                                       int Dab, double* __restrict__ out) {
    __shared__ double a[kSpTile][kSpTile + 1];
    __shared__ double b[kSpTile][kSpTile + 1];
    const long long n = (long long)chi * Dab;
    const long long i0 = (long long)blockIdx.y * kSpTile, j0 = (long long)blockIdx.x * kSpTile;
    const int tx = threadIdx.x % kSpTile, ty = threadIdx.x / kSpTile;  // 32 x 8
    for (int r = ty; r < kSpTile; r += 8) {
        const long long i = i0 + r, j = j0 + tx;
        a[r][tx] = (i < n && j < n) ? S[i * n + j] : 0.0;       // S[i0 + r][j0 + tx]
        const long long i2 = j0 + r, j2 = i0 + tx;
        b[r][tx] = (i2 < n && j2 < n) ? S[i2 * n + j2] : 0.0;   // S[j0 + r][i0 + tx]
    }
    __syncthreads();
    const long long D2 = (long long)Dab * Dab;
    for (int r = ty; r < kSpTile; r += 8) {
        const long long i = i0 + r, j = j0 + tx;
        if (i >= n || j >= n) continue;
        const long long al = i / Dab, rr = i % Dab, f = j / Dab, dd = j % Dab;
        out[al * (long long)chi * D2 + f * D2 + rr * Dab + dd] = 0.5 * (a[r][tx] + b[tx][r]);
    }
}

// rho[(s1 s1'),(s2 s2')] of a diagonal (next-nearest-neighbour) pair from the
// 2x2 plaquette (J1-J2 paragraph): the cyclic product of four enlarged
// corners, two of them with the site open.  By C4v every enlarged corner is
// the same symmetric matrix Cc, so rho = Tr(Co_{s1 s1'} Cc Co_{s2 s2'} Cc).
// The enlarged corners are built with the step's own contractions (reduced
// corner, 3a, 3b with the closed or the open double layer).
Status nnn_rho(const EnergyArgs& ea, const ELayout& L, hipStream_t st) {
    Status s;
    const int d = ea.d, D = ea.D, chi = ea.chi, Dab = D * D;
    const long long n = (long long)chi * Dab, nn = n * n, D8 = (long long)Dab * Dab * Dab * Dab;
    if (nn < D8) {
        s.code = -1;
        s.msg = "energy: the next-nearest-neighbour term needs chi >= D^2";
        return s;
    }
    char* b = ea.ws;
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    void* sk = b + L.splitk;
    const size_t skb = L.splitk_bytes;
    StepPtrs sp{};
    sp.C = ea.C; sp.T = ea.T; sp.a = ea.a;
    sp.Q = ea.Qbuf; sp.Y = ea.Ybuf; sp.Z = ea.Zbuf;
    QRCTM_TRY(gemm_f64(g_reduced_corner(sp, chi, Dab), sk, skb, st));
    QRCTM_TRY(gemm_f64(g_edge_a(sp, sp.Q, chi, chi, Dab), sk, skb, st));
    QRCTM_TRY(gemm_f64(g_edge_b(sp, chi, chi, Dab), sk, skb, st));
    const int blocks = (int)std::min<long long>(ceil_div(nn, 256), 65536);
    double* Cc = P(L.E2);
    hipLaunchKernelGGL(sym_square_kernel, dim3(blocks), dim3(256), 0, st, sp.Z, n, Cc);
    QRCTM_TRY(launch_check("sym_square_kernel"));
    const int d2 = d * d;
    double* aop = P(L.Yb);
    for (int q = 0; q < d2; ++q) {
        hipLaunchKernelGGL(open_layer_kernel, dim3((int)std::min<long long>(ceil_div(D8, 256), 65536)),
                           dim3(256), 0, st, ea.As, D, q / d, q % d, aop);
        QRCTM_TRY(launch_check("open_layer_kernel"));
        StepPtrs so = sp;
        so.a = aop;
        so.Z = P(L.E3);
        QRCTM_TRY(gemm_f64(g_edge_b(so, chi, chi, Dab), sk, skb, st));
        hipLaunchKernelGGL(sym_square_kernel, dim3(blocks), dim3(256), 0, st, so.Z, n,
                           P(L.E4) + (size_t)q * nn);
        QRCTM_TRY(launch_check("sym_square_kernel"));
    }
    for (int q = 0; q < d2; ++q) {
        GemmDesc g;  // X_q = Co_q Cc
        g.M = n; g.N = n; g.K = n;
        g.A = P(L.E4) + (size_t)q * nn; g.lda = n; g.B = Cc; g.ldb = n;
        g.C = P(L.E4p) + (size_t)q * nn; g.map = OutMap::plain(n, n, n);
        QRCTM_TRY(gemm_f64(g, sk, skb, st));
    }
    for (int q1 = 0; q1 < d2; ++q1)
        for (int q2 = 0; q2 < d2; ++q2)
            QRCTM_TRY(dot(P(L.E4p) + (size_t)q1 * nn, P(L.E4p) + (size_t)q2 * nn, nn, n, n, 1,
                          P(L.red), P(L.rho2) + q1 * d2 + q2, st));
    return s;
}

// Reverse of the plaquette term e2 = 2 J2 Tr(rm2 h2)/Tr(rm2), after nnn_rho
// (Cc in E2, Co_q in E4, X_q = Co_q Cc in E4p, the 3a output Y of the reduced
// corner in Ybuf, the reduced corner in Qbuf) and after the nearest-neighbour
// reverse (whose tape it reuses).  Adds to Cb, Tb (device) and Asb.
// With S = rhob2 (symmetrised), the cotangent of X_q is (sum_q2 S[q][q2] X_q2)^T
// = V_q^T (rho2[q1][q2] = Tr(X_q1 X_q2)); hence, Cc and Co_q being symmetric,
//   Cobar_q = V_q^T Cc,   Ccbar = sum_q Co_q V_q^T,
// each symmetrised (Co_q = sym(Z_q), Cc = sym(Z)), then the enlarged corners'
// 3b (closed and open double layers), 3a and reduced corner are reversed.
Status nnn_backward(const EnergyArgs& ea, const ELayout& L, double J2, double* Cb, double* Tb,
                    double* Asb, hipStream_t st) {
    char* b = ea.ws;
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    void* sk = b + L.splitk;
    const size_t skb = L.splitk_bytes;
    const int d = ea.d, D = ea.D, chi = ea.chi, Dab = D * D, d2 = d * d;
    const long long c = chi, Db = Dab, n = c * Db, nn = n * n, Q2 = Db * Db;
    if (d2 > 16) {
        Status s;
        s.code = -1;
        s.msg = "energy gradient: the next-nearest-neighbour term supports d <= 4";
        return s;
    }
    double* Cc = P(L.E2);
    double* Co = P(L.E4);
    double* X = P(L.E4p);
    // S = symmetrised dE2/drho2, then X_q -> V_q = sum_q2 S[q][q2] X_q2 in place
    hipLaunchKernelGGL(rho_bar_kernel, dim3(1), dim3(64), 0, st, P(L.rho2), P(L.h) + d2 * d2, d,
                       2.0 * J2, P(L.rhob2));
    QRCTM_TRY(launch_check("rho_bar_kernel"));
    const int blocks = (int)std::min<long long>(ceil_div(nn, 256), 65536);
    hipLaunchKernelGGL(mix_planes_kernel, dim3(blocks), dim3(256), 0, st, X, nn, d2, P(L.rhob2));
    QRCTM_TRY(launch_check("mix_planes_kernel"));
    // Ccbar (into Yb) = sum_q Co_q V_q^T; then Cobar_q = V_q^T Cc over Co_q
    double* Ccb = P(L.Yb);
    for (int q = 0; q < d2; ++q) {
        GemmDesc g;
        g.trans_b = 1;
        g.M = n; g.N = n; g.K = n;
        g.A = Co + (size_t)q * nn; g.lda = n; g.B = X + (size_t)q * nn; g.ldb = n;
        g.C = Ccb; g.map = OutMap::plain(n, n, n); g.beta = q ? 1.0 : 0.0;
        QRCTM_TRY(gemm_f64(g, sk, skb, st));
    }
    for (int q = 0; q < d2; ++q) {
        GemmDesc g;
        g.trans_a = 1;
        g.M = n; g.N = n; g.K = n;
        g.A = X + (size_t)q * nn; g.lda = n; g.B = Cc; g.ldb = n;
        g.C = Co + (size_t)q * nn; g.map = OutMap::plain(n, n, n);
        QRCTM_TRY(gemm_f64(g, sk, skb, st));
    }
    // reverse of 3b, Z_x[(al,f),(r,d)] = sum_(u,l) Y[(al,f),(u,l)] a_x[(u,l),(r,d)],
    // for the closed corner and the d^2 open ones: Ybar (layout [u][al][f][l], in
    // E3) accumulates Zbar'_x a_x^T, and a_x's cotangent Y^T Zbar'_x (D^8 <= n^2
    // doubles over the dead V_0) goes to the site tensor's cotangent
    double* Zb = ea.Zbuf;
    double* Ybar = P(L.E3);
    double* xbar = X;
    const dim3 sp_grid((unsigned)ceil_div(n, kSpTile), (unsigned)ceil_div(n, kSpTile));
    auto reverse_3b = [&](const double* Sx, const double* ax, bool first) -> Status {
        hipLaunchKernelGGL(sym_perm_kernel, sp_grid, dim3(256), 0, st, Sx, chi, Dab, Zb);
        QRCTM_TRY(launch_check("sym_perm_kernel"));
        QRCTM_TRY(gemm_f64(gd(0, 1, c * c, Q2, Q2, Zb, Q2, ax, Q2, Ybar,
                              OutMap{c, c * Db, Db, Db, c * c * Db, 1}, first ? 0.0 : 1.0),
                           sk, skb, st));
        return gemm_f64(gd(1, 0, Q2, Q2, c * c, ea.Ybuf, Q2, Zb, Q2, xbar, plain(Q2, Q2)), sk, skb,
                        st);
    };
    QRCTM_TRY(reverse_3b(Ccb, ea.a, true));
    QRCTM_TRY(double_layer_backward(xbar, ea.As, d, D, Asb, st));
    double* aop = P(L.Yb);  // Ccbar is dead now
    const long long D8 = Q2 * Q2;
    for (int q = 0; q < d2; ++q) {
        hipLaunchKernelGGL(open_layer_kernel, dim3((int)std::min<long long>(ceil_div(D8, 256), 65536)),
                           dim3(256), 0, st, ea.As, D, q / d, q % d, aop);
        QRCTM_TRY(launch_check("open_layer_kernel"));
        QRCTM_TRY(reverse_3b(Co + (size_t)q * nn, aop, false));
        QRCTM_TRY(open_layer_backward(xbar, ea.As, D, q / d, q % d, Asb, st));
    }
    // reverse of 3a, Y[al,f,u,l] = sum_e ct[(e,u),al] T[f,l,e]: ctbar (in Fb) and Tb
    double* ctb = P(L.Fb);
    QRCTM_TRY(gemm_f64(gd(0, 0, Db * c, c, c * Db, Ybar, c * Db, ea.T, c, ctb,
                          OutMap{Db * c, 0, 1, c, 0, Db * c}), sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 1, c * Db, c, Db * c, Ybar, c * Db, ea.Qbuf, Db * c, Tb,
                          plain(c * Db, c), 1.0), sk, skb, st));
    // reverse of the reduced corner ct = C T
    QRCTM_TRY(gemm_f64(gd(0, 1, c, c, Db * c, ctb, Db * c, ea.T, Db * c, Cb, plain(c, c), 1.0), sk,
                       skb, st));
    return gemm_f64(gd(1, 0, c, Db * c, c, ea.C, c, ctb, Db * c, Tb, plain(c, Db * c), 1.0), sk, skb,
                    st);
}

}  // namespace

Status energy_eval(const EnergyArgs& ea, const double* h_nn, const double* h_nnn, double J2,
                   double* E, hipStream_t st) {
    Status s;
    const int d = ea.d;
    const ELayout L = e_layout(d, ea.D, ea.chi);
    if (ea.ws_bytes < L.total) {
        s.code = -2;
        s.msg = "energy: scratch too small";
        return s;
    }
    char* b = ea.ws;
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    const int d4 = d * d * d * d;
    QRCTM_TRY(nn_rho_forward(ea, L, st));
    QRCTM_HIP(hipMemcpyAsync(P(L.h), h_nn, sizeof(double) * d4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(bond_energy_kernel, dim3(1), dim3(64), 0, st, P(L.rho), P(L.h), d, 2.0,
                       P(L.scal), 0);
    QRCTM_TRY(launch_check("bond_energy_kernel"));
    if (h_nnn != nullptr && J2 != 0.0) {
        // 2 J2 <h_nnn>: two diagonal pairs per site
        QRCTM_TRY(nnn_rho(ea, L, st));
        QRCTM_HIP(hipMemcpyAsync(P(L.h) + d4, h_nnn, sizeof(double) * d4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(bond_energy_kernel, dim3(1), dim3(64), 0, st, P(L.rho2), P(L.h) + d4, d,
                           2.0 * J2, P(L.scal), 1);
        QRCTM_TRY(launch_check("bond_energy_kernel"));
    }
    double hv = NAN;
    QRCTM_HIP(hipMemcpyAsync(&hv, P(L.scal), sizeof(double), hipMemcpyDeviceToHost, st));
    QRCTM_HIP(hipStreamSynchronize(st));
    *E = hv;
    return s;
}

Status energy_grad_eval(const EnergyArgs& ea, const double* h_nn, const double* h_nnn, double J2,
                        double* E, double* Cb, double* Tb, double* Asb, hipStream_t st) {
    Status s;
    const int d = ea.d, D = ea.D, chi = ea.chi;
    const ELayout L = e_layout(d, D, chi);
    if (ea.ws_bytes < L.total) {
        s.code = -2;
        s.msg = "energy: scratch too small";
        return s;
    }
    char* b = ea.ws;
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    const long long c = chi, DD = D, D2 = (long long)D * D, dd = d;
    void* sk = b + L.splitk;
    const size_t skb = L.splitk_bytes;
    QRCTM_TRY(nn_rho_forward(ea, L, st));
    QRCTM_HIP(hipMemcpyAsync(P(L.h), h_nn, sizeof(double) * d * d * d * d, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(bond_energy_kernel, dim3(1), dim3(64), 0, st, P(L.rho), P(L.h), d, 2.0,
                       P(L.scal), 0);
    QRCTM_TRY(launch_check("bond_energy_kernel"));
    hipLaunchKernelGGL(rho_bar_kernel, dim3(1), dim3(64), 0, st, P(L.rho), P(L.h), d, 2.0, P(L.rhob));
    QRCTM_TRY(launch_check("rho_bar_kernel"));
    const long long K = c * D2 * c;
    // Lpb = rhob_sym Lp
    QRCTM_TRY(gemm_f64(gd(0, 0, dd * dd, K, dd * dd, P(L.rhob), dd * dd, P(L.Lp), K, P(L.Lpb),
                          plain(dd * dd, K)), sk, skb, st));
    {   // Leftb[w][s][s'][R][v] from Lpb[(s,s'),(w,R,v)]
        const long long dims[5] = {dd, dd, c, D2, c};
        const int axes[5] = {2, 0, 1, 3, 4};
        QRCTM_TRY(permute(P(L.Lpb), P(L.Leftb), 5, dims, axes, st));
    }
    const long long Mleft = c * dd * dd * D2;
    // E4pb = Leftb T^T  (into E4);  Tb = E4p^T Leftb
    QRCTM_TRY(gemm_f64(gd(0, 1, Mleft, c * D2, c, P(L.Leftb), c, ea.T, c, P(L.E4),
                          plain(Mleft, c * D2)), sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 0, c * D2, c, Mleft, P(L.E4p), c * D2, P(L.Leftb), c, Tb,
                          plain(c * D2, c)), sk, skb, st));
    {   // E4b [w][t][s][d][r][s'][d'][r'] from E4pb [w][s][s'][r][r'][t][d][d']  (into E4p)
        const long long dims[8] = {c, dd, dd, DD, DD, c, DD, DD};
        const int axes[8] = {0, 5, 1, 6, 3, 2, 7, 4};
        QRCTM_TRY(permute(P(L.E4), P(L.E4p), 8, dims, axes, st));
    }
    // bra reverse: E3b (ket-GEMM layout [(w,t,u',l'),(s,d,r)]) into E4; Akb = E3^T E4b
    QRCTM_TRY(gemm_f64(gd(0, 1, c * c * dd * D2, D2, dd * D2, P(L.E4p), dd * D2, P(L.Ak), dd * D2,
                          P(L.E4), OutMap{dd * D2, D2 * dd * D2, 1, D2, 0, dd * D2}), sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 0, D2, dd * D2, c * c * dd * D2, P(L.E3), D2, P(L.E4p), dd * D2,
                          P(L.Akb), plain(D2, dd * D2)), sk, skb, st));
    // ket reverse: Ybb = E3b Ak^T (into E2);  Akb += Yb^T E3b
    QRCTM_TRY(gemm_f64(gd(0, 1, c * c * D2, D2, dd * D2, P(L.E4), dd * D2, P(L.Ak), dd * D2,
                          P(L.E2), plain(c * c * D2, D2)), sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 0, D2, dd * D2, c * c * D2, P(L.Yb), D2, P(L.E4), dd * D2, P(L.Akb),
                          plain(D2, dd * D2), 1.0), sk, skb, st));
    {   // E2b [u][u'][w][l][l'][t] from Ybb [w][t][u'][l'][u][l]  (into E3)
        const long long dims[6] = {c, c, DD, DD, DD, DD};
        const int axes[6] = {4, 2, 0, 5, 3, 1};
        QRCTM_TRY(permute(P(L.E2), P(L.E3), 6, dims, axes, st));
    }
    // E2 = T^T-contract E1: Tb += E1 E2b^T ; E1b = T E2b
    QRCTM_TRY(gemm_f64(gd(0, 1, c, D2 * c, D2 * c, P(L.E1), D2 * c, P(L.E3), D2 * c, Tb,
                          plain(c, D2 * c), 1.0), sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(0, 0, c, D2 * c, D2 * c, ea.T, D2 * c, P(L.E3), D2 * c, P(L.E1b),
                          plain(c, D2 * c)), sk, skb, st));
    // E1 = F C: Fb = E1b C^T ; Cb = F^T E1b
    QRCTM_TRY(gemm_f64(gd(0, 1, c * D2, c, c, P(L.E1b), c, ea.C, c, P(L.Fb), plain(c * D2, c)), sk,
                       skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 0, c, c, c * D2, P(L.F), c, P(L.E1b), c, Cb, plain(c, c)), sk, skb, st));
    // F = C T: Cb += Fb T^T ; Tb += C^T Fb
    QRCTM_TRY(gemm_f64(gd(0, 1, c, c, D2 * c, P(L.Fb), D2 * c, ea.T, D2 * c, Cb, plain(c, c), 1.0),
                       sk, skb, st));
    QRCTM_TRY(gemm_f64(gd(1, 0, c, D2 * c, c, ea.C, c, P(L.Fb), D2 * c, Tb, plain(c, D2 * c), 1.0),
                       sk, skb, st));
    {   // Asb[s][u][l][d][r] from Akb[u][l][s][d][r]
        const long long dims[5] = {DD, DD, dd, DD, DD};
        const int axes[5] = {2, 0, 1, 3, 4};
        QRCTM_TRY(permute(P(L.Akb), Asb, 5, dims, axes, st));
    }
    if (h_nnn != nullptr && J2 != 0.0) {
        // 2 J2 <h_nnn> and its reverse (the plaquette reuses the tape above)
        const int d4 = d * d * d * d;
        QRCTM_TRY(nnn_rho(ea, L, st));
        QRCTM_HIP(hipMemcpyAsync(P(L.h) + d4, h_nnn, sizeof(double) * d4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(bond_energy_kernel, dim3(1), dim3(64), 0, st, P(L.rho2), P(L.h) + d4, d,
                           2.0 * J2, P(L.scal), 1);
        QRCTM_TRY(launch_check("bond_energy_kernel"));
        QRCTM_TRY(nnn_backward(ea, L, J2, Cb, Tb, Asb, st));
    }
    double hv = NAN;
    QRCTM_HIP(hipMemcpyAsync(&hv, P(L.scal), sizeof(double), hipMemcpyDeviceToHost, st));
    QRCTM_HIP(hipStreamSynchronize(st));
    *E = hv;
    return s;
}

}  // namespace qrctm
