// Kernels of the hand-written reverse pass (automatic-differentiation
// paragraph: gradient through k tracked QR-CTMRG steps).  The GEMM adjoints
// reuse gemm.hip; this file holds the non-GEMM pieces:
//   sym_norm_backward   reverse of "symmetrise, divide by the Frobenius norm",
//   copyltu             tril(M) + tril(M,-1)^T for the thin-QR adjoint
//                       Abar = (Qbar + Q copyltu(R Rbar^T - Qbar^T Q)) R^{-T},
//   tri_inv_upper       R^{-1} of the upper-triangular R (one workgroup per column,
//                       the triangle of R in LDS, or for large n R^T read from L2),
//   double_layer_backward, c4v_backward (reverse of a2 and a1),
//   ratio_min           running minimum of min|R_ii|/max|R_ii| over tracked steps.
#include "adjoint.h"

#include <vector>

#include "common.h"

namespace qrctm {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 512;

__global__ __launch_bounds__(kThreads) void dots_kernel(const double* __restrict__ Cn,
                                                        const double* __restrict__ Cb,
                                                        const double* __restrict__ Tn,
                                                        const double* __restrict__ Tb, long long nC,
                                                        long long nT, double* part) {
    __shared__ double rc[kThreads], rt[kThreads];
    double sc = 0.0, st = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nC) sc += Cn[e] * Cb[e];
        else st += Tn[e - nC] * Tb[e - nC];
    }
    rc[threadIdx.x] = sc;
    rt[threadIdx.x] = st;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rc[threadIdx.x] += rc[threadIdx.x + w];
            rt[threadIdx.x] += rt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rc[0];
        part[2 * blockIdx.x + 1] = rt[0];
    }
}

// Cpb[x,y] = (sym(Cb)[x,y] - <Cn,Cb> Cn[x,y]) / ||Cs||, same for T over (x <-> y)
__global__ __launch_bounds__(kThreads) void sym_norm_bwd_kernel(
    const double* __restrict__ part, int nparts, const double* __restrict__ norms,
    const double* __restrict__ Cn, const double* __restrict__ Cb, const double* __restrict__ Tn,
    const double* __restrict__ Tb, int chi, int Dab, double* Cpb, double* Tpb) {
    __shared__ double s[2];
    __shared__ double ra[kThreads], rb[kThreads];
    {
        double a = 0.0, b = 0.0;
        for (int q = threadIdx.x; q < nparts; q += kThreads) {
            a += part[2 * q];
            b += part[2 * q + 1];
        }
        ra[threadIdx.x] = a;
        rb[threadIdx.x] = b;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ra[threadIdx.x] += ra[threadIdx.x + w];
                rb[threadIdx.x] += rb[threadIdx.x + w];
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        s[0] = ra[0];
        s[1] = rb[0];
    }
    __syncthreads();
    const double dc = s[0], dt = s[1];
    const double ic = 1.0 / norms[0], it = 1.0 / norms[1];
    const long long nC = (long long)chi * chi, nT = nC * Dab;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nC) {
            const long long x = e / chi, y = e % chi;
            Cpb[e] = (0.5 * (Cb[e] + Cb[y * chi + x]) - dc * Cn[e]) * ic;
        } else {
            const long long f = e - nC;
            const long long x = f / ((long long)Dab * chi), m = (f / chi) % Dab, y = f % chi;
            Tpb[f] = (0.5 * (Tb[f] + Tb[(y * Dab + m) * chi + x]) - dt * Tn[f]) * it;
        }
    }
}

__global__ void copyltu_kernel(const double* __restrict__ M, int n, double* Ms) {
    const long long nn = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, j = e % n;
        Ms[e] = i >= j ? M[e] : M[j * n + i];
    }
}

// x / R_ii, or x dinv[i] for the regularised inverse
__device__ __forceinline__ double div_diag(double x, double rii, const double* dinv, int i) {
    return dinv ? x * dinv[i] : x / rii;
}

// column j of R^{-1}: back substitution R x = e_j, x_i = 0 for i > j
__global__ void tri_inv_upper_kernel(const double* __restrict__ R, int n, double* Ri,
                                     const double* __restrict__ dinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int i = n - 1; i > j; --i) Ri[(size_t)i * n + j] = 0.0;
    for (int i = j; i >= 0; --i) {
        double acc = (i == j) ? 1.0 : 0.0;
        for (int k = i + 1; k <= j; ++k) acc -= R[(size_t)i * n + k] * Ri[(size_t)k * n + j];
        Ri[(size_t)i * n + j] = div_diag(acc, R[(size_t)i * n + i], dinv, i);
    }
}

// Tikhonov-regularised reciprocals of R's diagonal (one workgroup)
__global__ __launch_bounds__(256) void reg_recip_diag_kernel(const double* __restrict__ R, int n,
                                                             double eps_rel, double* dinv) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(R[(size_t)i * n + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double eps = eps_rel * red[0];
    for (int i = threadIdx.x; i < n; i += 256) {
        const double r = R[(size_t)i * n + i];
        dinv[i] = r / (r * r + eps * eps);
    }
}

// Column j of R^{-1} by one workgroup: the upper triangle of R is copied to
// LDS (packed by rows: row k starts at k n - k (k - 1) / 2), thread k keeps
// b_k; for i = j down to 0, x_i = b_i / R_ii (thread i, through LDS) and every
// thread k < i updates b_k -= R_ki x_i.  One workgroup barrier per step.
constexpr int kTriThreads = 256;
constexpr int kTriMaxLds = 150 * 1024;

__global__ __launch_bounds__(kTriThreads) void tri_inv_col_kernel(const double* __restrict__ R,
                                                                  int n, double* Ri,
                                                                  const double* __restrict__ dinv) {
    extern __shared__ double tri[];
    double* x = tri + (size_t)n * (n + 1) / 2;
    const int j = blockIdx.x, k = threadIdx.x;
    for (int r = 0; r <= j; ++r) {
        const size_t off = (size_t)r * n - (size_t)r * (r - 1) / 2;
        for (int c = r + k; c <= j; c += kTriThreads) tri[off + (c - r)] = R[(size_t)r * n + c];
    }
    double b = (k == j) ? 1.0 : 0.0;
    __syncthreads();
    for (int i = j; i >= 0; --i) {
        if (k == i) x[i] = div_diag(b, tri[(size_t)i * n - (size_t)i * (i - 1) / 2], dinv, i);
        __syncthreads();
        if (k < i) b -= tri[(size_t)k * n - (size_t)k * (k - 1) / 2 + (i - k)] * x[i];
    }
    for (int i = k; i < n; i += kTriThreads) Ri[(size_t)i * n + j] = i <= j ? x[i] : 0.0;
}

// Rt = R^T (n x n, row-major), 16 x 16 tiles through LDS.
__global__ void transpose_kernel(const double* __restrict__ R, int n, double* __restrict__ Rt) {
    __shared__ double tile[16][17];
    const int bx = blockIdx.x * 16, by = blockIdx.y * 16, tx = threadIdx.x, ty = threadIdx.y;
    if (by + ty < n && bx + tx < n) tile[ty][tx] = R[(size_t)(by + ty) * n + bx + tx];
    __syncthreads();
    if (bx + ty < n && by + tx < n) Rt[(size_t)(bx + ty) * n + by + tx] = tile[tx][ty];
}

// Column j of R^{-1} by one workgroup when R's triangle does not fit in LDS:
// the same back substitution, with column i of R read as row i of Rt (in L2,
// one coalesced read per step, issued a step ahead).  b lives in LDS (thread
// k owns entries k, k + 256, ...), x_i is handed over through a double buffer,
// so one barrier per step suffices.  n <= 1024.
__global__ __launch_bounds__(kTriThreads) void tri_inv_col_l2_kernel(const double* __restrict__ Rt,
                                                                     int n, double* Ri,
                                                                     const double* __restrict__ dinv) {
    __shared__ double bs[1024];
    __shared__ double xs[2];
    const int j = blockIdx.x, t = threadIdx.x;
    for (int k = t; k < n; k += kTriThreads) {
        bs[k] = k == j ? 1.0 : 0.0;
        if (k > j) Ri[(size_t)k * n + j] = 0.0;
    }
    constexpr int KPT = 1024 / kTriThreads;
    double r[KPT];
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
        const int k = t + u * kTriThreads;
        r[u] = k < j ? Rt[(size_t)j * n + k] : 0.0;
    }
    __syncthreads();
    for (int i = j; i >= 0; --i) {
        if (t == i % kTriThreads) {
            const double x = div_diag(bs[i], Rt[(size_t)i * n + i], dinv, i);
            xs[i & 1] = x;
            Ri[(size_t)i * n + j] = x;
        }
        __syncthreads();
        const double x = xs[i & 1];
        double rn[KPT];
#pragma unroll
        for (int u = 0; u < KPT; ++u) {
            const int k = t + u * kTriThreads;
            rn[u] = (i > 0 && k < i - 1) ? Rt[(size_t)(i - 1) * n + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KPT; ++u) {
            const int k = t + u * kTriThreads;
            if (k < i) bs[k] -= r[u] * x;
            r[u] = rn[u];
        }
    }
}

// Asb[s,u,l,d,r] += sum_{u',l',d',r'} (abar[(u u'),(l l'),(r r'),(d d')] +
//                   abar[(u' u),(l' l),(r' r),(d' d)]) As[s,u',l',d',r']
__global__ void dl_backward_kernel(const double* __restrict__ abar, const double* __restrict__ As,
                                   int d, int D, double* Asb) {
    const int D4 = D * D * D * D;
    const int D2 = D * D;
    const int n = d * D4;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int s = e / D4;
        int rem = e % D4;
        const int r = rem % D; rem /= D;
        const int dd = rem % D; rem /= D;
        const int l = rem % D; rem /= D;
        const int u = rem;
        double acc = 0.0;
        for (int q = 0; q < D4; ++q) {
            int t = q;
            const int r2 = t % D; t /= D;
            const int d2 = t % D; t /= D;
            const int l2 = t % D; t /= D;
            const int u2 = t;
            const double x = As[(size_t)s * D4 + q];
            const size_t i1 = (((size_t)(u * D + u2) * D2 + (l * D + l2)) * D2 + (r * D + r2)) * D2 +
                              (dd * D + d2);
            const size_t i2 = (((size_t)(u2 * D + u) * D2 + (l2 * D + l)) * D2 + (r2 * D + r)) * D2 +
                              (d2 * D + dd);
            acc += (abar[i1] + abar[i2]) * x;
        }
        Asb[e] += acc;
    }
}

// Reverse of a_open[(u u'),(l l'),(r r'),(d d')] = As[s,u,l,d,r] As[t,u',l',d',r']
// (ket s, bra t; a_int layout): bra = 0 adds sum over the bra indices of
// aob * As[t] to Asb[s] (the ket factor's cotangent), bra = 1 adds sum over
// the ket indices of aob * As[s] to Asb[t].
__global__ void open_layer_bw_kernel(const double* __restrict__ aob, const double* __restrict__ As,
                                     int D, int s, int t, int bra, double* Asb) {
    const int D4 = D * D * D * D, D2 = D * D;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D4) return;
    int rem = e;
    const int r = rem % D; rem /= D;
    const int dn = rem % D; rem /= D;
    const int l = rem % D; rem /= D;
    const int u = rem;
    const double* other = As + (size_t)(bra ? s : t) * D4;
    double acc = 0.0;
    for (int q = 0; q < D4; ++q) {
        int w = q;
        const int r2 = w % D; w /= D;
        const int d2 = w % D; w /= D;
        const int l2 = w % D; w /= D;
        const int u2 = w;
        // (this element, the other factor's element q) in ket-bra order
        const int U = bra ? u2 * D + u : u * D + u2;
        const int L = bra ? l2 * D + l : l * D + l2;
        const int R = bra ? r2 * D + r : r * D + r2;
        const int Dn = bra ? d2 * D + dn : dn * D + d2;
        acc += aob[(((size_t)U * D2 + L) * D2 + R) * D2 + Dn] * other[q];
    }
    Asb[(size_t)(bra ? t : s) * D4 + e] += acc;
}

__device__ __forceinline__ int c4v_pos(int g, int i) {
    const int k = g >> 1;
    return (g & 1) ? ((k - i) & 3) : ((i + k) & 3);
}

// dA = P(Asb)/m - sign * <Asb, P(A)>/m^2 * P(e_imax), As = P(A)/m (so <Asb,P(A)> = m <Asb,As>)
__global__ __launch_bounds__(1024) void c4v_backward_kernel(const double* __restrict__ Asb,
                                                            const double* __restrict__ As,
                                                            const double* __restrict__ scale,
                                                            const int* __restrict__ imax, int d,
                                                            int D, double* dA) {
    __shared__ double red[1024];
    const int D4 = D * D * D * D;
    const int n = d * D4;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) acc += Asb[e] * As[e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double m = *scale;
    const int im = *imax;
    const double sgn = As[im] < 0.0 ? -1.0 : 1.0;
    const double coef = sgn * red[0] * m / (m * m);
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int s = e / D4;
        int rem = e % D4;
        int idx[4];
        for (int q = 3; q >= 0; --q) { idx[q] = rem % D; rem /= D; }
        double g = 0.0, pe = 0.0;
        for (int gg = 0; gg < 8; ++gg) {
            int src[4];
            for (int q = 0; q < 4; ++q) src[q] = idx[c4v_pos(gg, q)];
            const int j = s * D4 + ((src[0] * D + src[1]) * D + src[2]) * D + src[3];
            g += Asb[j];
            pe += (j == im) ? 1.0 : 0.0;
        }
        dA[e] = 0.125 * g / m - coef * 0.125 * pe;
    }
}

__global__ void ratio_min_kernel(const double* __restrict__ r, double* acc, int reset) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc = reset ? *r : fmin(*acc, *r);
}

int grid(long long n) {
    long long b = ceil_div(n, kThreads);
    if (b < 1) b = 1;
    if (b > kBlocks) b = kBlocks;
    return (int)b;
}

}  // namespace

size_t sym_norm_backward_scratch_bytes() { return sizeof(double) * 2 * kBlocks; }

Status sym_norm_backward(const double* Cn, const double* Tn, const double* Cb, const double* Tb,
                         const double* norms, int chi, int Dab, double* Cpb, double* Tpb,
                         double* part, hipStream_t st) {
    const long long nC = (long long)chi * chi, nT = nC * Dab;
    const int b = grid(nC + nT);
    hipLaunchKernelGGL(dots_kernel, dim3(b), dim3(kThreads), 0, st, Cn, Cb, Tn, Tb, nC, nT, part);
    QRCTM_TRY(launch_check("dots_kernel"));
    hipLaunchKernelGGL(sym_norm_bwd_kernel, dim3(b), dim3(kThreads), 0, st, part, b, norms, Cn, Cb, Tn,
                       Tb, chi, Dab, Cpb, Tpb);
    return launch_check("sym_norm_bwd_kernel");
}

__global__ __launch_bounds__(kThreads) void diff_sq_kernel(const double* __restrict__ C1,
                                                           const double* __restrict__ C0,
                                                           const double* __restrict__ T1,
                                                           const double* __restrict__ T0,
                                                           long long nC, long long nT, double* part) {
    __shared__ double r[kThreads];
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        const double v = e < nC ? C1[e] - C0[e] : T1[e - nC] - T0[e - nC];
        acc += v * v;
    }
    r[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r[0];
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

Status sq_diff(const double* C1, const double* C0, const double* T1, const double* T0,
               long long nC, long long nT, double* part, double* out, hipStream_t st) {
    const int b = grid(nC + nT);
    hipLaunchKernelGGL(diff_sq_kernel, dim3(b), dim3(kThreads), 0, st, C1, C0, T1, T0, nC, nT, part);
    QRCTM_TRY(launch_check("diff_sq_kernel"));
    std::vector<double> h(2 * (size_t)b);
    QRCTM_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    QRCTM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v;
    *out = s;
    return Status{};
}

Status sq_norm(const double* Cb, const double* Tb, long long nC, long long nT, double* part,
               double* out, hipStream_t st) {
    const int b = grid(nC + nT);
    hipLaunchKernelGGL(dots_kernel, dim3(b), dim3(kThreads), 0, st, Cb, Cb, Tb, Tb, nC, nT, part);
    QRCTM_TRY(launch_check("dots_kernel"));
    std::vector<double> h(2 * (size_t)b);
    QRCTM_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    QRCTM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v;
    *out = s;
    return Status{};
}

Status copyltu(const double* M, int n, double* Ms, hipStream_t st) {
    hipLaunchKernelGGL(copyltu_kernel, dim3(grid((long long)n * n)), dim3(kThreads), 0, st, M, n, Ms);
    return launch_check("copyltu_kernel");
}

Status reg_recip_diag(const double* R, int n, double eps_rel, double* dinv, hipStream_t st) {
    hipLaunchKernelGGL(reg_recip_diag_kernel, dim3(1), dim3(256), 0, st, R, n, eps_rel, dinv);
    return launch_check("reg_recip_diag_kernel");
}

Status tri_inv_upper(const double* R, int n, double* Ri, double* scratch, hipStream_t st,
                     const double* dinv) {
    const size_t lds = sizeof(double) * ((size_t)n * (n + 1) / 2 + (size_t)n);
    if (n <= kTriThreads && lds <= (size_t)kTriMaxLds) {
        QRCTM_HIP(hipFuncSetAttribute((const void*)tri_inv_col_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(tri_inv_col_kernel, dim3(n), dim3(kTriThreads), lds, st, R, n, Ri, dinv);
        return launch_check("tri_inv_col_kernel");
    }
    if (scratch != nullptr && n <= 1024) {
        const int nb = (int)ceil_div(n, 16);
        hipLaunchKernelGGL(transpose_kernel, dim3(nb, nb), dim3(16, 16), 0, st, R, n, scratch);
        QRCTM_TRY(launch_check("transpose_kernel"));
        hipLaunchKernelGGL(tri_inv_col_l2_kernel, dim3(n), dim3(kTriThreads), 0, st, scratch, n, Ri,
                           dinv);
        return launch_check("tri_inv_col_l2_kernel");
    }
    hipLaunchKernelGGL(tri_inv_upper_kernel, dim3((int)ceil_div(n, 64)), dim3(64), 0, st, R, n, Ri,
                       dinv);
    return launch_check("tri_inv_upper_kernel");
}

Status double_layer_backward(const double* abar, const double* As, int d, int D, double* Asb,
                             hipStream_t st) {
    const long long n = (long long)d * D * D * D * D;
    hipLaunchKernelGGL(dl_backward_kernel, dim3((int)ceil_div(n, 64)), dim3(64), 0, st, abar, As, d,
                       D, Asb);
    return launch_check("dl_backward_kernel");
}

Status open_layer_backward(const double* aob, const double* As, int D, int s, int t, double* Asb,
                           hipStream_t st) {
    const int D4 = D * D * D * D;
    for (int bra = 0; bra < 2; ++bra) {
        hipLaunchKernelGGL(open_layer_bw_kernel, dim3((int)ceil_div(D4, 64)), dim3(64), 0, st, aob, As,
                           D, s, t, bra, Asb);
        QRCTM_TRY(launch_check("open_layer_bw_kernel"));
    }
    return Status{};
}

Status c4v_backward(const double* Asb, const double* As, const double* scale, const int* imax,
                    int d, int D, double* dA, hipStream_t st) {
    hipLaunchKernelGGL(c4v_backward_kernel, dim3(1), dim3(1024), 0, st, Asb, As, scale, imax, d, D,
                       dA);
    return launch_check("c4v_backward_kernel");
}

Status ratio_min(const double* r, double* acc, bool reset, hipStream_t st) {
    hipLaunchKernelGGL(ratio_min_kernel, dim3(1), dim3(64), 0, st, r, acc, reset ? 1 : 0);
    return launch_check("ratio_min_kernel");
}

}  // namespace qrctm
