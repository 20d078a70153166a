// Corner spectrum and its change, the convergence measure of the CTMRG loop
// (standard-CTMRG paragraph: iterate "until convergence"; the change in the
// normalised corner spectrum is the measure used here).
//
// One workgroup of 1024 threads: Householder tridiagonalisation of the
// symmetric chi x chi corner (packed lower triangle in LDS up to chi = 176;
// beyond that in global scratch, L2 resident, both triangles kept so every
// access is a coalesced row access), eigenvalues of the
// tridiagonal matrix by Sturm-sequence bisection (one eigenvalue per thread),
// |lambda| ranked in descending order (ties by index), normalised by their sum,
// and delta = || s - s_prev ||_2 with the shorter spectrum padded by zeros.
#include "common.h"
#include "spectrum.h"

namespace qrctm {
namespace {

constexpr int kSpecThreads = 1024;
constexpr int kMaxN = 1024;

__device__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = kSpecThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    for (int j = 1; j < n; ++j) {
        q = d[j] - x - e2[j - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Symmetric matrix storage: full rows in global scratch (any n), or the packed
// lower triangle in LDS (n <= kLdsMaxN), index i(i+1)/2 + j for i >= j.
struct GlobalSym {
    double* S;
    int n;
    __device__ double get(int i, int j) const { return S[(size_t)i * n + j]; }
    __device__ void sub(int i, int j, double v) { S[(size_t)i * n + j] -= v; }
    __device__ void set(int i, int j, double v) { S[(size_t)i * n + j] = v; }
    static constexpr bool kBothTriangles = true;
};
struct LdsSym {
    double* S;
    int n;
    __device__ static int idx(int i, int j) { return i * (i + 1) / 2 + j; }
    __device__ double get(int i, int j) const { return i >= j ? S[idx(i, j)] : S[idx(j, i)]; }
    __device__ void sub(int i, int j, double v) { S[idx(i, j)] -= v; }
    __device__ void set(int i, int j, double v) { S[idx(i, j)] = v; }
    static constexpr bool kBothTriangles = false;
};

constexpr int kLdsMaxN = 176;

template <class Store, int MAXN>
__global__ __launch_bounds__(kSpecThreads) void spectrum_kernel(const double* __restrict__ C, int n,
                                                                double* Sg, const double* s_prev,
                                                                int n_prev, double* s_out,
                                                                double* delta_out) {
    __shared__ double v[MAXN], p[MAXN], dd[MAXN], ee[MAXN], lam[MAXN], red[kSpecThreads];
    extern __shared__ double dyn[];
    Store A;
    A.S = Store::kBothTriangles ? Sg : dyn;
    A.n = n;
    const int t = threadIdx.x;
    for (long long q = t; q < (long long)n * n; q += kSpecThreads) {
        const int i = (int)(q / n), j = (int)(q % n);
        if (Store::kBothTriangles || i >= j) A.set(i, j, 0.5 * (C[q] + C[(size_t)j * n + i]));
    }
    __syncthreads();

    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        // x = column k below the diagonal (rows k+1 .. n-1)
        double part = 0.0;
        for (int i = 1 + t; i < m; i += kSpecThreads) {
            const double xi = A.get(k + 1 + i, k);
            part += xi * xi;
        }
        const double sigma2 = block_sum(part, red);
        const double alpha = A.get(k + 1, k);
        if (t == 0) dd[k] = A.get(k, k);
        if (sigma2 == 0.0) {
            if (t == 0) ee[k] = alpha;
            __syncthreads();
            continue;
        }
        const double beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
        const double tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int i = t; i < m; i += kSpecThreads) v[i] = (i == 0) ? 1.0 : A.get(k + 1 + i, k) * scal;
        if (t == 0) ee[k] = beta;
        __syncthreads();
        // p = tau * A22 v (A22 symmetric; the global store reads column i as row i):
        // row i is split into nc chunks handled by different threads, the
        // chunk sums are combined through LDS in a fixed order
        {
            const int nc = max(1, min(kSpecThreads / m, 32));
            const int len = (m + nc - 1) / nc;
            const int i = t % m, c = t / m;
            if (c < nc) {
                const int j0 = c * len, j1 = min(m, j0 + len);
                double acc = 0.0;
                for (int jx = j0; jx < j1; ++jx) acc += A.get(k + 1 + jx, k + 1 + i) * v[jx];
                red[c * m + i] = acc;
            }
            __syncthreads();
            for (int ii = t; ii < m; ii += kSpecThreads) {
                double acc = 0.0;
                for (int cc = 0; cc < nc; ++cc) acc += red[cc * m + ii];
                p[ii] = tau * acc;
            }
            __syncthreads();
        }
        double pv = 0.0;
        for (int i = t; i < m; i += kSpecThreads) pv += p[i] * v[i];
        const double K = 0.5 * tau * block_sum(pv, red);
        for (int i = t; i < m; i += kSpecThreads) p[i] -= K * v[i];  // w
        __syncthreads();
        {   // rank-2 update, 32 column lanes x 32 row groups
            const int cl = t % 32, rg = t / 32;
            for (int i = rg; i < m; i += kSpecThreads / 32) {
                const int jend = Store::kBothTriangles ? m : i + 1;
                const double vi = v[i], pi = p[i];
                for (int jx = cl; jx < jend; jx += 32)
                    A.sub(k + 1 + i, k + 1 + jx, vi * p[jx] + pi * v[jx]);
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            dd[n - 2] = A.get(n - 2, n - 2);
            dd[n - 1] = A.get(n - 1, n - 1);
            ee[n - 2] = A.get(n - 1, n - 2);
        } else {
            dd[0] = A.get(0, 0);
        }
    }
    __syncthreads();
    // Gershgorin interval
    double lo = INFINITY, hi = -INFINITY, me2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double el = i > 0 ? fabs(ee[i - 1]) : 0.0;
        const double er = i + 1 < n ? fabs(ee[i]) : 0.0;
        lo = fmin(lo, dd[i] - el - er);
        hi = fmax(hi, dd[i] + el + er);
        if (i + 1 < n) me2 = fmax(me2, ee[i] * ee[i]);
    }
    __syncthreads();
    for (int i = t; i + 1 < n; i += kSpecThreads) ee[i] = ee[i] * ee[i];
    __syncthreads();
    const double pivmin = 1e-300 * fmax(1.0, me2);
    const double span = fmax(fabs(lo), fabs(hi));
    lo -= 2.2e-16 * span * n + pivmin;
    hi += 2.2e-16 * span * n + pivmin;
    if (t < n) {
        double a = lo, b = hi;
        for (int it = 0; it < 256; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid == a || mid == b) break;
            if (sturm_count(dd, ee, n, mid, pivmin) > t) b = mid;
            else a = mid;
            if (b - a <= 2.0 * 2.2e-16 * fmax(fabs(a), fabs(b)) + pivmin) break;
        }
        lam[t] = fabs(0.5 * (a + b));
    }
    __syncthreads();
    // rank by |lambda| descending, ties by index
    double mine = 0.0;
    int rank = 0;
    if (t < n) {
        mine = lam[t];
        for (int jx = 0; jx < n; ++jx) {
            const double o = lam[jx];
            rank += (o > mine) || (o == mine && jx < t);
        }
    }
    __syncthreads();
    if (t < n) v[rank] = mine;
    __syncthreads();
    double ps = 0.0;
    for (int i = t; i < n; i += kSpecThreads) ps += v[i];
    const double total = block_sum(ps, red);
    const double inv = 1.0 / total;
    double dl = 0.0;
    const int nmax = n > n_prev ? n : n_prev;
    for (int i = t; i < nmax; i += kSpecThreads) {
        const double si = i < n ? v[i] * inv : 0.0;
        const double sp = (s_prev != nullptr && i < n_prev) ? s_prev[i] : 0.0;
        if (i < n) s_out[i] = si;
        dl += (si - sp) * (si - sp);
    }
    const double dsum = block_sum(dl, red);
    if (t == 0) *delta_out = sqrt(dsum);
}

}  // namespace

size_t spectrum_scratch_bytes(int n) { return sizeof(double) * (size_t)n * n; }

Status corner_spectrum(const double* C, int n, double* S, const double* s_prev, int n_prev,
                       double* s_out, double* delta_out, hipStream_t st) {
    Status s;
    if (n < 1 || n > kMaxN) {
        s.code = -1;
        s.msg = "spectrum: chi must be in [1, 1024]";
        return s;
    }
    if (n <= kLdsMaxN) {
        const size_t lds = sizeof(double) * (size_t)n * (n + 1) / 2;
        auto kern = spectrum_kernel<LdsSym, kLdsMaxN>;
        QRCTM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
        hipLaunchKernelGGL(kern, dim3(1), dim3(kSpecThreads), lds, st, C, n, S, s_prev, n_prev, s_out,
                           delta_out);
    } else {
        hipLaunchKernelGGL((spectrum_kernel<GlobalSym, kMaxN>), dim3(1), dim3(kSpecThreads), 0, st, C, n,
                           S, s_prev, n_prev, s_out, delta_out);
    }
    return launch_check("spectrum_kernel");
}

}  // namespace qrctm
