// Corner spectrum and its change, the convergence measure of the CTMRG loop
// (the standard-CTMRG paragraph iterates the step to convergence; the change
// in the normalised corner spectrum is the measure used here).
//
// Three kernels on the caller's stream:
//  * tridiag_kernel, one workgroup of 512 threads: Householder
//    tridiagonalisation of the symmetric chi x chi corner, keeping only its
//    lower triangle (packed in LDS up to chi = 176, beyond that row-major in
//    global scratch, L2 resident).  The rank-2 update of each reflection is
//    applied lazily, in the same sweep of the trailing triangle that forms the
//    next reflection's product A v, so each reflection reads and writes the
//    triangle once.  Writes the diagonal, the squared off-diagonal and a
//    Gershgorin interval;
//  * bisect_kernel, one wave per eigenvalue over as many workgroups as needed:
//    Sturm-sequence multisection, the 64 lanes each placing two of the 128
//    interior points that cut the interval, until it stops shrinking or is
//    within 2 eps relative / 4 eps |T| absolute;
//  * rank_kernel, one workgroup: |lambda| ranked in descending order (ties by
//    index), normalised by their sum, and delta = || s - s_prev ||_2 with the
//    shorter spectrum padded by zeros.
// Every reduction has a fixed order, so the result does not vary between runs.
#include "common.h"
#include "spectrum.h"

namespace qrctm {
namespace {

constexpr int kSpecThreads = 512;
constexpr int kSpecWaves = kSpecThreads / 64;
constexpr int kMaxN = 1024;
constexpr int kLdsMaxN = 176;

// lane permutation of a double within rows of 16 lanes (DPP control word CTRL)
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave (all lanes active); every lane gets the same
// value.  Butterfly within rows of 16 (xor 1, xor 2, mirror of 8, mirror of
// 16), then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_perm<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_perm<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_perm<0x141>(v);  // row_half_mirror
    v += dpp_perm<0x140>(v);  // row_mirror
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sums over the 64 lanes of eight values at once.  Each fold adds lanes a
// distance apart and keeps, per lane, the half belonging to one value, so one
// register ends up holding all eight: lane l (of any 16) holds the sum of
// value row8(l & 15).  Folds: distance 8 (row_ror:8), mirror within 8, xor 2,
// xor 1 (within rows of 16), then across the four rows of 16.
__device__ __forceinline__ int row8(int p) { return ((p & 2) ? 4 : 0) + ((p & 4) ? 2 : 0) + ((p & 8) ? 1 : 0); }
__device__ __forceinline__ double sum8(const double* v) {
    const int p = threadIdx.x & 15;
    double s4[4], s2[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double a = v[2 * q] + dpp_perm<0x128>(v[2 * q]);
        const double b = v[2 * q + 1] + dpp_perm<0x128>(v[2 * q + 1]);
        s4[q] = (p & 8) ? b : a;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double a = s4[2 * q] + dpp_perm<0x141>(s4[2 * q]);
        const double b = s4[2 * q + 1] + dpp_perm<0x141>(s4[2 * q + 1]);
        s2[q] = (p & 4) ? b : a;
    }
    const double a = s2[0] + dpp_perm<0x4E>(s2[0]);
    const double b = s2[1] + dpp_perm<0x4E>(s2[1]);
    double x = (p & 2) ? b : a;
    x += dpp_perm<0xB1>(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// Sum over the workgroup, the same value in every thread.  part holds one
// slot per wave; two calls in a row must use different part buffers (the
// barrier of the second call orders the first call's reads before the third
// call's writes).
__device__ double block_sum(double v, double* part) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSpecWaves; ++w) s += part[w];
    return s;
}

// Sturm counts (eigenvalues below x) of the tridiagonal matrix (d, e^2) at NP
// points, their recurrences interleaved.  1/q is the hardware reciprocal with
// two Newton steps; |q| >= pivmin = 1e-300 max(1, max e^2) keeps every value
// finite.
template <int NP>
__device__ void sturm_counts(const double* d, const double* e2, int n, const double* x,
                             double pivmin, int* cnt) {
    double q[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        q[p] = d[0] - x[p];
        if (fabs(q[p]) < pivmin) q[p] = -pivmin;
        cnt[p] = q[p] < 0.0;
    }
    auto step = [&](double dj, double ej) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double r = __builtin_amdgcn_rcp(q[p]);
            double h = fma(-q[p], r, 1.0);
            r = fma(r, h, r);
            h = fma(-q[p], r, 1.0);
            r = fma(r, h, r);
            double qq = fma(-ej, r, dj - x[p]);
            if (fabs(qq) < pivmin) qq = -pivmin;
            q[p] = qq;
            cnt[p] += qq < 0.0;
        }
    };
    // eight entries of (d, e^2) read ahead of their use
    int j = 1;
    for (; j + 8 <= n; j += 8) {
        double dv[8], ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dv[u] = d[j + u];
            ev[u] = e2[j + u - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) step(dv[u], ev[u]);
    }
    for (; j < n; ++j) step(d[j], e2[j - 1]);
}

// Lower triangle of the symmetric matrix: rows of a row-major n x n array in
// global scratch, or the packed triangle in LDS (row i at i(i+1)/2).
struct GlobalSym {
    double* S;
    int n;
    __device__ double* row(int i) const { return S + (size_t)i * n; }
    static constexpr bool kInLds = false;
};
struct LdsSym {
    double* S;
    int n;
    __device__ double* row(int i) const { return S + i * (i + 1) / 2; }
    static constexpr bool kInLds = true;
};


template <class Store, int MAXN>
__global__ __launch_bounds__(kSpecThreads) void tridiag_kernel(const double* __restrict__ C, int n,
                                                               double* Sg, double* tri) {
    constexpr int R = (MAXN + kSpecThreads - 1) / kSpecThreads;  // rows / eigenvalues per thread
    constexpr int NC = (MAXN + 63) / 64;                            // 64-column chunks of a row
    // vp, wp: the reflection whose rank-2 update is still pending; vk: the
    // current reflection; prow: row part of A v; dd, ee: the tridiagonal matrix
    __shared__ double vp[MAXN], wp[MAXN], vk[MAXN], prow[MAXN], dd[MAXN], ee[MAXN];
    __shared__ double part[2][kSpecWaves];
    __shared__ double alpha_sh;
    extern __shared__ double dyn[];
    double* pcol = dyn;  // [kSpecWaves][n]: column part of A v, one row per wave
    Store A;
    A.S = Store::kInLds ? dyn + (size_t)kSpecWaves * n : Sg;
    A.n = n;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int pb = 0;

    for (int i = wv; i < n; i += kSpecWaves) {
        double* ri = A.row(i);
        for (int j = lane; j <= i; j += 64) ri[j] = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
    }
    for (int i = t; i < n; i += kSpecThreads) {
        vp[i] = 0.0;
        wp[i] = 0.0;
    }
    __syncthreads();

    // Reflection k zeroes column k below the subdiagonal of the current matrix
    // A_k = S - vp wp^T - wp vp^T (on rows and columns > k-1); vph, wph are
    // vp[k], wp[k], held by every thread.
    double vph = 0.0, wph = 0.0;
    for (int k = 0; k + 2 < n; ++k) {
        double x[R];
        double s2 = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kSpecThreads;
            x[r] = 0.0;
            if (i > k && i < n) {
                const double c = A.row(i)[k] - vp[i] * wph - wp[i] * vph;
                x[r] = c;
                if (i > k + 1) s2 += c * c;
                else alpha_sh = c;
            }
        }
        if (t == 0) dd[k] = A.row(k)[k] - 2.0 * vph * wph;
        const double sigma2 = block_sum(s2, part[pb]);
        pb ^= 1;
        const double alpha = alpha_sh;
        double tau = 0.0, scal = 0.0, beta = alpha;
        if (sigma2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (t == 0) ee[k] = beta;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kSpecThreads;
            if (i > k && i < n) vk[i] = (i == k + 1) ? 1.0 : x[r] * scal;
        }
        __syncthreads();

        // one sweep of the trailing triangle (rows, columns > k): apply the
        // pending update, store, and accumulate A_{k+1} v by rows (prow) and,
        // for the strictly lower part, by columns (pc, per lane).  A wave takes
        // its rows eight at a time, every 64-column chunk of the eight loaded
        // together, and sums the eight row parts in one reduction.
        // (for the widest rows the column parts stay in the wave's pcol row:
        // lane (j - k - 1) % 64 alone touches entry j)
        constexpr bool kPcInLds = MAXN > 512;
        double pc[kPcInLds ? 1 : NC];
        if (kPcInLds) {
            for (int j = k + 1 + lane; j < n; j += 64) pcol[wv * n + j] = 0.0;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) pc[c] = 0.0;
        }
        for (int i0 = k + 1 + wv; i0 < n; i0 += 8 * kSpecWaves) {
            double acc[8], vi[8], wi[8], vki[8];
            int nchm = 0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int i = i0 + b * kSpecWaves;
                const int ii = i < n ? i : k + 1;
                vi[b] = vp[ii];
                wi[b] = wp[ii];
                vki[b] = vk[ii];
                acc[b] = 0.0;
                if (i < n) nchm = (i - k - 1) / 64 + 1;
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < nchm) {
                    const int j = k + 1 + c * 64 + lane;
                    const int jj = j < n ? j : n - 1;
                    const double vpj = vp[jj], wpj = wp[jj], vkj = vk[jj];
                    double a[8];
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        const int i = i0 + b * kSpecWaves;
                        if (i < n && j <= i) a[b] = A.row(i)[j];
                    }
                    double col = 0.0;
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        const int i = i0 + b * kSpecWaves;
                        if (i < n && j <= i) {
                            const double y = a[b] - vi[b] * wpj - wi[b] * vpj;
                            A.row(i)[j] = y;
                            acc[b] += y * vkj;
                            if (j < i) col += y * vki[b];
                        }
                    }
                    if (kPcInLds) {
                        if (j < n) pcol[wv * n + j] += col;
                    } else {
                        pc[c] += col;
                    }
                }
            }
            const double rs = sum8(acc);
            const int i = i0 + row8(lane & 15) * kSpecWaves;
            if (lane < 16 && (lane & 1) == 0 && i < n) prow[i] = rs;
        }
        if (!kPcInLds) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int j = k + 1 + c * 64 + lane;
                if (j < n) pcol[wv * n + j] = pc[kPcInLds ? 0 : c];
            }
        }
        __syncthreads();

        // p = tau A_{k+1} v, K = tau p^T v / 2, w = p - K v becomes the pending update
        double pr[R];
        double pv = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kSpecThreads;
            pr[r] = 0.0;
            if (i > k && i < n) {
                double sum = prow[i];
#pragma unroll
                for (int w = 0; w < kSpecWaves; ++w) sum += pcol[w * n + i];
                pr[r] = tau * sum;
                pv += pr[r] * vk[i];
            }
        }
        double head = prow[k + 1];
#pragma unroll
        for (int w = 0; w < kSpecWaves; ++w) head += pcol[w * n + k + 1];
        const double K = 0.5 * tau * block_sum(pv, part[pb]);
        pb ^= 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kSpecThreads;
            if (i > k && i < n) {
                const double v = vk[i];
                vp[i] = v;
                wp[i] = pr[r] - K * v;
            }
        }
        vph = 1.0;  // vk[k+1]
        wph = tau * head - K;
    }
    __syncthreads();
    if (t == 0) {
        if (n >= 2) {
            const double va = vp[n - 2], vb = vp[n - 1], wa = wp[n - 2], wb = wp[n - 1];
            dd[n - 2] = A.row(n - 2)[n - 2] - 2.0 * va * wa;
            dd[n - 1] = A.row(n - 1)[n - 1] - 2.0 * vb * wb;
            ee[n - 2] = A.row(n - 1)[n - 2] - vb * wa - wb * va;
        } else {
            dd[0] = A.row(0)[0];
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
    const double pivmin = 1e-300 * fmax(1.0, me2);
    const double span = fmax(fabs(lo), fabs(hi));
    // d, e^2, the widened Gershgorin interval and the absolute tolerance
    // (4 eps |T|) of the eigenvalues
    for (int i = t; i < n; i += kSpecThreads) {
        tri[i] = dd[i];
        tri[n + i] = i + 1 < n ? ee[i] * ee[i] : 0.0;
    }
    if (t == 0) {
        tri[2 * n] = lo - (2.2e-16 * span * n + pivmin);
        tri[2 * n + 1] = hi + (2.2e-16 * span * n + pivmin);
        tri[2 * n + 2] = pivmin;
        tri[2 * n + 3] = 4.0 * 2.2e-16 * span + pivmin;
    }
}

// |lambda_e| of the tridiagonal matrix for e = one per wave (ascending index):
// multisection over the Gershgorin interval, 128 points per round (two per
// lane, interleaved recurrences), the wave keeping the part that holds the
// eigenvalue, until the width is 2 eps max(|a|, |b|) + atol or stops falling.
constexpr int kBisWaves = 4;
__global__ __launch_bounds__(64 * kBisWaves) void bisect_kernel(const double* __restrict__ tri, int n,
                                                                double* lam) {
    extern __shared__ double sh[];
    double* d = sh;
    double* e2 = sh + n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        d[i] = tri[i];
        e2[i] = tri[n + i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * kBisWaves + (threadIdx.x >> 6);
    if (e >= n) return;
    double a = tri[2 * n], b = tri[2 * n + 1];
    const double pivmin = tri[2 * n + 2], atol = tri[2 * n + 3];
    constexpr int NP = 2, M = 64 * NP;
    for (int it = 0; it < 64; ++it) {
        if (!(b - a > 2.0 * 2.2e-16 * fmax(fabs(a), fabs(b)) + atol)) break;
        const double h = (b - a) / (M + 1);
        double x[NP];
        int cnt[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) x[p] = a + (double)(lane * NP + p + 1) * h;
        sturm_counts<NP>(d, e2, n, x, pivmin, cnt);
        double na = a, nb = b;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (cnt[p] > e) nb = fmin(nb, x[p]);
            else na = fmax(na, x[p]);
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            na = fmax(na, __shfl_xor(na, o, 64));
            nb = fmin(nb, __shfl_xor(nb, o, 64));
        }
        if (na == a && nb == b) break;
        a = na;
        b = nb;
    }
    if (lane == 0) lam[e] = fabs(0.5 * (a + b));
}

// Rank |lambda| descending (ties by index), normalise, and the change against
// s_prev (one workgroup).
constexpr int kRankThreads = 1024;
__global__ __launch_bounds__(kRankThreads) void rank_kernel(const double* __restrict__ lam, int n,
                                                            const double* s_prev, int n_prev,
                                                            double* s_out, double* delta_out) {
    __shared__ double sorted[kMaxN];
    __shared__ double part[2][kRankThreads / 64];
    const int t = threadIdx.x;
    for (int e = t; e < n; e += kRankThreads) {
        const double mine = lam[e];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double o = lam[j];
            rank += (o > mine) || (o == mine && j < e);
        }
        sorted[rank] = mine;
    }
    __syncthreads();
    auto bsum = [&](double v, double* pt) {
        v = wave_sum(v);
        if ((t & 63) == 0) pt[t >> 6] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kRankThreads / 64; ++w) s += pt[w];
        return s;
    };
    double ps = 0.0;
    for (int i = t; i < n; i += kRankThreads) ps += sorted[i];
    const double inv = 1.0 / bsum(ps, part[0]);
    double dl = 0.0;
    const int nmax = n > n_prev ? n : n_prev;
    for (int i = t; i < nmax; i += kRankThreads) {
        const double si = i < n ? sorted[i] * inv : 0.0;
        const double sp = (s_prev != nullptr && i < n_prev) ? s_prev[i] : 0.0;
        if (i < n) s_out[i] = si;
        dl += (si - sp) * (si - sp);
    }
    const double dsum = bsum(dl, part[1]);
    if (t == 0) *delta_out = sqrt(dsum);
}

}  // namespace

size_t spectrum_scratch_bytes(int n) { return sizeof(double) * ((size_t)n * n + 3 * (size_t)n + 8); }

Status corner_spectrum(const double* C, int n, double* S, const double* s_prev, int n_prev,
                       double* s_out, double* delta_out, hipStream_t st) {
    Status s;
    if (n < 1 || n > kMaxN) {
        s.code = -1;
        s.msg = "spectrum: chi must be in [1, 1024]";
        return s;
    }
    double* tri = S + (size_t)n * n;      // d, e^2, interval, tolerance
    double* lam = tri + 2 * (size_t)n + 4;
    auto launch = [&](auto kern, size_t tri_doubles) -> Status {
        const size_t dyn = sizeof(double) * ((size_t)kSpecWaves * n + tri_doubles);
        QRCTM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)dyn));
        hipLaunchKernelGGL(kern, dim3(1), dim3(kSpecThreads), dyn, st, C, n, S, tri);
        return launch_check("tridiag_kernel");
    };
    if (n <= kLdsMaxN) QRCTM_TRY(launch(tridiag_kernel<LdsSym, kLdsMaxN>, (size_t)n * (n + 1) / 2));
    else if (n <= 512) QRCTM_TRY(launch(tridiag_kernel<GlobalSym, 512>, 0));
    else QRCTM_TRY(launch(tridiag_kernel<GlobalSym, kMaxN>, 0));
    hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)ceil_div(n, kBisWaves)), dim3(64 * kBisWaves),
                       sizeof(double) * 2 * (size_t)n, st, tri, n, lam);
    QRCTM_TRY(launch_check("bisect_kernel"));
    hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(kRankThreads), 0, st, lam, n, s_prev, n_prev, s_out,
                       delta_out);
    return launch_check("rank_kernel");
}

}  // namespace qrctm
