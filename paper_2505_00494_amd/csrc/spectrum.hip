// Corner spectrum and its change, the convergence measure of the CTMRG loop
// (the standard-CTMRG paragraph iterates the step to convergence; the change
// in the normalised corner spectrum is the measure used here).
//
// One kernel of one workgroup (512 threads) on the caller's stream, so that
// beside a running step it occupies a single CU (with all of that CU's LDS, so
// that no workgroup of the step shares it):
//  * Householder tridiagonalisation of the symmetric chi x chi corner, keeping
//    only its lower triangle (packed in LDS up to chi = 176, beyond that
//    row-major in global scratch, L2 resident).  The rank-2 update of each
//    reflection is applied lazily, in the same sweep of the trailing triangle
//    that forms the next reflection's product A v, so each reflection reads and
//    writes the triangle once;
//  * Sturm-sequence multisection over the Gershgorin interval: one round of
//    512 evenly spaced points brackets every eigenvalue, then each eigenvalue
//    gets a group of lanes of one wave (64 / ceil(chi / 8) of them), which cut
//    its interval at one point each per round, until it stops shrinking or is
//    within 2 eps relative / 4 eps |T| absolute;
//  * |lambda| ranked in descending order (ties by index), normalised by their
//    sum, and delta = || s - s_prev ||_2 with the shorter spectrum padded by
//    zeros.
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
// points, their recurrences interleaved.  The count is the number of negative
// pivots q_j = d_j - x - e^2_{j-1} / q_{j-1} of T - x I = L D L^T; here without
// the division, through the leading minors p_j = (d_j - x) p_{j-1} - e^2_{j-1}
// p_{j-2} (q_j = p_j / p_{j-1}, negative where the two signs differ), the pair
// (p_j, p_{j-1}) scaled by a power of two after every step so that p_j lies in
// [1/2, 1).  A pivot below pivmin = 1e-300 max(1, max e^2) in magnitude is
// replaced by -pivmin (p_j = -pivmin p_{j-1}), which keeps every value finite.
template <int NP>
__device__ void sturm_counts(const double* d, const double* e2, int n, const double* x,
                             double pivmin, int* cnt) {
    double u[NP], v[NP];  // p_j and p_{j-1}, scaled
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        u[p] = d[0] - x[p];
        if (fabs(u[p]) < pivmin) u[p] = -pivmin;
        v[p] = 1.0;
        cnt[p] = u[p] < 0.0;
    }
    auto step = [&](double dj, double ej) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double un = fma(dj - x[p], u[p], -(ej * v[p]));
            if (fabs(un) < pivmin * fabs(u[p])) un = -pivmin * u[p];
            cnt[p] += (un < 0.0) != (u[p] < 0.0);
            // 2^(1022 - e) for the biased exponent e of un, built from its bits
            // (pivmin <= |un / u| <= 1/pivmin keeps e within [24, 2020])
            const unsigned ex = (unsigned)(__double_as_longlong(un) >> 52) & 0x7ffu;
            const double sc = __longlong_as_double((long long)(2045u - ex) << 52);
            v[p] = u[p] * sc;
            u[p] = un * sc;
        }
    };
    // eight entries of (d, e^2) read ahead of their use
    int j = 1;
    for (; j + 8 <= n; j += 8) {
        double dv[8], ev[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            dv[w] = d[j + w];
            ev[w] = e2[j + w - 1];
        }
#pragma unroll
        for (int w = 0; w < 8; ++w) step(dv[w], ev[w]);
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
__global__ __launch_bounds__(kSpecThreads) void spectrum_kernel(const double* __restrict__ C, int n,
                                                                double* Sg, const double* s_prev,
                                                                int n_prev, double* s_out,
                                                                double* delta_out) {
    constexpr int R = (MAXN + kSpecThreads - 1) / kSpecThreads;  // rows / eigenvalues per thread
    constexpr int NC = (MAXN + 63) / 64;                            // 64-column chunks of a row
    // vp, wp: the reflection whose rank-2 update is still pending; vk: the
    // current reflection; prow: row part of A v; dd, ee: the tridiagonal matrix
    __shared__ double vp[MAXN], wp[MAXN], vk[MAXN], prow[MAXN], dd[MAXN], ee[MAXN];
    __shared__ double part[2][kSpecWaves];
    __shared__ int cgrid[kSpecThreads];  // Sturm counts of the bracketing points
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
    // the widened interval and the absolute tolerance (4 eps |T|) of the eigenvalues
    lo -= 2.2e-16 * span * n + pivmin;
    hi += 2.2e-16 * span * n + pivmin;
    const double atol = 4.0 * 2.2e-16 * span + pivmin;
    // e^2 (in wp) and the eigenvalue magnitudes (in vk); the reflection arrays are free
    double* e2 = wp;
    double* lam = vk;
    for (int i = t; i < n; i += kSpecThreads) e2[i] = i + 1 < n ? ee[i] * ee[i] : 0.0;
    __syncthreads();

    // Bracketing: the counts at kSpecThreads evenly spaced points of the
    // interval, one per thread; eigenvalue e starts from the two neighbouring
    // points whose counts enclose it (found by bisection over the points, with
    // count(lo) = 0 and count(hi) = n at the ends).
    const double hg = (hi - lo) / (double)(kSpecThreads + 1);
    {
        const double x = lo + (double)(t + 1) * hg;
        int cnt;
        sturm_counts<1>(dd, e2, n, &x, pivmin, &cnt);
        cgrid[t] = cnt;
    }
    __syncthreads();
    // Multisection: eigenvalue e (ascending) gets a group of L lanes of one wave,
    // which cut its interval at one point each per round and keep the part that
    // holds it, until the width is 2 eps max(|a|, |b|) + atol or stops falling.  G groups per wave cover kSpecWaves G eigenvalues per pass.
    const int G = min(64, (n + kSpecWaves - 1) / kSpecWaves);
    const int L = 64 / G;
    const int g = lane / L, sub = lane % L;
    for (int base = 0; base < n; base += kSpecWaves * G) {
        const int e = base + wv * G + g;
        bool act = g < G && e < n;
        const bool valid = act;
        int jl = -1, jh = kSpecThreads;  // count(point jl) <= e < count(point jh)
        while (jh - jl > 1) {
            const int jm = (jl + jh) >> 1;
            if (cgrid[jm] <= (valid ? e : n)) jl = jm;
            else jh = jm;
        }
        double a = jl < 0 ? lo : lo + (double)(jl + 1) * hg;
        double b = jh >= kSpecThreads ? hi : lo + (double)(jh + 1) * hg;
        for (int it = 0; it < 4096; ++it) {
            act = act && (b - a > 2.0 * 2.2e-16 * fmax(fabs(a), fabs(b)) + atol);
            if (!__any(act)) break;
            const double x = a + (double)(sub + 1) * ((b - a) / (double)(L + 1));
            int cnt;
            sturm_counts<1>(dd, e2, n, &x, pivmin, &cnt);
            double na = cnt <= e ? x : a, nb = cnt > e ? x : b;
            for (int j = 0; j < L; ++j) {
                const int src = g * L + j;
                na = fmax(na, __shfl(na, src, 64));
                nb = fmin(nb, __shfl(nb, src, 64));
            }
            if (act) {
                if (na == a && nb == b) act = false;
                a = na;
                b = nb;
            }
        }
        if (valid && sub == 0) lam[e] = fabs(0.5 * (a + b));
    }
    __syncthreads();

    // |lambda| ranked in descending order (ties by index), normalised, and the
    // change against s_prev with the shorter spectrum padded by zeros
    double* sorted = prow;
    for (int e = t; e < n; e += kSpecThreads) {
        const double mine = lam[e];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double o = lam[j];
            rank += (o > mine) || (o == mine && j < e);
        }
        sorted[rank] = mine;
    }
    __syncthreads();
    double ps = 0.0;
    for (int i = t; i < n; i += kSpecThreads) ps += sorted[i];
    const double inv = 1.0 / block_sum(ps, part[pb]);
    pb ^= 1;
    double dl = 0.0;
    const int nmax = n > n_prev ? n : n_prev;
    for (int i = t; i < nmax; i += kSpecThreads) {
        const double si = i < n ? sorted[i] * inv : 0.0;
        const double sp = (s_prev != nullptr && i < n_prev) ? s_prev[i] : 0.0;
        if (i < n) s_out[i] = si;
        dl += (si - sp) * (si - sp);
    }
    const double dsum = block_sum(dl, part[pb]);
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
    auto launch = [&](auto kern, size_t tri_doubles) -> Status {
        size_t dyn = sizeof(double) * ((size_t)kSpecWaves * n + tri_doubles);
        {
            // all of the CU's LDS, so that no workgroup of the step beside it
            // shares the CU (measured at D = 6, chi = 144: the spectrum beside the
            // step 866 -> 837 us, the step 1185 -> 1195 steps/s)
            hipFuncAttributes fa;
            QRCTM_HIP(hipFuncGetAttributes(&fa, (const void*)kern));
            const size_t whole = 160 * 1024;
            if (fa.sharedSizeBytes + dyn < whole) dyn = whole - fa.sharedSizeBytes;
        }
        QRCTM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)dyn));
        hipLaunchKernelGGL(kern, dim3(1), dim3(kSpecThreads), dyn, st, C, n, S, s_prev, n_prev, s_out,
                           delta_out);
        return launch_check("spectrum_kernel");
    };
    if (n <= kLdsMaxN) return launch(spectrum_kernel<LdsSym, kLdsMaxN>, (size_t)n * (n + 1) / 2);
    if (n <= 512) return launch(spectrum_kernel<GlobalSym, 512>, 0);
    return launch(spectrum_kernel<GlobalSym, kMaxN>, 0);
}

}  // namespace qrctm
