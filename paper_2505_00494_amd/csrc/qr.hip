// Thin Householder QR of a tall matrix M (m x n, m >= n) with diag(R) >= 0.
//
// QR-CTMRG replaces the eigen/SVD decomposition by an unpivoted QR of the
// reduced corner (QR-CTMRG paragraph, Fig. 1e).  The factorisation here is the
// Householder one, organised for a machine with 256 compute units:
//
//  1. qr_factor_kernel (cooperative launch, at most one workgroup per compute
//     unit): every workgroup keeps a contiguous block of rows of M in LDS for
//     the whole factorisation, using as few workgroups as LDS allows.  Column j
//     needs, over all rows below j, the sum of squares of column j and its dot
//     products with every later column; each workgroup reduces its rows
//     (wavefront-parallel over columns, LDS over row groups) in the same pass
//     that applies the previous reflector, publishes the partial sums, and after
//     ONE grid barrier (an atomic arrival counter) every workgroup combines
//     them in a fixed order, forms the reflector and updates its own rows.  The reflector is generated with beta = +||x|| (the
//     non-negative-diagonal variant, cancellation-free gamma = alpha - beta), so
//     R has diag(R) >= 0 without a sign fix.
//  2. the compact-WY factor T of H_0 ... H_{n-1} = I - V T V^T from the Gram
//     matrix G = V^T V (an FP64 MFMA GEMM) and tau (qr_tfactor_kernel);
//  3. the explicit thin factor Q = [I; 0] - V (T V1^T) by two more MFMA GEMMs
//     (V1 = first n rows of V).
#include "common.h"
#include "qr.h"

namespace qrctm {
namespace {

constexpr int kQrThreads = 512;
constexpr int kColGroup = 64;                      // column lanes of a row group
constexpr int kRowGroups = kQrThreads / kColGroup;  // row groups
constexpr int kMaxColsPerLane = 8;                  // n <= 512
constexpr size_t kQrLdsBudget = 155 * 1024;
constexpr unsigned kSpinLimit = 1u << 22;

struct QrLayout {
    int P;   // workgroups
    int rb;  // rows per workgroup
    size_t lds_bytes;
};

size_t lds_for(int rb, int n) {
    // row block + v (rb) + w (n) + row j (n) + row-group partials + scalars
    return sizeof(double) * ((size_t)rb * n + rb + 2 * (size_t)n + (size_t)kRowGroups * (n + 1) + 8);
}

// Grid-wide barrier of a cooperative launch.  After a workgroup barrier, one
// thread per workgroup arrives on a counter with release semantics (one L2
// write-back for the whole workgroup), polls it with relaxed loads, and
// issues a single acquire fence once target arrivals are seen.  The wait is
// bounded: on timeout *err is set and the kernel runs to its end (the result is
// then discarded by the host).
__device__ void grid_barrier(unsigned* cnt, unsigned target, int* err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit) {
                atomicOr(err, 2);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Apply H_{jc-1} = I - t v w^T to the local rows below jc-1 (t == 0: no
// update) and write the partial sums of column jc over the local rows strictly
// below jc: slot 0 = sum x_i^2, slot s = sum x_i a_i,jc+s.  Column jc is updated
// first (its new values are the next reflector's x); the other columns are
// updated and accumulated in the same pass (64 column lanes x row groups).
__device__ void update_and_partials(double* Ab, int nr, int r0, int n, int jc, double t,
                                    const double* vloc, const double* wv, double* red,
                                    double* out) {
    const int tid = threadIdx.x, cl = tid % kColGroup, rg = tid / kColGroup;
    const int iupd = max(0, jc - r0);  // first local row with global index > jc - 1
    if (t != 0.0) {
        const double wj = wv[jc];
        for (int i = iupd + tid; i < nr; i += kQrThreads) Ab[i * n + jc] -= t * vloc[i] * wj;
    }
    __syncthreads();
    const int nsl = n - jc;
    const int ncl = (nsl + kColGroup - 1) / kColGroup;
    double acc[kMaxColsPerLane];
#pragma unroll
    for (int c = 0; c < kMaxColsPerLane; ++c) acc[c] = 0.0;
    for (int i = iupd + rg; i < nr; i += kRowGroups) {
        double* row = Ab + i * n;
        const double x = (r0 + i > jc) ? row[jc] : 0.0;
        const double tv = t * vloc[i];
#pragma unroll
        for (int c = 0; c < kMaxColsPerLane; ++c) {
            const int s = cl + kColGroup * c;
            if (c < ncl && s < nsl) {
                double a = row[jc + s];
                if (s > 0 && t != 0.0) {
                    a -= tv * wv[jc + s];
                    row[jc + s] = a;
                }
                acc[c] += x * a;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kMaxColsPerLane; ++c) {
        const int s = cl + kColGroup * c;
        if (c < ncl && s < nsl) red[rg * (n + 1) + s] = acc[c];
    }
    __syncthreads();
    for (int s = tid; s < nsl; s += kQrThreads) {
        double a = 0.0;
        for (int g = 0; g < kRowGroups; ++g) a += red[g * (n + 1) + s];
        out[s] = a;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kQrThreads) void qr_factor_kernel(const double* __restrict__ M, int m,
                                                               int n, int rb, double* V, double* R,
                                                               double* tau, double* part,
                                                               double* rowbuf, unsigned* cnt,
                                                               int* err) {
    extern __shared__ double lds[];
    const int P = gridDim.x, p = blockIdx.x, tid = threadIdx.x;
    const int r0 = p * rb;
    const int nr = max(0, min(rb, m - r0));
    double* Ab = lds;
    double* vloc = Ab + (size_t)rb * n;
    double* wv = vloc + rb;
    double* rowj = wv + n;
    double* red = rowj + n;
    double* sc = red + kRowGroups * (n + 1);
    const size_t pstride = (size_t)P * (n + 1);

    for (int e = tid; e < nr * n; e += kQrThreads) Ab[e] = M[(size_t)r0 * n + e];
    __syncthreads();

    // column 0 partials and row 0
    update_and_partials(Ab, nr, r0, n, 0, 0.0, vloc, wv, red, part + (size_t)p * (n + 1));
    if (r0 <= 0 && 0 < r0 + nr)
        for (int k = tid; k < n; k += kQrThreads) rowbuf[k] = Ab[k];

    for (int j = 0; j < n; ++j) {
        grid_barrier(cnt, (unsigned)(j + 1) * (unsigned)P, err);
        const double* pp = part + (size_t)(j & 1) * pstride;
        const double* row = rowbuf + (size_t)(j & 1) * n;
        const int nslots = n - j;
        // combine partials in a fixed order: 64 slot lanes x 8 workgroup groups,
        // four independent running sums, then the groups through LDS
        {
            const int sl = tid % kColGroup, qg = tid / kColGroup;
            for (int s0 = 0; s0 < nslots; s0 += kColGroup) {
                const int sidx = s0 + sl;
                if (sidx < nslots) {
                    const double* col = pp + sidx;
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                    int q = qg;
                    for (; q + 3 * kRowGroups < P; q += 4 * kRowGroups) {
                        a0 += col[(size_t)q * (n + 1)];
                        a1 += col[(size_t)(q + kRowGroups) * (n + 1)];
                        a2 += col[(size_t)(q + 2 * kRowGroups) * (n + 1)];
                        a3 += col[(size_t)(q + 3 * kRowGroups) * (n + 1)];
                    }
                    for (; q < P; q += kRowGroups) a0 += col[(size_t)q * (n + 1)];
                    red[qg * (n + 1) + sidx] = (a0 + a1) + (a2 + a3);
                }
            }
            for (int k = j + tid; k < n; k += kQrThreads) rowj[k] = row[k];
            __syncthreads();
            for (int sidx = tid; sidx < nslots; sidx += kQrThreads) {
                double a = 0.0;
                for (int g = 0; g < kRowGroups; ++g) a += red[g * (n + 1) + sidx];
                wv[j + sidx] = a;  // wv[j] = sigma^2, wv[k] = x^T a_k over rows > j
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double alpha = rowj[j];
            const double sigma2 = wv[j];
            double beta, t, gamma;
            int mode;  // 0: H = I, 1: sign flip e_j, 2: general reflector
            if (sigma2 == 0.0) {
                if (alpha >= 0.0) { mode = 0; beta = alpha; t = 0.0; gamma = 1.0; }
                else { mode = 1; beta = -alpha; t = 2.0; gamma = 1.0; }
            } else {
                mode = 2;
                beta = sqrt(alpha * alpha + sigma2);
                gamma = alpha <= 0.0 ? alpha - beta : -sigma2 / (alpha + beta);
                t = -gamma / beta;
            }
            sc[0] = beta; sc[1] = t; sc[2] = gamma; sc[3] = (double)mode;
        }
        __syncthreads();
        const double beta = sc[0], t = sc[1], gamma = sc[2];
        const int mode = (int)sc[3];
        // w_k = v^T a_k over rows >= j (v_j = 1)
        for (int k = j + 1 + tid; k < n; k += kQrThreads)
            wv[k] = (mode == 2) ? wv[k] / gamma + rowj[k] : rowj[k];
        // v for the local rows
        for (int i = tid; i < nr; i += kQrThreads) {
            const int gi = r0 + i;
            double v;
            if (gi < j) v = 0.0;
            else if (gi == j) v = 1.0;
            else v = (mode == 2) ? Ab[i * n + j] / gamma : 0.0;
            vloc[i] = v;
            V[(size_t)gi * n + j] = v;
        }
        __syncthreads();
        if (p == 0) {
            for (int k = tid; k < n; k += kQrThreads) {
                double r;
                if (k < j) r = 0.0;
                else if (k == j) r = beta;
                else r = rowj[k] - t * wv[k];
                R[(size_t)j * n + k] = r;
            }
            if (tid == 0) tau[j] = t;
        }
        if (j + 1 < n) {
            update_and_partials(Ab, nr, r0, n, j + 1, t, vloc, wv, red,
                                part + (size_t)((j + 1) & 1) * pstride + (size_t)p * (n + 1));
            // publish row j+1 (final in columns > j)
            if (r0 <= j + 1 && j + 1 < r0 + nr) {
                double* nrow = rowbuf + (size_t)((j + 1) & 1) * n;
                for (int k = tid; k < n; k += kQrThreads) nrow[k] = Ab[(j + 1 - r0) * n + k];
            }
        }
    }
}

__global__ void zero_counter_kernel(unsigned* cnt) {
    if (threadIdx.x == 0) *cnt = 0u;
}

// T[i][j] (i <= j): T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j,0:j] G[0:j, j]
// (the forward compact-WY recurrence), in column blocks of kTb: the part of the
// triangular product over columns left of the block is one parallel pass over
// the whole block (partial results in LDS); the in-block part is sequential
// over the kTb columns.  Also min|R_ii| / max|R_ii| into diag_ratio.
constexpr int kTb = 16;
constexpr int kTMaxN = 512;

__global__ __launch_bounds__(1024) void qr_tfactor_kernel(const double* __restrict__ G,
                                                          const double* __restrict__ tau, int n,
                                                          double* T, const double* R,
                                                          double* diag_ratio) {
    __shared__ double W1[kTMaxN * kTb];  // W1[i*kTb + c] = sum_{l<b0} T[i][l] G[l][b0+c]
    __shared__ double Tb[kTMaxN * kTb];  // current block's columns of T: Tb[i*kTb + c]
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) T[e] = 0.0;
    __syncthreads();
    for (int b0 = 0; b0 < n; b0 += kTb) {
        const int nb = min(kTb, n - b0);
        for (int e = tid; e < b0 * nb; e += blockDim.x) {
            const int i = e / nb, c = e % nb;
            double acc = 0.0;
            for (int l = i; l < b0; ++l) acc += T[(size_t)i * n + l] * G[(size_t)l * n + b0 + c];
            W1[i * kTb + c] = acc;
        }
        for (int e = tid; e < (b0 + nb) * kTb; e += blockDim.x) Tb[e] = 0.0;
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            const int jj = b0 + c;
            const double tj = tau[jj];
            double val = 0.0;
            const int i = tid;
            if (i < jj) {
                double acc = i < b0 ? W1[i * kTb + c] : 0.0;
                for (int l = max(i, b0); l < jj; ++l) acc += Tb[i * kTb + (l - b0)] * G[(size_t)l * n + jj];
                val = -tj * acc;
            }
            __syncthreads();
            if (i < jj) Tb[i * kTb + c] = val;
            if (i == jj) Tb[i * kTb + c] = tj;
            __syncthreads();
        }
        for (int e = tid; e < (b0 + nb) * nb; e += blockDim.x) {
            const int i = e / nb, c = e % nb;
            T[(size_t)i * n + b0 + c] = Tb[i * kTb + c];
        }
        __syncthreads();
    }
    if (tid == 0 && diag_ratio != nullptr) {
        double mn = INFINITY, mx = 0.0;
        for (int k = 0; k < n; ++k) {
            const double d = fabs(R[(size_t)k * n + k]);
            mn = fmin(mn, d);
            mx = fmax(mx, d);
        }
        *diag_ratio = mx > 0.0 ? mn / mx : 0.0;
    }
}

__global__ void eye_kernel(double* Q, long long m, int n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m * n;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, c = e % n;
        Q[e] = (i == c) ? 1.0 : 0.0;
    }
}

QrLayout plan_qr(int m, int n) {
    QrLayout L{};
    // fewest workgroups whose row blocks fit in LDS: fewer partial sums to
    // combine and a cheaper grid barrier
    const size_t fixed = lds_for(0, n);
    const size_t per_row = sizeof(double) * (size_t)(n + 1);
    long long rb_max = fixed < kQrLdsBudget ? (long long)((kQrLdsBudget - fixed) / per_row) : 0;
    if (rb_max < 1) rb_max = 1;
    long long P = ceil_div(m, rb_max);
    if (P < 1) P = 1;
    L.rb = (int)ceil_div(m, P);
    L.P = (int)ceil_div(m, L.rb);
    L.lds_bytes = lds_for(L.rb, n);
    return L;
}

}  // namespace

QrScratch qr_scratch_layout(int m, int n) {
    QrScratch s{};
    const QrLayout L = plan_qr(m, n);
    size_t off = 0;
    auto take = [&](size_t count) {
        const size_t o = off;
        off += ((count * sizeof(double) + 255) / 256) * 256;
        return o;
    };
    s.off_V = take((size_t)m * n);
    s.off_tau = take(n);
    s.off_part = take(2 * (size_t)L.P * (n + 1));
    s.off_rowbuf = take(2 * (size_t)n);
    s.off_G = take((size_t)n * n);
    s.off_T = take((size_t)n * n);
    s.off_MT = take((size_t)n * n);
    s.off_ratio = take(1);
    s.off_cnt = take(1);
    s.off_err = take(1);
    GemmDesc gg;
    gg.M = n; gg.N = n; gg.K = m;
    const size_t sk = gemm_splitk_bytes(gg);
    s.off_splitk = take(sk / sizeof(double) + 1);
    s.splitk_bytes = sk;
    s.total = off;
    return s;
}

bool qr_fits(int m, int n) {
    if (m < n || n < 1 || n > kTMaxN) return false;
    const QrLayout L = plan_qr(m, n);
    return L.lds_bytes <= kQrLdsBudget && L.P <= 256;
}

Status qr_pos(const double* M, double* Q, double* R, int m, int n, void* ws, size_t ws_bytes,
              hipStream_t st, double* diag_ratio_dev, int* err_dev) {
    Status s;
    if (!qr_fits(m, n)) {
        s.code = -1;
        s.msg = "qr: shape not supported (need m >= n, n <= 512, at most 256 row blocks in LDS)";
        return s;
    }
    const QrScratch L = qr_scratch_layout(m, n);
    if (ws_bytes < L.total) {
        s.code = -2;
        s.msg = "qr: workspace too small";
        return s;
    }
    char* base = static_cast<char*>(ws);
    double* V = reinterpret_cast<double*>(base + L.off_V);
    double* tau = reinterpret_cast<double*>(base + L.off_tau);
    double* part = reinterpret_cast<double*>(base + L.off_part);
    double* rowbuf = reinterpret_cast<double*>(base + L.off_rowbuf);
    double* G = reinterpret_cast<double*>(base + L.off_G);
    double* T = reinterpret_cast<double*>(base + L.off_T);
    double* MT = reinterpret_cast<double*>(base + L.off_MT);
    double* ratio = diag_ratio_dev ? diag_ratio_dev : reinterpret_cast<double*>(base + L.off_ratio);
    void* sk = base + L.off_splitk;

    const QrLayout ql = plan_qr(m, n);
    unsigned* cnt = reinterpret_cast<unsigned*>(base + L.off_cnt);
    int* err = err_dev ? err_dev : reinterpret_cast<int*>(base + L.off_err);
    {
        int dev = 0;
        QRCTM_HIP(hipGetDevice(&dev));
        QRCTM_HIP(hipFuncSetAttribute((const void*)qr_factor_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)ql.lds_bytes));
        int nblk = 0;
        QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, qr_factor_kernel, kQrThreads,
                                                               ql.lds_bytes));
        int ncu = 0;
        QRCTM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if ((long long)nblk * ncu < ql.P) {
            s.code = -1;
            s.msg = "qr: cooperative grid does not fit on the device";
            return s;
        }
        hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, st, cnt);
        QRCTM_TRY(launch_check("zero_counter_kernel"));
        const double* Mp = M;
        int mm = m, nn = n, rbb = ql.rb;
        void* args[] = {(void*)&Mp,  (void*)&mm,   (void*)&nn,     (void*)&rbb,
                        (void*)&V,   (void*)&R,    (void*)&tau,    (void*)&part,
                        (void*)&rowbuf, (void*)&cnt, (void*)&err};
        QRCTM_HIP(hipLaunchCooperativeKernel((const void*)qr_factor_kernel, dim3(ql.P),
                                             dim3(kQrThreads), args, ql.lds_bytes, st));
    }
    // G = V^T V
    {
        GemmDesc g;
        g.trans_a = 1; g.trans_b = 0;
        g.M = n; g.N = n; g.K = m;
        g.A = V; g.lda = n; g.B = V; g.ldb = n;
        g.C = G; g.map = OutMap::plain(n, n, n);
        QRCTM_TRY(gemm_f64(g, sk, L.splitk_bytes, st));
    }
    hipLaunchKernelGGL(qr_tfactor_kernel, dim3(1), dim3(1024), 0, st, G, tau, n, T, R, ratio);
    QRCTM_TRY(launch_check("qr_tfactor_kernel"));
    // MT = T V1^T
    {
        GemmDesc g;
        g.trans_a = 0; g.trans_b = 1;
        g.M = n; g.N = n; g.K = n;
        g.A = T; g.lda = n; g.B = V; g.ldb = n;
        g.C = MT; g.map = OutMap::plain(n, n, n);
        QRCTM_TRY(gemm_f64(g, sk, L.splitk_bytes, st));
    }
    {
        const long long tot = (long long)m * n;
        const int blocks = (int)std::min<long long>(ceil_div(tot, 256), 4096);
        hipLaunchKernelGGL(eye_kernel, dim3(blocks), dim3(256), 0, st, Q, (long long)m, n);
        QRCTM_TRY(launch_check("eye_kernel"));
    }
    // Q = E - V MT
    {
        GemmDesc g;
        g.trans_a = 0; g.trans_b = 0;
        g.M = m; g.N = n; g.K = n;
        g.A = V; g.lda = n; g.B = MT; g.ldb = n;
        g.C = Q; g.map = OutMap::plain(m, n, n);
        g.alpha = -1.0; g.beta = 1.0;
        QRCTM_TRY(gemm_f64(g, sk, L.splitk_bytes, st));
    }
    return s;
}

}  // namespace qrctm
