// Elementwise / reduction kernels of the CTMRG path (gfx950):
//   a1  C4v average of the site tensor and scaling to max|A| = 1,
//   a2  double layer a = sum_s A (x) A, stored as a[U][L][R][Dn],
//   a3  initial C, T from the bulk tensor and a boundary vector,
//   a9  symmetrise C', T' and divide by their Frobenius norms (FP64).
#include "common.h"
#include "tensor_ops.h"

namespace qrctm {
namespace {

// The 8 elements of C4v acting on the virtual-leg positions (u,l,d,r) = (0..3):
// rotations i -> i + k and reflections i -> k - i (mod 4).
__device__ __forceinline__ int c4v_pos(int g, int i) {
    const int k = g >> 1;
    return (g & 1) ? ((k - i) & 3) : ((i + k) & 3);
}

__global__ __launch_bounds__(1024) void c4v_prepare_kernel(const double* __restrict__ A, int d,
                                                           int D, double* As, double* scale_out,
                                                           int* bad, int* imax_out) {
    __shared__ double red[1024];
    __shared__ int redi[1024];
    const int n = d * D * D * D * D;
    const int D4 = D * D * D * D;
    double mx = -1.0;
    int mi = 0;
    int nonfinite = 0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int s = e / D4;
        int rem = e % D4;
        int idx[4];
        for (int q = 3; q >= 0; --q) { idx[q] = rem % D; rem /= D; }
        double acc = 0.0;
        for (int g = 0; g < 8; ++g) {
            int src[4];
            for (int q = 0; q < 4; ++q) src[q] = idx[c4v_pos(g, q)];
            acc += A[(size_t)s * D4 + ((src[0] * D + src[1]) * D + src[2]) * D + src[3]];
        }
        acc *= 0.125;
        As[e] = acc;
        if (!isfinite(acc)) nonfinite = 1;
        if (fabs(acc) > mx) { mx = fabs(acc); mi = e; }  // first maximiser of this thread
    }
    red[threadIdx.x] = mx;
    redi[threadIdx.x] = mi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            const int oi = redi[threadIdx.x + w];
            if (o > red[threadIdx.x] || (o == red[threadIdx.x] && oi < redi[threadIdx.x])) {
                red[threadIdx.x] = o;
                redi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const double m = red[0];
    if (threadIdx.x == 0 && imax_out) *imax_out = redi[0];
    if (nonfinite) atomicOr(bad, 1);
    if (m == 0.0 || !isfinite(m)) {
        if (threadIdx.x == 0) atomicOr(bad, 1);
        return;
    }
    const double inv = 1.0 / m;
    for (int e = threadIdx.x; e < n; e += blockDim.x) As[e] *= inv;
    if (threadIdx.x == 0 && scale_out) *scale_out = m;
}

// a_int[U][L][R][Dn] with U = u*D + u' (ket major)
__global__ void double_layer_kernel(const double* __restrict__ As, int d, int D, double* a) {
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
        const int u = U / D, u2 = U % D, l = L / D, l2 = L % D;
        const int r = R / D, r2 = R % D, dd = Dn / D, d2 = Dn % D;
        const int ik = ((u * D + l) * D + dd) * D + r;
        const int ib = ((u2 * D + l2) * D + d2) * D + r2;
        double acc = 0.0;
        for (int s = 0; s < d; ++s) acc += As[(size_t)s * D4 + ik] * As[(size_t)s * D4 + ib];
        a[e] = acc;
    }
}

// user layout a[U][L][Dn][R] -> internal a_int[U][L][R][Dn]
__global__ void dl_to_internal_kernel(const double* __restrict__ a, int Dab, double* out) {
    const long long n = (long long)Dab * Dab * Dab * Dab;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        long long rem = e;
        const int Dn = (int)(rem % Dab); rem /= Dab;
        const int R = (int)(rem % Dab); rem /= Dab;
        const long long UL = rem;
        out[e] = a[(UL * Dab + Dn) * Dab + R];
    }
}

// C0[x,y] = sum_{U,L} b[U] b[L] a[U,L,Dn=y,R=x];  T0[x,m,y] = sum_L b[L] a[U=x,L,Dn=y,R=m]
__global__ void init_env_kernel(const double* __restrict__ aint, const double* __restrict__ b,
                                int Dab, double* C, double* T) {
    const long long D = Dab;
    const long long nC = D * D, nT = D * D * D;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nC) {
            const long long x = e / D, y = e % D;
            double acc = 0.0;
            for (long long U = 0; U < D; ++U)
                for (long long L = 0; L < D; ++L)
                    acc += b[U] * b[L] * aint[((U * D + L) * D + x) * D + y];
            C[e] = acc;
        } else {
            const long long f = e - nC;
            const long long x = f / (D * D), m = (f / D) % D, y = f % D;
            double acc = 0.0;
            for (long long L = 0; L < D; ++L) acc += b[L] * aint[((x * D + L) * D + m) * D + y];
            T[f] = acc;
        }
    }
}

// identity boundary vector vec(I_D) on a paired leg
__global__ void eye_vec_kernel(double* b, int D) {
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) b[e] = (e / D == e % D) ? 1.0 : 0.0;
}

constexpr int kNormThreads = 256;
constexpr int kNormBlocks = 512;

// pass 1: symmetrised C, T into Cn, Tn plus per-block partial sums of squares
__global__ __launch_bounds__(kNormThreads) void symmetrize_kernel(const double* __restrict__ Cp,
                                                                  const double* __restrict__ Tp,
                                                                  int chi, int Dab, double* Cn,
                                                                  double* Tn, double* part) {
    __shared__ double rc[kNormThreads], rt[kNormThreads];
    const long long nC = (long long)chi * chi, nT = nC * Dab;
    double sc = 0.0, st = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nC) {
            const long long x = e / chi, y = e % chi;
            const double v = 0.5 * (Cp[e] + Cp[y * chi + x]);
            Cn[e] = v;
            sc += v * v;
        } else {
            const long long f = e - nC;
            const long long x = f / ((long long)Dab * chi), m = (f / chi) % Dab, y = f % chi;
            const double v = 0.5 * (Tp[f] + Tp[(y * Dab + m) * chi + x]);
            Tn[f] = v;
            st += v * v;
        }
    }
    rc[threadIdx.x] = sc;
    rt[threadIdx.x] = st;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
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

// pass 2: every block combines the partials (fixed order) and scales its share
__global__ __launch_bounds__(kNormThreads) void normalize_kernel(const double* __restrict__ part,
                                                                 int nparts, int chi, int Dab,
                                                                 double* Cn, double* Tn,
                                                                 double* norms, int* bad) {
    __shared__ double s[2];
    __shared__ double ra[kNormThreads], rb[kNormThreads];
    {
        double a = 0.0, b = 0.0;
        for (int q = threadIdx.x; q < nparts; q += kNormThreads) {
            a += part[2 * q];
            b += part[2 * q + 1];
        }
        ra[threadIdx.x] = a;
        rb[threadIdx.x] = b;
        __syncthreads();
        for (int w = kNormThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ra[threadIdx.x] += ra[threadIdx.x + w];
                rb[threadIdx.x] += rb[threadIdx.x + w];
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        s[0] = sqrt(ra[0]);
        s[1] = sqrt(rb[0]);
        if (blockIdx.x == 0 && norms) {
            norms[0] = s[0];
            norms[1] = s[1];
        }
        if (!(isfinite(s[0]) && isfinite(s[1]) && s[0] > 0.0 && s[1] > 0.0) && blockIdx.x == 0)
            atomicOr(bad, 1);
    }
    __syncthreads();
    const double ic = 1.0 / s[0], it = 1.0 / s[1];
    const long long nC = (long long)chi * chi, nT = nC * Dab;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nC + nT;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nC) Cn[e] *= ic;
        else Tn[e - nC] *= it;
    }
}

int grid_for(long long n, int threads, int cap) {
    long long b = ceil_div(n, threads);
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

Status c4v_prepare(const double* A, int d, int D, double* As, double* scale_out, int* bad,
                   int* imax_out, hipStream_t st) {
    hipLaunchKernelGGL(c4v_prepare_kernel, dim3(1), dim3(1024), 0, st, A, d, D, As, scale_out, bad,
                       imax_out);
    return launch_check("c4v_prepare_kernel");
}

Status double_layer(const double* As, int d, int D, double* a, hipStream_t st) {
    const long long D2 = (long long)D * D;
    const long long n = D2 * D2 * D2 * D2;
    hipLaunchKernelGGL(double_layer_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, st, As, d,
                       D, a);
    return launch_check("double_layer_kernel");
}

Status dl_to_internal(const double* a, int Dab, double* out, hipStream_t st) {
    const long long n = (long long)Dab * Dab * Dab * Dab;
    hipLaunchKernelGGL(dl_to_internal_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, st, a,
                       Dab, out);
    return launch_check("dl_to_internal_kernel");
}

Status eye_vec(double* b, int D, hipStream_t st) {
    hipLaunchKernelGGL(eye_vec_kernel, dim3(1), dim3(256), 0, st, b, D);
    return launch_check("eye_vec_kernel");
}

Status init_env(const double* aint, const double* b, int Dab, double* C, double* T,
                hipStream_t st) {
    const long long n = (long long)Dab * Dab * (1 + Dab);
    hipLaunchKernelGGL(init_env_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, aint, b,
                       Dab, C, T);
    return launch_check("init_env_kernel");
}

size_t sym_norm_scratch_bytes() { return sizeof(double) * 2 * kNormBlocks; }

Status sym_norm(const double* Cp, const double* Tp, int chi, int Dab, double* Cn, double* Tn,
                double* part, double* norms, int* bad, hipStream_t st) {
    const long long n = (long long)chi * chi * (1 + Dab);
    const int blocks = grid_for(n, kNormThreads, kNormBlocks);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks), dim3(kNormThreads), 0, st, Cp, Tp, chi, Dab,
                       Cn, Tn, part);
    QRCTM_TRY(launch_check("symmetrize_kernel"));
    hipLaunchKernelGGL(normalize_kernel, dim3(blocks), dim3(kNormThreads), 0, st, part, blocks, chi,
                       Dab, Cn, Tn, norms, bad);
    return launch_check("normalize_kernel");
}

}  // namespace qrctm
