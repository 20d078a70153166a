// Symmetric eigensolver for the warm-up steps of standard CTMRG: the enlarged
// corner is diagonalised and the chi eigenvectors of largest |lambda| form the
// isometry U (standard-CTMRG paragraph, Fig. 1d).  The warm-up runs 1-4 times
// per tensor (QR-CTMRG paragraph), so this solver is set-up cost, not the loop.
//
// Method: two-sided cyclic Jacobi with the parallel round-robin ordering
// (n/2 disjoint rotations per round, n-1 rounds per sweep), all on the GPU:
//   jacobi_params_kernel  one thread per pair: rotation (c, s) that zeroes
//                         A[p][q] (Golub & Van Loan's symmetric Schur 2x2),
//                         skipped when |A_pq| <= eps sqrt(|A_pp A_qq|);
//   jacobi_apply_kernel   A <- J^T A J on 2x2 blocks (one thread per pair of
//                         pairs, in place, disjoint) and V <- V J.
// A sweep without any rotation ends the iteration (host reads one counter per
// sweep).  Then the kept eigenpairs are ranked by |lambda| (descending; ties by
// lambda ascending, then index), sign-fixed (first component with
// |v_i| >= max|v|/2 positive) and written out as U (n x k, row-major) and
// diag(lambda).
#include "common.h"
#include "eigh.h"

namespace qrctm {
namespace {

struct Rot {
    int p, q;
    double c, s;
};

__device__ __forceinline__ void rr_pair(int r, int i, int np, int* a, int* b) {
    const int m = np - 1;
    *a = (r + i) % m;
    *b = (i == 0) ? m : (r - i + m) % m;
}

__global__ void jacobi_params_kernel(const double* __restrict__ A, int n, int np, int r, Rot* rot,
                                     int* count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np / 2) return;
    int a, b;
    rr_pair(r, i, np, &a, &b);
    const int p = min(a, b), q = max(a, b);
    Rot o{p, q, 1.0, 0.0};
    if (q < n) {
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double apq = A[(size_t)p * n + q];
        if (apq != 0.0 && fabs(apq) > 2.2e-16 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            o.c = 1.0 / sqrt(1.0 + t * t);
            o.s = t * o.c;
            atomicAdd(count, 1);
        }
    }
    rot[i] = o;
}

// blocks [0, nb_a): A update, thread per (pair ia, pair ib); then V update,
// thread per (row, pair).
__global__ void jacobi_apply_kernel(double* A, double* V, int n, int np, const Rot* __restrict__ rot,
                                    long long nA) {
    const int half = np / 2;
    const long long nV = (long long)n * half;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nA + nV;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nA) {
            const int ia = (int)(e / half), ib = (int)(e % half);
            const Rot ra = rot[ia], rb = rot[ib];
            if (ra.s == 0.0 && rb.s == 0.0) continue;
            const bool qa = ra.q < n, qb = rb.q < n;
            const int pa = ra.p, pb = rb.p;
            const int qa_ = ra.q, qb_ = rb.q;
            double x00 = A[(size_t)pa * n + pb];
            double x01 = qb ? A[(size_t)pa * n + qb_] : 0.0;
            double x10 = qa ? A[(size_t)qa_ * n + pb] : 0.0;
            double x11 = (qa && qb) ? A[(size_t)qa_ * n + qb_] : 0.0;
            // columns (pair b)
            double y00 = rb.c * x00 - rb.s * x01, y01 = rb.s * x00 + rb.c * x01;
            double y10 = rb.c * x10 - rb.s * x11, y11 = rb.s * x10 + rb.c * x11;
            // rows (pair a)
            double z00 = ra.c * y00 - ra.s * y10, z10 = ra.s * y00 + ra.c * y10;
            double z01 = ra.c * y01 - ra.s * y11, z11 = ra.s * y01 + ra.c * y11;
            if (ia == ib && ra.s != 0.0) { z01 = 0.0; z10 = 0.0; }
            A[(size_t)pa * n + pb] = z00;
            if (qb) A[(size_t)pa * n + qb_] = z01;
            if (qa) A[(size_t)qa_ * n + pb] = z10;
            if (qa && qb) A[(size_t)qa_ * n + qb_] = z11;
        } else {
            const long long f = e - nA;
            const int row = (int)(f / half), ib = (int)(f % half);
            const Rot rb = rot[ib];
            if (rb.s == 0.0 || rb.q >= n) continue;
            const double vp = V[(size_t)row * n + rb.p], vq = V[(size_t)row * n + rb.q];
            V[(size_t)row * n + rb.p] = rb.c * vp - rb.s * vq;
            V[(size_t)row * n + rb.q] = rb.s * vp + rb.c * vq;
        }
    }
}

__global__ void sym_copy_eye_kernel(const double* __restrict__ Z, int n, double* A, double* V) {
    const long long nn = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, j = e % n;
        A[e] = 0.5 * (Z[e] + Z[j * n + i]);
        V[e] = (i == j) ? 1.0 : 0.0;
    }
}

__global__ void zero_int_kernel(int* x) { *x = 0; }

// rank of each eigenvalue: |lambda| descending, lambda ascending, index ascending
__global__ void rank_kernel(const double* __restrict__ A, int n, int* order_of_rank, double* lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double li = A[(size_t)i * n + i], ai = fabs(li);
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const double lj = A[(size_t)j * n + j], aj = fabs(lj);
        rank += (aj > ai) || (aj == ai && (lj < li || (lj == li && j < i)));
    }
    order_of_rank[rank] = i;
    lam[rank] = li;
}

// U[:, j] = sign * V[:, order[j]] for j < k; Cd = diag(lam[0:k])
__global__ void select_kernel(const double* __restrict__ V, int n, int k,
                              const int* __restrict__ order, const double* __restrict__ lam,
                              double* U, double* Cd) {
    const int j = blockIdx.x;
    if (j >= k) return;
    const int col = order[j];
    __shared__ double bv[256];
    __shared__ int bi[256];
    double best = -1.0;
    int bidx = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double a = fabs(V[(size_t)i * n + col]);
        if (a > best) { best = a; bidx = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = bv[threadIdx.x + w];
            const int oi = bi[threadIdx.x + w];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    // sign: the first component with |v_i| >= max|v| / 2 is made positive
    const double half = 0.5 * bv[0];
    __syncthreads();
    int first = n;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (fabs(V[(size_t)i * n + col]) >= half) { first = i; break; }
    bi[threadIdx.x] = first;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) bi[threadIdx.x] = min(bi[threadIdx.x], bi[threadIdx.x + w]);
        __syncthreads();
    }
    const double sg = V[(size_t)bi[0] * n + col] < 0.0 ? -1.0 : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) U[(size_t)i * k + j] = sg * V[(size_t)i * n + col];
    for (int i = threadIdx.x; i < k; i += blockDim.x) Cd[(size_t)j * k + i] = (i == j) ? lam[j] : 0.0;
}

struct EigLayout {
    size_t A, V, rot, order, lam, count, total;
};

EigLayout eig_layout(int n) {
    EigLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const int np = n + (n & 1);
    L.A = take(sizeof(double) * (size_t)n * n);
    L.V = take(sizeof(double) * (size_t)n * n);
    L.rot = take(sizeof(Rot) * (size_t)(np / 2));
    L.order = take(sizeof(int) * (size_t)n);
    L.lam = take(sizeof(double) * (size_t)n);
    L.count = take(sizeof(int) * 4);
    L.total = off;
    return L;
}

}  // namespace

size_t eigh_scratch_bytes(int n) { return eig_layout(n).total; }

Status eigh_select(const double* Z, int n, int k, double* U, double* Cd, void* ws, size_t ws_bytes,
                   hipStream_t st) {
    Status s;
    const EigLayout L = eig_layout(n);
    if (k < 1 || k > n) {
        s.code = -1;
        s.msg = "eigh: need 1 <= k <= n";
        return s;
    }
    if (ws_bytes < L.total) {
        s.code = -2;
        s.msg = "eigh: workspace too small";
        return s;
    }
    char* base = static_cast<char*>(ws);
    double* A = reinterpret_cast<double*>(base + L.A);
    double* V = reinterpret_cast<double*>(base + L.V);
    Rot* rot = reinterpret_cast<Rot*>(base + L.rot);
    int* order = reinterpret_cast<int*>(base + L.order);
    double* lam = reinterpret_cast<double*>(base + L.lam);
    int* count = reinterpret_cast<int*>(base + L.count);
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(sym_copy_eye_kernel, dim3((int)std::min<long long>(ceil_div(nn, 256), 8192)),
                       dim3(256), 0, st, Z, n, A, V);
    QRCTM_TRY(launch_check("sym_copy_eye_kernel"));
    if (n > 1) {
        const int np = n + (n & 1);
        const int half = np / 2;
        const long long nA = (long long)half * half;
        const long long work = nA + (long long)n * half;
        const int ablocks = (int)std::min<long long>(ceil_div(work, 256), 16384);
        const int pblocks = (int)ceil_div(half, 256);
        bool done = false;
        for (int sweep = 0; sweep < 60 && !done; ++sweep) {
            hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, count);
            for (int r = 0; r < np - 1; ++r) {
                hipLaunchKernelGGL(jacobi_params_kernel, dim3(pblocks), dim3(256), 0, st, A, n, np, r,
                                   rot, count);
                hipLaunchKernelGGL(jacobi_apply_kernel, dim3(ablocks), dim3(256), 0, st, A, V, n, np,
                                   rot, nA);
            }
            QRCTM_TRY(launch_check("jacobi sweep"));
            int h = 1;
            QRCTM_HIP(hipMemcpyAsync(&h, count, sizeof(int), hipMemcpyDeviceToHost, st));
            QRCTM_HIP(hipStreamSynchronize(st));
            done = (h == 0);
        }
        if (!done) {
            s.code = -3;
            s.msg = "eigh: Jacobi did not converge in 60 sweeps";
            return s;
        }
    }
    hipLaunchKernelGGL(rank_kernel, dim3((int)ceil_div(n, 256)), dim3(256), 0, st, A, n, order, lam);
    QRCTM_TRY(launch_check("rank_kernel"));
    hipLaunchKernelGGL(select_kernel, dim3(k), dim3(256), 0, st, V, n, k, order, lam, U, Cd);
    return launch_check("select_kernel");
}

}  // namespace qrctm
