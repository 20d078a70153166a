// Cholesky-QR2 of the reduced corner, with the Householder kernel as fallback.
//
// The QR-CTMRG paragraph factors the reduced corner c~ (m x n, m = chi Dab,
// n = chi) by an unpivoted QR.  On the benchmark tensors c~ is well
// conditioned (kappa ~ 1e1-1e3: its columns span D^2 copies of the corner's
// leading subspace), so the factorisation can be formed from the n x n Gram
// matrix instead of n dependent column reflections:
//
//   pass 1:  G1 = M^T M,   G1 = R1^T R1 (Cholesky),   Q1 = M R1^{-1}
//   pass 2:  G2 = Q1^T Q1, G2 = R2^T R2,              Q  = Q1 R2^{-1},  R = R2 R1
//
// (Cholesky-QR2, Yamamoto, Nakatsukasa, Yanagisawa and Fukaya 2015: the second
// pass restores orthogonality to rounding level for kappa(M) up to about
// u^{-1/2}).  diag(R) > 0 by construction, so Q and R are the unique thin QR
// factors with a positive diagonal, the same ones the Householder kernel
// computes (up to rounding).
//
// Every pass is three kernels, none of them cooperative:
//  * gram_kernel: 32 x 32 tiles of the upper block triangle of X^T X, each
//    split over S row ranges (FP64 matrix cores); the workgroup that takes a
//    tile's last ticket adds the S partial tiles in a fixed order (the sum is
//    deterministic) and writes the tile and its mirror;
//  * chol_kernel: one workgroup, right-looking blocked Cholesky with 16 x 16
//    blocks (kept in LDS for n <= 176, in global memory beyond).  Wave 0
//    factors a diagonal block in registers, eliminating on [B | I] so that it
//    also yields W = R_KK^{-T}; all waves then form the block row
//    W B_KJ and the trailing update B_IJ -= B_KI^T B_KJ on the matrix cores;
//  * trsm_kernel: X = M R^{-1}, one wave per 16 rows, block column by block
//    column (X_K = (M_K - X_{<K} R_{<K,K}) W_K^T), with no barrier between
//    waves; in pass 2 further workgroups form R = R2 R1 and
//    min|R_ii| / max|R_ii|.
//
// Pass 1 is rejected (state 1) when a pivot is not positive or not finite,
// or min R1_ii < 1e-5 max R1_ii; pass 2 (state 2) when max |G2 - I| > 0.1,
// i.e. when Q1 is too far from orthonormal for the second pass to be
// accurate.  The kernels after a rejection return at once, and the cooperative
// Householder kernel, launched behind them, runs only when the state is
// non-zero.  The input M is read by pass 1 only and the output Q is written by
// the last kernel only, so Q may alias M.
#include "common.h"
#include "qr.h"

namespace qrctm {
namespace {

constexpr int kB = 16;                 // block (one FP64 MFMA tile)
constexpr int kGT = 32;                // Gram output tile
constexpr int kCholThreads = 512;
constexpr int kCholWaves = kCholThreads / 64;
constexpr int kCholLdsMaxNb = 11;      // n <= 176: the block triangle in LDS
constexpr double kPass1MinRatio = 1e-5;
constexpr double kPass2MaxDev = 0.1;

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// LDS written by some lanes of a wave and read by others: wait for the writes
// and keep the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int tri_index(int I, int J, int nb) {  // I <= J
    return I * nb - I * (I - 1) / 2 + (J - I);
}

// tile t of the upper triangle of an nt x nt tile grid, row by row
__device__ __forceinline__ void tile_of(int t, int nt, int& I, int& J) {
    int i = 0;
    while (t >= nt - i) {
        t -= nt - i;
        ++i;
    }
    I = i;
    J = i + t;
}

// ---------------------------------------------------------------------------
// G = X^T X (n x n, both triangles written).  Grid: ntri tiles x S splits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ X, int m, int n,
                                                   int nt, int S, int chunk, double* part,
                                                   unsigned* cnt, double* G,
                                                   const int* __restrict__ state) {
    if (state != nullptr && *state != 0) return;
    const int t = blockIdx.x / S, s = blockIdx.x % S;
    int I, J;
    tile_of(t, nt, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int sr = wave >> 1, sc = wave & 1;
    const int ca = I * kGT + sr * kB + (lane & 15), cb = J * kGT + sc * kB + (lane & 15);
    const int k0 = s * chunk, k1 = min(m, k0 + chunk);
    const int kl = lane >> 4;
    const bool va = ca < n, vb = cb < n;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < k1; k += 16) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int row = k + 4 * u + kl;
            const bool vr = row < k1;
            av[u] = (vr && va) ? X[(size_t)row * n + ca] : 0.0;
            bv[u] = (vr && vb) ? X[(size_t)row * n + cb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    // element (row, col) of the 32 x 32 tile held by this lane: (sr 16 + 4 r + kl, sc 16 + lane % 16)
    if (S == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gi = I * kGT + sr * kB + 4 * r + kl, gj = cb;
            if (gi < n && gj < n) {
                G[(size_t)gi * n + gj] = acc[r];
                G[(size_t)gj * n + gi] = acc[r];
            }
        }
        return;
    }
    double* my = part + ((size_t)t * S + s) * (kGT * kGT);
#pragma unroll
    for (int r = 0; r < 4; ++r) my[(sr * kB + 4 * r + kl) * kGT + sc * kB + (lane & 15)] = acc[r];
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(&cnt[t], 1u) == (unsigned)(S - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int e = tid; e < kGT * kGT; e += 256) {
        double v = 0.0;
        for (int q = 0; q < S; ++q) v += part[((size_t)t * S + q) * (kGT * kGT) + e];
        const int gi = I * kGT + e / kGT, gj = J * kGT + e % kGT;
        if (gi < n && gj < n) {
            G[(size_t)gi * n + gj] = v;
            G[(size_t)gj * n + gi] = v;
        }
    }
    if (tid == 0) cnt[t] = 0u;  // ready for the next launch on this scratch
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R of the n x n G (one workgroup).  Writes R (upper, zeros
// below), W[K] = R_KK^{-T} (nb blocks of 16 x 16), the state word and, in
// pass 1, the extreme pivots.
// ---------------------------------------------------------------------------
template <bool kLds>
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const double* __restrict__ G, int n,
                                                            int pass, double* work, double* R,
                                                            double* W, int* state,
                                                            double* stats) {
    extern __shared__ double lds[];
    if (pass == 2 && *state != 0) return;
    const int nb = (n + kB - 1) / kB;
    const int nblk = nb * (nb + 1) / 2;
    double* B = kLds ? lds : work;                // block triangle
    double* Wl = kLds ? lds + (size_t)nblk * 256 : lds;  // W of the current block
    __shared__ int bad;
    __shared__ double dev_max;
    __shared__ double piv_min, piv_max;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        bad = 0;
        dev_max = 0.0;
        piv_min = INFINITY;
        piv_max = 0.0;
    }
    __syncthreads();
    auto blk = [&](int I, int J) { return B + (size_t)tri_index(I, J, nb) * 256; };
    // load the upper block triangle (identity beyond n)
    {
        double dv = 0.0;
        int nf = 0;
        for (long long e = tid; e < (long long)nblk * 256; e += kCholThreads) {
            const int b = (int)(e / 256), w = (int)(e % 256);
            int I = 0, rem = b;
            while (rem >= nb - I) {
                rem -= nb - I;
                ++I;
            }
            const int J = I + rem;
            const int gi = I * kB + w / kB, gj = J * kB + w % kB;
            double v;
            if (gi < n && gj < n) {
                v = G[(size_t)gi * n + gj];
                if (!isfinite(v)) nf = 1;
                dv = fmax(dv, fabs(v - (gi == gj ? 1.0 : 0.0)));
            } else {
                v = gi == gj ? 1.0 : 0.0;
            }
            B[(size_t)b * 256 + w] = v;
        }
        if (nf) atomicOr(&bad, 1);
        if (pass == 2) {
            // max |G - I| over the workgroup (non-negative doubles order as integers)
            atomicMax(reinterpret_cast<unsigned long long*>(&dev_max),
                      (unsigned long long)__double_as_longlong(dv));
        }
    }
    __syncthreads();
    const int kl = lane >> 4, cl = lane & 15;
    for (int K = 0; K < nb; ++K) {
        // (a) diagonal block: wave 0 eliminates on [B_KK | I] (lane c < 16: column
        // c of B_KK, lane 16 + c: column c of I); rows become R_KK and R_KK^{-T}
        if (wave == 0) {
            double* bk = blk(K, K);
            const int c = lane & 31;
            double b[kB];
#pragma unroll
            for (int r = 0; r < kB; ++r) {
                if (lane < 16) b[r] = r <= c ? bk[r * kB + c] : bk[c * kB + r];
                else if (lane < 32) b[r] = (r == c - 16) ? 1.0 : 0.0;
                else b[r] = 0.0;
            }
            double pmin = INFINITY, pmax = 0.0;
            int nonpos = 0;
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                double p = readlane_d(b[j], j);
                if (!(p > 0.0) || !isfinite(p)) {
                    nonpos = 1;
                    p = 1.0;
                }
                const double dj = sqrt(p);
                const double inv = 1.0 / dj;
                if (K * kB + j < n) {
                    pmin = fmin(pmin, dj);
                    pmax = fmax(pmax, dj);
                }
                b[j] *= inv;
#pragma unroll
                for (int i = j + 1; i < kB; ++i) b[i] -= readlane_d(b[j], i) * b[j];
            }
            if (lane < 16) {
#pragma unroll
                for (int r = 0; r < kB; ++r) bk[r * kB + c] = r <= c ? b[r] : 0.0;
            } else if (lane < 32) {
#pragma unroll
                for (int r = 0; r < kB; ++r) {
                    Wl[r * kB + (c - 16)] = b[r];
                    W[(size_t)K * 256 + r * kB + (c - 16)] = b[r];
                }
            }
            if (lane == 0) {
                if (nonpos) bad |= 2;
                piv_min = fmin(piv_min, pmin);
                piv_max = fmax(piv_max, pmax);
            }
        }
        __syncthreads();
        // (b) block row: B_KJ <- W B_KJ for J > K
        for (int J = K + 1 + wave; J < nb; J += kCholWaves) {
            double* bj = blk(K, J);
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int k = 4 * s4 + kl;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[cl * kB + k], bj[k * kB + cl], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) bj[(4 * r + kl) * kB + cl] = acc[r];
        }
        __syncthreads();
        // (c) trailing blocks: B_IJ -= B_KI^T B_KJ for K < I <= J
        {
            int p = 0;
            for (int I = K + 1; I < nb; ++I) {
                for (int J = I; J < nb; ++J, ++p) {
                    if (p % kCholWaves != wave) continue;
                    const double* bi = blk(K, I);
                    const double* bj = blk(K, J);
                    double* bij = blk(I, J);
                    dbl4 acc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = bij[(4 * r + kl) * kB + cl];
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int k = 4 * s4 + kl;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-bi[k * kB + cl], bj[k * kB + cl], acc, 0,
                                                                   0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) bij[(4 * r + kl) * kB + cl] = acc[r];
                }
            }
        }
        __syncthreads();
    }
    // R (n x n, upper) and the verdict
    for (long long e = tid; e < (long long)n * n; e += kCholThreads) {
        const int gi = (int)(e / n), gj = (int)(e % n);
        R[e] = gj >= gi ? blk(gi / kB, gj / kB)[(gi % kB) * kB + gj % kB] : 0.0;
    }
    if (tid == 0) {
        int st = 0;
        if (pass == 1) {
            if (bad || !(piv_min >= kPass1MinRatio * piv_max)) st = 1;
            stats[0] = piv_min;
            stats[1] = piv_max;
        } else {
            if (bad || !(dev_max <= kPass2MaxDev)) st = 2;
        }
        *state = st;
    }
}

// ---------------------------------------------------------------------------
// X = M R^{-1} (R upper with W[K] = R_KK^{-T}); one wave per 16 rows, waves
// per workgroup wpg.  Workgroups from nrow_wg on (pass 2) form Rout = R2 R1
// (upper, zeros below) one 16 x 16 block per wave, and the diagonal ratio.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trsm_kernel(const double* __restrict__ M, int m, int n,
                                                   const double* __restrict__ R,
                                                   const double* __restrict__ W, double* X,
                                                   int wpg, int nrow_wg, const int* state,
                                                   const double* __restrict__ R1, double* Rout,
                                                   double* ratio) {
    extern __shared__ double lds[];
    if (*state != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kl = lane >> 4, cl = lane & 15;
    const int nb = (n + kB - 1) / kB;
    if ((int)blockIdx.x >= nrow_wg) {
        // Rout = R R1 by upper blocks (R = R2 here), and the ratio
        const int q = ((int)blockIdx.x - nrow_wg) * (blockDim.x / 64) + wave;
        const int nblk = nb * (nb + 1) / 2;
        if (q == nblk) {
            double lo = INFINITY, hi = 0.0;
            for (int i = lane; i < n; i += 64) {
                const double v = fabs(R[(size_t)i * n + i] * R1[(size_t)i * n + i]);
                lo = fmin(lo, v);
                hi = fmax(hi, v);
            }
            for (int o = 32; o > 0; o >>= 1) {
                lo = fmin(lo, __shfl_xor(lo, o));
                hi = fmax(hi, __shfl_xor(hi, o));
            }
            if (lane == 0 && ratio != nullptr) *ratio = hi > 0.0 ? lo / hi : 0.0;
            return;
        }
        if (q > nblk) return;
        int I = 0, rem = q;
        while (rem >= nb - I) {
            rem -= nb - I;
            ++I;
        }
        const int J = I + rem;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = I * kB; k0 < min(n, (J + 1) * kB); k0 += 4) {
            const int k = k0 + kl;
            const int ri = I * kB + cl, cj = J * kB + cl;
            const double a = (k < n && ri < n) ? R[(size_t)ri * n + k] : 0.0;
            const double b = (k < n && cj < n) ? R1[(size_t)k * n + cj] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gi = I * kB + 4 * r + kl, gj = J * kB + cl;
            if (gi < n && gj < n) {
                Rout[(size_t)gi * n + gj] = gj >= gi ? acc[r] : 0.0;
                if (I != J) Rout[(size_t)gj * n + gi] = 0.0;
            }
        }
        return;
    }
    if (wave >= wpg) return;
    const int ld = nb * kB + 1;  // odd row stride: the 16 rows of a fragment hit different banks
    double* Xl = lds + (size_t)wave * kB * ld;
    const long long r0 = ((long long)blockIdx.x * wpg + wave) * kB;
    for (int K = 0; K < nb; ++K) {
        const int col = K * kB + cl;
        dbl4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long row = r0 + 4 * r + kl;
            acc[r] = (row < m && col < n) ? M[(size_t)row * n + col] : 0.0;
        }
        for (int kk = 0; kk < K; ++kk) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int k = kk * kB + 4 * s4 + kl;
                const double a = -Xl[cl * ld + k];
                const double b = (k < n && col < n) ? R[(size_t)k * n + col] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
        }
        // X_K = acc W_K^T: acc to LDS (C layout), back as the A operand
#pragma unroll
        for (int r = 0; r < 4; ++r) Xl[(4 * r + kl) * ld + K * kB + cl] = acc[r];
        wave_lds_sync();
        dbl4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int k = 4 * s4 + kl;
            x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xl[cl * ld + K * kB + k], W[(size_t)K * 256 + cl * kB + k], x,
                                                     0, 0, 0);
        }
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Xl[(4 * r + kl) * ld + K * kB + cl] = x[r];
            const long long row = r0 + 4 * r + kl;
            if (row < m && col < n) X[(size_t)row * n + col] = x[r];
        }
        wave_lds_sync();
    }
}

struct GramPlan {
    int nt, ntri, S, chunk;
};

GramPlan gram_plan(int m, int n) {
    GramPlan g;
    g.nt = (n + kGT - 1) / kGT;
    g.ntri = g.nt * (g.nt + 1) / 2;
    // about 768 workgroups, row ranges of at least 256 rows (multiples of 16)
    long long S = ceil_div(768, g.ntri);
    S = std::min<long long>(S, std::max<long long>(1, m / 256));
    S = std::max<long long>(1, S);
    g.chunk = (int)(ceil_div(ceil_div(m, S), 16) * 16);
    g.S = (int)ceil_div(m, g.chunk);
    return g;
}

int trsm_waves(int n) {
    const int nb = (n + kB - 1) / kB;
    const size_t per_wave = sizeof(double) * kB * (size_t)(nb * kB + 1);
    int w = (int)std::min<size_t>(4, (150 * 1024) / per_wave);
    return std::max(1, w);
}

}  // namespace

bool cholqr_supported(int m, int n) {
    if (m < n || n < 1) return false;
    const int nb = (n + kB - 1) / kB;
    // one wave's 16 rows of X in LDS; the block triangle (global beyond n = 176)
    return sizeof(double) * kB * (size_t)(nb * kB + 1) <= 150 * 1024;
}

CholQrScratch cholqr_scratch_layout(int m, int n) {
    CholQrScratch s{};
    if (!cholqr_supported(m, n)) return s;
    const GramPlan g = gram_plan(m, n);
    const int nb = (n + kB - 1) / kB;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += ((bytes + 255) / 256) * 256;
        return o;
    };
    s.off_Q1 = take(sizeof(double) * (size_t)m * n);
    s.off_part = take(sizeof(double) * (size_t)g.ntri * (g.S > 1 ? g.S : 0) * kGT * kGT);
    s.off_G = take(sizeof(double) * (size_t)n * n);
    s.off_R1 = take(sizeof(double) * (size_t)n * n);
    s.off_R2 = take(sizeof(double) * (size_t)n * n);
    s.off_W1 = take(sizeof(double) * (size_t)nb * 256);
    s.off_W2 = take(sizeof(double) * (size_t)nb * 256);
    s.off_work = take(nb > kCholLdsMaxNb ? sizeof(double) * (size_t)nb * (nb + 1) / 2 * 256 : 0);
    s.off_stats = take(sizeof(double) * 4);
    s.off_state = take(sizeof(int));
    s.off_cnt = take(sizeof(unsigned) * (size_t)g.ntri);
    s.cnt_words = g.ntri;
    s.total = off;
    return s;
}

Status cholqr2(const double* M, double* Q, double* R, int m, int n, char* base,
               const CholQrScratch& L, double* diag_ratio_dev, int** state_out, hipStream_t st) {
    const GramPlan g = gram_plan(m, n);
    const int nb = (n + kB - 1) / kB;
    double* Q1 = reinterpret_cast<double*>(base + L.off_Q1);
    double* part = reinterpret_cast<double*>(base + L.off_part);
    double* G = reinterpret_cast<double*>(base + L.off_G);
    double* R1 = reinterpret_cast<double*>(base + L.off_R1);
    double* R2 = reinterpret_cast<double*>(base + L.off_R2);
    double* W1 = reinterpret_cast<double*>(base + L.off_W1);
    double* W2 = reinterpret_cast<double*>(base + L.off_W2);
    double* work = reinterpret_cast<double*>(base + L.off_work);
    double* stats = reinterpret_cast<double*>(base + L.off_stats);
    int* state = reinterpret_cast<int*>(base + L.off_state);
    unsigned* cnt = reinterpret_cast<unsigned*>(base + L.off_cnt);
    *state_out = state;

    const bool in_lds = nb <= kCholLdsMaxNb;
    const size_t chol_lds =
        sizeof(double) * (in_lds ? (size_t)nb * (nb + 1) / 2 * 256 + 256 : 256);
    const void* chol = in_lds ? (const void*)chol_kernel<true> : (const void*)chol_kernel<false>;
    QRCTM_HIP(hipFuncSetAttribute(chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds));
    const int wpg = trsm_waves(n);
    const size_t trsm_lds = sizeof(double) * (size_t)wpg * kB * (nb * kB + 1);
    QRCTM_HIP(hipFuncSetAttribute((const void*)trsm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)trsm_lds));
    const int nrow_wg = (int)ceil_div(ceil_div(m, kB), wpg);
    const int nblk = nb * (nb + 1) / 2;
    const int nr_wg = (int)ceil_div(nblk + 1, 4);  // R = R2 R1 blocks and the ratio, 4 waves each

    for (int pass = 1; pass <= 2; ++pass) {
        const double* X = pass == 1 ? M : Q1;
        hipLaunchKernelGGL(gram_kernel, dim3(g.ntri * g.S), dim3(256), 0, st, X, m, n, g.nt, g.S, g.chunk,
                           part, cnt, G, pass == 1 ? nullptr : state);
        QRCTM_TRY(launch_check("gram_kernel"));
        double* Rp = pass == 1 ? R1 : R2;
        double* Wp = pass == 1 ? W1 : W2;
        if (in_lds)
            hipLaunchKernelGGL(chol_kernel<true>, dim3(1), dim3(kCholThreads), chol_lds, st, G, n, pass,
                               work, Rp, Wp, state, stats);
        else
            hipLaunchKernelGGL(chol_kernel<false>, dim3(1), dim3(kCholThreads), chol_lds, st, G, n, pass,
                               work, Rp, Wp, state, stats);
        QRCTM_TRY(launch_check("chol_kernel"));
        if (pass == 1) {
            hipLaunchKernelGGL(trsm_kernel, dim3(nrow_wg), dim3(64 * wpg), trsm_lds, st, M, m, n, R1, W1, Q1,
                               wpg, nrow_wg, state, nullptr, nullptr, nullptr);
        } else {
            hipLaunchKernelGGL(trsm_kernel, dim3(nrow_wg + nr_wg), dim3(64 * std::max(wpg, 4)), trsm_lds, st,
                               Q1, m, n, R2, W2, Q, wpg, nrow_wg, state, R1, R, diag_ratio_dev);
        }
        QRCTM_TRY(launch_check("trsm_kernel"));
    }
    return Status{};
}

}  // namespace qrctm
