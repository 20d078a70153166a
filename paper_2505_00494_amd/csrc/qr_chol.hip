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
// Per pass, none of the kernels cooperative:
//  * gram_kernel: 32 x 32 tiles of the upper block triangle of X^T X, each
//    split over S row ranges (FP64 matrix cores; the loads of the next 64 rows
//    in flight while the current ones are multiplied), and gram_reduce_kernel,
//    which adds the S partial tiles in a fixed order (the sum is
//    deterministic) and writes each tile and its mirror.  (A last-arriving
//    workgroup could add them in the same kernel, but the device-scope fences
//    that would need drop every XCD's L2 for all workgroups);
//  * chol_kernel: one workgroup, right-looking blocked Cholesky with 16 x 16
//    blocks (kept in LDS for n <= 176, in global memory beyond).  Wave 0
//    factors a diagonal block in registers, eliminating on [B | I] so that it
//    also yields W_K = R_KK^{-T}; all waves form the block row W_K B_KJ, and in
//    the trailing update B_IJ -= B_KI^T B_KJ (matrix cores) wave 0 takes the
//    next diagonal block and factors it at once while the others update the
//    rest (two barriers per block column).  The same row operations applied
//    to the identity give R^{-T} (Gauss-Jordan), kept in the slots of the
//    finished block rows of R; the waves that do not factor write R and
//    R^{-1} out block by block as they become final.  In pass
//    2, when max |G2 - I| is below 1e-8, R2 = I + E_u (E = G2 - I, E_u its
//    upper triangle with half the diagonal) and R2^{-1} = I - E_u, exact to
//    |E|^2, below the rounding unit, replace the factorisation: the Gram
//    reduction of pass 2 writes them and max |G2 - I| (one atomic maximum per
//    wave), and the Cholesky kernel then only sets the state word;
//  * the two products M R^{-1} on the FP64 GEMM of the step (the second gated
//    by the state word, as it overwrites M when Q aliases M), and
//    rprod_kernel: R = R2 R1 by upper 16 x 16 blocks, and min|R_ii|/max|R_ii|.
//
// Pass 1 is rejected (state 1) when a pivot is not positive or not finite,
// or min R1_ii < 1e-5 max R1_ii; pass 2 (state 2) when max |G2 - I| > 0.1,
// i.e. when Q1 is too far from orthonormal for the second pass to be
// accurate.  The kernels after a rejection return at once, and the Householder
// kernel, launched behind them (an ordinary launch), runs only when the state
// is non-zero.  The input M is read by pass 1 only and the output Q is written by
// the last product only, so Q may alias M.
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
constexpr double kFirstOrderMaxDev = 1e-8;  // pass 2: |E|^2 below the rounding unit

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
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
                                                   int nt, int S, int chunk, double* part, double* G,
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
    // 64 rows per round: 16 operand pairs per lane, the next round's in flight
    constexpr int kU = 16;
    double av[kU], bv[kU], an[kU], bn[kU];
    auto load = [&](int k, double* A_, double* B_) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int row = k + 4 * u + kl;
            const bool vr = row < k1;
            A_[u] = (vr && va) ? X[(size_t)row * n + ca] : 0.0;
            B_[u] = (vr && vb) ? X[(size_t)row * n + cb] : 0.0;
        }
    };
    if (k0 < k1) load(k0, av, bv);
    for (int k = k0; k < k1; k += 4 * kU) {
        const bool more = k + 4 * kU < k1;
        if (more) load(k + 4 * kU, an, bn);
#pragma unroll
        for (int u = 0; u < kU; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        if (more) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                av[u] = an[u];
                bv[u] = bn[u];
            }
        }
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
}

// G tiles from the S partial tiles (gram_kernel with S > 1), summed in a fixed
// order: workgroup (t, quarter) adds 256 entries of tile t, eight partials'
// loads in flight at a time.
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part, int n, int nt,
                                                          int S, double* G, const int* __restrict__ state,
                                                          double* R, double* Ri, unsigned long long* devw) {
    if (state != nullptr && *state != 0) return;
    const int t = blockIdx.x / 4, e = (blockIdx.x % 4) * 256 + threadIdx.x;
    int I, J;
    tile_of(t, nt, I, J);
    const double* pt = part + (size_t)t * S * (kGT * kGT) + e;
    double v = 0.0;
    for (int s0 = 0; s0 < S; s0 += 8) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = s0 + u < S ? pt[(size_t)(s0 + u) * (kGT * kGT)] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) v += w[u];
    }
    const int gi = I * kGT + e / kGT, gj = J * kGT + e % kGT;
    const bool in = gi < n && gj < n;
    if (in) {
        G[(size_t)gi * n + gj] = v;
        G[(size_t)gj * n + gi] = v;
    }
    if (R == nullptr) return;
    // second pass: the first-order factors R2 = I + E_u, R2^{-1} = I - E_u
    // (E_u the upper triangle of E = G - I with half its diagonal), kept when
    // max |G - I| <= 1e-8, and that maximum (a non-finite entry counts as +inf;
    // non-negative doubles order as their bit patterns)
    double dev = 0.0;
    if (in) {
        const bool up = gj >= gi;
        const double x = gj > gi ? v : 0.5 * (v - 1.0);
        R[(size_t)gi * n + gj] = up ? (gi == gj ? 1.0 : 0.0) + x : 0.0;
        Ri[(size_t)gi * n + gj] = up ? (gi == gj ? 1.0 : 0.0) - x : 0.0;
        if (I != J) {
            R[(size_t)gj * n + gi] = 0.0;
            Ri[(size_t)gj * n + gi] = 0.0;
        }
        if (up) dev = isfinite(v) ? fabs(v - (gi == gj ? 1.0 : 0.0)) : INFINITY;
    }
    for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o));
    if ((threadIdx.x & 63) == 0) atomicMax(devw, (unsigned long long)__double_as_longlong(dev));
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R of the n x n G (one workgroup) and R^{-1} with it.
// Writes R and Ri = R^{-1} (n x n, upper, zeros below), the state word and,
// in pass 1, the extreme pivots.
//
// Row operations that take G to R take [G | I] to [R | R^{-T}], so R^{-1} is
// accumulated beside the factorisation (Gauss-Jordan on the block triangle):
// block row K of R^{-T}, X_KJ (J < K), goes through the same steps as R's,
// X_KJ <- W_K X_KJ with W_K = R_KK^{-T}, and its trailing update is
// X_IJ -= R_KI^T X_KJ (I > K).  X_IJ (J < I) lives in the slot of R_JI, which
// step J still reads; the slot turns into X_IJ at step J + 1, whose first
// touch also adds the term X_IJ = -R_JI^T W_J that step J would have written.
// Each slot is written by one wave per phase and read by no other in it.
// ---------------------------------------------------------------------------
template <bool kLds>
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const double* __restrict__ G, int n,
                                                            int pass, double* work, double* R,
                                                            double* Ri, int* state, double* stats,
                                                            unsigned long long* devw) {
    extern __shared__ double lds[];
    if (pass == 2 && *state != 0) return;
    if (pass == 1 && devw != nullptr && threadIdx.x == 0) *devw = 0ull;
    if (pass == 2 && devw != nullptr &&
        __longlong_as_double((long long)*devw) <= kFirstOrderMaxDev) {
        // the Gram reduction wrote the first-order factors
        if (threadIdx.x == 0) *state = 0;
        return;
    }
    const int nb = (n + kB - 1) / kB;
    const int nblk = nb * (nb + 1) / 2;
    double* B = kLds ? lds : work;                                 // block triangle
    double* const Wr = kLds ? lds + (size_t)nblk * 256 : lds;      // W_K, ring of three
    __shared__ int bad;
    __shared__ double dev_max;
    __shared__ double piv_min, piv_max;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kl = lane >> 4, cl = lane & 15;
    if (tid == 0) {
        bad = 0;
        dev_max = 0.0;
        piv_min = INFINITY;
        piv_max = 0.0;
    }
    __syncthreads();
    auto blk = [&](int I, int J) { return B + (size_t)tri_index(I, J, nb) * 256; };
    auto wblk = [&](int K) { return Wr + (K % 3) * 256; };
    // load the upper block triangle (identity beyond n): element e of the
    // triangle is element e % 256 of block e / 256 (row by row), thread t takes
    // e = t, t + 512, ...: a wave reads whole rows of 16 of G, and kU loads per
    // lane are in flight (one round up to chi = 144, two up to 176)
    {
        constexpr int kU = 24;
        const int total = nblk * 256;
        double dv = 0.0;
        int nf = 0;
        const bool first_order = pass == 2 && devw == nullptr;
        for (int e0 = tid; e0 < total; e0 += kU * kCholThreads) {
            int bi, bj;
            tile_of(e0 >> 8, nb, bi, bj);
            int I = bi, J = bj;
            double v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {  // block of e0 + 512 u: two blocks on each time
                const int e = e0 + u * kCholThreads;
                const int gi = I * kB + ((e >> 4) & 15), gj = J * kB + (e & 15);
                v[u] = (e < total && gi < n && gj < n) ? G[(size_t)gi * n + gj] : (gi == gj ? 1.0 : 0.0);
                J += 2;
                while (J >= nb && I < nb) {
                    ++I;
                    J += I - nb;
                }
            }
            I = bi;
            J = bj;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + u * kCholThreads;
                if (e < total) {
                    const int gi = I * kB + ((e >> 4) & 15), gj = J * kB + (e & 15);
                    blk(I, J)[e & 255] = v[u];
                    if (gi < n && gj < n && gj >= gi) {
                        if (!isfinite(v[u])) nf = 1;
                        dv = fmax(dv, fabs(v[u] - (gi == gj ? 1.0 : 0.0)));
                        if (first_order) {
                            // the first-order factors (kept if max |G - I| <= 1e-8, else
                            // overwritten below): R2 = I + E_u, R2^{-1} = I - E_u, E_u the
                            // upper triangle of E = G - I with half its diagonal
                            const double x = gj > gi ? v[u] : 0.5 * (v[u] - 1.0);
                            R[(size_t)gi * n + gj] = (gi == gj ? 1.0 : 0.0) + x;
                            Ri[(size_t)gi * n + gj] = (gi == gj ? 1.0 : 0.0) - x;
                        }
                    }
                }
                J += 2;
                while (J >= nb && I < nb) {
                    ++I;
                    J += I - nb;
                }
            }
        }
        if (first_order) {
            for (int e = tid; e < n * n; e += kCholThreads) {
                const int gi = e / n, gj = e % n;
                if (gj < gi) R[e] = Ri[e] = 0.0;
            }
        }
        if (nf) atomicOr(&bad, 1);
        if (pass == 2) {
            // max |G - I| over the workgroup (non-negative doubles order as integers)
            atomicMax(reinterpret_cast<unsigned long long*>(&dev_max),
                      (unsigned long long)__double_as_longlong(dv));
        }
    }
    __syncthreads();
    if (pass == 2 && dev_max <= kFirstOrderMaxDev) {  // |E|^2 below the rounding unit
        if (tid == 0) *state = bad ? 2 : 0;
        return;
    }
    // diagonal block K: wave 0 eliminates on [B_KK | I] (lane c < 16: column c of
    // B_KK, lane 16 + c: column c of I); its rows become R_KK and W_K = R_KK^{-T}.
    // Per pivot j (p = B_jj): row i > j loses B_ji / p times row j (the
    // multipliers B_ji read from lane i), row j + 1 first, as its lane j + 1
    // holds the next pivot; then row j is scaled by 1/sqrt(p).  Only 1/p lies
    // on the chain from one pivot to the next (the hardware estimate and two
    // Newton steps); 1/sqrt(p) likewise, beside it.  A pivot that is not
    // positive or not finite is recorded and replaced by 1 (the pass is then
    // rejected).
    auto factor_diag = [&](int K) {
        double* bk = blk(K, K);
        double* wk = wblk(K);
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
            double m[kB];
#pragma unroll
            for (int i = j; i < kB; ++i) m[i] = readlane_d(b[j], i);
            double p = m[j];
            if (!(p > 0.0) || !isfinite(p)) {
                nonpos = 1;
                p = 1.0;
            }
            double y = __builtin_amdgcn_rcp(p);
            y = fma(y, fma(-p, y, 1.0), y);
            y = fma(y, fma(-p, y, 1.0), y);
            const double tj = b[j] * y;
#pragma unroll
            for (int i = j + 1; i < kB; ++i) b[i] = fma(-m[i], tj, b[i]);
            double r = __builtin_amdgcn_rsq(p);
            const double hp = 0.5 * p;
            r = r * fma(-hp * r, r, 1.5);
            r = r * fma(-hp * r, r, 1.5);
            b[j] *= r;
            const double dj = p * r;
            if (K * kB + j < n) {
                pmin = fmin(pmin, dj);
                pmax = fmax(pmax, dj);
            }
        }
        if (lane < 16) {
#pragma unroll
            for (int r = 0; r < kB; ++r) bk[r * kB + c] = r <= c ? b[r] : 0.0;
        } else if (lane < 32) {
#pragma unroll
            for (int r = 0; r < kB; ++r) wk[r * kB + (c - 16)] = b[r];
        }
        if (lane == 0) {
            if (nonpos) bad |= 2;
            piv_min = fmin(piv_min, pmin);
            piv_max = fmax(piv_max, pmax);
        }
    };
    // 16 x 16 products of one wave on the matrix cores.  acc in the accumulator
    // layout (lane l, register r: element (4 r + l / 16, l % 16)), which is also
    // the B-operand layout of a next product.  mm_tn: acc -= a^T b; mm_nn2:
    // a b; mm_nr: acc += a t with t held in registers.
    auto ld = [&](const double* d) {
        dbl4 x;
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = d[(4 * r + kl) * kB + cl];
        return x;
    };
    auto st = [&](double* d, const dbl4& x) {
#pragma unroll
        for (int r = 0; r < 4; ++r) d[(4 * r + kl) * kB + cl] = x[r];
    };
    auto mm_tn = [&](dbl4 acc, const double* a, const double* b) {
        double av[4], bv[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            av[s4] = -a[(4 * s4 + kl) * kB + cl];
            bv[s4] = b[(4 * s4 + kl) * kB + cl];
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], bv[s4], acc, 0, 0, 0);
        return acc;
    };
    auto mm_nn2 = [&](const double* a, const double* b) {  // a b, two chains of two steps
        double av[4], bv[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            av[s4] = a[cl * kB + 4 * s4 + kl];
            bv[s4] = b[(4 * s4 + kl) * kB + cl];
        }
        dbl4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bv[0], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[2], bv[2], c1, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bv[1], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[3], bv[3], c1, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) c0[r] += c1[r];
        return c0;
    };
    auto mm_nr = [&](dbl4 acc, const double* a, const dbl4& t) {
        double av[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) av[s4] = a[cl * kB + 4 * s4 + kl];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], t[s4], acc, 0, 0, 0);
        return acc;
    };
    const dbl4 zero4 = {0.0, 0.0, 0.0, 0.0};
    // block (K, J) of R and block (J, K) of Ri = X^T (X_KJ, J < K, in the slot
    // of (J, K); X_KK = W_K), zeros outside the triangles, to global memory
    auto write_out = [&](int K, int J) {
        const double* rs = J >= K ? blk(K, J) : nullptr;
        const double* xs = J < K ? blk(J, K) : (J == K ? wblk(K) : nullptr);
        double rv[4], xv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            rv[r] = rs != nullptr ? rs[(4 * r + kl) * kB + cl] : 0.0;
            xv[r] = xs != nullptr ? xs[cl * kB + 4 * r + kl] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 4 * r + kl;
            const int ri = K * kB + a, rj = J * kB + cl;  // R element (ri, rj)
            if (ri < n && rj < n) R[(size_t)ri * n + rj] = rv[r];
            const int xi = J * kB + a, xj = K * kB + cl;  // Ri element (xi, xj) = X_KJ[cl][a]
            if (xi < n && xj < n) Ri[(size_t)xi * n + xj] = xv[r];
        }
    };
    // one trailing block: s -= a^T b, where s first becomes -s^T w if `first`
    // (the slot's first touch); two of them at a time, so that the loads and
    // the two chains of matrix-core steps overlap
    struct Item {
        double* s;
        const double* a;
        const double* b;
        const double* w;
        bool first;
    };
    auto two_items = [&](const Item& x, const Item& y, bool store_y) {
        double xs[4], ys[4], xa[4], xb[4], ya[4], yb[4], xw[4], yw[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int o = (4 * s4 + kl) * kB + cl;
            xs[s4] = x.s[o];
            ys[s4] = y.s[o];
            xa[s4] = -x.a[o];
            xb[s4] = x.b[o];
            ya[s4] = -y.a[o];
            yb[s4] = y.b[o];
            xw[s4] = x.w[o];
            yw[s4] = y.w[o];
        }
        dbl4 ax = {xs[0], xs[1], xs[2], xs[3]}, ay = {ys[0], ys[1], ys[2], ys[3]};
        if (x.first) {
            ax = zero4;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) ax = __builtin_amdgcn_mfma_f64_16x16x4f64(-xs[s4], xw[s4], ax, 0, 0, 0);
        }
        if (y.first) {
            ay = zero4;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) ay = __builtin_amdgcn_mfma_f64_16x16x4f64(-ys[s4], yw[s4], ay, 0, 0, 0);
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            ax = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s4], xb[s4], ax, 0, 0, 0);
            ay = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[s4], yb[s4], ay, 0, 0, 0);
        }
        st(x.s, ax);
        if (store_y) st(y.s, ay);
    };
    if (wave == 0) factor_diag(0);
    __syncthreads();
    for (int K = 0; K < nb; ++K) {
        // block row K: R_KJ = W_K B_KJ (J > K) and X_KJ <- W_K X_KJ (J < K); the
        // slot of (K - 1, K) still holds R_{K-1,K}, so X_{K,K-1} = -W_K R_{K-1,K}^T W_{K-1}
        for (int t = wave; t < nb - 1; t += kCholWaves) {
            const int J = t < K ? t : t + 1;
            double* s = J > K ? blk(K, J) : blk(J, K);
            if (J == K - 1) {
                const dbl4 u = mm_tn(zero4, s, wblk(K - 1));
                st(s, mm_nr(zero4, wblk(K), u));
            } else {
                st(s, mm_nn2(wblk(K), s));
            }
        }
        __syncthreads();
        if (K + 1 == nb) {
            for (int J = wave; J < nb; J += kCholWaves) write_out(K, J);
            break;
        }
        // trailing blocks: wave 0 updates B_{K+1,K+1} and factors it (lookahead);
        // the other waves take B_IJ -= R_KI^T R_KJ (K < I <= J), X_IJ -= R_KI^T X_KJ
        // (I > K, J < K; at J = K - 1 the slot's first touch, X_IJ = -R_JI^T W_J
        // first), and write block row K of R and block column K of Ri
        if (wave == 0) {
            double* s = blk(K + 1, K + 1);
            st(s, mm_tn(ld(s), blk(K, K + 1), blk(K, K + 1)));
            factor_diag(K + 1);
        } else {
            // items: the trailing blocks of B after (K+1, K+1), row by row; the
            // blocks X_IJ (I > K, J < K); the write-outs.  Wave w takes items
            // w - 1, w + 6, ..., two at a time.
            const int nt = nb - K - 1;
            const int nleft = nt * (nt + 1) / 2 - 1, nx = nt * K;
            auto item = [&](int q) {
                Item it;
                if (q < nleft) {
                    int i, j;
                    tile_of(q + 1, nt, i, j);
                    it.s = blk(K + 1 + i, K + 1 + j);
                    it.a = blk(K, K + 1 + i);
                    it.b = blk(K, K + 1 + j);
                    it.w = it.s;
                    it.first = false;
                } else {
                    const int t = q - nleft, I = K + 1 + t / K, J = t % K;
                    it.s = blk(J, I);
                    it.a = blk(K, I);
                    it.b = blk(J, K);
                    it.first = J == K - 1;
                    it.w = it.first ? wblk(J) : it.s;
                }
                return it;
            };
            constexpr int kTw = kCholWaves - 1;
            for (int q = wave - 1; q < nleft + nx; q += 2 * kTw) {
                const bool two = q + kTw < nleft + nx;
                const Item x = item(q);
                two_items(x, two ? item(q + kTw) : x, two);
            }
            for (int q = nleft + nx; q < nleft + nx + nb; ++q)
                if (q % kTw == wave - 1) write_out(K, q - nleft - nx);
        }
        __syncthreads();
    }
    if (tid == 0) {
        int st_ = 0;
        if (pass == 1) {
            if (bad || !(piv_min >= kPass1MinRatio * piv_max)) st_ = 1;
            stats[0] = piv_min;
            stats[1] = piv_max;
        } else {
            if (bad || !(dev_max <= kPass2MaxDev)) st_ = 2;
        }
        *state = st_;
    }
}

// R = R2 R1 (upper, zeros below) by 16 x 16 blocks, one per wave, and the
// ratio min|R_ii| / max|R_ii| (diag(R) = diag(R2) diag(R1)) by wave nblk.
__global__ __launch_bounds__(256) void rprod_kernel(const double* __restrict__ R2,
                                                    const double* __restrict__ R1, int n,
                                                    double* Rout, double* ratio,
                                                    const int* __restrict__ state) {
    if (*state != 0) return;
    const int lane = threadIdx.x & 63, kl = lane >> 4, cl = lane & 15;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nb = (n + kB - 1) / kB;
    const int nblk = nb * (nb + 1) / 2;
    if (q == nblk) {
        double lo = INFINITY, hi = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double v = fabs(R2[(size_t)i * n + i] * R1[(size_t)i * n + i]);
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
    int I, J;
    tile_of(q, nb, I, J);
    // k over [16 I, 16 (J + 1)), eight MFMA steps per batch with their 16 loads
    // issued together (indices clamped into the matrices, values masked)
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const int kend = min(n, (J + 1) * kB);
    const int ri = min(I * kB + cl, n - 1), cj = min(J * kB + cl, n - 1);
    const bool rok = I * kB + cl < n, cok = J * kB + cl < n;
    for (int k0 = I * kB; k0 < kend; k0 += 32) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = min(k0 + 4 * u + kl, n - 1);
            a[u] = R2[ri * n + k];
            b[u] = R1[k * n + cj];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool kok = k0 + 4 * u + kl < kend;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(kok && rok ? a[u] : 0.0, kok && cok ? b[u] : 0.0,
                                                       acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gi = I * kB + 4 * r + kl, gj = J * kB + cl;
        if (gi < n && gj < n) {
            Rout[(size_t)gi * n + gj] = gj >= gi ? acc[r] : 0.0;
            if (I != J) Rout[(size_t)gj * n + gi] = 0.0;
        }
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

GemmDesc solve_desc(const double* X, const double* Rinv, double* out, int m, int n) {
    GemmDesc g;  // out = X Rinv (m x n times n x n)
    g.M = m; g.N = n; g.K = n;
    g.A = X; g.lda = n; g.B = Rinv; g.ldb = n;
    g.C = out; g.map = OutMap::plain(m, n, n);
    return g;
}

}  // namespace

bool cholqr_supported(int m, int n) { return m >= n && n >= 1 && n <= 1024; }

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
    s.off_Ri = take(sizeof(double) * (size_t)n * n);
    s.off_work = take(nb > kCholLdsMaxNb ? sizeof(double) * (size_t)nb * (nb + 1) / 2 * 256 : 0);
    s.off_stats = take(sizeof(double) * 4);
    s.off_state = take(sizeof(int));
    s.off_dev = take(sizeof(unsigned long long));
    s.splitk_bytes = gemm_splitk_bytes(solve_desc(nullptr, nullptr, nullptr, m, n));
    s.off_splitk = take(s.splitk_bytes);
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
    double* Ri = reinterpret_cast<double*>(base + L.off_Ri);
    double* work = reinterpret_cast<double*>(base + L.off_work);
    double* stats = reinterpret_cast<double*>(base + L.off_stats);
    int* state = reinterpret_cast<int*>(base + L.off_state);
    unsigned long long* devw = reinterpret_cast<unsigned long long*>(base + L.off_dev);
    void* sk = base + L.off_splitk;
    *state_out = state;

    const bool in_lds = nb <= kCholLdsMaxNb;
    const size_t chol_lds =
        sizeof(double) * ((in_lds ? (size_t)nb * (nb + 1) / 2 * 256 : 0) + 3 * 256);
    const void* chol = in_lds ? (const void*)chol_kernel<true> : (const void*)chol_kernel<false>;
    QRCTM_HIP(hipFuncSetAttribute(chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds));
    const int nblk = nb * (nb + 1) / 2;

    for (int pass = 1; pass <= 2; ++pass) {
        const double* X = pass == 1 ? M : Q1;
        const int* gate = pass == 1 ? nullptr : state;
        hipLaunchKernelGGL(gram_kernel, dim3(g.ntri * g.S), dim3(256), 0, st, X, m, n, g.nt, g.S, g.chunk,
                           part, G, gate);
        QRCTM_TRY(launch_check("gram_kernel"));
        if (g.S > 1) {
            hipLaunchKernelGGL(gram_reduce_kernel, dim3(g.ntri * 4), dim3(256), 0, st, part, n, g.nt, g.S, G,
                               gate, pass == 2 ? R2 : nullptr, pass == 2 ? Ri : nullptr, devw);
            QRCTM_TRY(launch_check("gram_reduce_kernel"));
        }
        double* Rp = pass == 1 ? R1 : R2;
        // the first-order shortcut of pass 2 comes from the Gram reduction
        unsigned long long* dw = g.S > 1 ? devw : nullptr;
        if (in_lds)
            hipLaunchKernelGGL(chol_kernel<true>, dim3(1), dim3(kCholThreads), chol_lds, st, G, n, pass,
                               work, Rp, Ri, state, stats, dw);
        else
            hipLaunchKernelGGL(chol_kernel<false>, dim3(1), dim3(kCholThreads), chol_lds, st, G, n, pass,
                               work, Rp, Ri, state, stats, dw);
        QRCTM_TRY(launch_check("chol_kernel"));
        // Q1 = M R1^{-1} into scratch; Q = Q1 R2^{-1} only if both passes were accepted
        GemmDesc sd = solve_desc(X, Ri, pass == 1 ? Q1 : Q, m, n);
        sd.gate = pass == 1 ? nullptr : state;
        QRCTM_TRY(gemm_f64(sd, sk, L.splitk_bytes, st));
    }
    hipLaunchKernelGGL(rprod_kernel, dim3((unsigned)ceil_div(nblk + 1, 4)), dim3(256), 0, st, R2, R1, n, R,
                       diag_ratio_dev, state);
    return launch_check("rprod_kernel");
}

}  // namespace qrctm
