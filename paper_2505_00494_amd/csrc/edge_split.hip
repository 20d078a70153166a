// Fused edge contraction 3b: ket layer, then bra layer (see edge_split.h for
// the formulas).
//
// Work unit: one (al, f) block of Y, D^4 contiguous doubles.  A workgroup takes
// P consecutive blocks (a batch) at a time, so that the P D^2 rows of its two
// products fill 16-row MFMA tiles, and loops over batches (persistent grid).
// Batches are handed out by an atomic ticket counter, so a workgroup that
// starts late (its CU busy with other work) simply takes fewer of them; the
// workgroup that draws the last ticket of the launch resets the counter.
// Per batch and per physical index s:
//   GEMM 1  x[(p u_b l_b)][(r_k d_k)] = sum_{(u_k l_k)} ys[..] Bk[s]   (LDS A, register B)
//   GEMM 2  z[(p r_k d_k)][(r_b d_b)] += sum_{(u_b l_b)} xs[..] Bk[s]
// Both are M = P D^2, K = D^2, N = D^2 products on v_mfma_f64_16x16x4f64.
// Each wave owns one 16-column tile and a group of row tiles of both
// products; its B fragments (the same matrix Bk[s] for both) stay in
// registers for the whole launch, or (D = 6, where three waves per SIMD leave
// no room for them) come from a copy of Bk in LDS.  The Y block is staged in LDS transposed (ys[k][m], m
// contiguous), and GEMM 1 writes its result transposed (xs[k][m]), so every
// A fragment is a 16-double contiguous read per quarter-wave.  The next
// batch's Y is loaded into registers once GEMM 1 of the last s has consumed
// ys (while x is dead), in flight during GEMM 2, and written to LDS after it.  HBM traffic is Y
// once and Z once; the double-layer tensor is never read.
#include "edge_split.h"

namespace qrctm {
namespace {

// unsigned ticket counters kept after the prepared operand
constexpr int kTickets = 16;

// Batch size P, row groups G and register budget (waves per SIMD) per bond
// dimension.  P D^2 rows are padded to MT tiles of 16; wave w takes the
// column tile w % NB and the MT / G row tiles of group w / NB.
constexpr int kPairs[9] = {0, 80, 20, 8, 5, 3, 5, 1, 1};
constexpr int kGroups[9] = {0, 5, 5, 5, 5, 5, 4, 2, 1};
constexpr int kWavesPerSimd[9] = {0, 2, 2, 2, 2, 2, 3, 2, 2};
// B fragments read from an LDS copy of Bk instead of being held in registers
// (where the register budget of three waves per SIMD is too small for them)
constexpr bool kBInLds[9] = {false, false, false, false, false, false, true, false, false};

template <int D>
struct Shape3b {
    static constexpr int R = D * D;                    // one double-layer leg
    static constexpr int KP = (R + 3) / 4 * 4;         // contraction length (MFMA depth 4)
    static constexpr int NP = (R + 15) / 16 * 16;      // output columns (MFMA width 16)
    static constexpr int NB = NP / 16;                 // column tiles
    static constexpr int P = kPairs[D];                // (al, f) blocks per batch
    static constexpr int MP = (P * R + 15) / 16 * 16;  // rows, padded to the tile
    static constexpr int MT = MP / 16;                 // row tiles
    static constexpr int G = kGroups[D];
    static constexpr int MTW = MT / G;                 // row tiles per wave
    static constexpr int NT = NB * G * 64;             // threads
    static constexpr int LDM = MP;                     // LDS row length (doubles)
    static constexpr int NY = P * R * R;               // Y doubles per batch
    static constexpr int NL = (NY + NT - 1) / NT;      // ... per thread
    static constexpr int WPE = kWavesPerSimd[D];
    static constexpr bool BLDS = kBInLds[D];
    static constexpr int NBS = BLDS ? 2 * KP * NP : 1;  // LDS doubles for Bk (d = 2)
    static constexpr int KU = BLDS ? 3 : KP / 4;         // k steps unrolled
    static_assert(MT % G == 0, "row tiles split evenly over the groups");
};

// The products on the FP64 matrix cores (CT = double) or, for the mixed
// forms, on the FP32 ones (CT = float: Y and Bk rounded to FP32 in LDS and
// registers, FP32 accumulation, Z stored as double).
template <class CT> struct SplitMma;
template <> struct SplitMma<double> {
    typedef dbl4 acc_t;
    __device__ static acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row (within the 16-row tile) of accumulator element r of quarter-wave q
    __device__ static int row(int r, int q) { return 4 * r + q; }
};
template <> struct SplitMma<float> {
    typedef flt4 acc_t;
    __device__ static acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int r, int q) { return 4 * q + r; }
};

template <class CT, int D, int DP>
__global__ __launch_bounds__(Shape3b<D>::NT)
__attribute__((amdgpu_waves_per_eu(Shape3b<D>::WPE))) void edge_split_kernel(
    const double* __restrict__ Y, const double* __restrict__ Bk, int chi, int npairs,
    double* __restrict__ Z, unsigned* ticket) {
    using S = Shape3b<D>;
    using M = SplitMma<CT>;
    typedef typename M::acc_t acc_t;
    constexpr int R = S::R, KP = S::KP, NP = S::NP, NB = S::NB, P = S::P, MTW = S::MTW;
    constexpr int LDM = S::LDM, NT = S::NT, NY = S::NY, NL = S::NL, KS = KP / 4;
    __shared__ CT ys[KP * LDM];  // ys[(u_k l_k)][(p u_b l_b)]
    __shared__ CT xs[KP * LDM];  // xs[(u_b l_b)][(p r_k d_k)]
    __shared__ int next_batch;
    __shared__ CT bs[S::NBS];    // Bk (when S::BLDS)
    constexpr bool BLDS = S::BLDS;
    constexpr int KU = S::KU;

    const int tid = threadIdx.x;
    const int lane = tid & 63, q = lane >> 4, l16 = lane & 15;
    const int w = tid >> 6;
    const int nt = w % NB, mt0 = (w / NB) * MTW;
    const int nbatch = (npairs + P - 1) / P;
    // one ticket per batch, plus one that ends each workgroup: nbatch + gridDim.x in all
    auto draw = [&]() {
        if (tid == 0) {
            const unsigned t = atomicAdd(ticket, 1u);
            if (t == (unsigned)(nbatch + gridDim.x - 1)) atomicExch(ticket, 0u);
            next_batch = (int)min(t, (unsigned)nbatch);
        }
    };
    draw();
    __syncthreads();
    int b = next_batch;
    if (b >= nbatch) return;

    // padding rows and columns stay zero for the whole launch
    for (int i = tid; i < KP * LDM; i += NT) {
        ys[i] = (CT)0;
        xs[i] = (CT)0;
    }

    // this wave's B fragments: k rows 4 kk .. 4 kk + 3, columns 16 nt .. 16 nt + 15 of Bk[s]
    CT bf[BLDS ? 1 : DP][BLDS ? 1 : KS];
    if constexpr (BLDS) {
        for (int i = tid; i < DP * KP * NP; i += NT) bs[i] = (CT)Bk[i];
    } else {
#pragma unroll
        for (int s = 0; s < DP; ++s)
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
                bf[s][kk] = (CT)Bk[((long long)s * KP + 4 * kk + q) * NP + 16 * nt + l16];
    }
    auto bfrag = [&](int s, int kk) -> CT {
        if constexpr (BLDS) return bs[(s * KP + 4 * kk + q) * NP + 16 * nt + l16];
        else return bf[s][kk];
    };

    // 32-bit offsets: the host guarantees npairs D^4 + 2^16 < 2^31
    const int ylim = npairs * R * R;
    double pre[NL];
    auto load = [&](int b) {
        const int base = b * NY;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + i * NT;
            pre[i] = (e < NY && base + e < ylim) ? Y[base + e] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + i * NT;
            if (e < NY) {
                const int p = e / (R * R), v = e % (R * R);
                const int uk = v / (D * R), ub = (v / R) % D, lk = (v / D) % D, lb = v % D;
                ys[(uk * D + lk) * LDM + p * R + ub * D + lb] = (CT)pre[i];
            }
        }
    };

    __syncthreads();
    load(b);
    store();
    while (true) {
        draw();
        __syncthreads();  // ys holds batch b; xs reads of the previous batch are done
        const int bn = next_batch;  // read before the next barrier; rewritten after it

        acc_t z[MTW];
#pragma unroll
        for (int i = 0; i < MTW; ++i) z[i] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < DP; ++s) {
            acc_t x[MTW];
#pragma unroll
            for (int i = 0; i < MTW; ++i) x[i] = acc_t{0, 0, 0, 0};
#pragma unroll KU
            for (int kk = 0; kk < KS; ++kk) {
                const CT* row = ys + (4 * kk + q) * LDM + 16 * mt0 + l16;
                const CT bv = bfrag(s, kk);
#pragma unroll
                for (int i = 0; i < MTW; ++i) x[i] = M::run(row[16 * i], bv, x[i]);
            }
            if (s > 0) __syncthreads();  // xs reads of the previous s are done
#pragma unroll
            for (int i = 0; i < MTW; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * (mt0 + i) + M::row(r, q), c = 16 * nt + l16;
                    if (m < P * R && c < R) xs[(m % R) * LDM + (m / R) * R + c] = x[i][r];
                }
            __syncthreads();  // xs complete; every wave is past its last read of ys
            if (s == DP - 1 && bn < nbatch) load(bn);
#pragma unroll KU
            for (int kk = 0; kk < KS; ++kk) {
                const CT* row = xs + (4 * kk + q) * LDM + 16 * mt0 + l16;
                const CT bv = bfrag(s, kk);
#pragma unroll
                for (int i = 0; i < MTW; ++i) z[i] = M::run(row[16 * i], bv, z[i]);
            }
        }

        const int n = 16 * nt + l16;
        if (n < R) {
            const double inv_chi = 1.0 / (double)chi;
            const int rb = n / D, db = n % D;
#pragma unroll
            for (int i = 0; i < MTW; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * (mt0 + i) + M::row(r, q);
                    if (m >= P * R) continue;
                    const int pg = b * P + m / R;
                    if (pg >= npairs) continue;
                    const int c = m % R, al = div_inv(pg, chi, inv_chi), f = pg - al * chi;
                    const int rk = c / D, dk = c % D;
                    Z[(al * R + rk * D + rb) * chi * R + f * R + dk * D + db] = (double)z[i][r];
                }
        }
        if (bn >= nbatch) break;
        store();
        b = bn;
    }
}

// ---------------------------------------------------------------------------
// FP64 forward at D = 6 with both physical indices in one ket product.
//   GEMM 1  x[(p u_b l_b)][(s r_k d_k)] = sum_{(u_k l_k)} ys[..] Bk[s][(u_k l_k)][(r_k d_k)]
//           M = 4 * 36 = 144 (9 row tiles, no padding), N = 72, K = 36
//   GEMM 2  z[(p r_k d_k)][(r_b d_b)] = sum_{(s u_b l_b)} xs[..] Bk[s][(u_b l_b)][(r_b d_b)]
//           M = 144, N = 36, K = 72 (the prepared Bk is this K x N operand as it stands)
// Columns that do not fill a 16-wide tile (GEMM 1: 64..71, GEMM 2: 32..35) go
// to v_mfma_f64_4x4x4f64, four 4 x 4 blocks per instruction.  Its block b takes
// A[4b + i][k] from lane 16k + 4b + i, which is the 16 x 16 x 4 A fragment as it
// stands, B[k][j] from lane 16k + 4b + j (here the same four columns for every
// block), and leaves D[4b + i][j] in lane 16i + 4b + j (lane layouts measured
// on gfx950).  Instead of 5 x 16 and 3 x 16 columns of 16-wide tiles that is
// 4 x 16 + 8 and 2 x 16 + 4, and M needs no padding: 729 16x16x4-equivalents
// per batch of four blocks in place of 1296 for five.
// GEMM 2 of batch b and GEMM 1 of batch b + 1 run between the same two
// barriers (x waits in registers while GEMM 2 reads the previous x from xs), so
// each wave's share of the phase balances across both products.  Waves come in
// three groups of four; group g holds row tiles 3g .. 3g + 2.  In GEMM 1 wave c
// of a group takes column tile c of the group's rows; in GEMM 2 waves 0-2 take
// two of the group's six (row tile, column tile) pairs each, and wave 3 takes
// the narrow columns of both products.
// ---------------------------------------------------------------------------
namespace es6 {
constexpr int D = 6, R = 36, P = 4, M = P * R, LDM = M, NT = 768, NY = P * R * R;
constexpr int NL = (NY + NT - 1) / NT;
constexpr int NPB = 48;  // columns of the prepared Bk
}  // namespace es6

__global__ __launch_bounds__(es6::NT) __attribute__((amdgpu_waves_per_eu(3))) void edge_split6_kernel(
    const double* __restrict__ Y, const double* __restrict__ Bk, int chi, int npairs,
    double* __restrict__ Z, unsigned* ticket) {
    using namespace es6;
    __shared__ double ys[R * LDM];       // ys[(u_k l_k)][(p u_b l_b)]
    __shared__ double xs[2 * R * LDM];   // xs[(s u_b l_b)][(p r_k d_k)]
    __shared__ double bs[2 * R * NPB];   // Bk[(s k)][n]
    __shared__ int tk[2];

    const int tid = threadIdx.x;
    const int lane = tid & 63, q = lane >> 4, l16 = lane & 15;
    const int w = tid >> 6, c = w & 3, g = w >> 2;
    // 4x4x4 lane roles: block row 4 bq + q of the tile, column j4
    const int bq = (lane >> 2) & 3, j4 = lane & 3;
    const int nbatch = (npairs + P - 1) / P;
    // one ticket per batch, plus one that ends each workgroup: nbatch + gridDim.x in all
    auto draw = [&](int slot) {
        if (tid == 0) {
            const unsigned t = atomicAdd(ticket, 1u);
            if (t == (unsigned)(nbatch + gridDim.x - 1)) atomicExch(ticket, 0u);
            tk[slot] = (int)min(t, (unsigned)nbatch);
        }
    };
    draw(0);
    __syncthreads();
    const int b0 = tk[0];
    if (b0 >= nbatch) return;

    for (int i = tid; i < 2 * R * NPB; i += NT) bs[i] = Bk[i];

    // 32-bit offsets: the host guarantees npairs D^4 + 2^16 < 2^31
    const int ylim = npairs * R * R;
    double pre[NL];
    auto load = [&](int b) {
        const int base = b * NY;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + i * NT;
            pre[i] = (e < NY && base + e < ylim) ? Y[base + e] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + i * NT;
            if (e < NY) {
                const int p = e / (R * R), v = e % (R * R);
                const int uk = v / (D * R), ub = (v / R) % D, lk = (v / D) % D, lb = v % D;
                ys[(uk * D + lk) * LDM + p * R + ub * D + lb] = pre[i];
            }
        }
    };

    // GEMM 1 operands of this lane: B column 16 c + l16 of the stacked x columns (s r_k d_k)
    const int col1 = 16 * c + l16;
    const int boff1 = (col1 / R) * R * NPB + col1 % R;
    const int rt0 = 3 * g;  // first row tile of the group
    dbl4 x1[3];
    double xr[3][2];  // wave 3: columns 64 + 4 cb + j4
    auto gemm1 = [&]() {
#pragma unroll
        for (int i = 0; i < 3; ++i) x1[i] = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 3; ++i) xr[i][0] = xr[i][1] = 0.0;
        if (c < 3) {
#pragma unroll 3
            for (int kk = 0; kk < R / 4; ++kk) {
                const double* a = ys + (4 * kk + q) * LDM + 16 * rt0 + l16;
                const double bv = bs[boff1 + (4 * kk + q) * NPB];
#pragma unroll
                for (int i = 0; i < 3; ++i) x1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[16 * i], bv, x1[i], 0, 0, 0);
            }
        } else {
#pragma unroll 3
            for (int kk = 0; kk < R / 4; ++kk) {
                const double* a = ys + (4 * kk + q) * LDM + 16 * rt0 + l16;
                const double bv = bs[boff1 + (4 * kk + q) * NPB];
                const double* br = bs + (R + 4 * kk + q) * NPB + 28 + j4;
                const double b0v = br[0], b1v = br[4];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double av = a[16 * i];
                    x1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, x1[i], 0, 0, 0);
                    xr[i][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b0v, xr[i][0], 0, 0, 0);
                    xr[i][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b1v, xr[i][1], 0, 0, 0);
                }
            }
        }
    };
    // x[m][cc] -> xs[(cc / 36) 36 + m % 36][(m / 36) 36 + cc % 36]
    auto put_x = [&]() {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 16 * (rt0 + i) + 4 * r + q;
                xs[((col1 / R) * R + m % R) * LDM + (m / R) * R + col1 % R] = x1[i][r];
            }
        if (c == 3) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int m = 16 * (rt0 + i) + 4 * bq + q, cc = 64 + 4 * cb + j4;
                    xs[(R + m % R) * LDM + (m / R) * R + cc - R] = xr[i][cb];
                }
        }
    };

    // GEMM 2 pairs of waves 0-2: pair j = 2 c + h has row tile rt0 + j % 3 and column tile j / 3
    int rt2[2], ct2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = 2 * c + h;
        rt2[h] = rt0 + j % 3;
        ct2[h] = j / 3;
    }
    dbl4 z2[2];
    double zr[3];  // wave 3: columns 32 + j4
    auto gemm2 = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) z2[h] = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 3; ++i) zr[i] = 0.0;
        if (c < 3) {
#pragma unroll 3
            for (int kk = 0; kk < 2 * R / 4; ++kk) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double av = xs[(4 * kk + q) * LDM + 16 * rt2[h] + l16];
                    const double bv = bs[(4 * kk + q) * NPB + 16 * ct2[h] + l16];
                    z2[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, z2[h], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 3
            for (int kk = 0; kk < 2 * R / 4; ++kk) {
                const double* a = xs + (4 * kk + q) * LDM + 16 * rt0 + l16;
                const double bv = bs[(4 * kk + q) * NPB + 32 + j4];
#pragma unroll
                for (int i = 0; i < 3; ++i) zr[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[16 * i], bv, zr[i], 0, 0, 0);
            }
        }
    };
    const double inv_chi = 1.0 / (double)chi;
    // z[n2][n] of batch b: n2 = (p r_k d_k), n = (r_b d_b)
    auto put_z = [&](int b, int n2, int n, double v) {
        const int pg = b * P + n2 / R;
        if (pg >= npairs) return;
        const int cc = n2 % R, al = div_inv(pg, chi, inv_chi), f = pg - al * chi;
        const int rk = cc / D, dk = cc % D, rb = n / D, db = n % D;
        Z[(al * R + rk * D + rb) * chi * R + f * R + dk * D + db] = v;
    };
    auto store_z = [&](int b) {
        if (c < 3) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r) put_z(b, 16 * rt2[h] + 4 * r + q, 16 * ct2[h] + l16, z2[h][r]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) put_z(b, 16 * (rt0 + i) + 4 * bq + q, 32 + j4, zr[i]);
        }
    };

    // prologue: batch b0 through GEMM 1, its x in xs, the next batch's Y in ys
    load(b0);
    store();
    draw(1);
    __syncthreads();
    int nxt = tk[1];
    if (nxt < nbatch) load(nxt);
    gemm1();
    __syncthreads();
    put_x();
    if (nxt < nbatch) {
        store();
        draw(0);
    }
    __syncthreads();
    int cur_x = b0, cur_y = nxt, slot = 0;
    while (true) {
        nxt = cur_y < nbatch ? tk[slot] : nbatch;
        if (nxt < nbatch) load(nxt);
        gemm2();
        if (cur_y < nbatch) gemm1();
        __syncthreads();  // every read of xs and ys in this phase is done
        store_z(cur_x);
        if (cur_y >= nbatch) break;
        put_x();
        if (nxt < nbatch) {
            store();
            draw(slot ^ 1);
        }
        __syncthreads();
        cur_x = cur_y;
        cur_y = nxt;
        slot ^= 1;
    }
}

// Bk[s][k][n] = As[s][u][l][dd][r] (k = u D + l, n = r D + dd) and, after it,
// BkT[s][k][n] = Bk[s][n][k], both [d][KP][NP] and zero outside k, n < D^2;
// then the ticket counters.
__global__ void edge_split_prepare_kernel(const double* __restrict__ As, int d, int D, int KP,
                                          int NP, double* Bk) {
    const int R = D * D, n = d * KP * NP;
    if (blockIdx.x == 0 && threadIdx.x < kTickets)
        reinterpret_cast<unsigned*>(Bk + 2 * n)[threadIdx.x] = 0u;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int s = e / (KP * NP), k = (e / NP) % KP, c = e % NP;
        const double* A = As + (long long)s * R * R;
        Bk[e] = (k < R && c < R) ? A[k * R + (c % D) * D + c / D] : 0.0;
        Bk[n + e] = (k < R && c < R) ? A[c * R + (k % D) * D + k / D] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Reverse of 3b in the split form.  With Zb the cotangent of Z, per (al, f)
// block and per s (X_s as in the forward pass):
//   Xb_s[(r_k d_k)][(u_b l_b)] = sum_{(r_b d_b)} Zb[(r_k r_b)][(d_k d_b)] Bk[s][(u_b l_b)][(r_b d_b)]
//   Yb[(u_k u_b)][(l_k l_b)]  += sum_{(r_k d_k)} Xb_s[(r_k d_k)][(u_b l_b)] Bk[s][(u_k l_k)][(r_k d_k)]
//   Bkb[s] (bra) += sum_{blocks, (r_k d_k)} X_s[(u_b l_b)][(r_k d_k)] Zb[(r_k r_b)][(d_k d_b)]
//   Bkb[s] (ket) += sum_{blocks, (u_b l_b)} Y[(u_k u_b)][(l_k l_b)] Xb_s[(r_k d_k)][(u_b l_b)]
// in one kernel: Y and Zb staged in LDS (transposed), X_s and Xb_s computed
// into LDS, Yb accumulated over s in registers and written once, the Bkb
// sums accumulated over the workgroup's batches in registers and written
// per workgroup; a second kernel adds the workgroups' sums into the site
// tensor's cotangent.  Per batch and s: five M x N x K products on
// v_mfma_f64_16x16x4f64, the last two with K over the batch's blocks.  The
// LDS row length is odd so that those two read columns conflict-free.
// ---------------------------------------------------------------------------
constexpr int kBwPairs[9] = {0, 80, 20, 8, 5, 3, 2, 1, 1};

// x returned through an empty asm statement: index arithmetic on it is redone
// where it is used instead of being hoisted out of the batch loop into
// registers (which the accumulators need)
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
constexpr int kBwGroups[9] = {0, 5, 5, 5, 5, 5, 5, 4, 4};
constexpr int kBwWavesPerSimd[9] = {0, 2, 2, 2, 2, 2, 4, 4, 4};
constexpr int kBwMaxGrid = 512;

template <int D>
struct ShapeBw {
    static constexpr int R = D * D;
    static constexpr int KP = (R + 3) / 4 * 4;
    static constexpr int NP = (R + 15) / 16 * 16;
    static constexpr int NB = NP / 16;
    static constexpr int P = kBwPairs[D];
    static constexpr int MP = (P * R + 15) / 16 * 16;
    static constexpr int MT = MP / 16;
    static constexpr int G = kBwGroups[D];
    static constexpr int MTW = MT / G;
    static constexpr int W = NB * G;                  // waves
    static constexpr int NT = W * 64;
    static constexpr int LDM = MP + 1;                // odd row length
    static constexpr int NY = P * R * R;
    static constexpr int NL = (NY + NT - 1) / NT;
    static constexpr int TS = 2 * NB * NB;            // Bkb tiles per s (bra, ket)
    static constexpr int TPW = (TS + W - 1) / W;      // ... per wave
    static constexpr int WPE = kBwWavesPerSimd[D];
    // k steps unrolled per iteration; at D >= 7 none, so that the B fragment
    // loads are not hoisted into registers the accumulators need
    static constexpr int KU = D >= 7 ? 1 : 3;
    static constexpr int KU2 = D >= 7 ? 1 : 2;
    static_assert(MT % G == 0, "row tiles split evenly over the groups");
};

template <int D>
__global__ __launch_bounds__(ShapeBw<D>::NT)
__attribute__((amdgpu_waves_per_eu(ShapeBw<D>::WPE))) void edge_split_bw_kernel(
    const double* __restrict__ Y, const double* __restrict__ Zb, const double* __restrict__ Bk,
    const double* __restrict__ BkT, int npairs, double* __restrict__ Yb,
    double* __restrict__ part, unsigned* ticket) {
    using S = ShapeBw<D>;
    constexpr int R = S::R, KP = S::KP, NP = S::NP, NB = S::NB, P = S::P, MP = S::MP;
    constexpr int MTW = S::MTW, W = S::W, NT = S::NT, LDM = S::LDM, NY = S::NY, NL = S::NL;
    constexpr int KS = KP / 4, TS = S::TS, TPW = S::TPW;
    constexpr int DP = 2;
    __shared__ double ys[NP * LDM];   // ys[(u_k l_k)][(p u_b l_b)]
    __shared__ double zs[NP * LDM];   // zs[(r_b d_b)][(p r_k d_k)]
    __shared__ double xs[NP * LDM];   // xs[(u_b l_b)][(p r_k d_k)]   X_s
    __shared__ double xbs[NP * LDM];  // xbs[(r_k d_k)][(p u_b l_b)]  Xb_s
    __shared__ int next_batch;

    const int tid = threadIdx.x;
    const int lane = tid & 63, q = lane >> 4, l16 = lane & 15;
    const int w = tid >> 6;
    const int nt = w % NB, mt0 = (w / NB) * MTW;
    const int nbatch = (npairs + P - 1) / P;
    auto draw = [&]() {
        if (tid == 0) {
            const unsigned t = atomicAdd(ticket, 1u);
            if (t == (unsigned)(nbatch + gridDim.x - 1)) atomicExch(ticket, 0u);
            next_batch = (int)min(t, (unsigned)nbatch);
        }
    };

    for (int i = tid; i < NP * LDM; i += NT) {
        ys[i] = 0.0;
        zs[i] = 0.0;
        xs[i] = 0.0;
        xbs[i] = 0.0;
    }
    dbl4 ab[DP][TPW];
#pragma unroll
    for (int s = 0; s < DP; ++s)
#pragma unroll
        for (int t = 0; t < TPW; ++t) ab[s][t] = dbl4{0.0, 0.0, 0.0, 0.0};

    // 32-bit offsets: the host guarantees npairs D^4 + 2^16 < 2^31
    const int ylim = npairs * R * R;
    double py[NL], pz[NL];
    auto load = [&](int b) {
        const int base = b * NY;
        const int tv = opaque(tid);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tv + i * NT;
            const bool in = e < NY && base + e < ylim;
            py[i] = in ? Y[base + e] : 0.0;
            pz[i] = in ? Zb[base + e] : 0.0;
        }
    };
    // block digits v = ((a0 D + a1) D + a2) D + a3: Y [u_k][u_b][l_k][l_b],
    // Zb [r_k][r_b][d_k][d_b]
    auto store = [&]() {
        const int tv = opaque(tid);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tv + i * NT;
            if (e < NY) {
                const int p = e / (R * R), v = e % (R * R);
                const int a0 = v / (D * R), a1 = (v / R) % D, a2 = (v / D) % D, a3 = v % D;
                ys[(a0 * D + a2) * LDM + p * R + a1 * D + a3] = py[i];
                zs[(a1 * D + a3) * LDM + p * R + a0 * D + a2] = pz[i];
            }
        }
    };

    draw();
    __syncthreads();
    int b = next_batch;
    if (b < nbatch) {
        load(b);
        store();
        while (true) {
            draw();
            __syncthreads();  // ys, zs hold batch b
            const int bn = next_batch;
            dbl4 yb[MTW];
#pragma unroll
            for (int i = 0; i < MTW; ++i) yb[i] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < DP; ++s) {
                // B fragments (rows 4 kk + q, this wave's 16 columns) of Bk[s] and BkT[s]
                const double* B1 = Bk + (s * KP + q) * NP + 16 * nt + l16;
                const double* B2 = BkT + (s * KP + q) * NP + 16 * nt + l16;
                dbl4 x[MTW], xb[MTW];
#pragma unroll
                for (int i = 0; i < MTW; ++i) {
                    x[i] = dbl4{0.0, 0.0, 0.0, 0.0};
                    xb[i] = dbl4{0.0, 0.0, 0.0, 0.0};
                }
#pragma unroll S::KU
                for (int kk = 0; kk < KS; ++kk) {
                    const int o = (4 * kk + q) * LDM + 16 * mt0 + l16;
                    const double b1 = B1[4 * kk * NP], b2 = B2[4 * kk * NP];
#pragma unroll
                    for (int i = 0; i < MTW; ++i) {
                        x[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ys[o + 16 * i], b1, x[i], 0, 0, 0);
                        xb[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(zs[o + 16 * i], b2, xb[i], 0, 0, 0);
                    }
                }
                if (s > 0) __syncthreads();  // reads of xs, xbs for the previous s are done
#pragma unroll
                for (int i = 0; i < MTW; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = 16 * (mt0 + i) + 4 * r + q, c = 16 * nt + l16;
                        if (m < P * R && c < R) {
                            const int o = (m % R) * LDM + (m / R) * R + c;
                            xs[o] = x[i][r];
                            xbs[o] = xb[i][r];
                        }
                    }
                __syncthreads();  // xs, xbs complete
                if (s == DP - 1 && bn < nbatch) load(bn);
                // Yb += Xb_s^T-contract Bk[s] (B fragments of BkT[s], as for Xb_s)
#pragma unroll S::KU
                for (int kk = 0; kk < KS; ++kk) {
                    const int o = (4 * kk + q) * LDM + 16 * mt0 + l16;
                    const double b2 = B2[4 * kk * NP];
#pragma unroll
                    for (int i = 0; i < MTW; ++i)
                        yb[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(xbs[o + 16 * i], b2, yb[i], 0, 0, 0);
                }
                // Bkb[s] tiles: bra (xs, zs) and ket (ys, xbs), K over the batch
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int u = w + W * t;
                    if (u < TS) {
                        const int kind = u / (NB * NB), it = (u % (NB * NB)) / NB, jt = u % NB;
                        const double* As_ = kind ? ys : xs;
                        const double* Bs_ = kind ? xbs : zs;
                        const int oa = (16 * it + l16) * LDM + q, ob = (16 * jt + l16) * LDM + q;
                        if constexpr (D <= 6) {
                            // the K sum in two chains (even and odd k steps), so that
                            // consecutive matrix-core steps do not wait for each other
                            dbl4 a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll S::KU2
                            for (int kk = 0; kk < MP / 4; kk += 2) {
                                ab[s][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                    As_[oa + 4 * kk], Bs_[ob + 4 * kk], ab[s][t], 0, 0, 0);
                                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(As_[oa + 4 * kk + 4],
                                                                         Bs_[ob + 4 * kk + 4], a1, 0,
                                                                         0, 0);
                            }
#pragma unroll
                            for (int r = 0; r < 4; ++r) ab[s][t][r] += a1[r];
                        } else {
#pragma unroll S::KU2
                            for (int kk = 0; kk < MP / 4; ++kk)
                                ab[s][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                    As_[oa + 4 * kk], Bs_[ob + 4 * kk], ab[s][t], 0, 0, 0);
                        }
                    }
                }
            }
            // Yb[(u_k u_b)][block][(l_k l_b)], rows (p u_b l_b), columns (u_k l_k)
            const int lv = opaque(lane);
            const int n = 16 * nt + (lv & 15);
            if (n < R) {
                const int uk = n / D, lk = n % D;
#pragma unroll
                for (int i = 0; i < MTW; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = 16 * (mt0 + i) + 4 * r + (lv >> 4);
                        if (m >= P * R) continue;
                        const int pg = b * P + m / R;
                        if (pg >= npairs) continue;
                        const int c = m % R, ub = c / D, lb = c % D;
                        Yb[((uk * D + ub) * npairs + pg) * R + lk * D + lb] = yb[i][r];
                    }
            }
            if (bn >= nbatch) break;
            __syncthreads();  // every read of ys, zs for batch b is done
            store();
            b = bn;
        }
    }
    // this workgroup's sums: part[wg][kind][s][NP][NP]
#pragma unroll
    for (int s = 0; s < DP; ++s)
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int u = w + W * t;
            if (u < TS) {
                const int kind = u / (NB * NB), it = (u % (NB * NB)) / NB, jt = u % NB;
                double* o = part + ((size_t)(blockIdx.x * 2 + kind) * DP + s) * NP * NP;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[(16 * it + 4 * r + q) * NP + 16 * jt + l16] = ab[s][t][r];
            }
        }
}

// Asb[s][u][l][dd][r] += sum over workgroups and both kinds of part[..][s][u D + l][r D + dd]:
// a block per 32 outputs, its 8 thread rows each summing a share of the partials
constexpr int kRedOut = 32, kRedRows = 8;
__global__ __launch_bounds__(kRedOut * kRedRows) void edge_split_bw_reduce_kernel(
    const double* __restrict__ part, int nwg, int d, int D, int NP, double* Asb) {
    __shared__ double acc_s[kRedRows][kRedOut];
    const int R = D * D, n = d * R * R;
    const int lo = threadIdx.x % kRedOut, row = threadIdx.x / kRedOut;
    const int e = blockIdx.x * kRedOut + lo;
    double acc = 0.0;
    if (e < n) {
        const int s = e / (R * R), v = e % (R * R);
        const int k = v / R, r = v % D, dd = (v / D) % D;
        const size_t o = (size_t)k * NP + r * D + dd;
        for (int g = row; g < 2 * nwg; g += kRedRows) acc += part[((size_t)g * d + s) * NP * NP + o];
    }
    acc_s[row][lo] = acc;
    __syncthreads();
    if (row == 0 && e < n) {
        double t = 0.0;
        for (int q = 0; q < kRedRows; ++q) t += acc_s[q][lo];
        Asb[e] += t;
    }
}

template <int D>
Status launch_3b_bw(const double* Y, const double* Zb, const double* Bk, const double* BkT,
                    unsigned* ticket, int npairs, double* Yb, double* part, size_t part_doubles,
                    double* Asb, hipStream_t st) {
    using S = ShapeBw<D>;
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        QRCTM_HIP(hipGetDevice(&dev));
        QRCTM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edge_split_bw_kernel<D>,
                                                               S::NT, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const long long nbatch = ceil_div(npairs, S::P);
    long long grid = std::min<long long>(nbatch, (long long)per_cu * cus);
    grid = std::min<long long>(grid, kBwMaxGrid);
    Status s;
    if ((size_t)grid * 4 * S::NP * S::NP > part_doubles) {
        s.code = -2;
        s.msg = "edge_split_3b_backward: partial-sum scratch too small";
        return s;
    }
    hipLaunchKernelGGL(edge_split_bw_kernel<D>, dim3((int)grid), dim3(S::NT), 0, st, Y, Zb, Bk, BkT,
                       npairs, Yb, part, ticket);
    QRCTM_TRY(launch_check("edge_split_bw_kernel"));
    const int nout = 2 * S::R * S::R;
    hipLaunchKernelGGL(edge_split_bw_reduce_kernel, dim3((nout + kRedOut - 1) / kRedOut),
                       dim3(kRedOut * kRedRows), 0, st, part, (int)grid, 2, D, S::NP, Asb);
    return launch_check("edge_split_bw_reduce_kernel");
}

Status launch_3b6(const double* Y, const double* Bk, unsigned* ticket, int chi, int npairs,
                  double* Z, hipStream_t st) {
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        QRCTM_HIP(hipGetDevice(&dev));
        QRCTM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edge_split6_kernel, es6::NT, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const long long nbatch = ceil_div(npairs, es6::P);
    const int grid = (int)std::min<long long>(nbatch, (long long)per_cu * cus);
    hipLaunchKernelGGL(edge_split6_kernel, dim3(grid), dim3(es6::NT), 0, st, Y, Bk, chi, npairs, Z,
                       ticket);
    return launch_check("edge_split6_kernel");
}

template <class CT, int D>
Status launch_3b_t(const double* Y, const double* Bk, unsigned* ticket, int chi, int npairs,
                   double* Z, hipStream_t st) {
    if constexpr (D == 6 && sizeof(CT) == 8) return launch_3b6(Y, Bk, ticket, chi, npairs, Z, st);
    using S = Shape3b<D>;
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        QRCTM_HIP(hipGetDevice(&dev));
        QRCTM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edge_split_kernel<CT, D, 2>,
                                                               S::NT, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const long long nbatch = ceil_div(npairs, S::P);
    const int grid = (int)std::min<long long>(nbatch, (long long)per_cu * cus);
    hipLaunchKernelGGL((edge_split_kernel<CT, D, 2>), dim3(grid), dim3(S::NT), 0, st, Y, Bk, chi,
                       npairs, Z, ticket);
    return launch_check("edge_split_kernel");
}
template <int D>
Status launch_3b(const double* Y, const double* Bk, unsigned* ticket, int chi, int npairs,
                 double* Z, bool fp32, hipStream_t st) {
    return fp32 ? launch_3b_t<float, D>(Y, Bk, ticket, chi, npairs, Z, st)
                : launch_3b_t<double, D>(Y, Bk, ticket, chi, npairs, Z, st);
}

int kp_of(int D) { return (D * D + 3) / 4 * 4; }
int np_of(int D) { return (D * D + 15) / 16 * 16; }

}  // namespace

bool edge_split_supported(int d, int D) { return d == 2 && D >= 1 && D <= 8; }

size_t edge_split_operand_size(int d, int D) {
    return edge_split_supported(d, D) ? 2 * (size_t)d * kp_of(D) * np_of(D) + kTickets / 2 : 0;
}

bool edge_split_bw_supported(int d, int D) { return edge_split_supported(d, D); }

size_t edge_split_bw_part_size(int d, int D) {
    return edge_split_bw_supported(d, D) ? (size_t)kBwMaxGrid * 2 * d * np_of(D) * np_of(D) : 0;
}

Status edge_split_prepare(const double* As, int d, int D, double* Bk, hipStream_t st) {
    Status s;
    if (!edge_split_supported(d, D)) {
        s.code = -1;
        s.msg = "edge_split_prepare: unsupported (d, D)";
        return s;
    }
    hipLaunchKernelGGL(edge_split_prepare_kernel, dim3(16), dim3(256), 0, st, As, d, D, kp_of(D),
                       np_of(D), Bk);
    return launch_check("edge_split_prepare_kernel");
}

Status edge_split_3b(const double* Y, double* Bk, int d, int D, int chi, int chio, double* Z,
                     hipStream_t st, bool fp32) {
    Status s;
    if (!edge_split_supported(d, D) || chi < 0 || chio < 0 ||
        (long long)chi * chio * D * D * D * D + (1LL << 16) >= (1LL << 31)) {
        s.code = -1;
        s.msg = "edge_split_3b: unsupported shape";
        return s;
    }
    const int npairs = chi * chio;
    if (npairs == 0) return s;
    unsigned* tk = reinterpret_cast<unsigned*>(Bk + 2 * (size_t)d * kp_of(D) * np_of(D));
    switch (D) {
        case 1: return launch_3b<1>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 2: return launch_3b<2>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 3: return launch_3b<3>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 4: return launch_3b<4>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 5: return launch_3b<5>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 6: return launch_3b<6>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        case 7: return launch_3b<7>(Y, Bk, tk, chi, npairs, Z, fp32, st);
        default: return launch_3b<8>(Y, Bk, tk, chi, npairs, Z, fp32, st);
    }
}


Status edge_split_3b_backward(const double* Y, const double* Zb, double* Bk, int d, int D, int chi,
                              int chio, double* Yb, double* part, size_t part_doubles, double* Asb,
                              hipStream_t st) {
    Status s;
    if (!edge_split_bw_supported(d, D) || chi < 0 || chio < 0 ||
        (long long)chi * chio * D * D * D * D + (1LL << 16) >= (1LL << 31)) {
        s.code = -1;
        s.msg = "edge_split_3b_backward: unsupported shape";
        return s;
    }
    const int npairs = chi * chio;
    if (npairs == 0) return s;
    const size_t n = (size_t)d * kp_of(D) * np_of(D);
    const double* BkT = Bk + n;
    unsigned* tk = reinterpret_cast<unsigned*>(Bk + 2 * n) + 1;
    switch (D) {
        case 1: return launch_3b_bw<1>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 2: return launch_3b_bw<2>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 3: return launch_3b_bw<3>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 4: return launch_3b_bw<4>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 5: return launch_3b_bw<5>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 6: return launch_3b_bw<6>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        case 7: return launch_3b_bw<7>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
        default: return launch_3b_bw<8>(Y, Zb, Bk, BkT, tk, npairs, Yb, part, part_doubles, Asb, st);
    }
}

}  // namespace qrctm
