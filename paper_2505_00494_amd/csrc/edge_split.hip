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

template <int D, int DP>
__global__ __launch_bounds__(Shape3b<D>::NT)
__attribute__((amdgpu_waves_per_eu(Shape3b<D>::WPE))) void edge_split_kernel(
    const double* __restrict__ Y, const double* __restrict__ Bk, int chi, int npairs,
    double* __restrict__ Z, unsigned* ticket) {
    using S = Shape3b<D>;
    constexpr int R = S::R, KP = S::KP, NP = S::NP, NB = S::NB, P = S::P, MTW = S::MTW;
    constexpr int LDM = S::LDM, NT = S::NT, NY = S::NY, NL = S::NL, KS = KP / 4;
    __shared__ double ys[KP * LDM];  // ys[(u_k l_k)][(p u_b l_b)]
    __shared__ double xs[KP * LDM];  // xs[(u_b l_b)][(p r_k d_k)]
    __shared__ int next_batch;
    __shared__ double bs[S::NBS];    // Bk (when S::BLDS)
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
        ys[i] = 0.0;
        xs[i] = 0.0;
    }

    // this wave's B fragments: k rows 4 kk .. 4 kk + 3, columns 16 nt .. 16 nt + 15 of Bk[s]
    double bf[BLDS ? 1 : DP][BLDS ? 1 : KS];
    if constexpr (BLDS) {
        for (int i = tid; i < DP * KP * NP; i += NT) bs[i] = Bk[i];
    } else {
#pragma unroll
        for (int s = 0; s < DP; ++s)
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
                bf[s][kk] = Bk[((long long)s * KP + 4 * kk + q) * NP + 16 * nt + l16];
    }
    auto bfrag = [&](int s, int kk) -> double {
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
                ys[(uk * D + lk) * LDM + p * R + ub * D + lb] = pre[i];
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

        dbl4 z[MTW];
#pragma unroll
        for (int i = 0; i < MTW; ++i) z[i] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < DP; ++s) {
            dbl4 x[MTW];
#pragma unroll
            for (int i = 0; i < MTW; ++i) x[i] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll KU
            for (int kk = 0; kk < KS; ++kk) {
                const double* row = ys + (4 * kk + q) * LDM + 16 * mt0 + l16;
                const double bv = bfrag(s, kk);
#pragma unroll
                for (int i = 0; i < MTW; ++i)
                    x[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * i], bv, x[i], 0, 0, 0);
            }
            if (s > 0) __syncthreads();  // xs reads of the previous s are done
#pragma unroll
            for (int i = 0; i < MTW; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * (mt0 + i) + 4 * r + q, c = 16 * nt + l16;
                    if (m < P * R && c < R) xs[(m % R) * LDM + (m / R) * R + c] = x[i][r];
                }
            __syncthreads();  // xs complete; every wave is past its last read of ys
            if (s == DP - 1 && bn < nbatch) load(bn);
#pragma unroll KU
            for (int kk = 0; kk < KS; ++kk) {
                const double* row = xs + (4 * kk + q) * LDM + 16 * mt0 + l16;
                const double bv = bfrag(s, kk);
#pragma unroll
                for (int i = 0; i < MTW; ++i)
                    z[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * i], bv, z[i], 0, 0, 0);
            }
        }

        const int n = 16 * nt + l16;
        if (n < R) {
            const int rb = n / D, db = n % D;
#pragma unroll
            for (int i = 0; i < MTW; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * (mt0 + i) + 4 * r + q;
                    if (m >= P * R) continue;
                    const int pg = b * P + m / R;
                    if (pg >= npairs) continue;
                    const int c = m % R, al = pg / chi, f = pg - al * chi;
                    const int rk = c / D, dk = c % D;
                    Z[(al * R + rk * D + rb) * chi * R + f * R + dk * D + db] = z[i][r];
                }
        }
        if (bn >= nbatch) break;
        store();
        b = bn;
    }
}

__global__ void edge_split_prepare_kernel(const double* __restrict__ As, int d, int D, int KP,
                                          int NP, double* Bk) {
    const int R = D * D, n = d * KP * NP;
    // ticket counters after the operand
    if (blockIdx.x == 0 && threadIdx.x < kTickets) reinterpret_cast<unsigned*>(Bk + n)[threadIdx.x] = 0u;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int s = e / (KP * NP), k = (e / NP) % KP, c = e % NP;
        Bk[e] = (k < R && c < R) ? As[(long long)s * R * R + k * R + (c % D) * D + c / D] : 0.0;
    }
}

template <int D>
Status launch_3b(const double* Y, const double* Bk, unsigned* ticket, int chi, int npairs,
                 double* Z, hipStream_t st) {
    using S = Shape3b<D>;
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        QRCTM_HIP(hipGetDevice(&dev));
        QRCTM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edge_split_kernel<D, 2>,
                                                               S::NT, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const long long nbatch = ceil_div(npairs, S::P);
    const int grid = (int)std::min<long long>(nbatch, (long long)per_cu * cus);
    hipLaunchKernelGGL((edge_split_kernel<D, 2>), dim3(grid), dim3(S::NT), 0, st, Y, Bk, chi,
                       npairs, Z, ticket);
    return launch_check("edge_split_kernel");
}

int kp_of(int D) { return (D * D + 3) / 4 * 4; }
int np_of(int D) { return (D * D + 15) / 16 * 16; }

}  // namespace

bool edge_split_supported(int d, int D) { return d == 2 && D >= 1 && D <= 8; }

size_t edge_split_operand_size(int d, int D) {
    return edge_split_supported(d, D) ? (size_t)d * kp_of(D) * np_of(D) + kTickets / 2 : 0;
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
                     hipStream_t st) {
    Status s;
    if (!edge_split_supported(d, D) || chi < 0 || chio < 0 ||
        (long long)chi * chio * D * D * D * D + (1LL << 16) >= (1LL << 31)) {
        s.code = -1;
        s.msg = "edge_split_3b: unsupported shape";
        return s;
    }
    const int npairs = chi * chio;
    if (npairs == 0) return s;
    unsigned* tk = reinterpret_cast<unsigned*>(Bk + (size_t)d * kp_of(D) * np_of(D));
    switch (D) {
        case 1: return launch_3b<1>(Y, Bk, tk, chi, npairs, Z, st);
        case 2: return launch_3b<2>(Y, Bk, tk, chi, npairs, Z, st);
        case 3: return launch_3b<3>(Y, Bk, tk, chi, npairs, Z, st);
        case 4: return launch_3b<4>(Y, Bk, tk, chi, npairs, Z, st);
        case 5: return launch_3b<5>(Y, Bk, tk, chi, npairs, Z, st);
        case 6: return launch_3b<6>(Y, Bk, tk, chi, npairs, Z, st);
        case 7: return launch_3b<7>(Y, Bk, tk, chi, npairs, Z, st);
        default: return launch_3b<8>(Y, Bk, tk, chi, npairs, Z, st);
    }
}

}  // namespace qrctm
