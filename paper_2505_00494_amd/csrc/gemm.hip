// GEMM on the CDNA4 matrix cores, gfx950: FP64 (v_mfma_f64_16x16x4_f64) or, for
// the mixed-precision form, FP32 products with FP32 accumulation
// (v_mfma_f32_16x16x4_f32) on FP64 operands converted while they are staged.
//
// Every contraction of the QR-CTMRG step is one call of this kernel: the index
// permutations of the tensor network are absorbed into the operand strides
// (row- or column-major A and B) and into a two-level output map, so no tensor
// is ever transposed in memory.
//
// Tiling: a workgroup computes a BM x BN tile of C with (BM/WM) x (BN/WN) waves;
// each wave owns a WM x WN sub-tile held in (WM/16) x (WN/16) MFMA accumulators.
// K advances in slabs of BK staged through LDS (double buffered, one barrier per
// slab).  LDS holds each row of A and each column of B k-contiguous (row stride
// BK plus 16 bytes), and within a slab quarter-wave q of the MFMA's k slots
// takes the k range [q BK/4, (q+1) BK/4): every lane fetches all of its
// operand values for the slab with 16-byte reads, and the 16 lanes of a
// quarter-wave (16 rows, stride BK * size + 16 bytes) hit distinct banks.
//
// The one exception: a plain FP64 product (row-major C, no gate, no split
// planes) of at least kVendorMinFlop with at least kVendorMinTiles output
// tiles goes to the vendor BLAS (rocBLAS dgemm, atomics off, so the result is
// reproducible) unless its caller keeps it here (GemmDesc::vendor).  On the step's shapes it runs at
// 0.83-0.94 of the FP64 peak at chi D^2 = 16384 where these kernels reach
// 0.55-0.58; below that size they are as fast or the persistent grid of the
// kernel above wins beside the corner spectrum.
#include "common.h"

#include <rocblas/rocblas.h>

#include <mutex>

#ifndef MMA_F32_ROW
#define MMA_F32_ROW(r, q) (4 * (q) + (r))
#endif

namespace qrctm {
namespace {

struct KArgs {
    long long M, N, K;
    const double* A;
    long long lda;
    const double* B;
    long long ldb;
    double* C;
    OutMap map;
    double alpha, beta;
    long long kchunk;  // K range per split (split index = blockIdx.y)
    int tiles_m, tiles_n;
    int partial;       // 1: write raw sums to C + split*M*N (plain M x N)
    unsigned short* C16;  // non-null: the result split into three bf16 planes,
    long long pC16;       // plane s at C16[s pC16 + map(m, n)] (alpha only)
    const int* gate;      // non-null: skip unless *gate == 0
    unsigned* ticket;     // non-null: persistent grid drawing its items (tile, split) here
    int items;            // tiles_m tiles_n splits
};

// Matrix-core operation per compute type.  FP64: v_mfma_f64_16x16x4_f64; FP32:
// v_mfma_f32_16x16x4_f32 (FP32 products, FP32 accumulation).  Operands are fed
// as A[lane%16][lane/16] and B[lane/16][lane%16]; row_of(r, q) gives the row of
// accumulator element r held by a lane of quarter q = lane/16 (measured lane
// layouts on gfx950).
template <class CT>
struct Mma;
template <>
struct Mma<double> {
    typedef dbl4 acc_t;
    __device__ static acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row_of(int r, int q) { return 4 * r + q; }
};
template <>
struct Mma<float> {
    typedef flt4 acc_t;
    __device__ static acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row_of(int r, int q) { return MMA_F32_ROW(r, q); }
};

// (m, n < 2^31, which gemm_f64 checks)
__device__ __forceinline__ long long out_index(const OutMap& mp, int m, int n) {
    const int qm = div_inv(m, (int)mp.mdiv, mp.minv), qn = div_inv(n, (int)mp.ndiv, mp.ninv);
    return qm * mp.ms1 + (m - qm * (int)mp.mdiv) * mp.ms2 + qn * mp.ns1 +
           (n - qn * (int)mp.ndiv) * mp.ns2;
}

template <class CT, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool PERS>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void gemm_kernel(KArgs p) {
    if (p.gate != nullptr && *p.gate != 0) return;
    typedef typename Mma<CT>::acc_t acc_t;
    constexpr int NWN = BN / WN;
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int LA = (BM * BK + NT - 1) / NT, LB = (BN * BK + NT - 1) / NT;
    constexpr int KP = BK + 16 / (int)sizeof(CT);  // row stride in LDS (elements)
    constexpr int KQ = BK / 4;                      // k values per quarter-wave
    static_assert((KQ * sizeof(CT)) % 16 == 0, "k range of a quarter-wave in 16-byte units");
    __shared__ __attribute__((aligned(16))) CT As[2][BM][KP];
    __shared__ __attribute__((aligned(16))) CT Bs[2][BN][KP];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;

    // Item (bid, split): tile bid of the K range split.  A fixed grid has one
    // item per workgroup; a persistent grid (PERS, p.ticket) draws items from
    // the counter, so that a workgroup that starts late or runs slowly (its CU
    // shared with other work) simply takes fewer.  One ticket per item plus
    // one that ends each workgroup; the workgroup that draws the last ticket
    // of the launch resets the counter.
    auto body = [&](const int bid, const int split) {

    // grouped tile order: GROUP consecutive tile rows share B columns in L2
    constexpr int GROUP = 8;
    const int per_group = GROUP * p.tiles_n;
    const int g = bid / per_group;
    const int first_m = g * GROUP;
    const int gsz = min(p.tiles_m - first_m, GROUP);
    const int tm = first_m + (bid % per_group) % gsz;
    const int tn = (bid % per_group) / gsz;
    const long long m0 = (long long)tm * BM, n0 = (long long)tn * BN;

    const long long kbeg = (long long)split * p.kchunk;
    const long long kend = min(p.K, kbeg + p.kchunk);

    // raw operand values of the next two slabs, held in registers across the
    // MFMAs (two register sets, used alternately: a load has two slabs of
    // matrix-core work to arrive in) for the FP64 128 x 128 tiles, whose two
    // waves per SIMD have the registers; the other builds keep one slab ahead,
    // so that as many workgroups as before fit on a CU
    constexpr bool kPf2 = BM == 128 && BN == 128 && sizeof(CT) == 8;
    double ra0[LA], rb0[LB], ra1[LA], rb1[LB];

    // Out-of-range elements are loaded from a clamped (valid) address; they
    // are replaced by zero (and converted to CT) only when stored to LDS, after
    // the MFMAs of the current slab, so that the loads are not waited for
    // before the matrix-core work.
    auto a_in = [&](int i, long long k0, long long& gm, long long& gk) {
        const int e = tid + i * NT;
        int mm, kk;
        if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
        gm = m0 + mm;
        gk = k0 + kk;
        return (BM * BK % NT == 0 || e < BM * BK) && gm < p.M && gk < kend;
    };
    auto b_in = [&](int i, long long k0, long long& gn, long long& gk) {
        const int e = tid + i * NT;
        int nn, kk;
        if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
        gn = n0 + nn;
        gk = k0 + kk;
        return (BN * BK % NT == 0 || e < BN * BK) && gn < p.N && gk < kend;
    };
    auto load = [&](long long k0, double (&ra)[LA], double (&rb)[LB]) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            long long gm, gk;
            const bool in = a_in(i, k0, gm, gk);
            const long long cm = in ? gm : 0, ck = in ? gk : kbeg;
            ra[i] = TA ? p.A[ck * p.lda + cm] : p.A[cm * p.lda + ck];
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            long long gn, gk;
            const bool in = b_in(i, k0, gn, gk);
            const long long cn = in ? gn : 0, ck = in ? gk : kbeg;
            rb[i] = TB ? p.B[cn * p.ldb + ck] : p.B[ck * p.ldb + cn];
        }
    };
    auto store = [&](int buf, long long k0, const double (&ra)[LA], const double (&rb)[LB]) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + i * NT;
            if (BM * BK % NT != 0 && e >= BM * BK) break;
            long long gm, gk;
            const bool in = a_in(i, k0, gm, gk);
            int mm, kk;
            if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
            As[buf][mm][kk] = in ? (CT)ra[i] : (CT)0;
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = tid + i * NT;
            if (BN * BK % NT != 0 && e >= BN * BK) break;
            long long gn, gk;
            const bool in = b_in(i, k0, gn, gk);
            int nn, kk;
            if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
            Bs[buf][nn][kk] = in ? (CT)rb[i] : (CT)0;
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int lrow = lane & 15;  // operand row/col within a 16-block
    const int lk = lane >> 4;    // quarter-wave: MFMA k slot, k range [lk KQ, (lk+1) KQ)

    int buf = 0;
    if (kbeg < kend) {
        load(kbeg, ra0, rb0);
        store(0, kbeg, ra0, rb0);
    }
    if (kPf2 && kbeg + BK < kend) load(kbeg + BK, ra1, rb1);
    __syncthreads();
    // one slab: the loads of slab k0 + 2 BK go into (na, nb) while slab k0 is
    // multiplied from LDS; then slab k0 + BK, loaded a slab earlier into (ca,
    // cb), is stored to the other LDS buffer
    auto slab = [&](long long k0, double (&ca)[LA], double (&cb)[LB], double (&na)[LA],
                    double (&nb)[LB]) {
        const bool more = k0 + BK < kend;
        if (kPf2) {
            if (k0 + 2 * BK < kend) load(k0 + 2 * BK, na, nb);
        } else if (more) {
            load(k0 + BK, ca, cb);
        }
        CT af[FM][KQ], bf[FN][KQ];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const CT* src = &As[buf][wm * WM + i * 16 + lrow][lk * KQ];
#pragma unroll
            for (int q = 0; q < KQ; ++q) af[i][q] = src[q];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const CT* src = &Bs[buf][wn * WN + j * 16 + lrow][lk * KQ];
#pragma unroll
            for (int q = 0; q < KQ; ++q) bf[j][q] = src[q];
        }
        // k step q: slot lk of the MFMA carries k = lk KQ + q for A and B alike
#pragma unroll
        for (int q = 0; q < KQ; ++q)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = Mma<CT>::run(af[i][q], bf[j][q], acc[i][j]);
        if (more) store(buf ^ 1, k0 + BK, ca, cb);
        __syncthreads();
        buf ^= 1;
    };
    if (kPf2) {
        for (long long k0 = kbeg; k0 < kend; k0 += 2 * BK) {
            slab(k0, ra1, rb1, ra0, rb0);
            if (k0 + BK < kend) slab(k0 + BK, ra0, rb0, ra1, rb1);
        }
    } else {
        for (long long k0 = kbeg; k0 < kend; k0 += BK) slab(k0, ra1, rb1, ra0, rb0);
    }

    // epilogue: accumulator element r of a lane is D[row_of(r, lane/16)][lane%16]
    // Row and column offsets are computed once per accumulator row / column.
    const long long MN = p.M * p.N;
    long long noff[FN];
    bool nok[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const long long n = n0 + wn * WN + j * 16 + lrow;
        nok[j] = n < p.N;
        const int qn = div_inv((int)n, (int)p.map.ndiv, p.map.ninv);
        noff[j] = p.partial ? n : qn * p.map.ns1 + (n - qn * p.map.ndiv) * p.map.ns2;
    }
    double* Cb = p.partial ? p.C + (long long)split * MN : p.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long m = m0 + wm * WM + i * 16 + Mma<CT>::row_of(r, lk);
            if (m >= p.M) continue;
            const int qm = div_inv((int)m, (int)p.map.mdiv, p.map.minv);
            const long long moff =
                p.partial ? m * p.N : qm * p.map.ms1 + (m - qm * p.map.mdiv) * p.map.ms2;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if (!nok[j]) continue;
                const double v = (double)acc[i][j][r];
                if (p.C16) {
                    unsigned short h, mm, l;
                    bf16_split3((float)(p.alpha * v), h, mm, l);
                    const long long o16 = moff + noff[j];
                    p.C16[o16] = h;
                    p.C16[p.pC16 + o16] = mm;
                    p.C16[2 * p.pC16 + o16] = l;
                    continue;
                }
                double* o = Cb + moff + noff[j];
                if (p.partial) *o = v;
                else *o = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *o;
            }
        }
    };
    if constexpr (PERS) {
        __shared__ int item_s;
        const int ntiles = p.tiles_m * p.tiles_n;
        while (true) {
            __syncthreads();  // the previous item's reads of item_s and LDS are done
            if (tid == 0) {
                const unsigned t = atomicAdd(p.ticket, 1u);
                if (t == (unsigned)(p.items + gridDim.x - 1)) atomicExch(p.ticket, 0u);
                item_s = (int)min(t, (unsigned)p.items);
            }
            __syncthreads();
            const int item = item_s;
            if (item >= p.items) break;
            body(item % ntiles, item / ntiles);
        }
    } else {
        body(blockIdx.x, blockIdx.y);
    }
}

// Sum of split-K partials, then the output map / alpha / beta.
__global__ void splitk_reduce_kernel(const double* __restrict__ part, int splits, long long M,
                                     long long N, double* C, OutMap mp, double alpha,
                                     double beta, const int* gate) {
    if (gate != nullptr && *gate != 0) return;
    // M, N < 2^31 and M N < 2^40 (checked by gemm_f64)
    const long long MN = M * N;
    const double invN = 1.0 / (double)N;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < MN;
         e += (long long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += part[z * MN + e];
        const long long m = div_inv64(e, N, invN);
        const int n = (int)(e - m * N);
        const long long o = out_index(mp, (int)m, n);
        C[o] = beta == 0.0 ? alpha * s : alpha * s + beta * C[o];
    }
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, class CT = double>
void launch_cfg(const KArgs& a, int splits, hipStream_t st) {
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    if (a.ticket != nullptr) {
        auto kern = gemm_kernel<CT, BM, BN, BK, WM, WN, TA, TB, true>;
        // persistent: as many workgroups as fit on the device at once
        static int slots = 0;
        if (slots == 0) {
            int dev = 0, cus = 0, per_cu = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0) != hipSuccess)
                per_cu = cus = 0;
            slots = std::max(1, per_cu * cus);
        }
        const int grid = std::min(a.items, slots);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, st, a);
        return;
    }
    dim3 grid(a.tiles_m * a.tiles_n, splits);
    hipLaunchKernelGGL((gemm_kernel<CT, BM, BN, BK, WM, WN, TA, TB, false>), grid, dim3(NT), 0, st, a);
}

template <int BM, int BN, int BK, int WM, int WN, class CT>
void launch_t(const KArgs& a, int ta, int tb, int splits, hipStream_t st) {
    if (!ta && !tb) launch_cfg<BM, BN, BK, WM, WN, false, false, CT>(a, splits, st);
    else if (!ta && tb) launch_cfg<BM, BN, BK, WM, WN, false, true, CT>(a, splits, st);
    else if (ta && !tb) launch_cfg<BM, BN, BK, WM, WN, true, false, CT>(a, splits, st);
    else launch_cfg<BM, BN, BK, WM, WN, true, true, CT>(a, splits, st);
}

struct Plan {
    int cfg;  // 0: 128x128 (8 waves of 64x32; K slabs of 32 in FP64, 16 in FP32);
              // 1: 64x64 (8 waves of 32x16);
              // 2: 128x48 (12 waves of 32x16) for skinny N;
              // 3: 64x128 (8 waves of 32x32, K slabs of 16) for many tiles and K <= 192
              //    (FP64): the smaller LDS footprint lets two workgroups share a CU, which
              //    hides the prologue and epilogue of a short K (measured: 3a at
              //    chi = 144, K = 144: 0.25 -> 0.21 ms; at K = 256 the 128x128 tile wins)
    int bm, bn;
    int splits;
    long long kchunk;
};

constexpr int kTargetBlocks = 512;
// FP32 accumulation (mixed forms): the longest K range one block sums in FP32;
// longer contractions are split and their partial sums added in FP64 (measured
// energy error after 20 steps at D = 6 / 8: unsplit 1.2e-7 / 5.1e-7, chunks of
// 1024 1.25e-7 / 2.3e-8, 512 4.2e-8 / 7.3e-8, 256 4.0e-8 / 3.0e-8 but slower)
constexpr long long kF32Chunk = 512;

// compute units of the current device (256 if the query fails)
long long device_cus() {
    static long long cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus = n;
    }
    return cus;
}

// Tile choice measured on the step's shapes: large M and N take 128x128; a
// skinny N (the edge contraction 3c, N = chi) takes 128x48 tiles with split-K;
// everything else 64x64.  Split-K brings small grids to about 2 blocks per CU.
Plan make_plan(const GemmDesc& g) {
    Plan pl{};
    if (g.prec == 0 && g.K <= 192 && ceil_div(g.M, 128) * ceil_div(g.N, 128) >= 256) {
        pl.cfg = 3; pl.bm = 64; pl.bn = 128;
    } else if (ceil_div(g.M, 128) * ceil_div(g.N, 128) >= 256 ||
        (g.M >= 512 && g.N >= 512 && g.K >= 4096)) {
        // large tiles; a long K with fewer tiles is split below
        pl.cfg = 0; pl.bm = 128; pl.bn = 128;
    } else if (g.N <= 256 && g.M >= 1024 && g.K > 192) {
        // (with a short K the smaller tiles below fill the chip better: the
        // QR's 5184 x 144 x 144 products take 15 instead of 18 us)
        pl.cfg = 2; pl.bm = 128; pl.bn = 48;
    } else {
        pl.cfg = 1; pl.bm = 64; pl.bn = 64;
    }
    const long long tiles = ceil_div(g.M, pl.bm) * ceil_div(g.N, pl.bn);
    pl.splits = 1;
    pl.kchunk = g.K > 0 ? g.K : 1;
    if (tiles < kTargetBlocks / 2 && g.K >= 512) {
        long long s = ceil_div(kTargetBlocks, tiles);
        const long long max_s = g.K / 256;  // keep >= 256 of K per split
        if (s > max_s) s = max_s;
        if (s > 64) s = 64;
        // an even number of splits (measured on 3c at chi = 144, 123 tiles of
        // 128 x 48: 3 splits 259 us, 4: 198, 5: 225, 6: 189, 8: 186)
        if (s % 2 == 1 && s >= 3 && s + 1 <= max_s && s + 1 <= 64) ++s;
        if (s >= 2) {
            long long kc = ceil_div(g.K, s);
            kc = ceil_div(kc, 16) * 16;
            pl.splits = (int)ceil_div(g.K, kc);
            pl.kchunk = kc;
        }
    }
    // Tiles a little over a multiple of the CU count leave a last, nearly empty
    // round of tiles (measured: 3c at D = 6, chi = 320, 270 tiles of 128 x 128,
    // took twice 3a's time for the same flops).  Where there are at least as
    // many tiles as CUs, K is split into the s that minimises the rounds per
    // unit of work, ceil(tiles s / CUs) / s, if that beats no split by 10%.
    if (pl.splits == 1 && tiles >= device_cus() && g.K >= 1024 && g.C16 == nullptr) {
        const long long cus = device_cus();
        auto cost = [&](long long s) { return (double)ceil_div(tiles * s, cus) / (double)s; };
        long long best = 1;
        for (long long s = 2; s <= 8 && g.K / s >= 256; ++s)
            if (cost(s) < cost(best) - 1e-9) best = s;
        if (cost(best) < 0.9 * cost(1)) {
            long long kc = ceil_div(ceil_div(g.K, best), 16) * 16;
            pl.splits = (int)ceil_div(g.K, kc);
            pl.kchunk = kc;
        }
    }
    if (g.prec != 0 && g.C16 == nullptr && pl.kchunk > kF32Chunk) {
        const long long s = std::min<long long>(ceil_div(g.K, kF32Chunk), 64);
        const long long kc = ceil_div(ceil_div(g.K, s), 16) * 16;
        pl.splits = (int)ceil_div(g.K, kc);
        pl.kchunk = kc;
    }
    return pl;
}

}  // namespace

size_t gemm_splitk_bytes(const GemmDesc& g) {
    const Plan pl = make_plan(g);
    return pl.splits > 1 ? (size_t)pl.splits * g.M * g.N * sizeof(double) : 0;
}

namespace {

constexpr double kVendorMinFlop = 3.0e10;  // 2 M N K (chi D^2 = 16384: 3c 1.4e11)
// and enough output tiles for the chip: with few tiles and a long K (an inner
// product of the adjoint, 1 tile) the library ran one workgroup for 0.68 s,
// where the kernel above splits K
constexpr long long kVendorMinTiles = 256;
constexpr int kMaxDevices = 16;

bool plain_output(const GemmDesc& g) {
    const OutMap& m = g.map;
    return m.ms1 == 0 && m.ns1 == 0 && m.ns2 == 1 && m.mdiv >= g.M && m.ndiv >= g.N && m.ms2 >= g.N;
}

bool vendor_eligible(const GemmDesc& g) {
    return g.vendor && g.prec == 0 && g.gate == nullptr && g.A16 == nullptr && g.B16 == nullptr && g.C16 == nullptr &&
           plain_output(g) && 2.0 * (double)g.M * (double)g.N * (double)g.K >= kVendorMinFlop &&
           ceil_div(g.M, 128) * ceil_div(g.N, 128) >= kVendorMinTiles;
}

// one handle per device, made on first use (rocBLAS takes its own workspace
// then); calls on one device are serialised, as a handle has one stream
std::mutex g_vendor_mu;
rocblas_handle g_vendor[kMaxDevices] = {};

Status vendor_dgemm(const GemmDesc& g, hipStream_t st) {
    Status s;
    int dev = 0;
    QRCTM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        s.code = -1;
        s.msg = "gemm_f64: device index out of range for the vendor BLAS";
        return s;
    }
    std::lock_guard<std::mutex> lk(g_vendor_mu);
    if (g_vendor[dev] == nullptr) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success ||
            rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success) {
            if (h) rocblas_destroy_handle(h);
            s.code = -3;
            s.msg = "gemm_f64: rocblas handle";
            return s;
        }
        g_vendor[dev] = h;
    }
    rocblas_handle h = g_vendor[dev];
    // row-major C = op(A) op(B) is column-major C^T = op(B)^T op(A)^T
    const rocblas_operation ta = g.trans_b ? rocblas_operation_transpose : rocblas_operation_none;
    const rocblas_operation tb = g.trans_a ? rocblas_operation_transpose : rocblas_operation_none;
    const double alpha = g.alpha, beta = g.beta;
    if (rocblas_set_stream(h, st) != rocblas_status_success ||
        rocblas_dgemm(h, ta, tb, (rocblas_int)g.N, (rocblas_int)g.M, (rocblas_int)g.K, &alpha, g.B,
                      (rocblas_int)g.ldb, g.A, (rocblas_int)g.lda, &beta, g.C, (rocblas_int)g.map.ms2) !=
            rocblas_status_success) {
        s.code = -3;
        s.msg = "gemm_f64: rocblas_dgemm";
        return s;
    }
    return s;
}

}  // namespace

Status gemm_f64(const GemmDesc& g, void* splitk_ws, size_t splitk_bytes, hipStream_t st) {
    Status s;
    if (g.M <= 0 || g.N <= 0) return s;
    if (g.M >= (1ll << 31) || g.N >= (1ll << 31) || g.M * g.N >= (1ll << 40)) {
        // the kernels index rows and columns in 32 bits
        s.code = -1;
        s.msg = "gemm_f64: M and N must be below 2^31 and M * N below 2^40";
        return s;
    }
    if (g.K <= 0) {
        // C = beta * C (alpha * empty sum)
        // handled by a split-less pass of the reduce kernel with zero partials
        // is wasteful; K == 0 never occurs on the CTMRG path.
        s.code = -1;
        s.msg = "gemm_f64: K must be positive";
        return s;
    }
    // split-BF16 products when the operands come as planes; a result wanted
    // as planes (with FP64 operands) comes from the FP32 matrix cores
    if (g.prec == 2 && (g.A16 || g.B16)) return gemm_bf16x6(g, st);
    if (vendor_eligible(g)) return vendor_dgemm(g, st);
    const Plan pl = make_plan(g);
    KArgs a{};
    a.M = g.M; a.N = g.N; a.K = g.K;
    a.A = g.A; a.lda = g.lda; a.B = g.B; a.ldb = g.ldb;
    a.alpha = g.alpha; a.beta = g.beta; a.map = g.map.with_inv();
    a.kchunk = pl.kchunk;
    a.C16 = g.prec == 2 ? g.C16 : nullptr;
    a.pC16 = g.pC16;
    a.gate = g.gate;
    if (a.C16 && (pl.splits > 1 || g.beta != 0.0)) {
        s.code = -1;
        s.msg = "gemm_f64: a split result needs an unsplit K and beta = 0";
        return s;
    }
    a.tiles_m = (int)ceil_div(g.M, pl.bm);
    a.tiles_n = (int)ceil_div(g.N, pl.bn);
    a.ticket = g.ticket;
    a.items = a.tiles_m * a.tiles_n * pl.splits;
    if (pl.splits > 1) {
        const size_t need = (size_t)pl.splits * g.M * g.N * sizeof(double);
        if (splitk_ws == nullptr || splitk_bytes < need) {
            s.code = -2;
            s.msg = "gemm_f64: split-K scratch too small";
            return s;
        }
        a.C = static_cast<double*>(splitk_ws);
        a.partial = 1;
    } else {
        a.C = g.C;
        a.partial = 0;
    }
    if (g.prec != 0) {
        if (pl.cfg == 0) launch_t<128, 128, 16, 64, 32, float>(a, g.trans_a, g.trans_b, pl.splits, st);
        else if (pl.cfg == 2) launch_t<128, 48, 16, 32, 16, float>(a, g.trans_a, g.trans_b, pl.splits, st);
        else launch_t<64, 64, 16, 32, 16, float>(a, g.trans_a, g.trans_b, pl.splits, st);
    } else {
        if (pl.cfg == 0) launch_t<128, 128, 32, 64, 32, double>(a, g.trans_a, g.trans_b, pl.splits, st);
        else if (pl.cfg == 3) launch_t<64, 128, 16, 32, 32, double>(a, g.trans_a, g.trans_b, pl.splits, st);
        else if (pl.cfg == 2) launch_t<128, 48, 16, 32, 16, double>(a, g.trans_a, g.trans_b, pl.splits, st);
        else launch_t<64, 64, 16, 32, 16, double>(a, g.trans_a, g.trans_b, pl.splits, st);
    }
    QRCTM_TRY(launch_check("gemm_kernel"));
    if (pl.splits > 1) {
        const long long MN = g.M * g.N;
        const int blocks = (int)std::min<long long>(ceil_div(MN, 256), 4096);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, st,
                           static_cast<const double*>(splitk_ws), pl.splits, g.M, g.N, g.C, g.map.with_inv(),
                           g.alpha, g.beta, g.gate);
        QRCTM_TRY(launch_check("splitk_reduce_kernel"));
    }
    return s;
}

}  // namespace qrctm
