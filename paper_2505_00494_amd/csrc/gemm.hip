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
// slab), stored k-major so that every MFMA operand fetch is 16 consecutive
// doubles per quarter-wave.
#include "common.h"

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

__device__ __forceinline__ long long out_index(const OutMap& mp, long long m, long long n) {
    return (m / mp.mdiv) * mp.ms1 + (m % mp.mdiv) * mp.ms2 + (n / mp.ndiv) * mp.ns1 +
           (n % mp.ndiv) * mp.ns2;
}

template <class CT, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void gemm_kernel(KArgs p) {
    typedef typename Mma<CT>::acc_t acc_t;
    constexpr int NWN = BN / WN;
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int LA = (BM * BK + NT - 1) / NT, LB = (BN * BK + NT - 1) / NT;
    constexpr int PAD = 2;  // doubles; breaks the power-of-two row stride
    __shared__ CT As[2][BK][BM + PAD];
    __shared__ CT Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;

    // grouped tile order: GROUP consecutive tile rows share B columns in L2
    constexpr int GROUP = 8;
    const int bid = blockIdx.x;
    const int per_group = GROUP * p.tiles_n;
    const int g = bid / per_group;
    const int first_m = g * GROUP;
    const int gsz = min(p.tiles_m - first_m, GROUP);
    const int tm = first_m + (bid % per_group) % gsz;
    const int tn = (bid % per_group) / gsz;
    const long long m0 = (long long)tm * BM, n0 = (long long)tn * BN;

    const long long kbeg = (long long)blockIdx.y * p.kchunk;
    const long long kend = min(p.K, kbeg + p.kchunk);

    CT ra[LA], rb[LB];

    // Out-of-range elements are loaded from a clamped (valid) address and
    // replaced by zero, so the loads carry no branches.
    auto load = [&](long long k0) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + i * NT;
            int mm, kk;
            if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
            const long long gm = m0 + mm, gk = k0 + kk;
            const bool in = (BM * BK % NT == 0 || e < BM * BK) && gm < p.M && gk < kend;
            const long long cm = in ? gm : 0, ck = in ? gk : kbeg;
            const double v = TA ? p.A[ck * p.lda + cm] : p.A[cm * p.lda + ck];
            ra[i] = in ? (CT)v : (CT)0;
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = tid + i * NT;
            int nn, kk;
            if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
            const long long gn = n0 + nn, gk = k0 + kk;
            const bool in = (BN * BK % NT == 0 || e < BN * BK) && gn < p.N && gk < kend;
            const long long cn = in ? gn : 0, ck = in ? gk : kbeg;
            const double v = TB ? p.B[cn * p.ldb + ck] : p.B[ck * p.ldb + cn];
            rb[i] = in ? (CT)v : (CT)0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + i * NT;
            if (BM * BK % NT != 0 && e >= BM * BK) break;
            int mm, kk;
            if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
            As[buf][kk][mm] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = tid + i * NT;
            if (BN * BK % NT != 0 && e >= BN * BK) break;
            int nn, kk;
            if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
            Bs[buf][kk][nn] = rb[i];
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int lrow = lane & 15;  // operand row/col within a 16-block
    const int lk = lane >> 4;    // k within a 4-slab

    int buf = 0;
    if (kbeg < kend) {
        load(kbeg);
        store(0);
    }
    __syncthreads();
    for (long long k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = k0 + BK < kend;
        if (more) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            CT af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[i] = As[buf][kk * 4 + lk][wm * WM + i * 16 + lrow];
#pragma unroll
            for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kk * 4 + lk][wn * WN + j * 16 + lrow];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = Mma<CT>::run(af[i], bf[j], acc[i][j]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
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
        noff[j] = p.partial ? n : (n / p.map.ndiv) * p.map.ns1 + (n % p.map.ndiv) * p.map.ns2;
    }
    double* Cb = p.partial ? p.C + (long long)blockIdx.y * MN : p.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long m = m0 + wm * WM + i * 16 + Mma<CT>::row_of(r, lk);
            if (m >= p.M) continue;
            const long long moff =
                p.partial ? m * p.N : (m / p.map.mdiv) * p.map.ms1 + (m % p.map.mdiv) * p.map.ms2;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if (!nok[j]) continue;
                const double v = (double)acc[i][j][r];
                double* o = Cb + moff + noff[j];
                if (p.partial) *o = v;
                else *o = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *o;
            }
        }
}

// Sum of split-K partials, then the output map / alpha / beta.
__global__ void splitk_reduce_kernel(const double* __restrict__ part, int splits, long long M,
                                     long long N, double* C, OutMap mp, double alpha,
                                     double beta) {
    const long long MN = M * N;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < MN;
         e += (long long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < splits; ++z) s += part[z * MN + e];
        const long long m = e / N, n = e % N;
        const long long o = out_index(mp, m, n);
        C[o] = beta == 0.0 ? alpha * s : alpha * s + beta * C[o];
    }
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, class CT = double>
void launch_cfg(const KArgs& a, int splits, hipStream_t st) {
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    dim3 grid(a.tiles_m * a.tiles_n, splits);
    hipLaunchKernelGGL((gemm_kernel<CT, BM, BN, BK, WM, WN, TA, TB>), grid, dim3(NT), 0, st, a);
}

template <int BM, int BN, int BK, int WM, int WN, class CT>
void launch_t(const KArgs& a, int ta, int tb, int splits, hipStream_t st) {
    if (!ta && !tb) launch_cfg<BM, BN, BK, WM, WN, false, false, CT>(a, splits, st);
    else if (!ta && tb) launch_cfg<BM, BN, BK, WM, WN, false, true, CT>(a, splits, st);
    else if (ta && !tb) launch_cfg<BM, BN, BK, WM, WN, true, false, CT>(a, splits, st);
    else launch_cfg<BM, BN, BK, WM, WN, true, true, CT>(a, splits, st);
}

struct Plan {
    int cfg;  // 0: 128x128 (8 waves of 64x32); 1: 64x64 (8 waves of 32x16);
              // 2: 128x48 (12 waves of 32x16) for skinny N
    int bm, bn;
    int splits;
    long long kchunk;
};

constexpr int kTargetBlocks = 512;

// Tile choice measured on the step's shapes: large M and N take 128x128; a
// skinny N (the edge contraction 3c, N = chi) takes 128x48 tiles with split-K;
// everything else 64x64.  Split-K brings small grids to about 2 blocks per CU.
Plan make_plan(const GemmDesc& g) {
    Plan pl{};
    if (ceil_div(g.M, 128) * ceil_div(g.N, 128) >= 256) {
        pl.cfg = 0; pl.bm = 128; pl.bn = 128;
    } else if (g.N <= 256 && g.M >= 1024) {
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
        if (s >= 2) {
            long long kc = ceil_div(g.K, s);
            kc = ceil_div(kc, 16) * 16;
            pl.splits = (int)ceil_div(g.K, kc);
            pl.kchunk = kc;
        }
    }
    return pl;
}

}  // namespace

size_t gemm_splitk_bytes(const GemmDesc& g) {
    const Plan pl = make_plan(g);
    return pl.splits > 1 ? (size_t)pl.splits * g.M * g.N * sizeof(double) : 0;
}

Status gemm_f64(const GemmDesc& g, void* splitk_ws, size_t splitk_bytes, hipStream_t st) {
    Status s;
    if (g.M <= 0 || g.N <= 0) return s;
    if (g.K <= 0) {
        // C = beta * C (alpha * empty sum)
        // handled by a split-less pass of the reduce kernel with zero partials
        // is wasteful; K == 0 never occurs on the CTMRG path.
        s.code = -1;
        s.msg = "gemm_f64: K must be positive";
        return s;
    }
    const Plan pl = make_plan(g);
    KArgs a{};
    a.M = g.M; a.N = g.N; a.K = g.K;
    a.A = g.A; a.lda = g.lda; a.B = g.B; a.ldb = g.ldb;
    a.alpha = g.alpha; a.beta = g.beta; a.map = g.map;
    a.kchunk = pl.kchunk;
    a.tiles_m = (int)ceil_div(g.M, pl.bm);
    a.tiles_n = (int)ceil_div(g.N, pl.bn);
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
    if (g.prec == 1) {
        if (pl.cfg == 0) launch_t<128, 128, 16, 64, 32, float>(a, g.trans_a, g.trans_b, pl.splits, st);
        else if (pl.cfg == 2) launch_t<128, 48, 16, 32, 16, float>(a, g.trans_a, g.trans_b, pl.splits, st);
        else launch_t<64, 64, 16, 32, 16, float>(a, g.trans_a, g.trans_b, pl.splits, st);
    } else {
        if (pl.cfg == 0) launch_t<128, 128, 16, 64, 32, double>(a, g.trans_a, g.trans_b, pl.splits, st);
        else if (pl.cfg == 2) launch_t<128, 48, 16, 32, 16, double>(a, g.trans_a, g.trans_b, pl.splits, st);
        else launch_t<64, 64, 16, 32, 16, double>(a, g.trans_a, g.trans_b, pl.splits, st);
    }
    QRCTM_TRY(launch_check("gemm_kernel"));
    if (pl.splits > 1) {
        const long long MN = g.M * g.N;
        const int blocks = (int)std::min<long long>(ceil_div(MN, 256), 4096);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, st,
                           static_cast<const double*>(splitk_ws), pl.splits, g.M, g.N, g.C, g.map,
                           g.alpha, g.beta);
        QRCTM_TRY(launch_check("splitk_reduce_kernel"));
    }
    return s;
}

}  // namespace qrctm
