// Split-BF16 GEMM on the CDNA4 bf16 matrix cores (v_mfma_f32_16x16x32_bf16),
// for the mixed-precision form of the bulk contractions.
//
// Every operand element x is rounded to FP32 and split exactly into three
// bf16 parts, x32 = hi + mid + lo (8 + 8 + 8 significant bits: hi = bf16(x32),
// mid = bf16(x32 - hi), lo = x32 - hi - mid, each difference exact in FP32).
// A product keeps the six terms down to 2^-24 relative,
//   lo*hi + hi*lo + mid*mid + mid*hi + hi*mid + hi*hi
// (smallest first), accumulated in FP32 by the matrix cores: FP32-level
// accuracy at six bf16 products, whose dense rate is 16x the FP32 one.
//
// Operands come either as FP64 (split while staged) or already split into
// three bf16 planes in HBM ("planes": element (row, k) of plane s at
// base[s * plane + row * ld + k], k contiguous), and the result goes either to
// FP64 through the output map or, split, into three planes at the mapped
// index.  On the CTMRG step the edge contraction 3a writes Y as planes (from
// the FP32 matrix cores) and 3b reads Y and the double layer (transposed,
// split once per tensor) as planes here, so the split work is done once per
// element instead of once per tile.
//
// Tiling: a 256 x 128 tile of C per workgroup of eight waves (two per SIMD),
// 64 x 64 per wave (4 x 4 MFMA blocks); K advances in slabs of 32 staged through LDS as the
// three bf16 planes, stored [plane][k group of 8][row] in 16-byte units: each
// operand fetch is one 16-byte read (8 consecutive k) per lane, and the 16
// lanes of a quarter-wave (consecutive rows, one k group) read or write one
// contiguous 256-byte run, free of bank conflicts.  LDS is double
// buffered and the next slab is loaded into registers during the MFMAs.
// Operand lane layout (measured): lane l feeds row/column l % 16 and the k
// group l / 16; accumulator element r holds D[4 (l / 16) + r][l % 16].
#include "common.h"

namespace qrctm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

struct BArgs {
    long long M, N, K;
    const double* A;  // FP64 A: opA(m, k) = A[m lda + k] (TA false) or A[k lda + m]
    long long lda;
    const unsigned short* A16;  // planes: (m, k) of plane s at A16[s pA + m lda16 + k]
    long long lda16, pA;
    const double* B;  // FP64 B: opB(k, n) = B[k ldb + n] (TB false) or B[n ldb + k]
    long long ldb;
    const unsigned short* B16;  // planes: (n, k) of plane s at B16[s pB + n ldb16 + k]
    long long ldb16, pB;
    double* C;  // FP64 result through map (alpha, beta)
    unsigned short* C16;  // or split result: plane s at C16[s pC + map(m, n)] (alpha only)
    long long pC;
    OutMap map;
    double alpha, beta;
    int tiles_m, tiles_n;
};

constexpr int kBM = 256, kBN = 128, kBK = 32, kWM = 64, kWN = 64;
constexpr int kWaves = (kBM / kWM) * (kBN / kWN);
constexpr int kThreads = kWaves * 64;
constexpr int kGroups = kBK / 8;
constexpr int kItemsA = kBM * kGroups / kThreads;  // 8-k groups of A staged per thread
constexpr int kItemsB = kBN * kGroups / kThreads;  // and of B
static_assert(kItemsA * kThreads == kBM * kGroups && kItemsB * kThreads == kBN * kGroups,
              "whole staging rounds");

__device__ __forceinline__ void split1(float x, unsigned short& h, unsigned short& m,
                                       unsigned short& l) {
    bf16_split3(x, h, m, l);
}
__device__ __forceinline__ void split8(const double (&v)[8], us8 (&s)[3]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        unsigned short h, m, l;
        split1((float)v[e], h, m, l);
        s[0][e] = h;
        s[1][e] = m;
        s[2][e] = l;
    }
}

// One staged operand: 8 consecutive k of one row (A) or column (B) per item.
// load() only issues the loads (clamped addresses); the mask and the split are
// applied in split(), when the slab is stored to LDS after the MFMAs of the
// current slab, so the loads are never waited for before the matrix-core work.
template <bool PLANES, bool T, int kItems>
struct Stage {
    double v[kItems][8];
    us8 raw[kItems][3];
    us8 s[kItems][3];
    // row: global row/column index, k0: first k of the group
    __device__ __forceinline__ void load(int it, const double* X, long long ldx,
                                         const unsigned short* X16, long long ld16, long long pl,
                                         long long row, bool row_ok, long long k0, long long K) {
        if (PLANES) {
            const bool in = row_ok && k0 < K;  // K is a multiple of 8
            const long long base = (in ? row : 0) * ld16 + (in ? k0 : 0);
#pragma unroll
            for (int q = 0; q < 3; ++q) raw[it][q] = *reinterpret_cast<const us8*>(X16 + q * pl + base);
        } else {
            const long long cr = row_ok ? row : 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const long long gk = k0 + e;
                const bool in = row_ok && gk < K;
                const long long ck = in ? gk : 0;
                v[it][e] = T ? X[ck * ldx + cr] : X[cr * ldx + ck];
            }
        }
    }
    __device__ __forceinline__ void split(int it, bool row_ok, long long k0, long long K) {
        if (PLANES) {
            const bool in = row_ok && k0 < K;
#pragma unroll
            for (int q = 0; q < 3; ++q) s[it][q] = in ? raw[it][q] : us8{0, 0, 0, 0, 0, 0, 0, 0};
        } else {
            double w[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = (row_ok && k0 + e < K) ? v[it][e] : 0.0;
            split8(w, s[it]);
        }
    }
};

// (m, n < 2^31, which gemm_f64 checks)
__device__ __forceinline__ long long map_index(const OutMap& mp, int m, int n) {
    const int qm = div_inv(m, (int)mp.mdiv, mp.minv), qn = div_inv(n, (int)mp.ndiv, mp.ninv);
    return qm * mp.ms1 + (m - qm * (int)mp.mdiv) * mp.ms2 + qn * mp.ns1 +
           (n - qn * (int)mp.ndiv) * mp.ns2;
}

template <bool APL, bool BPL, bool TA, bool TB, bool OPL>
__global__ __launch_bounds__(kThreads) void gemm_bf16x6_kernel(BArgs p) {
    __shared__ us8 As[2][3][kGroups][kBM];
    __shared__ us8 Bs[2][3][kGroups][kBN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / (kBN / kWN), wn = wave % (kBN / kWN);

    constexpr int GROUP = 8;
    const int bid = blockIdx.x;
    const int per_group = GROUP * p.tiles_n;
    const int g = bid / per_group;
    const int first_m = g * GROUP;
    const int gsz = min(p.tiles_m - first_m, GROUP);
    const int tm = first_m + (bid % per_group) % gsz;
    const int tn = (bid % per_group) / gsz;
    const long long m0 = (long long)tm * kBM, n0 = (long long)tn * kBN;

    Stage<APL, TA, kItemsA> sa;
    Stage<BPL, !TB, kItemsB> sb;  // B's "row" is the output column n: opB(k, n) = B[n ldb + k] if TB

    auto load = [&](long long k0) {
#pragma unroll
        for (int it = 0; it < kItemsA; ++it) {
            const int item = tid + it * kThreads;
            const int row = item % kBM, grp = item / kBM;
            const long long gm = m0 + row, gk = k0 + 8 * grp;
            sa.load(it, p.A, p.lda, p.A16, p.lda16, p.pA, gm, gm < p.M, gk, p.K);
        }
#pragma unroll
        for (int it = 0; it < kItemsB; ++it) {
            const int item = tid + it * kThreads;
            const int row = item % kBN, grp = item / kBN;
            const long long gn = n0 + row, gk = k0 + 8 * grp;
            sb.load(it, p.B, p.ldb, p.B16, p.ldb16, p.pB, gn, gn < p.N, gk, p.K);
        }
    };
    auto store = [&](int buf, long long k0) {
#pragma unroll
        for (int it = 0; it < kItemsA; ++it) {
            const int item = tid + it * kThreads;
            const int row = item % kBM, grp = item / kBM;
            sa.split(it, m0 + row < p.M, k0 + 8 * grp, p.K);
#pragma unroll
            for (int q = 0; q < 3; ++q) As[buf][q][grp][row] = sa.s[it][q];
        }
#pragma unroll
        for (int it = 0; it < kItemsB; ++it) {
            const int item = tid + it * kThreads;
            const int row = item % kBN, grp = item / kBN;
            sb.split(it, n0 + row < p.N, k0 + 8 * grp, p.K);
#pragma unroll
            for (int q = 0; q < 3; ++q) Bs[buf][q][grp][row] = sb.s[it][q];
        }
    };

    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int FM = kWM / 16, FN = kWN / 16;
    f4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int lr = lane & 15, lg = lane >> 4;
    int buf = 0;
    load(0);
    store(0, 0);
    __syncthreads();
    for (long long k0 = 0; k0 < p.K; k0 += kBK) {
        const bool more = k0 + kBK < p.K;
        if (more) load(k0 + kBK);
        bf16x8 af[3][FM], bfr[3][FN];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
                af[s][i] = __builtin_bit_cast(bf16x8, As[buf][s][lg][wm * kWM + i * 16 + lr]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bfr[s][j] = __builtin_bit_cast(bf16x8, Bs[buf][s][lg][wn * kWN + j * 16 + lr]);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                f4 c = acc[i][j];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], c, 0, 0, 0);
                acc[i][j] = c;
            }
        if (more) store(buf ^ 1, k0 + kBK);
        __syncthreads();
        buf ^= 1;
    }

    // epilogue: element r of a lane is D[4 (lane / 16) + r][lane % 16]
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long m = m0 + wm * kWM + i * 16 + 4 * lg + r;
            if (m >= p.M) continue;
            const int qm = div_inv((int)m, (int)p.map.mdiv, p.map.minv);
            const long long moff = qm * p.map.ms1 + (m - qm * p.map.mdiv) * p.map.ms2;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const long long n = n0 + wn * kWN + j * 16 + lr;
                if (n >= p.N) continue;
                const int qn = div_inv((int)n, (int)p.map.ndiv, p.map.ninv);
                const long long o = moff + qn * p.map.ns1 + (n - qn * p.map.ndiv) * p.map.ns2;
                if (OPL) {
                    unsigned short h, mm, l;
                    split1((float)(p.alpha * (double)acc[i][j][r]), h, mm, l);
                    p.C16[o] = h;
                    p.C16[p.pC + o] = mm;
                    p.C16[2 * p.pC + o] = l;
                } else {
                    const double v = (double)acc[i][j][r];
                    double* c = p.C + o;
                    *c = p.beta == 0.0 ? p.alpha * v : p.alpha * v + p.beta * *c;
                }
            }
        }
}

// planes[s][n][k] = split_s(X[k][n]) for a rows x cols FP64 matrix X (k < rows,
// n < cols): the transposed split of an operand used as B.
__global__ void split_planes_t_kernel(const double* __restrict__ X, long long rows, long long cols,
                                      unsigned short* __restrict__ out) {
    const long long total = rows * cols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long n = e / rows, k = e % rows;
        unsigned short h, m, l;
        split1((float)X[k * cols + n], h, m, l);
        out[e] = h;
        out[total + e] = m;
        out[2 * total + e] = l;
    }
}

}  // namespace

Status split_planes_t(const double* X, long long rows, long long cols, unsigned short* out,
                      hipStream_t st) {
    const long long total = rows * cols;
    const int blocks = (int)std::min<long long>(ceil_div(total, 256), 8192);
    hipLaunchKernelGGL(split_planes_t_kernel, dim3(blocks), dim3(256), 0, st, X, rows, cols, out);
    return launch_check("split_planes_t_kernel");
}

Status gemm_bf16x6(const GemmDesc& g, hipStream_t st) {
    Status s;
    BArgs a{};
    a.M = g.M; a.N = g.N; a.K = g.K;
    a.A = g.A; a.lda = g.lda; a.A16 = g.A16; a.lda16 = g.lda16; a.pA = g.pA16;
    a.B = g.B; a.ldb = g.ldb; a.B16 = g.B16; a.ldb16 = g.ldb16; a.pB = g.pB16;
    a.C = g.C; a.C16 = g.C16; a.pC = g.pC16;
    a.map = g.map.with_inv(); a.alpha = g.alpha; a.beta = g.beta;
    a.tiles_m = (int)ceil_div(g.M, kBM);
    a.tiles_n = (int)ceil_div(g.N, kBN);
    const dim3 grid((unsigned)(a.tiles_m * a.tiles_n)), block(kThreads);
    const bool apl = g.A16 != nullptr, bpl = g.B16 != nullptr, opl = g.C16 != nullptr;
    if ((apl && (g.K % 8 != 0 || g.lda16 % 8 != 0)) || (bpl && (g.K % 8 != 0 || g.ldb16 % 8 != 0)) ||
        (opl && g.beta != 0.0)) {
        s.code = -1;
        s.msg = "gemm_bf16x6: planes need K and their row stride to be multiples of 8, and beta = 0";
        return s;
    }
    if (apl && bpl && !opl)
        hipLaunchKernelGGL((gemm_bf16x6_kernel<true, true, false, false, false>), grid, block, 0, st, a);
    else {
        s.code = -1;
        s.msg = "gemm_bf16x6: operand/result form not provided";
        return s;
    }
    return launch_check("gemm_bf16x6_kernel");
}

}  // namespace qrctm
