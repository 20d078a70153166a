// Shared host/device helpers of the QR-CTMRG library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace qrctm {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Error carried out of the internal launchers; the ABI layer turns it into a
// status code and a message.
struct Status {
    int code = 0;
    std::string msg;
    bool ok() const { return code == 0; }
};

inline Status hip_status(hipError_t e, const char* what) {
    Status s;
    if (e != hipSuccess) {
        s.code = -3;
        s.msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return s;
}

#define QRCTM_TRY(expr)                          \
    do {                                         \
        ::qrctm::Status _s = (expr);             \
        if (!_s.ok()) return _s;                 \
    } while (0)

#define QRCTM_HIP(expr) QRCTM_TRY(::qrctm::hip_status((expr), #expr))

inline Status launch_check(const char* what) { return hip_status(hipGetLastError(), what); }

inline long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// GEMM on the FP64 matrix cores (gemm.hip).
//   C[map(m,n)] = alpha * sum_k opA(m,k) opB(k,n) + beta * C[map(m,n)]
// opA(m,k) = A[m*lda + k] (trans_a = 0) or A[k*lda + m] (trans_a = 1)
// opB(k,n) = B[k*ldb + n] (trans_b = 0) or B[n*ldb + k] (trans_b = 1)
// map(m,n) = (m / mdiv) * ms1 + (m % mdiv) * ms2 + (n / ndiv) * ns1 + (n % ndiv) * ns2
// A plain row-major C with leading dimension ldc is mdiv = M, ms2 = ldc,
// ndiv = N, ns2 = 1.
// ---------------------------------------------------------------------------
// x (FP32) = hi + mid + lo exactly, each a bf16 (round to nearest even; the
// remainders x - hi and x - hi - mid are exact in FP32).  Bit patterns.
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}
__device__ __forceinline__ void bf16_split3(float x, unsigned short& h, unsigned short& m,
                                            unsigned short& l) {
    h = bf16_rne(x);
    const float r1 = x - bf16_value(h);
    m = bf16_rne(r1);
    l = bf16_rne(r1 - bf16_value(m));
}

struct OutMap {
    long long mdiv, ms1, ms2, ndiv, ns1, ns2;
    // 1 / mdiv and 1 / ndiv (set by with_inv before a launch)
    double minv = 0.0, ninv = 0.0;
    static OutMap plain(long long M, long long N, long long ldc) {
        return OutMap{M > 0 ? M : 1, 0, ldc, N > 0 ? N : 1, 0, 1};
    }
    OutMap with_inv() const {
        OutMap o = *this;
        o.minv = 1.0 / (double)mdiv;
        o.ninv = 1.0 / (double)ndiv;
        return o;
    }
};

// m / d for 0 <= m < 2^31, 1 <= d < 2^31, with inv = 1 / d rounded: the
// product is within 2^-21 of m / d, so its truncation is the quotient or one
// below it, and one comparison of the remainder corrects it (an integer
// division is a long instruction sequence on the GPU)
__device__ __forceinline__ int div_inv(int m, int d, double inv) {
    int q = (int)((double)m * inv);
    const int r = m - q * d;
    q += (r >= d ? 1 : 0) - (r < 0 ? 1 : 0);
    return q;
}
// the same for 0 <= m < 2^40 (the product is then within 2^-12 of m / d)
__device__ __forceinline__ long long div_inv64(long long m, long long d, double inv) {
    long long q = (long long)((double)m * inv);
    const long long r = m - q * d;
    q += (r >= d ? 1 : 0) - (r < 0 ? 1 : 0);
    return q;
}

struct GemmDesc {
    int trans_a = 0, trans_b = 0;
    long long M = 0, N = 0, K = 0;
    const double* A = nullptr;
    long long lda = 0;
    const double* B = nullptr;
    long long ldb = 0;
    double* C = nullptr;
    OutMap map{};
    double alpha = 1.0, beta = 0.0;
    int prec = 0;  // 0: FP64 matrix cores; 1: FP32 products and accumulation;
                   // 2: split-BF16 (six bf16 products, FP32 accumulation) when an
                   //    operand or the result is given as bf16 planes, else as 1
    // split-BF16 planes (three bf16 parts; element (row, k) of plane s at
    // base[s * plane + row * ld + k]): A16 (rows m), B16 (rows n = output
    // columns), and the split result C16 (plane s at C16[s * pC16 + map(m, n)])
    const unsigned short* A16 = nullptr;
    long long lda16 = 0, pA16 = 0;
    const unsigned short* B16 = nullptr;
    long long ldb16 = 0, pB16 = 0;
    unsigned short* C16 = nullptr;
    long long pC16 = 0;
    // if non-null: the product is skipped (C untouched) unless *gate == 0
    const int* gate = nullptr;
    // if non-null: a persistent grid (as many workgroups as fit at once) draws
    // the (tile, K split) items from this counter, which must be zero before
    // the launch and is zero again after it (launches sharing one counter must
    // be ordered, e.g. on one stream)
    unsigned* ticket = nullptr;
    // may run as the vendor BLAS's dgemm when it is a plain FP64 product of at
    // least 3e10 flop with at least 256 output tiles of 128 x 128
    bool vendor = true;
};

// Scratch needed by gemm_f64 for split-K partial sums (bytes); 0 when the
// shape does not split.
size_t gemm_splitk_bytes(const GemmDesc& g);
Status gemm_f64(const GemmDesc& g, void* splitk_ws, size_t splitk_bytes, hipStream_t st);
// split-BF16 GEMM (gemm_bf16.hip): planes in and FP64 out, or FP64 (transposed
// A and B) in and planes out; no split-K, no scratch
Status gemm_bf16x6(const GemmDesc& g, hipStream_t st);
// out[s][n][k] = part s of X[k][n] (X rows x cols FP64): the split of an
// operand used as B, transposed so that k is contiguous
Status split_planes_t(const double* X, long long rows, long long cols, unsigned short* out,
                      hipStream_t st);

}  // namespace qrctm
