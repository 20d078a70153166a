// Thin Householder QR of a tall matrix M (m x n, m >= n) with diag(R) >= 0.
//
// QR-CTMRG replaces the eigen/SVD decomposition by an unpivoted QR of the
// reduced corner (QR-CTMRG paragraph, Fig. 1e).  The factorisation here is a
// blocked Householder QR organised for a machine with 256 compute units, all
// in ONE cooperative kernel:
//
//  * rows are dealt cyclically to P workgroups (row g to workgroup g mod P), so
//    every workgroup keeps the same number of active rows as the elimination
//    moves down; each workgroup's rows live in a private working copy in HBM,
//    touched by no other workgroup;
//  * the columns are taken in panels of 16.  For column j of a panel every
//    workgroup reduces, over its rows below j, the squared norm of column j and
//    its dot products with the later panel columns and publishes these 16
//    partial sums; all workgroups then combine the partial sums in one fixed
//    order (bitwise identical everywhere), form the reflector with
//    beta = +||x|| (the non-negative diagonal variant, cancellation-free gamma)
//    and update the panel rows they hold in LDS.  One exchange per column,
//    of 16 numbers per workgroup, not n - j;
//  * after a panel, the trailing columns get the panel's reflectors in compact
//    WY form, I - V T V^T: V^T [V | A_trail] is reduced over all rows (FP64
//    matrix-core tiles per workgroup, then a reduction of the partial products
//    spread over the workgroups), T^T (V^T A_trail) follows from V^T V and the
//    tau's by substitution (T itself is never formed), and
//    A_trail -= V (T^T (V^T A_trail)) is a matrix-core update of each
//    workgroup's own rows;
//  * the explicit thin factor Q = H_0 ... H_{n-1} [I; 0] is formed in the same
//    kernel by applying the panels in reverse order to [I; 0], with the same
//    reduction pattern.
//
// Workgroups exchange data without grid barriers or cache flushes: every
// double sent to another workgroup travels as two 64-bit words, each holding
// 32 bits of the value and a 32-bit tag naming the exchange it belongs to
// (tags grow through the kernel from a base that differs between launches on
// the same buffers; the buffers are cleared to tag 0 when the caller asks,
// which it must on their first use and whenever the base starts over).  Writers and readers use relaxed agent-scope atomics, so each word
// is read whole; a reader polls its words until both carry the expected tag.
// Every exchange only waits for data of the previous one, all workgroups are
// co-resident (a cooperative launch; behind Cholesky-QR2, where it rarely runs,
// an ordinary launch of at most one workgroup per CU on an otherwise idle
// device), and every wait is bounded (on timeout an error bit is set and the
// kernel runs to its end).  Exchange buffers are
// double-buffered where a fast workgroup could otherwise overwrite data a slow
// one has not read: before a workgroup writes exchange t + 2 into a buffer it
// has read exchange t + 1 from every workgroup, which each sent only after
// reading exchange t.
//
// The reflectors are the textbook ones (column by column, in order), so R and Q
// agree with any other Householder QR with diag(R) >= 0 up to rounding.
#include "common.h"
#include "qr.h"

namespace qrctm {
namespace {

constexpr int kQrThreads = 512;
constexpr int kWaves = kQrThreads / 64;
constexpr int kPb = 16;                        // panel width (one MFMA tile)
constexpr int kRowGroups = kQrThreads / kPb;   // 32 row groups x 16 column lanes
constexpr int kRowsPerWg = 32;                 // target rows per workgroup (measured best)
constexpr int kMaxWg = 256;
constexpr int kMaxN = 1024;                    // columns (the LDS budget may allow fewer)
constexpr unsigned kSpinLimit = 1u << 17;      // polls of about a microsecond: ~0.1 s
constexpr size_t kQrLdsBudget = 150 * 1024;
// tags per launch (more than the n + 4 n / 16 + 3 one launch uses for n <=
// 1024) and launches before the tag bases start over
constexpr unsigned kQrTagSpan = 2048;
constexpr unsigned long long kQrEpochs = (1ull << 32) / kQrTagSpan;
static_assert(kMaxWg == 8 * kRowGroups, "the combine sums eight workgroups per row group");

struct QrPlan {
    int P;   // workgroups
    int rb;  // rows held by workgroup 0 (the most)
    size_t lds_bytes;
};

size_t lds_doubles(int rb, int n) {
    // panel rows + Y (16 x n) + G (16 x 16) + reduction scratch (32 x 16)
    // + w, pivot row (16 each) + tau (n) + scalars
    return (size_t)rb * kPb + (size_t)kPb * n + kPb * kPb + kRowGroups * kPb + 2 * kPb +
           (size_t)n + 8;
}

QrPlan plan_qr(int m, int n) {
    QrPlan L{};
    long long P = ceil_div(m, kRowsPerWg);
    if (P > kMaxWg) P = kMaxWg;
    if (P < 1) P = 1;
    L.P = (int)P;
    L.rb = (int)ceil_div(m, P);
    L.lds_bytes = sizeof(double) * lds_doubles(L.rb, n);
    return L;
}

typedef unsigned long long u64;

// A double sent to other workgroups: word 0 holds the low 32 bits, word 1 the
// high 32 bits, each with the tag in its upper half.
__device__ __forceinline__ void ll_put(u64* w, double v, unsigned tag) {
    const u64 b = (u64)__double_as_longlong(v);
    const u64 t = (u64)tag << 32;
    __hip_atomic_store(w, (b & 0xffffffffull) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (b >> 32) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Receive n <= N doubles (word pairs at addr(k)) sent with the given tag: all
// pending pairs are loaded in one round, those with both tags right are taken,
// the rest polled again.  On timeout the missing values are 0 and err gets 2.
template <int N, class Addr>
__device__ __forceinline__ void ll_get(const Addr& addr, int n, unsigned tag, double* out, int* err) {
    unsigned pending = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    unsigned spins = 0;
    while (pending) {
        u64 lo[N], hi[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if ((pending >> k) & 1u) {
                const u64* w = addr(k);
                lo[k] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                hi[k] = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (((pending >> k) & 1u) && (unsigned)(lo[k] >> 32) == tag &&
                (unsigned)(hi[k] >> 32) == tag) {
                out[k] = __longlong_as_double((long long)((hi[k] << 32) | (lo[k] & 0xffffffffull)));
                pending &= ~(1u << k);
            }
        }
        if (pending && ++spins > kSpinLimit) {
            atomicOr(err, 2);
#pragma unroll
            for (int k = 0; k < N; ++k)
                if ((pending >> k) & 1u) out[k] = 0.0;
            break;
        }
    }
}

// v + (v of the lane 16 or 32 apart): the row swap of gfx950 applied to v and
// itself leaves lane l's value and its partner's in the two results.
template <bool BY32>
__device__ __forceinline__ double fold_rows(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned l = (unsigned)b, h = (unsigned)(b >> 32);
    const auto lo = BY32 ? __builtin_amdgcn_permlane32_swap(l, l, false, false)
                         : __builtin_amdgcn_permlane16_swap(l, l, false, false);
    const auto hi = BY32 ? __builtin_amdgcn_permlane32_swap(h, h, false, false)
                         : __builtin_amdgcn_permlane16_swap(h, h, false, false);
    const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double c = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return a + c;
}

// Sum of v over the four lanes of a wave that share lane % 16 (the four row
// groups of a wave), in a fixed order; every lane gets the sum.  All lanes of
// the wave must be active.
__device__ __forceinline__ double quarter_sum(double v) { return fold_rows<true>(fold_rows<false>(v)); }

// Everything a workgroup needs to address its rows.
struct Rows {
    int p, P, nr;  // workgroup, workgroups, rows held (local i <-> global p + i P)
    __device__ __forceinline__ int global(int i) const { return p + i * P; }
    // first local row with global index >= g
    __device__ __forceinline__ int first_at_or_after(int g) const {
        if (g <= p) return 0;
        return (g - p + P - 1) / P;
    }
};

// Householder vector entry of local row i for panel column q (global column
// c0 + q): the stored value below the diagonal, 1 on it, 0 above it and for
// columns past the panel's width nb.
struct PanelV {
    const double* base;  // element (i, q) at base[i * ld + q]
    long long ld;
    Rows rows;
    int c0, nb;
    __device__ __forceinline__ double operator()(int i, int q) const {
        if (i >= rows.nr || q >= nb) return 0.0;
        const int gi = rows.global(i), jq = c0 + q;
        if (gi > jq) return base[(size_t)i * ld + q];
        return gi == jq ? 1.0 : 0.0;
    }
};

// The same for Householder vectors read from the working copy (row g of the
// matrix at A + g * n): panel columns c0 .. c0 + nb - 1.
struct GlobalV {
    const double* A;
    int n;
    Rows rows;
    int c0, nb;
    __device__ __forceinline__ double operator()(int i, int q) const {
        if (i >= rows.nr || q >= nb) return 0.0;
        const int gi = rows.global(i), jq = c0 + q;
        if (gi > jq) return A[(size_t)gi * n + jq];
        return gi == jq ? 1.0 : 0.0;
    }
};

// out[r][c] (16 x (16 + nx), row stride 16 + nx, sent with tag) = sum over local rows i >= ilo
// of V(i, r) * X(i, c), X = [V | X_g(:, xc0 : xc0 + nx)], on the FP64 matrix
// cores: one 16 x 16 output tile per wave at a time, 4 rows per MFMA, the
// operands of 16 rows loaded before the four MFMAs that use them.
template <class VF>
__device__ __forceinline__ void panel_vt_x(const VF& V, const Rows& rows, int ilo, const double* Xg, int ldx,
                           int xc0, int nx, u64* out, unsigned tag) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = kPb + nx;
    const int ntile = (L + 15) / 16;
    const int col_l = lane & 15, k_l = lane >> 4;
    for (int tile = wave; tile < ntile; tile += kWaves) {
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        const int c = tile * 16 + col_l;
        for (int i16 = ilo; i16 < rows.nr; i16 += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i16 + 4 * u + k_l;
                av[u] = V(i, col_l);
                if (c < kPb) bv[u] = V(i, c);
                else if (c < L && i < rows.nr) bv[u] = Xg[(size_t)rows.global(i) * ldx + xc0 + (c - kPb)];
                else bv[u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
        if (c < L) {
#pragma unroll
            for (int r = 0; r < 4; ++r) ll_put(out + 2 * ((size_t)(4 * r + k_l) * L + c), acc[r], tag);
        }
    }
}

// X_g(row, xc0 + c) -= sum_q V(i, q) Y[q][c] for local rows i >= ilo and c < nx
// (Y is 16 x nx in LDS, row stride nx), on the FP64 matrix cores: 16 x 16
// tiles, K = 16 in four steps.
template <class VF>
__device__ __forceinline__ void panel_update(const VF& V, const Rows& rows, int ilo, double* Xg, int ldx, int xc0,
                             int nx, const double* Y) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nrt = (rows.nr - ilo + 15) / 16, nct = (nx + 15) / 16;
    const int col_l = lane & 15, k_l = lane >> 4;
    for (int t = wave; t < nrt * nct; t += kWaves) {
        const int i0 = ilo + (t / nct) * 16, ct = (t % nct) * 16;
        const int c = ct + col_l;
        dbl4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * r + k_l;
            acc[r] = (i < rows.nr && c < nx) ? Xg[(size_t)rows.global(i) * ldx + xc0 + c] : 0.0;
        }
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
            const int q = 4 * kq + k_l;
            const double a = -V(i0 + col_l, q);
            const double b = (c < nx) ? Y[(size_t)q * nx + c] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * r + k_l;
            if (i < rows.nr && c < nx) Xg[(size_t)rows.global(i) * ldx + xc0 + c] = acc[r];
        }
    }
}

// Sum of the P partial products part[q][0:E] (q = 0..P-1, in that order) for
// the entries owned by this workgroup (a contiguous chunk of E / P), sent on
// to sum.  Entries are spread over ew lanes and the partial products over
// 512 / ew thread groups (at most 32 per thread, received 16 at a time).
__device__ __forceinline__ void reduce_chunk(const u64* part, u64* sum, int P, int p, int E, unsigned tag_in,
                             unsigned tag_out, double* red, int* err) {
    const int tid = threadIdx.x;
    const int chunk = (E + P - 1) / P;
    const int e0 = p * chunk, e1 = min(E, e0 + chunk);
    const int ew = chunk <= 16 ? 16 : (chunk <= 32 ? 32 : 64);
    const int ng = kQrThreads / ew;
    const int el = tid % ew, g = tid / ew;
    const int cnt = g < P ? (P - g + ng - 1) / ng : 0;
    for (int base = e0; base < e1; base += ew) {
        const int e = base + el;
        double a = 0.0;
        if (e < e1) {
            for (int k0 = 0; k0 < cnt; k0 += 16) {
                double v[16];
                const int nk = min(16, cnt - k0);
                ll_get<16>([&](int k) { return part + 2 * ((size_t)(g + (k0 + k) * ng) * E + e); },
                           nk, tag_in, v, err);
                for (int k = 0; k < nk; ++k) a += v[k];
            }
        }
        red[g * ew + el] = a;
        __syncthreads();
        if (tid < ew && base + tid < e1) {
            double s = 0.0;
            for (int gg = 0; gg < ng; ++gg) s += red[gg * ew + tid];
            ll_put(sum + 2 * (size_t)(base + tid), s, tag_out);
        }
        __syncthreads();
    }
}

// Y = T^T W (trans) or Y = T W, where I - V T V^T = H_{c0} ... H_{c0+nb-1} in
// compact WY form, without forming T: from the recurrences that define T,
// column by column (T[q][q] = tau_q, T[0:q, q] = -tau_q T[0:q, 0:q] G[0:q, q])
// or row by row (T[q, q+1:] = -tau_q G[q, q+1:] T[q+1:, q+1:]), with G = V^T V,
//   (T^T W)[q] = tau_q (W[q] - sum_{l<q} G[l][q] (T^T W)[l])   (forward),
//   (T W)[q]   = tau_q (W[q] - sum_{l>q} G[q][l] (T W)[l])     (backward).
// The reduced products redsum (16 x L, L = 16 + nx, sent with tag) hold G in
// their first 16 columns and W after them: G goes to LDS and column tid of W to
// registers in one round of loads; thread tid then writes columns tid, tid +
// 512, ... of Y into Ys (16 x nx, row stride nx), receiving the later columns
// of W as it goes.
// Column c of Y from column c of W (in w) and G (in Gs).
__device__ __forceinline__ void y_column(const double* w, const double* tau, int nb, bool trans,
                                         const double* Gs, double* y) {
    if (trans) {
#pragma unroll
        for (int q = 0; q < kPb; ++q) {
            double s = w[q];
#pragma unroll
            for (int l = 0; l < q; ++l) s -= Gs[l * kPb + q] * y[l];
            y[q] = q < nb ? tau[q] * s : 0.0;
        }
    } else {
#pragma unroll
        for (int q = kPb - 1; q >= 0; --q) {
            double s = w[q];
#pragma unroll
            for (int l = q + 1; l < kPb; ++l) s -= Gs[q * kPb + l] * y[l];
            y[q] = q < nb ? tau[q] * s : 0.0;
        }
    }
}

template <bool kWide>
__device__ __forceinline__ void form_y(const u64* redsum, int L, int nx, unsigned tag,
                                       const double* tau, int nb, bool trans, double* Gs,
                                       double* Ys, int* err) {
    const int tid = threadIdx.x;
    double w[kPb];
    if (tid < kPb * kPb) {
        ll_get<1>([&](int) { return redsum + 2 * ((size_t)(tid / kPb) * L + (tid % kPb)); }, 1, tag,
                  w, err);
        Gs[tid] = w[0];
    }
    auto get_w = [&](int c) {
        ll_get<kPb>([&](int r) { return redsum + 2 * ((size_t)r * L + kPb + c); }, kPb, tag, w, err);
    };
    if (tid < nx) get_w(tid);
    __syncthreads();
    double y[kPb];
    if (tid < nx) {
        y_column(w, tau, nb, trans, Gs, y);
#pragma unroll
        for (int q = 0; q < kPb; ++q) Ys[(size_t)q * nx + tid] = y[q];
    }
    // columns beyond the thread count (nx > 512: the kernel built for n > 512)
    if (kWide)
    for (int c = tid + kQrThreads; c < nx; c += kQrThreads) {
        get_w(c);
        y_column(w, tau, nb, trans, Gs, y);
#pragma unroll
        for (int q = 0; q < kPb; ++q) Ys[(size_t)q * nx + c] = y[q];
    }
    __syncthreads();
}

struct QrArgs {
    const double* M;
    int m, n;
    double* A;       // m x n working copy (rows owned cyclically)
    double* Q;       // m x n output (may alias M)
    double* R;       // n x n output
    // exchange buffers (two words per double, see ll_put)
    u64* part;       // 2 x P x 16 column partial sums
    u64* rowbuf;     // 2 x 16 pivot-row entries
    u64* red;        // P x 16 x (16 + n) partial products
    u64* redsum;     // 16 x (16 + n) reduced products
    double* ratio;   // min |R_ii| / max |R_ii|
    int* err;
};

// kWide: built for n > 512 (more columns of Y than threads)
template <bool kWide>
__global__ __launch_bounds__(kQrThreads) void qr_kernel(
    const double* M, int m_, int n_, double* __restrict__ Aw, double* Qo, double* __restrict__ Ro,
    u64* __restrict__ part, u64* __restrict__ rowbuf, u64* __restrict__ redp,
    u64* __restrict__ redsum, double* __restrict__ ratio, int* __restrict__ err, unsigned tag_base,
    const int* __restrict__ run_if, unsigned long long* fallbacks) {
    // behind Cholesky-QR2: run only where it rejected the factorisation
    if (run_if != nullptr) {
        if (*run_if == 0) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(fallbacks, 1ull);
    }
    QrArgs a{M, m_, n_, Aw, Qo, Ro, part, rowbuf, redp, redsum, ratio, err};
    extern __shared__ double lds[];
    const int P = gridDim.x, p = blockIdx.x, tid = threadIdx.x;
    const int m = a.m, n = a.n;
    Rows rows{p, P, (m - p + P - 1) / P};
    const int rbmax = (m + P - 1) / P;
    double* Pn = lds;                          // rbmax x 16 panel rows
    double* Ys = Pn + (size_t)rbmax * kPb;     // 16 x n
    double* Gs = Ys + (size_t)kPb * n;         // 16 x 16
    double* red = Gs + kPb * kPb;              // 32 x 16
    // within the column loop: red (first 8 x 16) for the combine, reda (next
    // 8 x 16) for the partial sums of the next column, so that no barrier is
    // needed between one column's last reads and the next column's writes
    double* reda = red + kWaves * kPb;
    double* wv = red + kRowGroups * kPb;       // 16
    double* rowj = wv + kPb;                   // 16
    double* tau = rowj + kPb;                  // n
    double bmin = INFINITY, bmax = 0.0;
    const int npanel = (n + kPb - 1) / kPb;
    // exchange tags: column round j, then two per panel for the trailing
    // updates and two per panel for the formation of Q
    // (offset by the launch's tag base, so words left by earlier launches on
    // the same buffers never carry a tag this launch waits for)
    auto tag_round = [&](int j) { return tag_base + (unsigned)(1 + j); };
    auto tag_trail = [&](int pk) { return tag_base + (unsigned)(n + 1 + 2 * pk); };
    auto tag_q = [&](int pk) { return tag_base + (unsigned)(n + 1 + 2 * npanel + 2 * pk); };

    // working copy of this workgroup's rows
    for (int e = tid; e < rows.nr * n; e += kQrThreads) {
        const int i = e / n, c = e - i * n;
        a.A[(size_t)rows.global(i) * n + c] = a.M[(size_t)rows.global(i) * n + c];
    }
    __syncthreads();

    const int cl = tid % kPb, rg = tid / kPb, lane = tid & 63, wave = tid >> 6;
    for (int pk = 0; pk < npanel; ++pk) {
        const int c0 = pk * kPb, nb = min(kPb, n - c0), c1 = c0 + nb;
        const int ilo = rows.first_at_or_after(c0);
        // panel rows into LDS; partial sums of column c0 and pivot row c0
        for (int e = tid; e < (rows.nr - ilo) * kPb; e += kQrThreads) {
            const int i = ilo + e / kPb, q = e % kPb;
            Pn[i * kPb + q] = q < nb ? a.A[(size_t)rows.global(i) * n + c0 + q] : 0.0;
        }
        __syncthreads();
        {
            double acc = 0.0;
            for (int i = ilo + rg; i < rows.nr; i += kRowGroups) {
                const int gi = rows.global(i);
                const double x = Pn[i * kPb];
                const double v = Pn[i * kPb + cl];
                if (gi > c0) acc += x * v;
                if (gi == c0) ll_put(a.rowbuf + 2 * ((size_t)(c0 & 1) * kPb + cl), v, tag_round(c0));
            }
            acc = quarter_sum(acc);
            if (lane < kPb) reda[wave * kPb + lane] = acc;
            __syncthreads();
            if (tid < kPb) {
                double s = 0.0;
                for (int w = 0; w < kWaves; ++w) s += reda[w * kPb + tid];
                ll_put(a.part + 2 * (((size_t)(c0 & 1) * P + p) * kPb + tid), s, tag_round(c0));
            }
        }
        for (int q = 0; q < nb; ++q) {
            const int j = c0 + q;
            const int buf = j & 1;
            // combine: slot s = column j + s (slot 0: squared norm below j)
            {
                // row group rg sums workgroups rg, rg + 32, ... (all loads
                // issued before the first add), then the four groups of a
                // wave, then the eight waves
                // (only the slots s < nb - q of this round are sent)
                double v[kMaxWg / kRowGroups];
                const int nw = (rg < P && cl < nb - q) ? (P - rg + kRowGroups - 1) / kRowGroups : 0;
#pragma unroll
                for (int k = 0; k < kMaxWg / kRowGroups; ++k) v[k] = 0.0;
                ll_get<kMaxWg / kRowGroups>(
                    [&](int k) { return a.part + 2 * (((size_t)buf * P + rg + kRowGroups * k) * kPb + cl); },
                    nw, tag_round(j), v, a.err);
                double acc = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
                acc = quarter_sum(acc);
                if (lane < kPb) red[wave * kPb + lane] = acc;
                // pivot row j, panel columns q .. nb - 1 (the ones sent)
                if (tid >= 64 + q && tid < 64 + nb) {
                    double r1[1];
                    ll_get<1>([&](int) { return a.rowbuf + 2 * ((size_t)buf * kPb + tid - 64); }, 1,
                              tag_round(j), r1, a.err);
                    rowj[tid - 64] = r1[0];
                }
                __syncthreads();
                if (tid < kPb) {
                    double t = 0.0;
                    for (int w = 0; w < kWaves; ++w) t += red[w * kPb + tid];
                    wv[tid] = t;
                }
                __syncthreads();
            }
            // reflector (every thread, same values)
            const double alpha = rowj[q], sigma2 = wv[0];
            double beta, t, gamma;
            int mode;  // 0: H = I, 1: sign flip of e_j, 2: general reflector
            if (sigma2 == 0.0) {
                if (alpha >= 0.0) { mode = 0; beta = alpha; t = 0.0; gamma = 1.0; }
                else { mode = 1; beta = -alpha; t = 2.0; gamma = 1.0; }
            } else {
                mode = 2;
                beta = sqrt(alpha * alpha + sigma2);
                gamma = alpha <= 0.0 ? alpha - beta : -sigma2 / (alpha + beta);
                t = -gamma / beta;
            }
            // v = x / gamma below j (as a product with the reciprocal); w_k =
            // v^T a_k over rows >= j for the panel columns k > j
            const double rgam = 1.0 / gamma;
            auto wcol = [&](int qq) {  // panel column qq > q
                const double rj = rowj[qq];
                return mode == 2 ? wv[qq - q] * rgam + rj : rj;
            };
            if (tid == 0) {
                tau[j] = t;
                bmin = fmin(bmin, fabs(beta));
                bmax = fmax(bmax, fabs(beta));
            }
            if (p == 0) {
                for (int k = tid; k < c1; k += kQrThreads) {
                    double r;
                    if (k < j) r = 0.0;
                    else if (k == j) r = beta;
                    else r = rowj[k - c0] - t * wcol(k - c0);
                    a.R[(size_t)j * n + k] = r;
                }
            }
            // apply H_j to the panel rows >= j, store v in column q, and
            // reduce column j+1 against the later panel columns (rows > j+1)
            const bool next = q + 1 < nb;
            const double w1 = next ? wcol(q + 1) : 0.0;
            const double wc = (cl > q && cl < nb) ? wcol(cl) : 0.0;
            const int ij = rows.first_at_or_after(j);
            double acc = 0.0;
            for (int i = ij + rg; i < rows.nr; i += kRowGroups) {
                const int gi = rows.global(i);
                double* row = Pn + i * kPb;
                const double xj = row[q];
                const double v = gi > j ? (mode == 2 ? xj * rgam : 0.0) : 1.0;
                const double tv = t * v;
                const double x1 = next ? row[q + 1] - tv * w1 : 0.0;
                if (cl == q && gi > j) row[q] = v;
                if (cl > q && cl < nb) {
                    const double u = row[cl] - tv * wc;
                    row[cl] = u;
                    if (gi > j + 1) acc += x1 * u;
                    if (gi == j + 1)
                        ll_put(a.rowbuf + 2 * ((size_t)((j + 1) & 1) * kPb + cl), u, tag_round(j + 1));
                }
            }
            if (next) {
                acc = quarter_sum(acc);
                if (lane < kPb) reda[wave * kPb + lane] = acc;
                __syncthreads();
                if (tid < kPb && tid > q) {
                    double s = 0.0;
                    for (int w = 0; w < kWaves; ++w) s += reda[w * kPb + tid];
                    // slot tid - (q + 1) for column j + 1 + (tid - q - 1)
                    ll_put(a.part + 2 * (((size_t)((j + 1) & 1) * P + p) * kPb + (tid - q - 1)), s,
                           tag_round(j + 1));
                }
            }
        }
        __syncthreads();
        // Householder vectors of the panel back to the working copy
        for (int e = tid; e < (rows.nr - ilo) * kPb; e += kQrThreads) {
            const int i = ilo + e / kPb, q = e % kPb;
            if (q < nb) a.A[(size_t)rows.global(i) * n + c0 + q] = Pn[i * kPb + q];
        }
        if (c1 < n) {
            const int nt = n - c1, L = kPb + nt;
            PanelV V{Pn, kPb, rows, c0, nb};
            panel_vt_x(V, rows, ilo, a.A, n, c1, nt, a.red + 2 * (size_t)p * kPb * L, tag_trail(pk));
            reduce_chunk(a.red, a.redsum, P, p, kPb * L, tag_trail(pk), tag_trail(pk) + 1, red, a.err);
            // Y = T^T W, W = V^T A_trail
            form_y<kWide>(a.redsum, L, nt, tag_trail(pk) + 1, tau + c0, nb, true, Gs, Ys, a.err);
            panel_update(V, rows, ilo, a.A, n, c1, nt, Ys);
            __syncthreads();
            // rows c0..c1-1 are final beyond the panel: they are R's rows there
            for (int e = tid; e < nb * nt; e += kQrThreads) {
                const int j = c0 + e / nt, c = c1 + e % nt;
                if (j % P == p) a.R[(size_t)j * n + c] = a.A[(size_t)j * n + c];
            }
        }
    }
    if (p == 0 && tid == 0) *a.ratio = bmax > 0.0 ? bmin / bmax : 0.0;

    // explicit Q: [I; 0], then the panels in reverse order
    __syncthreads();
    for (int e = tid; e < rows.nr * n; e += kQrThreads) {
        const int i = e / n, c = e - i * n;
        const int gi = rows.global(i);
        a.Q[(size_t)gi * n + c] = gi == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int pk = npanel - 1; pk >= 0; --pk) {
        const int c0 = pk * kPb, nb = min(kPb, n - c0);
        const int nq = n - c0, L = kPb + nq;
        const int ilo = rows.first_at_or_after(c0);
        GlobalV VG{a.A, n, rows, c0, nb};
        panel_vt_x(VG, rows, ilo, a.Q, n, c0, nq, a.red + 2 * (size_t)p * kPb * L, tag_q(pk));
        reduce_chunk(a.red, a.redsum, P, p, kPb * L, tag_q(pk), tag_q(pk) + 1, red, a.err);
        // Y = T W, W = V^T Q
        form_y<kWide>(a.redsum, L, nq, tag_q(pk) + 1, tau + c0, nb, false, Gs, Ys, a.err);
        panel_update(VG, rows, ilo, a.Q, n, c0, nq, Ys);
        __syncthreads();
    }
}

// Tag 0 into the exchange buffers (a range of 64-bit words).
__global__ void clear_words_kernel(u64* w, long long count) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        w[e] = 0ull;
}

}  // namespace

QrScratch qr_scratch_layout(int m, int n) {
    QrScratch s{};
    const QrPlan L = plan_qr(m, n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += ((bytes + 255) / 256) * 256;
        return o;
    };
    const size_t w = kPb + (size_t)n;
    s.off_A = take(sizeof(double) * (size_t)m * n);
    // the exchange buffers are one contiguous range (cleared before each launch)
    s.off_part = take(2 * sizeof(u64) * 2 * (size_t)L.P * kPb);
    s.off_rowbuf = take(2 * sizeof(u64) * 2 * kPb);
    s.off_red = take(2 * sizeof(u64) * (size_t)L.P * kPb * w);
    s.off_redsum = take(2 * sizeof(u64) * kPb * w);
    s.off_fallbacks = take(sizeof(unsigned long long));
    s.off_xend = off;
    s.off_ratio = take(sizeof(double));
    s.off_err = take(sizeof(int));
    s.off_chol = take(cholqr_scratch_layout(m, n).total);
    s.total = off;
    return s;
}

int qr_grid(int m, int n) { return plan_qr(m, n).P; }

bool qr_fits(int m, int n) {
    if (m < n || n < 1 || n > kMaxN) return false;
    const QrPlan L = plan_qr(m, n);
    return L.lds_bytes <= kQrLdsBudget && L.P <= kMaxWg;
}

Status qr_fallback_count(const void* ws, int m, int n, hipStream_t st, unsigned long long* out) {
    const QrScratch S = qr_scratch_layout(m, n);
    QRCTM_HIP(hipMemcpyAsync(out, static_cast<const char*>(ws) + S.off_fallbacks, sizeof(*out),
                             hipMemcpyDeviceToHost, st));
    return hip_status(hipStreamSynchronize(st), "hipStreamSynchronize");
}

Status qr_pos(const double* M, double* Q, double* R, int m, int n, void* ws, size_t ws_bytes,
              hipStream_t st, double* diag_ratio_dev, int* err_dev, unsigned long long epoch,
              int method) {
    Status s;
    if (!qr_fits(m, n)) {
        s.code = -1;
        s.msg = "qr: shape not supported (need m >= n >= 1, n <= 1024, rows and panel state within LDS)";
        return s;
    }
    const QrScratch S = qr_scratch_layout(m, n);
    if (ws_bytes < S.total) {
        s.code = -2;
        s.msg = "qr: workspace too small";
        return s;
    }
    const QrPlan L = plan_qr(m, n);
    char* base = static_cast<char*>(ws);
    QrArgs a;
    a.M = M;
    a.m = m;
    a.n = n;
    a.A = reinterpret_cast<double*>(base + S.off_A);
    a.Q = Q;
    a.R = R;
    a.part = reinterpret_cast<u64*>(base + S.off_part);
    a.rowbuf = reinterpret_cast<u64*>(base + S.off_rowbuf);
    a.red = reinterpret_cast<u64*>(base + S.off_red);
    a.redsum = reinterpret_cast<u64*>(base + S.off_redsum);
    a.ratio = diag_ratio_dev ? diag_ratio_dev : reinterpret_cast<double*>(base + S.off_ratio);
    a.err = err_dev ? err_dev : reinterpret_cast<int*>(base + S.off_err);

    const void* kern = n > kQrThreads ? (const void*)qr_kernel<true> : (const void*)qr_kernel<false>;
    int dev = 0;
    QRCTM_HIP(hipGetDevice(&dev));
    QRCTM_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes));
    int nblk = 0;
    QRCTM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, kern, kQrThreads, L.lds_bytes));
    int ncu = 0;
    QRCTM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if ((long long)nblk * ncu < L.P) {
        s.code = -1;
        s.msg = "qr: cooperative grid does not fit on the device";
        return s;
    }
    const unsigned long long e = epoch % kQrEpochs;
    if (e == 0) {
        const long long nwords = (long long)((S.off_xend - S.off_part) / sizeof(u64));
        hipLaunchKernelGGL(clear_words_kernel,
                           dim3((unsigned)std::min<long long>(ceil_div(nwords, 256), 2048)), dim3(256), 0,
                           st, a.part, nwords);
        QRCTM_TRY(launch_check("clear_words_kernel"));
    }
    const bool chol = method == kQrAuto && cholqr_supported(m, n);
    int* run_if = nullptr;
    unsigned long long* fallbacks = reinterpret_cast<unsigned long long*>(base + S.off_fallbacks);
    if (chol) {
        const CholQrScratch C = cholqr_scratch_layout(m, n);
        QRCTM_TRY(cholqr2(M, Q, R, m, n, base + S.off_chol, C, a.ratio, &run_if, st));
    }
    unsigned tag_base = (unsigned)e * kQrTagSpan;
    void* args[] = {(void*)&a.M,    (void*)&a.m,     (void*)&a.n,   (void*)&a.A,
                    (void*)&a.Q,    (void*)&a.R,     (void*)&a.part, (void*)&a.rowbuf,
                    (void*)&a.red,  (void*)&a.redsum, (void*)&a.ratio, (void*)&a.err,
                    (void*)&tag_base, (void*)&run_if, (void*)&fallbacks};
    if (run_if != nullptr) {
        // behind Cholesky-QR2 the kernel returns at once unless the state word
        // asks for it: an ordinary launch, since a cooperative one drains the
        // device before and after it (about 11 us each way at 5184 x 144).  When
        // it does run, its grid (at most one workgroup per CU, fewer than the
        // CUs) is placed at once on the otherwise idle device, and every wait in
        // it is bounded: a workgroup that could not be placed would cost a
        // time-out error, not a hang
        if (n > kQrThreads)
            hipLaunchKernelGGL(qr_kernel<true>, dim3(L.P), dim3(kQrThreads), L.lds_bytes, st, a.M, a.m,
                               a.n, a.A, a.Q, a.R, a.part, a.rowbuf, a.red, a.redsum, a.ratio, a.err,
                               tag_base, run_if, fallbacks);
        else
            hipLaunchKernelGGL(qr_kernel<false>, dim3(L.P), dim3(kQrThreads), L.lds_bytes, st, a.M, a.m,
                               a.n, a.A, a.Q, a.R, a.part, a.rowbuf, a.red, a.redsum, a.ratio, a.err,
                               tag_base, run_if, fallbacks);
        return launch_check("qr_kernel");
    }
    QRCTM_HIP(hipLaunchCooperativeKernel(kern, dim3(L.P), dim3(kQrThreads), args, L.lds_bytes, st));
    return s;
}

}  // namespace qrctm
