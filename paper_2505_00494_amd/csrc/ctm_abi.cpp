// C ABI and step driver of the QR-CTMRG library.
//
// A context owns host state only; all device memory is carved out of the
// caller's workspace (plan_workspace).  All GPU work of a context goes to its
// stream in order; host scalars are read after a stream synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qrctm.h"
#include "adjoint.h"
#include "common.h"
#include "edge_split.h"
#include "eigh.h"
#include "energy.h"
#include "qr.h"
#include "step_gemms.h"
#include "spectrum.h"
#include "tensor_ops.h"

using namespace qrctm;

namespace {

thread_local std::string g_create_error;

struct Buf {
    size_t off = 0, bytes = 0;
};

struct Plan {
    // device buffers (byte offsets into the workspace)
    Buf As, a, bvec, C0, C1, T0, T1, Q, R, Y, Z, Tp, W, Cp, S, spec0, spec1, small, normpart, qr,
        splitk, eig, energy, grad;
    // split-BF16 form: Y and the (transposed) double layer as three bf16 planes
    Buf Y16, a16;
    // ket/bra-split 3b: the site tensor as its GEMM operand (empty: not used)
    Buf Bk;
    size_t total = 0;
    size_t qr_bytes = 0, splitk_bytes = 0, eig_bytes = 0, energy_bytes = 0, grad_bytes = 0;
};

struct Shape {
    int d = 0, D = 0, Dab = 0, chi = 0;
    bool quantum = false;
};

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// split-K scratch of the step's GEMMs; the mixed forms (FP32 accumulation) split
// long contractions further
size_t step_splitk_bytes(int chi, int Dab, bool mixed) {
    StepPtrs p{};
    size_t s = 0;
    auto gemm_splitk_bytes = [mixed](GemmDesc g) {
        size_t b = qrctm::gemm_splitk_bytes(g);
        if (mixed) {
            g.prec = 1;
            b = std::max(b, qrctm::gemm_splitk_bytes(g));
        }
        return b;
    };
    for (int c = 1; c <= chi; ++c) {
        s = std::max(s, gemm_splitk_bytes(g_reduced_corner(p, c, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_a(p, nullptr, c, c, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_b(p, c, c, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_c(p, nullptr, c, c, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_corner_w(p, c, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_corner_c(p, c, Dab)));
    }
    // warm-up shapes (chi_in < chi_out)
    for (int ci = 1; ci <= chi; ++ci) {
        const int co = std::min(chi, ci * Dab);
        s = std::max(s, gemm_splitk_bytes(g_edge_a(p, nullptr, ci, ci, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_b(p, ci, ci, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_a(p, nullptr, ci, co, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_b(p, ci, co, Dab)));
        s = std::max(s, gemm_splitk_bytes(g_edge_c(p, nullptr, ci, co, Dab)));
    }
    return s;
}

// ---------------------------------------------------------------------------
// Reverse pass of one QR step: the GEMM adjoints, in order.  Each entry is the
// adjoint of one forward contraction (see qr_step_backward for the sequence).
// ---------------------------------------------------------------------------
struct BwPtrs {
    const double *C, *T, *a, *Q, *R, *Y, *Z, *Tp, *W;
    double *Cpb, *Tpb, *Wb, *Rb, *Qb, *Zg, *Y2, *abar, *Mm, *Ms, *Rinv, *ctb, *Cb2, *Tb2;
};

constexpr int kBwGemms = 16;

GemmDesc bw_gemm(int id, const BwPtrs& p, int chi, int Dab) {
    const long long c = chi, Db = Dab, Db2 = (long long)Dab * Dab;
    auto G = [](int ta, int tb, long long M, long long N, long long K, const double* A, long long lda,
                const double* B, long long ldb, double* C, OutMap mp, double alpha, double beta) {
        GemmDesc g;
        g.trans_a = ta; g.trans_b = tb;
        g.M = M; g.N = N; g.K = K;
        g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
        g.C = C; g.map = mp; g.alpha = alpha; g.beta = beta;
        return g;
    };
    auto pl = [](long long M, long long N) { return OutMap::plain(M, N, N); };
    switch (id) {
        // a8: C' = sum T'[g,r,a] W[g,r,b]
        case 0: return G(0, 1, c * Db, c, c, p.W, c, p.Cpb, c, p.Tpb, pl(c * Db, c), 1.0, 1.0);
        case 1: return G(0, 0, c * Db, c, c, p.Tp, c, p.Cpb, c, p.Wb, pl(c * Db, c), 1.0, 0.0);
        // a8: W = R Q
        case 2: return G(0, 1, c, c, Db * c, p.Wb, Db * c, p.Q, Db * c, p.Rb, pl(c, c), 1.0, 0.0);
        case 3: return G(1, 0, c, Db * c, c, p.R, c, p.Wb, Db * c, p.Qb, pl(c, Db * c), 1.0, 0.0);
        // a7 3c: T'[(a,r),b] = Z[(a,r),(f,d)] Q[(f,d),b]; Zbar stored as [a][f][r][d]
        case 4: return G(0, 1, c * Db, c * Db, c, p.Tpb, c, p.Q, c, p.Zg,
                         OutMap{Db, c * Db2, Db, Db, Db2, 1}, 1.0, 0.0);
        case 5: return G(1, 0, c * Db, c, c * Db, p.Z, c * Db, p.Tpb, c, p.Qb, pl(c * Db, c), 1.0, 1.0);
        // a7 3b: Z[(a,f),(r,d)] = Y[(a,f),(u,l)] a[(u,l),(r,d)]; Ybar stored as [u][a][f][l]
        case 6: return G(0, 1, c * c, Db2, Db2, p.Zg, Db2, p.a, Db2, p.Y2,
                         OutMap{c, c * Db, Db, Db, c * c * Db, 1}, 1.0, 0.0);
        case 7: return G(1, 0, Db2, Db2, c * c, p.Y, Db2, p.Zg, Db2, p.abar, pl(Db2, Db2), 1.0, 1.0);
        // a7 3a: Y[(u,a),(f,l)] = sum_e Q[(e,u),a] T[(f,l),e]
        case 8: return G(0, 0, Db * c, c, c * Db, p.Y2, c * Db, p.T, c, p.Qb,
                         OutMap{Db * c, 0, 1, c, 0, Db * c}, 1.0, 1.0);
        case 9: return G(1, 1, c * Db, c, Db * c, p.Y2, c * Db, p.Q, Db * c, p.Tb2, pl(c * Db, c), 1.0, 0.0);
        // a6: thin-QR adjoint
        case 10: return G(0, 1, c, c, c, p.R, c, p.Rb, c, p.Mm, pl(c, c), 1.0, 0.0);
        case 11: return G(1, 0, c, c, c * Db, p.Qb, c, p.Q, c, p.Mm, pl(c, c), -1.0, 1.0);
        case 12: return G(0, 0, c * Db, c, c, p.Q, c, p.Ms, c, p.Qb, pl(c * Db, c), 1.0, 1.0);
        case 13: return G(0, 1, c * Db, c, c, p.Qb, c, p.Rinv, c, p.ctb, pl(c * Db, c), 1.0, 0.0);
        // a5: ct = C T
        case 14: return G(0, 1, c, c, Db * c, p.ctb, Db * c, p.T, Db * c, p.Cb2, pl(c, c), 1.0, 0.0);
        default: return G(1, 0, c, Db * c, c, p.C, c, p.ctb, Db * c, p.Tb2, pl(c, Db * c), 1.0, 1.0);
    }
}

struct GradLayout {
    size_t ckC, ckT, Cb, Tb, Cb2, Tb2, Ctmp, Ttmp, Cpb, Tpb, Wb, Rb, Qb, Zg, Mm, Ms, Rinv, ctb, abar,
        Asb, part, ratio, dinv, splitk, bwpart;
    // per reversed step: the forward step's Q, R, T', W and its two norms, kept
    // so that the reverse sweep recomputes only Y and Z (3a, 3b); with
    // grad_keep_yz, Y and Z too (sY, sZ, else empty)
    size_t sQ, sR, sTp, sW, sN, sY = 0, sZ = 0;
    bool keep_yz = false;
    size_t splitk_bytes = 0, bwpart_doubles = 0, total = 0;
};

// 3b as the fused split kernel (forward), and its fused reverse where built
bool use_split(const Shape& sh, const ctm_opts& o) {
    // the kernels index Y and Z with 32-bit offsets
    const long long D4 = (long long)sh.D * sh.D * sh.D * sh.D;
    return sh.quantum && o.edge_split == 1 && edge_split_supported(sh.d, sh.D) &&
           (long long)sh.chi * sh.chi * D4 + (1LL << 16) < (1LL << 31);
}
bool use_split_bw(const Shape& sh, const ctm_opts& o) {
    return use_split(sh, o) && edge_split_bw_supported(sh.d, sh.D);
}

GradLayout grad_layout(const Shape& sh, int k, bool split_bw, bool keep_yz) {
    GradLayout L;
    if (!sh.quantum) return L;
    size_t off = 0;
    auto take = [&](size_t count) {
        const size_t o = off;
        off += (count * sizeof(double) + 255) / 256 * 256;
        return o;
    };
    const size_t c = sh.chi, Db = sh.Dab, c2 = c * c;
    // checkpoints C_0..C_k; at least three (the fixed-point scheme's env, F(env), F(F(env)))
    const size_t nck = (size_t)std::max(k + 1, 3);
    L.ckC = take(nck * c2);
    L.ckT = take(nck * c2 * Db);
    L.Cb = take(c2); L.Tb = take(c2 * Db);
    L.Cb2 = take(c2); L.Tb2 = take(c2 * Db);
    L.Ctmp = take(c2); L.Ttmp = take(c2 * Db);
    L.Cpb = take(c2); L.Tpb = take(c2 * Db); L.Wb = take(c2 * Db); L.Rb = take(c2);
    L.Qb = take(c2 * Db); L.Zg = take(c2 * Db * Db);
    L.Mm = take(c2); L.Ms = take(c2); L.Rinv = take(c2); L.ctb = take(c2 * Db);
    const size_t nslot = (size_t)std::max(k, 2);
    L.sQ = take(nslot * c2 * Db); L.sR = take(nslot * c2); L.sTp = take(nslot * c2 * Db);
    L.sW = take(nslot * c2 * Db); L.sN = take(nslot * 8);
    if (keep_yz) {
        L.keep_yz = true;
        L.sY = take(nslot * c2 * Db * Db);
        L.sZ = take(nslot * c2 * Db * Db);
    }
    L.abar = take(Db * Db * Db * Db);
    L.Asb = take((size_t)sh.d * sh.D * sh.D * sh.D * sh.D);
    L.part = take(sym_norm_backward_scratch_bytes() / sizeof(double) + 1);
    L.ratio = take(8);
    L.dinv = take(c);
    BwPtrs p{};
    size_t sk = 0;
    for (int cc = 1; cc <= sh.chi; ++cc)
        for (int id = 0; id < kBwGemms; ++id) sk = std::max(sk, gemm_splitk_bytes(bw_gemm(id, p, cc, sh.Dab)));
    L.splitk_bytes = sk;
    L.splitk = take(sk / sizeof(double) + 1);
    L.bwpart_doubles = split_bw ? edge_split_bw_part_size(sh.d, sh.D) : 0;
    L.bwpart = take(L.bwpart_doubles + 1);
    L.total = off;
    return L;
}

Plan plan_workspace(const Shape& sh, const ctm_opts& o) {
    Plan P;
    size_t off = 0;
    auto take = [&](Buf& b, size_t bytes) {
        b.off = off;
        b.bytes = bytes;
        off += align_up(bytes);
    };
    const size_t d8 = sizeof(double);
    const size_t chi = sh.chi, Dab = sh.Dab;
    const size_t D4 = (size_t)sh.D * sh.D * sh.D * sh.D;
    take(P.As, sh.quantum ? d8 * sh.d * D4 : 0);
    take(P.a, d8 * Dab * Dab * Dab * Dab);
    take(P.bvec, d8 * Dab);
    take(P.C0, d8 * chi * chi);
    take(P.C1, d8 * chi * chi);
    take(P.T0, d8 * chi * chi * Dab);
    take(P.T1, d8 * chi * chi * Dab);
    take(P.Q, d8 * chi * Dab * chi);
    take(P.R, d8 * chi * chi);
    take(P.Y, d8 * chi * chi * Dab * Dab);
    take(P.Z, d8 * chi * chi * Dab * Dab);
    take(P.Tp, d8 * chi * chi * Dab);
    take(P.W, d8 * chi * chi * Dab);
    take(P.Cp, d8 * chi * chi);
    take(P.S, spectrum_scratch_bytes((int)chi));
    take(P.spec0, d8 * chi);
    take(P.spec1, d8 * chi);
    take(P.small, d8 * 64);
    take(P.normpart, sym_norm_scratch_bytes());
    P.qr_bytes = 0;
    for (int c = 1; c <= sh.chi; ++c)
        P.qr_bytes = std::max(P.qr_bytes, qr_scratch_layout(c * sh.Dab, c).total);
    take(P.qr, P.qr_bytes);
    P.splitk_bytes = step_splitk_bytes(sh.chi, sh.Dab, o.precision != CTM_PREC_FP64);
    take(P.splitk, P.splitk_bytes);
    // warm-up eigensolver scratch: order chi_in * Dab of the largest warm-up step
    {
        int nmax = 0, cc = sh.Dab, steps = 0;
        const int want = o.n_warmup < 0 ? -1 : o.n_warmup;
        while (want < 0 ? true : steps < want) {
            nmax = std::max(nmax, cc * sh.Dab);
            const int cn = std::min(sh.chi, cc * sh.Dab);
            ++steps;
            if (want < 0 && (cn >= sh.chi || cn == cc)) break;
            cc = cn;
        }
        P.eig_bytes = nmax > 0 ? eigh_scratch_bytes(nmax) : 0;
    }
    take(P.eig, P.eig_bytes);
    P.energy_bytes = sh.quantum ? energy_scratch_bytes(sh.d, sh.D, sh.chi)
                                : classical_scratch_bytes(sh.Dab, sh.chi);
    take(P.energy, P.energy_bytes);
    P.grad_bytes = grad_layout(sh, o.k_tracked, use_split_bw(sh, o), o.grad_keep_yz != 0).total;
    take(P.grad, P.grad_bytes);
    // planes need the contraction length Dab^2 to be a multiple of 8 (D even);
    // the split 3b has no bf16 build, so it takes no planes
    const bool planes = o.precision == CTM_PREC_BF16X6_MFMA && (Dab * Dab) % 8 == 0 && !use_split(sh, o);
    take(P.Y16, planes ? 3 * sizeof(unsigned short) * chi * chi * Dab * Dab : 0);
    take(P.a16, planes ? 3 * sizeof(unsigned short) * Dab * Dab * Dab * Dab : 0);
    take(P.Bk, use_split(sh, o) ? d8 * edge_split_operand_size(sh.d, sh.D) : 0);
    P.total = off;
    return P;
}

constexpr int kPhases = 8;  // reduced corner, QR, 3a, 3b, 3c, corner, sym/norm, spectrum
// largest relative change of (C, T) under two QR steps that the fixed-point
// gradient accepts as a fixed point
constexpr double kFpMaxResidual = 1e-8;
// largest grid (workgroups) of a cooperative Householder QR that runs beside
// the corner spectrum without waiting for it (measured: grids of 162 and 225
// never did, 240 and 256 did).  Behind Cholesky-QR2 the Householder kernel is
// an ordinary launch and nothing waits for the spectrum.
constexpr int kQrGridBeside = 224;

// small-scalar slots (doubles) inside Plan::small
// SL_DELTA: ring of kDeltaSlots deltas (one per QR step, written on the
// auxiliary stream); SL_DELTA_SCRATCH: delta of spectra computed outside the loop.
constexpr int kDeltaSlots = 8;
enum { SL_NORMS = 2, SL_RATIO = 4, SL_SCALE = 5, SL_BAD = 8, SL_IMAX = 10, SL_E = 16,
       SL_DELTA = 32, SL_DELTA_SCRATCH = 48, SL_TICKET = 56 };

}  // namespace

struct ctm_ctx {
    Shape sh;
    ctm_opts opts{};
    hipStream_t st = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Plan plan;
    int chi_cur = 0;
    int cur = 0;       // which of (C0,T0)/(C1,T1) holds the environment
    bool fp64_steps = false;  // FP64 refinement phase of ctm_converge
    int spec_cur = 0;  // which spectrum buffer holds the spectrum of C
    int n_spec = 0;    // its length
    long long steps = 0;
    double last_delta = NAN;
    double last_ratio = NAN;
    std::string err;
    // optional per-phase timing of QR steps (hipEvents on the context stream)
    bool timing = false;
    long long grad_steps = 0;  // steps reversed by the last gradient
    double fp_residual = 0.0;  // |G(env) - env| / |env| of the last fixed-point gradient
    hipEvent_t ev[kPhases + 1] = {};
    hipEvent_t ev_sp[2] = {};
    double ms_phase[kPhases] = {};
    long long timed_steps = 0;
    // The corner spectrum of step i runs on an auxiliary stream, concurrently
    // with step i+1 on the main stream.  ev_specdone[b] marks the end of the
    // spectrum that reads environment buffer b; the main stream waits on it
    // before overwriting b two steps later.
    hipStream_t aux = nullptr;
    hipEvent_t ev_normed = nullptr, ev_join = nullptr, ev_specdone[2] = {}, ev_qrdone = nullptr;
    bool spec_pending[2] = {false, false};
    // When the QR's cooperative grid covers nearly every CU, the spectrum of a
    // step is queued only once the next step's QR is done (or when its result
    // is needed): a QR workgroup that finds no room beside the running
    // spectrum would stall the whole QR until the spectrum ends.  Smaller
    // grids leave room, and the spectrum runs beside the whole next step.
    struct OwedSpectrum {
        bool live = false;
        const double* C = nullptr;
        int n = 0;
        const double* s_prev = nullptr;
        int n_prev = 0;
        double* s_out = nullptr;
        double* delta = nullptr;
        int target = 0;  // environment buffer it reads
    } owed;
    int last_slot = 0;
    // QR launches on the context's QR workspace (numbers their exchange tags)
    // since its layout was last set for chi_cur = qr_chi (a new size starts
    // over at 0, which clears the exchange words and counters first)
    unsigned long long qr_launches = 0;
    int qr_chi = 0;
    ~ctm_ctx() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : ev_sp)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : ev_specdone)
            if (e) (void)hipEventDestroy(e);
        if (ev_normed) (void)hipEventDestroy(ev_normed);
        if (ev_qrdone) (void)hipEventDestroy(ev_qrdone);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
    }

    template <class T = double>
    T* ptr(const Buf& b) const {
        return reinterpret_cast<T*>(ws + b.off);
    }
    double* C() const { return ptr(cur ? plan.C1 : plan.C0); }
    double* T() const { return ptr(cur ? plan.T1 : plan.T0); }
    double* Cn() const { return ptr(cur ? plan.C0 : plan.C1); }
    double* Tn() const { return ptr(cur ? plan.T0 : plan.T1); }
    double* spec() const { return ptr(spec_cur ? plan.spec1 : plan.spec0); }
    double* spec_next() const { return ptr(spec_cur ? plan.spec0 : plan.spec1); }
    double* small() const { return ptr(plan.small); }
    int* bad() const { return reinterpret_cast<int*>(ptr(plan.small) + SL_BAD); }
    int* imax() const { return reinterpret_cast<int*>(ptr(plan.small) + SL_IMAX); }
    // counter of the step's persistent 3c GEMM (zero between launches)
    unsigned* gemm_ticket() const { return reinterpret_cast<unsigned*>(ptr(plan.small) + SL_TICKET); }
};

namespace {

int fail(ctm_ctx* c, const Status& s) {
    if (c) c->err = s.msg;
    else g_create_error = s.msg;
    return s.code;
}
int fail(ctm_ctx* c, int code, const std::string& msg) {
    Status s;
    s.code = code;
    s.msg = msg;
    return fail(c, s);
}

Status sync(hipStream_t st) { return hip_status(hipStreamSynchronize(st), "hipStreamSynchronize"); }

// Queue the owed spectrum on the auxiliary stream once `after` has completed.
Status launch_owed_spectrum(ctm_ctx* c, hipEvent_t after) {
    if (!c->owed.live) return Status{};
    const auto o = c->owed;
    c->owed.live = false;
    QRCTM_HIP(hipStreamWaitEvent(c->aux, after, 0));
    QRCTM_TRY(corner_spectrum(o.C, o.n, c->ptr(c->plan.S), o.s_prev, o.n_prev, o.s_out, o.delta,
                              c->aux));  // a10
    QRCTM_HIP(hipEventRecord(c->ev_specdone[o.target], c->aux));
    c->spec_pending[o.target] = true;
    return Status{};
}

// Make the main stream wait for all work queued on the auxiliary stream
// (queueing an owed spectrum first).
Status join_aux(ctm_ctx* c) {
    QRCTM_TRY(launch_owed_spectrum(c, c->ev_normed));
    QRCTM_HIP(hipEventRecord(c->ev_join, c->aux));
    QRCTM_HIP(hipStreamWaitEvent(c->st, c->ev_join, 0));
    c->spec_pending[0] = c->spec_pending[1] = false;
    return Status{};
}

Status read_bad(ctm_ctx* c, bool* bad) {
    int h = 0;
    QRCTM_HIP(hipMemcpyAsync(&h, c->bad(), sizeof(int), hipMemcpyDeviceToHost, c->st));
    QRCTM_TRY(sync(c->st));
    *bad = h != 0;
    return Status{};
}

Status clear_bad(ctm_ctx* c) {
    return hip_status(hipMemsetAsync(c->bad(), 0, sizeof(int), c->st), "hipMemsetAsync");
}

// The device error word, read after the stream's work: bit 2 (an exchange of
// the QR's workgroups timed out; its results are zeros) is a runtime error,
// bit 1 (a non-finite or zero tensor where a norm was taken) a numerical one.
Status check_bad(ctm_ctx* c, const char* where) {
    int h = 0;
    QRCTM_HIP(hipMemcpyAsync(&h, c->bad(), sizeof(int), hipMemcpyDeviceToHost, c->st));
    QRCTM_TRY(sync(c->st));
    Status s;
    if (h & 2) {
        s.code = CTM_EHIP;
        s.msg = std::string(where) + ": an exchange between the QR's workgroups timed out";
    } else if (h & 1) {
        s.code = CTM_ENONFINITE;
        s.msg = std::string(where) + ": non-finite or zero environment";
    }
    return s;
}

// One renormalisation of (C, T) with isometry Q (chi*Dab x chio) into Tp, W, Cp.
Status renormalise_edge(ctm_ctx* c, const StepPtrs& p, const double* Q, int chi, int chio) {
    const int Dab = c->sh.Dab;
    void* sk = c->ptr<void>(c->plan.splitk);
    const size_t skb = c->plan.splitk_bytes;
    QRCTM_TRY(gemm_f64(g_edge_a(p, Q, chi, chio, Dab), sk, skb, c->st));
    if (c->plan.Bk.bytes > 0)
        QRCTM_TRY(edge_split_3b(p.Y, c->ptr(c->plan.Bk), c->sh.d, c->sh.D, chi, chio, p.Z, c->st));
    else
        QRCTM_TRY(gemm_f64(g_edge_b(p, chi, chio, Dab), sk, skb, c->st));
    QRCTM_TRY(gemm_f64(g_edge_c(p, Q, chi, chio, Dab), sk, skb, c->st));
    return Status{};
}

StepPtrs step_ptrs(ctm_ctx* c) {
    StepPtrs p;
    p.C = c->C(); p.T = c->T(); p.a = c->ptr(c->plan.a);
    p.Q = c->ptr(c->plan.Q); p.R = c->ptr(c->plan.R);
    p.Y = c->ptr(c->plan.Y); p.Z = c->ptr(c->plan.Z);
    p.Tp = c->ptr(c->plan.Tp); p.W = c->ptr(c->plan.W); p.Cp = c->ptr(c->plan.Cp);
    return p;
}

Status mark(ctm_ctx* c, int i) {
    if (!c->timing) return Status{};
    return hip_status(hipEventRecord(c->ev[i], c->st), "hipEventRecord");
}

// GEMM precision of the forward step (the reverse pass always runs FP64).
int step_prec(const ctm_ctx* c) {
    if (c->fp64_steps) return 0;
    return c->opts.precision == CTM_PREC_FP32_MFMA    ? 1
           : c->opts.precision == CTM_PREC_BF16X6_MFMA ? 2
                                                        : 0;
}

// Operands derived from the site tensor (the double layer's split-BF16 planes,
// the ket/bra-split operand) after a new tensor.
Status refresh_planes(ctm_ctx* c) {
    if (c->plan.Bk.bytes > 0)
        QRCTM_TRY(edge_split_prepare(c->ptr(c->plan.As), c->sh.d, c->sh.D, c->ptr(c->plan.Bk), c->st));
    if (c->plan.a16.bytes == 0) return Status{};
    const long long D2 = (long long)c->sh.Dab * c->sh.Dab;
    return split_planes_t(c->ptr(c->plan.a), D2, D2, c->ptr<unsigned short>(c->plan.a16), c->st);
}

// a5-a9 from (Cin, Tin) into (Cout, Tout); intermediates stay in the step
// buffers (Q, R, Y, Z, Tp, W, Cp) and the norms in the small-scalar slots.
Status qr_step_core(ctm_ctx* c, const double* Cin, const double* Tin, double* Cout, double* Tout,
                    bool timed, int prec, hipEvent_t after_qr = nullptr, double* Yo = nullptr,
                    double* Zo = nullptr) {
    const int chi = c->chi_cur, Dab = c->sh.Dab;
    StepPtrs p = step_ptrs(c);
    p.C = Cin;
    p.T = Tin;
    if (Yo) p.Y = Yo;  // Y and Z into caller buffers (the gradient keeping them)
    if (Zo) p.Z = Zo;
    const bool tm = timed && c->timing;
    auto mark = [&](int i) -> Status {
        if (!tm) return Status{};
        return hip_status(hipEventRecord(c->ev[i], c->st), "hipEventRecord");
    };
    void* sk = c->ptr<void>(c->plan.splitk);
    const size_t skb = c->plan.splitk_bytes;
    // mixed forms (prec 1, 2): the contractions on the FP32 matrix cores, or
    // 3a/3b as split-BF16 products through bf16 planes of Y and of the double
    // layer; the fused split 3b on the FP32 matrix cores in both; QR,
    // normalisation and the spectrum stay FP64
    auto G = [&](GemmDesc g) {
        g.prec = prec;
        return gemm_f64(g, sk, skb, c->st);
    };
    // 3b as the fused ket/bra-split kernel (FP64) when the plan holds its operand
    const bool split = c->plan.Bk.bytes > 0;
    const bool planes = prec == 2 && c->plan.Y16.bytes > 0 && !split;
    unsigned short* Y16 = planes ? c->ptr<unsigned short>(c->plan.Y16) : nullptr;
    QRCTM_TRY(mark(0));
    QRCTM_TRY(G(g_reduced_corner(p, chi, Dab)));                                       // a5
    QRCTM_TRY(mark(1));
    if (c->qr_chi != chi) {
        c->qr_chi = chi;
        c->qr_launches = 0;
    }
    QRCTM_TRY(qr_pos(p.Q, p.Q, p.R, chi * Dab, chi, c->ptr<void>(c->plan.qr), c->plan.qr_bytes,
                     c->st, c->small() + SL_RATIO, c->bad(), c->qr_launches++,
                     c->opts.qr_method == CTM_QR_HOUSEHOLDER ? kQrHouseholder : kQrAuto));  // a6
    if (after_qr) QRCTM_HIP(hipEventRecord(after_qr, c->st));
    QRCTM_TRY(mark(2));
    {
        GemmDesc ga = g_edge_a(p, p.Q, chi, chi, Dab);                                 // a7 3a
        if (planes) {
            ga.C16 = Y16;
            ga.pC16 = ga.M * ga.N;
        }
        QRCTM_TRY(G(ga));
    }
    QRCTM_TRY(mark(3));
    if (split) {
        QRCTM_TRY(edge_split_3b(p.Y, c->ptr(c->plan.Bk), c->sh.d, c->sh.D, chi, chi, p.Z, c->st,
                                prec > 0));                                            // a7 3b
    } else {
        GemmDesc gb = g_edge_b(p, chi, chi, Dab);                                      // a7 3b
        if (planes) {
            const long long D2 = (long long)Dab * Dab;
            gb.A16 = Y16;
            gb.lda16 = D2;
            gb.pA16 = gb.M * gb.K;
            gb.B16 = c->ptr<unsigned short>(c->plan.a16);
            gb.ldb16 = D2;
            gb.pB16 = D2 * D2;
        }
        QRCTM_TRY(G(gb));
    }
    QRCTM_TRY(mark(4));
    {
        // 3c on a persistent grid: the corner spectrum of the previous step runs
        // beside it and holds a CU (measured at D = 6: a fixed grid 239 us beside
        // it and 195 alone, the persistent one 200 and 193; 3a, with many more
        // tiles, loses less and gains nothing)
        GemmDesc gc = g_edge_c(p, p.Q, chi, chi, Dab);                                 // a7 3c
        gc.ticket = c->gemm_ticket();
        QRCTM_TRY(G(gc));
    }
    QRCTM_TRY(mark(5));
    QRCTM_TRY(G(g_corner_w(p, chi, Dab)));                                             // a8
    QRCTM_TRY(G(g_corner_c(p, chi, Dab)));
    QRCTM_TRY(mark(6));
    QRCTM_TRY(sym_norm(p.Cp, p.Tp, chi, Dab, Cout, Tout, c->ptr(c->plan.normpart),
                       c->small() + SL_NORMS, c->bad(), c->st));                     // a9
    return mark(7);
}

// a5-a10 once; environment moves to the other buffer; spectrum likewise.
// a10 (the corner spectrum) is queued on the auxiliary stream.
Status qr_step_once(ctm_ctx* c) {
    const int chi = c->chi_cur;
    const int target = c->cur ^ 1;  // environment buffer this step writes
    if (c->spec_pending[target]) QRCTM_HIP(hipStreamWaitEvent(c->st, c->ev_specdone[target], 0));
    const bool owed = c->owed.live;
    QRCTM_TRY(qr_step_core(c, c->C(), c->T(), c->Cn(), c->Tn(), true, step_prec(c),
                           owed ? c->ev_qrdone : nullptr));
    if (owed) QRCTM_TRY(launch_owed_spectrum(c, c->ev_qrdone));  // the previous step's
    QRCTM_HIP(hipEventRecord(c->ev_normed, c->st));
    const int slot = (int)(c->steps % kDeltaSlots);
    c->owed = ctm_ctx::OwedSpectrum{true,          c->Cn(),          chi, c->spec(), c->n_spec,
                                    c->spec_next(), c->small() + SL_DELTA + slot, target};
    if (c->timing) {  // timed steps run one at a time: the spectrum right after its step
        QRCTM_HIP(hipStreamWaitEvent(c->aux, c->ev_normed, 0));
        QRCTM_HIP(hipEventRecord(c->ev_sp[0], c->aux));
        QRCTM_TRY(launch_owed_spectrum(c, c->ev_normed));
        QRCTM_HIP(hipEventRecord(c->ev_sp[1], c->aux));
    } else if (c->opts.qr_method != CTM_QR_HOUSEHOLDER ||
               qr_grid(chi * c->sh.Dab, chi) <= kQrGridBeside) {
        QRCTM_TRY(launch_owed_spectrum(c, c->ev_normed));
    }
    c->last_slot = slot;
    if (c->timing) {
        QRCTM_HIP(hipEventSynchronize(c->ev[kPhases - 1]));
        QRCTM_HIP(hipEventSynchronize(c->ev_sp[1]));
        for (int i = 0; i < kPhases - 1; ++i) {
            float ms = 0.f;
            QRCTM_HIP(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
            c->ms_phase[i] += ms;
        }
        float ms = 0.f;
        QRCTM_HIP(hipEventElapsedTime(&ms, c->ev_sp[0], c->ev_sp[1]));
        c->ms_phase[kPhases - 1] += ms;
        c->timed_steps++;
    }
    c->cur ^= 1;
    c->spec_cur ^= 1;
    c->n_spec = chi;
    c->steps++;
    return Status{};
}

// Standard step (warm-up): eigh of the enlarged corner, chi grows to
// min(chi_target, chi_cur * Dab).
Status eigh_step_once(ctm_ctx* c) {
    QRCTM_TRY(join_aux(c));
    const int chi = c->chi_cur, Dab = c->sh.Dab;
    const int n = chi * Dab;
    const int chio = std::min(c->sh.chi, n);
    StepPtrs p = step_ptrs(c);
    void* sk = c->ptr<void>(c->plan.splitk);
    const size_t skb = c->plan.splitk_bytes;
    // c~ into Q, enlarged corner into Z (Z[(al,r),(f,d)] = Ct[(f,d),(al,r)])
    QRCTM_TRY(gemm_f64(g_reduced_corner(p, chi, Dab), sk, skb, c->st));
    QRCTM_TRY(gemm_f64(g_edge_a(p, p.Q, chi, chi, Dab), sk, skb, c->st));
    QRCTM_TRY(gemm_f64(g_edge_b(p, chi, chi, Dab), sk, skb, c->st));
    // eigenpairs; U (n x chio) into Q, kept eigenvalues on the diagonal of Cp
    QRCTM_TRY(eigh_select(p.Z, n, chio, p.Q, p.Cp, c->ptr<void>(c->plan.eig), c->plan.eig_bytes,
                          c->st));
    QRCTM_TRY(renormalise_edge(c, p, p.Q, chi, chio));
    QRCTM_TRY(sym_norm(p.Cp, p.Tp, chio, Dab, c->Cn(), c->Tn(), c->ptr(c->plan.normpart),
                       c->small() + SL_NORMS, c->bad(), c->st));
    QRCTM_TRY(corner_spectrum(c->Cn(), chio, c->ptr(c->plan.S), c->spec(), c->n_spec,
                              c->spec_next(), c->small() + SL_DELTA_SCRATCH, c->st));
    c->cur ^= 1;
    c->spec_cur ^= 1;
    c->n_spec = chio;
    c->chi_cur = chio;
    return Status{};
}

struct GradPtrs {
    double *ckC, *ckT, *Cb, *Tb, *Cb2, *Tb2, *Ctmp, *Ttmp, *Cpb, *Tpb, *Wb, *Rb, *Qb, *Zg, *Mm, *Ms,
        *Rinv, *ctb, *abar, *Asb, *part, *ratio, *dinv, *bwpart, *sQ, *sR, *sTp, *sW, *sN;
    double *sY = nullptr, *sZ = nullptr;  // kept Y and Z per step (grad_keep_yz)
    void* splitk;
    size_t splitk_bytes, bwpart_doubles;
};

GradPtrs grad_ptrs(ctm_ctx* c) {
    const GradLayout L =
        grad_layout(c->sh, c->opts.k_tracked, use_split_bw(c->sh, c->opts), c->opts.grad_keep_yz != 0);
    char* b = c->ptr<char>(c->plan.grad);
    auto P = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    GradPtrs g;
    g.ckC = P(L.ckC); g.ckT = P(L.ckT); g.Cb = P(L.Cb); g.Tb = P(L.Tb); g.Cb2 = P(L.Cb2);
    g.Tb2 = P(L.Tb2); g.Ctmp = P(L.Ctmp); g.Ttmp = P(L.Ttmp); g.Cpb = P(L.Cpb); g.Tpb = P(L.Tpb);
    g.Wb = P(L.Wb); g.Rb = P(L.Rb); g.Qb = P(L.Qb); g.Zg = P(L.Zg); g.Mm = P(L.Mm); g.Ms = P(L.Ms);
    g.Rinv = P(L.Rinv); g.ctb = P(L.ctb); g.abar = P(L.abar); g.Asb = P(L.Asb); g.part = P(L.part);
    g.ratio = P(L.ratio);
    g.dinv = P(L.dinv);
    g.splitk = b + L.splitk;
    g.splitk_bytes = L.splitk_bytes;
    g.bwpart = P(L.bwpart);
    g.bwpart_doubles = L.bwpart_doubles;
    g.sQ = P(L.sQ); g.sR = P(L.sR); g.sTp = P(L.sTp); g.sW = P(L.sW); g.sN = P(L.sN);
    if (L.keep_yz) {
        g.sY = P(L.sY);
        g.sZ = P(L.sZ);
    }
    return g;
}

// Keep the forward step's Q, R, T', W and norms (just computed by qr_step_core)
// in reverse-pass slot i.
Status save_step(ctm_ctx* c, const GradPtrs& g, int i) {
    const size_t c2 = (size_t)c->chi_cur * c->chi_cur, nQ = c2 * c->sh.Dab;
    StepPtrs sp = step_ptrs(c);
    auto cp = [&](double* dst, const double* src, size_t n) {
        return hip_status(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToDevice, c->st),
                          "hipMemcpyAsync");
    };
    QRCTM_TRY(cp(g.sQ + i * nQ, sp.Q, nQ));
    QRCTM_TRY(cp(g.sR + i * c2, sp.R, c2));
    QRCTM_TRY(cp(g.sTp + i * nQ, sp.Tp, nQ));
    QRCTM_TRY(cp(g.sW + i * nQ, sp.W, nQ));
    return cp(g.sN + i * 8, c->small() + SL_NORMS, 2);
}

// Reverse of the QR step kept in slot i, which mapped (Ci, Ti) to (Co, To).
// Only Y and Z are recomputed (3a from the kept Q, then 3b), unless they were
// kept too; the cotangents (g.Cb, g.Tb) of (Co, To) become (g.Cb2, g.Tb2) of
// (Ci, Ti).
Status qr_step_backward(ctm_ctx* c, const GradPtrs& g, int i, const double* Ci, const double* Ti,
                        const double* Co, const double* To) {
    const int chi = c->chi_cur, Dab = c->sh.Dab;
    const size_t c2 = (size_t)chi * chi, nQ = c2 * Dab;
    StepPtrs sp = step_ptrs(c);
    sp.C = Ci;
    sp.T = Ti;
    const double* Qi = g.sQ + i * nQ;
    // scratch for Ybar: the step buffer Z (dead once Zbar and Qbar += Z^T Tpbar
    // are formed when Z is recomputed there; unused when Z is kept)
    double* ybar = sp.Z;
    if (g.sY != nullptr) {
        const size_t nY = nQ * Dab;
        sp.Y = g.sY + i * nY;
        sp.Z = g.sZ + i * nY;
    } else {
        QRCTM_TRY(gemm_f64(g_edge_a(sp, Qi, chi, chi, Dab), c->ptr<void>(c->plan.splitk),
                           c->plan.splitk_bytes, c->st));
        if (c->plan.Bk.bytes > 0)
            QRCTM_TRY(edge_split_3b(sp.Y, c->ptr(c->plan.Bk), c->sh.d, c->sh.D, chi, chi, sp.Z, c->st));
        else
            QRCTM_TRY(gemm_f64(g_edge_b(sp, chi, chi, Dab), c->ptr<void>(c->plan.splitk),
                               c->plan.splitk_bytes, c->st));
    }
    BwPtrs p;
    p.C = Ci; p.T = Ti; p.a = sp.a; p.Q = Qi; p.R = g.sR + i * c2; p.Y = sp.Y; p.Z = sp.Z;
    p.Tp = g.sTp + i * nQ;
    p.W = g.sW + i * nQ;
    p.Cpb = g.Cpb; p.Tpb = g.Tpb; p.Wb = g.Wb; p.Rb = g.Rb; p.Qb = g.Qb; p.Zg = g.Zg;
    p.Y2 = ybar;
    p.abar = g.abar; p.Mm = g.Mm; p.Ms = g.Ms; p.Rinv = g.Rinv; p.ctb = g.ctb;
    p.Cb2 = g.Cb2; p.Tb2 = g.Tb2;
    auto run = [&](int id) { return gemm_f64(bw_gemm(id, p, chi, Dab), g.splitk, g.splitk_bytes, c->st); };
    // a9: symmetrise / normalise
    QRCTM_TRY(sym_norm_backward(Co, To, g.Cb, g.Tb, g.sN + i * 8, chi, Dab, g.Cpb,
                                g.Tpb, g.part, c->st));
    if (g.bwpart_doubles > 0) {
        // a8, a7 (3c), the split reverse of 3b (Ybar into Y2, the site tensor's
        // cotangent straight into Asb), a7 (3a)
        for (int id = 0; id <= 5; ++id) QRCTM_TRY(run(id));
        QRCTM_TRY(edge_split_3b_backward(sp.Y, g.Zg, c->ptr(c->plan.Bk), c->sh.d, c->sh.D, chi, chi,
                                         p.Y2, g.bwpart, g.bwpart_doubles, g.Asb, c->st));
        for (int id = 8; id <= 9; ++id) QRCTM_TRY(run(id));
    } else {
        for (int id = 0; id <= 9; ++id) QRCTM_TRY(run(id));   // a8, a7 (3c, 3b, 3a)
    }
    QRCTM_TRY(run(10));                                    // a6: M = R Rbar^T - Qbar^T Q
    QRCTM_TRY(run(11));
    QRCTM_TRY(copyltu(g.Mm, chi, g.Ms, c->st));
    QRCTM_TRY(run(12));                                    // Qbar + Q copyltu(M)
    // R^{-1}, or its regularised form (opts.qr_reg_eps > 0; M is dead once Ms
    // holds copyltu(M))
    double* dinv = nullptr;
    if (c->opts.qr_reg_eps > 0.0) {
        QRCTM_TRY(reg_recip_diag(p.R, chi, c->opts.qr_reg_eps, g.dinv, c->st));
        dinv = g.dinv;
    }
    QRCTM_TRY(tri_inv_upper(p.R, chi, g.Rinv, g.Mm, c->st, dinv));
    QRCTM_TRY(run(13));                                    // ... R^{-T}
    QRCTM_TRY(run(14));                                    // a5
    QRCTM_TRY(run(15));
    return Status{};
}

__global__ void zero_kernel(double* x, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        x[e] = 0.0;
}

Status energy_grad_impl(ctm_ctx* c, const double* h_nn, const double* h_nnn, double J2, double* E,
                        double* dA, bool* series_done) {
    QRCTM_TRY(join_aux(c));
    QRCTM_TRY(clear_bad(c));
    const bool fixed_point = c->opts.grad_mode == CTM_GRAD_FIXED_POINT;
    const int k = c->opts.k_tracked;
    const int chi = c->chi_cur, Dab = c->sh.Dab;
    const size_t nC = (size_t)chi * chi, nT = nC * Dab;
    const GradPtrs g = grad_ptrs(c);
    // checkpoints: C_0..C_k (checkpointed), or env, F(env), F(F(env)) (fixed point)
    const int nfwd = fixed_point ? 2 : k;
    QRCTM_HIP(hipMemcpyAsync(g.ckC, c->C(), nC * 8, hipMemcpyDeviceToDevice, c->st));
    QRCTM_HIP(hipMemcpyAsync(g.ckT, c->T(), nT * 8, hipMemcpyDeviceToDevice, c->st));
    const size_t nY = nT * Dab;
    for (int i = 0; i < nfwd; ++i) {
        QRCTM_TRY(qr_step_core(c, g.ckC + i * nC, g.ckT + i * nT, g.ckC + (i + 1) * nC,
                               g.ckT + (i + 1) * nT, false, 0, nullptr,
                               g.sY ? g.sY + i * nY : nullptr, g.sZ ? g.sZ + i * nY : nullptr));
        QRCTM_TRY(ratio_min(c->small() + SL_RATIO, g.ratio, i == 0, c->st));
        QRCTM_TRY(save_step(c, g, i));
    }
    if (fixed_point) {
        // the scheme needs env = G(env) elementwise (C and T each have unit norm)
        double r2 = 0.0;
        QRCTM_TRY(sq_diff(g.ckC + 2 * nC, g.ckC, g.ckT + 2 * nT, g.ckT, (long long)nC,
                          (long long)nT, g.part, &r2, c->st));
        c->fp_residual = std::sqrt(r2 / 2.0);
        if (!(c->fp_residual <= kFpMaxResidual)) {
            Status s;
            s.code = CTM_ESTATE;
            s.msg = "fixed-point gradient: the environment is not a fixed point of two QR steps "
                    "(relative change " + std::to_string(c->fp_residual) +
                    "); converge it further or use the checkpointed scheme";
            return s;
        }
    }
    // the energy of the tracked steps' end (checkpointed) or of env itself
    const size_t ke = fixed_point ? 0 : (size_t)k;
    EnergyArgs ea{};
    ea.d = c->sh.d; ea.D = c->sh.D; ea.chi = chi;
    ea.C = g.ckC + ke * nC; ea.T = g.ckT + ke * nT; ea.As = c->ptr(c->plan.As);
    // the plaquette term (h_nnn) builds enlarged corners in the step buffers,
    // which hold nothing between the forward sweep and the reverse one
    ea.a = c->ptr(c->plan.a);
    ea.Qbuf = c->ptr(c->plan.Q); ea.Ybuf = c->ptr(c->plan.Y); ea.Zbuf = c->ptr(c->plan.Z);
    ea.ws = c->ptr<char>(c->plan.energy); ea.ws_bytes = c->plan.energy_bytes;
    ea.splitk = nullptr; ea.splitk_bytes = 0;
    QRCTM_TRY(energy_grad_eval(ea, h_nn, h_nnn, J2, E, g.Cb, g.Tb, g.Asb, c->st));
    const long long na = (long long)Dab * Dab * Dab * Dab;
    hipLaunchKernelGGL(zero_kernel, dim3((int)std::min<long long>(ceil_div(na, 256), 4096)), dim3(256),
                       0, c->st, g.abar, na);
    QRCTM_TRY(launch_check("zero_kernel"));
    double* Cb = g.Cb;
    double* Tb = g.Tb;
    double* Cb2 = g.Cb2;
    double* Tb2 = g.Tb2;
    auto reverse_step = [&](int i) -> Status {
        GradPtrs gi = g;
        gi.Cb = Cb; gi.Tb = Tb; gi.Cb2 = Cb2; gi.Tb2 = Tb2;
        QRCTM_TRY(qr_step_backward(c, gi, i, g.ckC + i * nC, g.ckT + i * nT, g.ckC + (i + 1) * nC,
                                   g.ckT + (i + 1) * nT));
        std::swap(Cb, Cb2);
        std::swap(Tb, Tb2);
        return Status{};
    };
    *series_done = true;
    if (!fixed_point) {
        for (int i = k - 1; i >= 0; --i) QRCTM_TRY(reverse_step(i));
        c->grad_steps = k;
    } else {
        // lam = sum_n ebar (dG/denv)^n, G = F o F: reverse env1 -> env, then env -> env1,
        // accumulating the a-cotangent of every reversed step, until a term is small
        double n0 = 0.0, nn = 0.0;
        QRCTM_TRY(sq_norm(Cb, Tb, (long long)nC, (long long)nT, g.part, &n0, c->st));
        const double stop = c->opts.fp_tol * c->opts.fp_tol * n0;
        double least = n0;
        long long steps = 0;
        *series_done = false;
        while (steps < c->opts.fp_max_iter) {
            QRCTM_TRY(reverse_step(1));
            QRCTM_TRY(reverse_step(0));
            steps += 2;
            QRCTM_TRY(sq_norm(Cb, Tb, (long long)nC, (long long)nT, g.part, &nn, c->st));
            if (!std::isfinite(nn)) {
                Status s;
                s.code = CTM_ENONFINITE;
                s.msg = "non-finite cotangent in the fixed-point series";
                return s;
            }
            if (nn <= stop) {
                *series_done = true;
                break;
            }
            // a term whose norm is a hundred times the smallest so far (squared
            // norms compared): the linearised step pair does not contract here
            least = std::min(least, nn);
            if (nn > 1e4 * least) break;
        }
        c->grad_steps = steps;
    }
    // the double layer's cotangent is zero when every reversed 3b was the split form
    if (g.bwpart_doubles == 0)
        QRCTM_TRY(double_layer_backward(g.abar, c->ptr(c->plan.As), c->sh.d, c->sh.D, g.Asb, c->st));
    QRCTM_TRY(c4v_backward(g.Asb, c->ptr(c->plan.As), c->small() + SL_SCALE, c->imax(), c->sh.d,
                           c->sh.D, dA, c->st));
    double ratio = 1.0;
    if (nfwd > 0)
        QRCTM_HIP(hipMemcpyAsync(&ratio, g.ratio, sizeof(double), hipMemcpyDeviceToHost, c->st));
    QRCTM_TRY(check_bad(c, "ctm_energy_grad"));
    if (nfwd > 0 && c->opts.qr_reg_eps == 0.0 && !(ratio >= c->opts.qr_sing_tol)) {
        Status s;
        s.code = CTM_ESINGULAR;
        s.msg = "reduced corner numerically rank deficient in a tracked step (min|R_ii|/max|R_ii| = " +
                std::to_string(ratio) + "); the QR adjoint needs R^{-1}";
        return s;
    }
    if (!std::isfinite(*E)) {
        Status s;
        s.code = CTM_ENONFINITE;
        s.msg = "non-finite energy";
        return s;
    }
    return Status{};
}

int warmup_needed(int chi0, int Dab, int chi) {
    int n = 0, cc = chi0;
    while (true) {
        ++n;
        const int cn = std::min(chi, cc * Dab);
        if (cn >= chi || cn == cc) return n;
        cc = cn;
    }
}

Status fresh_spectrum(ctm_ctx* c) {
    QRCTM_TRY(join_aux(c));
    QRCTM_TRY(corner_spectrum(c->C(), c->chi_cur, c->ptr(c->plan.S), nullptr, 0, c->spec(),
                              c->small() + SL_DELTA_SCRATCH, c->st));
    c->n_spec = c->chi_cur;
    return Status{};
}

Status start_environment(ctm_ctx* c) {
    const int Dab = c->sh.Dab;
    QRCTM_TRY(init_env(c->ptr(c->plan.a), c->ptr(c->plan.bvec), Dab, c->ptr(c->plan.Cp),
                       c->ptr(c->plan.Tp), c->st));
    c->chi_cur = Dab;
    QRCTM_TRY(sym_norm(c->ptr(c->plan.Cp), c->ptr(c->plan.Tp), Dab, Dab, c->C(), c->T(),
                       c->ptr(c->plan.normpart), c->small() + SL_NORMS, c->bad(), c->st));
    QRCTM_TRY(fresh_spectrum(c));
    int nw = c->opts.n_warmup < 0 ? warmup_needed(Dab, Dab, c->sh.chi) : c->opts.n_warmup;
    for (int i = 0; i < nw; ++i) QRCTM_TRY(eigh_step_once(c));
    bool bad = false;
    QRCTM_TRY(read_bad(c, &bad));
    if (bad) {
        Status s;
        s.code = CTM_ENONFINITE;
        s.msg = "non-finite or zero environment during initialisation";
        return s;
    }
    return Status{};
}

bool valid_opts(const ctm_opts& o) {
    return (o.precision == CTM_PREC_FP64 || o.precision == CTM_PREC_FP32_MFMA ||
            o.precision == CTM_PREC_BF16X6_MFMA) &&
           o.k_tracked >= -1 && (o.edge_split == 0 || o.edge_split == 1) &&
           (o.grad_mode == CTM_GRAD_CHECKPOINT || o.grad_mode == CTM_GRAD_FIXED_POINT) &&
           o.fp_tol > 0.0 && o.fp_max_iter >= 2 && (o.grad_keep_yz == 0 || o.grad_keep_yz == 1) &&
           o.qr_reg_eps >= 0.0 && std::isfinite(o.qr_reg_eps) &&
           (o.qr_method == CTM_QR_AUTO || o.qr_method == CTM_QR_HOUSEHOLDER);
}

// Tracked steps per bond dimension when opts.k_tracked = -1: the paper's timing
// study (Fig. 3 caption) uses 10, 12, 14, 16, 20, 24 for D = 2..7; D = 8 is not
// listed there and continues the step of 4 (28), which also covers larger D.
int default_k_tracked(int D) {
    static const int k[] = {10, 10, 10, 12, 14, 16, 20, 24, 28};
    return D < 1 ? 10 : (D <= 8 ? k[D] : 28);
}

ctm_opts resolved(const Shape& sh, const ctm_opts& in) {
    ctm_opts o = in;
    if (o.k_tracked < 0) o.k_tracked = default_k_tracked(sh.quantum ? sh.D : 0);
    return o;
}

int create(ctm_ctx** out, const Shape& sh, const ctm_opts* opts, void* ws, size_t ws_bytes,
           void* stream, ctm_ctx** made) {
    if (out == nullptr) return fail(nullptr, CTM_EINVAL, "out is NULL");
    *out = nullptr;
    ctm_opts o;
    ctm_default_opts(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return fail(nullptr, CTM_EINVAL, "invalid ctm_opts");
    o = resolved(sh, o);
    if (sh.chi < 1 || sh.chi > 1024 || sh.Dab < 1)
        return fail(nullptr, CTM_EINVAL, "chi must be in [1, 1024] and Dab >= 1");
    if (sh.chi < sh.Dab)
        return fail(nullptr, CTM_EINVAL, "chi must be at least the bond dimension Dab of the bulk tensor");
    if (!qr_fits(sh.chi * sh.Dab, sh.chi))
        return fail(nullptr, CTM_EINVAL, "chi*Dab x chi reduced corner exceeds the QR kernel limits");
    Plan P = plan_workspace(sh, o);
    if (ws == nullptr || ws_bytes < P.total)
        return fail(nullptr, CTM_EWORKSPACE, "workspace missing or smaller than ctm_workspace_bytes");
    ctm_ctx* c = new ctm_ctx();
    c->sh = sh;
    c->opts = o;
    c->st = static_cast<hipStream_t>(stream);
    c->ws = static_cast<char*>(ws);
    c->ws_bytes = ws_bytes;
    c->plan = P;
    bool ok = hipMemsetAsync(c->gemm_ticket(), 0, sizeof(unsigned), c->st) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_normed, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_qrdone, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_specdone[0], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_specdone[1], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        delete c;
        return fail(nullptr, CTM_EHIP, "could not create the auxiliary stream / events");
    }
    *made = c;
    return 0;
}

template <class F>
int guarded(ctm_ctx* c, F&& f) {
    try {
        Status s = f();
        if (!s.ok()) return fail(c, s);
        return s.code;
    } catch (const std::exception& e) {
        return fail(c, CTM_EHIP, std::string("exception: ") + e.what());
    } catch (...) {
        return fail(c, CTM_EHIP, "unknown exception");
    }
}

// Algorithmic flops of one QR step (Dab = D^2): reduced corner 2 chi^3 Dab,
// Householder QR 4 m n^2 - 4 n^3 / 3 with m = chi Dab, n = chi, edge
// renormalisation 2 chi^3 Dab^2 + 3b + 2 chi^3 Dab^2 with 3b 2 chi^2 Dab^4 (double
// layer) or 4 d chi^2 Dab^3 (ket/bra split, d > 0), accelerated corner 4 chi^3 Dab.
double step_flops(int chi, int Dab, int d_split) {
    const double c = chi, Db = Dab, Db2 = Db * Db;
    const double f3b = d_split > 0 ? 4.0 * d_split * c * c * Db2 * Db : 2 * c * c * Db2 * Db2;
    return 2 * c * c * c * Db + (4 * c * c * c * Db - 4.0 / 3.0 * c * c * c) +
           2 * c * c * c * Db2 + f3b + 2 * c * c * c * Db2 + 4 * c * c * c * Db;
}

}  // namespace

extern "C" {

void ctm_default_opts(ctm_opts* o) {
    if (!o) return;
    o->precision = CTM_PREC_FP64;
    o->n_warmup = -1;
    o->k_tracked = -1;
    o->qr_sing_tol = 1e-14;
    o->mixed_tol = 1e-6;
    o->edge_split = 1;
    o->grad_mode = CTM_GRAD_CHECKPOINT;
    o->fp_tol = 1e-10;
    o->fp_max_iter = 1000;
    o->grad_keep_yz = 0;
    o->qr_reg_eps = 0.0;
    o->qr_method = CTM_QR_AUTO;
}

size_t ctm_workspace_bytes(int d, int D, int chi, const ctm_opts* opts) {
    if (d < 1 || D < 1 || chi < 1) return 0;
    ctm_opts o;
    ctm_default_opts(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return 0;
    Shape sh{d, D, D * D, chi, true};
    return plan_workspace(sh, resolved(sh, o)).total;
}

size_t ctm_workspace_bytes_dl(int Dab, int chi, const ctm_opts* opts) {
    if (Dab < 1 || chi < 1) return 0;
    ctm_opts o;
    ctm_default_opts(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return 0;
    Shape sh{0, 0, Dab, chi, false};
    return plan_workspace(sh, resolved(sh, o)).total;
}

int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi, const ctm_opts* opts, void* ws,
             size_t ws_bytes, void* stream) {
    if (A == nullptr || d < 1 || D < 1) return fail(nullptr, CTM_EINVAL, "invalid A, d or D");
    Shape sh{d, D, D * D, chi, true};
    ctm_ctx* c = nullptr;
    int rc = create(out, sh, opts, ws, ws_bytes, stream, &c);
    if (rc != 0) return rc;
    rc = guarded(c, [&]() -> Status {
        QRCTM_TRY(clear_bad(c));
        QRCTM_TRY(c4v_prepare(A, d, D, c->ptr(c->plan.As), c->small() + SL_SCALE, c->bad(),
                              c->imax(), c->st));
        QRCTM_TRY(double_layer(c->ptr(c->plan.As), d, D, c->ptr(c->plan.a), c->st));
        QRCTM_TRY(refresh_planes(c));
        QRCTM_TRY(eye_vec(c->ptr(c->plan.bvec), D, c->st));
        bool bad = false;
        QRCTM_TRY(read_bad(c, &bad));
        if (bad) {
            Status s;
            s.code = CTM_ENONFINITE;
            s.msg = "site tensor is non-finite or zero after the C4v average";
            return s;
        }
        return start_environment(c);
    });
    if (rc < 0) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return rc;
}

int ctm_init_dl(ctm_ctx** out, const double* a, const double* bvec, int Dab, int chi,
                const ctm_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    if (a == nullptr || bvec == nullptr) return fail(nullptr, CTM_EINVAL, "a or bvec is NULL");
    Shape sh{0, 0, Dab, chi, false};
    ctm_ctx* c = nullptr;
    int rc = create(out, sh, opts, ws, ws_bytes, stream, &c);
    if (rc != 0) return rc;
    rc = guarded(c, [&]() -> Status {
        QRCTM_TRY(clear_bad(c));
        QRCTM_TRY(dl_to_internal(a, Dab, c->ptr(c->plan.a), c->st));
        QRCTM_TRY(refresh_planes(c));
        QRCTM_HIP(hipMemcpyAsync(c->ptr(c->plan.bvec), bvec, sizeof(double) * Dab,
                                 hipMemcpyDeviceToDevice, c->st));
        return start_environment(c);
    });
    if (rc < 0) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return rc;
}

int ctm_set_tensor(ctm_ctx* c, const double* A) {
    if (!c || !A) return fail(c, CTM_EINVAL, "NULL argument");
    if (!c->sh.quantum) return fail(c, CTM_ESTATE, "context was built from a double-layer tensor");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        QRCTM_TRY(clear_bad(c));
        QRCTM_TRY(c4v_prepare(A, c->sh.d, c->sh.D, c->ptr(c->plan.As), c->small() + SL_SCALE,
                              c->bad(), c->imax(), c->st));
        QRCTM_TRY(double_layer(c->ptr(c->plan.As), c->sh.d, c->sh.D, c->ptr(c->plan.a), c->st));
        QRCTM_TRY(refresh_planes(c));
        bool bad = false;
        QRCTM_TRY(read_bad(c, &bad));
        if (bad) {
            Status s;
            s.code = CTM_ENONFINITE;
            s.msg = "site tensor is non-finite or zero";
            return s;
        }
        return Status{};
    });
}

int ctm_step(ctm_ctx* c, int nsteps, double* delta) {
    if (!c || nsteps < 0) return fail(c, CTM_EINVAL, "invalid arguments");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(clear_bad(c));
        for (int i = 0; i < nsteps; ++i) QRCTM_TRY(qr_step_once(c));
        double h[2] = {NAN, NAN};
        if (nsteps > 0) {
            QRCTM_TRY(launch_owed_spectrum(c, c->ev_normed));
            QRCTM_HIP(hipMemcpyAsync(h, c->small() + SL_DELTA + c->last_slot, sizeof(double),
                                     hipMemcpyDeviceToHost, c->aux));
            QRCTM_HIP(hipStreamSynchronize(c->aux));
        } else {
            h[0] = c->last_delta;
        }
        c->last_delta = h[0];
        if (delta) *delta = h[0];
        QRCTM_TRY(check_bad(c, "ctm_step"));
        // nsteps = 0 reports the last step's change (NaN before the first step)
        if (nsteps > 0 && !std::isfinite(h[0])) {
            Status s;
            s.code = CTM_ENONFINITE;
            s.msg = "non-finite environment in ctm_step";
            return s;
        }
        return Status{};
    });
}

int ctm_converge(ctm_ctx* c, double tol, int max_steps, int* steps, double* delta) {
    if (!c || max_steps < 0) return fail(c, CTM_EINVAL, "invalid arguments");
    int taken = 0;
    double dl = NAN;
    int rc = guarded(c, [&]() -> Status {
        QRCTM_TRY(clear_bad(c));
        // Step i+1 is queued before delta_i is read, so the GPU never waits
        // for the host; if step i has converged, step i+1 is discarded (its
        // outputs live in the other environment / spectrum buffers).
        auto run = [&](double tl, int budget) -> Status {
            if (budget <= 0) return Status{};
            QRCTM_TRY(qr_step_once(c));
            int n = 1;
            while (true) {
                const int slot = c->last_slot;
                const bool speculate = n < budget;
                // step i's spectrum is queued by step i+1 (after its QR), or here
                if (speculate) QRCTM_TRY(qr_step_once(c));
                else QRCTM_TRY(launch_owed_spectrum(c, c->ev_normed));
                QRCTM_HIP(hipMemcpyAsync(&dl, c->small() + SL_DELTA + slot, sizeof(double),
                                         hipMemcpyDeviceToHost, c->aux));
                QRCTM_TRY(hip_status(hipStreamSynchronize(c->aux), "hipStreamSynchronize"));
                if (!std::isfinite(dl) || dl < tl) {
                    if (speculate) {
                        c->owed.live = false;  // step i+1 is discarded with its spectrum
                        QRCTM_TRY(join_aux(c));
                        QRCTM_TRY(sync(c->st));
                        c->cur ^= 1;
                        c->spec_cur ^= 1;
                        c->steps--;
                        c->last_slot = slot;
                    }
                    break;
                }
                if (!speculate) break;
                ++n;
            }
            taken += n;
            return Status{};
        };
        // mixed forms: mixed steps down to mixed_tol, then FP64 refinement
        const bool refine = c->opts.precision != CTM_PREC_FP64 && c->opts.mixed_tol > 0.0 &&
                            c->opts.mixed_tol > tol;
        if (refine) {
            QRCTM_TRY(run(c->opts.mixed_tol, max_steps));
            if (std::isfinite(dl) && dl < c->opts.mixed_tol) {
                c->fp64_steps = true;
                const Status s = run(tol, max_steps - taken);
                c->fp64_steps = false;
                QRCTM_TRY(s);
            }
        } else {
            QRCTM_TRY(run(tol, max_steps));
        }
        c->last_delta = dl;
        QRCTM_TRY(check_bad(c, "ctm_converge"));
        if (!std::isfinite(dl)) {
            Status s;
            s.code = CTM_ENONFINITE;
            s.msg = "non-finite environment in ctm_converge";
            return s;
        }
        return Status{};
    });
    if (steps) *steps = taken;
    if (delta) *delta = dl;
    if (rc < 0) return rc;
    return (dl < tol) ? CTM_OK : CTM_NOTCONV;
}

int ctm_get_env(ctm_ctx* c, double* C, double* T, int* chi_cur) {
    if (!c) return fail(c, CTM_EINVAL, "NULL context");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        const size_t nC = (size_t)c->chi_cur * c->chi_cur;
        if (C) QRCTM_HIP(hipMemcpyAsync(C, c->C(), nC * 8, hipMemcpyDeviceToDevice, c->st));
        if (T) QRCTM_HIP(hipMemcpyAsync(T, c->T(), nC * c->sh.Dab * 8, hipMemcpyDeviceToDevice, c->st));
        if (chi_cur) *chi_cur = c->chi_cur;
        return sync(c->st);
    });
}

int ctm_set_env(ctm_ctx* c, const double* C, const double* T, int chi_cur) {
    if (!c || !C || !T) return fail(c, CTM_EINVAL, "NULL argument");
    if (chi_cur < 1 || chi_cur > c->sh.chi) return fail(c, CTM_EINVAL, "chi_cur out of range");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        const size_t nC = (size_t)chi_cur * chi_cur;
        QRCTM_HIP(hipMemcpyAsync(c->C(), C, nC * 8, hipMemcpyDeviceToDevice, c->st));
        QRCTM_HIP(hipMemcpyAsync(c->T(), T, nC * c->sh.Dab * 8, hipMemcpyDeviceToDevice, c->st));
        c->chi_cur = chi_cur;
        QRCTM_TRY(fresh_spectrum(c));
        return sync(c->st);
    });
}

int ctm_spectrum(ctm_ctx* c, double* s) {
    if (!c || !s) return fail(c, CTM_EINVAL, "NULL argument");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        QRCTM_HIP(hipMemcpyAsync(s, c->spec(), sizeof(double) * c->n_spec, hipMemcpyDeviceToHost,
                                 c->st));
        return sync(c->st);
    });
}

int ctm_energy(ctm_ctx* c, const double* h_nn, const double* h_nnn, double J2, double* E) {
    if (!c || !h_nn || !E) return fail(c, CTM_EINVAL, "NULL argument");
    if (!c->sh.quantum) return fail(c, CTM_ESTATE, "energy needs a site tensor (ctm_init)");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        EnergyArgs ea{};
        ea.d = c->sh.d; ea.D = c->sh.D; ea.chi = c->chi_cur;
        ea.C = c->C(); ea.T = c->T(); ea.As = c->ptr(c->plan.As);
        ea.a = c->ptr(c->plan.a);
        ea.Qbuf = c->ptr(c->plan.Q); ea.Ybuf = c->ptr(c->plan.Y); ea.Zbuf = c->ptr(c->plan.Z);
        ea.ws = c->ptr<char>(c->plan.energy); ea.ws_bytes = c->plan.energy_bytes;
        ea.splitk = c->ptr<void>(c->plan.splitk); ea.splitk_bytes = c->plan.splitk_bytes;
        return energy_eval(ea, h_nn, h_nnn, J2, E, c->st);
    });
}

int ctm_energy_grad(ctm_ctx* c, const double* h_nn, const double* h_nnn, double J2, double* E,
                    double* dA) {
    if (!c || !h_nn || !E || !dA) return fail(c, CTM_EINVAL, "NULL argument");
    if (!c->sh.quantum) return fail(c, CTM_ESTATE, "gradient needs a site tensor (ctm_init)");
    bool series_done = true;
    const int rc = guarded(c, [&]() -> Status {
        return energy_grad_impl(c, h_nn, h_nnn, J2, E, dA, &series_done);
    });
    return (rc == CTM_OK && !series_done) ? CTM_NOTCONV : rc;
}

int ctm_lnz_per_site(ctm_ctx* c, double* lnk) {
    if (!c || !lnk) return fail(c, CTM_EINVAL, "NULL argument");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        ClassicalArgs ca{};
        ca.Dab = c->sh.Dab; ca.chi = c->chi_cur;
        ca.C = c->C(); ca.T = c->T(); ca.a = c->ptr(c->plan.a);
        ca.ws = c->ptr<char>(c->plan.energy); ca.ws_bytes = c->plan.energy_bytes;
        return classical_lnz(ca, lnk, c->st);
    });
}

int ctm_expect_site(ctm_ctx* c, const double* imp, double* v) {
    if (!c || !imp || !v) return fail(c, CTM_EINVAL, "NULL argument");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        ClassicalArgs ca{};
        ca.Dab = c->sh.Dab; ca.chi = c->chi_cur;
        ca.C = c->C(); ca.T = c->T(); ca.a = c->ptr(c->plan.a);
        ca.ws = c->ptr<char>(c->plan.energy); ca.ws_bytes = c->plan.energy_bytes;
        return classical_expect(ca, imp, v, c->st);
    });
}

int ctm_stats(ctm_ctx* c, ctm_stats_t* st) {
    if (!c || !st) return fail(c, CTM_EINVAL, "NULL argument");
    return guarded(c, [&]() -> Status {
        QRCTM_TRY(join_aux(c));
        double r = NAN;
        QRCTM_HIP(hipMemcpyAsync(&r, c->small() + SL_RATIO, sizeof(double), hipMemcpyDeviceToHost,
                                 c->st));
        QRCTM_TRY(sync(c->st));
        st->chi = c->sh.chi;
        st->chi_cur = c->chi_cur;
        st->Dab = c->sh.Dab;
        st->steps = c->steps;
        st->last_delta = c->last_delta;
        st->flops_per_step =
            step_flops(c->chi_cur, c->sh.Dab, c->plan.Bk.bytes > 0 ? c->sh.d : 0);
        st->r_diag_ratio = c->steps > 0 ? r : NAN;
        st->timed_steps = c->timed_steps;
        for (int i = 0; i < kPhases; ++i) st->ms_phase[i] = c->ms_phase[i];
        st->grad_steps = c->grad_steps;
        st->fp_residual = c->fp_residual;
        unsigned long long fb = 0;
        if (c->qr_launches > 0)
            QRCTM_TRY(qr_fallback_count(c->ptr<void>(c->plan.qr), c->qr_chi * c->sh.Dab, c->qr_chi,
                                        c->st, &fb));
        st->qr_fallbacks = (long long)fb;
        const bool split = c->plan.Bk.bytes > 0;
        const int prec = c->opts.precision;
        if (split) st->edge_3b_form = prec == CTM_PREC_FP64 ? CTM_3B_SPLIT_FP64 : CTM_3B_SPLIT_FP32;
        else if (prec == CTM_PREC_FP64) st->edge_3b_form = CTM_3B_DOUBLE_LAYER_FP64;
        else if (prec == CTM_PREC_BF16X6_MFMA && c->plan.Y16.bytes > 0)
            st->edge_3b_form = CTM_3B_DOUBLE_LAYER_BF16X6;
        else st->edge_3b_form = CTM_3B_DOUBLE_LAYER_FP32;
        return Status{};
    });
}

int ctm_set_timing(ctm_ctx* c, int on) {
    if (!c) return fail(c, CTM_EINVAL, "NULL context");
    return guarded(c, [&]() -> Status {
        if (on && !c->ev[0]) {
            for (auto& e : c->ev) QRCTM_HIP(hipEventCreate(&e));
            for (auto& e : c->ev_sp) QRCTM_HIP(hipEventCreate(&e));
        }
        QRCTM_TRY(join_aux(c));
        c->timing = on != 0;
        for (double& m : c->ms_phase) m = 0.0;
        c->timed_steps = 0;
        return Status{};
    });
}

const char* ctm_last_error(const ctm_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

void ctm_destroy(ctm_ctx* c) { delete c; }

size_t ctm_qr_workspace_bytes(int m, int n) {
    if (m < n || n < 1) return 0;
    return qr_scratch_layout(m, n).total;
}

}  // extern "C"

namespace {

__global__ void zero_int_word_kernel(int* w) { *w = 0; }

// One thin QR on scratch ws (ws_bytes), as ctm_qr and ctm_qr_noalloc do it:
// the error word cleared by a kernel, the exchange buffers by qr_pos (epoch
// 0), then the factorisation; reads back the error word and the fallback count.
int run_qr(const double* M, double* Q, double* R, int m, int n, int method, void* ws,
           size_t ws_bytes, hipStream_t st, int* used_householder) {
    return guarded(nullptr, [&]() -> Status {
        const QrScratch L = qr_scratch_layout(m, n);
        if (ws == nullptr || ws_bytes < L.total) {
            Status s;
            s.code = CTM_EWORKSPACE;
            s.msg = "qr: workspace missing or smaller than ctm_qr_workspace_bytes";
            return s;
        }
        int* err = reinterpret_cast<int*>(static_cast<char*>(ws) + L.off_err);
        hipLaunchKernelGGL(zero_int_word_kernel, dim3(1), dim3(1), 0, st, err);
        QRCTM_TRY(launch_check("zero_int_word_kernel"));
        QRCTM_TRY(qr_pos(M, Q, R, m, n, ws, ws_bytes, st, nullptr, err, 0,
                         method == CTM_QR_HOUSEHOLDER ? kQrHouseholder : kQrAuto));
        int h = 0;
        QRCTM_HIP(hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, st));
        unsigned long long fb = 0;
        QRCTM_TRY(qr_fallback_count(ws, m, n, st, &fb));
        if (used_householder) *used_householder = (method == CTM_QR_HOUSEHOLDER || fb > 0) ? 1 : 0;
        if (h != 0) {
            Status s;
            s.code = CTM_EHIP;
            s.msg = "qr: an exchange between the workgroups of the Householder factorisation timed out";
            return s;
        }
        return Status{};
    });
}

int check_qr_args(const double* M, double* Q, double* R, int m, int n, int method) {
    if (!M || !Q || !R) return fail(nullptr, CTM_EINVAL, "NULL argument");
    if (m < n || n < 1) return fail(nullptr, CTM_EINVAL, "need m >= n >= 1");
    if (method != CTM_QR_AUTO && method != CTM_QR_HOUSEHOLDER)
        return fail(nullptr, CTM_EINVAL, "unknown QR method");
    return 0;
}

// Scratch of ctm_qr_noalloc: a fixed array in device memory, one copy per GPU,
// held until the process ends.  Its host-side name is not a device address;
// kernels get the address hipGetSymbolAddress returns for each device, taken
// once per device with that device current.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

Status noalloc_scratch(void** out) {
    int dev = -1;
    QRCTM_HIP(hipGetDevice(&dev));
    Status s;
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        s.code = CTM_EINVAL;
        s.msg = "ctm_qr_noalloc: device index beyond the library's table";
        return s;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[dev] == nullptr) {
        void* p = nullptr;
        QRCTM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) {
            s.code = CTM_EHIP;
            s.msg = "ctm_qr_noalloc: no device address for the scratch array";
            return s;
        }
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return s;
}

}  // namespace

extern "C" {

int ctm_qr(const double* M, double* Q, double* R, int m, int n, int method, void* ws,
           size_t ws_bytes, void* stream, int* used_householder) {
    const int bad = check_qr_args(M, Q, R, m, n, method);
    if (bad) return bad;
    return run_qr(M, Q, R, m, n, method, ws, ws_bytes, static_cast<hipStream_t>(stream),
                  used_householder);
}

size_t ctm_qr_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int ctm_qr_noalloc(const double* M, double* Q, double* R, int m, int n, int method, void* stream,
                   int* used_householder) {
    const int bad = check_qr_args(M, Q, R, m, n, method);
    if (bad) return bad;
    const size_t need = qr_scratch_layout(m, n).total;
    if (need > kNoAllocScratchBytes)
        return fail(nullptr, CTM_EWORKSPACE,
                    "ctm_qr_noalloc: an " + std::to_string(m) + " x " + std::to_string(n) +
                        " factorisation needs " + std::to_string(need) +
                        " bytes of scratch, more than the fixed " +
                        std::to_string(kNoAllocScratchBytes) + " (use ctm_qr with a workspace)");
    void* ws = nullptr;
    const int rc = guarded(nullptr, [&]() -> Status { return noalloc_scratch(&ws); });
    if (rc != 0) return rc;
    return run_qr(M, Q, R, m, n, method, ws, kNoAllocScratchBytes, static_cast<hipStream_t>(stream),
                  used_householder);
}

size_t ctm_gemm_workspace_bytes(int M, int N, int K) {
    if (M < 0 || N < 0 || K < 1) return 0;
    GemmDesc g;
    g.M = M; g.N = N; g.K = K;
    return gemm_splitk_bytes(g);
}

int ctm_gemm(int trans_a, int trans_b, int M, int N, int K, double alpha, const double* A, int lda,
             const double* B, int ldb, double beta, double* C, int ldc, void* ws, size_t ws_bytes,
             void* stream) {
    if (!A || !B || !C || M < 0 || N < 0 || K < 1) return fail(nullptr, CTM_EINVAL, "invalid GEMM");
    return guarded(nullptr, [&]() -> Status {
        hipStream_t st = static_cast<hipStream_t>(stream);
        GemmDesc g;
        g.trans_a = trans_a ? 1 : 0;
        g.trans_b = trans_b ? 1 : 0;
        g.M = M; g.N = N; g.K = K;
        g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
        g.C = C; g.map = OutMap::plain(M, N, ldc);
        g.alpha = alpha; g.beta = beta;
        QRCTM_TRY(gemm_f64(g, ws, ws_bytes, st));
        return sync(st);
    });
}

}  // extern "C"
