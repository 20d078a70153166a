/*
 * qrctm.h - C ABI of the MI355X QR-CTMRG library (libqrctm.so).
 *
 * The library runs C4v-symmetric corner-transfer-matrix renormalisation with a
 * QR decomposition of the reduced corner in place of the eigen/SVD
 * decomposition (Zhang, Yang, Corboz, arXiv:2505.00494, "QR-CTMRG" paragraph
 * and Fig. 1e/f), on one GPU, in FP64.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays named "device" are GPU pointers; "host" arrays are CPU pointers.
 *    Every array is FP64 and row-major (C order) with the leg order given.
 *      A[s,u,l,d,r]   site tensor, d*D^4 (physical, up, left, down, right).
 *      a[U,L,Dn,R]    double-layer / classical tensor, Dab^4.
 *      C[x,y]         corner, chi*chi, symmetric.
 *      T[x,m,y]       edge, chi*Dab*chi; x, y boundary legs (T[x,m,y]=T[y,m,x]),
 *                     m the leg facing the bulk.
 *  - Ownership: the caller owns every buffer it passes and keeps it alive while
 *    the context uses it.  All device scratch comes from ONE caller-provided
 *    workspace (size from ctm_workspace_bytes*); the library allocates no
 *    device memory.  The context itself is a small host object.
 *  - Streams: each context enqueues all its GPU work on the HIP stream given at
 *    creation (a hipStream_t passed as void*; NULL = the null stream).  Calls
 *    that return host scalars synchronise that stream.  A context is not
 *    thread-safe.
 *  - Errors: every int-returning call returns 0 on success, >0 for a warning,
 *    <0 for an error (codes below).  No C++ exception crosses the ABI.  After an
 *    error the context keeps its previous environment unless the message from
 *    ctm_last_error() says the context is invalid.
 */
#ifndef QRCTM_H
#define QRCTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CTM_OK          0
#define CTM_NOTCONV     1   /* warning: max_steps reached before tol        */
#define CTM_EINVAL     -1   /* invalid argument (sizes, null pointers)      */
#define CTM_EWORKSPACE -2   /* workspace missing or too small               */
#define CTM_EHIP       -3   /* HIP runtime error (text in ctm_last_error)   */
#define CTM_ENONFINITE -4   /* NaN/Inf produced or found in the input       */
#define CTM_ESINGULAR  -5   /* R of the reduced corner numerically singular */
#define CTM_ESTATE     -6   /* call not valid for this context              */

/* precision of the bulk contractions */
#define CTM_PREC_FP64      0
#define CTM_PREC_FP32_MFMA 1
/* split-BF16: each FP64 operand rounded to FP32 and split exactly into three
   bf16 parts; six bf16 products (all terms down to 2^-24 relative) with FP32
   accumulation on the bf16 matrix cores.  Used for the large products of the
   plain form's step (3a writes Y as planes, 3b is the double-layer product of
   planes, at the usual sizes with D even); the smaller products take the FP32
   path.  With the ket/bra split 3b (edge_split = 1) there is no bf16 build:
   every product then runs on the FP32 matrix cores, as CTM_PREC_FP32_MFMA
   (ctm_stats reports the 3b kernel). */
#define CTM_PREC_BF16X6_MFMA 2

/* Gradient schemes of ctm_energy_grad (ctm_opts.grad_mode). */
#define CTM_GRAD_CHECKPOINT  0   /* k tracked steps from the current environment  */
#define CTM_GRAD_FIXED_POINT 1   /* implicit differentiation at a converged one   */

typedef struct ctm_ctx ctm_ctx;

typedef struct ctm_opts {
    int precision;      /* CTM_PREC_*; QR, normalisation and the spectrum stay FP64 */
    int n_warmup;       /* standard (eigh) warm-up steps; -1 = as many as needed for
                           chi to reach its target (QR-CTMRG paragraph: 1-4 steps) */
    int k_tracked;      /* tracked QR steps in ctm_energy_grad (AD paragraph); -1 =
                           the per-D choice of the paper's timing study (Fig. 3
                           caption): 10, 12, 14, 16, 20, 24 for D = 2..7, 28 for
                           D >= 8 (not given there), 10 for D = 1                   */
    double qr_sing_tol; /* ctm_energy_grad fails with CTM_ESINGULAR when
                           min|R_ii| / max|R_ii| of a tracked step is below this
                           (unless qr_reg_eps > 0)                                  */
    double mixed_tol;   /* mixed precisions only: ctm_converge takes mixed steps until
                           the spectrum change is below max(tol, mixed_tol), then FP64
                           steps until it is below tol, so the converged environment is
                           an FP64 fixed point; 0 = mixed steps throughout             */
    int edge_split;     /* 1: the edge contraction T a of the QR step applies the ket
                           layer A and then the bra layer A (Fig. 1b) instead of the
                           double-layer tensor a: 4 d chi^2 D^6 in place of 2 chi^2 D^8
                           flops, same result up to rounding (FP64, or the FP32
                           matrix cores in the mixed precisions).
                           Used where available (quantum contexts with d = 2, D <= 8
                           and chi^2 D^4 < 2^31 - 2^16), otherwise ignored.  0: always
                           the double-layer product.                                     */
    int grad_mode;      /* CTM_GRAD_CHECKPOINT or CTM_GRAD_FIXED_POINT (ctm_energy_grad) */
    double fp_tol;      /* fixed point: the series stops when a term's norm is below
                           fp_tol times the norm of dE/d(C, T)                        */
    int fp_max_iter;    /* fixed point: at most this many reversed steps (rounded up
                           to even); ctm_energy_grad returns CTM_NOTCONV beyond it     */
    int grad_keep_yz;   /* 1: ctm_energy_grad keeps each tracked step's Y and Z (3a and
                           3b outputs, chi^2 D^4 doubles each) instead of recomputing
                           them in the reverse sweep: 2 max(k_tracked, 2) chi^2 D^4
                           doubles more workspace, the same result.  0: recompute.    */
    double qr_reg_eps;  /* QR adjoint: 0 = the exact R^{-1}; > 0 = a Tikhonov-regularised
                           one, each division by R_ii in the back substitution
                           replaced by a product with R_ii / (R_ii^2 + eps^2),
                           eps = qr_reg_eps * max|R_ii|, so that a rank-deficient
                           reduced corner gives a finite (regularised) gradient
                           instead of CTM_ESINGULAR                                   */
    int qr_method;      /* QR of the reduced corner (QR-CTMRG paragraph): CTM_QR_AUTO =
                           Cholesky-QR2 (Gram matrix, Cholesky, product with R^-1, twice;
                           the same unique factors with diag(R) > 0), with the
                           Householder factorisation run instead on the GPU whenever the
                           Cholesky step rejects the matrix (a non-positive pivot,
                           min R_ii < 1e-5 max R_ii, or a first-pass Q too far from
                           orthonormal, e.g. a rank-deficient reduced corner);
                           CTM_QR_HOUSEHOLDER = the Householder factorisation always  */
} ctm_opts;

#define CTM_QR_AUTO        0
#define CTM_QR_HOUSEHOLDER 1

/* Fill *o with defaults: FP64, n_warmup = -1, k_tracked = -1 (per D), qr_sing_tol =
   1e-14, mixed_tol = 1e-6, edge_split = 1, grad_mode = CTM_GRAD_CHECKPOINT, fp_tol =
   1e-10, fp_max_iter = 1000, grad_keep_yz = 0, qr_reg_eps = 0, qr_method = CTM_QR_AUTO. */
void ctm_default_opts(ctm_opts* o);

/*
 * Workspace sizes in bytes for a context built by ctm_init (site tensor, d, D,
 * target chi) or by ctm_init_dl (double-layer / classical tensor of bond Dab).
 * opts may be NULL (defaults).  Returns 0 for invalid sizes or options.
 */
size_t ctm_workspace_bytes(int d, int D, int chi, const ctm_opts* opts);
size_t ctm_workspace_bytes_dl(int Dab, int chi, const ctm_opts* opts);

/*
 * ctm_init: a1-a4 for a quantum iPEPS.
 *   A      device, d*D^4, raw site tensor (read during the call only).  The
 *          library applies the C4v average over the 8 leg permutations and
 *          scales to max|A| = 1 (iPEPS paragraph, C4v footnote), builds the
 *          double layer a = sum_s A (x) A (Fig. 1b), initialises C, T by
 *          contracting ket with bra on the open legs (footnote on the initial
 *          boundary), and runs the standard-CTMRG warm-up steps (eigh of the
 *          enlarged corner, Fig. 1d) that grow chi to its target.
 *   chi    target boundary dimension, Dab <= chi <= 1024, as far as the QR's
 *          workgroups hold their rows and the panel state in LDS (e.g. chi up to
 *          1024 at Dab = 4, 600 at Dab = 36, 512 at Dab = 64); CTM_EINVAL beyond.
 *   ws     device workspace of at least ctm_workspace_bytes(d, D, chi, opts).
 *   stream hipStream_t as void*.
 * Returns CTM_OK, CTM_EINVAL, CTM_EWORKSPACE, CTM_ENONFINITE or CTM_EHIP.
 */
int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi,
             const ctm_opts* opts, void* ws, size_t ws_bytes, void* stream);

/*
 * ctm_init_dl: same for a tensor network given directly by its bulk tensor
 * (Discussion paragraph: classical 2D partition functions).
 *   a      device, Dab^4, layout a[U,L,Dn,R]; must be C4v symmetric.
 *   bvec   device, Dab: vector contracted with every open boundary leg to form
 *          the initial C and T (all ones = free boundary).
 * ctm_energy / ctm_energy_grad return CTM_ESTATE on such a context.
 */
int ctm_init_dl(ctm_ctx** out, const double* a, const double* bvec, int Dab, int chi,
                const ctm_opts* opts, void* ws, size_t ws_bytes, void* stream);

/*
 * ctm_set_tensor: replace the site tensor (same d, D) and rebuild a; C and T
 * are kept (environment reuse between optimisation steps, AD paragraph).
 */
int ctm_set_tensor(ctm_ctx* ctx, const double* A);

/*
 * ctm_step: nsteps QR-CTMRG steps (QR-CTMRG paragraph, Fig. 1e/f):
 *   reduced corner c~ = C.T (chi*Dab x chi); Householder QR c~ = Q R with
 *   diag(R) >= 0; T' = Q^T (T a) Q; C' = T'.R.Q (accelerated corner);
 *   symmetrise and divide C', T' by their Frobenius norms; corner spectrum
 *   s = sort(|eig C'|)/sum and delta = ||s - s_prev||_2.
 * delta (host, may be NULL) receives the change of the last step.
 */
int ctm_step(ctm_ctx* ctx, int nsteps, double* delta);

/*
 * ctm_converge: QR steps until delta < tol or max_steps steps were taken
 * (the standard-CTMRG paragraph iterates the step to convergence).  steps / delta are
 * host outputs (may be NULL).  Returns CTM_NOTCONV when max_steps is reached.
 */
int ctm_converge(ctm_ctx* ctx, double tol, int max_steps, int* steps, double* delta);

/* Environment access (device arrays sized for the current chi_cur <= chi). */
int ctm_get_env(ctm_ctx* ctx, double* C, double* T, int* chi_cur /* host */);
int ctm_set_env(ctm_ctx* ctx, const double* C, const double* T, int chi_cur);

/* Normalised corner spectrum of the current C (host array of chi_cur entries). */
int ctm_spectrum(ctm_ctx* ctx, double* s);

/*
 * ctm_energy: energy per site from the current environment (Heisenberg and
 * J1-J2 paragraphs).  h_nn, h_nnn are HOST d^2 x d^2 bond operators, row index
 * (s1 s2), column index (s1' s2'); h_nnn may be NULL.
 *   E = 2 <h_nn> + 2 J2 <h_nnn>   (two bonds of each kind per site),
 * where <h> = Tr(rho h)/Tr(rho) of the two-site reduced density matrix of a
 * nearest-neighbour pair (2x1 cluster) or a diagonal pair (2x2 plaquette).
 */
int ctm_energy(ctm_ctx* ctx, const double* h_nn, const double* h_nnn, double J2,
               double* E);

/*
 * ctm_energy_grad: E and dE/dA (AD paragraph).  dA is a device array of d*D^4
 * entries, the gradient with respect to the raw A given to ctm_init /
 * ctm_set_tensor; E is a host output.  The environment is left unchanged.
 * h_nn, h_nnn, J2 as in ctm_energy: with h_nnn (J1-J2 paragraph) the
 * plaquette term and its reverse are included (d <= 4; chi >= D^2; four open
 * enlarged corners of (chi D^2)^2 doubles in the workspace's energy part).
 * Two schemes (opts.grad_mode):
 *   CTM_GRAD_CHECKPOINT: starting from the current environment, held fixed,
 *     run opts.k_tracked QR steps, evaluate E, and reverse the whole
 *     computation by hand-written adjoints (contraction adjoints, the thin-QR
 *     adjoint, the double layer and the C4v average).  (C_i, T_i) and each
 *     tracked step's Q, R, T', W are kept (k (4 chi^2 D^2 + 2 chi^2) doubles);
 *     the large intermediates Y and Z (chi^2 D^4 each) are recomputed in the
 *     reverse sweep, or kept too when opts.grad_keep_yz = 1.
 *   CTM_GRAD_FIXED_POINT: the fixed-point scheme (Discussion paragraph): the
 *     current environment must be converged.  With F one QR step and G = F o F
 *     (T may alternate between two gauges from step to step; the pair of
 *     steps is a fixed point in either case), dE/dA follows from the implicit
 *     function theorem, lam = ebar (I - dG/denv)^{-1} being summed as a
 *     Neumann series of reversed step pairs until a term's norm is below
 *     opts.fp_tol times |ebar|.  Memory: two environments, no checkpoints
 *     (with opts.grad_keep_yz = 1, the two steps' Y and Z as well).
 *     The environment must be a fixed point of G elementwise: CTM_ESTATE when
 *     |G(env) - env| / |env| > 1e-8 (the corner spectrum can converge while
 *     C and T still drift; the series then need not converge).  Returns
 *     CTM_NOTCONV (dA still written) after opts.fp_max_iter reversed steps, or
 *     when the terms grow (the linearised step pair does not contract);
 *     ctm_stats reports the steps taken and the residual.
 * Returns CTM_ESINGULAR when a reversed step's R has min|R_ii|/max|R_ii| below
 * opts.qr_sing_tol.
 */
int ctm_energy_grad(ctm_ctx* ctx, const double* h_nn, const double* h_nnn, double J2,
                    double* E, double* dA);

/* Classical networks: ln of the partition function per site, and <O> at one
 * site from a device impurity tensor imp[U,L,Dn,R] (Dab^4). */
int ctm_lnz_per_site(ctm_ctx* ctx, double* lnk);
int ctm_expect_site(ctm_ctx* ctx, const double* imp, double* v);

typedef struct ctm_stats_t {
    int chi, chi_cur, Dab;
    long long steps;          /* QR steps taken since creation                 */
    double last_delta;
    double flops_per_step;    /* algorithmic flops of one QR step              */
    double r_diag_ratio;      /* min|R_ii|/max|R_ii| of the last QR            */
    long long timed_steps;    /* QR steps timed since ctm_set_timing(ctx, 1)   */
    double ms_phase[8];       /* GPU ms summed over the timed steps, per phase:
                                 0 reduced corner, 1 QR, 2 T.Q (3a),
                                 3 double-layer contraction (3b), 4 .Q (3c),
                                 5 accelerated corner, 6 symmetrise/normalise,
                                 7 corner spectrum                             */
    long long grad_steps;     /* steps reversed by the last ctm_energy_grad    */
    double fp_residual;       /* |G(env) - env| / |env| seen by the last
                                 fixed-point ctm_energy_grad (G: two steps)    */
    long long qr_fallbacks;   /* QRs (steps and tracked steps) that ran the
                                 Householder factorisation because Cholesky-QR2
                                 rejected the reduced corner (CTM_QR_AUTO),
                                 counted since chi_cur last changed            */
    int edge_3b_form;         /* kernel of the middle edge product (3b) in the
                                 context's QR steps: CTM_3B_* below            */
} ctm_stats_t;

/* ctm_stats_t.edge_3b_form */
#define CTM_3B_DOUBLE_LAYER_FP64   0  /* one GEMM with the double layer, FP64     */
#define CTM_3B_DOUBLE_LAYER_FP32   1  /* the same on the FP32 matrix cores         */
#define CTM_3B_DOUBLE_LAYER_BF16X6 2  /* the same as six bf16 products of split
                                         planes (FP32 accumulation)               */
#define CTM_3B_SPLIT_FP64          3  /* fused ket/bra split, FP64                 */
#define CTM_3B_SPLIT_FP32          4  /* fused ket/bra split, FP32 matrix cores    */
int ctm_stats(ctm_ctx* ctx, ctm_stats_t* st);

/* Per-phase timing of QR steps with HIP events on the context stream (on = 1)
 * or off (0); switching resets the accumulated times.  Timing synchronises the
 * stream once per step. */
int ctm_set_timing(ctm_ctx* ctx, int on);

/* Message of the last failing call on ctx (or on creation if ctx is NULL). */
const char* ctm_last_error(const ctm_ctx* ctx);
void ctm_destroy(ctm_ctx* ctx);

/*
 * Component entry points (one kernel chain each), exposed for tests at full
 * size.  All arrays device, row-major; stream as above; they synchronise.
 *
 * ctm_qr: thin QR of M (m x n, m >= n) with diag(R) >= 0 (QR-CTMRG paragraph:
 *   unpivoted QR of the reduced corner).  Q is m x n, R n x n upper
 *   triangular; Q may alias M.  method: CTM_QR_AUTO or CTM_QR_HOUSEHOLDER as
 *   for ctm_opts.qr_method.  used_householder (host, may be NULL) receives 1
 *   when the Householder factorisation ran (always for CTM_QR_HOUSEHOLDER; for
 *   CTM_QR_AUTO when Cholesky-QR2 rejected M), else 0.  ws of
 *   ctm_qr_workspace_bytes(m, n).
 */
size_t ctm_qr_workspace_bytes(int m, int n);
int ctm_qr(const double* M, double* Q, double* R, int m, int n, int method, void* ws,
           size_t ws_bytes, void* stream, int* used_householder);

/*
 * ctm_qr_noalloc: ctm_qr for callers that cannot allocate device memory (code
 *   under stream capture, tight serving loops, hosts that forbid allocation):
 *   the same factorisation and result, with its scratch in a fixed array of
 *   ctm_qr_noalloc_max_bytes() (64 MiB) that the library holds on every GPU it
 *   runs on until the process ends.  Nothing is allocated on any call.  The
 *   caller passes M, Q, R (device) as for ctm_qr.  Sizes whose scratch
 *   (ctm_qr_workspace_bytes(m, n)) exceeds the array fail with CTM_EWORKSPACE
 *   before any GPU work (e.g. 5184 x 144 and 9604 x 196 fit, 16384 x 256 does
 *   not).  All calls on one GPU share that GPU's array, whose contents persist
 *   from call to call: calls that overlap on one GPU (other streams, other
 *   threads) race and must be serialised by the caller.  Synchronises stream.
 */
size_t ctm_qr_noalloc_max_bytes(void);
int ctm_qr_noalloc(const double* M, double* Q, double* R, int m, int n, int method, void* stream,
                   int* used_householder);

/*
 * ctm_gemm: C = alpha * op(A) op(B) + beta * C, FP64 on the matrix cores (the
 *   kernel behind every contraction of the step; products of at least 3e10
 *   flop, 2 M N K, with at least 256 output tiles of 128 x 128 run as rocBLAS
 *   dgemm with atomics off, reproducibly).
 *   op(A) is M x K: trans_a = 0 -> A[m*lda + k], 1 -> A[k*lda + m].
 *   op(B) is K x N: trans_b = 0 -> B[k*ldb + n], 1 -> B[n*ldb + k].
 *   C is M x N at C[m*ldc + n].  ws: device scratch of at least
 *   ctm_gemm_workspace_bytes(M, N, K) bytes (0 for most shapes; may be NULL then).
 */
size_t ctm_gemm_workspace_bytes(int M, int N, int K);
int ctm_gemm(int trans_a, int trans_b, int M, int N, int K, double alpha,
             const double* A, int lda, const double* B, int ldb, double beta,
             double* C, int ldc, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QRCTM_H */
